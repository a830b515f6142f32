// The approximate inverse pseudo-Hessian of the comparison with alternative methods
// (Synthetic example): the per-shot zero-lag velocity autocorrelations (accumulated by the
// forward step kernel) are summed over shots into the full grid, clipped from below at a
// fraction of their maximum, inverted and scaled to a largest value of 1.
#include <algorithm>

#include "efwi_internal.h"

namespace efwi {
namespace {

constexpr int PB = 256;          // threads per block
constexpr int MAX_PARTIALS = 1024;

// h[z0 + i][x0 + j] += acc[i][j] over one shot's window (acc has row pitch cp, h pitch mld).
__global__ __launch_bounds__(PB) void k_add_window(const float* __restrict__ acc, int cp, int nz, int nx,
                                                   float* __restrict__ h, long mld, int z0, int x0) {
  const int j = blockIdx.x * PB + threadIdx.x, i = blockIdx.y;
  if (j >= nx || i >= nz) return;
  h[(long)(z0 + i) * mld + (x0 + j)] += acc[(long)i * cp + j];
}

__device__ __forceinline__ float block_max(float v, float* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = PB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  return sh[0];
}

// Largest value of each block's grid-stride share of h (h >= 0, so 0 is the identity).
__global__ __launch_bounds__(PB) void k_max_partials(const float* __restrict__ h, long n,
                                                     float* __restrict__ partial) {
  __shared__ float sh[PB];
  float m = 0.0f;
  for (long q = (long)blockIdx.x * PB + threadIdx.x; q < n; q += (long)gridDim.x * PB) m = fmaxf(m, h[q]);
  m = block_max(m, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = m;
}

// p = c top / max(h, c top), top = max(h) from the partials (every block reduces them
// itself); p = 1 everywhere when top is 0.
__global__ __launch_bounds__(PB) void k_inverse_diag(const float* __restrict__ h, long n,
                                                     const float* __restrict__ partial, int np, float clip,
                                                     float* __restrict__ p) {
  __shared__ float sh[PB];
  float m = 0.0f;
  for (int k = threadIdx.x; k < np; k += PB) m = fmaxf(m, partial[k]);
  const float top = block_max(m, sh);
  const float floor_ = clip * top;
  for (long q = (long)blockIdx.x * PB + threadIdx.x; q < n; q += (long)gridDim.x * PB)
    p[q] = top > 0.0f ? floor_ / fmaxf(h[q], floor_) : 1.0f;
}

}  // namespace

hipError_t launch_add_window(const float* acc, int cp, int nz, int nx, float* h, long mld, int z0, int x0,
                             hipStream_t st) {
  if (nz <= 0 || nx <= 0) return hipSuccess;
  k_add_window<<<dim3((nx + PB - 1) / PB, nz), PB, 0, st>>>(acc, cp, nz, nx, h, mld, z0, x0);
  return hipGetLastError();
}

int inverse_diag_partials(long n) {
  const long b = (n + PB - 1) / PB;
  return (int)std::max(1L, std::min(b, (long)MAX_PARTIALS));
}

hipError_t launch_inverse_diag(const float* h, long n, float clip, float* p, float* partial, hipStream_t st) {
  const int nb = inverse_diag_partials(n);
  k_max_partials<<<nb, PB, 0, st>>>(h, n, partial);
  k_inverse_diag<<<nb, PB, 0, st>>>(h, n, partial, nb, clip, p);
  return hipGetLastError();
}

}  // namespace efwi
