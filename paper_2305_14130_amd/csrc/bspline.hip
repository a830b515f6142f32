// Cubic B-spline model parameterization (the smoothing regularization of the field
// example): planes of coefficients c [np][Nz][Nx] on a coarse node grid expand to model
// planes m [np][nz][nx] = Bz c Bx^T, and gradients map back as Bz^T g Bx. Along an axis
// with node spacing D cells, node k sits at cell (k - 1) D with the uniform cubic B-spline
// B((i - (k - 1) D) / D), support |t| < 2; N = ceil((n - 1) / D) + 3 nodes. FP64 weights
// and sums, rounded once; gather form (one thread per output), so results are
// deterministic.
#include <algorithm>

#include "efwi_internal.h"

namespace efwi {
namespace {

constexpr int BB = 256;

__device__ __forceinline__ double bsp(double t) {
  const double a = fabs(t);
  if (a < 1.0) return 2.0 / 3.0 - a * a + 0.5 * a * a * a;
  if (a < 2.0) {
    const double u = 2.0 - a;
    return u * u * u / 6.0;
  }
  return 0.0;
}


__global__ __launch_bounds__(BB) void k_bspline_expand(int np, int nz, int nx, int Dz, int Dx, int Nz, int Nx,
                                                       const float* __restrict__ c, float* __restrict__ m) {
  extern __shared__ double wtab[];   // weight tables as in k_bspline_adjoint
  double* wxs = wtab;
  double* wzs = wtab + 4 * Dx - 1;
  for (int u = threadIdx.x; u < 4 * Dx - 1; u += BB) wxs[u] = bsp((double)(u - 2 * Dx + 1) * (1.0 / Dx));
  for (int u = threadIdx.x; u < 4 * Dz - 1; u += BB) wzs[u] = bsp((double)(u - 2 * Dz + 1) * (1.0 / Dz));
  __syncthreads();
  const long total = (long)np * nz * nx;
  for (long q = blockIdx.x * (long)BB + threadIdx.x; q < total; q += (long)gridDim.x * BB) {
    const int j = (int)(q % nx);
    const long r = q / nx;
    const int i = (int)(r % nz), p = (int)(r / nz);
    const int a0 = i / Dz, b0 = j / Dx;
    const float* cp = c + (long)p * Nz * Nx;
    // node b0 + u at cell j: offset j - (b0 + u - 1) Dx, table index that + 2 Dx - 1; it is
    // -1 (offset -2 Dx, weight 0) for u = 3 when j is a multiple of Dx, hence the guard
    const int tx = j - (b0 - 1) * Dx + 2 * Dx - 1, tz = i - (a0 - 1) * Dz + 2 * Dz - 1;
    double s = 0.0;
    for (int v = 0; v < 4 && a0 + v < Nz; ++v) {
      const int iv = tz - v * Dz;
      if (iv < 0) break;
      const float* row_c = cp + (long)(a0 + v) * Nx + b0;
      double row = 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int iu = tx - u * Dx;
        if (b0 + u < Nx && iu >= 0) row += (double)row_c[u] * wxs[iu];
      }
      s += wzs[iv] * row;
    }
    m[q] = (float)s;
  }
}

// The weight of node k at cell i depends on the offset i - (k - 1) D only: tables of the
// 4 D - 1 nonzero weights per axis (offsets -2 D + 1 .. 2 D - 1) in LDS, filled once per
// workgroup; the dynamic LDS holds the x table then the z table.
__global__ __launch_bounds__(BB) void k_bspline_adjoint(int np, int nz, int nx, int Dz, int Dx, int Nz, int Nx,
                                                        const float* __restrict__ g, float* __restrict__ cb) {
  extern __shared__ double wtab[];
  double* wxs = wtab;                 // wxs[d + 2 Dx - 1] = B(d / Dx)
  double* wzs = wtab + 4 * Dx - 1;    // wzs[d + 2 Dz - 1] = B(d / Dz)
  const double iz = 1.0 / Dz, ix = 1.0 / Dx;
  for (int u = threadIdx.x; u < 4 * Dx - 1; u += BB) wxs[u] = bsp((double)(u - 2 * Dx + 1) * ix);
  for (int u = threadIdx.x; u < 4 * Dz - 1; u += BB) wzs[u] = bsp((double)(u - 2 * Dz + 1) * iz);
  __syncthreads();
  const long total = (long)np * Nz * Nx;
  for (long q = blockIdx.x * (long)BB + threadIdx.x; q < total; q += (long)gridDim.x * BB) {
    const int b = (int)(q % Nx);
    const long r = q / Nx;
    const int a = (int)(r % Nz), p = (int)(r / Nz);
    // cells in the node's support: (k - 3) D < i < (k + 1) D
    const int i0 = std::max(0, (a - 3) * Dz + 1), i1 = std::min(nz - 1, (a + 1) * Dz - 1);
    const int j0 = std::max(0, (b - 3) * Dx + 1), j1 = std::min(nx - 1, (b + 1) * Dx - 1);
    const float* gp = g + (long)p * nz * nx;
    const int ox = 2 * Dx - 1 - (b - 1) * Dx, oz = 2 * Dz - 1 - (a - 1) * Dz;   // wxs[j + ox]: node b, cell j
    double s = 0.0;
    for (int i = i0; i <= i1; ++i) {
      const float* gr = gp + (long)i * nx;
      double r0 = 0.0, r1 = 0.0, r2 = 0.0, r3 = 0.0;   // four partial sums: independent chains
      int j = j0;
      for (; j + 3 <= j1; j += 4) {
        r0 += (double)gr[j] * wxs[j + ox];
        r1 += (double)gr[j + 1] * wxs[j + 1 + ox];
        r2 += (double)gr[j + 2] * wxs[j + 2 + ox];
        r3 += (double)gr[j + 3] * wxs[j + 3 + ox];
      }
      for (; j <= j1; ++j) r0 += (double)gr[j] * wxs[j + ox];
      s += wzs[i + oz] * ((r0 + r1) + (r2 + r3));
    }
    cb[q] = (float)s;
  }
}

int grid_for(long total) { return (int)std::max(1L, std::min((total + BB - 1) / BB, 8192L)); }

}  // namespace

int bspline_nodes(int n, int D) { return (n - 1 + D - 1) / D + 3; }

hipError_t launch_bspline_expand(int np, int nz, int nx, int Dz, int Dx, const float* c, float* m, hipStream_t st) {
  const long total = (long)np * nz * nx;
  const size_t lds = (size_t)(4 * Dx - 1 + 4 * Dz - 1) * sizeof(double);
  if (lds > 64 * 1024) return hipErrorInvalidValue;   // the entry points refuse such spacings
  k_bspline_expand<<<grid_for(total), BB, lds, st>>>(np, nz, nx, Dz, Dx, bspline_nodes(nz, Dz), bspline_nodes(nx, Dx),
                                                     c, m);
  return hipGetLastError();
}

hipError_t launch_bspline_adjoint(int np, int nz, int nx, int Dz, int Dx, const float* g, float* cb, hipStream_t st) {
  const int Nz = bspline_nodes(nz, Dz), Nx = bspline_nodes(nx, Dx);
  const long total = (long)np * Nz * Nx;
  const size_t lds = (size_t)(4 * Dx - 1 + 4 * Dz - 1) * sizeof(double);
  if (lds > 64 * 1024) return hipErrorInvalidValue;   // the entry points refuse such spacings
  k_bspline_adjoint<<<grid_for(total), BB, lds, st>>>(np, nz, nx, Dz, Dx, Nz, Nx, g, cb);
  return hipGetLastError();
}

}  // namespace efwi
