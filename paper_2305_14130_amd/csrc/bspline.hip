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

// Weight of node k at cell i (node spacing D).
__device__ __forceinline__ double wgt(int i, int k, int D) { return bsp((double)(i - (k - 1) * D) / (double)D); }

__global__ __launch_bounds__(BB) void k_bspline_expand(int np, int nz, int nx, int Dz, int Dx, int Nz, int Nx,
                                                       const float* __restrict__ c, float* __restrict__ m) {
  const long total = (long)np * nz * nx;
  for (long q = blockIdx.x * (long)BB + threadIdx.x; q < total; q += (long)gridDim.x * BB) {
    const int j = (int)(q % nx);
    const long r = q / nx;
    const int i = (int)(r % nz), p = (int)(r / nz);
    const int a0 = i / Dz, b0 = j / Dx;
    const float* cp = c + (long)p * Nz * Nx;
    double s = 0.0;
    for (int a = a0; a < std::min(a0 + 4, Nz); ++a) {
      const double wz = wgt(i, a, Dz);
      double row = 0.0;
      for (int b = b0; b < std::min(b0 + 4, Nx); ++b) row += (double)cp[(long)a * Nx + b] * wgt(j, b, Dx);
      s += wz * row;
    }
    m[q] = (float)s;
  }
}

__global__ __launch_bounds__(BB) void k_bspline_adjoint(int np, int nz, int nx, int Dz, int Dx, int Nz, int Nx,
                                                        const float* __restrict__ g, float* __restrict__ cb) {
  const long total = (long)np * Nz * Nx;
  for (long q = blockIdx.x * (long)BB + threadIdx.x; q < total; q += (long)gridDim.x * BB) {
    const int b = (int)(q % Nx);
    const long r = q / Nx;
    const int a = (int)(r % Nz), p = (int)(r / Nz);
    // cells in the node's support: (k - 3) D < i < (k + 1) D
    const int i0 = std::max(0, (a - 3) * Dz + 1), i1 = std::min(nz - 1, (a + 1) * Dz - 1);
    const int j0 = std::max(0, (b - 3) * Dx + 1), j1 = std::min(nx - 1, (b + 1) * Dx - 1);
    const float* gp = g + (long)p * nz * nx;
    double s = 0.0;
    for (int i = i0; i <= i1; ++i) {
      double row = 0.0;
      for (int j = j0; j <= j1; ++j) row += (double)gp[(long)i * nx + j] * wgt(j, b, Dx);
      s += wgt(i, a, Dz) * row;
    }
    cb[q] = (float)s;
  }
}

int grid_for(long total) { return (int)std::max(1L, std::min((total + BB - 1) / BB, 8192L)); }

}  // namespace

int bspline_nodes(int n, int D) { return (n - 1 + D - 1) / D + 3; }

hipError_t launch_bspline_expand(int np, int nz, int nx, int Dz, int Dx, const float* c, float* m, hipStream_t st) {
  const long total = (long)np * nz * nx;
  k_bspline_expand<<<grid_for(total), BB, 0, st>>>(np, nz, nx, Dz, Dx, bspline_nodes(nz, Dz), bspline_nodes(nx, Dx), c,
                                                   m);
  return hipGetLastError();
}

hipError_t launch_bspline_adjoint(int np, int nz, int nx, int Dz, int Dx, const float* g, float* cb, hipStream_t st) {
  const int Nz = bspline_nodes(nz, Dz), Nx = bspline_nodes(nx, Dx);
  const long total = (long)np * Nz * Nx;
  k_bspline_adjoint<<<grid_for(total), BB, 0, st>>>(np, nz, nx, Dz, Dx, Nz, Nx, g, cb);
  return hipGetLastError();
}

}  // namespace efwi
