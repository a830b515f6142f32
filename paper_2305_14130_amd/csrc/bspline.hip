// Cubic B-spline model parameterization (the smoothing regularization of the field
// example): planes of coefficients c [np][Nz][Nx] on a coarse node grid expand to model
// planes m [np][nz][nx] = Bz c Bx^T, and gradients map back as Bz^T g Bx. Along an axis
// with node spacing D cells, node k sits at cell (k - 1) D with the uniform cubic B-spline
// B((i - (k - 1) D) / D), support |t| < 2; N = ceil((n - 1) / D) + 3 nodes. FP64 weights
// and sums, rounded once; gather form (each output summed by one thread in a fixed order,
// no atomics), so results are deterministic. Both maps are separable: a workgroup takes one
// row (or row segment) of outputs and combines along z once per row, along x per output.
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


// Expansion: one workgroup per segment of `cols` columns of one output row (plane p, row
// i). The z-combination of the (up to four) coefficient rows the row uses is formed once per
// node the segment reaches (in LDS, after the x weight table), then each column sums its (up
// to four) nodes with the tabulated x weights. Segments of up to 4096 columns and 1024
// nodes: longer ones amortize the table over more columns (1000 x 3000 planes, nodes every
// 20 columns: 0.32 ms at 1024 columns, 0.23 ms at 4096), more nodes cost occupancy (every
// column a node: 0.68 ms at 1024 columns, 0.94 ms at 4096).
__global__ __launch_bounds__(BB) void k_bspline_expand(int nz, int nx, int Dz, int Dx, int Nz, int Nx, int cols,
                                                       const float* __restrict__ c, float* __restrict__ m) {
  extern __shared__ double wtab[];
  double* wxs = wtab;                 // wxs[d + 2 Dx - 1] = B(d / Dx)
  double* tn = wtab + 4 * Dx - 1;     // z-combined coefficients of the segment's nodes
  for (int u = threadIdx.x; u < 4 * Dx - 1; u += BB) wxs[u] = bsp((double)(u - 2 * Dx + 1) * (1.0 / Dx));
  const int row = blockIdx.x, i = row % nz, p = row / nz;
  const int j0 = blockIdx.y * cols, j1 = min(nx, j0 + cols) - 1;
  const int a0 = i / Dz, blo = j0 / Dx, bhi = min(Nx - 1, j1 / Dx + 3);
  // node a0 + v at row i: offset i - (a0 + v - 1) Dz (index tz - v Dz of a z table)
  const int tz = i - (a0 - 1) * Dz + 2 * Dz - 1;
  const float* cp = c + (size_t)p * Nz * Nx;
  for (int b = blo + (int)threadIdx.x; b <= bhi; b += BB) {
    double t = 0.0;
    for (int v = 0; v < 4 && a0 + v < Nz; ++v) {
      const int iv = tz - v * Dz;
      if (iv < 0) break;
      t += bsp((double)(iv - 2 * Dz + 1) * (1.0 / Dz)) * (double)cp[(size_t)(a0 + v) * Nx + b];
    }
    tn[b - blo] = t;
  }
  __syncthreads();
  float* mrow = m + (size_t)row * nx;
  // the thread's columns step by BB: carry j's node b0 = j / Dx and remainder r = j - b0 Dx
  // from one to the next instead of dividing per column
  const int qs = BB / Dx, rs = BB - qs * Dx;
  int j = j0 + (int)threadIdx.x, b0 = j / Dx, r = j - b0 * Dx;
  for (; j <= j1; j += BB) {
    // node b0 + u at cell j: offset r + (1 - u) Dx, table index that + 2 Dx - 1; it is -1
    // (offset -2 Dx, weight 0) for u = 3 when r = 0, hence the guard
    const int tx = r + 3 * Dx - 1;
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int iu = tx - u * Dx;
      if (b0 + u < Nx && iu >= 0) s += wxs[iu] * tn[b0 + u - blo];
    }
    mrow[j] = (float)s;
    b0 += qs;
    r += rs;
    if (r >= Dx) r -= Dx, ++b0;
  }
}

// Transpose: one workgroup per group of ADJ_NODES nodes of `rows` (at most ADJ_ROWS)
// consecutive coefficient rows (plane p, node rows a0 ..). The input rows in the union of those rows' z supports are
// staged in LDS one after the other, in chunks of `chunk` cells (after the x weight table);
// each thread sums, for each of its nodes, the staged cells in the node's support with the
// tabulated x weights (every lane of a wave reads the same table entry), once per input row,
// and adds that sum times the row's z weight to each coefficient row whose support holds the
// input row (each in ascending input-row order, as one row at a time would).
constexpr int ADJ_NPT = 4, ADJ_NODES = ADJ_NPT * BB, ADJ_ROWS = 4;

__global__ __launch_bounds__(BB) void k_bspline_adjoint(int nz, int nx, int Dz, int Dx, int Nz, int Nx, int chunk,
                                                        int rows, const float* __restrict__ g,
                                                        float* __restrict__ cb) {
  extern __shared__ double wtab[];
  double* wxs = wtab;                                   // wxs[d + 2 Dx - 1] = B(d / Dx)
  float* gs = reinterpret_cast<float*>(wtab + 4 * Dx - 1);
  for (int u = threadIdx.x; u < 4 * Dx - 1; u += BB) wxs[u] = bsp((double)(u - 2 * Dx + 1) * (1.0 / Dx));
  const int rgroups = (Nz + rows - 1) / rows;
  const int p = blockIdx.x / rgroups, a0 = (blockIdx.x - p * rgroups) * rows;
  const int a1 = min(Nz, a0 + rows) - 1;
  const int bfirst = blockIdx.y * ADJ_NODES, blast = min(Nx, bfirst + ADJ_NODES) - 1;
  // cells the group's nodes reach; rows in node row a's support: (a - 3) D < i < (a + 1) D
  const int cfirst = max(0, (bfirst - 3) * Dx + 1), clast = min(nx - 1, (blast + 1) * Dx - 1);
  const int i0 = max(0, (a0 - 3) * Dz + 1), i1 = min(nz - 1, (a1 + 1) * Dz - 1);
  const float* gp = g + (size_t)p * nz * nx;
  double acc[ADJ_ROWS][ADJ_NPT], h[ADJ_NPT];
#pragma unroll
  for (int r = 0; r < ADJ_ROWS; ++r)
#pragma unroll
    for (int q = 0; q < ADJ_NPT; ++q) acc[r][q] = 0.0;
  for (int i = i0; i <= i1; ++i) {
#pragma unroll
    for (int q = 0; q < ADJ_NPT; ++q) h[q] = 0.0;
    for (int c0 = cfirst; c0 <= clast; c0 += chunk) {
      const int c1 = min(clast, c0 + chunk - 1);
      __syncthreads();   // the previous chunk (and the table) is complete and no longer read
      for (int j = c0 + (int)threadIdx.x; j <= c1; j += BB) gs[j - c0] = gp[(size_t)i * nx + j];
      __syncthreads();
#pragma unroll
      for (int q = 0; q < ADJ_NPT; ++q) {
        const int b = bfirst + (int)threadIdx.x + q * BB;
        if (b > blast) continue;
        const int jl = max(max((b - 3) * Dx + 1, c0), 0), jh = min(min((b + 1) * Dx - 1, c1), nx - 1);
        const int ox = 2 * Dx - 1 - (b - 1) * Dx;   // wxs[j + ox]: node b, cell j
        double rs = 0.0;
        for (int j = jl; j <= jh; ++j) rs += (double)gs[j - c0] * wxs[j + ox];
        h[q] += rs;
      }
    }
#pragma unroll
    for (int r = 0; r < ADJ_ROWS; ++r) {
      const int a = a0 + r;
      if (a > a1 || i <= (a - 3) * Dz || i >= (a + 1) * Dz) continue;   // i outside row a's support
      const double wz = bsp((double)(i - (a - 1) * Dz) * (1.0 / Dz));
#pragma unroll
      for (int q = 0; q < ADJ_NPT; ++q) acc[r][q] += wz * h[q];
    }
  }
#pragma unroll
  for (int r = 0; r < ADJ_ROWS; ++r) {
    if (a0 + r > a1) continue;
    float* crow = cb + ((size_t)p * Nz + a0 + r) * Nx;
#pragma unroll
    for (int q = 0; q < ADJ_NPT; ++q) {
      const int b = bfirst + (int)threadIdx.x + q * BB;
      if (b <= blast) crow[b] = (float)acc[r][q];
    }
  }
}

}  // namespace

int bspline_nodes(int n, int D) { return (n - 1 + D - 1) / D + 3; }

hipError_t launch_bspline_expand(int np, int nz, int nx, int Dz, int Dx, const float* c, float* m, hipStream_t st) {
  if ((long)np * nz <= 0 || nx <= 0) return hipSuccess;
  if ((long)np * nz > 0x7fffffffL) return hipErrorInvalidValue;   // one workgroup row per output row
  const int cols = std::min(4096, 1024 * Dx);
  const size_t lds = (size_t)(4 * Dx - 1 + cols / Dx + 5) * sizeof(double);
  if (lds > 64 * 1024) return hipErrorInvalidValue;   // the entry points refuse such spacings
  if ((nx + cols - 1) / cols > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((long)np * nz), (unsigned)((nx + cols - 1) / cols));
  k_bspline_expand<<<grid, BB, lds, st>>>(nz, nx, Dz, Dx, bspline_nodes(nz, Dz), bspline_nodes(nx, Dx), cols, c, m);
  return hipGetLastError();
}

hipError_t launch_bspline_adjoint(int np, int nz, int nx, int Dz, int Dx, const float* g, float* cb, hipStream_t st) {
  const int Nz = bspline_nodes(nz, Dz), Nx = bspline_nodes(nx, Dx);
  if ((long)np * Nz <= 0) return hipSuccess;
  // coefficient rows per workgroup: four share each staged input row's x sums (an input row
  // lies in four rows' z supports), one where that would leave the GPU too few workgroups
  const int rows = (long)np * Nz >= 2048 ? ADJ_ROWS : 1;
  const long rgroups = (Nz + rows - 1) / rows;
  if ((long)np * rgroups > 0x7fffffffL || (Nx + ADJ_NODES - 1) / ADJ_NODES > 65535) return hipErrorInvalidValue;
  const size_t table = (size_t)(4 * Dx - 1) * sizeof(double);
  if (table + sizeof(float) > 64 * 1024) return hipErrorInvalidValue;   // the entry points refuse such spacings
  // staged cells: what the 64 KB of LDS leave beside the table, at most 4096
  const int chunk = (int)std::min<size_t>(4096, (64 * 1024 - table) / sizeof(float));
  const size_t lds = table + (size_t)chunk * sizeof(float);
  const dim3 grid((unsigned)(np * rgroups), (unsigned)((Nx + ADJ_NODES - 1) / ADJ_NODES));
  k_bspline_adjoint<<<grid, BB, lds, st>>>(nz, nx, Dz, Dx, Nz, Nx, chunk, rows, g, cb);
  return hipGetLastError();
}

}  // namespace efwi
