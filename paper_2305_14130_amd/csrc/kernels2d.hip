// 2D isotropic elastic velocity-stress kernels for gfx950 (forward, exact transpose,
// imaging condition, chain rule, misfit).
//
// Method passages: Forward problem eq.(1) (wave equation), eq.(2) (moment-tensor point
// source), eq.(3) (sampling operator, here DAS e_xx); Solving the inverse problem eq.(4)
// (L2 misfit) and eq.(6) (per-shot gradient J_s^T r by the adjoint-state method); Model
// extension eq.(8) (shot s differentiates only its own component m_s).
//
// Staggering: sxx, szz at (i, j); vx at (i, j+1/2); vz at (i+1/2, j); sxz at (i+1/2, j+1/2).
// Differences are 4th order with coefficients 9/8 and -1/24, values outside the grid are
// zero (zero halo of the padded arrays), time stepping is leapfrog, the absorbing
// boundary is an unsplit CPML with kappa = 1 whose memory variables live only in strips.
//
// The stencils are bandwidth bound (well under 1 flop/byte), so there is no MFMA: each
// thread owns one cell (one node of every type), a wavefront covers 64 consecutive x, and
// neighbour reads are served by L1/L2. The adjoint kernels are the exact transposes of the
// forward sub-steps: material parameters sit inside the transposed differences, so they
// are separate kernels rather than the forward run backwards.
#include "efwi_internal.h"

// Contract a * b + c into one fused multiply-add only inside a single expression, never
// across statements: every template instance of a kernel then rounds the same source the
// same way, so runs that differ only in what they store stay bitwise identical.
#pragma clang fp contract(on)

namespace efwi {
namespace {

static_assert(BX == 64, "a wavefront must cover exactly one row of a block");

constexpr float K1 = 1.125f;              // 9/8
constexpr float K2 = -0.041666666666666664f;  // -1/24

// Strip slots (see Shot2D): x-strips
constexpr int X_VXX = 0, X_VZX = 1, X_XX = 2, X_XZ = 3;
// z-strips
constexpr int Z_VXZ = 0, Z_VZZ = 1, Z_ZZ = 2, Z_XZ = 3;

__device__ __forceinline__ const gfloat* axi(const Shot2D& s) { return s.prof; }
__device__ __forceinline__ const gfloat* bxi(const Shot2D& s) { return s.prof + s.nx; }
__device__ __forceinline__ const gfloat* axh(const Shot2D& s) { return s.prof + 2 * s.nx; }
__device__ __forceinline__ const gfloat* bxh(const Shot2D& s) { return s.prof + 3 * s.nx; }
__device__ __forceinline__ const gfloat* azi(const Shot2D& s) { return s.prof + 4 * s.nx; }
__device__ __forceinline__ const gfloat* bzi(const Shot2D& s) { return s.prof + 4 * s.nx + s.nz; }
__device__ __forceinline__ const gfloat* azh(const Shot2D& s) { return s.prof + 4 * s.nx + 2 * s.nz; }
__device__ __forceinline__ const gfloat* bzh(const Shot2D& s) { return s.prof + 4 * s.nx + 3 * s.nz; }

// Staged parameters at their own nodes, derived from lambda, mu and rho at the normal
// nodes (k_stage repeats the last row and column into the halo, so the averages clamp at
// the far edges): lambda + 2 mu; mu_xz, the harmonic mean of the four surrounding mu (0 if
// any is 0, since the reciprocal of 0 is infinite); b_x, b_z, the inverse of the arithmetic
// mean density of the two surrounding normal nodes. v_rcp_f32 (1 ulp); the forward and the
// transposed kernels evaluate the same expressions, so the transpose stays exact.
__device__ __forceinline__ float rcpf(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float l2m_of(const Shot2D& s, long o) { return s.lam[o] + 2.0f * s.mu[o]; }
__device__ __forceinline__ float bx_of(const Shot2D& s, long o) { return 2.0f * rcpf(s.rho[o] + s.rho[o + 1]); }
__device__ __forceinline__ float bz_of(const Shot2D& s, long o) { return 2.0f * rcpf(s.rho[o] + s.rho[o + s.ld]); }
__device__ __forceinline__ float muxz_of(const Shot2D& s, long o) {
  const long ld = s.ld;
  return 4.0f * rcpf(rcpf(s.mu[o]) + rcpf(s.mu[o + 1]) + rcpf(s.mu[o + ld]) + rcpf(s.mu[o + ld + 1]));
}

// Forward D+ at the half node after index k, and D- at integer node k (array index k holds
// the half node k+1/2); `st` is the element stride along the axis.
template <class P>
__device__ __forceinline__ float dplus(P f, long o, long st, float r) {
  return (K1 * (f[o + st] - f[o]) + K2 * (f[o + 2 * st] - f[o - st])) * r;
}
template <class P>
__device__ __forceinline__ float dminus(P f, long o, long st, float r) {
  return (K1 * (f[o] - f[o - st]) + K2 * (f[o + st] - f[o - 2 * st])) * r;
}

// Work decomposition. A launch covers the tiles of every shot of a batch: tiles are listed
// shot by shot, row band by row band (x fastest), and `tile_first[s]` is shot s's first
// tile. The hardware deals workgroup w to XCD (w mod 8); the host-built schedule gives
// XCD k one contiguous run of the tile list, cut so that every XCD gets the same weighted
// cost (tiles touching the CPML strips cost more), and workgroup w = k + 8 m takes the
// m-th tile of run k. Contiguous runs keep each stencil's z-halo rows in the XCD's own L2.
// Schedule entries of -1 pad the shorter runs.
constexpr int NXCD = 8;
template <int ROWS>
__device__ __forceinline__ bool batch_tile(const int* __restrict__ sched, const int* __restrict__ tile_shot,
                                           const int* __restrict__ tile_first, const Shot2D* __restrict__ shots,
                                           int& sh, int& i0, int& j0) {
  const int t = sched[blockIdx.x];
  if (t < 0) return false;
  sh = tile_shot[t];
  const int local = t - tile_first[sh];
  const int ntx = (shots[sh].nx + BX - 1) / BX;
  i0 = (local / ntx) * ROWS;
  j0 = (local % ntx) * BX;
  return true;
}

#define BATCH_PARAMS                                                                           \
  const Shot2D* __restrict__ shots, const int* __restrict__ tile_shot, const int* __restrict__ tile_first, \
      const int* __restrict__ sched
#define STEP_PARAMS BATCH_PARAMS
#define BATCH_TILE()                                                                           \
  int sh_, i0, j0;                                                                              \
  if (!batch_tile<BZ>(sched, tile_shot, tile_first, shots, sh_, i0, j0)) return;               \
  const Shot2D& s = shots[sh_]

// Does the tile of `rows` rows touch a CPML strip (with `pad` extra cells of neighbourhood)?
__device__ __forceinline__ bool block_in_pml(const Shot2D& s, int j0, int i0, int rows, int pad) {
  if (s.P <= 0) return false;
  const int j1 = j0 + BX - 1 + pad, i1 = i0 + rows - 1 + pad;
  return (j0 - pad < s.P) || (j1 >= s.nx - s.P) || (i0 - pad < s.P) || (i1 >= s.nz - s.P);
}

// Every cell function below issues all of its loads before its first store: the
// compiler cannot prove that the shot's arrays do not alias, so a store placed before a
// load would force another memory round trip per wavefront.

// ------------------------------------------------------------------------------------
// Fused forward time step n, eq.(1)-(3), on tiles of TZ rows x 64 columns. The forward
// state is double-buffered by step parity: buffer n & 1 holds sigma^n, v^{n-1/2} and the
// CPML memory variables, and the step writes buffer (n + 1) & 1, so no tile reads what
// another tile of the same launch writes. Per tile:
//   1. sigma^n of the tile and a 4-node halo is staged in LDS by one coalesced sweep;
//   2. velocity half step v^{n+1/2} = v^{n-1/2} + dt b div(sigma^n) on the tile and a
//      2-node halo, from LDS (halo nodes are recomputed rather than exchanged); owned
//      nodes go to HBM, all of them to LDS;
//   3. stress half step sigma^{n+1} = sigma^n + dt C (strain rate of v^{n+1/2}) on the
//      tile from the LDS velocities, with the moment-tensor injection at t_{n+1/2}
//      (eq.(2)) and the DAS strain record (eq.(3)).
// Each step reads sigma, v and the parameters once and writes sigma and v once, instead of
// re-reading sigma and v between two half-step kernels.
// ------------------------------------------------------------------------------------
template <int TZ>
struct StepTile {
  static_assert(TZ % BZ == 0, "tile rows must be a multiple of the block's rows");
  static constexpr int SR = TZ + 8, SC = BX + 8;  // sigma: rows i0-4 .. i0+TZ+3, columns j0-4 .. j0+67
  static constexpr int VR = TZ + 4, VC = BX + 4;  // velocity: rows i0-2 .. i0+TZ+1, columns j0-2 .. j0+65
  static constexpr int NS = 3 * SR * SC;
  static constexpr int LDS_FLOATS = NS + 2 * VR * VC;
};

// Uniform (scalar) base pointers of one fused step. Every per-lane index below is a
// non-negative 32-bit element offset from one of them, so an access is a scalar base plus
// a 32-bit lane offset rather than per-lane 64-bit address arithmetic.
struct StepPtrs {
  const gfloat *sxx, *szz, *sxz, *vx, *vz;   // buffer n & 1, padded plane origins
  gfloat *wsxx, *wszz, *wsxz, *wvx, *wvz;    // buffer (n + 1) & 1
  const gfloat *lam, *mu, *rho;              // staged parameters, padded plane origins
  const gfloat *rpx[4], *rpz[4];             // memory variables of buffer n & 1
  gfloat *wpx[4], *wpz[4];                   // and of buffer (n + 1) & 1
  const gfloat *axi, *bxi, *axh, *bxh, *azi, *bzi, *azh, *bzh;
  gfloat* seg;                               // this step's slot of the history (STORE)
  int ld, nx, nz, P2;                        // row pitch, window, strip width 2P
};

__device__ __forceinline__ StepPtrs step_ptrs(const Shot2D& s, int n, gfloat* seg) {
  StepPtrs p;
  const long org = (long)HALO * s.ld + XOFF;   // interior origin inside a padded plane
  const long rd = (long)(n & 1) * s.sbuf, wr = (long)((n + 1) & 1) * s.sbuf;
  p.sxx = s.sxx - org + rd;
  p.szz = s.szz - org + rd;
  p.sxz = s.sxz - org + rd;
  p.vx = s.vx - org + rd;
  p.vz = s.vz - org + rd;
  p.wsxx = s.sxx - org + wr;
  p.wszz = s.szz - org + wr;
  p.wsxz = s.sxz - org + wr;
  p.wvx = s.vx - org + wr;
  p.wvz = s.vz - org + wr;
  p.lam = s.lam - org;
  p.mu = s.mu - org;
  p.rho = s.rho - org;
  for (int k = 0; k < 4; ++k) {
    p.rpx[k] = s.psx[k] + rd;
    p.rpz[k] = s.psz[k] + rd;
    p.wpx[k] = s.psx[k] + wr;
    p.wpz[k] = s.psz[k] + wr;
  }
  p.axi = axi(s), p.bxi = bxi(s), p.axh = axh(s), p.bxh = bxh(s);
  p.azi = azi(s), p.bzi = bzi(s), p.azh = azh(s), p.bzh = bzh(s);
  p.seg = seg;
  p.ld = s.ld, p.nx = s.nx, p.nz = s.nz, p.P2 = 2 * s.P;
  return p;
}

// Offset of padded node (i, j), i >= -HALO, j >= -XOFF, from its plane origin.
__device__ __forceinline__ unsigned pofs(const StepPtrs& p, int i, int j) {
  return (unsigned)((i + HALO) * p.ld + XOFF + j);
}

// Element `e` of a global array as a 32-bit byte offset from a uniform base (the form the
// hardware's scalar-base global loads and stores take).
template <class P>
__device__ __forceinline__ auto& G(P* base, unsigned e) {
  typedef __attribute__((address_space(1))) char gchar;
  return *(P*)((gchar*)base + e * 4u);
}
template <class P>
__device__ __forceinline__ const auto& G(const P* base, unsigned e) {
  typedef const __attribute__((address_space(1))) char gchar;
  return *(const P*)((gchar*)base + e * 4u);
}

// Inputs of one velocity node (loads only).
struct VelLoads {
  float vx, vz, r0, rx, rz;
  float p1, p2, p3, p4;        // velocity-side memory variables (CPML tiles)
};

template <bool PML>
__device__ __forceinline__ VelLoads vel_loads(const StepPtrs& p, const Shot2D& s, int gi, int gj) {
  VelLoads L;
  const int ic = min(max(gi, 0), p.nz - 1), jc = min(max(gj, 0), p.nx - 1);
  const unsigned o = pofs(p, ic, jc);
  L.vx = G(p.vx, o);
  L.vz = G(p.vz, o);
  L.r0 = G(p.rho, o);
  L.rx = G(p.rho, o + 1);
  L.rz = G(p.rho, o + p.ld);
  L.p1 = L.p2 = L.p3 = L.p4 = 0.0f;
  if (PML) {
    const int sx = max(strip_index(jc, p.nx, s.P), 0), sz = max(strip_index(ic, p.nz, s.P), 0);
    const unsigned qx = (unsigned)(ic * p.P2 + sx), qz = (unsigned)(sz * p.nx + jc);
    L.p1 = G(p.rpx[X_VXX], qx);
    L.p3 = G(p.rpx[X_VZX], qx);
    L.p2 = G(p.rpz[Z_VXZ], qz);
    L.p4 = G(p.rpz[Z_VZZ], qz);
  }
  return L;
}

// Velocity node (gi, gj): the four stress differences d1 = D+x sxx, d2 = D-z sxz (vx) and
// d3 = D-x sxz, d4 = D+z szz (vz) come from LDS. Returns v^{n+1/2} (0 outside the grid);
// with `owned`, writes v, the memory variables and the stored divergences.
template <bool STORE, bool PML>
__device__ __forceinline__ void vel_node(const StepPtrs& p, const Shot2D& s, int gi, int gj, bool owned,
                                         const VelLoads& L, float d1, float d2, float d3, float d4, float& vxn,
                                         float& vzn) {
  const bool in = gi >= 0 && gi < p.nz && gj >= 0 && gj < p.nx;
  int sx = -1, sz = -1;
  float p1 = 0.0f, p2 = 0.0f, p3 = 0.0f, p4 = 0.0f;
  if (PML) {
    const int ic = min(max(gi, 0), p.nz - 1), jc = min(max(gj, 0), p.nx - 1);
    sx = strip_index(jc, p.nx, s.P);
    sz = strip_index(ic, p.nz, s.P);
    p1 = G(p.bxh, jc) * L.p1 + G(p.axh, jc) * d1;
    p3 = G(p.bxi, jc) * L.p3 + G(p.axi, jc) * d3;
    p2 = G(p.bzi, ic) * L.p2 + G(p.azi, ic) * d2;
    p4 = G(p.bzh, ic) * L.p4 + G(p.azh, ic) * d4;
    if (sx >= 0) {
      d1 += p1;
      d3 += p3;
    }
    if (sz >= 0) {
      d2 += p2;
      d4 += p4;
    }
  }
  const float qx = d1 + d2, qz = d3 + d4;
  const float bx = 2.0f * rcpf(L.r0 + L.rx), bz = 2.0f * rcpf(L.r0 + L.rz);
  const float m = in ? 1.0f : 0.0f;
  vxn = m * (L.vx + s.dt * bx * qx);
  vzn = m * (L.vz + s.dt * bz * qz);
  if (owned) {
    const unsigned o = pofs(p, gi, gj);
    G(p.wvx, o) = vxn;
    G(p.wvz, o) = vzn;
    if (PML) {
      if (sx >= 0) {
        const unsigned q = (unsigned)(gi * p.P2 + sx);
        G(p.wpx[X_VXX], q) = p1;
        G(p.wpx[X_VZX], q) = p3;
      }
      if (sz >= 0) {
        const unsigned q = (unsigned)(sz * p.nx + gj);
        G(p.wpz[Z_VXZ], q) = p2;
        G(p.wpz[Z_VZZ], q) = p4;
      }
    }
    if (STORE) {  // divergences times b/2: the rho imaging terms (d b / d rho = -b^2/2)
      const unsigned c = (unsigned)(gi * s.cp + gj);
      G(p.seg, 3 * s.cells + c) = 0.5f * qx * bx;
      G(p.seg, 4 * s.cells + c) = 0.5f * qz * bz;
    }
  }
}

// Inputs of one stress node (loads only; the DAS channel, in the rare channel rows, is
// looked up in str_node).
struct StrLoads {
  float lam, mu, mu_x, mu_z, mu_xz;
  float p1, p2, p3, p4;        // stress-side memory variables (CPML tiles)
};

template <bool PML>
__device__ __forceinline__ StrLoads str_loads(const StepPtrs& p, const Shot2D& s, int gi, int gj) {
  StrLoads L;
  const int ic = min(gi, p.nz - 1), jc = min(gj, p.nx - 1);
  const unsigned o = pofs(p, ic, jc);
  L.lam = G(p.lam, o);
  L.mu = G(p.mu, o);
  L.mu_x = G(p.mu, o + 1);
  L.mu_z = G(p.mu, o + p.ld);
  L.mu_xz = G(p.mu, o + p.ld + 1);
  L.p1 = L.p2 = L.p3 = L.p4 = 0.0f;
  if (PML) {
    const int sx = max(strip_index(jc, p.nx, s.P), 0), sz = max(strip_index(ic, p.nz, s.P), 0);
    const unsigned qx = (unsigned)(ic * p.P2 + sx), qz = (unsigned)(sz * p.nx + jc);
    L.p1 = G(p.rpx[X_XX], qx);
    L.p2 = G(p.rpx[X_XZ], qx);
    L.p3 = G(p.rpz[Z_ZZ], qz);
    L.p4 = G(p.rpz[Z_XZ], qz);
  }
  return L;
}

// Stress node (i, j) from the LDS strain rates pxx = D-x vx, pzz = D-z vz, pzx = D+z vx,
// pxz = D+x vz and the LDS sigma^n.
template <bool STORE, bool RECORD, bool PML>
__device__ __forceinline__ void str_node(const StepPtrs& p, const Shot2D& s, int i, int j, int n, const StrLoads& L,
                                         int slot, float pxx, float pzz, float pzx, float pxz, float sxx, float szz,
                                         float sxz, float f_xx, float f_zz, float f_xz) {
  const float raw_pxx = pxx;
  const float mu = L.mu, lam = L.lam, l2m = lam + 2.0f * mu;
  const float mxz = 4.0f * rcpf(rcpf(mu) + rcpf(L.mu_x) + rcpf(L.mu_z) + rcpf(L.mu_xz));
  int sx = -1, sz = -1;
  float p1 = 0.0f, p2 = 0.0f, p3 = 0.0f, p4 = 0.0f;
  if (PML) {
    sx = strip_index(j, p.nx, s.P);
    sz = strip_index(i, p.nz, s.P);
    p1 = G(p.bxi, j) * L.p1 + G(p.axi, j) * pxx;
    p2 = G(p.bxh, j) * L.p2 + G(p.axh, j) * pxz;
    p3 = G(p.bzi, i) * L.p3 + G(p.azi, i) * pzz;
    p4 = G(p.bzh, i) * L.p4 + G(p.azh, i) * pzx;
    if (sx >= 0) {
      pxx += p1;
      pxz += p2;
    }
    if (sz >= 0) {
      pzz += p3;
      pzx += p4;
    }
  }
  const float ps = pzx + pxz;
  sxx += s.dt * (l2m * pxx + lam * pzz);
  szz += s.dt * (lam * pxx + l2m * pzz);
  sxz += s.dt * mxz * ps;
  if (i == s.si && j == s.sj) {
    sxx -= s.w * f_xx;
    szz -= s.w * f_zz;
  }
  if ((i == s.si || i == s.si - 1) && (j == s.sj || j == s.sj - 1)) sxz -= 0.25f * s.w * f_xz;
  if (PML) {
    if (sx >= 0) {
      const unsigned q = (unsigned)(i * p.P2 + sx);
      G(p.wpx[X_XX], q) = p1;
      G(p.wpx[X_XZ], q) = p2;
    }
    if (sz >= 0) {
      const unsigned q = (unsigned)(sz * p.nx + j);
      G(p.wpz[Z_ZZ], q) = p3;
      G(p.wpz[Z_XZ], q) = p4;
    }
  }
  const unsigned o = pofs(p, i, j);
  G(p.wsxx, o) = sxx;
  G(p.wszz, o) = szz;
  G(p.wsxz, o) = sxz;
  if (RECORD && slot >= 0) {  // slot: the row's DAS slot, uniform over the wavefront
    const int ch = s.rowch[(long)slot * s.nx + j];
    if (ch >= 0) {
      const float e = s.e[ch] + s.dt * raw_pxx;
      s.e[ch] = e;
      s.d[(long)ch * s.nt + n] = e;
    }
  }
  if (STORE) {  // strain rates times the factors of the lambda and mu imaging terms
    const unsigned c = (unsigned)(i * s.cp + j);
    G(p.seg, c) = (pxx + pzz) / (l2m + lam);
    G(p.seg, s.cells + c) = 0.5f * (pxx - pzz) * mu;
    G(p.seg, 2 * s.cells + c) = 0.25f * ps * mxz;
  }
}

template <int TZ, bool STORE, bool RECORD, bool PML>
__device__ __forceinline__ void fwd_step_tile(const Shot2D& s, int i0, int j0, int n, gfloat* seg, float* lds) {
  using T = StepTile<TZ>;
  constexpr int SR = T::SR, SC = T::SC, VR = T::VR, VC = T::VC, NS = T::NS;
  constexpr int NT = BX * BZ;
  constexpr int NV = VR / BZ, NSR = TZ / BZ;
  constexpr int Q = SC / 4;                         // float4 per staged row
  constexpr int NQ = 3 * SR * Q;
  constexpr int PER = (NQ + NT - 1) / NT;           // float4 loads per thread
  static_assert(SC % 4 == 0, "staged rows are whole float4s");
  typedef float f4 __attribute__((ext_vector_type(4)));
  const StepPtrs p = step_ptrs(s, n, seg);
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * BX + tx;
  const int tyu = __builtin_amdgcn_readfirstlane(ty);   // a wavefront's row is uniform
  float* SXX = lds;
  float* SZZ = lds + SR * SC;
  float* SXZ = lds + 2 * SR * SC;
  float* VXL = lds + NS;
  float* VZL = VXL + VR * VC;
  const int hv = min(tid >> 2, VR - 1), hc = tid & 3;
  const int hcol = hc < 2 ? hc : VC - 4 + hc;      // LDS velocity column 0, 1, 66, 67

  // ---- every global load of the tile, issued before the first LDS write ----
  int slot[NSR];                                    // DAS slots of the thread's stress rows
#pragma unroll
  for (int k = 0; k < NSR; ++k) slot[k] = RECORD ? s.row_slot[min(i0 + tyu + k * BZ, p.nz - 1)] : -1;
  // sigma^n of the tile and a 4-node halo, zero outside the grid: rows are clamped into the
  // grid (the masked values of a clamped row are discarded) and a float4 that crosses the
  // right edge reads the row's zero padding or the halo rows below it
  // thread tid takes float4 e = tid + k NT, i.e. (field f, row r, float4 c4) of the
  // [3][SR][Q] staging area, advanced by NT = 256 float4s per k without divisions
  constexpr int DC = NT % Q, DR = (NT / Q) % SR, DF = NT / (SR * Q);
  static_assert(DF == 0, "one step of NT float4s stays inside a field's staging area");
  int sf[PER], sr_[PER], sc4[PER];
  {
    int f = tid / (SR * Q), rem = tid - f * (SR * Q);
    int r = rem / Q, c4 = rem - r * Q;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      sf[k] = f, sr_[k] = r, sc4[k] = c4;
      c4 += DC;
      r += DR;
      if (c4 >= Q) c4 -= Q, ++r;
      if (r >= SR) r -= SR, ++f;
    }
  }
  f4 sv[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int f = min(sf[k], 2);   // past the last field only when e >= NQ: load a valid float4
    const int ic = min(max(i0 - 4 + sr_[k], 0), p.nz - 1);
    const gfloat* src = f == 0 ? p.sxx : f == 1 ? p.szz : p.sxz;
    typedef const __attribute__((address_space(1))) char gchar;
    sv[k] = *(const __attribute__((address_space(1))) f4*)((gchar*)src + pofs(p, ic, j0 - 4 + 4 * sc4[k]) * 4u);
  }
  VelLoads L[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) L[k] = vel_loads<PML>(p, s, i0 - 2 + ty + k * BZ, j0 + tx);
  const VelLoads H = vel_loads<PML>(p, s, i0 - 2 + hv, j0 - 2 + hcol);
  StrLoads SL[NSR];
#pragma unroll
  for (int k = 0; k < NSR; ++k) SL[k] = str_loads<PML>(p, s, i0 + tyu + k * BZ, j0 + tx);
  const float f_xx = s.src[n], f_zz = s.src[s.nt + n], f_xz = s.src[2 * s.nt + n];

  // ---- 1. staged sigma to LDS ----
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    if (sf[k] < 3) {
      const int f = sf[k], r = sr_[k], c4 = sc4[k];
      const int gi = i0 - 4 + r, gj = j0 - 4 + 4 * c4;
      const bool row_in = gi >= 0 && gi < p.nz;
      f4 v;
      v.x = (row_in && gj + 0 >= 0 && gj + 0 < p.nx) ? sv[k].x : 0.0f;
      v.y = (row_in && gj + 1 >= 0 && gj + 1 < p.nx) ? sv[k].y : 0.0f;
      v.z = (row_in && gj + 2 >= 0 && gj + 2 < p.nx) ? sv[k].z : 0.0f;
      v.w = (row_in && gj + 3 >= 0 && gj + 3 < p.nx) ? sv[k].w : 0.0f;
      *(f4*)(lds + f * SR * SC + r * SC + 4 * c4) = v;
    }
  }
  __syncthreads();

  // ---- 2. velocities: the 64 tile columns over VR rows (thread row ty, ty + 4, ...), then
  //         the four halo columns j0-2, j0-1, j0+64, j0+65 (threads 0 .. 4 VR - 1) ----
  auto vel = [&](int vr, int lcol, const VelLoads& LL, bool owned) {
    const int gi = i0 - 2 + vr, gj = j0 - 2 + lcol;
    const int sr = vr + 2, sc = lcol + 2;   // LDS sigma coordinates of the node
    const float d1 = (K1 * (SXX[sr * SC + sc + 1] - SXX[sr * SC + sc]) +
                      K2 * (SXX[sr * SC + sc + 2] - SXX[sr * SC + sc - 1])) * s.rdx;
    const float d2 = (K1 * (SXZ[sr * SC + sc] - SXZ[(sr - 1) * SC + sc]) +
                      K2 * (SXZ[(sr + 1) * SC + sc] - SXZ[(sr - 2) * SC + sc])) * s.rdz;
    const float d3 = (K1 * (SXZ[sr * SC + sc] - SXZ[sr * SC + sc - 1]) +
                      K2 * (SXZ[sr * SC + sc + 1] - SXZ[sr * SC + sc - 2])) * s.rdx;
    const float d4 = (K1 * (SZZ[(sr + 1) * SC + sc] - SZZ[sr * SC + sc]) +
                      K2 * (SZZ[(sr + 2) * SC + sc] - SZZ[(sr - 1) * SC + sc])) * s.rdz;
    float vxn, vzn;
    vel_node<STORE, PML>(p, s, gi, gj, owned, LL, d1, d2, d3, d4, vxn, vzn);
    VXL[vr * VC + lcol] = vxn;
    VZL[vr * VC + lcol] = vzn;
  };
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int vr = ty + k * BZ, gi = i0 - 2 + vr;
    vel(vr, tx + 2, L[k], gi >= i0 && gi < i0 + TZ && gi < p.nz && j0 + tx < p.nx);
  }
  if ((tid >> 2) < VR) vel(hv, hcol, H, false);
  __syncthreads();

  // ---- 3. stresses of the tile ----
#pragma unroll
  for (int k = 0; k < NSR; ++k) {
    const int i = i0 + tyu + k * BZ, j = j0 + tx;
    if (i >= p.nz || j >= p.nx) continue;
    const int vr = tyu + k * BZ + 2, vc = tx + 2;   // LDS velocity coordinates of the node
    const float* X = VXL + vr * VC + vc;
    const float* Z = VZL + vr * VC + vc;
    const float pxx = (K1 * (X[0] - X[-1]) + K2 * (X[1] - X[-2])) * s.rdx;
    const float pzz = (K1 * (Z[0] - Z[-VC]) + K2 * (Z[VC] - Z[-2 * VC])) * s.rdz;
    const float pzx = (K1 * (X[VC] - X[0]) + K2 * (X[2 * VC] - X[-VC])) * s.rdz;
    const float pxz = (K1 * (Z[1] - Z[0]) + K2 * (Z[2] - Z[-1])) * s.rdx;
    const int so = (vr + 2) * SC + tx + 4;           // LDS sigma of the node
    str_node<STORE, RECORD, PML>(p, s, i, j, n, SL[k], slot[k], pxx, pzz, pzx, pxz, SXX[so], SZZ[so], SXZ[so],
                                 f_xx, f_zz, f_xz);
  }
}

// Tile shape of the fused forward step: TSTEP rows x 64 columns.
template <int TZ, bool STORE, bool RECORD>
__global__ __launch_bounds__(BX * BZ) void k_fwd_step(STEP_PARAMS, int n, int kstore) {
  __shared__ float lds[StepTile<TZ>::LDS_FLOATS];
  int sh_, i0, j0;
  if (!batch_tile<TZ>(sched, tile_shot, tile_first, shots, sh_, i0, j0)) return;
  const Shot2D& s = shots[sh_];
  gfloat* seg = STORE ? s.seg + (size_t)kstore * NSEG_FIELDS * s.cells : nullptr;
  // block-uniform branch: every thread reaches the barriers
  if (block_in_pml(s, j0, i0, TZ, 2)) fwd_step_tile<TZ, STORE, RECORD, true>(s, i0, j0, n, seg, lds);
  else fwd_step_tile<TZ, STORE, RECORD, false>(s, i0, j0, n, seg, lds);
}

// ------------------------------------------------------------------------------------
// Adjoint (exact transpose) in scaled variables.
//
// With sigma_bar the adjoint of sigma^{n+1} and v_bar the adjoint of v^{n+1/2}, the
// transposed sub-steps of step n are (reverse order of the forward):
//   DAS:      v_bar_x += dt (D-x)^T e_bar at the channels, e_bar = sum_{k>=n} r[:, k]
//   stress:   p_bar = dt C sigma_bar (+ CPML transpose), v_bar += D^T p_bar
//   velocity: q_bar = dt b v_bar (+ CPML transpose),     sigma_bar += D^T q_bar
// Carrying u_bar = b v_bar and t_bar = C sigma_bar instead, p_bar~ = dt t_bar and
// q_bar~ = dt u_bar are read straight from the neighbours (no material parameters there),
// and the parameters act only on the owned node: u_bar += b D^T p_bar,
// t_bar += C D^T q_bar. D^T uses D-^T = -D+ and D+^T = -D- (zero outside the grid).
// CPML transpose of psi <- b psi + a D, D~ = D + psi: psi_bar += y_bar; x_bar = y_bar +
// a psi_bar; psi_bar <- b psi_bar (double-buffered: neighbours read the old value).
// Imaging (the adjoint-state correlations of eq.(6)), gathered at the normal node (i, j)
// from the stored forward quantities h0..h4 (see NSEG_FIELDS) into three sums:
//   A += dt (t_xx + t_zz) h0                                    g_lambda
//   E += dt [(t_xx - t_zz) h1 + sum_k c_k t_xz(k) h2(k)]        mu^2 g_mu
//   R -= dt [sum_b c_b u_x(b) h3(b) + sum_a c_a u_z(a) h4(a)]   g_rho through b_x, b_z
// over the four shear nodes k and the two vx nodes b and two vz nodes a whose staged
// value uses mu(i, j) or rho(i, j), c counting how often (twice at a clamped edge).
// With t = C sigma_bar, t_xx + t_zz = 2(l+m)(s_xx + s_zz) and t_xx - t_zz = 2m(s_xx - s_zz);
// d mu_xz / d mu = mu_xz^2 / (4 mu^2) per corner and d b / d rho = -b^2 / 2, so the chain
// rule at the end of each block of steps needs only g_mu = A + E / mu^2 and R.
// ------------------------------------------------------------------------------------

// How often the shear node (a, b) (harmonic mean over the clamped corners (a, b),
// (a+1, b), (a, b+1), (a+1, b+1)) uses the normal node (i, j).
__device__ __forceinline__ int corner_count(int a, int b, int i, int j, int nz, int nx) {
  if (a < 0 || b < 0) return 0;
  const int ap = min(a + 1, nz - 1), bp = min(b + 1, nx - 1);
  return (a == i && b == j) + (ap == i && b == j) + (a == i && bp == j) + (ap == i && bp == j);
}
// How often the velocity node between k and k+1 (clamped) uses node m along that axis.
__device__ __forceinline__ int pair_count(int k, int m, int n) {
  if (k < 0) return 0;
  return (k == m) + (min(k + 1, n - 1) == m);
}

// ------------------------------------------------------------------------------------
template <bool PML>
struct AdjCtx {
  const Shot2D& s;
  int rd;                   // which buffer of the adjoint memory variables holds step n+1
};

// Corrected transposed operands at node (ii, jj); `a` is the profile coefficient for the
// node's coordinate along the derivative's axis and `psi` the matching adjoint memory
// variable, used only inside the CPML strips.
template <bool PML>
__device__ __forceinline__ float corr_x(const AdjCtx<PML>& c, float v, int ii, int jj, const gfloat* aprof, int slot) {
  const Shot2D& s = c.s;
  if (PML && ii >= 0 && ii < s.nz && jj >= 0 && jj < s.nx) {
    const int sx = strip_index(jj, s.nx, s.P);
    if (sx >= 0) v += aprof[jj] * (s.pbx[c.rd][slot][(long)ii * 2 * s.P + sx] + v);
  }
  return v;
}
template <bool PML>
__device__ __forceinline__ float corr_z(const AdjCtx<PML>& c, float v, int ii, int jj, const gfloat* aprof, int slot) {
  const Shot2D& s = c.s;
  if (PML && ii >= 0 && ii < s.nz && jj >= 0 && jj < s.nx) {
    const int sz = strip_index(ii, s.nz, s.P);
    if (sz >= 0) v += aprof[ii] * (s.pbz[c.rd][slot][(long)sz * s.nx + jj] + v);
  }
  return v;
}

// p_bar for pxx (x int, X_XX), pzz (z int, Z_ZZ), pzx (z half, Z_XZ), pxz (x half, X_XZ)
template <bool PML>
__device__ __forceinline__ float pb_xx(const AdjCtx<PML>& c, int ii, int jj) {
  return corr_x(c, c.s.dt * c.s.txxb[(long)ii * c.s.ld + jj], ii, jj, axi(c.s), X_XX);
}
template <bool PML>
__device__ __forceinline__ float pb_zz(const AdjCtx<PML>& c, int ii, int jj) {
  return corr_z(c, c.s.dt * c.s.tzzb[(long)ii * c.s.ld + jj], ii, jj, azi(c.s), Z_ZZ);
}
template <bool PML>
__device__ __forceinline__ float pb_zx(const AdjCtx<PML>& c, int ii, int jj) {
  return corr_z(c, c.s.dt * c.s.txzb[(long)ii * c.s.ld + jj], ii, jj, azh(c.s), Z_XZ);
}
template <bool PML>
__device__ __forceinline__ float pb_xz(const AdjCtx<PML>& c, int ii, int jj) {
  return corr_x(c, c.s.dt * c.s.txzb[(long)ii * c.s.ld + jj], ii, jj, axh(c.s), X_XZ);
}
// q_bar for qx with D+x sxx (x half, X_VXX), with D-z sxz (z int, Z_VXZ);
// for qz with D-x sxz (x int, X_VZX), with D+z szz (z half, Z_VZZ)
template <bool PML>
__device__ __forceinline__ float qb_xa(const AdjCtx<PML>& c, int ii, int jj) {
  return corr_x(c, c.s.dt * c.s.uxb[(long)ii * c.s.ld + jj], ii, jj, axh(c.s), X_VXX);
}
template <bool PML>
__device__ __forceinline__ float qb_xb(const AdjCtx<PML>& c, int ii, int jj) {
  return corr_z(c, c.s.dt * c.s.uxb[(long)ii * c.s.ld + jj], ii, jj, azi(c.s), Z_VXZ);
}
template <bool PML>
__device__ __forceinline__ float qb_za(const AdjCtx<PML>& c, int ii, int jj) {
  return corr_x(c, c.s.dt * c.s.uzb[(long)ii * c.s.ld + jj], ii, jj, axi(c.s), X_VZX);
}
template <bool PML>
__device__ __forceinline__ float qb_zb(const AdjCtx<PML>& c, int ii, int jj) {
  return corr_z(c, c.s.dt * c.s.uzb[(long)ii * c.s.ld + jj], ii, jj, azh(c.s), Z_VZZ);
}

__device__ __forceinline__ float ebar_at(const Shot2D& s, int slot, int jc, int n) {
  if (jc < 0 || jc >= s.nx) return 0.0f;
  const int c = s.rowch[(long)slot * s.nx + jc];
  return c >= 0 ? s.ebar[(long)n * s.nch + c] : 0.0f;
}

// CPML tiles stage the corrected transposed operands of the tile and its halo in LDS, so
// each node's correction (strip test, profile, adjoint memory variable) is computed once
// instead of once per neighbour that reads it. Four operands, each over the tile rows or
// columns it is differentiated along: x-operands cover columns [j0 + lo, j0 + 64 + hi] of
// the 4 tile rows, z-operands rows [i0 + lo, i0 + 4 + hi] of the 64 tile columns.
constexpr int LX = BX + 3;      // 67 columns (x-operands)
constexpr int LZ = BZ + 3;      // 7 rows (z-operands)
constexpr int LDS_OPS = 2 * BZ * LX + 2 * LZ * BX;

struct StageArea {
  float* x0;  // [BZ][LX]
  float* x1;  // [BZ][LX]
  float* z0;  // [LZ][BX]
  float* z1;  // [LZ][BX]
};

// One staged operand: dt * f at the nodes of its patch, plus, inside the CPML strips of its
// axis, a * (psi + dt * f) with the profile coefficient a of the node's coordinate and the
// adjoint memory variable psi. x-operands cover (i0 + r, j0 + c + lo), r < BZ, c < LX;
// z-operands (i0 + r + lo, j0 + c), r < LZ, c < BX. Nodes outside the grid hold zero.
struct StagedOp {
  const gfloat* f;
  const gfloat* a;
  const gfloat* psi;
  int lo;
};

// Every thread takes at most two nodes of each operand: all loads are issued before the
// first LDS write, so a tile costs one memory round trip.
template <bool XAXIS>
__device__ __forceinline__ void stage_load(const Shot2D& s, int i0, int j0, const StagedOp& op, int tid, float* v) {
  constexpr int N = XAXIS ? BZ * LX : LZ * BX;
  constexpr int W = XAXIS ? LX : BX;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int e = tid + k * BX * BZ;
    const int r = e / W, c = e % W;
    const int ii = i0 + r + (XAXIS ? 0 : op.lo), jj = j0 + c + (XAXIS ? op.lo : 0);
    // clamped indices keep every load valid and unconditional (no waits inside branches)
    const bool in = e < N && ii >= 0 && ii < s.nz && jj >= 0 && jj < s.nx;
    const int ic = min(max(ii, 0), s.nz - 1), jc = min(max(jj, 0), s.nx - 1);
    const int sidx = XAXIS ? strip_index(jc, s.nx, s.P) : strip_index(ic, s.nz, s.P);
    const int sc = max(sidx, 0);
    const float f = op.f[(long)ic * s.ld + jc];
    const float ps = XAXIS ? op.psi[(long)ic * 2 * s.P + sc] : op.psi[(long)sc * s.nx + jc];
    const float ac = op.a[XAXIS ? jc : ic];
    // 0/1 masks instead of branches keep the loads unconditional (the compiler would sink
    // loads used on one side of a select into a branch and wait there)
    const float m_in = in ? 1.0f : 0.0f, m_strip = sidx >= 0 ? 1.0f : 0.0f;
    const float val = s.dt * f;
    v[k] = m_in * (val + (m_strip * ac) * (ps + val));
  }
}
template <bool XAXIS>
__device__ __forceinline__ void stage_store(float* dst, int tid, const float* v) {
  constexpr int N = XAXIS ? BZ * LX : LZ * BX;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int e = tid + k * BX * BZ;
    if (e < N) dst[e] = v[k];
  }
}
// Stage the two x-operands and the two z-operands of a CPML tile.
__device__ __forceinline__ void stage_operands(const Shot2D& s, int i0, int j0, StageArea a, const StagedOp& x0,
                                               const StagedOp& x1, const StagedOp& z0, const StagedOp& z1) {
  static_assert(BZ * LX <= 2 * BX * BZ && LZ * BX <= 2 * BX * BZ, "two nodes per thread and operand");
  const int tid = threadIdx.y * BX + threadIdx.x;
  float v0[2], v1[2], v2[2], v3[2];
  stage_load<true>(s, i0, j0, x0, tid, v0);
  stage_load<true>(s, i0, j0, x1, tid, v1);
  stage_load<false>(s, i0, j0, z0, tid, v2);
  stage_load<false>(s, i0, j0, z1, tid, v3);
  stage_store<true>(a.x0, tid, v0);
  stage_store<true>(a.x1, tid, v1);
  stage_store<false>(a.z0, tid, v2);
  stage_store<false>(a.z1, tid, v3);
}

// Transposed stress sub-step (first at reverse step n): t_bar -> u_bar.
// ux, uz, wz, wx are the four transposed differences: D+x p_bar_xx, D-z p_bar_zx,
// D+z p_bar_zz and D-x p_bar_xz at the cell's velocity nodes (without 1/h).
template <bool GRAD, bool SRCADJ, bool PML>
__device__ __forceinline__ void adj_vel_finish(const Shot2D& s, int i, int j, int n, const gfloat* seg, bool first,
                                               float ux, float uz, float wz, float wx) {
  const long ld = s.ld;
  const long o = (long)i * ld + j;
  const int rd = (n + 1) & 1, wr = n & 1;
  // ---- loads ----
  const int slot = s.row_slot[i];  // DAS row slot (depends on the wavefront's row only)
  const float txx = s.txxb[o], tzz = s.tzzb[o], txz = s.txzb[o];
  const float u0x = s.uxb[o], u0z = s.uzb[o], bx = bx_of(s, o), bz = bz_of(s, o);
  int sx = -1, sz = -1;
  long qx_ = 0, qz_ = 0;
  float r1 = 0.0f, r2 = 0.0f, r3 = 0.0f, r4 = 0.0f;
  if (PML) {  // owned adjoint memory variables of the stress-side derivatives
    sx = strip_index(j, s.nx, s.P);
    sz = strip_index(i, s.nz, s.P);
    qx_ = (long)i * 2 * s.P + max(sx, 0);
    qz_ = (long)max(sz, 0) * s.nx + j;
    r1 = bxi(s)[j] * (s.pbx[rd][X_XX][qx_] + s.dt * txx);
    r2 = bxh(s)[j] * (s.pbx[rd][X_XZ][qx_] + s.dt * txz);
    r3 = bzi(s)[i] * (s.pbz[rd][Z_ZZ][qz_] + s.dt * tzz);
    r4 = bzh(s)[i] * (s.pbz[rd][Z_XZ][qz_] + s.dt * txz);
  }
  long cc = 0;
  float a0 = 0.0f, a1 = 0.0f, e = 0.0f, h0 = 0.0f;
  if (GRAD) {
    cc = (long)i * s.cp + j;
    const gfloat* h2 = seg + 2 * s.cells;
    h0 = seg[cc];
    e = (txx - tzz) * seg[s.cells + cc];
    // shear nodes (a, b), a in {i-1, i}, b in {j-1, j}; indices clamped so every load is
    // valid and issued up front, with weight 0 where the node does not use mu(i, j)
    for (int a = i - 1; a <= i; ++a) {
      for (int b = j - 1; b <= j; ++b) {
        const float c = (float)corner_count(a, b, i, j, s.nz, s.nx);
        const int aa = max(a, 0), bb = max(b, 0);
        e += c * s.txzb[(long)aa * ld + bb] * h2[(long)aa * s.cp + bb];
      }
    }
    if (!first) {
      a0 = s.acc[cc];
      a1 = s.acc[s.cells + cc];
    }
  }
  // DAS transpose: the channel at normal node jc feeds vx nodes jc (c1), jc-1 (-c1),
  // jc+1 (c2) and jc-2 (-c2) of its row
  float inj = 0.0f;
  if (slot >= 0)
    inj = K1 * (ebar_at(s, slot, j, n) - ebar_at(s, slot, j + 1, n)) +
          K2 * (ebar_at(s, slot, j - 1, n) - ebar_at(s, slot, j + 2, n));
  float sb0 = 0.0f, sb1 = 0.0f, sb2 = 0.0f;
  const bool at_src = SRCADJ && i == s.si && j == s.sj;
  if (at_src) {
    // sigma_bar at the source from t_bar: invert the 2x2 normal block and the shear moduli
    const float lam = s.lam[o], l2m = l2m_of(s, o);
    const float det = (l2m - lam) * (l2m + lam);
    sb0 = (l2m * txx - lam * tzz) / det;
    sb1 = (l2m * tzz - lam * txx) / det;
    auto sxz_at = [&](long oo) {
      const float m = muxz_of(s, oo);
      return m > 0.0f ? s.txzb[oo] / m : 0.0f;
    };
    sb2 = sxz_at(o) + sxz_at(o - 1) + sxz_at(o - ld) + sxz_at(o - ld - 1);
  }
  // ---- arithmetic ----
  // v_bar_x += -(D+x p_bar_xx + D-z p_bar_zx); v_bar_z += -(D+z p_bar_zz + D-x p_bar_xz)
  const float gx = -(ux * s.rdx + uz * s.rdz) + s.dt * s.rdx * inj;
  const float gz = -(wz * s.rdz + wx * s.rdx);
  // ---- stores ----
  if (PML) {
    if (sx >= 0) {
      s.pbx[wr][X_XX][qx_] = r1;
      s.pbx[wr][X_XZ][qx_] = r2;
    }
    if (sz >= 0) {
      s.pbz[wr][Z_ZZ][qz_] = r3;
      s.pbz[wr][Z_XZ][qz_] = r4;
    }
  }
  s.uxb[o] = u0x + bx * gx;
  s.uzb[o] = u0z + bz * gz;
  if (GRAD) {
    s.acc[cc] = a0 + s.dt * (txx + tzz) * h0;
    s.acc[s.cells + cc] = a1 + s.dt * e;
  }
  if (at_src) {
    s.src_bar[n] = -s.w * sb0;
    s.src_bar[s.nt + n] = -s.w * sb1;
    s.src_bar[2 * s.nt + n] = -0.25f * s.w * sb2;
  }
}

template <bool GRAD, bool SRCADJ>
__global__ __launch_bounds__(BX * BZ) void k_adj_vel(BATCH_PARAMS, int n, int k, int first) {
  BATCH_TILE();
  // all 64 lanes of a wavefront share threadIdx.y: keep the row index scalar
  const int j = j0 + threadIdx.x, i = i0 + __builtin_amdgcn_readfirstlane(threadIdx.y);
  const gfloat* seg = GRAD ? s.seg + (size_t)k * NSEG_FIELDS * s.cells : nullptr;
  const bool active = i < s.nz && j < s.nx;
  if (block_in_pml(s, j0, i0, BZ, 2)) {  // block-uniform: every thread reaches the barrier
    __shared__ float lds[LDS_OPS];
    const StageArea a{lds, lds + BZ * LX, lds + 2 * BZ * LX, lds + 2 * BZ * LX + LZ * BX};
    const int rd = (n + 1) & 1;
    // x0: p_bar_xx at columns j-1 .. j+2; x1: p_bar_xz at j-2 .. j+1;
    // z0: p_bar_zx at rows i-2 .. i+1;     z1: p_bar_zz at i-1 .. i+2
    stage_operands(s, i0, j0, a, StagedOp{s.txxb, axi(s), s.pbx[rd][X_XX], -1},
                   StagedOp{s.txzb, axh(s), s.pbx[rd][X_XZ], -2}, StagedOp{s.txzb, azh(s), s.pbz[rd][Z_XZ], -2},
                   StagedOp{s.tzzb, azi(s), s.pbz[rd][Z_ZZ], -1});
    __syncthreads();
    if (!active) return;
    const int r = threadIdx.y, q = threadIdx.x;
    const float* X0 = a.x0 + r * LX + q;   // X0[m] = p_bar_xx(i, j - 1 + m)
    const float* X1 = a.x1 + r * LX + q;   // X1[m] = p_bar_xz(i, j - 2 + m)
    const float* Z0 = a.z0 + r * BX + q;   // Z0[m BX] = p_bar_zx(i - 2 + m, j)
    const float* Z1 = a.z1 + r * BX + q;   // Z1[m BX] = p_bar_zz(i - 1 + m, j)
    const float ux = K1 * (X0[2] - X0[1]) + K2 * (X0[3] - X0[0]);
    const float uz = K1 * (Z0[2 * BX] - Z0[BX]) + K2 * (Z0[3 * BX] - Z0[0]);
    const float wz = K1 * (Z1[2 * BX] - Z1[BX]) + K2 * (Z1[3 * BX] - Z1[0]);
    const float wx = K1 * (X1[2] - X1[1]) + K2 * (X1[3] - X1[0]);
    adj_vel_finish<GRAD, SRCADJ, true>(s, i, j, n, seg, first != 0, ux, uz, wz, wx);
  } else if (active) {
    const AdjCtx<false> c{s, 0};
    const float ux = K1 * (pb_xx(c, i, j + 1) - pb_xx(c, i, j)) + K2 * (pb_xx(c, i, j + 2) - pb_xx(c, i, j - 1));
    const float uz = K1 * (pb_zx(c, i, j) - pb_zx(c, i - 1, j)) + K2 * (pb_zx(c, i + 1, j) - pb_zx(c, i - 2, j));
    const float wz = K1 * (pb_zz(c, i + 1, j) - pb_zz(c, i, j)) + K2 * (pb_zz(c, i + 2, j) - pb_zz(c, i - 1, j));
    const float wx = K1 * (pb_xz(c, i, j) - pb_xz(c, i, j - 1)) + K2 * (pb_xz(c, i, j + 1) - pb_xz(c, i, j - 2));
    adj_vel_finish<GRAD, SRCADJ, false>(s, i, j, n, seg, first != 0, ux, uz, wz, wx);
  }
}

// Transposed velocity sub-step (second at reverse step n): u_bar -> t_bar.
// txx, tzz, t1, t2: D-x q_bar_xa, D-z q_bar_zb, D+z q_bar_xb, D+x q_bar_za at the cell's
// stress nodes (without 1/h).
template <bool GRAD, bool PML>
__device__ __forceinline__ void adj_str_finish(const Shot2D& s, int i, int j, int n, const gfloat* seg, bool first,
                                               float txx, float tzz, float t1, float t2) {
  const long ld = s.ld;
  const long o = (long)i * ld + j;
  const int rd = (n + 1) & 1, wr = n & 1;
  // ---- loads ----
  const float ux = s.uxb[o], uz = s.uzb[o];
  const float lam = s.lam[o], l2m = l2m_of(s, o), mxz = muxz_of(s, o);
  const float t0xx = s.txxb[o], t0zz = s.tzzb[o], t0xz = s.txzb[o];
  int sx = -1, sz = -1;
  long qx_ = 0, qz_ = 0;
  float r1 = 0.0f, r2 = 0.0f, r3 = 0.0f, r4 = 0.0f;
  if (PML) {  // owned adjoint memory variables of the velocity-side derivatives
    sx = strip_index(j, s.nx, s.P);
    sz = strip_index(i, s.nz, s.P);
    qx_ = (long)i * 2 * s.P + max(sx, 0);
    qz_ = (long)max(sz, 0) * s.nx + j;
    r1 = bxh(s)[j] * (s.pbx[rd][X_VXX][qx_] + s.dt * ux);
    r2 = bxi(s)[j] * (s.pbx[rd][X_VZX][qx_] + s.dt * uz);
    r3 = bzi(s)[i] * (s.pbz[rd][Z_VXZ][qz_] + s.dt * ux);
    r4 = bzh(s)[i] * (s.pbz[rd][Z_VZZ][qz_] + s.dt * uz);
  }
  long cc = 0;
  float a2 = 0.0f, r = 0.0f;
  if (GRAD) {
    cc = (long)i * s.cp + j;
    const gfloat* h3 = seg + 3 * s.cells;
    const gfloat* h4 = seg + 4 * s.cells;
    // vx nodes (i, b + 1/2), b in {j-1, j}: b_x averages rho(i, b), rho(i, b + 1); vz nodes
    // (a + 1/2, j), a in {i-1, i}; clamped indices, weight 0 where rho(i, j) is not used
    const int jm = max(j - 1, 0), im = max(i - 1, 0);
    r = (float)pair_count(j - 1, j, s.nx) * s.uxb[(long)i * ld + jm] * h3[(long)i * s.cp + jm];
    r += (float)pair_count(j, j, s.nx) * ux * h3[cc];
    r += (float)pair_count(i - 1, i, s.nz) * s.uzb[(long)im * ld + j] * h4[(long)im * s.cp + j];
    r += (float)pair_count(i, i, s.nz) * uz * h4[cc];
    if (!first) a2 = s.acc[2 * s.cells + cc];
  }
  // ---- arithmetic ----
  // sigma_bar_xx += -D-x q_bar_xa ; sigma_bar_zz += -D-z q_bar_zb ;
  // sigma_bar_xz += -(D+z q_bar_xb + D+x q_bar_za)
  const float dsxx = -txx * s.rdx, dszz = -tzz * s.rdz, dsxz = -(t1 * s.rdz + t2 * s.rdx);
  // ---- stores ----
  if (PML) {
    if (sx >= 0) {
      s.pbx[wr][X_VXX][qx_] = r1;
      s.pbx[wr][X_VZX][qx_] = r2;
    }
    if (sz >= 0) {
      s.pbz[wr][Z_VXZ][qz_] = r3;
      s.pbz[wr][Z_VZZ][qz_] = r4;
    }
  }
  s.txxb[o] = t0xx + (l2m * dsxx + lam * dszz);
  s.tzzb[o] = t0zz + (lam * dsxx + l2m * dszz);
  s.txzb[o] = t0xz + mxz * dsxz;
  if (GRAD) s.acc[2 * s.cells + cc] = a2 - s.dt * r;
}

template <bool GRAD>
__global__ __launch_bounds__(BX * BZ) void k_adj_str(BATCH_PARAMS, int n, int k, int first) {
  BATCH_TILE();
  const int j = j0 + threadIdx.x, i = i0 + threadIdx.y;
  const gfloat* seg = GRAD ? s.seg + (size_t)k * NSEG_FIELDS * s.cells : nullptr;
  const bool active = i < s.nz && j < s.nx;
  if (block_in_pml(s, j0, i0, BZ, 2)) {  // block-uniform: every thread reaches the barrier
    __shared__ float lds[LDS_OPS];
    const StageArea a{lds, lds + BZ * LX, lds + 2 * BZ * LX, lds + 2 * BZ * LX + LZ * BX};
    const int rd = (n + 1) & 1;
    // x0: q_bar_xa at columns j-2 .. j+1; x1: q_bar_za at j-1 .. j+2;
    // z0: q_bar_zb at rows i-2 .. i+1;     z1: q_bar_xb at i-1 .. i+2
    stage_operands(s, i0, j0, a, StagedOp{s.uxb, axh(s), s.pbx[rd][X_VXX], -2},
                   StagedOp{s.uzb, axi(s), s.pbx[rd][X_VZX], -1}, StagedOp{s.uzb, azh(s), s.pbz[rd][Z_VZZ], -2},
                   StagedOp{s.uxb, azi(s), s.pbz[rd][Z_VXZ], -1});
    __syncthreads();
    if (!active) return;
    const int r = threadIdx.y, q = threadIdx.x;
    const float* X0 = a.x0 + r * LX + q;   // X0[m] = q_bar_xa(i, j - 2 + m)
    const float* X1 = a.x1 + r * LX + q;   // X1[m] = q_bar_za(i, j - 1 + m)
    const float* Z0 = a.z0 + r * BX + q;   // Z0[m BX] = q_bar_zb(i - 2 + m, j)
    const float* Z1 = a.z1 + r * BX + q;   // Z1[m BX] = q_bar_xb(i - 1 + m, j)
    const float txx = K1 * (X0[2] - X0[1]) + K2 * (X0[3] - X0[0]);
    const float tzz = K1 * (Z0[2 * BX] - Z0[BX]) + K2 * (Z0[3 * BX] - Z0[0]);
    const float t1 = K1 * (Z1[2 * BX] - Z1[BX]) + K2 * (Z1[3 * BX] - Z1[0]);
    const float t2 = K1 * (X1[2] - X1[1]) + K2 * (X1[3] - X1[0]);
    adj_str_finish<GRAD, true>(s, i, j, n, seg, first != 0, txx, tzz, t1, t2);
  } else if (active) {
    const AdjCtx<false> c{s, 0};
    const float txx = K1 * (qb_xa(c, i, j) - qb_xa(c, i, j - 1)) + K2 * (qb_xa(c, i, j + 1) - qb_xa(c, i, j - 2));
    const float tzz = K1 * (qb_zb(c, i, j) - qb_zb(c, i - 1, j)) + K2 * (qb_zb(c, i + 1, j) - qb_zb(c, i - 2, j));
    const float t1 = K1 * (qb_xb(c, i + 1, j) - qb_xb(c, i, j)) + K2 * (qb_xb(c, i + 2, j) - qb_xb(c, i - 1, j));
    const float t2 = K1 * (qb_za(c, i, j + 1) - qb_za(c, i, j)) + K2 * (qb_za(c, i, j + 2) - qb_za(c, i, j - 1));
    adj_str_finish<GRAD, false>(s, i, j, n, seg, first != 0, txx, tzz, t1, t2);
  }
}

// ------------------------------------------------------------------------------------
// Staging: (Vp, Vs, rho) of the window -> lambda, mu, rho at the normal nodes; the last row
// and column are repeated into the halo so that the averages of the staggered parameters
// clamp at the far edges (see bx_of, muxz_of).
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(BX * BZ) void k_stage(BATCH_PARAMS) {
  BATCH_TILE();
  const int j = j0 + threadIdx.x, i = i0 + threadIdx.y;
  if (i >= s.nz || j >= s.nx) return;
  const long mo = (long)i * s.mld + j;
  const float vp = s.mvp[mo], vs = s.mvs[mo], rho = s.mrho[mo];
  const float mu = rho * vs * vs;
  const float lam = rho * vp * vp - 2.0f * mu;
  const long o = (long)i * s.ld + j;
  const bool xe = j == s.nx - 1, ze = i == s.nz - 1;
  for (int c = 0; c < 4; ++c) {
    const bool dx = c & 1, dz = c >> 1;
    if ((dx && !xe) || (dz && !ze)) continue;
    const long oc = o + (dx ? 1 : 0) + (dz ? s.ld : 0);
    s.lam[oc] = lam;
    s.mu[oc] = mu;
    s.rho[oc] = rho;
  }
}

// ------------------------------------------------------------------------------------
// Chain rule of one block's FP32 imaging sums (A, E, R at the normal node, gathered over
// the staggered nodes by the adjoint kernels) into the FP64 (Vp, Vs, rho) gradient:
// g_lambda = A, g_mu = A + E / mu^2, g_rho(b) = R; lambda = rho(Vp^2 - 2Vs^2), mu = rho Vs^2.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(BX * BZ) void k_chain_flush(BATCH_PARAMS) {
  BATCH_TILE();
  const int j = j0 + threadIdx.x, i = i0 + threadIdx.y;
  if (i >= s.nz || j >= s.nx) return;
  const long cc = (long)i * s.cp + j;
  const long mo = (long)i * s.mld + j;
  const double vp = s.mvp[mo], vs = s.mvs[mo], rho = s.mrho[mo];
  const double mu = rho * vs * vs;
  const double gl = s.acc[cc];
  const double gmu = gl + (mu > 0.0 ? (double)s.acc[s.cells + cc] / (mu * mu) : 0.0);
  s.G[cc] += 2.0 * rho * vp * gl;
  s.G[s.cells + cc] += 2.0 * rho * vs * (gmu - 2.0 * gl);
  s.G[2 * s.cells + cc] += (vp * vp - 2.0 * vs * vs) * gl + vs * vs * gmu + (double)s.acc[2 * s.cells + cc];
}

__global__ __launch_bounds__(BX * BZ) void k_write_gradient(BATCH_PARAMS) {
  BATCH_TILE();
  gfloat* g = s.gout;
  const long mplane = s.mplane;
  const int z0 = s.z0, x0 = s.x0;
  const int j = j0 + threadIdx.x, i = i0 + threadIdx.y;
  if (i >= s.nz || j >= s.nx) return;
  const long cc = (long)i * s.cp + j;
  const long go = (long)(z0 + i) * s.mld + (x0 + j);
  for (int k = 0; k < 3; ++k) g[k * mplane + go] = (float)s.G[k * s.cells + cc];
}

// ------------------------------------------------------------------------------------
// Misfit (FP64) and the reverse cumulative residual that drives the DAS transpose:
// e_bar[n][c] = sum_{k >= n} r[c][k], r = d - d_obs. One thread per channel; the per-channel
// FP64 partial sums are reduced in a fixed order by a single block.
// ------------------------------------------------------------------------------------
__global__ void k_residual(const float* d, const float* dobs, int nch, int nt, double* partial, float* ebar) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nch) return;
  double acc = 0.0, sq = 0.0;
  for (int n = nt - 1; n >= 0; --n) {
    const long k = (long)c * nt + n;
    const double r = dobs ? (double)d[k] - (double)dobs[k] : (double)d[k];
    sq += r * r;
    acc += r;
    ebar[(long)n * nch + c] = (float)acc;
  }
  if (partial) partial[c] = sq;
}

__global__ void k_reduce_phi(const double* partial, int n, double* phi) {
  __shared__ double sh[256];
  double a = 0.0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) a += partial[k];
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *phi = 0.5 * sh[0];
}

inline dim3 grid_of(const Sched& q) { return dim3(q.n); }
inline dim3 block2d() { return dim3(BX, BZ); }
#define FWD_ARGS b.shots, b.tile_shot, b.tile_first, b.fwd.sched
#define ADJ_ARGS b.shots, b.tile_shot, b.tile_first, b.adj.sched

}  // namespace

hipError_t launch_stage2d(const Batch2D& b, hipStream_t st) {
  k_stage<<<grid_of(b.fwd), block2d(), 0, st>>>(FWD_ARGS);
  return hipGetLastError();
}

#define STEP_ARGS b.shots, b.step_tile_shot, b.step_tile_first, b.step.sched

hipError_t launch_fwd_step(const Batch2D& b, int n, int kstore, bool record, hipStream_t st) {
  const dim3 g = grid_of(b.step);
  if (kstore >= 0) {
    if (record) k_fwd_step<TSTEP, true, true><<<g, block2d(), 0, st>>>(STEP_ARGS, n, kstore);
    else k_fwd_step<TSTEP, true, false><<<g, block2d(), 0, st>>>(STEP_ARGS, n, kstore);
  } else {
    if (record) k_fwd_step<TSTEP, false, true><<<g, block2d(), 0, st>>>(STEP_ARGS, n, 0);
    else k_fwd_step<TSTEP, false, false><<<g, block2d(), 0, st>>>(STEP_ARGS, n, 0);
  }
  return hipGetLastError();
}

hipError_t launch_adj_vel(const Batch2D& b, int n, int k, bool grad, bool first, bool srcadj, hipStream_t st) {
  if (grad) k_adj_vel<true, false><<<grid_of(b.adj), block2d(), 0, st>>>(ADJ_ARGS, n, k, first);
  else if (srcadj) k_adj_vel<false, true><<<grid_of(b.adj), block2d(), 0, st>>>(ADJ_ARGS, n, 0, 0);
  else k_adj_vel<false, false><<<grid_of(b.adj), block2d(), 0, st>>>(ADJ_ARGS, n, 0, 0);
  return hipGetLastError();
}

hipError_t launch_adj_str(const Batch2D& b, int n, int k, bool grad, bool first, hipStream_t st) {
  if (grad) k_adj_str<true><<<grid_of(b.adj), block2d(), 0, st>>>(ADJ_ARGS, n, k, first);
  else k_adj_str<false><<<grid_of(b.adj), block2d(), 0, st>>>(ADJ_ARGS, n, 0, 0);
  return hipGetLastError();
}

hipError_t launch_chain_flush(const Batch2D& b, hipStream_t st) {
  k_chain_flush<<<grid_of(b.fwd), block2d(), 0, st>>>(FWD_ARGS);
  return hipGetLastError();
}

hipError_t launch_write_gradient(const Batch2D& b, hipStream_t st) {
  k_write_gradient<<<grid_of(b.fwd), block2d(), 0, st>>>(FWD_ARGS);
  return hipGetLastError();
}

hipError_t launch_misfit_raw(int nch, int nt, const float* d, const float* dobs, double* partial, double* phi,
                             float* ebar, hipStream_t st) {
  if (nch > 0) k_residual<<<(nch + 127) / 128, 128, 0, st>>>(d, dobs, nch, nt, partial, ebar);
  k_reduce_phi<<<1, 256, 0, st>>>(partial, nch > 0 ? nch : 0, phi);
  return hipGetLastError();
}

hipError_t launch_residual_cumsum_raw(int nch, int nt, const float* r, float* ebar, hipStream_t st) {
  if (nch > 0) k_residual<<<(nch + 127) / 128, 128, 0, st>>>(r, nullptr, nch, nt, nullptr, ebar);
  return hipGetLastError();
}

hipError_t launch_misfit(const Shot2D& s, const float* d, const float* dobs, double* partial, double* phi,
                         float* ebar, hipStream_t st) {
  return launch_misfit_raw(s.nch, s.nt, d, dobs, partial, phi, ebar, st);
}

hipError_t launch_residual_cumsum(const Shot2D& s, const float* r, float* ebar, hipStream_t st) {
  return launch_residual_cumsum_raw(s.nch, s.nt, r, ebar, st);
}

}  // namespace efwi
