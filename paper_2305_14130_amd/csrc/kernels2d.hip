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
// The stencils are bandwidth bound (well under 1 flop/byte), so there is no MFMA. One
// launch per time step fuses both half steps on tiles of 8, 12 or 16 rows x 64 columns
// (a wavefront covers 64 consecutive x): the tile's halo of the first half step's input is
// staged in LDS and the second half step's input is recomputed on a 2-node halo instead of
// being exchanged between tiles. The transposed step is the exact transpose of the forward
// step in scaled adjoint variables (material parameters applied at the owned node), not
// the forward scheme run backwards; it also gathers the imaging sums.
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
#define STEP_PARAMS const Shot2D* __restrict__ shots, const StepSlot* __restrict__ slots
#define BATCH_TILE()                                                                           \
  int sh_, i0, j0;                                                                              \
  if (!batch_tile<BZ>(sched, tile_shot, tile_first, shots, sh_, i0, j0)) return;               \
  const Shot2D& s = shots[sh_]

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
  const gfloat *c11, *c13;                   // VTI staged parameters (NULL: isotropic)
  const gfloat* rps;                         // memory variables of buffer n & 1 (see xv, zv)
  gfloat* wps;                               // and of buffer (n + 1) & 1
  const gfloat* prof;                        // CPML profiles (see xp, zp)
  gfloat* seg;                               // this step's slot of the history (STORE)
  int ld, nx, nz, P2;                        // row pitch, window, strip width 2P
  unsigned xs, zs;                           // elements of one x-strip and one z-strip array
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
  p.c11 = s.c11 ? s.c11 - org : nullptr;
  p.c13 = s.c13 ? s.c13 - org : nullptr;
  p.rps = s.psx[0] + rd;
  p.wps = s.psx[0] + wr;
  p.prof = s.prof;
  p.seg = seg;
  p.ld = s.ld, p.nx = s.nx, p.nz = s.nz, p.P2 = 2 * s.P;
  p.xs = (unsigned)(s.nz * 2 * s.P), p.zs = (unsigned)(2 * s.P * s.nx);
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

// Streaming (non-temporal) accesses of the history: written once per forward step, read
// once in the reverse sweep.
template <class P>
__device__ __forceinline__ void GS(P* base, unsigned e, float v) {
  typedef __attribute__((address_space(1))) char gchar;
  __builtin_nontemporal_store(v, (P*)((gchar*)base + e * 4u));
}
template <class P>
__device__ __forceinline__ float GL(const P* base, unsigned e) {
  typedef const __attribute__((address_space(1))) char gchar;
  return __builtin_nontemporal_load((const P*)((gchar*)base + e * 4u));
}

// Element offsets inside the strip block of one buffer (x-strip arrays [nz][2P] of the
// variables X_*, then z-strip arrays [2P][nx] of the variables Z_*) and inside the profile
// table (a_x, b_x at integer then half nodes [nx], then the same along z [nz]; k = 0 a at
// integer nodes, 1 b at integer nodes, 2 a at half nodes, 3 b at half nodes). One base
// pointer plus 32-bit offsets keeps the CPML paths' scalar registers few.
template <class P>
__device__ __forceinline__ unsigned xv(const P& p, int k) { return (unsigned)k * p.xs; }
template <class P>
__device__ __forceinline__ unsigned zv(const P& p, int k) { return 4u * p.xs + (unsigned)k * p.zs; }
template <class P>
__device__ __forceinline__ unsigned xp(const P& p, int k) { return (unsigned)(k * p.nx); }
template <class P>
__device__ __forceinline__ unsigned zp(const P& p, int k) { return (unsigned)(4 * p.nx + k * p.nz); }

// Inputs of one velocity node (loads only).
struct VelLoads {
  float vx, vz, r0, rx, rz;
};

// EDGE: the tile may reach the grid's edges (clamp indices, mask outside nodes); tiles away
// from every edge skip both. Neighbours at a fixed offset are addressed through a shifted
// uniform base, so the lane offset is shared by all of a node's loads.
template <bool PML, bool EDGE>
__device__ __forceinline__ VelLoads vel_loads(const StepPtrs& p, const Shot2D& s, int gi, int gj) {
  VelLoads L;
  const int ic = EDGE ? min(max(gi, 0), p.nz - 1) : gi, jc = EDGE ? min(max(gj, 0), p.nx - 1) : gj;
  const unsigned o = pofs(p, ic, jc);
  L.vx = G(p.vx, o);
  L.vz = G(p.vz, o);
  L.r0 = G(p.rho, o);
  L.rx = G(p.rho + 1, o);
  L.rz = G(p.rho + p.ld, o);
  return L;
}

// Velocity node (gi, gj): the four stress differences d1 = D+x sxx, d2 = D-z sxz (vx) and
// d3 = D-x sxz, d4 = D+z szz (vz) come from LDS. Returns v^{n+1/2} (0 outside the grid);
// with `owned`, writes v, the memory variables and the stored divergences.
template <bool STORE, bool PML, bool EDGE>
__device__ __forceinline__ void vel_node(const StepPtrs& p, const Shot2D& s, int gi, int gj, bool owned,
                                         const VelLoads& L, float d1, float d2, float d3, float d4, float& vxn,
                                         float& vzn) {
  const bool in = !EDGE || (gi >= 0 && gi < p.nz && gj >= 0 && gj < p.nx);
  int sx = -1, sz = -1;
  float p1 = 0.0f, p2 = 0.0f, p3 = 0.0f, p4 = 0.0f;
  if (PML) {
    const int ic = min(max(gi, 0), p.nz - 1), jc = min(max(gj, 0), p.nx - 1);
    sx = strip_index(jc, p.nx, s.P);
    sz = strip_index(ic, p.nz, s.P);
    // the velocity-side memory variables are loaded here, not with the node's other
    // inputs: CPML tiles keep fewer values live, so every tile kernel fits more waves
    const unsigned qx = (unsigned)(ic * p.P2 + max(sx, 0)), qz = (unsigned)(max(sz, 0) * p.nx + jc);
    p1 = G(p.prof, xp(p, 3) + jc) * G(p.rps, xv(p, X_VXX) + qx) + G(p.prof, xp(p, 2) + jc) * d1;
    p3 = G(p.prof, xp(p, 1) + jc) * G(p.rps, xv(p, X_VZX) + qx) + G(p.prof, xp(p, 0) + jc) * d3;
    p2 = G(p.prof, zp(p, 1) + ic) * G(p.rps, zv(p, Z_VXZ) + qz) + G(p.prof, zp(p, 0) + ic) * d2;
    p4 = G(p.prof, zp(p, 3) + ic) * G(p.rps, zv(p, Z_VZZ) + qz) + G(p.prof, zp(p, 2) + ic) * d4;
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
  if (EDGE) {
    const float m = in ? 1.0f : 0.0f;
    vxn = m * (L.vx + s.dt * bx * qx);
    vzn = m * (L.vz + s.dt * bz * qz);
  } else {
    vxn = L.vx + s.dt * bx * qx;
    vzn = L.vz + s.dt * bz * qz;
  }
  if (owned) {
    const unsigned o = pofs(p, gi, gj);
    G(p.wvx, o) = vxn;
    G(p.wvz, o) = vzn;
    if (PML) {
      if (sx >= 0) {
        const unsigned q = (unsigned)(gi * p.P2 + sx);
        G(p.wps, xv(p, X_VXX) + q) = p1;
        G(p.wps, xv(p, X_VZX) + q) = p3;
      }
      if (sz >= 0) {
        const unsigned q = (unsigned)(sz * p.nx + gj);
        G(p.wps, zv(p, Z_VXZ) + q) = p2;
        G(p.wps, zv(p, Z_VZZ) + q) = p4;
      }
    }
    if (STORE) {  // divergences times b/2: the rho imaging terms (d b / d rho = -b^2/2)
      const unsigned c = (unsigned)(gi * s.cp + gj);
      GS(p.seg, 3 * s.cells + c, 0.5f * qx * bx);
      GS(p.seg, 4 * s.cells + c, 0.5f * qz * bz);
    }
  }
}

// Inputs of one stress node (loads only; the DAS channel, in the rare channel rows, is
// looked up in str_node).
struct StrLoads {
  float lam, mu, mu_x, mu_z, mu_xz, c11, c13;
};

template <bool PML, bool EDGE, bool VTI>
__device__ __forceinline__ StrLoads str_loads(const StepPtrs& p, const Shot2D& s, int gi, int gj) {
  StrLoads L;
  const int ic = EDGE ? min(gi, p.nz - 1) : gi, jc = EDGE ? min(gj, p.nx - 1) : gj;
  const unsigned o = pofs(p, ic, jc);
  L.c11 = VTI ? G(p.c11, o) : 0.0f;
  L.c13 = VTI ? G(p.c13, o) : 0.0f;
  L.lam = G(p.lam, o);
  L.mu = G(p.mu, o);
  L.mu_x = G(p.mu + 1, o);
  L.mu_z = G(p.mu + p.ld, o);
  L.mu_xz = G(p.mu + p.ld + 1, o);
  return L;
}

// Stress node (i, j) from the LDS strain rates pxx = D-x vx, pzz = D-z vz, pzx = D+z vx,
// pxz = D+x vz and the LDS sigma^n.
// VTI: sigma_xx += dt (c11 p_xx + c13 p_zz), sigma_zz += dt (c13 p_xx + c33 p_zz), and the
// stored normal-block quantities are p_xx / det and p_zz / det, det = c11 c33 - c13^2.
template <bool STORE, bool RECORD, bool PML, bool VTI>
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
    // memory variables loaded here rather than with the node's inputs (fewer live values)
    const unsigned qx = (unsigned)(i * p.P2 + max(sx, 0)), qz = (unsigned)(max(sz, 0) * p.nx + j);
    p1 = G(p.prof, xp(p, 1) + j) * G(p.rps, xv(p, X_XX) + qx) + G(p.prof, xp(p, 0) + j) * pxx;
    p2 = G(p.prof, xp(p, 3) + j) * G(p.rps, xv(p, X_XZ) + qx) + G(p.prof, xp(p, 2) + j) * pxz;
    p3 = G(p.prof, zp(p, 1) + i) * G(p.rps, zv(p, Z_ZZ) + qz) + G(p.prof, zp(p, 0) + i) * pzz;
    p4 = G(p.prof, zp(p, 3) + i) * G(p.rps, zv(p, Z_XZ) + qz) + G(p.prof, zp(p, 2) + i) * pzx;
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
  const float c11 = VTI ? L.c11 : l2m, c13 = VTI ? L.c13 : lam;
  sxx += s.dt * (c11 * pxx + c13 * pzz);
  szz += s.dt * (c13 * pxx + l2m * pzz);
  sxz += s.dt * mxz * ps;
  if (i == s.si && j == s.sj) {
    sxx -= s.w * f_xx;
    szz -= s.w * f_zz;
  }
  if ((i == s.si || i == s.si - 1) && (j == s.sj || j == s.sj - 1)) sxz -= 0.25f * s.w * f_xz;
  if (PML) {
    if (sx >= 0) {
      const unsigned q = (unsigned)(i * p.P2 + sx);
      G(p.wps, xv(p, X_XX) + q) = p1;
      G(p.wps, xv(p, X_XZ) + q) = p2;
    }
    if (sz >= 0) {
      const unsigned q = (unsigned)(sz * p.nx + j);
      G(p.wps, zv(p, Z_ZZ) + q) = p3;
      G(p.wps, zv(p, Z_XZ) + q) = p4;
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
    if (VTI) {
      const float det = c11 * l2m - c13 * c13;
      GS(p.seg, c, pxx / det);
      GS(p.seg, s.cells + c, pzz / det);
    } else {
      GS(p.seg, c, (pxx + pzz) / (l2m + lam));
      GS(p.seg, s.cells + c, 0.5f * (pxx - pzz) * mu);
    }
    GS(p.seg, 2 * s.cells + c, 0.25f * ps * mxz);
  }
}

// ACORR: also add vx^2 + vz^2 of the new velocities at the owned nodes into acc[0] (the
// zero-lag autocorrelation of the particle velocity, for the approximate pseudo-Hessian).
template <int TZ, bool STORE, bool RECORD, bool PML, bool EDGE, bool ACORR, bool VTI>
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
  // a wavefront is one row of threads, so ty is the same in every lane: rows indexed through
  // tyu keep their addresses in scalar registers (the velocity rows too: 82 -> 80 VGPRs, 6
  // waves per SIMD instead of 5, 1000 x 3000 shot: forward step 33.3 -> 32.4 us, transposed
  // 58.9 -> 57.9 us; the LDS row of the transposed step's velocity store stays per lane,
  // which keeps two VGPRs fewer)
  const int tyu = __builtin_amdgcn_readfirstlane(ty);
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
    const int ic = EDGE ? min(max(i0 - 4 + sr_[k], 0), p.nz - 1) : i0 - 4 + sr_[k];
    const gfloat* src = f == 0 ? p.sxx : f == 1 ? p.szz : p.sxz;
    typedef const __attribute__((address_space(1))) char gchar;
    sv[k] = *(const __attribute__((address_space(1))) f4*)((gchar*)src + pofs(p, ic, j0 - 4 + 4 * sc4[k]) * 4u);
  }
  VelLoads L[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) L[k] = vel_loads<PML, EDGE>(p, s, i0 - 2 + tyu + k * BZ, j0 + tx);
  const VelLoads H = vel_loads<PML, EDGE>(p, s, i0 - 2 + hv, j0 - 2 + hcol);
  const float f_xx = s.src[n], f_zz = s.src[s.nt + n], f_xz = s.src[2 * s.nt + n];

  // ---- 1. staged sigma to LDS ----
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    if (sf[k] < 3) {
      const int f = sf[k], r = sr_[k], c4 = sc4[k];
      const int gi = i0 - 4 + r, gj = j0 - 4 + 4 * c4;
      f4 v = sv[k];
      if (EDGE) {
        const bool row_in = gi >= 0 && gi < p.nz;
        v.x = (row_in && gj + 0 >= 0 && gj + 0 < p.nx) ? v.x : 0.0f;
        v.y = (row_in && gj + 1 >= 0 && gj + 1 < p.nx) ? v.y : 0.0f;
        v.z = (row_in && gj + 2 >= 0 && gj + 2 < p.nx) ? v.z : 0.0f;
        v.w = (row_in && gj + 3 >= 0 && gj + 3 < p.nx) ? v.w : 0.0f;
      }
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
    vel_node<STORE, PML, EDGE>(p, s, gi, gj, owned, LL, d1, d2, d3, d4, vxn, vzn);
    VXL[vr * VC + lcol] = vxn;
    VZL[vr * VC + lcol] = vzn;
    if (ACORR && owned) {
      const unsigned c = (unsigned)(gi * s.cp + gj);
      s.acc[c] += vxn * vxn + vzn * vzn;
    }
  };
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int vr = tyu + k * BZ, gi = i0 - 2 + vr;
    vel(vr, tx + 2, L[k], gi >= i0 && gi < i0 + TZ && (!EDGE || (gi < p.nz && j0 + tx < p.nx)));
  }
  if ((tid >> 2) < VR) vel(hv, hcol, H, false);
  __syncthreads();

  // ---- 3. stresses of the tile (their parameter loads issued here, after the velocity
  //         phase, to bound the live registers) ----
  StrLoads SL[NSR];
#pragma unroll
  for (int k = 0; k < NSR; ++k) SL[k] = str_loads<PML, EDGE, VTI>(p, s, i0 + tyu + k * BZ, j0 + tx);
#pragma unroll
  for (int k = 0; k < NSR; ++k) {
    const int i = i0 + tyu + k * BZ, j = j0 + tx;
    if (EDGE && (i >= p.nz || j >= p.nx)) continue;
    const int vr = tyu + k * BZ + 2, vc = tx + 2;   // LDS velocity coordinates of the node
    const float* X = VXL + vr * VC + vc;
    const float* Z = VZL + vr * VC + vc;
    const float pxx = (K1 * (X[0] - X[-1]) + K2 * (X[1] - X[-2])) * s.rdx;
    const float pzz = (K1 * (Z[0] - Z[-VC]) + K2 * (Z[VC] - Z[-2 * VC])) * s.rdz;
    const float pzx = (K1 * (X[VC] - X[0]) + K2 * (X[2 * VC] - X[-VC])) * s.rdz;
    const float pxz = (K1 * (Z[1] - Z[0]) + K2 * (Z[2] - Z[-1])) * s.rdx;
    const int so = (vr + 2) * SC + tx + 4;           // LDS sigma of the node
    str_node<STORE, RECORD, PML, VTI>(p, s, i, j, n, SL[k], slot[k], pxx, pzz, pzx, pxz, SXX[so], SZZ[so], SXZ[so],
                                 f_xx, f_zz, f_xz);
  }
}

// Tile shape of the fused forward step: TSTEP rows x 64 columns.
// Workgroup w takes schedule slot w: its tile and code path come in one scalar load (the
// host classified the tile), so a workgroup starts its tile's loads after two dependent
// scalar round trips (the slot, then the shot's descriptor).
template <int TZ, bool STORE, bool RECORD, bool ACORR, bool VTI>
__global__ __launch_bounds__(BX * BZ) void k_fwd_step(STEP_PARAMS, int n, int kstore) {
  __shared__ float lds[StepTile<TZ>::LDS_FLOATS];
  const StepSlot slot = slots[blockIdx.x];
  if (slot.shot < 0) return;
  const Shot2D& s = shots[slot.shot];
  const int i0 = slot.i0, j0 = slot.j0;
  gfloat* seg = STORE ? s.seg + (size_t)kstore * NSEG_FIELDS * s.cells : nullptr;
  // block-uniform branch: every thread reaches the barriers. CPML tiles: within 2 nodes of
  // a strip (velocity halo); edge tiles (grids whose strips are under 2 nodes wide): the
  // staged halo may leave the grid; every other tile's staged halo lies inside it.
  if (slot.path == PATH_PML) fwd_step_tile<TZ, STORE, RECORD, true, true, ACORR, VTI>(s, i0, j0, n, seg, lds);
  else if (slot.path == PATH_EDGE) fwd_step_tile<TZ, STORE, RECORD, false, true, ACORR, VTI>(s, i0, j0, n, seg, lds);
  else fwd_step_tile<TZ, STORE, RECORD, false, false, ACORR, VTI>(s, i0, j0, n, seg, lds);
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

__device__ __forceinline__ float ebar_at(const Shot2D& s, int slot, int jc, int n) {
  if (jc < 0 || jc >= s.nx) return 0.0f;
  const int c = s.rowch[(long)slot * s.nx + jc];
  return c >= 0 ? s.ebar[(long)n * s.nch + c] : 0.0f;
}

// ------------------------------------------------------------------------------------
// Fused transposed step n (reverse time) on the forward step's tiles of TZ rows x 64
// columns: the transpose of the stress half step and then of the velocity half step, in
// the scaled variables above. The adjoint fields are double-buffered by step parity like
// the forward state: buffer (n + 1) & 1 holds t_bar, u_bar of step n + 1, the step writes
// buffer n & 1. Per tile:
//   1. the corrected transposed stress operands p_bar (dt t_bar, plus the CPML transpose
//      inside the strips) of the tile and a 4-node halo are staged in LDS;
//   2. u_bar += b (-D^T p_bar) (+ the DAS transpose) on the tile and a 2-node halo, kept in
//      LDS with the corrected transposed velocity operands q_bar;
//   3. t_bar += C (-D^T q_bar) on the tile, the memory variables, and the imaging sums.
// ------------------------------------------------------------------------------------
template <int TZ>
struct AdjTile {
  static constexpr int SR = TZ + 8, SC = BX + 8;  // p_bar: rows i0-4 .. i0+TZ+3, columns j0-4 .. j0+67
  static constexpr int VR = TZ + 4, VC = BX + 4;  // u_bar, q_bar: rows i0-2 .. i0+TZ+1, columns j0-2 .. j0+65
  static constexpr int NP = SR * SC, NU = VR * VC;
  // interior tiles: 3 p_bar arrays, then u_bar (2); CPML tiles: 4 p_bar arrays, then (after a
  // barrier) u_bar and the 4 q_bar operands over the same space
  static constexpr int LDS_INT = 3 * NP + 2 * NU;
  static constexpr int LDS_PML = (4 * NP > 6 * NU) ? 4 * NP : 6 * NU;
  static constexpr int LDS_MAIN = LDS_INT > LDS_PML ? LDS_INT : LDS_PML;
  // then t_bar_xx, t_bar_zz, t_bar_xz of the tile's own nodes, copied while staging: the
  // transposed stress update reads them from here rather than from HBM a second time
  static constexpr int LDS_FLOATS = LDS_MAIN + 3 * TZ * BX;
};

struct AdjPtrs {
  const gfloat *txx, *tzz, *txz, *ux, *uz;   // adjoint buffer (n + 1) & 1, padded plane origins
  gfloat *wtxx, *wtzz, *wtxz, *wux, *wuz;    // buffer n & 1
  const gfloat *lam, *mu, *rho;              // staged parameters, padded plane origins
  const gfloat *c11, *c13;                   // VTI staged parameters (NULL: isotropic)
  const gfloat* rps;                         // adjoint memory variables of step n + 1 (see xv, zv)
  gfloat* wps;                               // and of step n
  const gfloat* prof;                        // CPML profiles (see xp, zp)
  const gfloat* seg;                         // history slot of step n (imaging)
  gfloat* acc;
  int ld, nx, nz, P2;
  unsigned xs, zs;
};

__device__ __forceinline__ AdjPtrs adj_ptrs(const Shot2D& s, int n, int kseg) {
  AdjPtrs p;
  const long org = (long)HALO * s.ld + XOFF;
  const int prd = (n + 1) & 1, pwr = n & 1;
  const long rd = (long)prd * s.abuf, wr = (long)pwr * s.abuf;
  p.txx = s.txxb - org + rd;
  p.tzz = s.tzzb - org + rd;
  p.txz = s.txzb - org + rd;
  p.ux = s.uxb - org + rd;
  p.uz = s.uzb - org + rd;
  p.wtxx = s.txxb - org + wr;
  p.wtzz = s.tzzb - org + wr;
  p.wtxz = s.txzb - org + wr;
  p.wux = s.uxb - org + wr;
  p.wuz = s.uzb - org + wr;
  p.lam = s.lam - org;
  p.mu = s.mu - org;
  p.rho = s.rho - org;
  p.c11 = s.c11 ? s.c11 - org : nullptr;
  p.c13 = s.c13 ? s.c13 - org : nullptr;
  p.rps = s.pbx[prd][0];
  p.wps = s.pbx[pwr][0];
  p.prof = s.prof;
  p.seg = s.seg ? s.seg + (size_t)kseg * NSEG_FIELDS * s.cells : nullptr;
  p.acc = s.acc;
  p.ld = s.ld, p.nx = s.nx, p.nz = s.nz, p.P2 = 2 * s.P;
  p.xs = (unsigned)(s.nz * 2 * s.P), p.zs = (unsigned)(2 * s.P * s.nx);
  return p;
}

__device__ __forceinline__ unsigned pofs(const AdjPtrs& p, int i, int j) {
  return (unsigned)((i + HALO) * p.ld + XOFF + j);
}

// Inputs of one u_bar node (loads only).
struct UbLoads {
  int slot;                  // DAS slot of the node's row (-1: none or outside the grid)
  float ux, uz, r0, rx, rz;
};

template <bool PML, bool EDGE>
__device__ __forceinline__ UbLoads ub_loads(const AdjPtrs& p, const Shot2D& s, int gi, int gj) {
  UbLoads L;
  const int ic = EDGE ? min(max(gi, 0), p.nz - 1) : gi, jc = EDGE ? min(max(gj, 0), p.nx - 1) : gj;
  const unsigned o = pofs(p, ic, jc);
  const bool in = !EDGE || (gi >= 0 && gi < p.nz && gj >= 0 && gj < p.nx);
  const int slot = s.row_slot[ic];
  L.slot = in ? slot : -1;
  L.ux = G(p.ux, o);
  L.uz = G(p.uz, o);
  L.r0 = G(p.rho, o);
  L.rx = G(p.rho + 1, o);
  L.rz = G(p.rho + p.ld, o);
  return L;
}

// Inputs of one t_bar node (loads only).
struct TbLoads {
  float lam, mu, mu_x, mu_z, mu_xz, c11, c13;
  float h0, h1, h3m, h3, h4m, h4, a0, a1, a2, a3, a4;   // imaging inputs (a3, a4: VTI)
  float h2[4], c2[4];         // around the node's four shear nodes: stored h2 and how often
                              // the node's mu is used
};

// EDGE: the node may sit on the grid's first or clamped last row or column (tiles that
// touch a CPML strip, or any tile without CPML); elsewhere every count below is 1.
template <bool GRAD, bool PML, bool EDGE, bool VTI>
__device__ __forceinline__ TbLoads tb_loads(const AdjPtrs& p, const Shot2D& s, int gi, int gj, bool first) {
  TbLoads L;
  const int ic = EDGE ? min(gi, p.nz - 1) : gi, jc = EDGE ? min(gj, p.nx - 1) : gj;
  const unsigned o = pofs(p, ic, jc);
  L.c11 = VTI ? G(p.c11, o) : 0.0f;
  L.c13 = VTI ? G(p.c13, o) : 0.0f;
  L.lam = G(p.lam, o);
  L.mu = G(p.mu, o);
  L.mu_x = G(p.mu + 1, o);
  L.mu_z = G(p.mu + p.ld, o);
  L.mu_xz = G(p.mu + p.ld + 1, o);
  L.h0 = L.h1 = L.h3m = L.h3 = L.h4m = L.h4 = L.a0 = L.a1 = L.a2 = L.a3 = L.a4 = 0.0f;
  if (GRAD) {
    const unsigned cc = (unsigned)(ic * s.cp + jc), cells = (unsigned)s.cells;
    L.h0 = GL(p.seg, cc);
    L.h1 = GL(p.seg, cells + cc);
    // shear nodes (a, b), a in {i-1, i}, b in {j-1, j} (k = 2 (a - i + 1) + b - j + 1): the
    // stored (pzx + pxz) mu_xz / 4 and how often mu_xz(a, b) uses mu(i, j); t_bar_xz of
    // step n + 1 there is read here in CPML tiles, from the staged operands otherwise
    for (int k = 0; k < 4; ++k) {
      const int a = ic - 1 + (k >> 1), b = jc - 1 + (k & 1);
      if (EDGE) {
        L.c2[k] = (float)corner_count(a, b, ic, jc, p.nz, p.nx);
        const int aa = max(a, 0), bb = max(b, 0);
        L.h2[k] = GL(p.seg, 2 * cells + (unsigned)(aa * s.cp + bb));
      } else {  // a shifted uniform base: the lane offset cc serves all four
        L.c2[k] = 1.0f;
        L.h2[k] = GL(p.seg + 2 * s.cells + ((k >> 1) - 1) * s.cp + (k & 1) - 1, cc);
      }
    }
    if (EDGE) {
      const int jm = max(jc - 1, 0), im = max(ic - 1, 0);
      L.h3m = GL(p.seg, 3 * cells + (unsigned)(ic * s.cp + jm));
      L.h4m = GL(p.seg, 4 * cells + (unsigned)(im * s.cp + jc));
    } else {
      L.h3m = GL(p.seg + 3 * s.cells - 1, cc);
      L.h4m = GL(p.seg + 4 * s.cells - s.cp, cc);
    }
    L.h3 = GL(p.seg, 3 * cells + cc);
    L.h4 = GL(p.seg, 4 * cells + cc);
    if (!first) {
      L.a0 = G(p.acc, cc);
      L.a1 = G(p.acc, cells + cc);
      L.a2 = G(p.acc, 2 * cells + cc);
      if (VTI) {
        L.a3 = G(p.acc, 3 * cells + cc);
        L.a4 = G(p.acc, 4 * cells + cc);
      }
    }
  }
  return L;
}

template <int TZ, bool GRAD, bool SRCADJ, bool PML, bool EDGE, bool VTI>
__device__ __forceinline__ void adj_step_tile(const Shot2D& s, int i0, int j0, int n, int kseg, bool first,
                                              float* lds) {
  using T = AdjTile<TZ>;
  constexpr int SR = T::SR, SC = T::SC, VR = T::VR, VC = T::VC, NP = T::NP, NU = T::NU;
  constexpr int NT = BX * BZ;
  constexpr int NV = VR / BZ, NSR = TZ / BZ;
  typedef float f4 __attribute__((ext_vector_type(4)));
  typedef const __attribute__((address_space(1))) char gchar;
  const AdjPtrs p = adj_ptrs(s, n, kseg);
  const float dt = s.dt;
  const int tx = threadIdx.x, ty = threadIdx.y, tid = ty * BX + tx;
  const int tyu = __builtin_amdgcn_readfirstlane(ty);
  // LDS: p_bar operands OX0 = p_xx, OX1 = p_xz (x-differentiated), OZ0 = p_zx, OZ1 = p_zz
  // (z-differentiated); in interior tiles OX1 and OZ0 are the same array (no correction)
  float* OX0 = lds;
  float* OZ1 = lds + NP;
  float* OX1 = lds + 2 * NP;
  float* OZ0 = PML ? lds + 3 * NP : OX1;
  float* UX = PML ? lds : lds + 3 * NP;   // CPML tiles overwrite the staged operands
  float* UZ = UX + NU;
  float* QXA = UZ + NU;      // q_bar operands (CPML tiles): x-differentiated from u_x, u_z,
  float* QZA = QXA + NU;     // z-differentiated from u_x, u_z
  float* QXB = QZA + NU;
  float* QZB = QXB + NU;
  float* TO = lds + T::LDS_MAIN;   // own t_bar_xx, t_bar_zz, t_bar_xz (TZ x 64 each)
  const int hv = min(tid >> 2, VR - 1), hc = tid & 3;
  const int hcol = hc < 2 ? hc : VC - 4 + hc;     // LDS u column 0, 1, 66, 67


  // ---- 1. stage p_bar ----
  if (!PML) {
    constexpr int Q = SC / 4, NQ = 3 * SR * Q, PER = (NQ + NT - 1) / NT;
    constexpr int DC = NT % Q, DR = (NT / Q) % SR;
    static_assert(NT / (SR * Q) == 0, "one step of NT float4s stays inside a field's staging area");
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
      const int f = min(sf[k], 2);
      const int ic = EDGE ? min(max(i0 - 4 + sr_[k], 0), p.nz - 1) : i0 - 4 + sr_[k];
      const gfloat* src = f == 0 ? p.txx : f == 1 ? p.tzz : p.txz;
      sv[k] = *(const __attribute__((address_space(1))) f4*)((gchar*)src + pofs(p, ic, j0 - 4 + 4 * sc4[k]) * 4u);
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      if (sf[k] < 3) {
        const int f = sf[k], r = sr_[k], c4 = sc4[k];
        const int gi = i0 - 4 + r, gj = j0 - 4 + 4 * c4;
        f4 v = dt * sv[k];
        if (EDGE) {
          const bool row_in = gi >= 0 && gi < p.nz;
          v.x = (row_in && gj + 0 >= 0 && gj + 0 < p.nx) ? v.x : 0.0f;
          v.y = (row_in && gj + 1 >= 0 && gj + 1 < p.nx) ? v.y : 0.0f;
          v.z = (row_in && gj + 2 >= 0 && gj + 2 < p.nx) ? v.z : 0.0f;
          v.w = (row_in && gj + 3 >= 0 && gj + 3 < p.nx) ? v.w : 0.0f;
        }
        *(f4*)(lds + f * NP + r * SC + 4 * c4) = v;
        if (r >= 4 && r < 4 + TZ && c4 >= 1 && c4 <= BX / 4)
          *(f4*)(TO + f * TZ * BX + (r - 4) * BX + 4 * (c4 - 1)) = sv[k];
      }
    }
  } else {
    // CPML tiles: four corrected operands, one after the other (a node's correction uses
    // the memory variable and profile of the operand's own axis)
    constexpr int PER = (NP + NT - 1) / NT;
#pragma unroll
    for (int op = 0; op < 4; ++op) {
      const gfloat* f = op == 0 ? p.txx : op == 3 ? p.tzz : p.txz;
      const bool xaxis = op < 2;
      const unsigned prof = op == 0 ? xp(p, 0) : op == 1 ? xp(p, 2) : op == 2 ? zp(p, 2) : zp(p, 0);
      const unsigned psi = op == 0 ? xv(p, X_XX) : op == 1 ? xv(p, X_XZ) : op == 2 ? zv(p, Z_XZ) : zv(p, Z_ZZ);
      float* dst = op == 0 ? OX0 : op == 1 ? OX1 : op == 2 ? OZ0 : OZ1;
      float* own = TO + (op == 0 ? 0 : op == 3 ? 1 : 2) * TZ * BX;
      float v[PER], raw[PER];
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int e = min(tid + k * NT, NP - 1);
        const int r = e / SC, c = e - r * SC;
        const int gi = i0 - 4 + r, gj = j0 - 4 + c;
        const bool in = gi >= 0 && gi < p.nz && gj >= 0 && gj < p.nx;
        const int ic = min(max(gi, 0), p.nz - 1), jc = min(max(gj, 0), p.nx - 1);
        const int sidx = xaxis ? strip_index(jc, p.nx, s.P) : strip_index(ic, p.nz, s.P);
        const int sc = max(sidx, 0);
        raw[k] = G(f, pofs(p, ic, jc));
        const float val = dt * raw[k];
        const float ps = G(p.rps, psi + (xaxis ? (unsigned)(ic * p.P2 + sc) : (unsigned)(sc * p.nx + jc)));
        const float ac = G(p.prof, prof + (unsigned)(xaxis ? jc : ic));
        const float m_in = in ? 1.0f : 0.0f, m_strip = sidx >= 0 ? 1.0f : 0.0f;
        v[k] = m_in * (val + (m_strip * ac) * (ps + val));
      }
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int e = tid + k * NT;
        if (e < NP) {
          dst[e] = v[k];
          const int r = e / SC, c = e - r * SC;
          if (op != 2 && r >= 4 && r < 4 + TZ && c >= 4 && c < 4 + BX) own[(r - 4) * BX + c - 4] = raw[k];
        }
      }
    }
  }
  // loads of the velocity nodes, issued before the barrier (after the staging loads, whose
  // registers are free by now)
  UbLoads UL[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) UL[k] = ub_loads<PML, EDGE>(p, s, i0 - 2 + tyu + k * BZ, j0 + tx);
  const UbLoads UH = ub_loads<PML, EDGE>(p, s, i0 - 2 + hv, j0 - 2 + hcol);
  __syncthreads();

  // ---- 2. u_bar on the tile and a 2-node halo ----
  struct Ub {
    float ux, uz;
  };
  auto ubar = [&](int vr, int lcol, const UbLoads& L, bool owned) -> Ub {
    const int gi = i0 - 2 + vr, gj = j0 - 2 + lcol;
    const int sr = vr + 2, sc = lcol + 2;   // LDS p_bar coordinates of the node
    const float ux_d = K1 * (OX0[sr * SC + sc + 1] - OX0[sr * SC + sc]) +
                       K2 * (OX0[sr * SC + sc + 2] - OX0[sr * SC + sc - 1]);
    const float uz_d = K1 * (OZ0[sr * SC + sc] - OZ0[(sr - 1) * SC + sc]) +
                       K2 * (OZ0[(sr + 1) * SC + sc] - OZ0[(sr - 2) * SC + sc]);
    const float wz_d = K1 * (OZ1[(sr + 1) * SC + sc] - OZ1[sr * SC + sc]) +
                       K2 * (OZ1[(sr + 2) * SC + sc] - OZ1[(sr - 1) * SC + sc]);
    const float wx_d = K1 * (OX1[sr * SC + sc] - OX1[sr * SC + sc - 1]) +
                       K2 * (OX1[sr * SC + sc + 1] - OX1[sr * SC + sc - 2]);
    const bool in = !EDGE || (gi >= 0 && gi < p.nz && gj >= 0 && gj < p.nx);
    // DAS transpose: the channel at normal node jc feeds vx nodes jc (c1), jc-1 (-c1),
    // jc+1 (c2) and jc-2 (-c2) of its row
    float inj = 0.0f;
    if (L.slot >= 0)
      inj = K1 * (ebar_at(s, L.slot, gj, n) - ebar_at(s, L.slot, gj + 1, n)) +
            K2 * (ebar_at(s, L.slot, gj - 1, n) - ebar_at(s, L.slot, gj + 2, n));
    // v_bar_x += -(D+x p_bar_xx + D-z p_bar_zx); v_bar_z += -(D+z p_bar_zz + D-x p_bar_xz)
    const float gx = -(ux_d * s.rdx + uz_d * s.rdz) + dt * s.rdx * inj;
    const float gz = -(wz_d * s.rdz + wx_d * s.rdx);
    const float bx = 2.0f * rcpf(L.r0 + L.rx), bz = 2.0f * rcpf(L.r0 + L.rz);
    const float m = in ? 1.0f : 0.0f;
    const Ub u{m * (L.ux + bx * gx), m * (L.uz + bz * gz)};
    if (owned) {
      const unsigned o = pofs(p, gi, gj);
      G(p.wux, o) = u.ux;
      G(p.wuz, o) = u.uz;
    }
    return u;
  };
  // u_bar of a node into LDS; CPML tiles also the corrected q_bar operands, dt u (+ a
  // (psi_bar + dt u) inside the strips), and the owned velocity-side adjoint memory
  // variables. In CPML tiles this runs after the barrier that ends the reads of the staged
  // operands (the LDS space is reused), so only u_bar is held across it.
  auto put = [&](int vr, int lcol, const Ub& u, bool owned) {
    UX[vr * VC + lcol] = u.ux;
    UZ[vr * VC + lcol] = u.uz;
    if (PML) {
      const int gi = i0 - 2 + vr, gj = j0 - 2 + lcol;
      const bool in = gi >= 0 && gi < p.nz && gj >= 0 && gj < p.nx;
      const float m = in ? 1.0f : 0.0f;
      const int ic = min(max(gi, 0), p.nz - 1), jc = min(max(gj, 0), p.nx - 1);
      const int sx = strip_index(jc, p.nx, s.P), sz = strip_index(ic, p.nz, s.P);
      // velocity-side adjoint memory variables of step n + 1
      const unsigned qx = (unsigned)(ic * p.P2 + max(sx, 0)), qz = (unsigned)(max(sz, 0) * p.nx + jc);
      const float q1 = G(p.rps, xv(p, X_VXX) + qx);
      const float q2 = G(p.rps, xv(p, X_VZX) + qx);
      const float q3 = G(p.rps, zv(p, Z_VXZ) + qz);
      const float q4 = G(p.rps, zv(p, Z_VZZ) + qz);
      const float mx = sx >= 0 ? 1.0f : 0.0f, mz = sz >= 0 ? 1.0f : 0.0f;
      const float dux = dt * u.ux, duz = dt * u.uz;
      QXA[vr * VC + lcol] = m * (dux + (mx * G(p.prof, xp(p, 2) + (unsigned)jc)) * (q1 + dux));
      QZA[vr * VC + lcol] = m * (duz + (mx * G(p.prof, xp(p, 0) + (unsigned)jc)) * (q2 + duz));
      QXB[vr * VC + lcol] = m * (dux + (mz * G(p.prof, zp(p, 0) + (unsigned)ic)) * (q3 + dux));
      QZB[vr * VC + lcol] = m * (duz + (mz * G(p.prof, zp(p, 2) + (unsigned)ic)) * (q4 + duz));
      if (owned) {
        if (sx >= 0) {
          const unsigned q = (unsigned)(gi * p.P2 + sx);
          G(p.wps, xv(p, X_VXX) + q) = G(p.prof, xp(p, 3) + (unsigned)gj) * (q1 + dt * u.ux);
          G(p.wps, xv(p, X_VZX) + q) = G(p.prof, xp(p, 1) + (unsigned)gj) * (q2 + dt * u.uz);
        }
        if (sz >= 0) {
          const unsigned q = (unsigned)(sz * p.nx + gj);
          G(p.wps, zv(p, Z_VXZ) + q) = G(p.prof, zp(p, 1) + (unsigned)gi) * (q3 + dt * u.ux);
          G(p.wps, zv(p, Z_VZZ) + q) = G(p.prof, zp(p, 3) + (unsigned)gi) * (q4 + dt * u.uz);
        }
      }
    }
  };
  Ub uo[NV];
  bool own[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int vr = tyu + k * BZ, gi = i0 - 2 + vr;
    own[k] = gi >= i0 && gi < i0 + TZ && (!EDGE || (gi < p.nz && j0 + tx < p.nx));
    uo[k] = ubar(vr, tx + 2, UL[k], own[k]);
  }
  const bool has_halo = (tid >> 2) < VR;
  Ub ho{0.0f, 0.0f};
  if (has_halo) ho = ubar(hv, hcol, UH, false);
  if (PML) __syncthreads();   // every thread is done reading the staged operands
#pragma unroll
  for (int k = 0; k < NV; ++k) put(ty + k * BZ, tx + 2, uo[k], own[k]);
  if (has_halo) put(hv, hcol, ho, false);
  __syncthreads();

  // ---- 3. t_bar, memory variables and imaging at the tile's normal nodes (their loads
  //         issued here, after the velocity phase, to bound the live registers) ----
  TbLoads TL[NSR];
#pragma unroll
  for (int k = 0; k < NSR; ++k) TL[k] = tb_loads<GRAD, PML, EDGE, VTI>(p, s, i0 + tyu + k * BZ, j0 + tx, first);
#pragma unroll
  for (int k = 0; k < NSR; ++k) {
    const int i = i0 + tyu + k * BZ, j = j0 + tx;
    if (EDGE && (i >= p.nz || j >= p.nx)) continue;
    const TbLoads& L = TL[k];
    const int ow = (tyu + k * BZ) * BX + tx;
    const float txx = TO[ow], tzz = TO[TZ * BX + ow], txz = TO[2 * TZ * BX + ow];
    const int vr = tyu + k * BZ + 2, vc = tx + 2;   // LDS u coordinates of the node
    const int u0 = vr * VC + vc;
    // q operands: interior tiles read dt u_bar directly
    auto qxa = [&](int d) { return PML ? QXA[u0 + d] : dt * UX[u0 + d]; };
    auto qxb = [&](int d) { return PML ? QXB[u0 + d] : dt * UX[u0 + d]; };
    auto qza = [&](int d) { return PML ? QZA[u0 + d] : dt * UZ[u0 + d]; };
    auto qzb = [&](int d) { return PML ? QZB[u0 + d] : dt * UZ[u0 + d]; };
    const float txx_d = K1 * (qxa(0) - qxa(-1)) + K2 * (qxa(1) - qxa(-2));
    const float tzz_d = K1 * (qzb(0) - qzb(-VC)) + K2 * (qzb(VC) - qzb(-2 * VC));
    const float t1 = K1 * (qxb(VC) - qxb(0)) + K2 * (qxb(2 * VC) - qxb(-VC));
    const float t2 = K1 * (qza(1) - qza(0)) + K2 * (qza(2) - qza(-1));
    // sigma_bar_xx += -D-x q_bar_xa ; sigma_bar_zz += -D-z q_bar_zb ;
    // sigma_bar_xz += -(D+z q_bar_xb + D+x q_bar_za)
    const float dsxx = -txx_d * s.rdx, dszz = -tzz_d * s.rdz, dsxz = -(t1 * s.rdz + t2 * s.rdx);
    const float mu = L.mu, lam = L.lam, l2m = lam + 2.0f * mu;
    const float mxz = 4.0f * rcpf(rcpf(mu) + rcpf(L.mu_x) + rcpf(L.mu_z) + rcpf(L.mu_xz));
    const unsigned o = pofs(p, i, j);
    if (PML) {  // owned stress-side adjoint memory variables, from t_bar of step n + 1
      const int sx = strip_index(j, p.nx, s.P), sz = strip_index(i, p.nz, s.P);
      if (sx >= 0) {
        const unsigned q = (unsigned)(i * p.P2 + sx);
        const float r1 = G(p.rps, xv(p, X_XX) + q), r2 = G(p.rps, xv(p, X_XZ) + q);
        G(p.wps, xv(p, X_XX) + q) = G(p.prof, xp(p, 1) + (unsigned)j) * (r1 + dt * txx);
        G(p.wps, xv(p, X_XZ) + q) = G(p.prof, xp(p, 3) + (unsigned)j) * (r2 + dt * txz);
      }
      if (sz >= 0) {
        const unsigned q = (unsigned)(sz * p.nx + j);
        const float r3 = G(p.rps, zv(p, Z_ZZ) + q), r4 = G(p.rps, zv(p, Z_XZ) + q);
        G(p.wps, zv(p, Z_ZZ) + q) = G(p.prof, zp(p, 1) + (unsigned)i) * (r3 + dt * tzz);
        G(p.wps, zv(p, Z_XZ) + q) = G(p.prof, zp(p, 3) + (unsigned)i) * (r4 + dt * txz);
      }
    }
    const float c11 = VTI ? L.c11 : l2m, c13 = VTI ? L.c13 : lam;
    G(p.wtxx, o) = txx + (c11 * dsxx + c13 * dszz);
    G(p.wtzz, o) = tzz + (c13 * dsxx + l2m * dszz);
    G(p.wtxz, o) = txz + mxz * dsxz;
    if (GRAD) {
      const unsigned cc = (unsigned)(i * s.cp + j), cells = (unsigned)s.cells;
      float e = VTI ? 0.0f : (txx - tzz) * L.h1;
      const int so = (vr + 2) * SC + tx + 4;   // LDS p_bar coordinates of the node
      const float rdt = 1.0f / dt;
      for (int q = 0; q < 4; ++q) {
        // the same arithmetic either way (the staged operand is dt t_bar_xz), so the result
        // does not depend on which tiles take the CPML path
        const int a = max(i - 1 + (q >> 1), 0), b = max(j - 1 + (q & 1), 0);
        const float txz = rdt * (PML ? dt * G(p.txz, pofs(p, a, b)) : OX1[so + ((q >> 1) - 1) * SC + (q & 1) - 1]);
        e += L.c2[q] * txz * L.h2[q];
      }
      // vx nodes (i, j-1/2), (i, j+1/2) and vz nodes (i-1/2, j), (i+1/2, j) around rho(i, j)
      const float c0 = EDGE ? (float)pair_count(j - 1, j, p.nx) : 1.0f;
      const float c1 = EDGE ? (float)pair_count(j, j, p.nx) : 1.0f;
      const float c2 = EDGE ? (float)pair_count(i - 1, i, p.nz) : 1.0f;
      const float c3 = EDGE ? (float)pair_count(i, i, p.nz) : 1.0f;
      float r = c0 * UX[u0 - 1] * L.h3m;
      r += c1 * UX[u0] * L.h3;
      r += c2 * UZ[u0 - VC] * L.h4m;
      r += c3 * UZ[u0] * L.h4;
      if (VTI) {  // sigma_bar = C^-1 t_bar on the normal block: (u, v) / det, det in h0, h1
        const float u = l2m * txx - c13 * tzz, v = c11 * tzz - c13 * txx;
        G(p.acc, cc) = L.a0 + dt * u * L.h0;                         // c11
        G(p.acc, 3 * cells + cc) = L.a3 + dt * v * L.h1;             // c33
        G(p.acc, 4 * cells + cc) = L.a4 + dt * (u * L.h1 + v * L.h0);  // c13
      } else {
        G(p.acc, cc) = L.a0 + dt * (txx + tzz) * L.h0;
      }
      G(p.acc, cells + cc) = L.a1 + dt * e;
      G(p.acc, 2 * cells + cc) = L.a2 - dt * r;
    }
    if (SRCADJ && i == s.si && j == s.sj) {
      // sigma_bar at the source from t_bar of step n + 1: invert the 2x2 normal block and
      // the shear moduli of the four shear nodes around the source
      const float det = VTI ? c11 * l2m - c13 * c13 : (l2m - lam) * (l2m + lam);
      const float sb0 = (l2m * txx - c13 * tzz) / det, sb1 = (c11 * tzz - c13 * txx) / det;
      float sb2 = 0.0f;
      for (int a = i - 1; a <= i; ++a) {
        for (int b = j - 1; b <= j; ++b) {
          const unsigned oo = pofs(p, a, b);
          const float m4 = 4.0f * rcpf(rcpf(G(p.mu, oo)) + rcpf(G(p.mu, oo + 1)) + rcpf(G(p.mu, oo + p.ld)) +
                                       rcpf(G(p.mu, oo + p.ld + 1)));
          sb2 += m4 > 0.0f ? G(p.txz, oo) / m4 : 0.0f;
        }
      }
      s.src_bar[n] = -s.w * sb0;
      s.src_bar[s.nt + n] = -s.w * sb1;
      s.src_bar[2 * s.nt + n] = -0.25f * s.w * sb2;
    }
  }
}

template <int TZ, bool GRAD, bool SRCADJ, bool VTI>
__global__ __launch_bounds__(BX * BZ) void k_adj_step(STEP_PARAMS, int n, int kseg, int first) {
  __shared__ float lds[AdjTile<TZ>::LDS_FLOATS];
  const StepSlot slot = slots[blockIdx.x];
  if (slot.shot < 0) return;
  const Shot2D& s = shots[slot.shot];
  const int i0 = slot.i0, j0 = slot.j0;
  // block-uniform branch: every thread reaches the barriers. The staged p_bar operands
  // reach 4 nodes beyond the tile, so tiles within 4 nodes of a strip take the CPML path;
  // with strips at all four edges every other tile and its 4-node halo lie inside the
  // grid and skip the edge handling (only a grid without strips needs it there).
  if (slot.path == PATH_PML) adj_step_tile<TZ, GRAD, SRCADJ, true, true, VTI>(s, i0, j0, n, kseg, first != 0, lds);
  else if (slot.path == PATH_EDGE)
    adj_step_tile<TZ, GRAD, SRCADJ, false, true, VTI>(s, i0, j0, n, kseg, first != 0, lds);
  else adj_step_tile<TZ, GRAD, SRCADJ, false, false, VTI>(s, i0, j0, n, kseg, first != 0, lds);
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
  // VTI (Thomsen eps, delta = eps / 2): c11 = c33 (1 + 2 eps),
  // c13 = sqrt((c33 - mu)(c33 (1 + 2 delta) - mu)) - mu, from the FP32 c33 and mu in FP64
  float c11 = 0.0f, c13 = 0.0f;
  if (s.meps) {
    const double c33 = (double)lam + 2.0 * (double)mu, eps = s.meps[mo], m = mu;
    c11 = (float)(c33 * (1.0 + 2.0 * eps));
    c13 = (float)(sqrt(fmax((c33 - m) * (c33 * (1.0 + eps) - m), 0.0)) - m);
  }
  const long o = (long)i * s.ld + j;
  const bool xe = j == s.nx - 1, ze = i == s.nz - 1;
  for (int c = 0; c < 4; ++c) {
    const bool dx = c & 1, dz = c >> 1;
    if ((dx && !xe) || (dz && !ze)) continue;
    const long oc = o + (dx ? 1 : 0) + (dz ? s.ld : 0);
    s.lam[oc] = lam;
    s.mu[oc] = mu;
    s.rho[oc] = rho;
    if (s.meps) {
      s.c11[oc] = c11;
      s.c13[oc] = c13;
    }
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
  // the model and the FP64 sums are touched once per flush: streaming accesses keep them
  // from displacing the time-step state in the caches
  const double vp = __builtin_nontemporal_load(s.mvp + mo), vs = __builtin_nontemporal_load(s.mvs + mo);
  const double rho = __builtin_nontemporal_load(s.mrho + mo);
  const double mu = rho * vs * vs;
  gdouble* G0 = s.G + cc;
  gdouble* G1 = s.G + s.cells + cc;
  gdouble* G2 = s.G + 2 * s.cells + cc;
  const double g0 = __builtin_nontemporal_load(G0), g1 = __builtin_nontemporal_load(G1);
  const double g2 = __builtin_nontemporal_load(G2);
  if (s.meps) {
    // VTI at fixed eps: sums of c11, c33, c13 at the node; c13 = R - mu with
    // R^2 = (c33 - mu)(c33 (1 + eps) - mu) moves with c33 and mu; the shear sum E / mu^2
    // and the buoyancy sum as in the isotropic case
    const double eps = __builtin_nontemporal_load(s.meps + mo);
    const double c33 = rho * vp * vp, A = c33 - mu, B = c33 * (1.0 + eps) - mu, R = sqrt(fmax(A * B, 0.0));
    const double d33 = R > 0.0 ? (B + A * (1.0 + eps)) / (2.0 * R) : 0.0;
    const double dmu = (R > 0.0 ? -(A + B) / (2.0 * R) : 0.0) - 1.0;
    const double a11 = s.acc[cc], a33 = s.acc[3 * s.cells + cc], a13 = s.acc[4 * s.cells + cc];
    const double g33 = a33 + (1.0 + 2.0 * eps) * a11 + d33 * a13;
    const double gm = (mu > 0.0 ? (double)s.acc[s.cells + cc] / (mu * mu) : 0.0) + dmu * a13;
    __builtin_nontemporal_store(g0 + 2.0 * rho * vp * g33, G0);
    __builtin_nontemporal_store(g1 + 2.0 * rho * vs * gm, G1);
    __builtin_nontemporal_store(g2 + (vp * vp * g33 + vs * vs * gm + (double)s.acc[2 * s.cells + cc]), G2);
    return;
  }
  const double gl = s.acc[cc];
  const double gmu = gl + (mu > 0.0 ? (double)s.acc[s.cells + cc] / (mu * mu) : 0.0);
  __builtin_nontemporal_store(g0 + 2.0 * rho * vp * gl, G0);
  __builtin_nontemporal_store(g1 + 2.0 * rho * vs * (gmu - 2.0 * gl), G1);
  __builtin_nontemporal_store(g2 + ((vp * vp - 2.0 * vs * vs) * gl + vs * vs * gmu + (double)s.acc[2 * s.cells + cc]),
                              G2);
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
// e_bar[n][c] = sum_{k >= n} r[c][k], r = d - d_obs. A block takes RES_T channels and walks
// the time axis from the end in tiles of RES_T samples: the tile is read along time
// (coalesced; d and e_bar are [nch][nt] and [nt][nch]), its residuals transposed through
// LDS in FP64, summed by one thread per channel in the order of a serial reverse sum (so the
// sums do not depend on the tiling), and written along the channels. The per-channel FP64
// partial sums of r^2 are reduced in a fixed order by a single block.
// ------------------------------------------------------------------------------------
constexpr int RES_T = 64;
__global__ __launch_bounds__(256) void k_residual(const float* d, const float* dobs, int nch, int nt,
                                                  double* partial, float* ebar) {
  // sample-major ([sample][channel]): the sequential scan below, one channel per lane,
  // then reads consecutive addresses across the wave (bank-conflict free)
  __shared__ double tile[RES_T][RES_T + 1];
  const int c0 = blockIdx.x * RES_T, tid = threadIdx.x;
  constexpr int ROWS = 256 / RES_T;   // channels (loads) or samples (stores) per pass of the block
  double acc = 0.0, sq = 0.0;         // of channel c0 + tid, in threads tid < RES_T
  for (int t0 = (nt - 1) / RES_T * RES_T; t0 >= 0; t0 -= RES_T) {
    // every load in bounds (index clamped, the value then kept or zeroed), so that the
    // loads of a pass issue together instead of one branch and round trip each
    for (int k = 0; k < RES_T / ROWS; ++k) {
      const int ch = tid / RES_T + ROWS * k, sm = tid % RES_T, c = c0 + ch, t = t0 + sm;
      const long e = (long)min(c, nch - 1) * nt + min(t, nt - 1);
      const double r = dobs ? (double)d[e] - (double)dobs[e] : (double)d[e];
      tile[sm][ch] = (c < nch && t < nt) ? r : 0.0;
    }
    __syncthreads();
    if (tid < RES_T) {
      for (int sm = RES_T - 1; sm >= 0; --sm) {   // samples past nt hold r = 0 and change nothing
        const double r = tile[sm][tid];
        sq += r * r;
        acc += r;
        tile[sm][tid] = acc;
      }
    }
    __syncthreads();
    for (int k = 0; k < RES_T / ROWS; ++k) {
      const int sm = tid / RES_T + ROWS * k, ch = tid % RES_T, c = c0 + ch, t = t0 + sm;
      if (c < nch && t < nt) ebar[(long)t * nch + c] = (float)tile[sm][ch];
    }
    __syncthreads();
  }
  if (partial && tid < RES_T && c0 + tid < nch) partial[c0 + tid] = sq;
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

}  // namespace

hipError_t launch_stage2d(const Batch2D& b, hipStream_t st) {
  k_stage<<<grid_of(b.fwd), block2d(), 0, st>>>(FWD_ARGS);
  return hipGetLastError();
}

#define STEP_ARGS b.shots, b.step.slot
#define ADJSTEP_ARGS b.shots, b.adj_step.slot

namespace {

template <int TZ, bool VTI>
void fwd_step_launch(const Batch2D& b, int n, int kstore, bool record, hipStream_t st) {
  const dim3 g(b.step.n);
  if (kstore >= 0) {
    if (record) k_fwd_step<TZ, true, true, false, VTI><<<g, block2d(), 0, st>>>(STEP_ARGS, n, kstore);
    else k_fwd_step<TZ, true, false, false, VTI><<<g, block2d(), 0, st>>>(STEP_ARGS, n, kstore);
  } else {
    if (record) k_fwd_step<TZ, false, true, false, VTI><<<g, block2d(), 0, st>>>(STEP_ARGS, n, 0);
    else k_fwd_step<TZ, false, false, false, VTI><<<g, block2d(), 0, st>>>(STEP_ARGS, n, 0);
  }
}

template <int TZ, bool VTI>
void adj_step_launch(const Batch2D& b, int n, int k, bool grad, bool first, bool srcadj, hipStream_t st) {
  const dim3 g(b.adj_step.n);
  if (grad) k_adj_step<TZ, true, false, VTI><<<g, block2d(), 0, st>>>(ADJSTEP_ARGS, n, k, first);
  else if (srcadj) k_adj_step<TZ, false, true, VTI><<<g, block2d(), 0, st>>>(ADJSTEP_ARGS, n, 0, 0);
  else k_adj_step<TZ, false, false, VTI><<<g, block2d(), 0, st>>>(ADJSTEP_ARGS, n, 0, 0);
}

template <bool VTI>
void fwd_acorr_launch(const Batch2D& b, int n, hipStream_t st) {
  const dim3 g(b.step.n);
  switch (b.fwd_rows) {
    case 8: k_fwd_step<8, false, false, true, VTI><<<g, block2d(), 0, st>>>(STEP_ARGS, n, 0); break;
    case 12: k_fwd_step<12, false, false, true, VTI><<<g, block2d(), 0, st>>>(STEP_ARGS, n, 0); break;
    default: k_fwd_step<16, false, false, true, VTI><<<g, block2d(), 0, st>>>(STEP_ARGS, n, 0); break;
  }
}

}  // namespace

hipError_t launch_fwd_step(const Batch2D& b, int n, int kstore, bool record, hipStream_t st) {
  switch (b.fwd_rows) {
    case 8: b.vti ? fwd_step_launch<8, true>(b, n, kstore, record, st) : fwd_step_launch<8, false>(b, n, kstore, record, st); break;
    case 12: b.vti ? fwd_step_launch<12, true>(b, n, kstore, record, st) : fwd_step_launch<12, false>(b, n, kstore, record, st); break;
    case 16: b.vti ? fwd_step_launch<16, true>(b, n, kstore, record, st) : fwd_step_launch<16, false>(b, n, kstore, record, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fwd_acorr(const Batch2D& b, int n, hipStream_t st) {
  if (b.fwd_rows != 8 && b.fwd_rows != 12 && b.fwd_rows != 16) return hipErrorInvalidValue;
  if (b.vti) fwd_acorr_launch<true>(b, n, st);
  else fwd_acorr_launch<false>(b, n, st);
  return hipGetLastError();
}

hipError_t launch_adj_step(const Batch2D& b, int n, int k, bool grad, bool first, bool srcadj, hipStream_t st) {
  switch (b.adj_rows) {
    case 8:
      b.vti ? adj_step_launch<8, true>(b, n, k, grad, first, srcadj, st)
            : adj_step_launch<8, false>(b, n, k, grad, first, srcadj, st);
      break;
    case 12:
      b.vti ? adj_step_launch<12, true>(b, n, k, grad, first, srcadj, st)
            : adj_step_launch<12, false>(b, n, k, grad, first, srcadj, st);
      break;
    case 16:
      b.vti ? adj_step_launch<16, true>(b, n, k, grad, first, srcadj, st)
            : adj_step_launch<16, false>(b, n, k, grad, first, srcadj, st);
      break;
    default: return hipErrorInvalidValue;
  }
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
  if (nch > 0) k_residual<<<(nch + RES_T - 1) / RES_T, 256, 0, st>>>(d, dobs, nch, nt, partial, ebar);
  k_reduce_phi<<<1, 256, 0, st>>>(partial, nch > 0 ? nch : 0, phi);
  return hipGetLastError();
}

hipError_t launch_residual_cumsum_raw(int nch, int nt, const float* r, float* ebar, hipStream_t st) {
  if (nch > 0) k_residual<<<(nch + RES_T - 1) / RES_T, 256, 0, st>>>(r, nullptr, nch, nt, nullptr, ebar);
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
