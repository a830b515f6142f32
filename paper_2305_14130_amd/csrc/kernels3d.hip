// 3D isotropic elastic velocity-stress kernels for gfx950: forward, exact transpose (in
// scaled adjoint variables), imaging condition, chain rule. The 3D counterpart of
// kernels2d.hip (Forward problem eqs.(1)-(3); Solving the inverse problem eqs.(4),(6);
// Model extension eq.(8)).
//
// Staggering: sxx, syy, szz at (i, k, j); vx (i, k, j+1/2); vy (i, k+1/2, j);
// vz (i+1/2, k, j); sxy (i, k+1/2, j+1/2); sxz (i+1/2, k, j+1/2); syz (i+1/2, k+1/2, j).
// i = z, k = y, j = x. 4th-order differences, zero outside the grid (zero halo), leapfrog,
// unsplit CPML (kappa = 1) with memory variables in strips on every face.
//
// Tiles are 64 (x) by 16 (y) cells of one z plane, four rows per thread. The adjoint
// carries u_bar = b v_bar and t_bar = C sigma_bar (C: lambda 1 1^T + 2 mu I on the normal
// block, the shear moduli on the shear components), so its transposed differences read one
// array per neighbour. The imaging condition gathers three sums at each normal node from
// forward quantities stored with the factors of the chain rule already applied, so that
// the transposed kernels read and write three sums per cell and step instead of one per
// modulus and buoyancy:
//   A += dt tr(t) tr(p) / (3l + 2m)                           g_lambda = A
//   E += dt dev(t) : (m dev(p)) + dt sum_s c_s t_xy(s) (mu_xy(s) / 4) (D+y vx + D+x vy)(s)
//        (and xz, yz)                                          g_mu = 2/3 A + E / m^2
//   R += dt sum_v c_v u_x(v) (b_x(v) / 2) q_x(v)  (and y, z)   g_rho = -R
// over the four shear nodes s of each type and the two velocity nodes v of each component
// whose harmonic modulus or buoyancy uses the node's mu or rho, c counting how often (twice
// at the last plane, row or column, where the neighbour is clamped): d mu_xy / d mu =
// mu_xy^2 / (4 mu^2) per corner and d b / d rho = -b^2 / 2.
#include "efwi_internal.h"

// Contract a * b + c into one fused multiply-add only inside a single expression, never
// across statements: every template instance of a kernel then rounds the same source the
// same way, so runs that differ only in what they store stay bitwise identical.
#pragma clang fp contract(on)

namespace efwi {
namespace {

constexpr float K1 = 1.125f;
constexpr float K2 = -0.041666666666666664f;
constexpr int TX = TILE3_X, TY = TILE3_TY;

// Strip slots. x-strips: vx(D+x sxx) vy(D-x sxy) vz(D-x sxz) pxx(D-x vx) sxy(D+x vy) sxz(D+x vz)
enum { XS_VX = 0, XS_VY, XS_VZ, XS_PXX, XS_SXY, XS_SXZ };
// y-strips: vx(D-y sxy) vy(D+y syy) vz(D-y syz) pyy(D-y vy) sxy(D+y vx) syz(D+y vz)
enum { YS_VX = 0, YS_VY, YS_VZ, YS_PYY, YS_SXY, YS_SYZ };
// z-strips: vx(D-z sxz) vy(D-z syz) vz(D+z szz) pzz(D-z vz) sxz(D+z vx) syz(D+z vy)
enum { ZS_VX = 0, ZS_VY, ZS_VZ, ZS_PZZ, ZS_SXZ, ZS_SYZ };
// profile tables: 0 a_int, 1 b_int, 2 a_half, 3 b_half (D- uses int, D+ uses half)
__device__ __forceinline__ const gfloat* px_(const Shot3D& s, int w) { return s.prof + w * s.nx; }
__device__ __forceinline__ const gfloat* py_(const Shot3D& s, int w) { return s.prof + 4 * s.nx + w * s.ny; }
__device__ __forceinline__ const gfloat* pz_(const Shot3D& s, int w) { return s.prof + 4 * s.nx + 4 * s.ny + w * s.nz; }

// Field accesses in the cell functions: a uniform base pointer at the padded plane's origin
// (PF) plus a non-negative 32-bit element offset (cell_ofs), so that a load is a scalar base
// and a 32-bit lane offset rather than per-lane 64-bit address arithmetic. Offsets stay far
// below 2^30 elements at the sizes the plans allow.
__device__ __forceinline__ long org3(const Shot3D& s) { return (long)HALO * s.pz + (long)HALO * s.ld + XOFF; }
#define PF(f) ((f) - org3(s))
__device__ __forceinline__ unsigned cell_ofs(const Shot3D& s, int i, int k, int j) {
  return (unsigned)(i + HALO) * (unsigned)s.pz + (unsigned)(k + HALO) * (unsigned)s.ld + (unsigned)(XOFF + j);
}
// Element e of a global array as a 32-bit byte offset from a uniform base (the form the
// hardware's scalar-base global loads and stores take; e < 2^30, checked on the host).
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

template <class P>
__device__ __forceinline__ float dplus(P f, unsigned o, unsigned st, float r) {
  return (K1 * (G(f, o + st) - G(f, o)) + K2 * (G(f, o + 2 * st) - G(f, o - st))) * r;
}
template <class P>
__device__ __forceinline__ float dminus(P f, unsigned o, unsigned st, float r) {
  return (K1 * (G(f, o) - G(f, o - st)) + K2 * (G(f, o + st) - G(f, o - 2 * st))) * r;
}

// Element offsets into the strip arrays (32-bit: a strip array holds far fewer than 2^30
// elements at the sizes the plans allow).
__device__ __forceinline__ unsigned xq(const Shot3D& s, int i, int k, int sx) {
  return ((unsigned)i * (unsigned)s.ny + (unsigned)k) * (2u * (unsigned)s.P) + (unsigned)sx;
}
__device__ __forceinline__ unsigned yq(const Shot3D& s, int i, int sy, int j) {
  return ((unsigned)i * (2u * (unsigned)s.P) + (unsigned)sy) * (unsigned)s.nx + (unsigned)j;
}
__device__ __forceinline__ unsigned zq(const Shot3D& s, int sz, int k, int j) {
  return ((unsigned)sz * (unsigned)s.ny + (unsigned)k) * (unsigned)s.nx + (unsigned)j;
}
// Strip node of coordinate k on an axis of n nodes (strip_index), clamped into 0 .. 2P-1 so
// that it always addresses the strip arrays; `in` tells whether k lies in a strip of the
// grid. The CPML code reads the strip arrays at the clamped node unconditionally and keeps
// the result only where `in` holds: no load sits in a (divergent) branch, so a cell's loads
// are issued together instead of one memory round trip per branch. Only the CPML code paths
// call it, which run only when the strips exist (P > 0, see pml_axes).
__device__ __forceinline__ int strip_clamp(int k, int n, int P, bool& in) {
  const bool lo = k < P, hi = k >= n - P;
  in = (lo && k >= 0) || (hi && k < n);
  const int sk = lo ? k : k - (n - 2 * P);
  return min(max(sk, 0), 2 * P - 1);
}

// Which axes' CPML strips a tile's cells (widened by pad on every side) reach: bit 0 x,
// bit 1 y, bit 2 z.
__device__ __forceinline__ int pml_axes(const Shot3D& s, int i, int k0, int j0, int pad) {
  if (s.P <= 0) return 0;
  const bool x = (j0 - pad < s.P) || (j0 + TX - 1 + pad >= s.nx - s.P);
  const bool y = (k0 - pad < s.P) || (k0 + TILE3_Y - 1 + pad >= s.ny - s.P);
  const bool z = (i - pad < s.P) || (i + pad >= s.nz - s.P);
  return (x ? 1 : 0) | (y ? 2 : 0) | (z ? 4 : 0);
}
#define DISPATCH_AXES(m, CALL)          \
  switch (m) {                          \
    case 0: CALL(false, false, false); break; \
    case 1: CALL(true, false, false); break;  \
    case 2: CALL(false, true, false); break;  \
    case 3: CALL(true, true, false); break;   \
    case 4: CALL(false, false, true); break;  \
    case 5: CALL(true, false, true); break;   \
    case 6: CALL(false, true, true); break;   \
    default: CALL(true, true, true); break;   \
  }

// Tile of schedule slot blockIdx.x (tile order: tile3_coords). Schedule as in 2D.
__device__ __forceinline__ bool tile3(const int* __restrict__ sched, const int* __restrict__ tile_shot,
                                      const int* __restrict__ tile_first, const Shot3D* __restrict__ shots, int& sh,
                                      int& i, int& k0, int& j0) {
  const int t = sched[blockIdx.x];
  if (t < 0) return false;
  sh = tile_shot[t];
  tile3_coords(t - tile_first[sh], shots[sh].nz, shots[sh].ny, shots[sh].nx, i, k0, j0);
  return true;
}

// The transposed kernels pass the row k through readfirstlane: a wave is one row of a tile
// (64 x 4 workgroups, four rows per thread), so k is the same in every lane, and saying so
// lets the compiler keep the row's addresses and y-profile values in scalar registers
// (transposed velocity 1.54 -> 1.47 ms, 125 -> 116 VGPRs; the forward kernels were 1-2%
// slower with it).
#define PARAMS3                                                                                      \
  const Shot3D* __restrict__ shots, const int* __restrict__ tile_shot, const int* __restrict__ tile_first, \
      const int* __restrict__ sched
// The tile, then a loop over the thread's rows k of it: the kernel body that follows is the
// loop's body (a row beyond the grid ends the thread, as every later row is beyond it too).
#define TILE3()                                                                                       \
  int sh_, i, k0, j0;                                                                                  \
  if (!tile3(sched, tile_shot, tile_first, shots, sh_, i, k0, j0)) return;                            \
  const Shot3D& s = shots[sh_];                                                                        \
  const int j = j0 + threadIdx.x;                                                                      \
  _Pragma("unroll 1") for (int k = k0 + (int)threadIdx.y; k < k0 + TILE3_Y; k += TILE3_TY)

// Streaming (non-temporal) accesses of the history: written once per forward step, read
// once in the reverse sweep, so they should not displace the wavefields in the caches.
__device__ __forceinline__ void hist_put(gfloat* base, unsigned e, float v) {
  typedef __attribute__((address_space(1))) char gchar;
  __builtin_nontemporal_store(v, (gfloat*)((gchar*)base + e * 4u));
}
__device__ __forceinline__ float hist_get(const gfloat* base, unsigned e) {
  typedef const __attribute__((address_space(1))) char gchar;
  return __builtin_nontemporal_load((const gfloat*)((gchar*)base + e * 4u));
}

// Harmonic mean of the four shear moduli around a shear node (0 if any is 0), and the
// buoyancy between two normal nodes. The staging kernel and the step kernels evaluate the
// shear moduli by the same expressions on the same FP32 values, so the derived moduli are
// bitwise the staged ones that the transposed stress kernel reads.
__device__ __forceinline__ float harm4(float a, float b, float c, float d) {
  return (a > 0.f && b > 0.f && c > 0.f && d > 0.f) ? 4.0f / (1.0f / a + 1.0f / b + 1.0f / c + 1.0f / d) : 0.0f;
}
__device__ __forceinline__ float buoy(float r0, float r1) { return 2.0f / (r0 + r1); }
// Derived parameters of cell offset o from the padded rho and mu arrays (see Shot3D).
__device__ __forceinline__ void buoyancies(const Shot3D& s, unsigned o, float& bx, float& by, float& bz) {
  const gfloat* r = PF(s.rho);
  const float r0 = G(r, o);
  bx = buoy(r0, G(r, o + 1u));
  by = buoy(r0, G(r, o + (unsigned)s.ld));
  bz = buoy(r0, G(r, o + (unsigned)s.pz));
}
__device__ __forceinline__ void shear_moduli(const Shot3D& s, unsigned o, float& mxy, float& mxz, float& myz) {
  const gfloat* m = PF(s.mu);
  const unsigned ld = (unsigned)s.ld, pz = (unsigned)s.pz;
  const float m0 = G(m, o), mx = G(m, o + 1u), my = G(m, o + ld), mz = G(m, o + pz);
  mxy = harm4(m0, my, mx, G(m, o + ld + 1u));
  mxz = harm4(m0, mz, mx, G(m, o + pz + 1u));
  myz = harm4(m0, mz, my, G(m, o + pz + ld));
}

// Every cell function below reads all it needs before its first store: the compiler cannot
// prove that the arrays do not alias, so a load placed after a store would cost another
// memory round trip per wavefront.

// CPML memory variable at an owned node: psi <- b psi + a D computed from the old value
// (read with the cell's other inputs, before any store) into p; returns D + psi. The caller
// stores p after the cell's field updates.
__device__ __forceinline__ float cpml_new(const gfloat* psi, unsigned q, const gfloat* a, const gfloat* b, int c,
                                          float d, float& p) {
  p = b[c] * G(psi, q) + a[c] * d;
  return d + p;
}

// ------------------------------------------------------------------------------------
// Forward velocity half step.
// ------------------------------------------------------------------------------------
template <bool STORE, bool PX, bool PY, bool PZ>
__device__ __forceinline__ void fwd_vel3(const Shot3D& s, int i, int k, int j, gfloat* seg) {
  const unsigned ld = (unsigned)s.ld, pz = (unsigned)s.pz;
  const unsigned o = cell_ofs(s, i, k, j);
  float a1 = dplus(PF(s.sxx), o, 1u, s.rdx), a2 = dminus(PF(s.sxy), o, ld, s.rdy), a3 = dminus(PF(s.sxz), o, pz, s.rdz);
  float b1 = dminus(PF(s.sxy), o, 1u, s.rdx), b2 = dplus(PF(s.syy), o, ld, s.rdy), b3 = dminus(PF(s.syz), o, pz, s.rdz);
  float c1 = dminus(PF(s.sxz), o, 1u, s.rdx), c2 = dminus(PF(s.syz), o, ld, s.rdy), c3 = dplus(PF(s.szz), o, pz, s.rdz);
  const float vx = G(PF(s.vx), o), vy = G(PF(s.vy), o), vz = G(PF(s.vz), o);
  float bx, by, bz;
  buoyancies(s, o, bx, by, bz);
  bool inx = false, iny = false, inz = false;
  unsigned qxs = 0, qys = 0, qzs = 0;
  float p[9];
  if (PX) {
    qxs = xq(s, i, k, strip_clamp(j, s.nx, s.P, inx));
    const float ta = cpml_new(s.psx[XS_VX], qxs, px_(s, 2), px_(s, 3), j, a1, p[0]);
    const float tb = cpml_new(s.psx[XS_VY], qxs, px_(s, 0), px_(s, 1), j, b1, p[1]);
    const float tc = cpml_new(s.psx[XS_VZ], qxs, px_(s, 0), px_(s, 1), j, c1, p[2]);
    a1 = inx ? ta : a1, b1 = inx ? tb : b1, c1 = inx ? tc : c1;
  }
  if (PY) {
    qys = yq(s, i, strip_clamp(k, s.ny, s.P, iny), j);
    const float ta = cpml_new(s.psy[YS_VX], qys, py_(s, 0), py_(s, 1), k, a2, p[3]);
    const float tb = cpml_new(s.psy[YS_VY], qys, py_(s, 2), py_(s, 3), k, b2, p[4]);
    const float tc = cpml_new(s.psy[YS_VZ], qys, py_(s, 0), py_(s, 1), k, c2, p[5]);
    a2 = iny ? ta : a2, b2 = iny ? tb : b2, c2 = iny ? tc : c2;
  }
  if (PZ) {
    qzs = zq(s, strip_clamp(i, s.nz, s.P, inz), k, j);
    const float ta = cpml_new(s.psz[ZS_VX], qzs, pz_(s, 0), pz_(s, 1), i, a3, p[6]);
    const float tb = cpml_new(s.psz[ZS_VY], qzs, pz_(s, 0), pz_(s, 1), i, b3, p[7]);
    const float tc = cpml_new(s.psz[ZS_VZ], qzs, pz_(s, 2), pz_(s, 3), i, c3, p[8]);
    a3 = inz ? ta : a3, b3 = inz ? tb : b3, c3 = inz ? tc : c3;
  }
  const float qx = a1 + a2 + a3, qy = b1 + b2 + b3, qz = c1 + c2 + c3;
  G(PF(s.vx), o) = vx + s.dt * bx * qx;
  G(PF(s.vy), o) = vy + s.dt * by * qy;
  G(PF(s.vz), o) = vz + s.dt * bz * qz;
  if (PX && inx) G(s.psx[XS_VX], qxs) = p[0], G(s.psx[XS_VY], qxs) = p[1], G(s.psx[XS_VZ], qxs) = p[2];
  if (PY && iny) G(s.psy[YS_VX], qys) = p[3], G(s.psy[YS_VY], qys) = p[4], G(s.psy[YS_VZ], qys) = p[5];
  if (PZ && inz) G(s.psz[ZS_VX], qzs) = p[6], G(s.psz[ZS_VY], qzs) = p[7], G(s.psz[ZS_VZ], qzs) = p[8];
  if (STORE) {
    const unsigned c = (unsigned)(((long)i * s.ny + k) * s.cp + j), cells = (unsigned)s.cells;
    hist_put(seg, 6 * cells + c, 0.5f * qx * bx);
    hist_put(seg, 7 * cells + c, 0.5f * qy * by);
    hist_put(seg, 8 * cells + c, 0.5f * qz * bz);
  }
}

template <bool STORE>
__global__ __launch_bounds__(TX * TY) void k3_fwd_vel(PARAMS3, int kstore) {
  TILE3() {
    if (k >= s.ny || j >= s.nx) return;
    gfloat* seg = STORE ? s.seg + (size_t)kstore * NSEG3 * s.cells : nullptr;
#define CALL(X, Y, Z) fwd_vel3<STORE, X, Y, Z>(s, i, k, j, seg)
    DISPATCH_AXES(pml_axes(s, i, k0, j0, 0), CALL);
#undef CALL
  }
}

// ------------------------------------------------------------------------------------
// Forward stress half step + six-component moment-tensor injection + DAS e_xx record.
// ------------------------------------------------------------------------------------
template <bool STORE, bool RECORD, bool PX, bool PY, bool PZ>
__device__ __forceinline__ void fwd_str3(const Shot3D& s, int i, int k, int j, int n, gfloat* seg) {
  const unsigned ld = (unsigned)s.ld, pz = (unsigned)s.pz;
  const unsigned o = cell_ofs(s, i, k, j);
  float pxx = dminus(PF(s.vx), o, 1u, s.rdx), pyy = dminus(PF(s.vy), o, ld, s.rdy), pzz = dminus(PF(s.vz), o, pz, s.rdz);
  float vx_y = dplus(PF(s.vx), o, ld, s.rdy), vy_x = dplus(PF(s.vy), o, 1u, s.rdx);
  float vx_z = dplus(PF(s.vx), o, pz, s.rdz), vz_x = dplus(PF(s.vz), o, 1u, s.rdx);
  float vy_z = dplus(PF(s.vy), o, pz, s.rdz), vz_y = dplus(PF(s.vz), o, ld, s.rdy);
  const float raw_pxx = pxx;
  const float l2m = G(PF(s.l2m), o), lam = G(PF(s.lam), o), two_mu = l2m - lam;
  float mxy, mxz, myz;
  shear_moduli(s, o, mxy, mxz, myz);
  const float sxx0 = G(PF(s.sxx), o), syy0 = G(PF(s.syy), o), szz0 = G(PF(s.szz), o), sxy0 = G(PF(s.sxy), o), sxz0 = G(PF(s.sxz), o), syz0 = G(PF(s.syz), o);
  const int slot = RECORD ? s.row_slot[(long)i * s.ny + k] : -1;
  bool inx = false, iny = false, inz = false;
  unsigned qxs = 0, qys = 0, qzs = 0;
  float p[9];
  if (PX) {
    qxs = xq(s, i, k, strip_clamp(j, s.nx, s.P, inx));
    const float ta = cpml_new(s.psx[XS_PXX], qxs, px_(s, 0), px_(s, 1), j, pxx, p[0]);
    const float tb = cpml_new(s.psx[XS_SXY], qxs, px_(s, 2), px_(s, 3), j, vy_x, p[1]);
    const float tc = cpml_new(s.psx[XS_SXZ], qxs, px_(s, 2), px_(s, 3), j, vz_x, p[2]);
    pxx = inx ? ta : pxx, vy_x = inx ? tb : vy_x, vz_x = inx ? tc : vz_x;
  }
  if (PY) {
    qys = yq(s, i, strip_clamp(k, s.ny, s.P, iny), j);
    const float ta = cpml_new(s.psy[YS_PYY], qys, py_(s, 0), py_(s, 1), k, pyy, p[3]);
    const float tb = cpml_new(s.psy[YS_SXY], qys, py_(s, 2), py_(s, 3), k, vx_y, p[4]);
    const float tc = cpml_new(s.psy[YS_SYZ], qys, py_(s, 2), py_(s, 3), k, vz_y, p[5]);
    pyy = iny ? ta : pyy, vx_y = iny ? tb : vx_y, vz_y = iny ? tc : vz_y;
  }
  if (PZ) {
    qzs = zq(s, strip_clamp(i, s.nz, s.P, inz), k, j);
    const float ta = cpml_new(s.psz[ZS_PZZ], qzs, pz_(s, 0), pz_(s, 1), i, pzz, p[6]);
    const float tb = cpml_new(s.psz[ZS_SXZ], qzs, pz_(s, 2), pz_(s, 3), i, vx_z, p[7]);
    const float tc = cpml_new(s.psz[ZS_SYZ], qzs, pz_(s, 2), pz_(s, 3), i, vy_z, p[8]);
    pzz = inz ? ta : pzz, vx_z = inz ? tb : vx_z, vy_z = inz ? tc : vy_z;
  }
  const float tr = pxx + pyy + pzz;
  const float sxy_r = vx_y + vy_x, sxz_r = vx_z + vz_x, syz_r = vy_z + vz_y;
  float sxx = sxx0 + s.dt * (lam * tr + two_mu * pxx);
  float syy = syy0 + s.dt * (lam * tr + two_mu * pyy);
  float szz = szz0 + s.dt * (lam * tr + two_mu * pzz);
  float sxy = sxy0 + s.dt * mxy * sxy_r;
  float sxz = sxz0 + s.dt * mxz * sxz_r;
  float syz = syz0 + s.dt * myz * syz_r;
  const int nt = s.nt;
  if (i == s.si && k == s.sk && j == s.sj) {
    sxx -= s.w * s.src[n];
    syy -= s.w * s.src[nt + n];
    szz -= s.w * s.src[2 * nt + n];
  }
  const bool ii = (i == s.si || i == s.si - 1), kk = (k == s.sk || k == s.sk - 1), jj = (j == s.sj || j == s.sj - 1);
  if (i == s.si && kk && jj) sxy -= 0.25f * s.w * s.src[3 * nt + n];
  if (ii && k == s.sk && jj) sxz -= 0.25f * s.w * s.src[4 * nt + n];
  if (ii && kk && j == s.sj) syz -= 0.25f * s.w * s.src[5 * nt + n];
  G(PF(s.sxx), o) = sxx;
  G(PF(s.syy), o) = syy;
  G(PF(s.szz), o) = szz;
  G(PF(s.sxy), o) = sxy;
  G(PF(s.sxz), o) = sxz;
  G(PF(s.syz), o) = syz;
  if (PX && inx) G(s.psx[XS_PXX], qxs) = p[0], G(s.psx[XS_SXY], qxs) = p[1], G(s.psx[XS_SXZ], qxs) = p[2];
  if (PY && iny) G(s.psy[YS_PYY], qys) = p[3], G(s.psy[YS_SXY], qys) = p[4], G(s.psy[YS_SYZ], qys) = p[5];
  if (PZ && inz) G(s.psz[ZS_PZZ], qzs) = p[6], G(s.psz[ZS_SXZ], qzs) = p[7], G(s.psz[ZS_SYZ], qzs) = p[8];
  if (RECORD) {
    if (slot >= 0) {
      const int c = s.rowch[(long)slot * s.nx + j];
      if (c >= 0) {
        const float e = s.e[c] + s.dt * raw_pxx;
        s.e[c] = e;
        s.d[(long)c * nt + n] = e;
      }
    }
  }
  if (STORE) {
    const unsigned c = (unsigned)(((long)i * s.ny + k) * s.cp + j), cells = (unsigned)s.cells;
    const float mu = 0.5f * two_mu, third = tr * (1.0f / 3.0f);
    hist_put(seg, c, tr / (l2m + 2.0f * lam));
    hist_put(seg, cells + c, (pxx - third) * mu);
    hist_put(seg, 2 * cells + c, (pyy - third) * mu);
    hist_put(seg, 3 * cells + c, 0.25f * mxy * sxy_r);
    hist_put(seg, 4 * cells + c, 0.25f * mxz * sxz_r);
    hist_put(seg, 5 * cells + c, 0.25f * myz * syz_r);
  }
}

template <bool STORE, bool RECORD>
__global__ __launch_bounds__(TX * TY) void k3_fwd_str(PARAMS3, int n, int kstore) {
  TILE3() {
    if (k >= s.ny || j >= s.nx) return;
    gfloat* seg = STORE ? s.seg + (size_t)kstore * NSEG3 * s.cells : nullptr;
#define CALL(X, Y, Z) fwd_str3<STORE, RECORD, X, Y, Z>(s, i, k, j, n, seg)
    DISPATCH_AXES(pml_axes(s, i, k0, j0, 0), CALL);
#undef CALL
  }
}

// ------------------------------------------------------------------------------------
// Adjoint. Corrected transposed operands at a neighbour node: v + a (psi_bar + v) inside
// the CPML strip of the derivative's axis (psi_bar from the buffer of step n+1), v outside.
// PX, PY, PZ: the tile's stencil reaches a strip on that axis (otherwise no correction on
// it is possible). A neighbour differs from the owned node only along the derivative's
// axis, so only that index is range-checked (strip_clamp).
// ------------------------------------------------------------------------------------
template <bool PX, bool PY, bool PZ>
struct Adj3 {
  const Shot3D& s;
  int rd;
  __device__ __forceinline__ float cx(float v, int i, int k, int j, int slot, int prof) const {
    if (!PX) return v;
    bool in;
    const unsigned q = xq(s, i, k, strip_clamp(j, s.nx, s.P, in));
    float c = v;
    c += px_(s, prof)[min(max(j, 0), s.nx - 1)] * (G(s.pbx[rd][slot], q) + c);
    return in ? c : v;
  }
  __device__ __forceinline__ float cy(float v, int i, int k, int j, int slot, int prof) const {
    if (!PY) return v;
    bool in;
    const unsigned q = yq(s, i, strip_clamp(k, s.ny, s.P, in), j);
    float c = v;
    c += py_(s, prof)[min(max(k, 0), s.ny - 1)] * (G(s.pby[rd][slot], q) + c);
    return in ? c : v;
  }
  __device__ __forceinline__ float cz(float v, int i, int k, int j, int slot, int prof) const {
    if (!PZ) return v;
    bool in;
    const unsigned q = zq(s, strip_clamp(i, s.nz, s.P, in), k, j);
    float c = v;
    c += pz_(s, prof)[min(max(i, 0), s.nz - 1)] * (G(s.pbz[rd][slot], q) + c);
    return in ? c : v;
  }
  __device__ __forceinline__ float at(const gfloat* f, int i, int k, int j) const {
    return s.dt * G(PF(f), cell_ofs(s, i, k, j));
  }
};

__device__ __forceinline__ float ebar3(const Shot3D& s, int slot, int jc, int n) {
  if (jc < 0 || jc >= s.nx) return 0.0f;
  const int c = s.rowch[(long)slot * s.nx + jc];
  return c >= 0 ? s.ebar[(long)n * s.nch + c] : 0.0f;
}

// Transposed stress sub-step: t_bar -> u_bar.
template <bool GRAD, bool SRCADJ, bool PX, bool PY, bool PZ>
__device__ __forceinline__ void adj_vel3(const Shot3D& s, int i, int k, int j, int n, const gfloat* seg, bool first) {
  const unsigned ld = (unsigned)s.ld, pz = (unsigned)s.pz;
  const unsigned o = cell_ofs(s, i, k, j);
  const int rd = (n + 1) & 1, wr = n & 1;
  const Adj3<PX, PY, PZ> A{s, rd};
  // operands: normal (int profile on their own axis), shear (half profile on the axis of
  // the velocity derivative they came from)
  auto Pxx = [&](int a, int b, int c) { return A.cx(A.at(s.txxb, a, b, c), a, b, c, XS_PXX, 0); };
  auto Pyy = [&](int a, int b, int c) { return A.cy(A.at(s.tyyb, a, b, c), a, b, c, YS_PYY, 0); };
  auto Pzz = [&](int a, int b, int c) { return A.cz(A.at(s.tzzb, a, b, c), a, b, c, ZS_PZZ, 0); };
  auto Pxy_vx = [&](int a, int b, int c) { return A.cy(A.at(s.txyb, a, b, c), a, b, c, YS_SXY, 2); };
  auto Pxy_vy = [&](int a, int b, int c) { return A.cx(A.at(s.txyb, a, b, c), a, b, c, XS_SXY, 2); };
  auto Pxz_vx = [&](int a, int b, int c) { return A.cz(A.at(s.txzb, a, b, c), a, b, c, ZS_SXZ, 2); };
  auto Pxz_vz = [&](int a, int b, int c) { return A.cx(A.at(s.txzb, a, b, c), a, b, c, XS_SXZ, 2); };
  auto Pyz_vy = [&](int a, int b, int c) { return A.cz(A.at(s.tyzb, a, b, c), a, b, c, ZS_SYZ, 2); };
  auto Pyz_vz = [&](int a, int b, int c) { return A.cy(A.at(s.tyzb, a, b, c), a, b, c, YS_SYZ, 2); };
  // t_bar one back along either axis of each shear type: operands of the differences and,
  // with the imaging, terms of its gather below (loaded once for both; without the imaging
  // the differences load them as the other operands, which keeps that instance's registers
  // below the cap)
  const float txy_km = GRAD ? G(PF(s.txyb), o - ld) : 0.0f, txy_jm = GRAD ? G(PF(s.txyb), o - 1u) : 0.0f;
  const float txz_im = GRAD ? G(PF(s.txzb), o - pz) : 0.0f, txz_jm = GRAD ? G(PF(s.txzb), o - 1u) : 0.0f;
  const float tyz_im = GRAD ? G(PF(s.tyzb), o - pz) : 0.0f, tyz_km = GRAD ? G(PF(s.tyzb), o - ld) : 0.0f;
  // v_bar_x += -(D+x Pxx + D-y Pxy_vx + D-z Pxz_vx)
  const float x1 = K1 * (Pxx(i, k, j + 1) - Pxx(i, k, j)) + K2 * (Pxx(i, k, j + 2) - Pxx(i, k, j - 1));
  const float x2 = K1 * (Pxy_vx(i, k, j) - (GRAD ? A.cy(s.dt * txy_km, i, k - 1, j, YS_SXY, 2) : Pxy_vx(i, k - 1, j))) + K2 * (Pxy_vx(i, k + 1, j) - Pxy_vx(i, k - 2, j));
  const float x3 = K1 * (Pxz_vx(i, k, j) - (GRAD ? A.cz(s.dt * txz_im, i - 1, k, j, ZS_SXZ, 2) : Pxz_vx(i - 1, k, j))) + K2 * (Pxz_vx(i + 1, k, j) - Pxz_vx(i - 2, k, j));
  // v_bar_y += -(D+y Pyy + D-x Pxy_vy + D-z Pyz_vy)
  const float y1 = K1 * (Pyy(i, k + 1, j) - Pyy(i, k, j)) + K2 * (Pyy(i, k + 2, j) - Pyy(i, k - 1, j));
  const float y2 = K1 * (Pxy_vy(i, k, j) - (GRAD ? A.cx(s.dt * txy_jm, i, k, j - 1, XS_SXY, 2) : Pxy_vy(i, k, j - 1))) + K2 * (Pxy_vy(i, k, j + 1) - Pxy_vy(i, k, j - 2));
  const float y3 = K1 * (Pyz_vy(i, k, j) - (GRAD ? A.cz(s.dt * tyz_im, i - 1, k, j, ZS_SYZ, 2) : Pyz_vy(i - 1, k, j))) + K2 * (Pyz_vy(i + 1, k, j) - Pyz_vy(i - 2, k, j));
  // v_bar_z += -(D+z Pzz + D-x Pxz_vz + D-y Pyz_vz)
  const float z1 = K1 * (Pzz(i + 1, k, j) - Pzz(i, k, j)) + K2 * (Pzz(i + 2, k, j) - Pzz(i - 1, k, j));
  const float z2 = K1 * (Pxz_vz(i, k, j) - (GRAD ? A.cx(s.dt * txz_jm, i, k, j - 1, XS_SXZ, 2) : Pxz_vz(i, k, j - 1))) + K2 * (Pxz_vz(i, k, j + 1) - Pxz_vz(i, k, j - 2));
  const float z3 = K1 * (Pyz_vz(i, k, j) - (GRAD ? A.cy(s.dt * tyz_km, i, k - 1, j, YS_SYZ, 2) : Pyz_vz(i, k - 1, j))) + K2 * (Pyz_vz(i, k + 1, j) - Pyz_vz(i, k - 2, j));
  float gx = -(x1 * s.rdx + x2 * s.rdy + x3 * s.rdz);
  const float gy = -(y1 * s.rdy + y2 * s.rdx + y3 * s.rdz);
  const float gz = -(z1 * s.rdz + z2 * s.rdx + z3 * s.rdy);
  const int slot = s.row_slot[(long)i * s.ny + k];
  if (slot >= 0) {
    const float inj = K1 * (ebar3(s, slot, j, n) - ebar3(s, slot, j + 1, n)) +
                      K2 * (ebar3(s, slot, j - 1, n) - ebar3(s, slot, j + 2, n));
    gx += s.dt * s.rdx * inj;
  }
  const float txx = G(PF(s.txxb), o), tyy = G(PF(s.tyyb), o), tzz = G(PF(s.tzzb), o);
  const float txy = G(PF(s.txyb), o), txz = G(PF(s.txzb), o), tyz = G(PF(s.tyzb), o);
  // Imaging terms of this normal node, formed before the stores below so that the t_bar
  // neighbours the differences above loaded are not loaded again. The four shear nodes of
  // a type (this node's and those one back along either or both of the type's axes a, b)
  // are weighted by how often their clamped corners use this node: twice at the last
  // plane, row or column (wa, wb), else once. A neighbour before the first plane, row or
  // column has its t_bar in the zero halo, and its stored quantity is read at this node
  // instead (in bounds and finite), so its term is zero. The stored shear quantities are
  // read through the caches: four normal nodes gather each.
  float img_a = 0.0f, img_e = 0.0f;
  if (GRAD) {
    const unsigned c = (unsigned)(((long)i * s.ny + k) * s.cp + j), cells = (unsigned)s.cells;
    const float h0 = hist_get(seg, c), D1 = hist_get(seg, cells + c), D2 = hist_get(seg, 2 * cells + c);
    const float trt = txx + tyy + tzz;
    const float da = txx - trt * (1.0f / 3.0f), db = tyy - trt * (1.0f / 3.0f);
    const unsigned hx = j > 0 ? 1u : 0u, hy = k > 0 ? (unsigned)s.cp : 0u, hz = i > 0 ? (unsigned)(s.ny * s.cp) : 0u;
    const float wx = j == s.nx - 1 ? 2.0f : 1.0f, wy = k == s.ny - 1 ? 2.0f : 1.0f, wz = i == s.nz - 1 ? 2.0f : 1.0f;
    const gfloat *hxy = seg + 3 * cells, *hxz = seg + 4 * cells, *hyz = seg + 5 * cells;
    const float sxy = wy * (wx * (txy * G(hxy, c)) + txy_jm * G(hxy, c - hx)) +
                      (wx * (txy_km * G(hxy, c - hy)) + G(PF(s.txyb), o - ld - 1u) * G(hxy, c - hy - hx));
    const float sxz = wz * (wx * (txz * G(hxz, c)) + txz_jm * G(hxz, c - hx)) +
                      (wx * (txz_im * G(hxz, c - hz)) + G(PF(s.txzb), o - pz - 1u) * G(hxz, c - hz - hx));
    const float syz = wz * (wy * (tyz * G(hyz, c)) + tyz_km * G(hyz, c - hy)) +
                      (wy * (tyz_im * G(hyz, c - hz)) + G(PF(s.tyzb), o - pz - ld) * G(hyz, c - hz - hy));
    img_a = trt * h0;
    img_e = (da * D1 + db * D2 + (da + db) * (D1 + D2)) + (sxy + sxz + syz);
  }
  const float ux = G(PF(s.uxb), o), uy = G(PF(s.uyb), o), uz = G(PF(s.uzb), o);
  float bx, by, bz;
  buoyancies(s, o, bx, by, bz);
  G(PF(s.uxb), o) = ux + bx * gx;
  G(PF(s.uyb), o) = uy + by * gy;
  G(PF(s.uzb), o) = uz + bz * gz;
  if (PX || PY || PZ) {  // adjoint memory variables: step n + 1 (read buffer) -> step n (write buffer)
    const float dt = s.dt;
    if (PX) {
      bool in;
      const unsigned q = xq(s, i, k, strip_clamp(j, s.nx, s.P, in));
      const float o0 = G(s.pbx[rd][XS_PXX], q), o1 = G(s.pbx[rd][XS_SXY], q), o2 = G(s.pbx[rd][XS_SXZ], q);
      if (in) {
        G(s.pbx[wr][XS_PXX], q) = px_(s, 1)[j] * (o0 + dt * txx);
        G(s.pbx[wr][XS_SXY], q) = px_(s, 3)[j] * (o1 + dt * txy);
        G(s.pbx[wr][XS_SXZ], q) = px_(s, 3)[j] * (o2 + dt * txz);
      }
    }
    if (PY) {
      bool in;
      const unsigned q = yq(s, i, strip_clamp(k, s.ny, s.P, in), j);
      const float o0 = G(s.pby[rd][YS_PYY], q), o1 = G(s.pby[rd][YS_SXY], q), o2 = G(s.pby[rd][YS_SYZ], q);
      if (in) {
        G(s.pby[wr][YS_PYY], q) = py_(s, 1)[k] * (o0 + dt * tyy);
        G(s.pby[wr][YS_SXY], q) = py_(s, 3)[k] * (o1 + dt * txy);
        G(s.pby[wr][YS_SYZ], q) = py_(s, 3)[k] * (o2 + dt * tyz);
      }
    }
    if (PZ) {
      bool in;
      const unsigned q = zq(s, strip_clamp(i, s.nz, s.P, in), k, j);
      const float o0 = G(s.pbz[rd][ZS_PZZ], q), o1 = G(s.pbz[rd][ZS_SXZ], q), o2 = G(s.pbz[rd][ZS_SYZ], q);
      if (in) {
        G(s.pbz[wr][ZS_PZZ], q) = pz_(s, 1)[i] * (o0 + dt * tzz);
        G(s.pbz[wr][ZS_SXZ], q) = pz_(s, 3)[i] * (o1 + dt * txz);
        G(s.pbz[wr][ZS_SYZ], q) = pz_(s, 3)[i] * (o2 + dt * tyz);
      }
    }
  }
  if (GRAD) {
    const unsigned c = (unsigned)(((long)i * s.ny + k) * s.cp + j), cells = (unsigned)s.cells;
    const float a0 = first ? 0.0f : G(s.acc, c), a1 = first ? 0.0f : G(s.acc, cells + c);
    G(s.acc, c) = a0 + s.dt * img_a;
    G(s.acc, cells + c) = a1 + s.dt * img_e;
  }
  if (SRCADJ && i == s.si && k == s.sk && j == s.sj) {
    // sigma_bar at the source: invert C on the normal block and the shear moduli
    const float l2m = G(PF(s.l2m), o), lam = G(PF(s.lam), o), two_mu = l2m - lam;
    const float trs = (txx + tyy + tzz) / (l2m + 2.0f * lam);
    const int nt = s.nt;
    s.src_bar[n] = -s.w * (txx - lam * trs) / two_mu;
    s.src_bar[nt + n] = -s.w * (tyy - lam * trs) / two_mu;
    s.src_bar[2 * nt + n] = -s.w * (tzz - lam * trs) / two_mu;
    auto sh = [&](const gfloat* t, const gfloat* mu, unsigned oo) {
      return G(PF(mu), oo) > 0.0f ? G(PF(t), oo) / G(PF(mu), oo) : 0.0f;
    };
    float a = 0.f, b = 0.f, c = 0.f;
    for (int q = 0; q < 4; ++q) {
      const int d1 = q & 1, d2 = q >> 1;
      a += sh(s.txyb, s.muxy, o - d1 * ld - d2);        // (i, k-d1, j-d2)
      b += sh(s.txzb, s.muxz, o - d1 * pz - d2);        // (i-d1, k, j-d2)
      c += sh(s.tyzb, s.muyz, o - d1 * pz - d2 * ld);   // (i-d1, k-d2, j)
    }
    s.src_bar[3 * nt + n] = -0.25f * s.w * a;
    s.src_bar[4 * nt + n] = -0.25f * s.w * b;
    s.src_bar[5 * nt + n] = -0.25f * s.w * c;
  }
}

template <bool GRAD, bool SRCADJ>
// At least 4 waves per SIMD (at most 128 VGPRs; the compiler takes 116 with the imaging
// gather and the wave-uniform row, without spilling): 1.47 ms per 300 x 400 x 400 launch. Before the gather, 1.59 ms
// at this cap against 1.73 ms with the compiler's own allocation (136 VGPRs, 3 waves) and
// 2.02 ms capped at 5 waves (spills).
__global__ __launch_bounds__(TX * TY) __attribute__((amdgpu_waves_per_eu(4))) void k3_adj_vel(PARAMS3, int n, int kseg, int first) {
  TILE3() {
    if (k >= s.ny || j >= s.nx) return;
    const gfloat* seg = GRAD ? s.seg + (size_t)kseg * NSEG3 * s.cells : nullptr;
#define CALL(X, Y, Z) adj_vel3<GRAD, SRCADJ, X, Y, Z>(s, i, __builtin_amdgcn_readfirstlane(k), j, n, seg, first != 0)
    DISPATCH_AXES(pml_axes(s, i, k0, j0, 2), CALL);
#undef CALL
  }
}

// Transposed velocity sub-step: u_bar -> t_bar.
template <bool GRAD, bool PX, bool PY, bool PZ>
__device__ __forceinline__ void adj_str3(const Shot3D& s, int i, int k, int j, int n, const gfloat* seg, bool first) {
  const unsigned ld = (unsigned)s.ld, pz = (unsigned)s.pz;
  const unsigned o = cell_ofs(s, i, k, j);
  const int rd = (n + 1) & 1, wr = n & 1;
  const Adj3<PX, PY, PZ> A{s, rd};
  auto Qxx = [&](int a, int b, int c) { return A.cx(A.at(s.uxb, a, b, c), a, b, c, XS_VX, 2); };  // vx: D+x sxx
  auto Qxy = [&](int a, int b, int c) { return A.cy(A.at(s.uxb, a, b, c), a, b, c, YS_VX, 0); };  // vx: D-y sxy
  auto Qxz = [&](int a, int b, int c) { return A.cz(A.at(s.uxb, a, b, c), a, b, c, ZS_VX, 0); };  // vx: D-z sxz
  auto Qyx = [&](int a, int b, int c) { return A.cx(A.at(s.uyb, a, b, c), a, b, c, XS_VY, 0); };  // vy: D-x sxy
  auto Qyy = [&](int a, int b, int c) { return A.cy(A.at(s.uyb, a, b, c), a, b, c, YS_VY, 2); };  // vy: D+y syy
  auto Qyz = [&](int a, int b, int c) { return A.cz(A.at(s.uyb, a, b, c), a, b, c, ZS_VY, 0); };  // vy: D-z syz
  auto Qzx = [&](int a, int b, int c) { return A.cx(A.at(s.uzb, a, b, c), a, b, c, XS_VZ, 0); };  // vz: D-x sxz
  auto Qzy = [&](int a, int b, int c) { return A.cy(A.at(s.uzb, a, b, c), a, b, c, YS_VZ, 0); };  // vz: D-y syz
  auto Qzz = [&](int a, int b, int c) { return A.cz(A.at(s.uzb, a, b, c), a, b, c, ZS_VZ, 2); };  // vz: D+z szz
  // sigma_bar_cc += -D-c Q; shear += -(D+ Q + D+ Q)
  const float dxx = -(K1 * (Qxx(i, k, j) - Qxx(i, k, j - 1)) + K2 * (Qxx(i, k, j + 1) - Qxx(i, k, j - 2))) * s.rdx;
  const float dyy = -(K1 * (Qyy(i, k, j) - Qyy(i, k - 1, j)) + K2 * (Qyy(i, k + 1, j) - Qyy(i, k - 2, j))) * s.rdy;
  const float dzz = -(K1 * (Qzz(i, k, j) - Qzz(i - 1, k, j)) + K2 * (Qzz(i + 1, k, j) - Qzz(i - 2, k, j))) * s.rdz;
  const float dxy = -((K1 * (Qxy(i, k + 1, j) - Qxy(i, k, j)) + K2 * (Qxy(i, k + 2, j) - Qxy(i, k - 1, j))) * s.rdy +
                      (K1 * (Qyx(i, k, j + 1) - Qyx(i, k, j)) + K2 * (Qyx(i, k, j + 2) - Qyx(i, k, j - 1))) * s.rdx);
  const float dxz = -((K1 * (Qxz(i + 1, k, j) - Qxz(i, k, j)) + K2 * (Qxz(i + 2, k, j) - Qxz(i - 1, k, j))) * s.rdz +
                      (K1 * (Qzx(i, k, j + 1) - Qzx(i, k, j)) + K2 * (Qzx(i, k, j + 2) - Qzx(i, k, j - 1))) * s.rdx);
  const float dyz = -((K1 * (Qyz(i + 1, k, j) - Qyz(i, k, j)) + K2 * (Qyz(i + 2, k, j) - Qyz(i - 1, k, j))) * s.rdz +
                      (K1 * (Qzy(i, k + 1, j) - Qzy(i, k, j)) + K2 * (Qzy(i, k + 2, j) - Qzy(i, k - 1, j))) * s.rdy);
  const float ux = G(PF(s.uxb), o), uy = G(PF(s.uyb), o), uz = G(PF(s.uzb), o);
  const float l2m = G(PF(s.l2m), o), lam = G(PF(s.lam), o), two_mu = l2m - lam;
  // the staged moduli here: deriving them (seven mu loads, three harmonic means) raised this
  // kernel from 102 to 141 VGPRs and 1.64 to 2.01 ms per 300 x 400 x 400 launch
  const float mxy = G(PF(s.muxy), o), mxz = G(PF(s.muxz), o), myz = G(PF(s.muyz), o);
  const float txx = G(PF(s.txxb), o), tyy = G(PF(s.tyyb), o), tzz = G(PF(s.tzzb), o), txy = G(PF(s.txyb), o), txz = G(PF(s.txzb), o), tyz = G(PF(s.tyzb), o);
  const float tr = dxx + dyy + dzz;
  G(PF(s.txxb), o) = txx + (lam * tr + two_mu * dxx);
  G(PF(s.tyyb), o) = tyy + (lam * tr + two_mu * dyy);
  G(PF(s.tzzb), o) = tzz + (lam * tr + two_mu * dzz);
  G(PF(s.txyb), o) = txy + mxy * dxy;
  G(PF(s.txzb), o) = txz + mxz * dxz;
  G(PF(s.tyzb), o) = tyz + myz * dyz;
  if (PX || PY || PZ) {  // adjoint memory variables: step n + 1 (read buffer) -> step n (write buffer)
    const float dt = s.dt;
    if (PX) {
      bool in;
      const unsigned q = xq(s, i, k, strip_clamp(j, s.nx, s.P, in));
      const float o0 = G(s.pbx[rd][XS_VX], q), o1 = G(s.pbx[rd][XS_VY], q), o2 = G(s.pbx[rd][XS_VZ], q);
      if (in) {
        G(s.pbx[wr][XS_VX], q) = px_(s, 3)[j] * (o0 + dt * ux);
        G(s.pbx[wr][XS_VY], q) = px_(s, 1)[j] * (o1 + dt * uy);
        G(s.pbx[wr][XS_VZ], q) = px_(s, 1)[j] * (o2 + dt * uz);
      }
    }
    if (PY) {
      bool in;
      const unsigned q = yq(s, i, strip_clamp(k, s.ny, s.P, in), j);
      const float o0 = G(s.pby[rd][YS_VX], q), o1 = G(s.pby[rd][YS_VY], q), o2 = G(s.pby[rd][YS_VZ], q);
      if (in) {
        G(s.pby[wr][YS_VX], q) = py_(s, 1)[k] * (o0 + dt * ux);
        G(s.pby[wr][YS_VY], q) = py_(s, 3)[k] * (o1 + dt * uy);
        G(s.pby[wr][YS_VZ], q) = py_(s, 1)[k] * (o2 + dt * uz);
      }
    }
    if (PZ) {
      bool in;
      const unsigned q = zq(s, strip_clamp(i, s.nz, s.P, in), k, j);
      const float o0 = G(s.pbz[rd][ZS_VX], q), o1 = G(s.pbz[rd][ZS_VY], q), o2 = G(s.pbz[rd][ZS_VZ], q);
      if (in) {
        G(s.pbz[wr][ZS_VX], q) = pz_(s, 1)[i] * (o0 + dt * ux);
        G(s.pbz[wr][ZS_VY], q) = pz_(s, 1)[i] * (o1 + dt * uy);
        G(s.pbz[wr][ZS_VZ], q) = pz_(s, 3)[i] * (o2 + dt * uz);
      }
    }
  }
  if (GRAD) {
    // The two velocity nodes of each component whose buoyancy uses this node's density
    // (this node's and the one back along the component's axis), weighted as the shear
    // nodes of the transposed stress sub-step.
    const unsigned c = (unsigned)(((long)i * s.ny + k) * s.cp + j), cells = (unsigned)s.cells;
    const unsigned hx = j > 0 ? 1u : 0u, hy = k > 0 ? (unsigned)s.cp : 0u, hz = i > 0 ? (unsigned)(s.ny * s.cp) : 0u;
    const float wx = j == s.nx - 1 ? 2.0f : 1.0f, wy = k == s.ny - 1 ? 2.0f : 1.0f, wz = i == s.nz - 1 ? 2.0f : 1.0f;
    auto pair = [&](const gfloat* u, float u0, unsigned f, unsigned oa, unsigned ha, float wa) {
      const gfloat* h = seg + f * cells;
      return wa * (u0 * G(h, c)) + G(PF(u), o - oa) * G(h, c - ha);
    };
    const float a0 = first ? 0.0f : G(s.acc, 2 * cells + c);
    const float rx = pair(s.uxb, ux, 6u, 1u, hx, wx), ry = pair(s.uyb, uy, 7u, ld, hy, wy);
    const float rz = pair(s.uzb, uz, 8u, pz, hz, wz);
    G(s.acc, 2 * cells + c) = a0 + s.dt * (rx + ry + rz);
  }
}

template <bool GRAD>
// The compiler's own allocation (88 VGPRs with the imaging gather and the wave-uniform row, 5
// waves per SIMD): 1.45 ms per 300 x 400 x 400 launch. Before the gather (102 VGPRs, 4 waves), 1.64 ms against 1.88
// ms capped at 8 waves (64 VGPRs, spills) and 2.00 ms at 7.
__global__ __launch_bounds__(TX * TY) void k3_adj_str(PARAMS3, int n, int kseg, int first) {
  TILE3() {
    if (k >= s.ny || j >= s.nx) return;
    const gfloat* seg = GRAD ? s.seg + (size_t)kseg * NSEG3 * s.cells : nullptr;
#define CALL(X, Y, Z) adj_str3<GRAD, X, Y, Z>(s, i, __builtin_amdgcn_readfirstlane(k), j, n, seg, first != 0)
    DISPATCH_AXES(pml_axes(s, i, k0, j0, 2), CALL);
#undef CALL
  }
}

// ------------------------------------------------------------------------------------
// Staging: (Vp, Vs, rho) -> lambda + 2 mu, lambda, harmonic shear moduli, padded rho and mu.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(TX * TY) void k3_stage(PARAMS3) {
  TILE3() {
    if (k >= s.ny || j >= s.nx) return;
    const int ip = min(i + 1, s.nz - 1), kp = min(k + 1, s.ny - 1), jp = min(j + 1, s.nx - 1);
    auto at = [&](const gfloat* f, int a, int b, int c) { return f[(long)a * s.mplanestride + (long)b * s.mld + c]; };
    auto mu_at = [&](int a, int b, int c) {
      const float v = at(s.mvs, a, b, c);
      return at(s.mrho, a, b, c) * v * v;
    };
    const float vp = at(s.mvp, i, k, j), rho = at(s.mrho, i, k, j);
    const float mu = mu_at(i, k, j);
    const unsigned o = cell_ofs(s, i, k, j);
    const float l2m = rho * vp * vp;
    G(PF(s.l2m), o) = l2m;
    G(PF(s.lam), o) = l2m - 2.0f * mu;
    G(PF(s.muxy), o) = harm4(mu, mu_at(i, kp, j), mu_at(i, k, jp), mu_at(i, kp, jp));
    G(PF(s.muxz), o) = harm4(mu, mu_at(ip, k, j), mu_at(i, k, jp), mu_at(ip, k, jp));
    G(PF(s.muyz), o) = harm4(mu, mu_at(ip, k, j), mu_at(i, kp, j), mu_at(ip, kp, j));
    // rho and mu, repeated one node beyond the last plane, row and column (the clamped
    // neighbours of the derivations above)
    const unsigned ld = (unsigned)s.ld, pz = (unsigned)s.pz;
    const bool ei = i == s.nz - 1, ek = k == s.ny - 1, ej = j == s.nx - 1;
    auto put = [&](unsigned oo) {
      G(PF(s.rho), oo) = rho;
      G(PF(s.mu), oo) = mu;
    };
    put(o);
    if (ej) put(o + 1u);
    if (ek) put(o + ld);
    if (ei) put(o + pz);
    if (ej && ek) put(o + ld + 1u);
    if (ej && ei) put(o + pz + 1u);
    if (ek && ei) put(o + pz + ld);
  }
}

// ------------------------------------------------------------------------------------
// Chain rule of one block of FP32 imaging sums into the FP64 (Vp, Vs, rho) gradient.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(TX * TY) void k3_chain_flush(PARAMS3) {
  TILE3() {
    if (k >= s.ny || j >= s.nx) return;
    const long cs = s.cells;
    auto ci = [&](int a, int b, int c) { return ((long)a * s.ny + b) * s.cp + c; };
    const long cc = ci(i, k, j);
    const long mo = (long)i * s.mplanestride + (long)k * s.mld + j;
    const float vp = s.mvp[mo], vs = s.mvs[mo], rho = s.mrho[mo];
    const double mu = (double)(rho * vs * vs);
    const double gl = s.acc[cc];
    const double gmu = 2.0 / 3.0 * gl + (mu > 0.0 ? (double)s.acc[cs + cc] / (mu * mu) : 0.0);
    const double grho = -(double)s.acc[2 * cs + cc];
    const double dvp = vp, dvs = vs, drho = rho;
    s.G[cc] += 2.0 * drho * dvp * gl;
    s.G[cs + cc] += 2.0 * drho * dvs * (gmu - 2.0 * gl);
    s.G[2 * cs + cc] += (dvp * dvp - 2.0 * dvs * dvs) * gl + dvs * dvs * gmu + grho;
  }
}

__global__ __launch_bounds__(TX * TY) void k3_write_gradient(PARAMS3) {
  TILE3() {
    if (k >= s.ny || j >= s.nx) return;
    const long cc = ((long)i * s.ny + k) * s.cp + j;
    const long go = (long)(s.z0 + i) * s.mplanestride + (long)(s.y0 + k) * s.mld + (s.x0 + j);
    for (int q = 0; q < 3; ++q) s.gout[q * s.mplane + go] = (float)s.G[q * s.cells + cc];
  }
}

inline dim3 grid3(const Sched& q) { return dim3(q.n); }
inline dim3 block3() { return dim3(TX, TY); }
#define FWD3 b.shots, b.tile_shot, b.tile_first, b.fwd.sched
#define ADJ3 b.shots, b.tile_shot, b.tile_first, b.adj.sched

}  // namespace

hipError_t launch3_stage(const Batch3D& b, hipStream_t st) {
  k3_stage<<<grid3(b.fwd), block3(), 0, st>>>(FWD3);
  return hipGetLastError();
}

hipError_t launch3_fwd_vel(const Batch3D& b, int kstore, hipStream_t st) {
  if (kstore >= 0) k3_fwd_vel<true><<<grid3(b.fwd), block3(), 0, st>>>(FWD3, kstore);
  else k3_fwd_vel<false><<<grid3(b.fwd), block3(), 0, st>>>(FWD3, 0);
  return hipGetLastError();
}

hipError_t launch3_fwd_str(const Batch3D& b, int n, int kstore, bool record, hipStream_t st) {
  if (kstore >= 0) {
    if (record) k3_fwd_str<true, true><<<grid3(b.fwd), block3(), 0, st>>>(FWD3, n, kstore);
    else k3_fwd_str<true, false><<<grid3(b.fwd), block3(), 0, st>>>(FWD3, n, kstore);
  } else {
    if (record) k3_fwd_str<false, true><<<grid3(b.fwd), block3(), 0, st>>>(FWD3, n, 0);
    else k3_fwd_str<false, false><<<grid3(b.fwd), block3(), 0, st>>>(FWD3, n, 0);
  }
  return hipGetLastError();
}

hipError_t launch3_adj_vel(const Batch3D& b, int n, int k, bool grad, bool first, bool srcadj, hipStream_t st) {
  if (grad) k3_adj_vel<true, false><<<grid3(b.adj), block3(), 0, st>>>(ADJ3, n, k, first);
  else if (srcadj) k3_adj_vel<false, true><<<grid3(b.adj), block3(), 0, st>>>(ADJ3, n, 0, 0);
  else k3_adj_vel<false, false><<<grid3(b.adj), block3(), 0, st>>>(ADJ3, n, 0, 0);
  return hipGetLastError();
}

hipError_t launch3_adj_str(const Batch3D& b, int n, int k, bool grad, bool first, hipStream_t st) {
  if (grad) k3_adj_str<true><<<grid3(b.adj), block3(), 0, st>>>(ADJ3, n, k, first);
  else k3_adj_str<false><<<grid3(b.adj), block3(), 0, st>>>(ADJ3, n, 0, 0);
  return hipGetLastError();
}

hipError_t launch3_chain_flush(const Batch3D& b, hipStream_t st) {
  k3_chain_flush<<<grid3(b.fwd), block3(), 0, st>>>(FWD3);
  return hipGetLastError();
}

hipError_t launch3_write_gradient(const Batch3D& b, hipStream_t st) {
  k3_write_gradient<<<grid3(b.fwd), block3(), 0, st>>>(FWD3);
  return hipGetLastError();
}

}  // namespace efwi
