// Internal declarations shared by the HIP kernels and the host-side C ABI.
// Not installed; the public interface is include/efwi.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace efwi {

// Padded field layout: every wavefield and staged-parameter array has HALO zero cells on
// each side in z and x so that the 4th-order stencils never branch on the grid edge.
constexpr int HALO = 2;
// The interior of every padded row starts XOFF floats into the row and the row pitch is a
// multiple of 32 floats, so each wavefront's 64 consecutive x values fill whole 128-byte
// lines. Unpadded per-cell arrays (segment buffer, imaging sums, gradient) use a row pitch
// `cp` rounded up to 32 for the same reason.
constexpr int XOFF = 32;
constexpr int ROW_ALIGN = 32;
// Thread-block shape of the 2D stencil kernels: 64 lanes along x (one wavefront per row)
// by 4 rows along z.
constexpr int BX = 64;
constexpr int BZ = 4;
// Number of per-step forward quantities kept for the imaging condition (see k_fwd_str and
// k_fwd_vel), each already multiplied by the factor it meets in the gradient of its
// parameter: (pxx+pzz)/(2(l+m)) and (pxx-pzz) mu/2 at the normal node, (pzx+pxz) mu_xz/4 at
// the shear node, qx b_x/2 and qz b_z/2 at the velocity nodes (p, q: CPML-corrected strain
// rates and stress divergences of the step).
constexpr int NSEG_FIELDS = 5;
// Number of imaging accumulators, all at the normal node: lambda; mu scaled by mu^2
// (the normal-node mu term plus the four surrounding mu_xz terms); rho through the
// buoyancies of the four surrounding velocity nodes.
constexpr int NACC = 3;
constexpr int NACC_VTI = 5;   // VTI: the c11, c33 and c13 sums replace the lambda sum
// Time steps summed in FP32 before the imaging sums are chained into the FP64 gradient
// (each flush reads and writes the FP64 sums: 64 steps keep it near 0.5% of a reverse sweep).
constexpr int FLUSH_STEPS = 64;

// Device pointers in the global address space. Kernels read each shot's descriptor from a
// device array; typing its pointer members as global keeps every access a global_load /
// global_store instead of a generic flat access.
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) int gint;
typedef __attribute__((address_space(1))) double gdouble;

// Everything a 2D kernel needs about one shot. Pointers to padded arrays point at the
// interior origin (i = 0, j = 0); element (i, j) is at p[i * ld + j].
struct Shot2D {
  int nz, nx, ld, P;            // window size, padded pitch, CPML strip half-width (0: none)
  int nt, nch;
  int si, sj;                   // source normal node, window coordinates
  float dt, rdx, rdz, w;        // w = dt / (dx dz)
  int cp;                       // row pitch of the unpadded per-cell arrays
  long cells;                   // nz * cp
  // forward state, double-buffered by step parity: these pointers address buffer 0 and
  // element p + sbuf is the same element of buffer 1
  long sbuf;
  gfloat *vx, *vz, *sxx, *szz, *sxz;
  gfloat* psx[4];                // x-strip memory variables [nz][2P]: VXX, VZX, XX, XZ
  gfloat* psz[4];                // z-strip memory variables [2P][nx]: VXZ, VZZ, ZZ, XZ
  // adjoint state in scaled variables: u_bar = b v_bar at the velocity nodes and
  // t_bar = C sigma_bar at the stress nodes (t_xx = (l+2m) s_xx + l s_zz, t_zz = l s_xx +
  // (l+2m) s_zz, t_xz = mu_xz s_xz), an invertible change of variables for Vs > 0
  // (double-buffered by step parity like the forward state: element p + abuf is the same
  // element of buffer 1)
  long abuf;
  gfloat *uxb, *uzb, *txxb, *tzzb, *txzb;
  gfloat* pbx[2][4];             // double-buffered x-strip adjoint memory variables
  gfloat* pbz[2][4];             // double-buffered z-strip adjoint memory variables
  // staged parameters at the normal nodes (padded; the halo repeats the last row and column)
  gfloat *lam, *mu, *rho;
  // VTI (Thomsen eps, delta = eps / 2): staged c11 and c13 at the normal nodes (c33 is
  // lambda + 2 mu), and the window of the eps model (unpadded, full-model pitch); NULL in
  // an isotropic medium
  gfloat *c11, *c13;
  const gfloat* meps;
  // CPML profiles: axi bxi axh bxh [nx] then azi bzi azh bzh [nz]
  const gfloat* prof;
  // source
  const gfloat* src;             // [3][nt]
  gfloat* src_bar;               // [3][nt] (adjoint only)
  // DAS
  const gint* row_slot;          // [nz]: slot of the row in rowch, or -1
  const gint* rowch;             // [nslots][nx]: channel id at normal node, or -1
  gfloat* e;                     // [nch] running strain
  gfloat* d;                     // [nch][nt]
  const gfloat* ebar;            // [nt][nch] reverse cumulative residual
  // model window (unpadded, full-model pitch) for the chain rule
  const gfloat *mvp, *mvs, *mrho;
  long mld;
  // imaging
  gfloat* seg;                   // [L][5][cells]
  gfloat* acc;                   // [5][cells]
  gdouble* G;                    // [3][cells]
  // gradient output: slot of the extended gradient, full-model plane size, window origin
  gfloat* gout;
  long mplane;
  int z0, x0;
};

// A batch of shots advanced together: device descriptors and the flat tile list (tiles of
// shot s are tile_first[s] .. tile_first[s] + tiles(s) - 1; tile_shot maps tile -> shot),
// and two launch schedules: workgroup w processes tile sched[w] (-1: none). Both cut the
// tile list into one contiguous run per XCD of equal weighted cost, with the weights of
// the forward (and pointwise) kernels in `fwd` and those of the adjoint kernels in `adj`.
struct Sched {
  const int* sched;
  int n;
};
// A slot of a fused-step schedule as the kernel reads it (one scalar load per workgroup):
// the tile's shot (-1: empty slot), first row, first column and code path.
constexpr int PATH_INTERIOR = 0;   // no CPML, halo inside the grid
constexpr int PATH_EDGE = 1;       // halo may leave the grid (a grid without CPML)
constexpr int PATH_PML = 2;        // the tile or its halo touches a CPML strip
struct StepSlot {
  int shot, i0, j0, path;
};
struct StepSched {
  const StepSlot* slot;
  int n;
};
struct Batch2D {
  const Shot2D* shots;
  const int* tile_shot;      // 4-row tiles (pointwise kernels)
  const int* tile_first;
  Sched fwd;
  int ns, ntiles;
  // schedules of the fused forward step (tiles of fwd_rows rows) and of the fused
  // transposed step (adj_rows rows), 64 columns wide
  StepSched step, adj_step;
  int fwd_rows, adj_rows;
  int vti;                   // the shots' medium is VTI (the fused steps' VTI instances)
};

// Rows of a fused-step tile (64 columns wide): the kernels are built for these heights and
// the autotuner picks one for each of the two fused steps.
constexpr int TILE_ROWS[3] = {8, 12, 16};
constexpr int DEFAULT_TILE_ROWS = 8;
inline bool valid_tile_rows(int r) { return r == 8 || r == 12 || r == 16; }

// Number of XCDs the hardware deals workgroups to, round robin.
constexpr int NUM_XCD = 8;

// 3D tiles: TILE3_X columns (x) by TILE3_Y rows (y) of one z plane, covered by a workgroup
// of TILE3_X x TILE3_TY threads (each thread takes every TILE3_TY-th row). A shot's tiles
// are listed by group of TILE3_BANDS y bands (slowest), then z plane, then y band inside the
// group, then x block, so consecutive tiles march down z through one group of bands: the z
// neighbours of a tile were touched a few tiles earlier, and so were the y-halo rows of the
// bands inside its group (2 bands: the 300 x 400 x 400 sample's four half steps 0.1-1.3%
// faster than with 1; 4 bands: the forward ones faster, the transposed velocity step slower).
constexpr int TILE3_X = 64, TILE3_Y = 16, TILE3_TY = 4, TILE3_BANDS = 2;
__host__ __device__ inline int tiles3(int nz, int ny, int nx) {
  return nz * ((ny + TILE3_Y - 1) / TILE3_Y) * ((nx + TILE3_X - 1) / TILE3_X);
}
__host__ __device__ inline void tile3_coords(int local, int nz, int ny, int nx, int& i, int& k0, int& j0) {
  const int ntx = (nx + TILE3_X - 1) / TILE3_X, nb = (ny + TILE3_Y - 1) / TILE3_Y;
  const int per_group = nz * ntx * TILE3_BANDS;          // tiles of a full group of bands
  const int g = local / per_group, b0 = g * TILE3_BANDS;  // groups before this one are full
  const int gb = min(TILE3_BANDS, nb - b0);               // bands in this group
  int rem = local - g * per_group;
  i = rem / (gb * ntx);
  rem -= i * gb * ntx;
  const int band = b0 + rem / ntx;
  j0 = (rem - (band - b0) * ntx) * TILE3_X;
  k0 = band * TILE3_Y;
}
// Per-step bytes of the shots advanced together in one wave of a batch: 256 MiB, about the
// MI355X's 256 MB Infinity Cache (a sweep of 96-384 MiB on 64 uneven windows measured
// 96 and 128 MiB 8% slower and 192 MiB 0.8% slower than 256 MiB; 384 MiB gave the same
// waves as 256 MiB there).
constexpr size_t WAVE_CACHE_BYTES = (size_t)256 << 20;
// Lanes of a 2D batch by default (efwi_set_wave_lanes): two lanes ran the 64 uneven windows
// with sqrt(nt) checkpoints 4% faster than one (MI355X).
constexpr int DEFAULT_WAVE_LANES = 2;
// Relative cost of an interior tile and of a tile that touches a CPML strip, as integer
// weights (measured on MI355X with the 2D kernels: CPML tiles cost ~1.5x in the forward
// kernels and ~2x in the adjoint kernels, which also update the adjoint memory variables
// and stage corrected operands). The 3D adjoint CPML weight is 3.
constexpr int FWD_W_INT = 2, FWD_W_PML = 3;
constexpr int ADJ_W_INT = 1, ADJ_W_PML = 2;
constexpr int ADJ3_W_INT = 1, ADJ3_W_PML = 3;
// Bound on W_PML / W_INT over all schedules (sizes the schedule arrays).
constexpr int SCHED_RATIO = 3;
static_assert(FWD_W_PML <= SCHED_RATIO * FWD_W_INT && ADJ_W_PML <= SCHED_RATIO * ADJ_W_INT &&
                  ADJ3_W_PML <= SCHED_RATIO * ADJ3_W_INT,
              "schedule capacity assumes W_PML <= SCHED_RATIO * W_INT");

// Strip index helpers (x: column j of width nx; z: row i of height nz).
__host__ __device__ inline int strip_index(int k, int n, int P) {
  if (P <= 0) return -1;
  if (k < P) return k;
  if (k >= n - P) return k - (n - 2 * P);
  return -1;
}

// Kernel launchers (kernels2d.hip). All enqueue on `st` and return hipGetLastError().
// `kstore` / `k` index the step inside the checkpoint segment buffer (-1: do not store).
hipError_t launch_stage2d(const Batch2D& b, hipStream_t st);
// Fused forward step n: reads state buffer n & 1, writes buffer (n + 1) & 1.
hipError_t launch_fwd_step(const Batch2D& b, int n, int kstore, bool record, hipStream_t st);
// Fused transposed step n: reads adjoint buffer (n + 1) & 1, writes buffer n & 1.
hipError_t launch_adj_step(const Batch2D& b, int n, int k, bool grad, bool first, bool srcadj, hipStream_t st);
hipError_t launch_chain_flush(const Batch2D& b, hipStream_t st);
hipError_t launch_write_gradient(const Batch2D& b, hipStream_t st);
// Per-shot (host copy of the shot's descriptor).
hipError_t launch_misfit(const Shot2D& s, const float* d, const float* dobs, double* partial,
                         double* phi, float* ebar, hipStream_t st);
hipError_t launch_residual_cumsum(const Shot2D& s, const float* r, float* ebar, hipStream_t st);
// The same on plain sizes (any dimension): d, d_obs, r [nch][nt]; e_bar [nt][nch].
hipError_t launch_misfit_raw(int nch, int nt, const float* d, const float* dobs, double* partial, double* phi,
                             float* ebar, hipStream_t st);
hipError_t launch_residual_cumsum_raw(int nch, int nt, const float* r, float* ebar, hipStream_t st);

// 16-bit checkpoints (checkpoint.hip): the fields of a state block (2D: five padded
// wavefields and eight CPML strip arrays; 3D: nine and eighteen), as element offsets and
// lengths; `n` is the number of fields used.
constexpr int CKPT_NFIELDS = 27;
constexpr int CKPT_HEADER = 256;          // bytes of per-field scales at the head of a slot
constexpr int CKPT_CODEC_BF16 = 1;        // values of efwi_shot.ckpt_mode
constexpr int CKPT_CODEC_FP16 = 2;
struct CkptFields {
  long off[CKPT_NFIELDS];
  long len[CKPT_NFIELDS];
  int n;
};
hipError_t launch_ckpt_encode(const float* state, const CkptFields& f, unsigned int* maxbits, void* slot, int codec,
                              hipStream_t st);
hipError_t launch_ckpt_decode(float* state, const CkptFields& f, const void* slot, int codec, hipStream_t st);

// Regularizer (regularizer.hip).
hipError_t launch_regularizer(int ns, long npts, long plane, const float* m_ext, const float* b,
                              const unsigned char* sink, float eta, float* g_ext, double* partial,
                              int nblocks, double* phi, hipStream_t st);
int regularizer_blocks(long npts);
// One source's zone of influence for k_zoi (efwi_zoi in FP64).
struct ZoiArgs {
  double src[3], icov[6], box[6], taper, n, nu;
};
// Up to ZOI_BATCH zones per launch, passed by value (the launch's arguments stay below 4 KB).
constexpr int ZOI_BATCH = 16;
struct ZoiBatch {
  ZoiArgs z[ZOI_BATCH];
};
// Zones zb.z[0 .. count) into b[s][npts], sink[s][npts] (s counted from the batch's first).
hipError_t launch_zoi(int three, int count, long npts, int nz, int ny, int nx, double dz, double dy, double dx,
                      const ZoiBatch& zb, float* b, unsigned char* sink, hipStream_t st);
hipError_t launch_final_model(int ns, long npts, const float* m_ext, const float* b, const unsigned char* sink,
                              float* m_out, hipStream_t st);
// Extension along groups of shots (regularizer.hip): one shot's FP64 gradient sums of its
// window, rounded to FP32, added into its group's gradient component.
hipError_t launch_add_gradient(const double* G, long cells, int cp, int nz, int ny, int nx, float* out, long mplane,
                               long mrow, long mslab, int z0, int y0, int x0, hipStream_t st);

// Cubic B-spline model parameterization (bspline.hip): node count of an axis of n cells with
// node spacing D, expansion of coefficient planes and its transpose.
int bspline_nodes(int n, int D);
hipError_t launch_bspline_expand(int np, int nz, int nx, int Dz, int Dx, const float* c, float* m, hipStream_t st);
hipError_t launch_bspline_adjoint(int np, int nz, int nx, int Dz, int Dx, const float* g, float* cb, hipStream_t st);

// Field-like DAS sampling of recorded point strains (receiver.hip): gauge mean of `gauge`
// consecutive channels, strain rate when `rate`, every decim-th sample. Identity when
// gauge = decim = 1 and rate = 0 (the library then keeps the plain misfit path).
struct Receiver {
  int nch, nt, gauge, decim, rate;
  float rdt;  // 1 / dt
  bool identity() const { return gauge == 1 && decim == 1 && rate == 0; }
  int nf() const { return nch - gauge + 1; }
  int ntf() const { return nt / decim; }
};
hipError_t launch_field_data(const Receiver& R, const float* e, float* out, hipStream_t st);
hipError_t launch_field_misfit(const Receiver& R, const float* e, const float* dobs, float* rf, double* partial,
                               double* phi, float* ebar, hipStream_t st);
hipError_t launch_field_cumsum(const Receiver& R, const float* rf, float* ebar, hipStream_t st);

// Approximate inverse pseudo-Hessian (precondition.hip): the forward step with the velocity
// autocorrelation into acc[0], the window sum into the full grid, the clipped inverse
// (partial: inverse_diag_partials(n) floats of scratch).
hipError_t launch_fwd_acorr(const Batch2D& b, int n, hipStream_t st);
hipError_t launch_add_window(const float* acc, int cp, int nz, int nx, float* h, long mld, int z0, int x0,
                             hipStream_t st);
int inverse_diag_partials(long n);
hipError_t launch_inverse_diag(const float* h, long n, float clip, float* p, float* partial, hipStream_t st);

// ---------------------------------------------------------------------------------------
// 3D. Arrays are [nz][ny][nx]; padded arrays have the same zero halo in z and y as in 2D
// and the XOFF / ROW_ALIGN layout in x; element (i, k, j) is at p[i * pz + k * ld + j].
// ---------------------------------------------------------------------------------------
constexpr int NSEG3 = 9;   // stored per step: tr/(3l+2m), dev_xx m, dev_yy m (normal node),
                           // the three shear strain rates x their modulus / 4 (shear nodes),
                           // qx bx / 2, qy by / 2, qz bz / 2 (velocity nodes)
constexpr int NACC3 = 3;   // imaging sums gathered at the normal node: lambda, mu^2 x (mu part
                           // beyond 2/3 lambda's), rho

struct Shot3D {
  int nz, ny, nx, ld, P;
  long pz;                      // padded plane stride
  int nt, nch;
  int si, sk, sj;               // source normal node (window coordinates)
  float dt, rdx, rdy, rdz, w;   // w = dt / (dx dy dz)
  int cp;                       // x pitch of the unpadded per-cell arrays
  long cells;                   // nz * ny * cp
  gfloat *vx, *vy, *vz, *sxx, *syy, *szz, *sxy, *sxz, *syz;
  gfloat* psx[6];               // x-strips [nz][ny][2P]
  gfloat* psy[6];               // y-strips [nz][2P][nx]
  gfloat* psz[6];               // z-strips [2P][ny][nx]
  gfloat *uxb, *uyb, *uzb, *txxb, *tyyb, *tzzb, *txyb, *txzb, *tyzb;   // scaled adjoint state
  gfloat* pbx[2][6];
  gfloat* pby[2][6];
  gfloat* pbz[2][6];
  gfloat *l2m, *lam, *muxy, *muxz, *muyz;
  // density and mu at the normal nodes, padded, with the last plane, row and column repeated
  // one node beyond the grid: the step kernels derive the buoyancies and harmonic shear
  // moduli from them (the moduli bitwise the staged ones, which the transposed stress
  // kernel and the source adjoint read)
  gfloat *rho, *mu;
  const gfloat* prof;           // x: a_int b_int a_half b_half [nx] each, then y [ny], then z [nz]
  const gfloat* src;            // [6][nt]
  gfloat* src_bar;
  const gint* row_slot;         // [nz * ny]
  const gint* rowch;            // [nslots][nx]
  gfloat* e;
  gfloat* d;
  const gfloat* ebar;
  const gfloat *mvp, *mvs, *mrho;
  long mld, mplanestride;       // x pitch and z-plane stride of the full model
  gfloat* seg;                  // [L][9][cells]
  gfloat* acc;                  // [8][cells]
  gdouble* G;                   // [3][cells]
  gfloat* gout;
  long mplane;                  // elements of one full-model parameter volume
  int z0, y0, x0;
};

struct Batch3D {
  const Shot3D* shots;
  const int* tile_shot;
  const int* tile_first;
  Sched fwd, adj;
  int ns, ntiles;
};

hipError_t launch3_stage(const Batch3D& b, hipStream_t st);
hipError_t launch3_fwd_vel(const Batch3D& b, int kstore, hipStream_t st);
hipError_t launch3_fwd_str(const Batch3D& b, int n, int kstore, bool record, hipStream_t st);
hipError_t launch3_adj_vel(const Batch3D& b, int n, int k, bool grad, bool first, bool srcadj, hipStream_t st);
hipError_t launch3_adj_str(const Batch3D& b, int n, int k, bool grad, bool first, hipStream_t st);
hipError_t launch3_chain_flush(const Batch3D& b, hipStream_t st);
hipError_t launch3_write_gradient(const Batch3D& b, hipStream_t st);

}  // namespace efwi
