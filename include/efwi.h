/*
 * efwi.h - C ABI of the MI355X (gfx950) library for the hot path of source-extended
 * elastic full-waveform inversion (Bader, Clapp, Nihei, Biondi: "Source footprint
 * elimination in full-waveform inversion by model extension").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Array arguments marked DEVICE are device pointers owned by the caller, contiguous,
 *   FP32 unless stated. Arrays marked HOST are read during the call only.
 * - Grid arrays are [nz][nx] with x fastest. A model m is [3][nz][nx] = (Vp, Vs, rho)
 *   in m/s, m/s, kg/m^3. An extended model is [ns][3][nz][nx].
 * - DAS data are [nch][nt]: d[c][n] is the horizontal strain e_xx at channel c at time
 *   t_{n+1} = (n+1) dt.
 * - Source components are [3][nt] = (f_xx, f_zz, f_xz): the moment-tensor components times
 *   the moment-rate wavelet, sampled at t_{n+1/2} (Forward problem, eq.(2), MT case).
 * - The library allocates no device memory. Scratch comes from a caller-provided
 *   workspace of at least efwi_workspace_size() bytes (256-byte aligned). Workspaces
 *   must not be shared by calls that may overlap in time. (The one exception is
 *   efwi_shot_gradient_noalloc, whose scratch is a fixed array the library holds per GPU.)
 * - Every call is asynchronous on the given HIP stream (hipStream_t passed as void*);
 *   scalar results (misfits) are written to DEVICE doubles.
 * - All arguments are validated on the host before anything is enqueued; on error the
 *   call returns a negative efwi_status, enqueues nothing, and efwi_last_error() holds a
 *   message (thread-local). No exception crosses the ABI.
 * - Results are deterministic: no floating-point atomics on any result path.
 *
 * Discretization (the paper gives none; this is the reading implemented): first-order
 * velocity-stress system, staggered grid (sxx, szz at (i,j); vx at (i,j+1/2); vz at
 * (i+1/2,j); sxz at (i+1/2,j+1/2)), 4th-order differences (9/8, -1/24), leapfrog in time,
 * values outside the grid zero, unsplit CPML (kappa = 1) in strips of npml cells.
 */
#ifndef EFWI_H
#define EFWI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EFWI_OK = 0,
  EFWI_E_INVAL = -1,        /* null pointer, bad size, duplicate channel, nt < 1 ...   */
  EFWI_E_RANGE = -2,        /* source or channel outside the window interior / in CPML */
  EFWI_E_CFL = -3,          /* dt * vp_max * (9/8 + 1/24) * sqrt(sum 1/h^2) >= 1       */
  EFWI_E_WORKSPACE = -4,    /* workspace smaller than efwi_workspace_size()            */
  EFWI_E_HIP = -5,          /* a HIP runtime call failed (message in efwi_last_error)  */
  EFWI_E_NONFINITE = -6,    /* reserved: non-finite value detected                      */
  EFWI_E_UNSUPPORTED = -7   /* option not supported (a VTI medium on a 3D grid, ...)    */
} efwi_status;

/* Simulation grid. In the batched call nz, nx are the extended model's full size and each
 * shot runs on its own window. */
typedef struct {
  int ndim;        /* 2                                                              */
  int nz, ny, nx;  /* grid points; ny = 1 in 2D                                      */
  float dz, dy, dx;/* spacing in m                                                   */
  float dt;        /* time step in s                                                 */
  int nt;          /* number of time steps                                           */
  int npml;        /* CPML thickness in cells, inside each window (0: rigid walls)   */
  float pml_R;     /* CPML target reflection coefficient (e.g. 1e-3)                 */
  float pml_f0;    /* CPML frequency-shift parameter alpha_max = pi * pml_f0         */
  float vp_max;    /* caller's bound on Vp: CFL check and CPML damping d0            */
  /* VTI medium (the field example's starting model: vertical symmetry axis, Thomsen eps,
   * delta = eps / 2): DEVICE [nz][nx] eps of the full model, or NULL for an isotropic
   * medium. The model's (Vp, Vs, rho) are then (Vp0, Vs0, rho): c33 = rho Vp0^2,
   * c55 = rho Vs0^2, c11 = c33 (1 + 2 eps), c13 = sqrt((c33 - c55)(c33 (1 + eps) - c55))
   * - c55; gradients are with respect to (Vp0, Vs0, rho) at fixed eps. vp_max must bound
   * the horizontal P speed Vp0 sqrt(1 + 2 eps). 2D only (EFWI_E_UNSUPPORTED in 3D). */
  const float* eps;
} efwi_grid;

/* Checkpoint storage modes for the reverse sweep (wavefield recomputation). */
enum { EFWI_CKPT_FP32 = 0, EFWI_CKPT_BF16 = 1, EFWI_CKPT_FP16 = 2 };

/* One shot: a moment-tensor source, its DAS channels and its subdomain window. */
typedef struct {
  int src_iz, src_iy, src_ix; /* normal node of the source, full-model coordinates       */
  int nch;                    /* number of DAS channels (>= 0)                           */
  const int* ch_iz;           /* HOST [nch] channel normal nodes (full-model coords)     */
  const int* ch_iy;           /* HOST [nch], may be NULL in 2D                           */
  const int* ch_ix;           /* HOST [nch]                                              */
  int z0, y0, x0;             /* window origin in the full model                         */
  int wz, wy, wx;             /* window size; 0 means "to the end of the model"          */
  int ckpt_interval;          /* time steps per checkpoint segment; 0 = ceil(sqrt(nt));
                                 >= nt = keep the whole forward history (no recompute)   */
  int ckpt_mode;              /* EFWI_CKPT_*                                             */
  /* DAS sampling K_r of eq.(3). The kernels record the x-x strain e_c(t_{n+1}) at every
   * channel's normal node; with the defaults (0 or 1, 1, 0) that point strain [nch][nt] is
   * the shot's data. Otherwise the data are field-like, [nch - gauge + 1][nt / decim]:
   * field channel f is the mean over the gauge of channels f .. f + gauge - 1 (consecutive
   * in the list, i.e. along the fiber), as strain rate (e(t_{n+1}) - e(t_n)) / dt with
   * e(t_0) = 0 when rate = 1, sampled at t_{n+1} = k decim dt, k = 1, 2, ... Every entry
   * point then reads and writes data in that shape (d, d_obs, r, v, d_out) and the misfit
   * and gradients are those of the field data.                                         */
  int gauge;                  /* channels per gauge length (0 or 1: point strain)        */
  int decim;                  /* resampling factor in time steps (0 or 1: every step)    */
  int rate;                   /* 1: strain rate, 0: strain                               */
} efwi_shot;

/* Which entry point a workspace is sized for. */
typedef enum {
  EFWI_WS_FORWARD = 0,
  EFWI_WS_ADJOINT = 1,
  EFWI_WS_GRADIENT = 2,
  EFWI_WS_BATCH = 3,
  EFWI_WS_REGULARIZER = 4
} efwi_ws_kind;

/* Workspace bytes needed by one call of the given kind (0 on invalid arguments; see
 * efwi_last_error). For EFWI_WS_BATCH, shots points to ns HOST descriptors. */
size_t efwi_workspace_size(efwi_ws_kind kind, const efwi_grid* grid, int ns, const efwi_shot* shots);

/* Checkpoint interval for a memory budget (host only, no HIP call): the largest
 * ckpt_interval L whose EFWI_WS_GRADIENT workspace for this shot (with its ckpt_mode) fits
 * in budget_bytes. L = nt keeps the whole forward history and the reverse sweep recomputes
 * nothing; otherwise it recomputes (ceil(nt / L) - 1) L of the nt steps, so the larger L
 * the less work. The search starts from ceil(sqrt(nt)), the default interval. (The
 * gradient of eq.(6) cross-correlates the forward and adjoint wavefields, Solving the
 * inverse problem; how the forward history is kept is an implementation choice.) Returns L > 0, or a
 * negative efwi_status: EFWI_E_WORKSPACE when even ceil(sqrt(nt)) does not fit, or the
 * status efwi_validate reports. */
int efwi_plan_interval(const efwi_grid* grid, const efwi_shot* shot, size_t budget_bytes);

/* Host-side validation only (no HIP call): the checks every entry point runs first. */
efwi_status efwi_validate(const efwi_grid* grid, int ns, const efwi_shot* shots);

/* model_forward: d = K_r u_s(m) for one shot (Forward problem, eqs.(1)-(3)).
 *   m   DEVICE [3][nz][nx] model (Vp, Vs, rho); only the shot's window is read.
 *   src DEVICE [3][nt] source components.
 *   d   DEVICE [nch][nt] output, overwritten. */
efwi_status efwi_model_forward(const efwi_grid* grid, const efwi_shot* shot, const float* m,
                               const float* src, float* d, void* ws, size_t ws_bytes, void* stream);

/* model_adjoint: src_bar = L^T r, the exact transpose of model_forward with respect to the
 * source components (used for the dot-product test <L f, r> = <f, L^T r>).
 *   r       DEVICE [nch][nt] data-space input.
 *   src_bar DEVICE [3][nt] output, overwritten. */
efwi_status efwi_model_adjoint(const efwi_grid* grid, const efwi_shot* shot, const float* m,
                               const float* r, float* src_bar, void* ws, size_t ws_bytes, void* stream);

/* shot_gradient: data misfit phi_s = 1/2 ||d_s(m_s) - d_obs||^2 (eq.(4), data term of
 * eq.(8)) and its gradient g_s = J_s^T (d_s - d_obs) (eq.(6)) with respect to m_s =
 * (Vp, Vs, rho): the exact transpose of the discrete forward map, computed by the
 * adjoint-state method with checkpointed recomputation of the forward wavefield.
 *   d_obs DEVICE [nch][nt].
 *   g     DEVICE [3][nz][nx] output, overwritten (zero outside the shot's window).
 *   phi   DEVICE double, overwritten.
 *   d_out DEVICE [nch][nt] predicted data, or NULL. */
efwi_status efwi_shot_gradient(const efwi_grid* grid, const efwi_shot* shot, const float* m,
                               const float* src, const float* d_obs, float* g, double* phi,
                               float* d_out, void* ws, size_t ws_bytes, void* stream);

/* shot_jt: g = J_s^T v for a data-space vector v [nch][nt] (eq.(6) with the residual
 * replaced by v): the backward of the differentiable map m_s -> d_s, for any data-space
 * loss. The forward wavefield is recomputed from checkpoints as in efwi_shot_gradient
 * (same workspace size).
 *   v     DEVICE [nch][nt]; g DEVICE [3][nz][nx] output (zero outside the window);
 *   d_out DEVICE [nch][nt] predicted data, or NULL. */
efwi_status efwi_shot_jt(const efwi_grid* grid, const efwi_shot* shot, const float* m, const float* src,
                         const float* v, float* g, float* d_out, void* ws, size_t ws_bytes, void* stream);

/* shot_gradient_noalloc: efwi_shot_gradient for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation): the
 * same arguments without a workspace, the same results bit for bit. Its scratch is one
 * library-owned device array per GPU of EFWI_NOALLOC_SCRATCH_BYTES (64 MiB), held from the
 * first call on that GPU until the process ends; the call allocates no device or pinned
 * memory and creates no events (the kernel timing sampler skips it). Every call on a GPU
 * shares that GPU's array, so calls that may overlap in time on one GPU (several streams or
 * host threads) race and must not be made; sequential calls on one stream are safe (each
 * clears what must start at zero). Its small per-call tables are copied from host memory and
 * the call waits for that copy (and so for the stream's earlier work) before enqueueing the
 * time steps.
 * Errors: as efwi_shot_gradient; EFWI_E_WORKSPACE when the shot's gradient workspace
 * (efwi_workspace_size(EFWI_WS_GRADIENT, ...) with its ckpt_interval and ckpt_mode) exceeds
 * the scratch: choose a smaller ckpt_interval (efwi_plan_interval with this budget) or use
 * efwi_shot_gradient with a workspace. */
#define EFWI_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
efwi_status efwi_shot_gradient_noalloc(const efwi_grid* grid, const efwi_shot* shot, const float* m,
                                       const float* src, const float* d_obs, float* g, double* phi, float* d_out,
                                       void* stream);
/* The scratch size of efwi_shot_gradient_noalloc in bytes (EFWI_NOALLOC_SCRATCH_BYTES). */
size_t efwi_noalloc_scratch_bytes(void);

/* batch_gradient: the data term of eq.(8) for ns shots at once, each shot s on its own
 * component m_s of the extended model and its own window, advanced in waves (one launch per
 * half step covers every tile of a wave's shots; the waves and lanes efwi_batch_waves
 * reports). Each shot's results are bitwise those of efwi_shot_gradient, whatever the waves.
 * With two lanes the call also enqueues work on the library's second stream of the current
 * device; the caller's stream waits for it before the call's work is complete there.
 *   m_ext DEVICE [ns][3][nz][nx]; src DEVICE [ns][3][nt];
 *   d_obs DEVICE concatenation of the shots' [nch_s][nt] blocks in shot order;
 *   g_ext DEVICE [ns][3][nz][nx] output, overwritten (slot s holds g_s);
 *   phi   DEVICE double [ns] output. */
efwi_status efwi_batch_gradient(const efwi_grid* grid, int ns, const efwi_shot* shots,
                                const float* m_ext, const float* src, const float* d_obs,
                                float* g_ext, double* phi, void* ws, size_t ws_bytes, void* stream);

/* batch_gradient_grouped: the data term of eq.(8) with the model extended along groups of
 * sources instead of single ones (the paper's suggestion for surveys with many shots):
 * shot s runs on component group[s] of an extended model with ng components, and each
 * component's gradient is the sum of its shots' gradients (each shot's FP64 sums rounded
 * to FP32, then added in shot order, so the result does not depend on the waves).
 *   group HOST int [ns], 0 <= group[s] < ng;
 *   m_ext DEVICE [ng][3][nz][nx]; src DEVICE [ns][3][nt]; d_obs as in efwi_batch_gradient;
 *   g_ext DEVICE [ng][3][nz][nx] output, overwritten; phi DEVICE double [ns] output.
 * The regularizer, zones and final model then take ng components. */
efwi_status efwi_batch_gradient_grouped(const efwi_grid* grid, int ns, const efwi_shot* shots, const int* group,
                                        int ng, const float* m_ext, const float* src, const float* d_obs,
                                        float* g_ext, double* phi, void* ws, size_t ws_bytes, void* stream);

/* batch_waves: how efwi_batch_gradient groups the ns shots into waves (shots advanced
 * together, one launch per half step) for a workspace of ws_bytes. 2D: the shots are packed
 * first fit, largest first (by workspace bytes), into as few waves as the workspace holds
 * while each wave's per-step state (both state buffers, imaging sums and parameters) stays
 * within 256 MiB, about the MI355X's 256 MB Infinity Cache, so that each step finds most of
 * the previous step's state cached (efwi_set_wave_cache_bytes); a wave holds at least one
 * shot. With two lanes (efwi_set_wave_lanes) the plan is that of each lane's half, waves
 * 2m and 2m+1 running side by side. 3D waves take the shots in order, limited by the
 * workspace only. (efwi_batch_gradient_grouped keeps the shot order and one lane.)
 *   nwaves     HOST int output: number of waves;
 *   wave_first HOST int [ns] output (may be NULL): start of each wave in `order`;
 *   order      HOST int [ns] output (may be NULL): the shots in the order the waves take them,
 *              wave w being order[wave_first[w]] .. order[wave_first[w+1] - 1], ascending;
 *   lanes      HOST int output (may be NULL): 1 or 2, the lanes that advance the waves.
 * EFWI_E_WORKSPACE if one shot alone does not fit. */
efwi_status efwi_batch_waves(const efwi_grid* grid, int ns, const efwi_shot* shots, size_t ws_bytes,
                             int* nwaves, int* wave_first, int* order, int* lanes);

/* Per-step state bound of a 2D wave (efwi_batch_waves, efwi_batch_gradient, and the calls
 * that advance shots in waves): a wave takes shots while their per-step state stays within
 * `bytes`; the default, 256 MiB, is about the MI355X's 256 MB Infinity Cache.
 * (size_t)-1 sizes waves by the workspace alone; 0 restores the default. Process-wide,
 * applies to calls planned after it; results do not depend on it (each shot's arithmetic is
 * the same in any wave). Always EFWI_OK. */
efwi_status efwi_set_wave_cache_bytes(size_t bytes);
size_t efwi_get_wave_cache_bytes(void);

/* Lanes of a 2D batch (efwi_batch_gradient, efwi_batch_waves): with 2, the workspace is split
 * into two halves and consecutive waves alternate between them, one half advanced on the
 * caller's stream and the other on a second stream the library creates on the current
 * device (default priority, once per device); every time step is enqueued for both waves in
 * turn, so one wave's launches fill the end of the other's. Each lane's waves keep half of
 * the per-step state bound (efwi_set_wave_cache_bytes). A batch uses two lanes when one lane
 * would take several waves, every shot fits half the workspace and the halves' plan has at
 * most about twice as many waves, none of them with more per-step state than the whole
 * bound, else one; shots whose
 * gradients add into a shared component (efwi_batch_gradient_grouped) always use one. The
 * caller's stream waits for the second one before the call returns its work; results are
 * bitwise those of one lane. lanes: 1 or 2, 0 restores the default (2). Process-wide,
 * applies to calls planned after it. EFWI_E_INVAL for other values. */
efwi_status efwi_set_wave_lanes(int lanes);
int efwi_get_wave_lanes(void);

/* extension_regularizer: value and gradient of 1/2 eta^2 ||(I - S^T S_w) W m~||^2 (eq.(8)
 * second term), with W from eq.(11) (sinkhole samples of m_s replaced by the b-weighted mix
 * of the other components; a row whose other weights sum to 0 is the identity), S_w from
 * eq.(12) (b'_s = 1 inside s's sinkhole, b_s elsewhere; points where sum b' = 0 contribute
 * nothing) and S^T the copy along shots. Pointwise in space, same weights for Vp, Vs, rho.
 *   m_ext DEVICE [ns][3][nz][nx]; b DEVICE [ns][nz][nx] weights in [0,1];
 *   sink  DEVICE unsigned char [ns][nz][nx], nonzero inside s's sinkhole;
 *   g_ext DEVICE [ns][3][nz][nx], ACCUMULATED (+=) so data and penalty gradients sum;
 *   phi   DEVICE double, overwritten with the penalty value. */
efwi_status efwi_extension_regularizer(const efwi_grid* grid, int ns, const float* m_ext,
                                       const float* b, const unsigned char* sink, float eta,
                                       float* g_ext, double* phi, void* ws, size_t ws_bytes,
                                       void* stream);

/* One source's zone of influence (Source zone of influence, eq.(10)). Node (i, k, j) of
 * the grid sits at (i dz, k dy, j dx) metres; the y entries are ignored in 2D. */
typedef struct {
  float src[3];   /* z, y, x of the sinkhole centre (normally the source), metres           */
  float icov[6];  /* zz, yy, xx, zy, zx, yx of the sinkhole's inverse covariance C^-1,
                     1/m^2, symmetric positive definite: the sinkhole is the ellipse
                     (ellipsoid) dp^T C^-1 dp < 1, dp = node - src                          */
  float box[6];   /* z0, z1, y0, y1, x0, x1: the zone's active part (b = 1 there outside
                     the sinkhole), metres                                                  */
  float taper;    /* width of the outer transition beyond the box, metres (0: a step)      */
} efwi_zoi;

/* zoi_weights: the ZOI weights b_s of eq.(10) and the sinkhole flags of ns sources on the
 * full grid: b = (cos^n(pi r / 2) - ln nu) / (1 - ln nu), r the larger of the outer
 * transition's (Euclidean distance to the box over the taper, capped at 1) and the
 * sinkhole's (1 - d inside the sinkhole, d the Mahalanobis distance to src), so b is 1 in
 * the active part and (-ln nu) / (1 - ln nu) at the source; sink = (d < 1), decided in
 * FP64 with a fixed summation order. The outputs feed efwi_extension_regularizer and
 * efwi_final_model.
 *   zones HOST [ns]; n > 0 sets the transition's stiffness, 0 < nu < 1 its height;
 *   b     DEVICE [ns][nz][nx] (3D [ns][nz][ny][nx]) FP32 output;
 *   sink  DEVICE unsigned char, same shape, output.
 * FP64 arithmetic, one launch per 16 sources on `stream`. EFWI_E_INVAL for a box with an upper
 * bound below its lower bound, a negative taper, an inverse covariance that is not positive
 * definite, non-finite values, or n, nu out of range. */
efwi_status efwi_zoi_weights(const efwi_grid* grid, int ns, const efwi_zoi* zones, float n, float nu,
                             float* b, unsigned char* sink, void* stream);

/* final_model: the physical model m = S_w W m~ of eq.(9) from an extended model, with W
 * (eq.(11)) and S_w (eq.(12)) as in efwi_extension_regularizer; 0 where the weights b'
 * sum to 0 (no source is useful there).
 *   m_ext DEVICE [ns][3][nz][nx]; b, sink as in efwi_extension_regularizer;
 *   m_out DEVICE [3][nz][nx] output (3D: [3][nz][ny][nx]).
 * FP64 arithmetic, one launch on `stream`. */
efwi_status efwi_final_model(const efwi_grid* grid, int ns, const float* m_ext, const float* b,
                             const unsigned char* sink, float* m_out, void* stream);

/* Cubic B-spline model parameterization (the smoothing regularization of the field example,
 * which describes the model by cubic B-spline coefficients on a node grid of 50 m in x and
 * the grid spacing in z). Along an axis of n cells with node spacing D cells (D >= 1), node
 * k = 0 .. N-1 sits at cell (k - 1) D and carries the uniform cubic B-spline
 * B((i - (k - 1) D) / D): 2/3 - t^2 + |t|^3/2 for |t| < 1, (2 - |t|)^3 / 6 for 1 <= |t| < 2,
 * 0 beyond; N = ceil((n - 1) / D) + 3 nodes, so the basis sums to one on the grid.
 * efwi_bspline_nodes: N (0 for n < 1 or D < 1).
 * efwi_bspline_expand: m = Bz c Bx^T for np planes; c DEVICE [np][Nz][Nx], m DEVICE
 *   [np][nz][nx] output.
 * efwi_bspline_adjoint: c_bar = Bz^T g Bx (the transpose: gradients with respect to the
 *   coefficients); g DEVICE [np][nz][nx], c_bar DEVICE [np][Nz][Nx] output.
 * FP64 weights and sums, one launch on `stream`; EFWI_E_INVAL for sizes or spacings below
 * 1, spacings summing to more than 2000 cells (the weight tables live in LDS) or NULL
 * arrays. */
int efwi_bspline_nodes(int n, int spacing);
efwi_status efwi_bspline_expand(int nz, int nx, int dz_nodes, int dx_nodes, int np, const float* c, float* m,
                                void* stream);
efwi_status efwi_bspline_adjoint(int nz, int nx, int dz_nodes, int dx_nodes, int np, const float* g, float* c_bar,
                                 void* stream);

/* das_field: the field data K e of a shot (see efwi_shot's DAS sampling) from recorded point
 * strains, e.g. of a shot with the default sampling.
 *   e   DEVICE [nch][nt] point strains (x-x strain at each channel at t_{n+1});
 *   out DEVICE [nch - gauge + 1][nt / decim] output.
 * FP64 arithmetic, one launch on `stream`. EFWI_E_INVAL for an invalid grid or shot. */
efwi_status efwi_das_field(const efwi_grid* grid, const efwi_shot* shot, const float* e, float* out, void* stream);

/* pseudo_hessian: the approximate inverse pseudo-Hessian that the paper gives l-BFGS as
 * its initial inverse Hessian in the comparison with alternative methods (synthetic
 * example): the zero-lag autocorrelation in time of the particle velocity, summed over
 * shots, clipped and scaled. Each shot s runs the forward problem on its own component
 * m_s and window (no data are recorded) and adds, at every normal node of its window,
 * vx^2 + vz^2 of the velocities of every step (vx at (i, j+1/2), vz at (i+1/2, j)); then
 *   h = sum over shots (0 outside every window), FP32 sums in time, shots added in order;
 *   p = c max(h) / max(h, c max(h)), c = clip: 1 where h <= c max(h), smallest (c) where
 *       h is largest; p = 1 everywhere if h is 0.
 * 2D only. Shots advance in waves as in efwi_batch_gradient.
 *   m_ext DEVICE [ns][3][nz][nx]; src DEVICE [ns][3][nt];
 *   clip  in (0, 1];
 *   h     DEVICE [nz][nx] output (raw sums); p DEVICE [nz][nx] output (the operator);
 *   ws    at least efwi_workspace_size(EFWI_WS_GRADIENT, ...) of the largest shot.
 * EFWI_E_INVAL for a 3D grid, a clip outside (0, 1] or NULL arrays; EFWI_E_WORKSPACE if
 * one shot does not fit. */
efwi_status efwi_pseudo_hessian(const efwi_grid* grid, int ns, const efwi_shot* shots, const float* m_ext,
                                const float* src, float clip, float* h, float* p, void* ws, size_t ws_bytes,
                                void* stream);

/* Tile shape of the fused 2D forward and transposed time-step kernels: tiles of 8, 12 or
 * 16 rows by 64 columns (the stencil halo is recomputed per tile, so taller tiles recompute
 * less but hold more LDS and registers). Results do not depend on the choice (every node
 * is computed by the same arithmetic whichever tile holds it). Process-wide; applies to
 * calls planned after it. efwi_set_tile_rows: 0 keeps a value; EFWI_E_INVAL for other
 * values. */
efwi_status efwi_set_tile_rows(int fwd_rows, int adj_rows);
efwi_status efwi_get_tile_rows(int* fwd_rows, int* adj_rows);

/* Autotuner of the tile shape: times the shot's forward and transposed sweeps over `steps`
 * time steps (whole history kept, FP32) for each tile height (a warm-up run, then the best
 * of two), on the given stream, keeps the fastest for each sweep (efwi_set_tile_rows) and
 * returns them in *fwd_rows and *adj_rows. Blocks until the timing runs end. 2D grids
 * only (EFWI_E_UNSUPPORTED for 3D).
 *   m, src   DEVICE as in efwi_shot_gradient (src is read for the first `steps` samples);
 *   ws       DEVICE workspace of efwi_autotune_workspace_size() bytes (0 on invalid input);
 *   times_ms HOST [3][2] (forward, transposed sweep ms for 8, 12, 16 rows), or NULL.
 * Must not overlap other calls that plan work. */
size_t efwi_autotune_workspace_size(const efwi_grid* grid, const efwi_shot* shot, int steps);
efwi_status efwi_autotune(const efwi_grid* grid, const efwi_shot* shot, const float* m, const float* src,
                          int steps, void* ws, size_t ws_bytes, void* stream, int* fwd_rows, int* adj_rows,
                          float* times_ms);

/* Kernel timing sampler (profiling aid, off by default). With sample_every = k > 0, every
 * k-th launch of each kernel kind (at least every 8th) opens a window of up to 8
 * consecutive launches of that kind, bracketed by two HIP events recorded on the launches'
 * stream; another kind's launch closes the window early; 0 turns sampling off.
 * efwi_timing_query() waits for the pending events of one kind and returns the number of
 * launches, of timed launches and their summed duration in ms. Kinds are
 * 0 .. efwi_kernel_count() - 1, named by efwi_kernel_name(). */
efwi_status efwi_timing_enable(int sample_every);
efwi_status efwi_timing_reset(void);
efwi_status efwi_timing_query(int kind, long* launches, long* timed, double* total_ms);
int efwi_kernel_count(void);
const char* efwi_kernel_name(int kind);

/* Human-readable name of a status code (static storage). */
const char* efwi_status_string(efwi_status s);
/* Message of the last failing call on this thread (static thread-local storage). */
const char* efwi_last_error(void);
/* Library version string. */
const char* efwi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EFWI_H */
