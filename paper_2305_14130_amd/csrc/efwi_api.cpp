// Host side of the C ABI declared in include/efwi.h: argument validation, workspace
// planning, upload of the small per-shot tables, and the time-stepping schedule
// (forward sweep with checkpoints, misfit, reverse sweep by segments with recomputation,
// chain rule into the shot's own component of the extended gradient).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "efwi.h"
#include "efwi_internal.h"

using namespace efwi;

namespace {

thread_local std::string g_last_error;

efwi_status fail(efwi_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) return fail(EFWI_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// ----------------------------------------------------------------------------------------
// Pinned staging ring for the small host -> device tables (CPML profiles, channel maps).
// A slot is reused only after the event recorded behind its copy has completed.
// ----------------------------------------------------------------------------------------
class Staging {
 public:
  hipError_t upload(void* dst, const void* src, size_t bytes, hipStream_t st) {
    std::lock_guard<std::mutex> lock(mu_);
    Slot& s = slots_[next_];
    next_ = (next_ + 1) % kSlots;
    hipError_t e;
    if (s.ev && s.used) {
      e = hipEventSynchronize(s.ev);
      if (e != hipSuccess) return e;
    }
    if (!s.ev) {
      e = hipEventCreateWithFlags(&s.ev, hipEventDisableTiming);
      if (e != hipSuccess) return e;
    }
    if (s.cap < bytes) {
      if (s.host) hipHostFree(s.host);
      s.host = nullptr;
      s.cap = 0;
      e = hipHostMalloc(&s.host, bytes, hipHostMallocDefault);
      if (e != hipSuccess) return e;
      s.cap = bytes;
    }
    std::memcpy(s.host, src, bytes);
    e = hipMemcpyAsync(dst, s.host, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    e = hipEventRecord(s.ev, st);
    s.used = (e == hipSuccess);
    return e;
  }

 private:
  static constexpr int kSlots = 8;
  struct Slot {
    void* host = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool used = false;
  };
  std::mutex mu_;
  Slot slots_[kSlots];
  int next_ = 0;
};

Staging& staging() {
  static Staging* s = new Staging();  // lives for the process; never torn down at exit
  return *s;
}

// ----------------------------------------------------------------------------------------
// Kernel timing sampler: when enabled, every `every`-th launch of each kernel kind is
// bracketed by two HIP events recorded on the launch stream; durations are collected when
// queried. Off by default (no events in the hot loop).
// ----------------------------------------------------------------------------------------
enum KernelKind { KK_FWD_VEL = 0, KK_FWD_STR, KK_ADJ_VEL, KK_ADJ_STR, KK_CHAIN, KK_MISFIT, KK_REG, KK_COUNT };
const char* const kKernelNames[KK_COUNT] = {"fwd_vel", "fwd_str", "adj_vel", "adj_str",
                                            "chain_flush", "misfit", "regularizer"};

class Sampler {
 public:
  void enable(int every) {
    std::lock_guard<std::mutex> lock(mu_);
    every_ = every;
  }
  template <class F>
  hipError_t run(int kind, hipStream_t st, F&& launch) {
    if (every_ <= 0) return launch();
    std::unique_lock<std::mutex> lock(mu_);
    const bool take = (launched_[kind]++ % every_) == 0;
    hipEvent_t a = nullptr, b = nullptr;
    if (take) {
      hipError_t e = get_event(&a);
      if (e == hipSuccess) e = get_event(&b);
      if (e != hipSuccess) return e;
      e = hipEventRecord(a, st);
      if (e != hipSuccess) return e;
    }
    lock.unlock();
    hipError_t e = launch();
    if (e != hipSuccess || !take) return e;
    e = hipEventRecord(b, st);
    lock.lock();
    pending_[kind].push_back({a, b});
    return e;
  }
  hipError_t query(int kind, long* launched, long* timed, double* total_ms) {
    std::lock_guard<std::mutex> lock(mu_);
    for (auto& pr : pending_[kind]) {
      hipError_t e = hipEventSynchronize(pr.second);
      if (e != hipSuccess) return e;
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, pr.first, pr.second);
      if (e != hipSuccess) return e;
      total_ms_[kind] += ms;
      ++timed_[kind];
      free_.push_back(pr.first);
      free_.push_back(pr.second);
    }
    pending_[kind].clear();
    *launched = launched_[kind];
    *timed = timed_[kind];
    *total_ms = total_ms_[kind];
    return hipSuccess;
  }
  hipError_t reset() {
    std::lock_guard<std::mutex> lock(mu_);
    for (int k = 0; k < KK_COUNT; ++k) {
      for (auto& pr : pending_[k]) {
        hipError_t e = hipEventSynchronize(pr.second);
        if (e != hipSuccess) return e;
        free_.push_back(pr.first);
        free_.push_back(pr.second);
      }
      pending_[k].clear();
      launched_[k] = timed_[k] = 0;
      total_ms_[k] = 0.0;
    }
    return hipSuccess;
  }

 private:
  hipError_t get_event(hipEvent_t* ev) {
    if (!free_.empty()) {
      *ev = free_.back();
      free_.pop_back();
      return hipSuccess;
    }
    return hipEventCreate(ev);
  }
  std::mutex mu_;
  int every_ = 0;
  long launched_[KK_COUNT] = {};
  long timed_[KK_COUNT] = {};
  double total_ms_[KK_COUNT] = {};
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending_[KK_COUNT];
  std::vector<hipEvent_t> free_;
};

Sampler& sampler() {
  static Sampler* s = new Sampler();
  return *s;
}

#define TIMED(kind, st, call) sampler().run((kind), (st), [&]() { return (call); })

// ----------------------------------------------------------------------------------------
// Validation.
// ----------------------------------------------------------------------------------------
struct Window {
  int z0, x0, wz, wx;
};

Window window_of(const efwi_grid& g, const efwi_shot& s) {
  Window w;
  w.z0 = s.z0;
  w.x0 = s.x0;
  w.wz = s.wz > 0 ? s.wz : g.nz - s.z0;
  w.wx = s.wx > 0 ? s.wx : g.nx - s.x0;
  return w;
}

int strip_width(const efwi_grid& g) { return g.npml > 0 ? g.npml + 1 : 0; }

efwi_status validate_grid(const efwi_grid* g) {
  if (!g) return fail(EFWI_E_INVAL, "grid is NULL");
  if (g->ndim == 3) return fail(EFWI_E_UNSUPPORTED, "3D grids are not supported by this entry point");
  if (g->ndim != 2) return fail(EFWI_E_INVAL, "ndim must be 2 (got %d)", g->ndim);
  if (g->nz < 1 || g->nx < 1) return fail(EFWI_E_INVAL, "grid size %d x %d", g->nz, g->nx);
  if (!(g->dx > 0.f) || !(g->dz > 0.f) || !(g->dt > 0.f))
    return fail(EFWI_E_INVAL, "dx, dz, dt must be positive");
  if (g->nt < 1) return fail(EFWI_E_INVAL, "nt must be >= 1 (got %d)", g->nt);
  if (g->npml < 0) return fail(EFWI_E_INVAL, "npml must be >= 0");
  if (!(g->vp_max > 0.f)) return fail(EFWI_E_INVAL, "vp_max must be positive");
  if (g->npml > 0 && !(g->pml_R > 0.f && g->pml_R < 1.f)) return fail(EFWI_E_INVAL, "pml_R must be in (0, 1)");
  if (g->npml > 0 && !(g->pml_f0 >= 0.f)) return fail(EFWI_E_INVAL, "pml_f0 must be >= 0");
  const double courant = (double)g->dt * g->vp_max * (9.0 / 8.0 + 1.0 / 24.0) *
                         std::sqrt(1.0 / ((double)g->dx * g->dx) + 1.0 / ((double)g->dz * g->dz));
  if (!(courant < 1.0)) return fail(EFWI_E_CFL, "unstable time step: Courant number %.4f >= 1", courant);
  return EFWI_OK;
}

efwi_status validate_shot(const efwi_grid& g, const efwi_shot* s, int index) {
  if (!s) return fail(EFWI_E_INVAL, "shot %d descriptor is NULL", index);
  const Window w = window_of(g, *s);
  const int P = strip_width(g);
  if (w.z0 < 0 || w.x0 < 0 || w.wz < 1 || w.wx < 1 || w.z0 + w.wz > g.nz || w.x0 + w.wx > g.nx)
    return fail(EFWI_E_RANGE, "shot %d: window [%d,+%d) x [%d,+%d) outside the %d x %d model", index, w.z0, w.wz,
                w.x0, w.wx, g.nz, g.nx);
  if (w.wz < 2 * P + 4 || w.wx < 2 * P + 4)
    return fail(EFWI_E_RANGE, "shot %d: window %d x %d too small for %d CPML cells", index, w.wz, w.wx, g.npml);
  const int si = s->src_iz - w.z0, sj = s->src_ix - w.x0;
  if (si < P + 1 || si > w.wz - P - 1 || sj < P + 1 || sj > w.wx - P - 1)
    return fail(EFWI_E_RANGE, "shot %d: source (%d,%d) not in the window interior outside the CPML", index,
                s->src_iz, s->src_ix);
  if (s->nch < 0) return fail(EFWI_E_INVAL, "shot %d: nch < 0", index);
  if (s->nch > 0 && (!s->ch_iz || !s->ch_ix)) return fail(EFWI_E_INVAL, "shot %d: channel arrays are NULL", index);
  std::vector<long> keys;
  keys.reserve(s->nch);
  for (int c = 0; c < s->nch; ++c) {
    const int ci = s->ch_iz[c] - w.z0, cj = s->ch_ix[c] - w.x0;
    if (ci < P || ci > w.wz - P - 1 || cj < P || cj > w.wx - P - 1)
      return fail(EFWI_E_RANGE, "shot %d: channel %d at (%d,%d) outside the window interior", index, c, s->ch_iz[c],
                  s->ch_ix[c]);
    keys.push_back((long)ci * w.wx + cj);
  }
  std::sort(keys.begin(), keys.end());
  if (std::adjacent_find(keys.begin(), keys.end()) != keys.end())
    return fail(EFWI_E_INVAL, "shot %d: two channels share one grid node", index);
  if (s->ckpt_interval < 0) return fail(EFWI_E_INVAL, "shot %d: ckpt_interval < 0", index);
  if (s->ckpt_mode != EFWI_CKPT_FP32 && s->ckpt_mode != EFWI_CKPT_BF16 && s->ckpt_mode != EFWI_CKPT_FP16)
    return fail(EFWI_E_INVAL, "shot %d: unknown ckpt_mode %d", index, s->ckpt_mode);
  return EFWI_OK;
}

// ----------------------------------------------------------------------------------------
// Workspace plan of one 2D shot.
// ----------------------------------------------------------------------------------------
struct Plan2D {
  Window w;
  int nz, nx, ld, cp, rows, P, nslots, nt, nch, L, nseg;
  long plane, cells;
  size_t state_bytes;  // padded fields + forward CPML strips (one checkpoint)
  size_t off_state, off_e, off_adj, off_par, off_tab, tab_bytes, off_ebar, off_partial, off_dint, off_acc, off_G,
      off_seg, off_ckpt, total;
  size_t adj_bytes, par_bytes;
};

size_t strips_floats(int nz, int nx, int P) { return (size_t)4 * nz * 2 * P + (size_t)4 * 2 * P * nx; }

int count_slots(const efwi_shot& s, const Window& w) {
  std::vector<int> rows;
  for (int c = 0; c < s.nch; ++c) rows.push_back(s.ch_iz[c] - w.z0);
  std::sort(rows.begin(), rows.end());
  rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
  return (int)rows.size();
}

Plan2D plan2d(const efwi_grid& g, const efwi_shot& s, efwi_ws_kind kind) {
  Plan2D p{};
  p.w = window_of(g, s);
  p.nz = p.w.wz;
  p.nx = p.w.wx;
  p.ld = (XOFF + p.nx + HALO + ROW_ALIGN - 1) / ROW_ALIGN * ROW_ALIGN;
  p.cp = (p.nx + ROW_ALIGN - 1) / ROW_ALIGN * ROW_ALIGN;
  p.rows = p.nz + 2 * HALO;
  p.plane = (long)p.rows * p.ld;
  p.cells = (long)p.nz * p.cp;
  p.P = strip_width(g);
  p.nt = g.nt;
  p.nch = s.nch;
  p.nslots = count_slots(s, p.w);
  int L = s.ckpt_interval > 0 ? s.ckpt_interval : (int)std::ceil(std::sqrt((double)g.nt));
  L = std::max(1, std::min(L, g.nt));
  p.L = L;
  p.nseg = (g.nt + L - 1) / L;
  const size_t strips = strips_floats(p.nz, p.nx, p.P);
  p.state_bytes = align_up(((size_t)5 * p.plane + strips) * sizeof(float));
  p.adj_bytes = align_up(((size_t)5 * p.plane + 2 * strips) * sizeof(float));
  p.par_bytes = align_up((size_t)5 * p.plane * sizeof(float));
  p.tab_bytes = align_up((size_t)(4 * p.nx + 4 * p.nz) * sizeof(float) + (size_t)p.nz * sizeof(int) +
                         (size_t)p.nslots * p.nx * sizeof(int));
  const bool fwd = kind != EFWI_WS_ADJOINT;
  const bool adj = kind != EFWI_WS_FORWARD;
  const bool grad = kind == EFWI_WS_GRADIENT || kind == EFWI_WS_BATCH;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align_up(bytes);
    return at;
  };
  p.off_par = take(p.par_bytes);
  p.off_tab = take(p.tab_bytes);
  p.off_state = fwd ? take(p.state_bytes) : 0;
  p.off_e = fwd ? take((size_t)std::max(1, p.nch) * sizeof(float)) : 0;
  p.off_adj = adj ? take(p.adj_bytes) : 0;
  p.off_ebar = adj ? take((size_t)std::max(1, p.nch) * p.nt * sizeof(float)) : 0;
  p.off_partial = grad ? take((size_t)std::max(1, p.nch) * sizeof(double)) : 0;
  p.off_dint = grad ? take((size_t)std::max(1, p.nch) * p.nt * sizeof(float)) : 0;
  p.off_acc = grad ? take((size_t)NACC * p.cells * sizeof(float)) : 0;
  p.off_G = grad ? take((size_t)3 * p.cells * sizeof(double)) : 0;
  p.off_seg = grad ? take((size_t)p.L * NSEG_FIELDS * p.cells * sizeof(float)) : 0;
  p.off_ckpt = grad ? take((size_t)std::max(0, p.nseg - 2) * p.state_bytes) : 0;
  p.total = o;
  return p;
}

// Host tables: CPML profiles (computed in double, stored FP32), row -> slot map, and the
// [slot][x] channel map.
void cpml_profile(std::vector<float>& a, std::vector<float>& b, int n, double h, const efwi_grid& g, bool half) {
  a.assign(n, 0.f);
  b.assign(n, 1.f);
  if (g.npml <= 0) return;
  const double L = g.npml;
  const double d0 = -3.0 * g.vp_max * std::log((double)g.pml_R) / (2.0 * L * h);
  for (int k = 0; k < n; ++k) {
    const double x = k + (half ? 0.5 : 0.0);
    const double xi = std::max(std::max(L - x, x - (n - 1 - L)), 0.0);
    const double r = std::min(xi / L, 1.0);
    const double d = d0 * r * r;
    const double alpha = M_PI * g.pml_f0 * (1.0 - r);
    const double bb = std::exp(-(d + alpha) * g.dt);
    const double den = d + alpha;
    a[k] = (float)(den > 0 ? d * (bb - 1.0) / den : 0.0);
    b[k] = (float)bb;
  }
}

std::vector<unsigned char> build_tables(const efwi_grid& g, const efwi_shot& s, const Plan2D& p) {
  std::vector<unsigned char> blob(p.tab_bytes, 0);
  float* prof = reinterpret_cast<float*>(blob.data());
  std::vector<float> a, b;
  const int nx = p.nx, nz = p.nz;
  cpml_profile(a, b, nx, g.dx, g, false);
  std::copy(a.begin(), a.end(), prof);
  std::copy(b.begin(), b.end(), prof + nx);
  cpml_profile(a, b, nx, g.dx, g, true);
  std::copy(a.begin(), a.end(), prof + 2 * nx);
  std::copy(b.begin(), b.end(), prof + 3 * nx);
  cpml_profile(a, b, nz, g.dz, g, false);
  std::copy(a.begin(), a.end(), prof + 4 * nx);
  std::copy(b.begin(), b.end(), prof + 4 * nx + nz);
  cpml_profile(a, b, nz, g.dz, g, true);
  std::copy(a.begin(), a.end(), prof + 4 * nx + 2 * nz);
  std::copy(b.begin(), b.end(), prof + 4 * nx + 3 * nz);
  int* row_slot = reinterpret_cast<int*>(prof + 4 * nx + 4 * nz);
  int* rowch = row_slot + nz;
  std::fill(row_slot, row_slot + nz, -1);
  std::fill(rowch, rowch + (size_t)p.nslots * nx, -1);
  int nslots = 0;
  for (int c = 0; c < s.nch; ++c) {
    const int ci = s.ch_iz[c] - p.w.z0, cj = s.ch_ix[c] - p.w.x0;
    if (row_slot[ci] < 0) row_slot[ci] = nslots++;
    rowch[(size_t)row_slot[ci] * nx + cj] = c;
  }
  return blob;
}

Shot2D make_desc(const efwi_grid& g, const efwi_shot& s, const Plan2D& p, unsigned char* ws, const float* m,
                 long mplane) {
  Shot2D d{};
  d.nz = p.nz;
  d.nx = p.nx;
  d.ld = p.ld;
  d.P = p.P;
  d.nt = p.nt;
  d.nch = p.nch;
  d.si = s.src_iz - p.w.z0;
  d.sj = s.src_ix - p.w.x0;
  d.dt = g.dt;
  d.rdx = (float)(1.0 / g.dx);
  d.rdz = (float)(1.0 / g.dz);
  d.w = (float)((double)g.dt / ((double)g.dx * g.dz));
  d.cp = p.cp;
  d.cells = p.cells;
  const long interior = (long)HALO * p.ld + XOFF;
  const size_t strips = strips_floats(p.nz, p.nx, p.P);
  auto fields = [&](size_t off, float** out, int count) {
    float* base = reinterpret_cast<float*>(ws + off);
    for (int k = 0; k < count; ++k) out[k] = base + k * p.plane + interior;
    return base + (size_t)5 * p.plane;  // strips follow the five planes
  };
  auto strips_at = [&](float* base, float** px, float** pz) {
    const size_t xs = (size_t)p.nz * 2 * p.P, zs = (size_t)2 * p.P * p.nx;
    for (int k = 0; k < 4; ++k) px[k] = base + k * xs;
    for (int k = 0; k < 4; ++k) pz[k] = base + 4 * xs + k * zs;
  };
  {
    float* f[5];
    float* st = fields(p.off_state, f, 5);
    d.vx = f[0];
    d.vz = f[1];
    d.sxx = f[2];
    d.szz = f[3];
    d.sxz = f[4];
    strips_at(st, d.psx, d.psz);
  }
  {
    float* f[5];
    float* st = fields(p.off_adj, f, 5);
    d.uxb = f[0];
    d.uzb = f[1];
    d.txxb = f[2];
    d.tzzb = f[3];
    d.txzb = f[4];
    strips_at(st, d.pbx[0], d.pbz[0]);
    strips_at(st + strips, d.pbx[1], d.pbz[1]);
  }
  {
    float* f[5];
    fields(p.off_par, f, 5);
    d.l2m = f[0];
    d.lam = f[1];
    d.muxz = f[2];
    d.bx = f[3];
    d.bz = f[4];
  }
  float* prof = reinterpret_cast<float*>(ws + p.off_tab);
  d.prof = prof;
  d.row_slot = reinterpret_cast<const int*>(prof + 4 * p.nx + 4 * p.nz);
  d.rowch = d.row_slot + p.nz;
  d.e = reinterpret_cast<float*>(ws + p.off_e);
  d.ebar = reinterpret_cast<const float*>(ws + p.off_ebar);
  d.acc = reinterpret_cast<float*>(ws + p.off_acc);
  d.G = reinterpret_cast<double*>(ws + p.off_G);
  d.seg = reinterpret_cast<float*>(ws + p.off_seg);
  const long mld = g.nx;
  const float* mw = m + (long)p.w.z0 * mld + p.w.x0;
  d.mvp = mw;
  d.mvs = mw + mplane;
  d.mrho = mw + 2 * mplane;
  d.mld = mld;
  return d;
}

efwi_status check_ws(const void* ws, size_t have, size_t need) {
  if (need > 0 && !ws) return fail(EFWI_E_INVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % ALIGN != 0) return fail(EFWI_E_INVAL, "workspace not 256-byte aligned");
  if (have < need) return fail(EFWI_E_WORKSPACE, "workspace has %zu bytes, needs %zu", have, need);
  return EFWI_OK;
}

// Common set-up: zero what must start at zero, upload the tables, stage the parameters.
efwi_status setup_shot(const efwi_grid& g, const efwi_shot& s, const Plan2D& p, unsigned char* ws, Shot2D& d,
                       bool fwd, bool adj, bool grad, hipStream_t st) {
  HIP_TRY(hipMemsetAsync(ws + p.off_par, 0, p.par_bytes, st));
  if (fwd) {
    HIP_TRY(hipMemsetAsync(ws + p.off_state, 0, p.state_bytes, st));
    HIP_TRY(hipMemsetAsync(ws + p.off_e, 0, (size_t)std::max(1, p.nch) * sizeof(float), st));
  }
  if (adj) HIP_TRY(hipMemsetAsync(ws + p.off_adj, 0, p.adj_bytes, st));
  if (grad) HIP_TRY(hipMemsetAsync(ws + p.off_G, 0, (size_t)3 * p.cells * sizeof(double), st));
  std::vector<unsigned char> tab = build_tables(g, s, p);
  HIP_TRY(staging().upload(ws + p.off_tab, tab.data(), tab.size(), st));
  HIP_TRY(launch_stage2d(d, st));
  return EFWI_OK;
}

efwi_status run_forward(Shot2D& d, const Plan2D& p, unsigned char* ws, bool checkpoints, hipStream_t st) {
  const int last0 = (p.nseg - 1) * p.L;
  for (int n = 0; n < p.nt; ++n) {
    if (checkpoints && n % p.L == 0 && n > 0 && n < last0) {
      const int k = n / p.L;
      HIP_TRY(hipMemcpyAsync(ws + p.off_ckpt + (size_t)(k - 1) * p.state_bytes, ws + p.off_state, p.state_bytes,
                             hipMemcpyDeviceToDevice, st));
    }
    float* seg = nullptr;
    if (checkpoints && n >= last0) seg = d.seg + (size_t)(n - last0) * NSEG_FIELDS * p.cells;
    HIP_TRY(TIMED(KK_FWD_VEL, st, launch_fwd_vel(d, n, seg, st)));
    HIP_TRY(TIMED(KK_FWD_STR, st, launch_fwd_str(d, n, seg, true, st)));
  }
  return EFWI_OK;
}

efwi_status run_reverse(Shot2D& d, const Plan2D& p, unsigned char* ws, hipStream_t st) {
  for (int k = p.nseg - 1; k >= 0; --k) {
    const int n0 = k * p.L, n1 = std::min(p.nt, n0 + p.L);
    if (k < p.nseg - 1) {
      if (k == 0) HIP_TRY(hipMemsetAsync(ws + p.off_state, 0, p.state_bytes, st));
      else
        HIP_TRY(hipMemcpyAsync(ws + p.off_state, ws + p.off_ckpt + (size_t)(k - 1) * p.state_bytes, p.state_bytes,
                               hipMemcpyDeviceToDevice, st));
      for (int n = n0; n < n1; ++n) {
        float* seg = d.seg + (size_t)(n - n0) * NSEG_FIELDS * p.cells;
        HIP_TRY(TIMED(KK_FWD_VEL, st, launch_fwd_vel(d, n, seg, st)));
        HIP_TRY(TIMED(KK_FWD_STR, st, launch_fwd_str(d, n, seg, false, st)));
      }
    }
    // Imaging sums run in FP32 over blocks of FLUSH_STEPS steps aligned on absolute step
    // numbers and are then added into the FP64 gradient, so the result does not depend on
    // the checkpoint interval.
    for (int n = n1 - 1; n >= n0; --n) {
      const float* seg = d.seg + (size_t)(n - n0) * NSEG_FIELDS * p.cells;
      const bool first = (n == p.nt - 1) || ((n + 1) % FLUSH_STEPS == 0);
      HIP_TRY(TIMED(KK_ADJ_VEL, st, launch_adj_vel(d, n, seg, true, first, false, st)));
      HIP_TRY(TIMED(KK_ADJ_STR, st, launch_adj_str(d, n, seg, true, first, st)));
      if (n % FLUSH_STEPS == 0) HIP_TRY(TIMED(KK_CHAIN, st, launch_chain_flush(d, st)));
    }
  }
  return EFWI_OK;
}

efwi_status shot_gradient_impl(const efwi_grid& g, const efwi_shot& s, const float* m, long mplane, const float* src,
                               const float* d_obs, float* gout, double* phi, float* d_out, unsigned char* ws,
                               size_t ws_bytes, hipStream_t st, bool zero_outside) {
  const Plan2D p = plan2d(g, s, EFWI_WS_GRADIENT);
  efwi_status rc = check_ws(ws, ws_bytes, p.total);
  if (rc != EFWI_OK) return rc;
  Shot2D d = make_desc(g, s, p, ws, m, mplane);
  d.src = src;
  d.d = d_out ? d_out : reinterpret_cast<float*>(ws + p.off_dint);
  rc = setup_shot(g, s, p, ws, d, true, true, true, st);
  if (rc != EFWI_OK) return rc;
  rc = run_forward(d, p, ws, true, st);
  if (rc != EFWI_OK) return rc;
  HIP_TRY(TIMED(KK_MISFIT, st,
                launch_misfit(d, d.d, d_obs, reinterpret_cast<double*>(ws + p.off_partial), phi,
                              reinterpret_cast<float*>(ws + p.off_ebar), st)));
  rc = run_reverse(d, p, ws, st);
  if (rc != EFWI_OK) return rc;
  const bool full = p.w.z0 == 0 && p.w.x0 == 0 && p.nz == g.nz && p.nx == g.nx;
  if (zero_outside && !full) HIP_TRY(hipMemsetAsync(gout, 0, (size_t)3 * mplane * sizeof(float), st));
  HIP_TRY(launch_write_gradient(d, gout, mplane, p.w.z0, p.w.x0, st));
  return EFWI_OK;
}

}  // namespace

// ========================================================================================
// C ABI
// ========================================================================================
extern "C" {

const char* efwi_status_string(efwi_status s) {
  switch (s) {
    case EFWI_OK: return "EFWI_OK";
    case EFWI_E_INVAL: return "EFWI_E_INVAL";
    case EFWI_E_RANGE: return "EFWI_E_RANGE";
    case EFWI_E_CFL: return "EFWI_E_CFL";
    case EFWI_E_WORKSPACE: return "EFWI_E_WORKSPACE";
    case EFWI_E_HIP: return "EFWI_E_HIP";
    case EFWI_E_NONFINITE: return "EFWI_E_NONFINITE";
    case EFWI_E_UNSUPPORTED: return "EFWI_E_UNSUPPORTED";
  }
  return "EFWI_E_UNKNOWN";
}

const char* efwi_last_error(void) { return g_last_error.c_str(); }

const char* efwi_version(void) { return "efwi-gfx950 0.1"; }

efwi_status efwi_timing_enable(int sample_every) {
  if (sample_every < 0) return fail(EFWI_E_INVAL, "sample_every < 0");
  sampler().enable(sample_every);
  return EFWI_OK;
}

efwi_status efwi_timing_reset(void) {
  HIP_TRY(sampler().reset());
  return EFWI_OK;
}

efwi_status efwi_timing_query(int kind, long* launches, long* timed, double* total_ms) {
  if (kind < 0 || kind >= KK_COUNT) return fail(EFWI_E_INVAL, "unknown kernel kind %d", kind);
  if (!launches || !timed || !total_ms) return fail(EFWI_E_INVAL, "NULL output");
  HIP_TRY(sampler().query(kind, launches, timed, total_ms));
  return EFWI_OK;
}

const char* efwi_kernel_name(int kind) { return (kind >= 0 && kind < KK_COUNT) ? kKernelNames[kind] : ""; }

int efwi_kernel_count(void) { return KK_COUNT; }

efwi_status efwi_validate(const efwi_grid* grid, int ns, const efwi_shot* shots) {
  g_last_error.clear();
  efwi_status rc = validate_grid(grid);
  if (rc != EFWI_OK) return rc;
  if (ns < 0) return fail(EFWI_E_INVAL, "ns < 0");
  if (ns > 0 && !shots) return fail(EFWI_E_INVAL, "shots is NULL");
  for (int k = 0; k < ns; ++k) {
    rc = validate_shot(*grid, shots + k, k);
    if (rc != EFWI_OK) return rc;
  }
  return EFWI_OK;
}

size_t efwi_workspace_size(efwi_ws_kind kind, const efwi_grid* grid, int ns, const efwi_shot* shots) {
  if (kind == EFWI_WS_REGULARIZER) {
    if (validate_grid(grid) != EFWI_OK) return 0;
    const long npts = (long)grid->nz * grid->nx;
    return align_up((size_t)regularizer_blocks(npts) * sizeof(double));
  }
  if (efwi_validate(grid, kind == EFWI_WS_BATCH ? ns : 1, shots) != EFWI_OK) return 0;
  if (kind == EFWI_WS_BATCH) {
    size_t mx = 0;
    for (int k = 0; k < ns; ++k) mx = std::max(mx, plan2d(*grid, shots[k], kind).total);
    return mx;
  }
  return plan2d(*grid, *shots, kind).total;
}

efwi_status efwi_model_forward(const efwi_grid* grid, const efwi_shot* shot, const float* m, const float* src,
                               float* d, void* ws, size_t ws_bytes, void* stream) {
  efwi_status rc = efwi_validate(grid, 1, shot);
  if (rc != EFWI_OK) return rc;
  if (!m || !src || (shot->nch > 0 && !d)) return fail(EFWI_E_INVAL, "NULL array argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const Plan2D p = plan2d(*grid, *shot, EFWI_WS_FORWARD);
  rc = check_ws(ws, ws_bytes, p.total);
  if (rc != EFWI_OK) return rc;
  unsigned char* w = static_cast<unsigned char*>(ws);
  Shot2D dd = make_desc(*grid, *shot, p, w, m, (long)grid->nz * grid->nx);
  dd.src = src;
  dd.d = d;
  rc = setup_shot(*grid, *shot, p, w, dd, true, false, false, st);
  if (rc != EFWI_OK) return rc;
  return run_forward(dd, p, w, false, st);
}

efwi_status efwi_model_adjoint(const efwi_grid* grid, const efwi_shot* shot, const float* m, const float* r,
                               float* src_bar, void* ws, size_t ws_bytes, void* stream) {
  efwi_status rc = efwi_validate(grid, 1, shot);
  if (rc != EFWI_OK) return rc;
  if (!m || !src_bar || (shot->nch > 0 && !r)) return fail(EFWI_E_INVAL, "NULL array argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const Plan2D p = plan2d(*grid, *shot, EFWI_WS_ADJOINT);
  rc = check_ws(ws, ws_bytes, p.total);
  if (rc != EFWI_OK) return rc;
  unsigned char* w = static_cast<unsigned char*>(ws);
  Shot2D dd = make_desc(*grid, *shot, p, w, m, (long)grid->nz * grid->nx);
  dd.src_bar = src_bar;
  rc = setup_shot(*grid, *shot, p, w, dd, false, true, false, st);
  if (rc != EFWI_OK) return rc;
  HIP_TRY(launch_residual_cumsum(dd, r, reinterpret_cast<float*>(w + p.off_ebar), st));
  for (int n = p.nt - 1; n >= 0; --n) {
    HIP_TRY(launch_adj_vel(dd, n, nullptr, false, false, true, st));
    HIP_TRY(launch_adj_str(dd, n, nullptr, false, false, st));
  }
  return EFWI_OK;
}

efwi_status efwi_shot_gradient(const efwi_grid* grid, const efwi_shot* shot, const float* m, const float* src,
                               const float* d_obs, float* g, double* phi, float* d_out, void* ws, size_t ws_bytes,
                               void* stream) {
  efwi_status rc = efwi_validate(grid, 1, shot);
  if (rc != EFWI_OK) return rc;
  if (shot->ckpt_mode != EFWI_CKPT_FP32) return fail(EFWI_E_UNSUPPORTED, "16-bit checkpoints not built yet");
  if (!m || !src || !g || !phi || (shot->nch > 0 && !d_obs)) return fail(EFWI_E_INVAL, "NULL array argument");
  return shot_gradient_impl(*grid, *shot, m, (long)grid->nz * grid->nx, src, d_obs, g, phi, d_out,
                            static_cast<unsigned char*>(ws), ws_bytes, reinterpret_cast<hipStream_t>(stream), true);
}

efwi_status efwi_batch_gradient(const efwi_grid* grid, int ns, const efwi_shot* shots, const float* m_ext,
                                const float* src, const float* d_obs, float* g_ext, double* phi, void* ws,
                                size_t ws_bytes, void* stream) {
  efwi_status rc = efwi_validate(grid, ns, shots);
  if (rc != EFWI_OK) return rc;
  if (ns < 1) return fail(EFWI_E_INVAL, "ns must be >= 1");
  if (!m_ext || !src || !g_ext || !phi) return fail(EFWI_E_INVAL, "NULL array argument");
  const long plane = (long)grid->nz * grid->nx;
  size_t off_obs = 0;
  for (int s = 0; s < ns; ++s) {
    if (shots[s].ckpt_mode != EFWI_CKPT_FP32) return fail(EFWI_E_UNSUPPORTED, "16-bit checkpoints not built yet");
    if (shots[s].nch > 0 && !d_obs) return fail(EFWI_E_INVAL, "d_obs is NULL");
    rc = shot_gradient_impl(*grid, shots[s], m_ext + (size_t)s * 3 * plane, plane, src + (size_t)s * 3 * grid->nt,
                            d_obs ? d_obs + off_obs : nullptr, g_ext + (size_t)s * 3 * plane, phi + s, nullptr,
                            static_cast<unsigned char*>(ws), ws_bytes, reinterpret_cast<hipStream_t>(stream), true);
    if (rc != EFWI_OK) return rc;
    off_obs += (size_t)shots[s].nch * grid->nt;
  }
  return EFWI_OK;
}

efwi_status efwi_extension_regularizer(const efwi_grid* grid, int ns, const float* m_ext, const float* b,
                                       const unsigned char* sink, float eta, float* g_ext, double* phi, void* ws,
                                       size_t ws_bytes, void* stream) {
  g_last_error.clear();
  efwi_status rc = validate_grid(grid);
  if (rc != EFWI_OK) return rc;
  if (ns < 1) return fail(EFWI_E_INVAL, "ns must be >= 1");
  if (!m_ext || !b || !sink || !g_ext || !phi) return fail(EFWI_E_INVAL, "NULL array argument");
  if (!std::isfinite(eta)) return fail(EFWI_E_INVAL, "eta is not finite");
  const long npts = (long)grid->nz * grid->nx;
  const int nb = regularizer_blocks(npts);
  rc = check_ws(ws, ws_bytes, align_up((size_t)nb * sizeof(double)));
  if (rc != EFWI_OK) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  HIP_TRY(TIMED(KK_REG, st,
                launch_regularizer(ns, npts, npts, m_ext, b, sink, eta, g_ext, static_cast<double*>(ws), nb, phi,
                                   st)));
  return EFWI_OK;
}

}  // extern "C"
