// Host side of the C ABI declared in include/efwi.h: argument validation, workspace
// planning, upload of the small per-shot tables, and the time-stepping schedule
// (forward sweep with checkpoints, misfit, reverse sweep by segments with recomputation,
// chain rule into the shot's own component of the extended gradient).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
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

// Calls that must not allocate (efwi_shot_gradient_noalloc) upload their header with a plain
// copy from the planning code's host buffer instead of the staging ring (whose pinned slots
// are allocated on first use), and wait for it, since that buffer is freed on return.
thread_local bool t_no_alloc = false;
struct NoAllocScope {
  NoAllocScope() { t_no_alloc = true; }
  ~NoAllocScope() { t_no_alloc = false; }
};

hipError_t upload_header(void* dst, const std::vector<unsigned char>& blob, hipStream_t st) {
  if (!t_no_alloc) return staging().upload(dst, blob.data(), blob.size(), st);
  hipError_t e = hipMemcpyAsync(dst, blob.data(), blob.size(), hipMemcpyHostToDevice, st);
  return e != hipSuccess ? e : hipStreamSynchronize(st);
}

// ----------------------------------------------------------------------------------------
// Kernel timing sampler: when enabled, every `every`-th launch of each kernel kind opens a
// window of up to WINDOW consecutive launches of that kind on one stream, bracketed by two
// HIP events recorded on that stream (one event pair per window, so the event overhead is
// spread over its launches); a launch of another kind on the same stream closes the window
// early. Windows are kept per stream, so the two lanes of a batch are timed separately (a
// window's launches then share the GPU with the other lane's). Durations are collected when
// queried. Off by default (no events in the hot loop).
// ----------------------------------------------------------------------------------------
// fwd_vel, fwd_str, adj_vel and adj_str are the 3D half steps; fwd_step and adj_step are the
// fused 2D forward and transposed steps.
enum KernelKind {
  KK_FWD_VEL = 0, KK_FWD_STR, KK_ADJ_VEL, KK_ADJ_STR, KK_CHAIN, KK_MISFIT, KK_REG, KK_FWD_STEP, KK_ADJ_STEP,
  KK_ZOI, KK_FINAL, KK_ACORR, KK_COUNT
};
const char* const kKernelNames[KK_COUNT] = {"fwd_vel", "fwd_str",     "adj_vel",  "adj_str", "chain_flush",
                                            "misfit",  "regularizer", "fwd_step", "adj_step",
                                            "zoi",     "final_model", "fwd_acorr"};

class Sampler {
 public:
  static constexpr int WINDOW = 8;
  void enable(int every) {
    std::lock_guard<std::mutex> lock(mu_);
    every_ = every;
  }
  template <class F>
  hipError_t run(int kind, hipStream_t st, F&& launch) {
    if (every_ <= 0 || t_no_alloc) return launch();   // allocation-free calls create no events
    std::unique_lock<std::mutex> lock(mu_);
    for (int k = 0; k < KK_COUNT; ++k) {  // another kind's launch on this stream closes its open window
      Window* o = find(k, st);
      if (k != kind && o && o->active) {
        hipError_t e = hipEventRecord(o->b, o->st);
        if (e != hipSuccess) return e;
        pending_[k].push_back(*o);
        o->active = false;
      }
    }
    Window& w = window(kind, st);
    if (!w.active && (launched_[kind] % std::max(every_, WINDOW)) == 0) {
      hipError_t e = get_event(&w.a);
      if (e == hipSuccess) e = get_event(&w.b);
      if (e == hipSuccess) e = hipEventRecord(w.a, st);
      if (e != hipSuccess) return e;
      w.active = true;
      w.valid = true;
      w.count = 0;
    }
    ++launched_[kind];
    lock.unlock();
    hipError_t e = launch();
    if (e != hipSuccess) return e;
    lock.lock();
    Window& v = window(kind, st);
    if (v.active && ++v.count == WINDOW) {
      e = hipEventRecord(v.b, st);
      pending_[kind].push_back(v);
      v.active = false;
    }
    return e;
  }
  hipError_t query(int kind, long* launched, long* timed, double* total_ms) {
    std::lock_guard<std::mutex> lock(mu_);
    for (auto& w : pending_[kind]) {
      hipError_t e = hipEventSynchronize(w.b);
      if (e != hipSuccess) return e;
      if (w.valid) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, w.a, w.b);
        if (e != hipSuccess) return e;
        total_ms_[kind] += ms;
        timed_[kind] += w.count;
      }
      free_.push_back(w.a);
      free_.push_back(w.b);
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
      for (auto& w : pending_[k]) {
        hipError_t e = hipEventSynchronize(w.b);
        if (e != hipSuccess) return e;
        free_.push_back(w.a);
        free_.push_back(w.b);
      }
      pending_[k].clear();
      for (Window& o : open_[k])
        if (o.active) o.valid = false;   // closes later; its events are then recycled
      launched_[k] = timed_[k] = 0;
      total_ms_[k] = 0.0;
    }
    return hipSuccess;
  }

 private:
  struct Window {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t st = nullptr;
    int count = 0;
    bool active = false, valid = false;
  };
  // the open window of a kind on a stream (created inactive on first use)
  Window* find(int kind, hipStream_t st) {
    for (Window& w : open_[kind])
      if (w.st == st) return &w;
    return nullptr;
  }
  Window& window(int kind, hipStream_t st) {
    if (Window* w = find(kind, st)) return *w;
    open_[kind].push_back(Window{});
    open_[kind].back().st = st;
    return open_[kind].back();
  }
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
  std::vector<Window> open_[KK_COUNT];
  std::vector<Window> pending_[KK_COUNT];
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
  int z0, y0, x0, wz, wy, wx;
};

Window window_of(const efwi_grid& g, const efwi_shot& s) {
  Window w;
  w.z0 = s.z0;
  w.x0 = s.x0;
  w.wz = s.wz > 0 ? s.wz : g.nz - s.z0;
  w.wx = s.wx > 0 ? s.wx : g.nx - s.x0;
  const bool three = g.ndim == 3;
  w.y0 = three ? s.y0 : 0;
  w.wy = three ? (s.wy > 0 ? s.wy : g.ny - s.y0) : 1;
  return w;
}

int strip_width(const efwi_grid& g) { return g.npml > 0 ? g.npml + 1 : 0; }

efwi_status validate_grid(const efwi_grid* g) {
  if (!g) return fail(EFWI_E_INVAL, "grid is NULL");
  if (g->ndim != 2 && g->ndim != 3) return fail(EFWI_E_INVAL, "ndim must be 2 or 3 (got %d)", g->ndim);
  const bool three = g->ndim == 3;
  if (g->nz < 1 || g->nx < 1 || (three && g->ny < 1)) return fail(EFWI_E_INVAL, "bad grid size");
  if (!(g->dx > 0.f) || !(g->dz > 0.f) || !(g->dt > 0.f) || (three && !(g->dy > 0.f)))
    return fail(EFWI_E_INVAL, "grid spacings and dt must be positive");
  if (g->nt < 1) return fail(EFWI_E_INVAL, "nt must be >= 1 (got %d)", g->nt);
  if (g->npml < 0) return fail(EFWI_E_INVAL, "npml must be >= 0");
  if (g->eps && three) return fail(EFWI_E_UNSUPPORTED, "VTI media are 2D only");
  if (!(g->vp_max > 0.f)) return fail(EFWI_E_INVAL, "vp_max must be positive");
  if (g->npml > 0 && !(g->pml_R > 0.f && g->pml_R < 1.f)) return fail(EFWI_E_INVAL, "pml_R must be in (0, 1)");
  if (g->npml > 0 && !(g->pml_f0 >= 0.f)) return fail(EFWI_E_INVAL, "pml_f0 must be >= 0");
  double inv2 = 1.0 / ((double)g->dx * g->dx) + 1.0 / ((double)g->dz * g->dz);
  if (three) inv2 += 1.0 / ((double)g->dy * g->dy);
  const double courant = (double)g->dt * g->vp_max * (9.0 / 8.0 + 1.0 / 24.0) * std::sqrt(inv2);
  if (!(courant < 1.0)) return fail(EFWI_E_CFL, "unstable time step: Courant number %.4f >= 1", courant);
  return EFWI_OK;
}

// The shot's DAS sampling (0 in gauge or decim means 1).
Receiver receiver_of(const efwi_grid& g, const efwi_shot& s) {
  Receiver R{};
  R.nch = s.nch;
  R.nt = g.nt;
  R.gauge = s.gauge > 0 ? s.gauge : 1;
  R.decim = s.decim > 0 ? s.decim : 1;
  R.rate = s.rate;
  R.rdt = (float)(1.0 / (double)g.dt);
  return R;
}

// Data rows and samples of a shot as the caller sees them (field shape).
size_t data_floats(const efwi_grid& g, const efwi_shot& s) {
  const Receiver R = receiver_of(g, s);
  return s.nch > 0 ? (size_t)std::max(0, R.nf()) * R.ntf() : 0;
}

efwi_status validate_shot(const efwi_grid& g, const efwi_shot* s, int index) {
  if (!s) return fail(EFWI_E_INVAL, "shot %d descriptor is NULL", index);
  const bool three = g.ndim == 3;
  const Window w = window_of(g, *s);
  const int P = strip_width(g);
  if (w.z0 < 0 || w.x0 < 0 || w.y0 < 0 || w.wz < 1 || w.wx < 1 || w.wy < 1 || w.z0 + w.wz > g.nz ||
      w.x0 + w.wx > g.nx || (three && w.y0 + w.wy > g.ny))
    return fail(EFWI_E_RANGE, "shot %d: window outside the model", index);
  if (w.wz < 2 * P + 4 || w.wx < 2 * P + 4 || (three && w.wy < 2 * P + 4))
    return fail(EFWI_E_RANGE, "shot %d: window too small for %d CPML cells", index, g.npml);
  {  // the kernels address a shot's arrays with 32-bit byte offsets from uniform bases
    const long ld = (XOFF + w.wx + HALO + ROW_ALIGN - 1) / ROW_ALIGN * ROW_ALIGN;
    const long cp = (w.wx + ROW_ALIGN - 1) / ROW_ALIGN * ROW_ALIGN;
    const long padded = (long)(w.wz + 2 * HALO) * (three ? w.wy + 2 * HALO : 1) * ld;
    const long cells = (long)w.wz * w.wy * cp;
    // per-cell arrays addressed from one base: the history slots of a step and the imaging
    // sums (2D: NSEG_FIELDS and up to NACC_VTI; 3D: NSEG3 and NACC3), and the CPML strips
    const long per_cell = three ? std::max(NSEG3, NACC3) : std::max(NSEG_FIELDS, NACC_VTI);
    const long strips = three ? 0 : 4L * ((long)w.wz * 2 * P + (long)2 * P * w.wx);
    if (padded >= (1L << 30) || per_cell * cells >= (1L << 30) || strips >= (1L << 30))
      return fail(EFWI_E_RANGE, "shot %d: window of %ld cells is beyond this library's 2^30-element arrays", index,
                  (long)w.wz * w.wy * w.wx);
  }
  const int si = s->src_iz - w.z0, sj = s->src_ix - w.x0, sk = three ? s->src_iy - w.y0 : 0;
  if (si < P + 1 || si > w.wz - P - 1 || sj < P + 1 || sj > w.wx - P - 1 ||
      (three && (sk < P + 1 || sk > w.wy - P - 1)))
    return fail(EFWI_E_RANGE, "shot %d: source not in the window interior outside the CPML", index);
  if (s->nch < 0) return fail(EFWI_E_INVAL, "shot %d: nch < 0", index);
  if (s->nch > 0 && (!s->ch_iz || !s->ch_ix || (three && !s->ch_iy)))
    return fail(EFWI_E_INVAL, "shot %d: channel arrays are NULL", index);
  std::vector<long> keys;
  keys.reserve(s->nch);
  for (int c = 0; c < s->nch; ++c) {
    const int ci = s->ch_iz[c] - w.z0, cj = s->ch_ix[c] - w.x0, ck = three ? s->ch_iy[c] - w.y0 : 0;
    if (ci < P || ci > w.wz - P - 1 || cj < P || cj > w.wx - P - 1 || (three && (ck < P || ck > w.wy - P - 1)))
      return fail(EFWI_E_RANGE, "shot %d: channel %d outside the window interior", index, c);
    keys.push_back(((long)ci * w.wy + ck) * w.wx + cj);
  }
  std::sort(keys.begin(), keys.end());
  if (std::adjacent_find(keys.begin(), keys.end()) != keys.end())
    return fail(EFWI_E_INVAL, "shot %d: two channels share one grid node", index);
  if (s->ckpt_interval < 0) return fail(EFWI_E_INVAL, "shot %d: ckpt_interval < 0", index);
  if (s->gauge < 0 || s->decim < 0 || (s->rate != 0 && s->rate != 1))
    return fail(EFWI_E_INVAL, "shot %d: gauge and decim must be >= 0 and rate 0 or 1", index);
  if (s->nch > 0 && s->gauge > s->nch)
    return fail(EFWI_E_INVAL, "shot %d: gauge of %d channels exceeds its %d channels", index, s->gauge, s->nch);
  if (s->decim > g.nt) return fail(EFWI_E_INVAL, "shot %d: decim %d exceeds nt", index, s->decim);
  if (s->ckpt_mode != EFWI_CKPT_FP32 && s->ckpt_mode != EFWI_CKPT_BF16 && s->ckpt_mode != EFWI_CKPT_FP16)
    return fail(EFWI_E_INVAL, "shot %d: unknown ckpt_mode %d", index, s->ckpt_mode);
  return EFWI_OK;
}

// ----------------------------------------------------------------------------------------
// Workspace plan of one 2D shot (its private region of the workspace).
// ----------------------------------------------------------------------------------------
// Rows of the fused forward-step and transposed-step tiles for the plans made from now on
// (set by efwi_set_tile_rows or efwi_autotune; process-wide).
std::atomic<int> g_fwd_rows{DEFAULT_TILE_ROWS}, g_adj_rows{DEFAULT_TILE_ROWS};
// Per-step state bound of a 2D wave (efwi_set_wave_cache_bytes; process-wide).
std::atomic<size_t> g_wave_cache_bytes{WAVE_CACHE_BYTES};
// Lanes of a 2D batch (efwi_set_wave_lanes; process-wide): 1 or 2.
std::atomic<int> g_wave_lanes{DEFAULT_WAVE_LANES};

struct Plan2D {
  Window w;
  int nz, nx, ld, cp, rows, P, nslots, nt, nch, L, nseg, ntiles;
  int fwd_rows, adj_rows, nfwd_tiles, nadj_tiles;   // fused-step tiles
  long plane, cells;
  size_t state_bytes;  // padded fields + forward CPML strips
  size_t state_elems;
  int ckpt_mode;
  size_t slot_bytes;   // one checkpoint (FP32 copy of the state block, or 16-bit codes)
  CkptFields fields;
  size_t tab_bytes;    // CPML profiles + channel maps (kept in the batch header)
  size_t off_state, off_e, off_adj, off_par, off_ebar, off_partial, off_dint, off_acc, off_G, off_seg, off_ckpt,
      off_maxbits, off_rf, total;
  size_t adj_bytes, par_bytes;
  Receiver R;
  bool field;          // the DAS sampling is not the identity
};

size_t strips_floats(int nz, int nx, int P) { return (size_t)4 * nz * 2 * P + (size_t)4 * 2 * P * nx; }

int count_slots(const efwi_shot& s, const Window& w) {
  std::vector<int> rows;
  for (int c = 0; c < s.nch; ++c) rows.push_back(s.ch_iz[c] - w.z0);
  std::sort(rows.begin(), rows.end());
  rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
  return (int)rows.size();
}

int interval_of(const efwi_grid& g, const efwi_shot& s) {
  int L = s.ckpt_interval > 0 ? s.ckpt_interval : (int)std::ceil(std::sqrt((double)g.nt));
  return std::max(1, std::min(L, g.nt));
}

Plan2D plan2d(const efwi_grid& g, const efwi_shot& s, efwi_ws_kind kind, int fwd_rows = 0, int adj_rows = 0) {
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
  p.ntiles = ((p.nx + BX - 1) / BX) * ((p.nz + BZ - 1) / BZ);
  p.fwd_rows = fwd_rows > 0 ? fwd_rows : g_fwd_rows.load();
  p.adj_rows = adj_rows > 0 ? adj_rows : g_adj_rows.load();
  p.nfwd_tiles = ((p.nx + BX - 1) / BX) * ((p.nz + p.fwd_rows - 1) / p.fwd_rows);
  p.nadj_tiles = ((p.nx + BX - 1) / BX) * ((p.nz + p.adj_rows - 1) / p.adj_rows);
  p.L = interval_of(g, s);
  p.nseg = (g.nt + p.L - 1) / p.L;
  const size_t strips = strips_floats(p.nz, p.nx, p.P);
  p.state_elems = (size_t)5 * p.plane + strips;
  p.state_bytes = align_up(p.state_elems * sizeof(float));
  p.ckpt_mode = s.ckpt_mode;
  p.slot_bytes = s.ckpt_mode == EFWI_CKPT_FP32 ? p.state_bytes
                                               : align_up(CKPT_HEADER + p.state_elems * sizeof(unsigned short));
  {
    const long xs = (long)p.nz * 2 * p.P, zs = (long)2 * p.P * p.nx;
    p.fields.n = 13;
    for (int k = 0; k < 5; ++k) {
      p.fields.off[k] = k * p.plane;
      p.fields.len[k] = p.plane;
    }
    for (int k = 0; k < 4; ++k) {
      p.fields.off[5 + k] = 5 * p.plane + k * xs;
      p.fields.len[5 + k] = xs;
      p.fields.off[9 + k] = 5 * p.plane + 4 * xs + k * zs;
      p.fields.len[9 + k] = zs;
    }
  }
  // adjoint fields double-buffered by step parity (10 planes), then the two buffers of the
  // adjoint memory variables
  p.adj_bytes = align_up(((size_t)10 * p.plane + 2 * strips) * sizeof(float));
  // staged lambda, mu, rho (+ c11, c13 in a VTI medium)
  p.par_bytes = align_up((size_t)(g.eps ? 5 : 3) * p.plane * sizeof(float));
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
  p.off_state = fwd ? take(2 * p.state_bytes) : 0;  // double-buffered by step parity
  p.off_e = fwd ? take((size_t)std::max(1, p.nch) * sizeof(float)) : 0;
  p.off_adj = adj ? take(p.adj_bytes) : 0;
  p.off_ebar = adj ? take((size_t)std::max(1, p.nch) * p.nt * sizeof(float)) : 0;
  p.off_partial = grad ? take((size_t)std::max(1, p.nch) * sizeof(double)) : 0;
  p.R = receiver_of(g, s);
  p.field = !p.R.identity();
  p.off_dint = (grad || (fwd && p.field)) ? take((size_t)std::max(1, p.nch) * p.nt * sizeof(float)) : 0;
  p.off_rf = (grad && p.field) ? take(std::max<size_t>(1, data_floats(g, s)) * sizeof(float)) : 0;
  p.off_acc = grad ? take((size_t)(g.eps ? NACC_VTI : NACC) * p.cells * sizeof(float)) : 0;
  p.off_G = grad ? take((size_t)3 * p.cells * sizeof(double)) : 0;
  p.off_seg = grad ? take((size_t)p.L * NSEG_FIELDS * p.cells * sizeof(float)) : 0;
  p.off_ckpt = grad ? take((size_t)std::max(0, p.nseg - 2) * p.slot_bytes) : 0;
  p.off_maxbits = grad ? take(CKPT_NFIELDS * sizeof(unsigned int)) : 0;
  p.total = o;
  return p;
}

// CPML profile of one axis, computed in double and stored FP32.
void cpml_profile(float* a, float* b, int n, double h, const efwi_grid& g, bool half) {
  for (int k = 0; k < n; ++k) {
    a[k] = 0.f;
    b[k] = 1.f;
  }
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

// Per-shot tables: CPML profiles, row -> slot map and the [slot][x] channel map.
void build_tables(const efwi_grid& g, const efwi_shot& s, const Plan2D& p, unsigned char* out) {
  std::memset(out, 0, p.tab_bytes);
  float* prof = reinterpret_cast<float*>(out);
  const int nx = p.nx, nz = p.nz;
  cpml_profile(prof, prof + nx, nx, g.dx, g, false);
  cpml_profile(prof + 2 * nx, prof + 3 * nx, nx, g.dx, g, true);
  cpml_profile(prof + 4 * nx, prof + 4 * nx + nz, nz, g.dz, g, false);
  cpml_profile(prof + 4 * nx + 2 * nz, prof + 4 * nx + 3 * nz, nz, g.dz, g, true);
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
}

// What one shot reads and writes (device pointers; unused ones are NULL).
struct ShotIO {
  const float* m = nullptr;   // window of the full-model [3][nz][nx] array
  long mplane = 0;
  const float* src = nullptr;
  const float* dobs = nullptr;
  const float* r = nullptr;
  float* d = nullptr;          // forward data output
  float* gout = nullptr;
  double* phi = nullptr;
  float* src_bar = nullptr;
  bool accumulate = false;     // add the gradient into gout (shots sharing a component)
};

Shot2D make_desc(const efwi_grid& g, const efwi_shot& s, const Plan2D& p, unsigned char* region,
                 const float* tab, const ShotIO& io) {
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
  auto fields = [&](size_t off, gfloat** out) {
    gfloat* base = (gfloat*)(region + off);
    for (int k = 0; k < 5; ++k) out[k] = base + k * p.plane + interior;
    return base + (size_t)5 * p.plane;  // strips follow the five planes
  };
  auto strips_at = [&](gfloat* base, gfloat** px, gfloat** pz) {
    const size_t xs = (size_t)p.nz * 2 * p.P, zs = (size_t)2 * p.P * p.nx;
    for (int k = 0; k < 4; ++k) px[k] = base + k * xs;
    for (int k = 0; k < 4; ++k) pz[k] = base + 4 * xs + k * zs;
  };
  gfloat* f[5];
  gfloat* st = fields(p.off_state, f);
  d.sbuf = (long)(p.state_bytes / sizeof(float));
  d.vx = f[0], d.vz = f[1], d.sxx = f[2], d.szz = f[3], d.sxz = f[4];
  strips_at(st, d.psx, d.psz);
  st = fields(p.off_adj, f) + (size_t)5 * p.plane;  // buffer 1's planes, then the strips
  d.abuf = (long)5 * p.plane;
  d.uxb = f[0], d.uzb = f[1], d.txxb = f[2], d.tzzb = f[3], d.txzb = f[4];
  strips_at(st, d.pbx[0], d.pbz[0]);
  strips_at(st + strips, d.pbx[1], d.pbz[1]);
  fields(p.off_par, f);
  d.lam = f[0], d.mu = f[1], d.rho = f[2];
  d.c11 = g.eps ? f[3] : nullptr;
  d.c13 = g.eps ? f[4] : nullptr;
  d.meps = g.eps ? (const gfloat*)(g.eps + (long)p.w.z0 * g.nx + p.w.x0) : nullptr;
  d.prof = (const gfloat*)(tab);
  d.row_slot = (const gint*)(tab + 4 * p.nx + 4 * p.nz);
  d.rowch = d.row_slot + p.nz;
  d.e = (gfloat*)(region + p.off_e);
  d.ebar = (const gfloat*)(region + p.off_ebar);
  d.acc = (gfloat*)(region + p.off_acc);
  d.G = (gdouble*)(region + p.off_G);
  d.seg = (gfloat*)(region + p.off_seg);
  const long mld = g.nx;
  if (io.m) {
    const gfloat* mw = (const gfloat*)(io.m + (long)p.w.z0 * mld + p.w.x0);
    d.mvp = mw;
    d.mvs = mw + io.mplane;
    d.mrho = mw + 2 * io.mplane;
  }
  d.mld = mld;
  d.src = (const gfloat*)(io.src);
  d.src_bar = (gfloat*)(io.src_bar);
  // with a field sampling the kernels record the point strains internally and the field
  // data are formed from them afterwards
  d.d = (gfloat*)((io.d && !p.field) ? io.d : reinterpret_cast<float*>(region + p.off_dint));
  d.gout = (gfloat*)(io.gout);
  d.mplane = io.mplane;
  d.z0 = p.w.z0;
  d.x0 = p.w.x0;
  return d;
}

efwi_status check_ws(const void* ws, size_t have, size_t need) {
  if (need > 0 && !ws) return fail(EFWI_E_INVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % ALIGN != 0) return fail(EFWI_E_INVAL, "workspace not 256-byte aligned");
  if (have < need) return fail(EFWI_E_WORKSPACE, "workspace has %zu bytes, needs %zu", have, need);
  return EFWI_OK;
}

// ----------------------------------------------------------------------------------------
// A wave: shots [first, first + count) of a call, advanced together. The workspace holds a
// header (descriptors, tile list, per-shot tables: uploaded once) followed by each shot's
// private region.
// ----------------------------------------------------------------------------------------
// Schedule entries needed for `tiles` tiles: a run's weight is below wtot / NUM_XCD plus one
// tile's weight, so it holds at most tiles * SCHED_RATIO / NUM_XCD + SCHED_RATIO + 1 tiles.
size_t sched_capacity(size_t tiles) {
  return (size_t)NUM_XCD * (tiles * SCHED_RATIO / NUM_XCD + SCHED_RATIO + 2);
}

size_t header_bytes(const std::vector<Plan2D>& plans, int first, int count) {
  size_t tiles = 0, ftiles = 0, atiles = 0, tabs = 0;
  for (int k = first; k < first + count; ++k) {
    tiles += plans[k].ntiles;
    ftiles += plans[k].nfwd_tiles;
    atiles += plans[k].nadj_tiles;
    tabs += plans[k].tab_bytes;
  }
  auto list = [&](size_t n) {  // tile_first, tile_shot and schedule of one tile list
    return align_up((size_t)count * sizeof(int)) + align_up(n * sizeof(int)) +
           align_up(sched_capacity(n) * sizeof(int));
  };
  auto step_list = [&](size_t n) { return align_up(sched_capacity(n) * sizeof(StepSlot)); };
  return align_up((size_t)count * sizeof(Shot2D)) + list(tiles) + step_list(ftiles) + step_list(atiles) + tabs;
}

size_t wave_bytes(const std::vector<Plan2D>& plans, int first, int count) {
  size_t t = header_bytes(plans, first, count);
  for (int k = first; k < first + count; ++k) t += plans[k].total;
  return t;
}

// Cut `weight` into NUM_XCD contiguous runs of equal total and write the schedule: slot
// m * NUM_XCD + k holds the m-th tile of XCD k's run (workgroups go to the XCDs round robin).
efwi_status build_sched(const std::vector<int>& weight, int* sched, int& nsched) {
  const int ntiles = (int)weight.size();
  long wtot = 0;
  for (int x : weight) wtot += x;
  std::vector<int> cut(NUM_XCD + 1, ntiles);
  cut[0] = 0;
  long acc = 0;
  for (int q = 0, k = 1; q < ntiles && k < NUM_XCD; ++q) {
    acc += weight[q];
    while (k < NUM_XCD && acc * NUM_XCD >= wtot * k) cut[k++] = q + 1;
  }
  int maxrun = 0;
  for (int k = 0; k < NUM_XCD; ++k) maxrun = std::max(maxrun, cut[k + 1] - cut[k]);
  if ((size_t)maxrun * NUM_XCD > sched_capacity(ntiles)) return fail(EFWI_E_INVAL, "tile schedule overflow");
  // inside a run the costlier tiles go first (the rest in list order), so that an XCD does
  // not end its share of the launch on a few slow tiles near a strip
  std::vector<int> order(ntiles);
  for (int q = 0; q < ntiles; ++q) order[q] = q;
  for (int k = 0; k < NUM_XCD; ++k)
    std::stable_sort(order.begin() + cut[k], order.begin() + cut[k + 1],
                     [&](int a, int b) { return weight[a] > weight[b]; });
  for (int m = 0; m < maxrun; ++m)
    for (int k = 0; k < NUM_XCD; ++k) sched[m * NUM_XCD + k] = (cut[k] + m < cut[k + 1]) ? order[cut[k] + m] : -1;
  nsched = maxrun * NUM_XCD;
  return EFWI_OK;
}

struct Wave {
  std::vector<Plan2D> plans;   // of the wave's shots
  std::vector<Shot2D> descs;   // host copies
  std::vector<size_t> regions; // byte offset of each shot's region
  Batch2D batch{};
  int L = 1, nseg = 1, nt = 0;
};

efwi_status setup_wave(const efwi_grid& g, const efwi_shot* shots, const std::vector<Plan2D>& plans, int first,
                       int count, const std::vector<ShotIO>& io, efwi_ws_kind kind, unsigned char* ws, Wave& wv,
                       hipStream_t st) {
  wv.plans.assign(plans.begin() + first, plans.begin() + first + count);
  wv.nt = g.nt;
  wv.L = wv.plans[0].L;
  wv.nseg = wv.plans[0].nseg;
  int ntiles = 0, nftiles = 0, natiles = 0;
  for (const Plan2D& p : wv.plans) {
    ntiles += p.ntiles;
    nftiles += p.nfwd_tiles;
    natiles += p.nadj_tiles;
  }
  // header layout: descriptors, the 4-row tile list (tile_first [count], tile_shot
  // [tiles], XCD schedule), the forward-step and transposed-step schedules (StepSlot per
  // slot), then the per-shot tables
  const size_t off_desc = 0;
  size_t off = off_desc + align_up((size_t)count * sizeof(Shot2D));
  struct ListAt {
    size_t first, shot, sched;
  };
  auto list_at = [&](size_t n) {
    ListAt l;
    l.first = off;
    l.shot = l.first + align_up((size_t)count * sizeof(int));
    l.sched = l.shot + align_up(n * sizeof(int));
    off = l.sched + align_up(sched_capacity(n) * sizeof(int));
    return l;
  };
  const ListAt l4 = list_at(ntiles);
  const size_t off_fs = off;   // the fused steps' schedules
  off += align_up(sched_capacity(nftiles) * sizeof(StepSlot));
  const size_t off_as = off;
  off += align_up(sched_capacity(natiles) * sizeof(StepSlot));
  size_t off_tab = off;
  const size_t hdr = header_bytes(plans, first, count);
  std::vector<unsigned char> blob(hdr, 0);
  auto ints = [&](size_t o) { return reinterpret_cast<int*>(blob.data() + o); };
  size_t region = hdr;
  int t4 = 0;
  wv.descs.clear();
  wv.regions.clear();
  for (int k = 0; k < count; ++k) {
    const Plan2D& p = wv.plans[k];
    const efwi_shot& s = shots[first + k];
    ints(l4.first)[k] = t4;
    for (int q = 0; q < p.ntiles; ++q) ints(l4.shot)[t4++] = k;
    build_tables(g, s, p, blob.data() + off_tab);
    const float* tab_dev = reinterpret_cast<const float*>(ws + off_tab);
    wv.descs.push_back(make_desc(g, s, p, ws + region, tab_dev, io[first + k]));
    wv.regions.push_back(region);
    off_tab += p.tab_bytes;
    region += p.total;
  }
  std::memcpy(blob.data() + off_desc, wv.descs.data(), (size_t)count * sizeof(Shot2D));
  // XCD schedules: cut each tile list into NUM_XCD contiguous runs of equal weighted cost.
  // Tiles near a CPML strip cost more: the 4-row tiles (pointwise kernels) that contain
  // strip nodes, forward-step tiles within two nodes of a strip (velocity halo) and
  // transposed-step tiles within four (staged operands). The fused steps' schedules hold
  // each slot's tile itself (shot, origin, code path) rather than its index.
  std::vector<StepSlot> info;
  auto weights = [&](int rows, int pad, int edge_below, int w_pml, int w_int, size_t n) {
    std::vector<int> w(n);
    info.assign(n, StepSlot{-1, 0, 0, 0});
    size_t q = 0;
    int sh = 0;
    for (const Plan2D& p : wv.plans) {
      const int ntx = (p.nx + BX - 1) / BX, nty = (p.nz + rows - 1) / rows;
      for (int l = 0; l < ntx * nty; ++l, ++q) {
        const int i0 = (l / ntx) * rows, j0 = (l % ntx) * BX;
        const bool pml = p.P > 0 && ((j0 - pad < p.P) || (j0 + BX - 1 + pad >= p.nx - p.P) || (i0 - pad < p.P) ||
                                     (i0 + rows - 1 + pad >= p.nz - p.P));
        w[q] = pml ? w_pml : w_int;
        info[q] = StepSlot{sh, i0, j0, pml ? PATH_PML : p.P < edge_below ? PATH_EDGE : PATH_INTERIOR};
      }
      ++sh;
    }
    return w;
  };
  auto step_slots = [&](const int* order, int nslots, size_t off_slots) {
    StepSlot* out = reinterpret_cast<StepSlot*>(blob.data() + off_slots);
    for (int q = 0; q < nslots; ++q) out[q] = order[q] < 0 ? StepSlot{-1, 0, 0, 0} : info[order[q]];
  };
  const int frows = wv.plans[0].fwd_rows, arows = wv.plans[0].adj_rows;
  int nsched[3];
  efwi_status rc = build_sched(weights(BZ, 0, 0, FWD_W_PML, FWD_W_INT, ntiles), ints(l4.sched), nsched[0]);
  if (rc != EFWI_OK) return rc;
  {
    // the halo of the forward step's staged stresses reaches 2 nodes beyond the velocity
    // halo, so without strips of at least 2 nodes a tile may read outside the grid; the
    // transposed step's reaches 4 nodes, inside the grid whenever there are strips
    std::vector<int> order(sched_capacity(nftiles));
    rc = build_sched(weights(frows, 2, 2, FWD_W_PML, FWD_W_INT, nftiles), order.data(), nsched[1]);
    if (rc != EFWI_OK) return rc;
    step_slots(order.data(), nsched[1], off_fs);
    order.assign(sched_capacity(natiles), -1);
    rc = build_sched(weights(arows, 4, 1, ADJ_W_PML, ADJ_W_INT, natiles), order.data(), nsched[2]);
    if (rc != EFWI_OK) return rc;
    step_slots(order.data(), nsched[2], off_as);
  }
  auto dev = [&](size_t o) { return reinterpret_cast<const int*>(ws + o); };
  wv.batch.tile_first = dev(l4.first);
  wv.batch.tile_shot = dev(l4.shot);
  wv.batch.fwd = Sched{dev(l4.sched), nsched[0]};
  wv.batch.step = StepSched{reinterpret_cast<const StepSlot*>(ws + off_fs), nsched[1]};
  wv.batch.adj_step = StepSched{reinterpret_cast<const StepSlot*>(ws + off_as), nsched[2]};
  wv.batch.fwd_rows = frows;
  wv.batch.adj_rows = arows;
  wv.batch.vti = g.eps != nullptr;
  wv.batch.shots = reinterpret_cast<const Shot2D*>(ws + off_desc);
  wv.batch.ns = count;
  wv.batch.ntiles = ntiles;
  // zero what must start at zero
  const bool fwd = kind != EFWI_WS_ADJOINT;
  const bool adj = kind != EFWI_WS_FORWARD;
  const bool grad = kind == EFWI_WS_GRADIENT || kind == EFWI_WS_BATCH;
  for (int k = 0; k < count; ++k) {
    const Plan2D& p = wv.plans[k];
    unsigned char* r = ws + wv.regions[k];
    HIP_TRY(hipMemsetAsync(r + p.off_par, 0, p.par_bytes, st));
    if (fwd) {
      HIP_TRY(hipMemsetAsync(r + p.off_state, 0, 2 * p.state_bytes, st));
      HIP_TRY(hipMemsetAsync(r + p.off_e, 0, (size_t)std::max(1, p.nch) * sizeof(float), st));
    }
    if (adj) HIP_TRY(hipMemsetAsync(r + p.off_adj, 0, p.adj_bytes, st));
    if (grad) HIP_TRY(hipMemsetAsync(r + p.off_G, 0, (size_t)3 * p.cells * sizeof(double), st));
  }
  HIP_TRY(upload_header(ws, blob, st));
  HIP_TRY(launch_stage2d(wv.batch, st));
  return EFWI_OK;
}

// A wave being advanced: its plan and descriptors, the workspace it was set up in and the
// stream its work goes to. The sweeps below advance one or more waves of the same schedule
// (nt, checkpoint interval) together, enqueuing each time step for every wave in turn, so
// that waves on different streams run their launches side by side.
struct Lane {
  Wave wv;
  unsigned char* ws = nullptr;
  hipStream_t st = nullptr;
};

// Forward sweep. With `checkpoints`, the state block of every shot is copied at the start of
// segments 1 .. nseg-2 (segment 0 starts from zero) and the last segment's imaging
// quantities are kept from this sweep, so the reverse sweep need not recompute it.
efwi_status run_forward(std::vector<Lane>& lanes, bool checkpoints) {
  const Wave& w0 = lanes[0].wv;
  const int last0 = (w0.nseg - 1) * w0.L;
  for (int n = 0; n < w0.nt; ++n) {
    for (Lane& l : lanes) {
      Wave& wv = l.wv;
      hipStream_t st = l.st;
      if (checkpoints && n % wv.L == 0 && n > 0 && n < last0) {
        const int k = n / wv.L;
        for (size_t q = 0; q < wv.plans.size(); ++q) {
          const Plan2D& p = wv.plans[q];
          unsigned char* r = l.ws + wv.regions[q];
          unsigned char* slot = r + p.off_ckpt + (size_t)(k - 1) * p.slot_bytes;
          unsigned char* state = r + p.off_state + (size_t)(n & 1) * p.state_bytes;  // state of step n
          if (p.ckpt_mode == EFWI_CKPT_FP32)
            HIP_TRY(hipMemcpyAsync(slot, state, p.state_bytes, hipMemcpyDeviceToDevice, st));
          else
            HIP_TRY(launch_ckpt_encode(reinterpret_cast<const float*>(state), p.fields,
                                       reinterpret_cast<unsigned int*>(r + p.off_maxbits), slot, p.ckpt_mode, st));
        }
      }
      const int kstore = (checkpoints && n >= last0) ? n - last0 : -1;
      HIP_TRY(TIMED(KK_FWD_STEP, st, launch_fwd_step(wv.batch, n, kstore, true, st)));
    }
  }
  return EFWI_OK;
}

efwi_status run_forward(Wave& wv, unsigned char* ws, bool checkpoints, hipStream_t st) {
  std::vector<Lane> one(1);
  one[0].wv = wv;
  one[0].ws = ws;
  one[0].st = st;
  return run_forward(one, checkpoints);
}

// Reverse sweep: segments last to first; each segment (but the last) is recomputed from its
// checkpoint while storing the imaging quantities, then stepped back.
efwi_status run_reverse(std::vector<Lane>& lanes) {
  const Wave& w0 = lanes[0].wv;
  for (int k = w0.nseg - 1; k >= 0; --k) {
    const int n0 = k * w0.L, n1 = std::min(w0.nt, n0 + w0.L);
    if (k < w0.nseg - 1) {
      for (Lane& l : lanes) {
        for (size_t q = 0; q < l.wv.plans.size(); ++q) {
          const Plan2D& p = l.wv.plans[q];
          unsigned char* r = l.ws + l.wv.regions[q];
          const unsigned char* slot = r + p.off_ckpt + (size_t)(k - 1) * p.slot_bytes;
          unsigned char* state = r + p.off_state + (size_t)(n0 & 1) * p.state_bytes;  // state of step n0
          if (k == 0) HIP_TRY(hipMemsetAsync(state, 0, p.state_bytes, l.st));
          else if (p.ckpt_mode == EFWI_CKPT_FP32)
            HIP_TRY(hipMemcpyAsync(state, slot, p.state_bytes, hipMemcpyDeviceToDevice, l.st));
          else
            HIP_TRY(launch_ckpt_decode(reinterpret_cast<float*>(state), p.fields, slot, p.ckpt_mode, l.st));
        }
      }
      for (int n = n0; n < n1; ++n)
        for (Lane& l : lanes) HIP_TRY(TIMED(KK_FWD_STEP, l.st, launch_fwd_step(l.wv.batch, n, n - n0, false, l.st)));
    }
    // Imaging sums run in FP32 over blocks of FLUSH_STEPS steps aligned on absolute step
    // numbers and are then added into the FP64 gradient, so the result does not depend on
    // the checkpoint interval.
    for (int n = n1 - 1; n >= n0; --n) {
      const bool first = (n == w0.nt - 1) || ((n + 1) % FLUSH_STEPS == 0);
      for (Lane& l : lanes) {
        HIP_TRY(TIMED(KK_ADJ_STEP, l.st, launch_adj_step(l.wv.batch, n, n - n0, true, first, false, l.st)));
        if (n % FLUSH_STEPS == 0) HIP_TRY(TIMED(KK_CHAIN, l.st, launch_chain_flush(l.wv.batch, l.st)));
      }
    }
  }
  return EFWI_OK;
}

efwi_status run_reverse(Wave& wv, unsigned char* ws, hipStream_t st) {
  std::vector<Lane> one(1);
  one[0].wv = wv;
  one[0].ws = ws;
  one[0].st = st;
  return run_reverse(one);
}

// Bytes that one time step of a shot reads and writes again at the next step: both
// buffers of the forward state, or both of the adjoint state and the imaging sums, plus
// the parameters.
size_t step_bytes(const Plan2D& p) {
  return std::max(2 * p.state_bytes, p.adj_bytes + (size_t)3 * p.cells * sizeof(float)) + p.par_bytes;
}

// Split shots [0, ns) into waves that fit ws_bytes. A wave also keeps its shots' step
// bytes within the wave bound (WAVE_CACHE_BYTES unless set; at least one shot per wave): while they fit in the
// 256 MB Infinity Cache, each step finds the previous step's state there, and one launch
// over more shots than fit is slower per cell than a launch per wave (measured on the
// 1000 x 3000 shots: a 2-shot launch took 1.5x (forward) and 1.1x (transposed) the time
// per cell of a 1-shot launch). Small windows are still advanced many at a time.
efwi_status plan_waves(const std::vector<Plan2D>& plans, size_t ws_bytes, std::vector<std::pair<int, int>>& waves,
                       size_t cache_bytes = 0) {
  const int ns = (int)plans.size();
  if (cache_bytes == 0) cache_bytes = g_wave_cache_bytes.load();
  int first = 0;
  while (first < ns) {
    int count = 0;
    size_t cached = 0;
    while (first + count < ns && wave_bytes(plans, first, count + 1) <= ws_bytes &&
           (count == 0 || cached + step_bytes(plans[first + count]) <= cache_bytes)) {
      cached += step_bytes(plans[first + count]);
      ++count;
    }
    if (count == 0)
      return fail(EFWI_E_WORKSPACE, "workspace has %zu bytes; shot %d alone needs %zu", ws_bytes, first,
                  wave_bytes(plans, first, 1));
    waves.push_back({first, count});
    first += count;
  }
  return EFWI_OK;
}

// First-fit-decreasing packing of a batch into waves, for calls whose shots do not depend on
// one another's order: the shots taken largest first (by workspace bytes), each into the
// first wave that still fits it in the workspace and, beyond its first shot, in the per-step
// state bound. Fewer, fuller waves than taking the shots in order (the batched workload's 64
// windows: 29 waves of 3.14 M cells against 39 of 2.34 M), so longer launches. `order` lists
// the shots wave by wave (ascending inside a wave); wave w is order[first, first + count).
efwi_status pack_waves(const std::vector<Plan2D>& plans, size_t ws_bytes, size_t cache_bytes, std::vector<int>& order,
                       std::vector<std::pair<int, int>>& waves) {
  const int ns = (int)plans.size();
  std::vector<int> idx(ns);
  for (int k = 0; k < ns; ++k) idx[k] = k;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return plans[a].total > plans[b].total; });
  struct Bin {
    std::vector<int> shots;
    size_t tiles = 0, ftiles = 0, atiles = 0, tabs = 0, total = 0, step = 0;
  };
  auto bytes_with = [&](const Bin& b, const Plan2D& p) {   // wave_bytes of the bin plus shot p
    const size_t count = b.shots.size() + 1, tiles = b.tiles + p.ntiles, ftiles = b.ftiles + p.nfwd_tiles,
                 atiles = b.atiles + p.nadj_tiles;
    auto list = [&](size_t n) {
      return align_up(count * sizeof(int)) + align_up(n * sizeof(int)) + align_up(sched_capacity(n) * sizeof(int));
    };
    auto step_list = [&](size_t n) { return align_up(sched_capacity(n) * sizeof(StepSlot)); };
    return align_up(count * sizeof(Shot2D)) + list(tiles) + step_list(ftiles) + step_list(atiles) + b.tabs + p.tab_bytes +
           b.total + p.total;
  };
  std::vector<Bin> bins;
  for (int k : idx) {
    const Plan2D& p = plans[k];
    Bin* into = nullptr;
    for (Bin& b : bins)
      if (b.step + step_bytes(p) <= cache_bytes && bytes_with(b, p) <= ws_bytes) {
        into = &b;
        break;
      }
    if (!into) {
      if (bytes_with(Bin{}, p) > ws_bytes)
        return fail(EFWI_E_WORKSPACE, "workspace has %zu bytes; shot %d alone needs %zu", ws_bytes, k,
                    bytes_with(Bin{}, p));
      bins.emplace_back();
      into = &bins.back();
    }
    into->shots.push_back(k);
    into->tiles += p.ntiles;
    into->ftiles += p.nfwd_tiles;
    into->atiles += p.nadj_tiles;
    into->tabs += p.tab_bytes;
    into->total += p.total;
    into->step += step_bytes(p);
  }
  order.clear();
  waves.clear();
  for (Bin& b : bins) {
    std::sort(b.shots.begin(), b.shots.end());
    waves.push_back({(int)order.size(), (int)b.shots.size()});
    order.insert(order.end(), b.shots.begin(), b.shots.end());
  }
  return EFWI_OK;
}

// The lane plan of a 2D batch: the waves (packed when `reorder`, else in shot order) and the
// lanes that advance them. With two lanes (efwi_set_wave_lanes) each lane takes half of the
// workspace and half of the per-step state bound (so that the two waves running side by side
// keep their state within the Infinity Cache together), and consecutive waves alternate
// between the lanes. Two lanes are used when `lanes2` holds, one lane would take more than
// one wave, every shot fits a lane's half, the two lanes' plan has at most about twice the
// waves of one lane's and none of its waves has more per-step state than the whole bound;
// otherwise one lane takes everything.
efwi_status plan_lanes(const std::vector<Plan2D>& plans, size_t ws_bytes, bool lanes2, bool reorder,
                       std::vector<int>& order, std::vector<std::pair<int, int>>& waves, int& nlanes,
                       size_t& lane_bytes) {
  const size_t cache = g_wave_cache_bytes.load();
  auto plan = [&](size_t ws, size_t cache_bytes) {
    if (reorder) return pack_waves(plans, ws, cache_bytes, order, waves);
    order.resize(plans.size());
    for (size_t k = 0; k < plans.size(); ++k) order[k] = (int)k;
    waves.clear();
    return plan_waves(plans, ws, waves, cache_bytes);
  };
  nlanes = 1;
  lane_bytes = ws_bytes;
  efwi_status rc = plan(ws_bytes, cache);
  if (rc != EFWI_OK || !lanes2 || g_wave_lanes.load() < 2 || waves.size() < 2) return rc;
  const size_t one_lane = waves.size();
  const size_t half = ws_bytes / 2 / ALIGN * ALIGN;
  for (size_t k = 0; k < plans.size(); ++k)
    if (wave_bytes(plans, (int)k, 1) > half) return EFWI_OK;
  const std::vector<int> order1 = order;
  const std::vector<std::pair<int, int>> waves1 = waves;
  // two lanes when each lane's waves are not finer than half of one lane's and no wave's
  // per-step state exceeds the whole bound (two such waves side by side overflow the cache:
  // two 1200 x 4000 shots, 300 MB of state each, ran 12% slower than one after the other)
  if (plan(half, std::max<size_t>(cache / 2, 1)) == EFWI_OK && waves.size() >= 2 && waves.size() <= 2 * one_lane + 1) {
    bool small = true;
    for (const auto& w : waves) {
      size_t st = 0;
      for (int q = w.first; q < w.first + w.second; ++q) st += step_bytes(plans[order[q]]);
      small = small && st <= cache;
    }
    if (small) {
      nlanes = 2;
      lane_bytes = half;
      return EFWI_OK;
    }
  }
  order = order1;
  waves = waves1;
  return EFWI_OK;
}

// The second lane's stream on the current device, created on first use (default priority,
// not synchronizing with the null stream: the calls order it with events).
hipError_t lane_stream(hipStream_t* out) {
  static std::mutex mu;
  static std::vector<hipStream_t>* streams = new std::vector<hipStream_t>();  // lives for the process
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)streams->size() <= dev) streams->resize(dev + 1, nullptr);
  if (!(*streams)[dev]) {
    e = hipStreamCreateWithFlags(&(*streams)[dev], hipStreamNonBlocking);
    if (e != hipSuccess) return e;
  }
  *out = (*streams)[dev];
  return hipSuccess;
}

// Event-ordered hand-over between two streams: `to` waits for what `from` has enqueued so far.
hipError_t join_streams(hipStream_t from, hipStream_t to) {
  hipEvent_t ev;
  hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e != hipSuccess) return e;
  e = hipEventRecord(ev, from);
  if (e == hipSuccess) e = hipStreamWaitEvent(to, ev, 0);
  const hipError_t d = hipEventDestroy(ev);
  return e != hipSuccess ? e : d;
}

efwi_status gradient_waves3(const efwi_grid& g, const efwi_shot* shots, int ns, const std::vector<ShotIO>& io,
                            unsigned char* ws, size_t ws_bytes, hipStream_t st);

// Misfit stage of a shot with a field sampling: the field data out of the recorded point
// strains when asked for, then e_bar from the given field-space vector (J^T v) or from the
// field residual K d - d_obs (with the misfit).
hipError_t field_misfit(const Receiver& R, unsigned char* region, size_t off_dint, size_t off_rf, size_t off_partial,
                        const ShotIO& io, float* ebar, hipStream_t st) {
  const float* e = reinterpret_cast<const float*>(region + off_dint);
  if (io.d) {
    const hipError_t rc = launch_field_data(R, e, io.d, st);
    if (rc != hipSuccess) return rc;
  }
  if (io.r) return launch_field_cumsum(R, io.r, ebar, st);
  return launch_field_misfit(R, e, io.dobs, reinterpret_cast<float*>(region + off_rf),
                             reinterpret_cast<double*>(region + off_partial), io.phi, ebar, st);
}

// The data term over a batch of 2D shots: waves set up in turn in the workspace (or in its
// two halves, one per lane), each swept forward, its misfit taken, swept back and its
// gradient written. Shots whose gradients add into a shared component (io.accumulate) use
// one lane, so that the additions keep the shot order.
efwi_status gradient_lanes(const efwi_grid& g, const efwi_shot* shots, const std::vector<ShotIO>& io,
                           const std::vector<Plan2D>& plans, const std::vector<std::pair<int, int>>& waves,
                           int nlanes, size_t lane_bytes, unsigned char* ws, hipStream_t st, hipStream_t st1) {
  efwi_status rc = EFWI_OK;
  for (size_t w = 0; w < waves.size(); w += nlanes) {
    std::vector<Lane> lanes(std::min<size_t>(nlanes, waves.size() - w));
    for (size_t l = 0; l < lanes.size(); ++l) {
      lanes[l].ws = ws + l * lane_bytes;
      lanes[l].st = l == 0 ? st : st1;
      rc = setup_wave(g, shots, plans, waves[w + l].first, waves[w + l].second, io, EFWI_WS_GRADIENT, lanes[l].ws,
                      lanes[l].wv, lanes[l].st);
      if (rc != EFWI_OK) return rc;
    }
    rc = run_forward(lanes, true);
    if (rc != EFWI_OK) return rc;
    for (size_t l = 0; l < lanes.size(); ++l) {
      const Wave& wv = lanes[l].wv;
      const int first = waves[w + l].first;
      hipStream_t ls = lanes[l].st;
      for (int k = 0; k < waves[w + l].second; ++k) {
        const Shot2D& d = wv.descs[k];
        unsigned char* r = lanes[l].ws + wv.regions[k];
        const Plan2D& p = wv.plans[k];
        float* ebar = reinterpret_cast<float*>(r + p.off_ebar);
        if (p.field) {
          HIP_TRY(TIMED(KK_MISFIT, ls, field_misfit(p.R, r, p.off_dint, p.off_rf, p.off_partial, io[first + k], ebar, ls)));
        } else if (io[first + k].r) {  // J^T v: the data-space vector drives the adjoint directly
          HIP_TRY(TIMED(KK_MISFIT, ls, launch_residual_cumsum(d, io[first + k].r, ebar, ls)));
        } else {
          HIP_TRY(TIMED(KK_MISFIT, ls,
                        launch_misfit(d, (const float*)(d.d), io[first + k].dobs,
                                      reinterpret_cast<double*>(r + p.off_partial), io[first + k].phi, ebar, ls)));
        }
      }
    }
    rc = run_reverse(lanes);
    if (rc != EFWI_OK) return rc;
    for (size_t l = 0; l < lanes.size(); ++l) {
      const Wave& wv = lanes[l].wv;
      const int first = waves[w + l].first, count = waves[w + l].second;
      hipStream_t ls = lanes[l].st;
      if (io[first].accumulate) {  // one launch per shot, in shot order: shots of a group add deterministically
        for (int k = 0; k < count; ++k) {
          const Plan2D& p = wv.plans[k];
          HIP_TRY(launch_add_gradient(reinterpret_cast<const double*>(lanes[l].ws + wv.regions[k] + p.off_G), p.cells,
                                      p.cp, p.nz, 1, p.nx, io[first + k].gout, io[first + k].mplane, g.nx, g.nx,
                                      p.w.z0, 0, p.w.x0, ls));
        }
        continue;
      }
      for (int k = 0; k < count; ++k) {
        const Plan2D& p = wv.plans[k];
        const bool full = p.w.z0 == 0 && p.w.x0 == 0 && p.nz == g.nz && p.nx == g.nx;
        if (!full) HIP_TRY(hipMemsetAsync(io[first + k].gout, 0, (size_t)3 * io[first + k].mplane * sizeof(float), ls));
      }
      HIP_TRY(launch_write_gradient(wv.batch, ls));
    }
  }
  return EFWI_OK;
}

efwi_status gradient_waves(const efwi_grid& g, const efwi_shot* shots, int ns, const std::vector<ShotIO>& io,
                           unsigned char* ws, size_t ws_bytes, hipStream_t st) {
  if (g.ndim == 3) return gradient_waves3(g, shots, ns, io, ws, ws_bytes, st);
  std::vector<Plan2D> plans;
  for (int k = 0; k < ns; ++k) plans.push_back(plan2d(g, shots[k], EFWI_WS_GRADIENT));
  efwi_status rc = check_ws(ws, ws_bytes, wave_bytes(plans, 0, 1));
  if (rc != EFWI_OK) return rc;
  std::vector<std::pair<int, int>> waves;
  std::vector<int> order;
  int nlanes = 1;
  size_t lane_bytes = ws_bytes;
  const bool independent = !io[0].accumulate;   // grouped shots add into shared components in shot order
  rc = plan_lanes(plans, ws_bytes, independent && !t_no_alloc, independent, order, waves, nlanes, lane_bytes);
  if (rc != EFWI_OK) return rc;
  // the shots, their plans and outputs in the order the waves take them
  std::vector<efwi_shot> sp(ns);
  std::vector<ShotIO> iop(ns);
  std::vector<Plan2D> pp(ns);
  for (int q = 0; q < ns; ++q) {
    sp[q] = shots[order[q]];
    iop[q] = io[order[q]];
    pp[q] = plans[order[q]];
  }
  if (nlanes == 1) return gradient_lanes(g, sp.data(), iop, pp, waves, 1, lane_bytes, ws, st, nullptr);
  hipStream_t st1 = nullptr;
  HIP_TRY(lane_stream(&st1));
  HIP_TRY(join_streams(st, st1));   // the second lane starts after the caller's earlier work
  rc = gradient_lanes(g, sp.data(), iop, pp, waves, nlanes, lane_bytes, ws, st, st1);
  // the caller's stream then waits for the second lane, also after an error, so that no
  // work on the workspace is left behind the caller's stream
  const hipError_t e = join_streams(st1, st);
  if (rc != EFWI_OK) return rc;
  if (e != hipSuccess) return fail(EFWI_E_HIP, "joining the lanes failed: %s", hipGetErrorString(e));
  return EFWI_OK;
}

efwi_status check_same_schedule(const efwi_grid& g, int ns, const efwi_shot* shots) {
  for (int k = 1; k < ns; ++k) {
    if (interval_of(g, shots[k]) != interval_of(g, shots[0]) || shots[k].ckpt_mode != shots[0].ckpt_mode)
      return fail(EFWI_E_INVAL, "shots of one batch must share ckpt_interval and ckpt_mode");
  }
  return EFWI_OK;
}

// ========================================================================================
// 3D: the same schedule on Shot3D descriptors.
// ========================================================================================
struct Plan3D {
  Window w;
  int nz, ny, nx, ld, cp, P, nslots, nt, nch, L, nseg, ntiles;
  long pz, plane, cells;
  size_t strips, state_elems, state_bytes, slot_bytes, tab_bytes, adj_bytes, par_bytes;
  int ckpt_mode;
  CkptFields fields;
  size_t off_par, off_state, off_e, off_adj, off_ebar, off_partial, off_dint, off_acc, off_G, off_seg, off_ckpt,
      off_maxbits, off_rf, total;
  Receiver R;
  bool field;
};

int count_rows3(const efwi_shot& s, const Window& w) {
  std::vector<long> rows;
  for (int c = 0; c < s.nch; ++c) rows.push_back((long)(s.ch_iz[c] - w.z0) * w.wy + (s.ch_iy[c] - w.y0));
  std::sort(rows.begin(), rows.end());
  rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
  return (int)rows.size();
}

Plan3D plan3d(const efwi_grid& g, const efwi_shot& s, efwi_ws_kind kind) {
  Plan3D p{};
  p.w = window_of(g, s);
  p.nz = p.w.wz;
  p.ny = p.w.wy;
  p.nx = p.w.wx;
  p.ld = (XOFF + p.nx + HALO + ROW_ALIGN - 1) / ROW_ALIGN * ROW_ALIGN;
  p.cp = (p.nx + ROW_ALIGN - 1) / ROW_ALIGN * ROW_ALIGN;
  p.pz = (long)(p.ny + 2 * HALO) * p.ld;
  p.plane = (long)(p.nz + 2 * HALO) * p.pz;
  p.cells = (long)p.nz * p.ny * p.cp;
  p.P = strip_width(g);
  p.nt = g.nt;
  p.nch = s.nch;
  p.nslots = count_rows3(s, p.w);
  p.ntiles = tiles3(p.nz, p.ny, p.nx);
  p.L = interval_of(g, s);
  p.nseg = (g.nt + p.L - 1) / p.L;
  const long xs = (long)p.nz * p.ny * 2 * p.P, ys = (long)p.nz * 2 * p.P * p.nx, zs = (long)2 * p.P * p.ny * p.nx;
  p.strips = (size_t)6 * (xs + ys + zs);
  p.state_elems = (size_t)9 * p.plane + p.strips;
  p.state_bytes = align_up(p.state_elems * sizeof(float));
  p.adj_bytes = align_up(((size_t)9 * p.plane + 2 * p.strips) * sizeof(float));
  p.par_bytes = align_up((size_t)7 * p.plane * sizeof(float));
  p.tab_bytes = align_up((size_t)(4 * p.nx + 4 * p.ny + 4 * p.nz) * sizeof(float) +
                         (size_t)p.nz * p.ny * sizeof(int) + (size_t)p.nslots * p.nx * sizeof(int));
  p.ckpt_mode = s.ckpt_mode;
  p.slot_bytes = s.ckpt_mode == EFWI_CKPT_FP32 ? p.state_bytes
                                               : align_up(CKPT_HEADER + p.state_elems * sizeof(unsigned short));
  p.fields.n = 27;
  for (int k = 0; k < 9; ++k) {
    p.fields.off[k] = k * p.plane;
    p.fields.len[k] = p.plane;
  }
  long off = 9 * p.plane;
  for (int k = 0; k < 18; ++k) {
    const long len = k < 6 ? xs : (k < 12 ? ys : zs);
    p.fields.off[9 + k] = off;
    p.fields.len[9 + k] = len;
    off += len;
  }
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
  p.off_state = fwd ? take(p.state_bytes) : 0;
  p.off_e = fwd ? take((size_t)std::max(1, p.nch) * sizeof(float)) : 0;
  p.off_adj = adj ? take(p.adj_bytes) : 0;
  p.off_ebar = adj ? take((size_t)std::max(1, p.nch) * p.nt * sizeof(float)) : 0;
  p.off_partial = grad ? take((size_t)std::max(1, p.nch) * sizeof(double)) : 0;
  p.R = receiver_of(g, s);
  p.field = !p.R.identity();
  p.off_dint = (grad || (fwd && p.field)) ? take((size_t)std::max(1, p.nch) * p.nt * sizeof(float)) : 0;
  p.off_rf = (grad && p.field) ? take(std::max<size_t>(1, data_floats(g, s)) * sizeof(float)) : 0;
  p.off_acc = grad ? take((size_t)NACC3 * p.cells * sizeof(float)) : 0;
  p.off_G = grad ? take((size_t)3 * p.cells * sizeof(double)) : 0;
  p.off_seg = grad ? take((size_t)p.L * NSEG3 * p.cells * sizeof(float)) : 0;
  p.off_ckpt = grad ? take((size_t)std::max(0, p.nseg - 2) * p.slot_bytes) : 0;
  p.off_maxbits = grad ? take(CKPT_NFIELDS * sizeof(unsigned int)) : 0;
  p.total = o;
  return p;
}

void build_tables3(const efwi_grid& g, const efwi_shot& s, const Plan3D& p, unsigned char* out) {
  std::memset(out, 0, p.tab_bytes);
  float* prof = reinterpret_cast<float*>(out);
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  cpml_profile(prof, prof + nx, nx, g.dx, g, false);
  cpml_profile(prof + 2 * nx, prof + 3 * nx, nx, g.dx, g, true);
  float* py = prof + 4 * nx;
  cpml_profile(py, py + ny, ny, g.dy, g, false);
  cpml_profile(py + 2 * ny, py + 3 * ny, ny, g.dy, g, true);
  float* pz = py + 4 * ny;
  cpml_profile(pz, pz + nz, nz, g.dz, g, false);
  cpml_profile(pz + 2 * nz, pz + 3 * nz, nz, g.dz, g, true);
  int* row_slot = reinterpret_cast<int*>(pz + 4 * nz);
  int* rowch = row_slot + (size_t)nz * ny;
  std::fill(row_slot, row_slot + (size_t)nz * ny, -1);
  std::fill(rowch, rowch + (size_t)p.nslots * nx, -1);
  int nslots = 0;
  for (int c = 0; c < s.nch; ++c) {
    const long row = (long)(s.ch_iz[c] - p.w.z0) * ny + (s.ch_iy[c] - p.w.y0);
    if (row_slot[row] < 0) row_slot[row] = nslots++;
    rowch[(size_t)row_slot[row] * nx + (s.ch_ix[c] - p.w.x0)] = c;
  }
}

Shot3D make_desc3(const efwi_grid& g, const efwi_shot& s, const Plan3D& p, unsigned char* region, const float* tab,
                  const ShotIO& io) {
  Shot3D d{};
  d.nz = p.nz, d.ny = p.ny, d.nx = p.nx, d.ld = p.ld, d.P = p.P, d.pz = p.pz;
  d.nt = p.nt, d.nch = p.nch;
  d.si = s.src_iz - p.w.z0, d.sk = s.src_iy - p.w.y0, d.sj = s.src_ix - p.w.x0;
  d.dt = g.dt;
  d.rdx = (float)(1.0 / g.dx), d.rdy = (float)(1.0 / g.dy), d.rdz = (float)(1.0 / g.dz);
  d.w = (float)((double)g.dt / ((double)g.dx * g.dy * g.dz));
  d.cp = p.cp, d.cells = p.cells;
  const long interior = (long)HALO * p.pz + (long)HALO * p.ld + XOFF;
  auto fields = [&](size_t off, gfloat** out, int count) {
    gfloat* base = (gfloat*)(region + off);
    for (int k = 0; k < count; ++k) out[k] = base + k * p.plane + interior;
    return base + (size_t)count * p.plane;
  };
  const long xs = (long)p.nz * p.ny * 2 * p.P, ys = (long)p.nz * 2 * p.P * p.nx, zs = (long)2 * p.P * p.ny * p.nx;
  auto strips_at = [&](gfloat* base, gfloat** sx, gfloat** sy, gfloat** sz) {
    for (int k = 0; k < 6; ++k) sx[k] = base + k * xs;
    for (int k = 0; k < 6; ++k) sy[k] = base + 6 * xs + k * ys;
    for (int k = 0; k < 6; ++k) sz[k] = base + 6 * xs + 6 * ys + k * zs;
  };
  gfloat* f[9];
  gfloat* st = fields(p.off_state, f, 9);
  d.vx = f[0], d.vy = f[1], d.vz = f[2], d.sxx = f[3], d.syy = f[4], d.szz = f[5], d.sxy = f[6], d.sxz = f[7],
  d.syz = f[8];
  strips_at(st, d.psx, d.psy, d.psz);
  st = fields(p.off_adj, f, 9);
  d.uxb = f[0], d.uyb = f[1], d.uzb = f[2], d.txxb = f[3], d.tyyb = f[4], d.tzzb = f[5], d.txyb = f[6],
  d.txzb = f[7], d.tyzb = f[8];
  strips_at(st, d.pbx[0], d.pby[0], d.pbz[0]);
  strips_at(st + p.strips, d.pbx[1], d.pby[1], d.pbz[1]);
  gfloat* pf[7];
  fields(p.off_par, pf, 7);
  d.l2m = pf[0], d.lam = pf[1], d.muxy = pf[2], d.muxz = pf[3], d.muyz = pf[4], d.rho = pf[5], d.mu = pf[6];
  d.prof = (const gfloat*)(tab);
  d.row_slot = (const gint*)(tab + 4 * p.nx + 4 * p.ny + 4 * p.nz);
  d.rowch = d.row_slot + (long)p.nz * p.ny;
  d.e = (gfloat*)(region + p.off_e);
  d.ebar = (const gfloat*)(region + p.off_ebar);
  d.acc = (gfloat*)(region + p.off_acc);
  d.G = (gdouble*)(region + p.off_G);
  d.seg = (gfloat*)(region + p.off_seg);
  d.mld = g.nx;
  d.mplanestride = (long)g.ny * g.nx;
  if (io.m) {
    const float* mw = io.m + (long)p.w.z0 * d.mplanestride + (long)p.w.y0 * d.mld + p.w.x0;
    d.mvp = (const gfloat*)(mw);
    d.mvs = (const gfloat*)(mw + io.mplane);
    d.mrho = (const gfloat*)(mw + 2 * io.mplane);
  }
  d.src = (const gfloat*)(io.src);
  d.src_bar = (gfloat*)(io.src_bar);
  // with a field sampling the kernels record the point strains internally and the field
  // data are formed from them afterwards
  d.d = (gfloat*)((io.d && !p.field) ? io.d : reinterpret_cast<float*>(region + p.off_dint));
  d.gout = (gfloat*)(io.gout);
  d.mplane = io.mplane;
  d.z0 = p.w.z0, d.y0 = p.w.y0, d.x0 = p.w.x0;
  return d;
}

size_t header_bytes3(const std::vector<Plan3D>& plans, int first, int count) {
  size_t tiles = 0, tabs = 0;
  for (int k = first; k < first + count; ++k) {
    tiles += plans[k].ntiles;
    tabs += plans[k].tab_bytes;
  }
  return align_up((size_t)count * sizeof(Shot3D)) + align_up((size_t)count * sizeof(int)) +
         align_up(tiles * sizeof(int)) + 2 * align_up(sched_capacity(tiles) * sizeof(int)) + tabs;
}

size_t wave_bytes3(const std::vector<Plan3D>& plans, int first, int count) {
  size_t t = header_bytes3(plans, first, count);
  for (int k = first; k < first + count; ++k) t += plans[k].total;
  return t;
}

struct Wave3 {
  std::vector<Plan3D> plans;
  std::vector<Shot3D> descs;
  std::vector<size_t> regions;
  Batch3D batch{};
  int L = 1, nseg = 1, nt = 0;
};

efwi_status setup_wave3(const efwi_grid& g, const efwi_shot* shots, const std::vector<Plan3D>& plans, int first,
                        int count, const std::vector<ShotIO>& io, efwi_ws_kind kind, unsigned char* ws, Wave3& wv,
                        hipStream_t st) {
  wv.plans.assign(plans.begin() + first, plans.begin() + first + count);
  wv.nt = g.nt;
  wv.L = wv.plans[0].L;
  wv.nseg = wv.plans[0].nseg;
  int ntiles = 0;
  for (const Plan3D& p : wv.plans) ntiles += p.ntiles;
  const size_t off_first = align_up((size_t)count * sizeof(Shot3D));
  const size_t off_tshot = off_first + align_up((size_t)count * sizeof(int));
  const size_t off_sched = off_tshot + align_up((size_t)ntiles * sizeof(int));
  const size_t off_sched2 = off_sched + align_up(sched_capacity(ntiles) * sizeof(int));
  size_t off_tab = off_sched2 + align_up(sched_capacity(ntiles) * sizeof(int));
  const size_t hdr = header_bytes3(plans, first, count);
  std::vector<unsigned char> blob(hdr, 0);
  int* tfirst = reinterpret_cast<int*>(blob.data() + off_first);
  int* tshot = reinterpret_cast<int*>(blob.data() + off_tshot);
  size_t region = hdr;
  int t = 0;
  std::vector<int> weight;
  wv.descs.clear();
  wv.regions.clear();
  for (int k = 0; k < count; ++k) {
    const Plan3D& p = wv.plans[k];
    const efwi_shot& s = shots[first + k];
    tfirst[k] = t;
    for (int q = 0; q < p.ntiles; ++q) {
      tshot[t++] = k;
      int i, k0, j0;
      tile3_coords(q, p.nz, p.ny, p.nx, i, k0, j0);
      const int pad = 2;
      const bool pml = p.P > 0 && ((j0 - pad < p.P) || (j0 + TILE3_X - 1 + pad >= p.nx - p.P) || (k0 - pad < p.P) ||
                                   (k0 + TILE3_Y - 1 + pad >= p.ny - p.P) || (i - pad < p.P) ||
                                   (i + pad >= p.nz - p.P));
      weight.push_back(pml ? ADJ3_W_PML : ADJ3_W_INT);
    }
    build_tables3(g, s, p, blob.data() + off_tab);
    wv.descs.push_back(make_desc3(g, s, p, ws + region, reinterpret_cast<const float*>(ws + off_tab),
                                  io[first + k]));
    wv.regions.push_back(region);
    off_tab += p.tab_bytes;
    region += p.total;
  }
  std::memcpy(blob.data(), wv.descs.data(), (size_t)count * sizeof(Shot3D));
  int nsched[2];
  efwi_status rc = build_sched(std::vector<int>(ntiles, 1), reinterpret_cast<int*>(blob.data() + off_sched), nsched[0]);
  if (rc != EFWI_OK) return rc;
  rc = build_sched(weight, reinterpret_cast<int*>(blob.data() + off_sched2), nsched[1]);
  if (rc != EFWI_OK) return rc;
  wv.batch.shots = reinterpret_cast<const Shot3D*>(ws);
  wv.batch.tile_first = reinterpret_cast<const int*>(ws + off_first);
  wv.batch.tile_shot = reinterpret_cast<const int*>(ws + off_tshot);
  wv.batch.fwd = Sched{reinterpret_cast<const int*>(ws + off_sched), nsched[0]};
  wv.batch.adj = Sched{reinterpret_cast<const int*>(ws + off_sched2), nsched[1]};
  wv.batch.ns = count;
  wv.batch.ntiles = ntiles;
  const bool fwd = kind != EFWI_WS_ADJOINT;
  const bool adj = kind != EFWI_WS_FORWARD;
  const bool grad = kind == EFWI_WS_GRADIENT || kind == EFWI_WS_BATCH;
  for (int k = 0; k < count; ++k) {
    const Plan3D& p = wv.plans[k];
    unsigned char* r = ws + wv.regions[k];
    HIP_TRY(hipMemsetAsync(r + p.off_par, 0, p.par_bytes, st));
    if (fwd) {
      HIP_TRY(hipMemsetAsync(r + p.off_state, 0, p.state_bytes, st));
      HIP_TRY(hipMemsetAsync(r + p.off_e, 0, (size_t)std::max(1, p.nch) * sizeof(float), st));
    }
    if (adj) HIP_TRY(hipMemsetAsync(r + p.off_adj, 0, p.adj_bytes, st));
    if (grad) HIP_TRY(hipMemsetAsync(r + p.off_G, 0, (size_t)3 * p.cells * sizeof(double), st));
  }
  HIP_TRY(upload_header(ws, blob, st));
  HIP_TRY(launch3_stage(wv.batch, st));
  return EFWI_OK;
}

efwi_status save_or_restore3(Wave3& wv, unsigned char* ws, int k, bool save, hipStream_t st) {
  for (size_t q = 0; q < wv.plans.size(); ++q) {
    const Plan3D& p = wv.plans[q];
    unsigned char* r = ws + wv.regions[q];
    unsigned char* slot = r + p.off_ckpt + (size_t)(k - 1) * p.slot_bytes;
    float* state = reinterpret_cast<float*>(r + p.off_state);
    if (save) {
      if (p.ckpt_mode == EFWI_CKPT_FP32)
        HIP_TRY(hipMemcpyAsync(slot, state, p.state_bytes, hipMemcpyDeviceToDevice, st));
      else
        HIP_TRY(launch_ckpt_encode(state, p.fields, reinterpret_cast<unsigned int*>(r + p.off_maxbits), slot,
                                   p.ckpt_mode, st));
    } else if (k == 0) {
      HIP_TRY(hipMemsetAsync(state, 0, p.state_bytes, st));
    } else if (p.ckpt_mode == EFWI_CKPT_FP32) {
      HIP_TRY(hipMemcpyAsync(state, slot, p.state_bytes, hipMemcpyDeviceToDevice, st));
    } else {
      HIP_TRY(launch_ckpt_decode(state, p.fields, slot, p.ckpt_mode, st));
    }
  }
  return EFWI_OK;
}

efwi_status run_forward3(Wave3& wv, unsigned char* ws, bool checkpoints, hipStream_t st) {
  const int last0 = (wv.nseg - 1) * wv.L;
  for (int n = 0; n < wv.nt; ++n) {
    if (checkpoints && n % wv.L == 0 && n > 0 && n < last0) {
      efwi_status rc = save_or_restore3(wv, ws, n / wv.L, true, st);
      if (rc != EFWI_OK) return rc;
    }
    const int kstore = (checkpoints && n >= last0) ? n - last0 : -1;
    HIP_TRY(TIMED(KK_FWD_VEL, st, launch3_fwd_vel(wv.batch, kstore, st)));
    HIP_TRY(TIMED(KK_FWD_STR, st, launch3_fwd_str(wv.batch, n, kstore, true, st)));
  }
  return EFWI_OK;
}

efwi_status run_reverse3(Wave3& wv, unsigned char* ws, hipStream_t st) {
  for (int k = wv.nseg - 1; k >= 0; --k) {
    const int n0 = k * wv.L, n1 = std::min(wv.nt, n0 + wv.L);
    if (k < wv.nseg - 1) {
      efwi_status rc = save_or_restore3(wv, ws, k, false, st);
      if (rc != EFWI_OK) return rc;
      for (int n = n0; n < n1; ++n) {
        HIP_TRY(TIMED(KK_FWD_VEL, st, launch3_fwd_vel(wv.batch, n - n0, st)));
        HIP_TRY(TIMED(KK_FWD_STR, st, launch3_fwd_str(wv.batch, n, n - n0, false, st)));
      }
    }
    for (int n = n1 - 1; n >= n0; --n) {
      const bool first = (n == wv.nt - 1) || ((n + 1) % FLUSH_STEPS == 0);
      HIP_TRY(TIMED(KK_ADJ_VEL, st, launch3_adj_vel(wv.batch, n, n - n0, true, first, false, st)));
      HIP_TRY(TIMED(KK_ADJ_STR, st, launch3_adj_str(wv.batch, n, n - n0, true, first, st)));
      if (n % FLUSH_STEPS == 0) HIP_TRY(TIMED(KK_CHAIN, st, launch3_chain_flush(wv.batch, st)));
    }
  }
  return EFWI_OK;
}

// 3D waves: as many shots as fit ws_bytes (a 3D shot's state exceeds the caches anyway).
efwi_status plan_waves3(const std::vector<Plan3D>& plans, size_t ws_bytes, std::vector<std::pair<int, int>>& waves) {
  const int ns = (int)plans.size();
  int first = 0;
  while (first < ns) {
    int count = 0;
    while (first + count < ns && wave_bytes3(plans, first, count + 1) <= ws_bytes) ++count;
    if (count == 0) return fail(EFWI_E_WORKSPACE, "workspace too small for shot %d", first);
    waves.push_back({first, count});
    first += count;
  }
  return EFWI_OK;
}

efwi_status gradient_waves3(const efwi_grid& g, const efwi_shot* shots, int ns, const std::vector<ShotIO>& io,
                            unsigned char* ws, size_t ws_bytes, hipStream_t st) {
  std::vector<Plan3D> plans;
  for (int k = 0; k < ns; ++k) plans.push_back(plan3d(g, shots[k], EFWI_WS_GRADIENT));
  efwi_status rc = check_ws(ws, ws_bytes, wave_bytes3(plans, 0, 1));
  if (rc != EFWI_OK) return rc;
  std::vector<std::pair<int, int>> waves;
  rc = plan_waves3(plans, ws_bytes, waves);
  if (rc != EFWI_OK) return rc;
  for (auto [first, count] : waves) {
    Wave3 wv;
    rc = setup_wave3(g, shots, plans, first, count, io, EFWI_WS_GRADIENT, ws, wv, st);
    if (rc != EFWI_OK) return rc;
    rc = run_forward3(wv, ws, true, st);
    if (rc != EFWI_OK) return rc;
    for (int k = 0; k < count; ++k) {
      const Plan3D& p = wv.plans[k];
      unsigned char* r = ws + wv.regions[k];
      float* ebar = reinterpret_cast<float*>(r + p.off_ebar);
      if (p.field)
        HIP_TRY(TIMED(KK_MISFIT, st, field_misfit(p.R, r, p.off_dint, p.off_rf, p.off_partial, io[first + k], ebar, st)));
      else if (io[first + k].r)
        HIP_TRY(TIMED(KK_MISFIT, st, launch_residual_cumsum_raw(p.nch, p.nt, io[first + k].r, ebar, st)));
      else
        HIP_TRY(TIMED(KK_MISFIT, st,
                      launch_misfit_raw(p.nch, p.nt, (const float*)(wv.descs[k].d), io[first + k].dobs,
                                        reinterpret_cast<double*>(r + p.off_partial), io[first + k].phi, ebar, st)));
    }
    rc = run_reverse3(wv, ws, st);
    if (rc != EFWI_OK) return rc;
    if (io[first].accumulate) {
      for (int k = 0; k < count; ++k) {
        const Plan3D& p = wv.plans[k];
        HIP_TRY(launch_add_gradient(reinterpret_cast<const double*>(ws + wv.regions[k] + p.off_G), p.cells, p.cp, p.nz,
                                    p.ny, p.nx, io[first + k].gout, io[first + k].mplane, g.nx, (long)g.ny * g.nx,
                                    p.w.z0, p.w.y0, p.w.x0, st));
      }
      continue;
    }
    for (int k = 0; k < count; ++k) {
      const Plan3D& p = wv.plans[k];
      const bool full = p.w.z0 == 0 && p.w.y0 == 0 && p.w.x0 == 0 && p.nz == g.nz && p.ny == g.ny && p.nx == g.nx;
      if (!full) HIP_TRY(hipMemsetAsync(io[first + k].gout, 0, (size_t)3 * io[first + k].mplane * sizeof(float), st));
    }
    HIP_TRY(launch3_write_gradient(wv.batch, st));
  }
  return EFWI_OK;
}

size_t workspace3(efwi_ws_kind kind, const efwi_grid& g, int n, const efwi_shot* shots) {
  std::vector<Plan3D> plans;
  for (int k = 0; k < n; ++k) plans.push_back(plan3d(g, shots[k], kind));
  return wave_bytes3(plans, 0, n);
}

}  // namespace

// ========================================================================================
// Scratch of the allocation-free entry point: one array per GPU, held until the process
// ends. Host code never passes the array's name (a host-side stand-in) to a kernel or copy:
// it uses the device address hipGetSymbolAddress returns for the current device.
// ========================================================================================
namespace {
static __device__ __align__(256) unsigned char scratch[EFWI_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::once_flag g_scratch_once[MAX_DEVICES];
void* g_scratch_ptr[MAX_DEVICES] = {};
hipError_t g_scratch_err[MAX_DEVICES] = {};

// The current device's scratch address (looked up once per device, with that device current).
efwi_status scratch_of_current_device(unsigned char** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(EFWI_E_UNSUPPORTED, "device %d beyond %d devices", dev, MAX_DEVICES);
  std::call_once(g_scratch_once[dev], [dev]() {
    void* ptr = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? ptr : nullptr;
  });
  if (g_scratch_err[dev] != hipSuccess || !g_scratch_ptr[dev])
    return fail(EFWI_E_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                hipGetErrorString(g_scratch_err[dev]));
  *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
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
    const long npts = (long)grid->nz * grid->nx * (grid->ndim == 3 ? grid->ny : 1);
    return align_up((size_t)regularizer_blocks(npts) * sizeof(double));
  }
  const int n = kind == EFWI_WS_BATCH ? ns : 1;
  if (efwi_validate(grid, n, shots) != EFWI_OK) return 0;
  if (grid->ndim == 3) return workspace3(kind, *grid, n, shots);
  std::vector<Plan2D> plans;
  for (int k = 0; k < n; ++k) plans.push_back(plan2d(*grid, shots[k], kind));
  return wave_bytes(plans, 0, n);
}

efwi_status efwi_set_tile_rows(int fwd_rows, int adj_rows) {
  if ((fwd_rows != 0 && !valid_tile_rows(fwd_rows)) || (adj_rows != 0 && !valid_tile_rows(adj_rows)))
    return fail(EFWI_E_INVAL, "tile rows must be 8, 12 or 16 (0 keeps the current value)");
  if (fwd_rows) g_fwd_rows.store(fwd_rows);
  if (adj_rows) g_adj_rows.store(adj_rows);
  return EFWI_OK;
}

efwi_status efwi_set_wave_cache_bytes(size_t bytes) {
  g_wave_cache_bytes.store(bytes == 0 ? WAVE_CACHE_BYTES : bytes);
  return EFWI_OK;
}

size_t efwi_get_wave_cache_bytes(void) { return g_wave_cache_bytes.load(); }

efwi_status efwi_set_wave_lanes(int lanes) {
  if (lanes < 0 || lanes > 2) return fail(EFWI_E_INVAL, "lanes must be 1 or 2 (0 restores the default)");
  g_wave_lanes.store(lanes == 0 ? DEFAULT_WAVE_LANES : lanes);
  return EFWI_OK;
}

int efwi_get_wave_lanes(void) { return g_wave_lanes.load(); }

efwi_status efwi_get_tile_rows(int* fwd_rows, int* adj_rows) {
  if (!fwd_rows || !adj_rows) return fail(EFWI_E_INVAL, "NULL output pointer");
  *fwd_rows = g_fwd_rows.load();
  *adj_rows = g_adj_rows.load();
  return EFWI_OK;
}

namespace {
// The short run the autotuner times: the shot on its window for `steps` time steps, whole
// history kept, FP32.
void tune_case(const efwi_grid& g, const efwi_shot& s, int steps, efwi_grid& gt, efwi_shot& st) {
  gt = g;
  gt.nt = std::max(1, std::min(steps, g.nt));
  st = s;
  st.ckpt_interval = gt.nt;
  st.ckpt_mode = EFWI_CKPT_FP32;
}
size_t tune_bytes(const efwi_grid& gt, const efwi_shot& st) {
  size_t need = 0;
  for (int r : TILE_ROWS) {
    std::vector<Plan2D> plans{plan2d(gt, st, EFWI_WS_GRADIENT, r, r)};
    need = std::max(need, wave_bytes(plans, 0, 1));
  }
  return need + align_up((size_t)std::max(1, st.nch) * gt.nt * sizeof(float));  // DAS data sink
}
}  // namespace

size_t efwi_autotune_workspace_size(const efwi_grid* grid, const efwi_shot* shot, int steps) {
  if (efwi_validate(grid, 1, shot) != EFWI_OK || grid->ndim != 2 || steps < 1) return 0;
  efwi_grid gt;
  efwi_shot st;
  tune_case(*grid, *shot, steps, gt, st);
  return tune_bytes(gt, st);
}

efwi_status efwi_autotune(const efwi_grid* grid, const efwi_shot* shot, const float* m, const float* src, int steps,
                          void* ws, size_t ws_bytes, void* stream, int* fwd_rows, int* adj_rows, float* times_ms) {
  efwi_status rc = efwi_validate(grid, 1, shot);
  if (rc != EFWI_OK) return rc;
  if (grid->ndim != 2) return fail(EFWI_E_UNSUPPORTED, "tile rows are tuned on 2D grids only");
  if (!m || !src || !fwd_rows || !adj_rows || steps < 1) return fail(EFWI_E_INVAL, "NULL argument or steps < 1");
  efwi_grid gt;
  efwi_shot sh;
  tune_case(*grid, *shot, steps, gt, sh);
  rc = check_ws(ws, ws_bytes, tune_bytes(gt, sh));
  if (rc != EFWI_OK) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  unsigned char* w = static_cast<unsigned char*>(ws);
  hipEvent_t ev[3];
  for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
  float best_f = 1e30f, best_a = 1e30f;
  int rf = g_fwd_rows.load(), ra = g_adj_rows.load();
  rc = EFWI_OK;
  for (int ci = 0; ci < 3; ++ci) {
    const int r = TILE_ROWS[ci];
    std::vector<Plan2D> plans{plan2d(gt, sh, EFWI_WS_GRADIENT, r, r)};
    const size_t wb = wave_bytes(plans, 0, 1);
    ShotIO io;
    io.m = m;
    io.mplane = (long)grid->nz * grid->nx;
    io.src = src;
    io.d = reinterpret_cast<float*>(w + wb);
    float mf = 1e30f, ma = 1e30f;
    for (int rep = 0; rep < 3 && rc == EFWI_OK; ++rep) {  // the first run warms up; best of the others
      Wave wv;
      rc = setup_wave(gt, &sh, plans, 0, 1, {io}, EFWI_WS_GRADIENT, w, wv, st);
      if (rc != EFWI_OK) break;
      const Plan2D& p = wv.plans[0];
      unsigned char* region = w + wv.regions[0];
      if (hipEventRecord(ev[0], st) != hipSuccess || (rc = run_forward(wv, w, true, st)) != EFWI_OK) break;
      // zero adjoint source: the sweep is timed, its result discarded
      if (hipMemsetAsync(region + p.off_ebar, 0, (size_t)std::max(1, p.nch) * p.nt * sizeof(float), st) !=
              hipSuccess ||
          hipEventRecord(ev[1], st) != hipSuccess || (rc = run_reverse(wv, w, st)) != EFWI_OK ||
          hipEventRecord(ev[2], st) != hipSuccess || hipEventSynchronize(ev[2]) != hipSuccess) {
        if (rc == EFWI_OK) rc = fail(EFWI_E_HIP, "autotune: HIP event or memset failed");
        break;
      }
      float tf = 0.f, ta = 0.f;
      hipEventElapsedTime(&tf, ev[0], ev[1]);
      hipEventElapsedTime(&ta, ev[1], ev[2]);
      if (rep > 0) {
        mf = std::min(mf, tf);
        ma = std::min(ma, ta);
      }
    }
    if (rc != EFWI_OK) break;
    if (mf < best_f) best_f = mf, rf = r;
    if (ma < best_a) best_a = ma, ra = r;
    if (times_ms) {
      times_ms[2 * ci] = mf;
      times_ms[2 * ci + 1] = ma;
    }
  }
  for (auto& e : ev) hipEventDestroy(e);
  if (rc != EFWI_OK) return rc;
  g_fwd_rows.store(rf);
  g_adj_rows.store(ra);
  *fwd_rows = rf;
  *adj_rows = ra;
  return EFWI_OK;
}

int efwi_plan_interval(const efwi_grid* grid, const efwi_shot* shot, size_t budget_bytes) {
  efwi_status rc = efwi_validate(grid, 1, shot);
  if (rc != EFWI_OK) return rc;
  efwi_shot s = *shot;
  auto need = [&](int L) {
    s.ckpt_interval = L;
    return efwi_workspace_size(EFWI_WS_GRADIENT, grid, 1, &s);
  };
  const int nt = grid->nt;
  if (need(nt) <= budget_bytes) return nt;
  int lo = std::min(nt, (int)std::ceil(std::sqrt((double)nt)));
  if (need(lo) > budget_bytes)
    return fail(EFWI_E_WORKSPACE, "even the sqrt(nt) checkpoint workspace (%zu bytes) exceeds the budget",
                need(lo));
  int hi = nt;  // need(lo) fits, need(hi) does not
  while (hi - lo > 1) {
    const int mid = lo + (hi - lo) / 2;
    if (need(mid) <= budget_bytes) lo = mid;
    else hi = mid;
  }
  return lo;
}

efwi_status efwi_model_forward(const efwi_grid* grid, const efwi_shot* shot, const float* m, const float* src,
                               float* d, void* ws, size_t ws_bytes, void* stream) {
  efwi_status rc = efwi_validate(grid, 1, shot);
  if (rc != EFWI_OK) return rc;
  if (!m || !src || (shot->nch > 0 && !d)) return fail(EFWI_E_INVAL, "NULL array argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  unsigned char* w = static_cast<unsigned char*>(ws);
  ShotIO io;
  io.m = m;
  io.mplane = (long)grid->nz * grid->nx * (grid->ndim == 3 ? grid->ny : 1);
  io.src = src;
  io.d = d;
  if (grid->ndim == 3) {
    std::vector<Plan3D> plans{plan3d(*grid, *shot, EFWI_WS_FORWARD)};
    rc = check_ws(ws, ws_bytes, wave_bytes3(plans, 0, 1));
    if (rc != EFWI_OK) return rc;
    Wave3 wv;
    rc = setup_wave3(*grid, shot, plans, 0, 1, {io}, EFWI_WS_FORWARD, w, wv, st);
    if (rc != EFWI_OK) return rc;
    rc = run_forward3(wv, w, false, st);
    if (rc != EFWI_OK || !plans[0].field) return rc;
    HIP_TRY(launch_field_data(plans[0].R, reinterpret_cast<const float*>(w + wv.regions[0] + plans[0].off_dint), d, st));
    return EFWI_OK;
  }
  std::vector<Plan2D> plans{plan2d(*grid, *shot, EFWI_WS_FORWARD)};
  rc = check_ws(ws, ws_bytes, wave_bytes(plans, 0, 1));
  if (rc != EFWI_OK) return rc;
  Wave wv;
  rc = setup_wave(*grid, shot, plans, 0, 1, {io}, EFWI_WS_FORWARD, w, wv, st);
  if (rc != EFWI_OK) return rc;
  rc = run_forward(wv, w, false, st);
  if (rc != EFWI_OK || !plans[0].field) return rc;
  HIP_TRY(launch_field_data(plans[0].R, reinterpret_cast<const float*>(w + wv.regions[0] + plans[0].off_dint), d, st));
  return EFWI_OK;
}

efwi_status efwi_model_adjoint(const efwi_grid* grid, const efwi_shot* shot, const float* m, const float* r,
                               float* src_bar, void* ws, size_t ws_bytes, void* stream) {
  efwi_status rc = efwi_validate(grid, 1, shot);
  if (rc != EFWI_OK) return rc;
  if (!m || !src_bar || (shot->nch > 0 && !r)) return fail(EFWI_E_INVAL, "NULL array argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  unsigned char* w = static_cast<unsigned char*>(ws);
  ShotIO io;
  io.m = m;
  io.mplane = (long)grid->nz * grid->nx * (grid->ndim == 3 ? grid->ny : 1);
  io.src_bar = src_bar;
  if (grid->ndim == 3) {
    std::vector<Plan3D> plans{plan3d(*grid, *shot, EFWI_WS_ADJOINT)};
    rc = check_ws(ws, ws_bytes, wave_bytes3(plans, 0, 1));
    if (rc != EFWI_OK) return rc;
    Wave3 wv;
    rc = setup_wave3(*grid, shot, plans, 0, 1, {io}, EFWI_WS_ADJOINT, w, wv, st);
    if (rc != EFWI_OK) return rc;
    const Plan3D& p = wv.plans[0];
    float* ebar3 = reinterpret_cast<float*>(w + wv.regions[0] + p.off_ebar);
    if (p.field) HIP_TRY(launch_field_cumsum(p.R, r, ebar3, st));
    else HIP_TRY(launch_residual_cumsum_raw(p.nch, p.nt, r, ebar3, st));
    for (int n = p.nt - 1; n >= 0; --n) {
      HIP_TRY(TIMED(KK_ADJ_VEL, st, launch3_adj_vel(wv.batch, n, 0, false, false, true, st)));
      HIP_TRY(TIMED(KK_ADJ_STR, st, launch3_adj_str(wv.batch, n, 0, false, false, st)));
    }
    return EFWI_OK;
  }
  std::vector<Plan2D> plans{plan2d(*grid, *shot, EFWI_WS_ADJOINT)};
  rc = check_ws(ws, ws_bytes, wave_bytes(plans, 0, 1));
  if (rc != EFWI_OK) return rc;
  Wave wv;
  rc = setup_wave(*grid, shot, plans, 0, 1, {io}, EFWI_WS_ADJOINT, w, wv, st);
  if (rc != EFWI_OK) return rc;
  const Plan2D& p = wv.plans[0];
  float* ebar = reinterpret_cast<float*>(w + wv.regions[0] + p.off_ebar);
  if (p.field) HIP_TRY(launch_field_cumsum(p.R, r, ebar, st));
  else HIP_TRY(launch_residual_cumsum(wv.descs[0], r, ebar, st));
  for (int n = p.nt - 1; n >= 0; --n) {
    HIP_TRY(TIMED(KK_ADJ_STEP, st, launch_adj_step(wv.batch, n, 0, false, false, true, st)));
  }
  return EFWI_OK;
}

efwi_status efwi_shot_gradient(const efwi_grid* grid, const efwi_shot* shot, const float* m, const float* src,
                               const float* d_obs, float* g, double* phi, float* d_out, void* ws, size_t ws_bytes,
                               void* stream) {
  efwi_status rc = efwi_validate(grid, 1, shot);
  if (rc != EFWI_OK) return rc;
  if (!m || !src || !g || !phi || (shot->nch > 0 && !d_obs)) return fail(EFWI_E_INVAL, "NULL array argument");
  ShotIO io;
  io.m = m;
  io.mplane = (long)grid->nz * grid->nx * (grid->ndim == 3 ? grid->ny : 1);
  io.src = src;
  io.dobs = d_obs;
  io.d = d_out;
  io.gout = g;
  io.phi = phi;
  return gradient_waves(*grid, shot, 1, {io}, static_cast<unsigned char*>(ws), ws_bytes,
                        reinterpret_cast<hipStream_t>(stream));
}

efwi_status efwi_shot_jt(const efwi_grid* grid, const efwi_shot* shot, const float* m, const float* src,
                         const float* v, float* g, float* d_out, void* ws, size_t ws_bytes, void* stream) {
  efwi_status rc = efwi_validate(grid, 1, shot);
  if (rc != EFWI_OK) return rc;
  if (!m || !src || !g || (shot->nch > 0 && !v)) return fail(EFWI_E_INVAL, "NULL array argument");
  ShotIO io;
  io.m = m;
  io.mplane = (long)grid->nz * grid->nx * (grid->ndim == 3 ? grid->ny : 1);
  io.src = src;
  io.r = v;
  io.d = d_out;
  io.gout = g;
  return gradient_waves(*grid, shot, 1, {io}, static_cast<unsigned char*>(ws), ws_bytes,
                        reinterpret_cast<hipStream_t>(stream));
}

size_t efwi_noalloc_scratch_bytes(void) { return EFWI_NOALLOC_SCRATCH_BYTES; }

efwi_status efwi_shot_gradient_noalloc(const efwi_grid* grid, const efwi_shot* shot, const float* m,
                                       const float* src, const float* d_obs, float* g, double* phi, float* d_out,
                                       void* stream) {
  efwi_status rc = efwi_validate(grid, 1, shot);
  if (rc != EFWI_OK) return rc;
  if (!m || !src || !g || !phi || (shot->nch > 0 && !d_obs)) return fail(EFWI_E_INVAL, "NULL array argument");
  const size_t need = efwi_workspace_size(EFWI_WS_GRADIENT, grid, 1, shot);
  if (need > EFWI_NOALLOC_SCRATCH_BYTES)
    return fail(EFWI_E_WORKSPACE,
                "the shot needs %zu bytes of scratch; the allocation-free entry point has %zu (use a smaller "
                "ckpt_interval or efwi_shot_gradient with a workspace)",
                need, (size_t)EFWI_NOALLOC_SCRATCH_BYTES);
  unsigned char* ws = nullptr;
  rc = scratch_of_current_device(&ws);
  if (rc != EFWI_OK) return rc;
  ShotIO io;
  io.m = m;
  io.mplane = (long)grid->nz * grid->nx * (grid->ndim == 3 ? grid->ny : 1);
  io.src = src;
  io.dobs = d_obs;
  io.d = d_out;
  io.gout = g;
  io.phi = phi;
  NoAllocScope scope;
  return gradient_waves(*grid, shot, 1, {io}, ws, EFWI_NOALLOC_SCRATCH_BYTES, reinterpret_cast<hipStream_t>(stream));
}

efwi_status efwi_batch_waves(const efwi_grid* grid, int ns, const efwi_shot* shots, size_t ws_bytes, int* nwaves,
                             int* wave_first, int* order, int* lanes) {
  efwi_status rc = efwi_validate(grid, ns, shots);
  if (rc != EFWI_OK) return rc;
  if (ns < 1 || !nwaves) return fail(EFWI_E_INVAL, "ns must be >= 1 and nwaves not NULL");
  std::vector<std::pair<int, int>> waves;
  std::vector<int> ord(ns);
  for (int k = 0; k < ns; ++k) ord[k] = k;
  int nlanes = 1;
  if (grid->ndim == 3) {
    std::vector<Plan3D> plans;
    for (int k = 0; k < ns; ++k) plans.push_back(plan3d(*grid, shots[k], EFWI_WS_GRADIENT));
    rc = plan_waves3(plans, ws_bytes, waves);
  } else {
    std::vector<Plan2D> plans;
    for (int k = 0; k < ns; ++k) plans.push_back(plan2d(*grid, shots[k], EFWI_WS_GRADIENT));
    size_t lane_bytes = ws_bytes;
    rc = plan_lanes(plans, ws_bytes, true, true, ord, waves, nlanes, lane_bytes);
  }
  if (rc != EFWI_OK) return rc;
  *nwaves = (int)waves.size();
  if (lanes) *lanes = nlanes;
  if (wave_first)
    for (size_t i = 0; i < waves.size(); ++i) wave_first[i] = waves[i].first;
  if (order)
    for (int k = 0; k < ns; ++k) order[k] = ord[k];
  return EFWI_OK;
}

efwi_status efwi_batch_gradient(const efwi_grid* grid, int ns, const efwi_shot* shots, const float* m_ext,
                                const float* src, const float* d_obs, float* g_ext, double* phi, void* ws,
                                size_t ws_bytes, void* stream) {
  efwi_status rc = efwi_validate(grid, ns, shots);
  if (rc != EFWI_OK) return rc;
  if (ns < 1) return fail(EFWI_E_INVAL, "ns must be >= 1");
  if (!m_ext || !src || !g_ext || !phi) return fail(EFWI_E_INVAL, "NULL array argument");
  rc = check_same_schedule(*grid, ns, shots);
  if (rc != EFWI_OK) return rc;
  const long plane = (long)grid->nz * grid->nx * (grid->ndim == 3 ? grid->ny : 1);
  const int ncomp = grid->ndim == 3 ? 6 : 3;
  std::vector<ShotIO> io(ns);
  size_t off_obs = 0;
  for (int s = 0; s < ns; ++s) {
    if (shots[s].nch > 0 && !d_obs) return fail(EFWI_E_INVAL, "d_obs is NULL");
    io[s].m = m_ext + (size_t)s * 3 * plane;
    io[s].mplane = plane;
    io[s].src = src + (size_t)s * ncomp * grid->nt;
    io[s].dobs = d_obs ? d_obs + off_obs : nullptr;
    io[s].gout = g_ext + (size_t)s * 3 * plane;
    io[s].phi = phi + s;
    off_obs += data_floats(*grid, shots[s]);
  }
  return gradient_waves(*grid, shots, ns, io, static_cast<unsigned char*>(ws), ws_bytes,
                        reinterpret_cast<hipStream_t>(stream));
}

efwi_status efwi_batch_gradient_grouped(const efwi_grid* grid, int ns, const efwi_shot* shots, const int* group,
                                        int ng, const float* m_ext, const float* src, const float* d_obs,
                                        float* g_ext, double* phi, void* ws, size_t ws_bytes, void* stream) {
  efwi_status rc = efwi_validate(grid, ns, shots);
  if (rc != EFWI_OK) return rc;
  if (ns < 1 || ng < 1) return fail(EFWI_E_INVAL, "ns and ng must be >= 1");
  if (!group || !m_ext || !src || !g_ext || !phi) return fail(EFWI_E_INVAL, "NULL array argument");
  for (int s = 0; s < ns; ++s)
    if (group[s] < 0 || group[s] >= ng) return fail(EFWI_E_INVAL, "shot %d: group %d outside [0, %d)", s, group[s], ng);
  rc = check_same_schedule(*grid, ns, shots);
  if (rc != EFWI_OK) return rc;
  const long plane = (long)grid->nz * grid->nx * (grid->ndim == 3 ? grid->ny : 1);
  const int ncomp = grid->ndim == 3 ? 6 : 3;
  std::vector<ShotIO> io(ns);
  size_t off_obs = 0;
  for (int s = 0; s < ns; ++s) {
    if (shots[s].nch > 0 && !d_obs) return fail(EFWI_E_INVAL, "d_obs is NULL");
    io[s].m = m_ext + (size_t)group[s] * 3 * plane;
    io[s].mplane = plane;
    io[s].src = src + (size_t)s * ncomp * grid->nt;
    io[s].dobs = d_obs ? d_obs + off_obs : nullptr;
    io[s].gout = g_ext + (size_t)group[s] * 3 * plane;
    io[s].phi = phi + s;
    io[s].accumulate = true;
    off_obs += data_floats(*grid, shots[s]);
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // the first shot's workspace is checked before anything is written
  rc = check_ws(ws, ws_bytes, efwi_workspace_size(EFWI_WS_GRADIENT, grid, 1, shots));
  if (rc != EFWI_OK) return rc;
  HIP_TRY(hipMemsetAsync(g_ext, 0, (size_t)ng * 3 * plane * sizeof(float), st));
  return gradient_waves(*grid, shots, ns, io, static_cast<unsigned char*>(ws), ws_bytes, st);
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
  const long npts = (long)grid->nz * grid->nx * (grid->ndim == 3 ? grid->ny : 1);
  const int nb = regularizer_blocks(npts);
  rc = check_ws(ws, ws_bytes, align_up((size_t)nb * sizeof(double)));
  if (rc != EFWI_OK) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  HIP_TRY(TIMED(KK_REG, st,
                launch_regularizer(ns, npts, npts, m_ext, b, sink, eta, g_ext, static_cast<double*>(ws), nb, phi,
                                   st)));
  return EFWI_OK;
}

efwi_status efwi_zoi_weights(const efwi_grid* grid, int ns, const efwi_zoi* zones, float n, float nu, float* b,
                             unsigned char* sink, void* stream) {
  g_last_error.clear();
  efwi_status rc = validate_grid(grid);
  if (rc != EFWI_OK) return rc;
  if (ns < 1) return fail(EFWI_E_INVAL, "ns must be >= 1");
  if (!zones || !b || !sink) return fail(EFWI_E_INVAL, "NULL argument");
  if (!(std::isfinite(n) && n > 0.0f)) return fail(EFWI_E_INVAL, "n must be finite and > 0 (got %g)", n);
  if (!(nu > 0.0f && nu < 1.0f)) return fail(EFWI_E_INVAL, "nu must lie in (0, 1) (got %g)", nu);
  const bool three = grid->ndim == 3;
  for (int s = 0; s < ns; ++s) {
    const efwi_zoi& z = zones[s];
    bool finite = std::isfinite(z.taper);
    for (float v : z.src) finite = finite && std::isfinite(v);
    for (float v : z.icov) finite = finite && std::isfinite(v);
    for (float v : z.box) finite = finite && std::isfinite(v);
    if (!finite) return fail(EFWI_E_INVAL, "zone %d has a non-finite entry", s);
    if (z.taper < 0.0f) return fail(EFWI_E_INVAL, "zone %d: negative taper", s);
    if (z.box[1] < z.box[0] || z.box[5] < z.box[4] || (three && z.box[3] < z.box[2]))
      return fail(EFWI_E_INVAL, "zone %d: box upper bound below lower bound", s);
    // positive definite: leading principal minors of [[zz, zy, zx], [zy, yy, yx], [zx, yx, xx]]
    // (2D: of [[zz, zx], [zx, xx]])
    const double zz = z.icov[0], yy = z.icov[1], xx = z.icov[2], zy = z.icov[3], zx = z.icov[4], yx = z.icov[5];
    bool pd;
    if (three) {
      const double m2 = zz * yy - zy * zy;
      const double m3 = zz * (yy * xx - yx * yx) - zy * (zy * xx - yx * zx) + zx * (zy * yx - yy * zx);
      pd = zz > 0.0 && m2 > 0.0 && m3 > 0.0;
    } else {
      pd = zz > 0.0 && zz * xx - zx * zx > 0.0;
    }
    if (!pd) return fail(EFWI_E_INVAL, "zone %d: inverse covariance is not positive definite", s);
  }
  const int ny = three ? grid->ny : 1;
  const long npts = (long)grid->nz * ny * grid->nx;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  for (int s0 = 0; s0 < ns; s0 += ZOI_BATCH) {   // up to ZOI_BATCH zones per launch
    const int count = std::min(ZOI_BATCH, ns - s0);
    ZoiBatch zb{};
    for (int q = 0; q < count; ++q) {
      const efwi_zoi& z = zones[s0 + q];
      ZoiArgs& a = zb.z[q];
      for (int k = 0; k < 3; ++k) a.src[k] = z.src[k];
      for (int k = 0; k < 6; ++k) a.icov[k] = z.icov[k], a.box[k] = z.box[k];
      a.taper = z.taper, a.n = n, a.nu = nu;
    }
    HIP_TRY(TIMED(KK_ZOI, st,
                  launch_zoi(three ? 1 : 0, count, npts, grid->nz, ny, grid->nx, grid->dz, three ? grid->dy : 0.0,
                             grid->dx, zb, b + (size_t)s0 * npts, sink + (size_t)s0 * npts, st)));
  }
  return EFWI_OK;
}

int efwi_bspline_nodes(int n, int spacing) { return (n >= 1 && spacing >= 1) ? bspline_nodes(n, spacing) : 0; }

static efwi_status check_bspline(int nz, int nx, int dz_nodes, int dx_nodes, int np, const void* a, const void* b) {
  if (nz < 1 || nx < 1 || np < 1) return fail(EFWI_E_INVAL, "nz, nx and np must be >= 1");
  if (dz_nodes < 1 || dx_nodes < 1) return fail(EFWI_E_INVAL, "node spacings must be >= 1 cell");
  if (dz_nodes + dx_nodes > 2000) return fail(EFWI_E_INVAL, "node spacings must sum to at most 2000 cells");
  if (!a || !b) return fail(EFWI_E_INVAL, "NULL array argument");
  return EFWI_OK;
}

efwi_status efwi_bspline_expand(int nz, int nx, int dz_nodes, int dx_nodes, int np, const float* c, float* m,
                                void* stream) {
  g_last_error.clear();
  const efwi_status rc = check_bspline(nz, nx, dz_nodes, dx_nodes, np, c, m);
  if (rc != EFWI_OK) return rc;
  HIP_TRY(launch_bspline_expand(np, nz, nx, dz_nodes, dx_nodes, c, m, reinterpret_cast<hipStream_t>(stream)));
  return EFWI_OK;
}

efwi_status efwi_bspline_adjoint(int nz, int nx, int dz_nodes, int dx_nodes, int np, const float* g, float* c_bar,
                                 void* stream) {
  g_last_error.clear();
  const efwi_status rc = check_bspline(nz, nx, dz_nodes, dx_nodes, np, g, c_bar);
  if (rc != EFWI_OK) return rc;
  HIP_TRY(launch_bspline_adjoint(np, nz, nx, dz_nodes, dx_nodes, g, c_bar, reinterpret_cast<hipStream_t>(stream)));
  return EFWI_OK;
}

efwi_status efwi_das_field(const efwi_grid* grid, const efwi_shot* shot, const float* e, float* out, void* stream) {
  efwi_status rc = efwi_validate(grid, 1, shot);
  if (rc != EFWI_OK) return rc;
  if (shot->nch > 0 && (!e || !out)) return fail(EFWI_E_INVAL, "NULL array argument");
  HIP_TRY(launch_field_data(receiver_of(*grid, *shot), e, out, reinterpret_cast<hipStream_t>(stream)));
  return EFWI_OK;
}

efwi_status efwi_pseudo_hessian(const efwi_grid* grid, int ns, const efwi_shot* shots, const float* m_ext,
                                const float* src, float clip, float* h, float* p, void* ws, size_t ws_bytes,
                                void* stream) {
  efwi_status rc = efwi_validate(grid, ns, shots);
  if (rc != EFWI_OK) return rc;
  if (grid->ndim != 2) return fail(EFWI_E_INVAL, "pseudo_hessian is 2D only");
  if (ns < 1) return fail(EFWI_E_INVAL, "ns must be >= 1");
  if (!m_ext || !src || !h || !p) return fail(EFWI_E_INVAL, "NULL array argument");
  if (!(clip > 0.0f && clip <= 1.0f)) return fail(EFWI_E_INVAL, "clip must be in (0, 1]");
  const efwi_grid& g = *grid;
  const long plane = (long)g.nz * g.nx;
  std::vector<ShotIO> io(ns);
  for (int s = 0; s < ns; ++s) {
    io[s].m = m_ext + (size_t)s * 3 * plane;
    io[s].mplane = plane;
    io[s].src = src + (size_t)s * 3 * g.nt;
  }
  std::vector<Plan2D> plans;
  for (int k = 0; k < ns; ++k) plans.push_back(plan2d(g, shots[k], EFWI_WS_GRADIENT));
  unsigned char* w = static_cast<unsigned char*>(ws);
  rc = check_ws(w, ws_bytes, std::max(wave_bytes(plans, 0, 1),
                                     align_up((size_t)inverse_diag_partials(plane) * sizeof(float))));
  if (rc != EFWI_OK) return rc;
  std::vector<std::pair<int, int>> waves;
  rc = plan_waves(plans, ws_bytes, waves);
  if (rc != EFWI_OK) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  HIP_TRY(hipMemsetAsync(h, 0, (size_t)plane * sizeof(float), st));
  for (auto [first, count] : waves) {
    Wave wv;
    rc = setup_wave(g, shots, plans, first, count, io, EFWI_WS_GRADIENT, w, wv, st);
    if (rc != EFWI_OK) return rc;
    for (int k = 0; k < count; ++k)
      HIP_TRY(hipMemsetAsync(w + wv.regions[k] + wv.plans[k].off_acc, 0, (size_t)wv.plans[k].cells * sizeof(float),
                             st));
    for (int n = 0; n < g.nt; ++n) HIP_TRY(TIMED(KK_ACORR, st, launch_fwd_acorr(wv.batch, n, st)));
    for (int k = 0; k < count; ++k) {  // one launch per shot: overlapping windows add in shot order
      const Plan2D& pl = wv.plans[k];
      HIP_TRY(launch_add_window(reinterpret_cast<const float*>(w + wv.regions[k] + pl.off_acc), pl.cp, pl.nz, pl.nx,
                                h, g.nx, pl.w.z0, pl.w.x0, st));
    }
  }
  HIP_TRY(launch_inverse_diag(h, plane, clip, p, reinterpret_cast<float*>(w), st));
  return EFWI_OK;
}

efwi_status efwi_final_model(const efwi_grid* grid, int ns, const float* m_ext, const float* b,
                             const unsigned char* sink, float* m_out, void* stream) {
  g_last_error.clear();
  efwi_status rc = validate_grid(grid);
  if (rc != EFWI_OK) return rc;
  if (ns < 1) return fail(EFWI_E_INVAL, "ns must be >= 1");
  if (!m_ext || !b || !sink || !m_out) return fail(EFWI_E_INVAL, "NULL array argument");
  const long npts = (long)grid->nz * grid->nx * (grid->ndim == 3 ? grid->ny : 1);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  HIP_TRY(TIMED(KK_FINAL, st, launch_final_model(ns, npts, m_ext, b, sink, m_out, st)));
  return EFWI_OK;
}

}  // extern "C"
