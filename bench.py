"""Throughput of the source-extended elastic FWI hot path on one MI355X.

One step = one pass of the whole hot path over the batched workload: 64 shots on uneven
windows (nz_s ~ U[400,1000], nx_s ~ U[800,3000], dx = 2.5 m, 40-cell CPML in each window)
cut around their moment-tensor sources from the 1000 x 3000 shale model, nt = 4000; each
shot's gradient (forward sweep with DAS recording, FP64 misfit, reverse sweep of transposed
stress/velocity steps, imaging condition, chain rule) into its own component m_s of the
64-component extended model, advanced in waves by efwi_batch_gradient, then the
consistency-regularizer value and gradient over the 64 components (hard sinkholes). The
forward history is kept with the largest checkpoint interval whose workspace fits in the
free HBM (every window's whole history fits in an MI355X, so nothing is recomputed).

Metric: Gcell-updates/s = sum over shots of window cells x nt / wall time (fwd + adj + grad),
inputs resident in HBM before the timed region.

Byte model (algorithmic bytes per cell-step, FP32, no temporal blocking; each array read or
written once per pass; the model is 3 values, the derived parameters are not counted):
  forward step           read 5 state + 3 model, write 5 state       52 B   (3D: 9 + 3, 9: 84 B)
  store v for imaging    write 2 (3D: 3)                               8 B   (12 B)
  adjoint step           as the forward step                          52 B   (84 B)
  imaging condition      read v at n+1/2 and n-1/2                    16 B   (24 B)
  gradient accumulators  3 x (read + write)                           24 B   (24 B)
  => 152 B per cell-step with the whole history, + 52 B per recomputed step (204 B with
  sqrt(nt) checkpoints); 3D 228 B and + 84 B (312 B). CPML memory variables add 32 B per
  strip cell and pass in 2D (4 variables read and written; a corner cell lies in both
  strips) and 48 B per strip cell, axis and pass in 3D, passes = forward, adjoint and the
  recomputed share. The library's own compulsory bytes (it stores 5 pre-multiplied imaging
  quantities instead of 2 velocities and keeps the staged parameters) are reported beside
  as `design_bytes_per_cell_step`.

The JSON line also carries:
* roofline: the dominant kernel's algorithmic bytes per launch (adj_step: 92 B per cell plus
  32 B per strip cell, averaged over the launches of the waves) over its mean launch time
  (HIP events around sampled launches on the library's stream), against 8 TB/s; `traffic`
  is the HBM bytes per launch from rocprofv3's read and write counters, measured per cell on
  the first windows of this workload and recorded below for the current kernel (else null);
* path: the whole step's algorithmic bytes (with CPML) over the step time;
* forms: the same 64 windows as 64 sequential shot_gradient calls (shots/s plain vs
  batched), the batched form with sqrt(nt) FP32, FP16 and BF16 checkpoints (accuracy of the
  16-bit ones against FP32) and with sqrt(nt) checkpoints in waves sized by the workspace
  alone instead of the Infinity Cache, the plain 1000 x 3000 workload (20 shots, whole
  history), the differentiation workload (1200 x 4000, nt = 8000, sqrt(nt) = 90-step checkpoints through
  torch.autograd, a stated subset of its 32 shots), one VTI shot, one full shot of the 3D precision workload (8-shot time extrapolated);
* cpu_baseline: the FP64 NumPy oracle on a bounded sample of the same workload, one process
  and one process per core (the host's core count and CPU model recorded);
* extension_ops: the zone-of-influence weights, final model, pseudo-Hessian, field DAS
  sampling and B-spline operators (once per inversion, not part of the step).
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per cell and pass (see the module docstring)
ALG2 = {"fwd": 52, "store": 8, "adj": 52, "img": 16, "acc": 24, "psi": 32}
ALG3 = {"fwd": 84, "store": 12, "adj": 84, "img": 24, "acc": 24, "psi": 48}
# the library's compulsory bytes per cell: fused forward step 52 (+20 storing the 5 imaging
# quantities), fused transposed step 96 (state, 3 staged parameters, 5 stored quantities,
# 3 imaging sums read and written)
DESIGN2 = {"fwd": 52, "fwd_store": 72, "adj": 96}
# HBM bytes per cell of one launch of the dominant kernel, measured with rocprofv3's read
# and write counters (FETCH_SIZE x 2.00 + WRITE_SIZE x 1.00 KiB, the factors of a 256 MiB
# device copy) on the first 3 windows of this workload at 400 steps (whole history, one wave
# each: 1.45 M cells per launch, 14.7% of them CPML strip cells against the full workload's
# 15.1%), keyed by (kernel, tile rows); profiles/batched2d_64windows_adj_step_counters.md.
# `traffic` is that figure times the cells of a launch of this run. A kernel changed since
# its measurement is removed from here.
MEASURED_TRAFFIC_PER_CELL = {("adj_step", 12): 109.77}


def strip_cells_2d(wz, wx, npml):
    """Cells of the x strips plus cells of the z strips (corners count twice: both sets of
    memory variables live there)."""
    return 2 * npml * wz + 2 * npml * wx


def path_bytes_2d(cells, strips, rf):
    """Algorithmic bytes of one cell-step summed over shots: cells and strip cells of the
    shots, recompute fraction rf."""
    a = ALG2
    per_cell = a["fwd"] + a["store"] + a["adj"] + a["img"] + a["acc"] + rf * a["fwd"]
    return per_cell * cells + a["psi"] * strips * (2.0 + rf)


def design_bytes_2d(rf):
    return DESIGN2["fwd_store"] + DESIGN2["adj"] + rf * DESIGN2["fwd"]


# ---------------------------------------------------------------------------------------
# CPU baseline: the FP64 oracle (test infrastructure) on a bounded sample, in child
# processes started before this process touches the GPU.
# ---------------------------------------------------------------------------------------
def _cpu_sample(steps):
    """One oracle shot gradient on the smallest window of the batched workload, `steps`
    time steps (fwd + adj + grad); returns (cells x steps, seconds, window shape)."""
    from oracle import elastic2d as E
    from paper_2305_14130_amd import inputs
    w = inputs.batched_2d(nshots=64, nt=max(steps, 1))
    k = int(np.argmin([s.wz * s.wx for s in w.shots]))
    s = w.shots[k]
    g = E.Grid2D(nz=s.wz, nx=s.wx, dz=w.dz, dx=w.dx, dt=w.dt, nt=steps, npml=w.npml, pml_R=w.pml_R, pml_f0=w.f0,
                 vp_max=w.vp_max)
    m = w.m_start[:, s.z0:s.z0 + s.wz, s.x0:s.x0 + s.wx]
    src = np.outer(s.M, w.stf[:steps])
    t0 = time.perf_counter()
    E.shot_gradient(g, m, s.src_iz - s.z0, s.src_ix - s.x0, src, s.ch_iz - s.z0, s.ch_ix - s.x0,
                    np.zeros((len(s.ch_ix), steps)))
    return s.wz * s.wx * steps, time.perf_counter() - t0, (s.wz, s.wx)


def _host_info():
    model = ""
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.lower().startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    return {"nproc": os.cpu_count(), "model": model}


def cpu_baseline(steps=240, workers=None):
    """One oracle process alone, then `workers` independent processes at once (shots are
    independent, one per core); NumPy single-threaded in each (its elementwise ops are)."""
    host = _host_info()
    workers = workers or min(16, host["nproc"] or 1)
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-worker", str(steps)]

    def run(n):
        procs = [subprocess.Popen(cmd, stdout=subprocess.PIPE, text=True, env=env, cwd=ROOT) for _ in range(n)]
        t0 = time.perf_counter()
        res = []
        for p in procs:
            out, _ = p.communicate(timeout=600)
            if p.returncode != 0:
                raise RuntimeError(f"oracle worker failed with {p.returncode}")
            res.append(json.loads(out.strip().splitlines()[-1]))
        return res, time.perf_counter() - t0

    one, _ = run(1)
    many, wall = run(workers)
    cs = one[0]["cell_steps"]
    rate1 = cs / one[0]["seconds"] / 1e9
    rate_n = sum(r["cell_steps"] for r in many) / max(r["seconds"] for r in many) / 1e9
    shape = one[0]["window"]
    return {"value": round(rate_n, 6), "unit": "Gcell-updates/s", "cores": workers, "kind": "oracle",
            "sample": f"{workers} independent processes, each one shot of the batched workload on its smallest "
                      f"window ({shape[0]}x{shape[1]}, CPML 40), {steps} of 4000 time steps, fwd+adj+grad, "
                      f"FP64 NumPy single-threaded; wall {wall:.1f} s",
            "one_core": {"value": round(rate1, 6), "seconds": round(one[0]["seconds"], 2)},
            "host": host,
            "note": "the oracle is a correctness reference, not a tuned CPU code"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------------------
# Forms beside the headline.
# ---------------------------------------------------------------------------------------
def plain_1000x3000_form(efwi, inputs, torch, dev, nt, nshots=20):
    """The plain workload: 20 shots on the whole 1000 x 3000 grid, one shot gradient after
    the other (whole history), then the regularizer; timed once after one untimed pass."""
    w = inputs.plain_2d(nshots=nshots, nt=nt)
    ns, nz, nx = len(w.shots), w.nz, w.nx
    grid = efwi.make_grid(nz, nx, w.dz, w.dx, w.dt, nt, w.npml, w.pml_R, w.f0, w.vp_max)
    T = lambda a: torch.tensor(np.asarray(a, np.float32), device=dev)
    shots = [efwi.Shot(s.src_iz, s.src_ix, s.ch_iz, s.ch_ix) for s in w.shots]
    m_start = T(w.m_start)
    src = T(np.stack([np.outer(s.M, w.stf) for s in w.shots]))
    fws = efwi.workspace(efwi.workspace_size(efwi.WS_FORWARD, grid, shots[:1]), dev)
    m_true = T(w.m_true)
    obs = [efwi.model_forward(grid, shots[k], m_true, src[k], ws=fws) for k in range(ns)]
    del fws, m_true
    noise = T(np.stack([inputs.smooth_random_field((nz, nx), 20.0, 77 + k, 0.01) for k in range(3)]))
    m_ext = torch.stack([m_start * (1.0 + torch.roll(noise, shifts=(0, 37 * k), dims=(1, 2))) for k in range(ns)])
    del noise
    b_np, sink_np = inputs.hard_sinkholes(ns, nz, nx, [s.src_iz for s in w.shots], [s.src_ix for s in w.shots])
    b, sink = T(b_np), torch.tensor(sink_np, device=dev)
    g_ext = torch.empty_like(m_ext)
    phi = torch.empty((ns,), dtype=torch.float64, device=dev)
    phi_reg = torch.empty((), dtype=torch.float64, device=dev)
    rws = efwi.workspace(efwi.workspace_size(efwi.WS_REGULARIZER, grid, []), dev)
    torch.cuda.synchronize()
    L = efwi.plan_interval(grid, shots[0], int(0.9 * torch.cuda.mem_get_info(dev)[0]))
    shots = [dataclasses.replace(s, ckpt_interval=L, _keep=[]) for s in shots]
    ws = efwi.workspace(efwi.workspace_size(efwi.WS_GRADIENT, grid, shots[:1]), dev)

    def step():
        for k in range(ns):
            efwi.shot_gradient(grid, shots[k], m_ext[k], src[k], obs[k], g=g_ext[k], phi=phi[k], ws=ws)
        efwi.extension_regularizer(grid, m_ext, b, sink, 1.0, g_ext, phi=phi_reg, ws=rws)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert bool(torch.isfinite(phi).all())
    rf = efwi.recompute_fraction(grid, L)
    cells = ns * nz * nx
    gcell = cells * nt / dt / 1e9
    alg = path_bytes_2d(cells, ns * strip_cells_2d(nz, nx, w.npml), rf) / cells
    out = {"shots": ns, "grid": [nz, nx], "nt": nt, "ckpt_interval": L, "recompute_fraction": round(rf, 4),
           "ms": round(dt * 1e3, 1), "gcell_per_s": round(gcell, 3), "shots_per_s": round(ns / dt, 3),
           "bytes_per_cell_step": round(alg, 1), "path_frac": round(alg * gcell / HBM_PEAK_GBS, 4),
           "note": "one shot's per-step state (about 160 MB) stays in the 256 MB Infinity Cache between steps"}
    del ws, rws, m_ext, g_ext, b, sink, obs, src, m_start
    torch.cuda.empty_cache()
    return out


def autograd_form(efwi, inputs, torch, dev, nt, subset=4, nshots=32):
    """The differentiation workload (1200 x 4000 at 2 m, nt = 8000, 32 shots along the well):
    each shot's misfit through autograd.ShotMisfit, backward to the model, with sqrt(nt) = 90-step
    checkpoints (recomputation in the reverse sweep) and, for comparison with storing the
    forward history, with the largest checkpoint interval whose workspace fits 85% of the free
    HBM (a shot's whole history, 5 x 4.8e6 x 8000 x 4 B = 768 GB, does not fit); `subset` of the
    32 shots timed once per form after one untimed shot, the 32-shot time extrapolated linearly
    (shots cost the same: same grid and channels). Both forms give the same gradient bit for
    bit (the imaging sums are blocked on absolute step numbers)."""
    from paper_2305_14130_amd import autograd as AG
    w = inputs.differentiation_2d(nt=nt, nshots=nshots)
    nz, nx = w.nz, w.nx
    grid = efwi.make_grid(nz, nx, w.dz, w.dx, w.dt, nt, w.npml, w.pml_R, w.f0, w.vp_max)
    T = lambda a: torch.tensor(np.asarray(a, np.float32), device=dev)
    picks = [int(round(k * (nshots - 1) / max(1, subset - 1))) for k in range(subset)]
    base = [efwi.Shot(w.shots[k].src_iz, w.shots[k].src_ix, w.shots[k].ch_iz, w.shots[k].ch_ix, ckpt_interval=0)
            for k in picks]
    srcs = [T(np.outer(w.shots[k].M, w.stf)) for k in picks]
    m_true = T(w.m_true)
    obs = [efwi.model_forward(grid, base[q], m_true, srcs[q]) for q in range(subset)]
    del m_true
    m = T(w.m_start).requires_grad_(True)
    torch.cuda.synchronize()
    # the workspace for the largest interval is planned on the shot with the most channels
    big = min(efwi.plan_interval(grid, s, int(0.85 * torch.cuda.mem_get_info(dev)[0])) for s in base)
    out = {"grid": [nz, nx], "nt": nt, "shots_timed": subset, "shots_total": nshots, "shot_indices": picks}
    grads = {}
    for name, interval in (("sqrt_nt", 0), ("largest_interval", big)):
        shots = [dataclasses.replace(s, ckpt_interval=interval, _keep=[]) for s in base]
        ws = efwi.workspace(max(efwi.workspace_size(efwi.WS_GRADIENT, grid, [s]) for s in shots), dev)

        def one(q):
            phi = AG.ShotMisfit.apply(m, srcs[q], obs[q], grid, shots[q], ws)
            phi.backward()

        one(0)
        torch.cuda.synchronize()
        m.grad = None
        t0 = time.perf_counter()
        for q in range(subset):
            one(q)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert bool(torch.isfinite(m.grad).all())
        grads[name] = m.grad.clone()
        m.grad = None
        rf = efwi.recompute_fraction(grid, interval)
        cells = nz * nx
        gcell = subset * cells * nt / dt / 1e9
        alg = path_bytes_2d(cells, strip_cells_2d(nz, nx, w.npml), rf) / cells
        out[name] = {"ckpt_interval": int(np.ceil(np.sqrt(nt))) if interval == 0 else interval,
                     "recompute_fraction": round(rf, 4), "ms": round(dt * 1e3, 1), "gcell_per_s": round(gcell, 3),
                     "extrapolated_32_shots_s": round(dt * nshots / subset, 2),
                     "bytes_per_cell_step": round(alg, 1), "path_frac": round(alg * gcell / HBM_PEAK_GBS, 4)}
        del ws
        torch.cuda.empty_cache()
    out["identical_gradients"] = bool(torch.equal(grads["sqrt_nt"], grads["largest_interval"]))
    del m, obs, srcs, grads
    torch.cuda.empty_cache()
    return out


def vti_shot_form(efwi, inputs, torch, dev, nt):
    """One shot of the plain workload (1000 x 3000, whole history) in a VTI medium (Thomsen
    eps 0.1 above the reservoir, 0.6 in it and 0.3 below, smoothed; delta = eps / 2), timed
    once after one untimed call. path_frac: the isotropic algorithmic bytes plus c11 and c13
    read in both passes and two more imaging sums (2 x 8 B + 16 B = 32 B)."""
    from scipy.ndimage import gaussian_filter
    w = inputs.plain_2d(nshots=1, nt=nt)
    nz, nx = w.nz, w.nx
    T = lambda a: torch.tensor(np.asarray(a, np.float32), device=dev)
    i = np.arange(nz)
    col = np.where(i < nz // 2 - 3, 0.1, np.where(i < nz // 2 + 3, 0.6, 0.3))
    eps = torch.tensor(np.repeat(gaussian_filter(col, 2.0)[:, None], nx, axis=1).astype(np.float32), device=dev)
    m_start = T(w.m_start)
    vmax = 1.01 * float((m_start[0] * torch.sqrt(1.0 + 2.0 * eps)).max())
    grid = efwi.make_grid(nz, nx, w.dz, w.dx, w.dt, nt, w.npml, w.pml_R, w.f0, vmax, eps=eps)
    iso = efwi.make_grid(nz, nx, w.dz, w.dx, w.dt, nt, w.npml, w.pml_R, w.f0, w.vp_max)
    s = w.shots[0]
    shot = efwi.Shot(s.src_iz, s.src_ix, s.ch_iz, s.ch_ix, ckpt_interval=nt)
    src = T(np.outer(s.M, w.stf))
    d_obs = efwi.model_forward(iso, shot, T(w.m_true), src)
    ws = efwi.workspace(efwi.workspace_size(efwi.WS_GRADIENT, grid, [shot]), dev)
    efwi.shot_gradient(grid, shot, m_start, src, d_obs, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g, _ = efwi.shot_gradient(grid, shot, m_start, src, d_obs, ws=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gcell = nz * nx * nt / dt / 1e9
    alg = path_bytes_2d(nz * nx, strip_cells_2d(nz, nx, w.npml), 0.0) / (nz * nx) + 32.0
    out = {"shots": 1, "ms": round(dt * 1e3, 1), "gcell_per_s": round(gcell, 3), "bytes_per_cell_step": round(alg, 1),
           "path_frac": round(alg * gcell / HBM_PEAK_GBS, 4), "finite": bool(torch.isfinite(g).all())}
    del ws, g
    torch.cuda.empty_cache()
    return out


def precision_3d_shot(efwi, inputs, torch, dev, nt=3000, nshots=8):
    """One shot of the 3D precision workload on its full 300 x 400 x 400 grid (5 m, CPML 20,
    two DAS wells along x with a channel at every interior node, 356 each and 712 in all,
    six-component moment tensor), all nt = 3000 steps with sqrt(nt) FP16 checkpoints, d_obs = 0;
    timed once after an untimed 16-step call on the same grid; the 8-shot time extrapolated
    linearly (the shots cost the same, and one shot's workspace, about 150 GB, leaves no room
    for a second in a wave). path_frac: 3D algorithmic bytes (228 B per cell-step + 84 B per
    recomputed step, CPML memory variables 48 B per strip cell, axis and pass) over the time."""
    w = inputs.precision_3d(nt=nt, nshots=1, anomalies=False)
    s = w.shots[0]
    shot = efwi.Shot(s.src_iz, s.src_ix, s.ch_iz, s.ch_ix, src_iy=s.src_iy, ch_iy=s.ch_iy, ckpt_mode=efwi.CKPT_FP16)
    m = torch.tensor(np.asarray(w.m_start, np.float32), device=dev)
    src = torch.tensor(np.asarray(np.outer(s.M, w.stf), np.float32), device=dev)
    warm = efwi.make_grid3d(w.nz, w.ny, w.nx, w.h, w.h, w.h, w.dt, 16, w.npml, w.pml_R, w.f0, w.vp_max)
    efwi.shot_gradient(warm, shot, m, src[:, :16].contiguous(),
                       torch.zeros((len(s.ch_ix), 16), dtype=torch.float32, device=dev))
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    grid = efwi.make_grid3d(w.nz, w.ny, w.nx, w.h, w.h, w.h, w.dt, nt, w.npml, w.pml_R, w.f0, w.vp_max)
    d_obs = torch.zeros((len(s.ch_ix), nt), dtype=torch.float32, device=dev)
    ws = efwi.workspace(efwi.workspace_size(efwi.WS_GRADIENT, grid, [shot]), dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g, _ = efwi.shot_gradient(grid, shot, m, src, d_obs, ws=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    cells = w.nz * w.ny * w.nx
    rf = efwi.recompute_fraction(grid, 0)
    a = ALG3
    P = w.npml
    strips = 2 * P * (w.ny * w.nx + w.nz * w.nx + w.nz * w.ny)
    alg = ((a["fwd"] + a["store"] + a["adj"] + a["img"] + a["acc"] + rf * a["fwd"]) * cells
           + a["psi"] * strips * (2.0 + rf)) / cells
    gcell = cells * nt / dt / 1e9
    out = {"grid": [w.nz, w.ny, w.nx], "nt": nt, "checkpoints": "sqrt(nt), FP16", "recompute_fraction": round(rf, 4),
           "channels": len(s.ch_ix), "workspace_GiB": round(ws.numel() / 2**30, 1), "ms": round(dt * 1e3, 1),
           "gcell_per_s": round(gcell, 3), f"extrapolated_{nshots}_shots_s": round(dt * nshots, 1),
           "bytes_per_cell_step": round(alg, 1), "path_GBs": round(alg * gcell, 1),
           "path_frac": round(alg * gcell / HBM_PEAK_GBS, 4), "finite": bool(torch.isfinite(g).all())}
    del ws, m, g
    torch.cuda.empty_cache()
    return out


def extension_ops(efwi, inputs, torch, dev, nt):
    """The sources' zones of influence (eq.(10)) and the final model S_w W m~ (eq.(9)) on the
    1000 x 3000 grid for 20 sources (median of 5 calls each; compulsory bytes: zones write b
    and the sinkhole flag, 5 B per point and source; final model reads m~, b and the flags,
    writes m); the approximate inverse pseudo-Hessian of the comparison methods for one shot
    over 200 steps (median of 3; 60 B per cell-step); the field-like DAS sampling of 1500
    channels x nt steps (10-channel gauge, strain rate, every 4th sample; median of 5); the
    cubic B-spline expansion of 40 model planes and its transpose (nodes every 50 m in x and
    every cell in z; median of 5)."""
    w = inputs.plain_2d(nshots=20, nt=nt)
    ns, nz, nx = len(w.shots), w.nz, w.nx
    grid = efwi.make_grid(nz, nx, w.dz, w.dx, w.dt, nt, w.npml, w.pml_R, w.f0, w.vp_max)
    m = torch.tensor(np.asarray(w.m_start, np.float32), device=dev)
    m_ext = m.unsqueeze(0).repeat(ns, 1, 1, 1).contiguous()
    zones = []
    for s in w.shots:
        xs = [s.src_ix] + list(s.ch_ix)
        zones.append(efwi.make_zone((s.src_iz * w.dz, 0.0, s.src_ix * w.dx),
                                    (1.0 / (20.0 ** 2), 0.0, 1.0 / (75.0 ** 2), 0.0, 0.0, 0.0),
                                    (0.0, (nz - 1) * w.dz, 0.0, 0.0, min(xs) * w.dx, max(xs) * w.dx), 200.0))
    b = torch.empty((ns, nz, nx), dtype=torch.float32, device=dev)
    sink = torch.empty((ns, nz, nx), dtype=torch.uint8, device=dev)
    m_out = torch.empty((3, nz, nx), dtype=torch.float32, device=dev)

    def med_ms(fn, reps=5):
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        return sorted(times)[reps // 2]

    zms = med_ms(lambda: efwi.zoi_weights(grid, zones, 2.0, 0.9, b=b, sink=sink))
    fms = med_ms(lambda: efwi.final_model(grid, m_ext, b, sink, m_out=m_out))
    zbytes, fbytes = 5 * nz * nx * ns, (17 * ns + 12) * nz * nx
    ph_steps = 200
    ph_grid = efwi.make_grid(nz, nx, w.dz, w.dx, w.dt, ph_steps, w.npml, w.pml_R, w.f0, w.vp_max)
    s0 = w.shots[0]
    ph_shot = [efwi.Shot(s0.src_iz, s0.src_ix, s0.ch_iz, s0.ch_ix)]
    ph_ws = efwi.workspace(efwi.workspace_size(efwi.WS_GRADIENT, ph_grid, ph_shot), dev)
    h = torch.empty((nz, nx), dtype=torch.float32, device=dev)
    pinv = torch.empty((nz, nx), dtype=torch.float32, device=dev)
    ph_src = torch.tensor(np.outer(s0.M, w.stf[:ph_steps])[None].astype(np.float32), device=dev)
    pms = med_ms(lambda: efwi.pseudo_hessian(ph_grid, ph_shot, m_ext[:1], ph_src, 0.01, h=h, p=pinv, ws=ph_ws), 3)
    pbytes = (60 * ph_steps + 12) * nz * nx
    fshot = efwi.Shot(s0.src_iz, s0.src_ix, s0.ch_iz, s0.ch_ix, gauge=10, decim=4, rate=True)
    e = torch.randn((len(s0.ch_ix), nt), dtype=torch.float32, device=dev)
    fout = torch.empty(fshot.data_shape(nt), dtype=torch.float32, device=dev)
    dms = med_ms(lambda: efwi.das_field(grid, fshot, e, out=fout))
    dbytes = 4 * (e.numel() + fout.numel())
    dzn, dxn = 1, max(1, int(round(50.0 / w.dx)))
    coef = torch.randn((ns, 2, efwi.bspline_nodes(nz, dzn), efwi.bspline_nodes(nx, dxn)), dtype=torch.float32,
                       device=dev)
    planes = torch.empty((ns, 2, nz, nx), dtype=torch.float32, device=dev)
    cbar = torch.empty_like(coef)
    ems = med_ms(lambda: efwi.bspline_expand(coef, nz, nx, dzn, dxn, out=planes))
    ams = med_ms(lambda: efwi.bspline_adjoint(planes, dzn, dxn, out=cbar))
    bbytes = 4 * (planes.numel() + coef.numel())

    def rate(nbytes, ms):
        return {"ms": round(ms, 3), "bytes": nbytes, "GBs": round(nbytes / ms / 1e6, 1),
                "frac": round(nbytes / ms / 1e6 / HBM_PEAK_GBS, 4)}

    out = {"zoi_weights": {"sources": ns, "sink_points": int(sink.sum().item()), **rate(zbytes, zms)},
           "final_model": {"components": ns, **rate(fbytes, fms)},
           "pseudo_hessian": {"shots": 1, "steps": ph_steps, "gcell_per_s": round(nz * nx * ph_steps / pms / 1e6, 2),
                              **rate(pbytes, pms)},
           "das_field": {"channels": int(e.shape[0]), "steps": int(e.shape[1]), "gauge": 10, "decim": 4,
                         "rate": True, **rate(dbytes, dms)},
           "bspline_expand": {"planes": 2 * ns, "nodes": [int(coef.shape[2]), int(coef.shape[3])], **rate(bbytes, ems)},
           "bspline_adjoint": {"planes": 2 * ns, **rate(bbytes, ams)}}
    del b, sink, m_out, h, pinv, ph_ws, e, fout, coef, planes, cbar, m_ext, m
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------------------
# The headline: the batched workload.
# ---------------------------------------------------------------------------------------
class Batched:
    """The batched workload resident in HBM: 64 windows, their sources, observed data (the
    true model's), the 64-component extended model (start model times 1% smooth noise per
    shot), hard sinkholes for the regularizer."""

    def __init__(self, efwi, inputs, torch, dev, nt, nshots=64, windows=None):
        w = inputs.batched_2d(nshots=nshots, nt=nt)
        if windows:   # the first `windows` of the 64 (profiling runs): the full run's first waves
            w.shots = w.shots[:windows]
        self.w, self.nt, self.dev = w, nt, dev
        T = lambda a: torch.tensor(np.asarray(a, np.float32), device=dev)
        self.grid = efwi.make_grid(w.nz, w.nx, w.dz, w.dx, w.dt, nt, w.npml, w.pml_R, w.f0, w.vp_max)
        self.shots = [efwi.Shot(s.src_iz, s.src_ix, s.ch_iz, s.ch_ix, z0=s.z0, x0=s.x0, wz=s.wz, wx=s.wx)
                      for s in w.shots]
        ns, nz, nx = len(self.shots), w.nz, w.nx
        self.ns = ns
        self.src = T(np.stack([np.outer(s.M, w.stf) for s in w.shots]))
        m_true = T(w.m_true)
        fws = efwi.workspace(max(efwi.workspace_size(efwi.WS_FORWARD, self.grid, [s]) for s in self.shots), dev)
        obs = [efwi.model_forward(self.grid, self.shots[k], m_true, self.src[k], ws=fws) for k in range(ns)]
        self.d_obs = torch.cat(obs)
        self.obs = list(torch.split(self.d_obs, [s.nch for s in self.shots]))
        del fws, m_true, obs
        m_start = T(w.m_start)
        noise = T(np.stack([inputs.smooth_random_field((nz, nx), 20.0, 177 + k, 0.01) for k in range(3)]))
        self.m_ext = torch.stack([m_start * (1.0 + torch.roll(noise, shifts=(0, 41 * k), dims=(1, 2)))
                                  for k in range(ns)])
        del noise, m_start
        b_np, sink_np = inputs.hard_sinkholes(ns, nz, nx, [s.src_iz for s in w.shots], [s.src_ix for s in w.shots])
        self.b, self.sink = T(b_np), torch.tensor(sink_np, device=dev)
        del b_np, sink_np
        self.g_ext = torch.empty_like(self.m_ext)
        self.phi = torch.empty((ns,), dtype=torch.float64, device=dev)
        self.phi_reg = torch.empty((), dtype=torch.float64, device=dev)
        self.rws = efwi.workspace(efwi.workspace_size(efwi.WS_REGULARIZER, self.grid, []), dev)
        self.cells = [s.wz * s.wx for s in w.shots]
        self.strips = [strip_cells_2d(s.wz, s.wx, w.npml) for s in w.shots]
        self.largest = int(np.argmax(self.cells))


def main():  # noqa: C901
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nt", type=int, default=4000, help="time steps of the 2D workloads (profiling runs use fewer)")
    ap.add_argument("--sample-every", type=int, default=16, help="time every k-th launch of each kernel")
    ap.add_argument("--interval", type=int, default=-1,
                    help="checkpoint interval of the headline (-1: largest that fits, 0: sqrt(nt))")
    ap.add_argument("--mem-fraction", type=float, default=0.9,
                    help="share of the free device memory the headline's workspace may take")
    ap.add_argument("--wave-cache-mib", type=int, default=0,
                    help="per-step state bound of a wave in MiB (0: the library's default, -1: the workspace alone)")
    ap.add_argument("--lanes", type=int, default=0, help="lanes of the batched calls (0: the library's default)")
    ap.add_argument("--nt3d", type=int, default=3000, help="time steps of the 3D shot (profiling runs use fewer)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="time the headline only (profiling runs)")
    for f in ("sequential", "sqrt", "compressed", "plain", "autograd", "vti", "3d", "extension-ops", "autotune"):
        ap.add_argument(f"--no-{f}", action="store_true")
    ap.add_argument("--tile-rows", default="",
                    help="FWD,ADJ: fix the step kernels' tile rows instead of autotuning them (counter runs, "
                         "whose serialised launches would distort the autotuner's timings)")
    ap.add_argument("--windows", type=int, default=0,
                    help="time the headline over the first K of its 64 windows only (counter runs: the launches "
                         "of the full run's first waves, without its hundreds of thousands of other launches)")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="first run a plain device copy of this many MiB (scales HBM byte counters)")
    ap.add_argument("--cpu-worker", type=int, default=0, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker:
        cs, sec, shape = _cpu_sample(args.cpu_worker)
        print(json.dumps({"cell_steps": cs, "seconds": sec, "window": shape}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: --gpus must be 1. On several GPUs the shots would be sharded, one "
                                   "process per GPU, with the regularizer's three per-point sums all-reduced; that "
                                   "path is not built"}))
        sys.exit(2)

    cpu = None
    if not args.no_cpu_baseline:   # before this process touches the GPU: the workers are children
        cpu = cpu_baseline()
        log(f"cpu baseline done: {cpu}")

    import torch
    from paper_2305_14130_amd import efwi, inputs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy_mb > 0:
        x = torch.ones(args.calibrate_copy_mb * (1 << 18), dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    nt = args.nt
    if args.lanes:
        efwi.set_wave_lanes(args.lanes)
    if args.wave_cache_mib:
        efwi.set_wave_cache_bytes(args.wave_cache_mib << 20 if args.wave_cache_mib > 0 else -1)
    B = Batched(efwi, inputs, torch, dev, nt, windows=args.windows)
    grid, ns = B.grid, B.ns
    torch.cuda.synchronize()
    log(f"set-up done: {ns} windows, {sum(B.cells) / 1e6:.2f} M cells")
    tune_ms = {}
    big = B.largest
    if args.tile_rows:
        efwi.set_tile_rows(*(int(x) for x in args.tile_rows.split(",")))
    tiles = efwi.get_tile_rows() if args.no_autotune or args.tile_rows else \
        efwi.autotune(grid, B.shots[big], B.m_ext[big], B.src[big], steps=64, times=tune_ms)
    log(f"tile rows (forward, transposed): {tiles}; sweep ms by rows: {tune_ms}")
    budget = int(args.mem_fraction * torch.cuda.mem_get_info(dev)[0])
    L = efwi.plan_interval(grid, B.shots[big], budget) if args.interval < 0 else args.interval
    shots = [dataclasses.replace(s, ckpt_interval=L, _keep=[]) for s in B.shots]
    need = efwi.workspace_size(efwi.WS_BATCH, grid, shots)
    ws = efwi.workspace(min(need, budget), dev)
    waves = efwi.batch_waves(grid, shots, ws.numel())
    torch.cuda.synchronize()
    log(f"checkpoint interval {L}, workspace {ws.numel() / 2**30:.1f} GiB, {len(waves)} waves")

    def batched_step(shot_list, wsp):
        efwi.batch_gradient(grid, shot_list, B.m_ext, B.src, B.d_obs, g_ext=B.g_ext, phi=B.phi, ws=wsp)
        efwi.extension_regularizer(grid, B.m_ext, B.b, B.sink, 1.0, B.g_ext, phi=B.phi_reg, ws=B.rws)

    for _ in range(args.warmup):
        batched_step(shots, ws)
    torch.cuda.synchronize()
    log("warm-up done")
    efwi.timing_reset()
    efwi.timing_enable(args.sample_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        batched_step(shots, ws)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timing = efwi.timing_query()
    efwi.timing_enable(0)
    assert bool(torch.isfinite(B.phi).all()) and bool(torch.isfinite(B.phi_reg))
    g_batched = B.g_ext.clone()
    log(f"timed steps done: {elapsed:.2f} s")
    del ws
    torch.cuda.empty_cache()

    cells = sum(B.cells)
    strips = sum(B.strips)
    rf = efwi.recompute_fraction(grid, L)
    value = cells * nt * args.steps / elapsed / 1e9
    step_s = elapsed / args.steps
    pb = path_bytes_2d(cells, strips, rf) / cells

    forms = {}
    run_forms = not args.no_forms
    if run_forms and not args.no_sequential:
        # the same 64 windows as 64 sequential shot gradients (one shot's workspace, the
        # largest window's), then the regularizer: shots/s plain vs batched
        sws = efwi.workspace(efwi.workspace_size(efwi.WS_GRADIENT, grid, [shots[big]]), dev)
        B.g_ext.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for k in range(ns):
            efwi.shot_gradient(grid, shots[k], B.m_ext[k], B.src[k], B.obs[k], g=B.g_ext[k], phi=B.phi[k], ws=sws)
        efwi.extension_regularizer(grid, B.m_ext, B.b, B.sink, 1.0, B.g_ext, phi=B.phi_reg, ws=B.rws)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        forms["plain_sequential_64"] = {"shots_per_s": round(ns / dt, 4),
                                        "gcell_per_s": round(cells * nt / dt / 1e9, 4),
                                        "ms_per_step": round(dt * 1e3, 1),
                                        "identical_to_batched": bool(torch.equal(B.g_ext, g_batched)),
                                        "path_frac": round(pb * cells * nt / dt / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"sequential form done: {forms['plain_sequential_64']}")
        del sws
        torch.cuda.empty_cache()

    def batched_form(name, mode, ref=None):
        sq = [dataclasses.replace(s, ckpt_interval=0, ckpt_mode=mode, _keep=[]) for s in shots]
        need_ = efwi.workspace_size(efwi.WS_BATCH, grid, sq)
        wsp = efwi.workspace(min(need_, int(args.mem_fraction * torch.cuda.mem_get_info(dev)[0])), dev)
        B.g_ext.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        batched_step(sq, wsp)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        rf_ = efwi.recompute_fraction(grid, 0)
        pb_ = path_bytes_2d(cells, strips, rf_) / cells
        gcell = cells * nt / dt / 1e9
        f = {"shots_per_s": round(ns / dt, 4), "gcell_per_s": round(gcell, 4), "ms_per_step": round(dt * 1e3, 1),
             "ckpt_interval": int(np.ceil(np.sqrt(nt))), "recompute_fraction": round(rf_, 4),
             "waves": len(efwi.batch_waves(grid, sq, wsp.numel())), "workspace_GiB": round(wsp.numel() / 2**30, 2),
             "bytes_per_cell_step": round(pb_, 1), "path_frac": round(pb_ * gcell / HBM_PEAK_GBS, 4)}
        if ref is None:
            f["identical_to_whole_history"] = bool(torch.equal(B.g_ext, g_batched))
        else:   # the 16-bit codes' error against the FP32 checkpoints, per parameter, worst of the first 4 shots
            f["grad_rel_l2_vs_fp32"] = [
                max(float(torch.linalg.vector_norm(B.g_ext[q, c].double() - ref[q, c].double()) /
                          torch.linalg.vector_norm(ref[q, c].double())) for q in range(4)) for c in range(3)]
        forms[name] = f
        log(f"{name} form done: {f}")
        del wsp
        torch.cuda.empty_cache()

    if run_forms and not args.no_sqrt:
        batched_form("batched_sqrt_nt", efwi.CKPT_FP32)
        # the same with waves sized by the workspace alone (the Infinity-Cache bound on a
        # wave's per-step state lifted): one launch per half step over many more shots
        efwi.set_wave_cache_bytes(-1)
        try:
            batched_form("batched_sqrt_nt_workspace_waves", efwi.CKPT_FP32)
        finally:
            efwi.set_wave_cache_bytes(0)
        if not args.no_compressed:
            ref = B.g_ext[:4].clone()
            batched_form("batched_sqrt_nt_fp16", efwi.CKPT_FP16, ref)
            batched_form("batched_sqrt_nt_bf16", efwi.CKPT_BF16, ref)
            del ref

    del B.m_ext, B.g_ext, B.b, B.sink, B.d_obs, B.obs, B.src, g_batched
    torch.cuda.empty_cache()
    if run_forms and not args.no_plain:
        forms["plain_1000x3000_20"] = plain_1000x3000_form(efwi, inputs, torch, dev, nt)
        log(f"plain 1000x3000 form done: {forms['plain_1000x3000_20']}")
    if run_forms and not args.no_autograd:
        forms["autograd_1200x4000"] = autograd_form(efwi, inputs, torch, dev, 2 * nt)
        log(f"autograd form done: {forms['autograd_1200x4000']}")
    if run_forms and not args.no_vti:
        forms["vti_1shot"] = vti_shot_form(efwi, inputs, torch, dev, nt)
        log(f"VTI form done: {forms['vti_1shot']}")
    if run_forms and not args.no_3d:
        forms["precision_3d_shot"] = precision_3d_shot(efwi, inputs, torch, dev, nt=args.nt3d)
        log(f"3D shot done: {forms['precision_3d_shot']}")
    ext_ops = None
    if run_forms and not args.no_extension_ops:
        ext_ops = extension_ops(efwi, inputs, torch, dev, nt)
        log(f"extension operators done: {ext_ops}")

    # ---- roofline of the dominant kernel ----
    kern = {}
    for name, (launches, timed, ms) in timing.items():
        if launches:
            kern[name] = {"launches": launches, "timed": timed, "mean_us": round(ms * 1e3, 2) if timed else None}
    total_ms = sum(k["launches"] * k["mean_us"] / 1e3 for k in kern.values() if k["mean_us"])
    for k in kern.values():
        k["share"] = round(k["launches"] * k["mean_us"] / 1e3 / total_ms, 4) if k["mean_us"] else None
    dominant = max((n for n in ("adj_step", "fwd_step") if n in kern and kern[n]["share"]),
                   key=lambda n: kern[n]["share"])
    # algorithmic bytes of the dominant kernel over one step's launches, per launch: each
    # wave runs nt launches of the transposed step over its shots' tiles (and nt (1 + rf)
    # forward ones)
    a = ALG2
    if dominant == "adj_step":
        per_step = (a["adj"] + a["img"] + a["acc"]) * cells + a["psi"] * strips
        launches_per_step = len(waves) * nt
    else:
        per_step = (a["fwd"] * (1 + rf) + a["store"]) * cells + a["psi"] * strips * (1 + rf)
        launches_per_step = len(waves) * nt * (1 + rf)
    bytes_launch = per_step * nt / launches_per_step
    achieved = bytes_launch / (kern[dominant]["mean_us"] * 1e-6) / 1e9
    rows = tiles[1] if dominant == "adj_step" else tiles[0]
    per_cell = MEASURED_TRAFFIC_PER_CELL.get((dominant, rows)) if rf == 0.0 else None
    traffic = int(per_cell * cells / len(waves)) if per_cell and dominant == "adj_step" else None
    out = {
        "metric": "Gcell-updates/s fwd+adj+grad (and % HBM roofline); shots/s batched vs plain",
        "value": round(value, 4),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched 2D elastic: {ns} MT shots on uneven windows (nz_s ~ U[400,1000], "
                               f"nx_s ~ U[800,3000], {cells / ns / 1e6:.2f} M cells on average) of the 1000x3000 "
                               f"dx=2.5m shale model, nt={nt}, DAS e_xx channels in each window, CPML {B.w.npml}, "
                               f"per-shot m_s gradients + extension regularizer (hard sinkholes), FP32, "
                               f"checkpoint interval {L}",
                   "shots": ns, "nt": nt, "cells": int(cells), "ckpt_interval": L,
                   "recompute_fraction": round(rf, 4), "waves": len(waves), "lanes_setting": efwi.get_wave_lanes(),
                   "form": "batched (efwi_batch_gradient, shots packed into waves largest first)",
                   "wave_cache_MiB": efwi.get_wave_cache_bytes() / 2**20 if efwi.get_wave_cache_bytes() < 2**63 else None,
                   "tile_rows": {"forward": tiles[0], "transposed": tiles[1],
                                 "autotune_ms": {str(k): [round(x, 3) for x in v] for k, v in tune_ms.items()}}},
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_basis": ("HBM bytes per launch: rocprofv3 FETCH_SIZE x 2 + WRITE_SIZE (KiB, "
                                       "copy-calibrated) per cell of this kernel on the first 3 windows, "
                                       f"{per_cell} B, times the cells of a launch here") if traffic else None,
                     "bytes_per_launch": int(bytes_launch), "mean_launch_us": kern[dominant]["mean_us"],
                     "bytes_model": "92 B per cell (adjoint step 52, imaging 16, accumulators 24) + 32 B per CPML "
                                    "strip cell, averaged over the launches of the waves"},
        "path": {"bytes_per_cell_step": round(pb, 1), "achieved_GBs": round(pb * cells * nt / step_s / 1e9, 1),
                 "frac": round(pb * cells * nt / step_s / 1e9 / HBM_PEAK_GBS, 4),
                 "design_bytes_per_cell_step": round(design_bytes_2d(rf), 1)},
        "shots_per_s": {"batched": round(ns / step_s, 4),
                        **{k: v["shots_per_s"] for k, v in forms.items() if "shots_per_s" in v}},
        "forms": forms,
        "extension_ops": ext_ops,
        "kernels": kern,
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
