"""Throughput of the source-extended elastic FWI hot path on one MI355X.

One step = one pass of the whole hot path over the plain per-shot workload: for each of the
20 shots of the 1000 x 3000 (dx = 2.5 m), nt = 4000 shale model, a full shot gradient
(forward sweep with DAS recording, FP64 misfit, reverse sweep with transposed
stress/velocity steps, imaging condition, chain rule into the shot's own component m_s of
the extended model), then the consistency-regularizer value and gradient over the
20-component extended model.

The forward history for the imaging condition is kept with the largest checkpoint interval
whose workspace fits in the free HBM (one shot's whole history, 224 GiB, fits in the 288 GB
of an MI355X, so nothing is recomputed); the sqrt(nt)-checkpoint form (recomputing all but
the last segment) and the batched form (shots advanced together, one launch per half step
over a wave's tiles, in waves whose per-step state fits the Infinity Cache) are timed once
each and must give the identical gradient; the FP16- and BF16-checkpoint forms are timed once
each with their gradient's relative L2 distance from the FP32 one, and the batched form on
64 uneven windows (nz_s ~ U[400,1000], nx_s ~ U[800,3000]) is timed once.

Metric: Gcell-updates/s = shots * nz * nx * nt / wall time (fwd + adj + grad), inputs
resident in HBM before the timed region. The JSON line also carries:
* roofline: the dominant kernel's algorithmic bytes per launch over its mean launch time
  (HIP events around sampled launches on the library's stream), against 8 TB/s, and the
  HBM traffic per launch that rocprofv3's counters measured for that kernel and tile shape
  on this grid (null when no such measurement applies);
* cpu_baseline: the FP64 NumPy oracle on a bounded sample (one shot, full grid, a few
  time steps), in the same unit;
* path: the whole step's algorithmic bytes (168 B per cell-step plus 52 B per recomputed
  cell-step) over the step time; each checkpointed form carries the same as path_frac.
* forms.vti_1shot: one shot of the workload in a VTI medium (Thomsen eps, delta = eps / 2),
  whole history, timed once, with its path_frac.
* forms.precision_3d_sample: one shot of the 3D precision workload (300 x 400 x 400) for
  200 of its 3000 steps with sqrt(nt) FP16 checkpoints, timed once, with its path_frac.
* extension_ops: the zones of influence (eq.(10)) of the 20 sources and the final model
  S_w W m~ (eq.(9)) on the full grid (once per inversion, not part of the step), and the
  approximate inverse pseudo-Hessian of the comparison methods (one shot, 200 steps), each
  with its time and compulsory-bytes rate.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Compulsory bytes per cell of each kernel launch (FP32; each array read or written once;
# lambda, mu, rho are the staged parameters, lambda + 2 mu, mu_xz and the buoyancies are
# derived from them in the kernels, so neighbours' values come from the caches):
#   fwd_step     fused forward step: read sxx szz sxz vx vz lambda mu rho,
#                write sxx szz sxz vx vz (state double-buffered)                52 B
#                + store the 5 imaging quantities of the step                  +20 B
#   adj_step     fused transposed step: read t_bar (3), u_bar (2), lambda mu rho,
#                the 5 stored quantities, 3 imaging sums; write t_bar, u_bar (5)
#                and the 3 sums (adjoint fields double-buffered)                 96 B
# (u_bar = b v_bar and t_bar = C sigma_bar are the scaled adjoint variables; the imaging
# sums are gathered at the normal node.)
KERNEL_BYTES = {"fwd_step": (52, 72), "adj_step": (96, 96)}
# HBM traffic per launch measured with rocprofv3 on one 1000 x 3000 shot, per tile shape
# (rows): FETCH_SIZE and WRITE_SIZE in KiB, scaled by 2.00 and 1.00 (the factors a 256 MiB
# device copy needs); see profiles/plain2d_1000x3000_hbm_counters.md. Valid for these
# kernels on this grid only.
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0
MEASURED_TRAFFIC = {
    "adj_step": {"cells": 3_000_000, "kib": {8: (108335.4, 99086.1), 12: (109512.9, 99026.9),
                                             16: (110407.7, 98984.8)}},
    "fwd_step": {"cells": 3_000_000, "kib": {8: (54604.5, 122430.2), 12: (55683.2, 122443.6),
                                             16: (56538.1, 122455.1)}},
}


def measured_traffic(name, cells, rows):
    """Measured HBM bytes per launch of kernel `name` at `rows` tile rows, or None."""
    mt = MEASURED_TRAFFIC.get(name)
    if not mt or mt["cells"] != cells or rows not in mt["kib"]:
        return None
    fetch, write = mt["kib"][rows]
    return int((fetch * FETCH_SCALE + write * WRITE_SCALE) * 1024)


def path_bytes_per_cell_step(recompute_fraction):
    """Whole-path algorithmic bytes per cell-step: every step runs forward once with storing
    (fwd_step with store) and backward once (adj_step); each recomputed
    step adds a forward step without storing in the first sweep."""
    fwd_plain, fwd_store = KERNEL_BYTES["fwd_step"]
    adj = KERNEL_BYTES["adj_step"][0]
    return fwd_store + adj + recompute_fraction * fwd_plain


def kernel_bytes_per_launch(name, cells, nt, L):
    """Mean compulsory bytes per launch: every step is stored once for the imaging condition
    (the last segment during the first sweep, the others during recomputation), and the
    first sweep's other steps run without storing."""
    plain, store = KERNEL_BYTES[name]
    if name.startswith("adj"):
        return plain * cells
    nseg = (nt + L - 1) // L
    nostore = (nseg - 1) * L
    return (nostore * plain + nt * store) / (nostore + nt) * cells


def cpu_baseline(w, target_s=12.0):
    """FP64 oracle on one shot of the same grid, truncated in time (fwd + adj + grad): 8 steps
    first, then a run sized to take about `target_s` seconds (at most 64 steps)."""
    from oracle import elastic2d as E
    sh = w.shots[0]

    def run(steps):
        g = E.Grid2D(nz=w.nz, nx=w.nx, dz=w.dz, dx=w.dx, dt=w.dt, nt=steps, npml=w.npml, pml_R=w.pml_R,
                     pml_f0=w.f0, vp_max=w.vp_max)
        src = np.outer(sh.M, w.stf[:steps])
        t0 = time.perf_counter()
        E.shot_gradient(g, w.m_start, sh.src_iz, sh.src_ix, src, sh.ch_iz, sh.ch_ix, np.zeros((len(sh.ch_iz), steps)))
        return time.perf_counter() - t0

    steps = 8
    dt = run(steps)
    if dt < 0.5 * target_s:
        steps = int(min(64, max(8, round(steps * target_s / dt))))
        dt = run(steps)
    return {"value": w.nz * w.nx * steps / dt / 1e9, "unit": "Gcell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"1 shot, full {w.nz}x{w.nx} grid, {steps} of {w.nt} time steps, fwd+adj+grad, "
                      f"FP64 NumPy (single-threaded elementwise), {dt:.1f} s"}


def uneven_batched_form(efwi, inputs, torch, dev, grid, nt, log):
    """64 shots on uneven windows (nz_s ~ U[400,1000], nx_s ~ U[800,3000]) cut from the same
    model, each with its own component of a 64-component extended model, advanced together
    (sqrt(nt) checkpoints), plus the regularizer over the 64 components; timed once."""
    w = inputs.batched_2d(nshots=64, nt=nt)
    T = lambda a: torch.tensor(np.asarray(a, np.float32), device=dev)
    shots = [efwi.Shot(s.src_iz, s.src_ix, s.ch_iz, s.ch_ix, z0=s.z0, x0=s.x0, wz=s.wz, wx=s.wx) for s in w.shots]
    ns, nz, nx = len(shots), w.nz, w.nx
    m_start, m_true = T(w.m_start), T(w.m_true)
    src = T(np.stack([np.outer(s.M, w.stf) for s in w.shots]))
    fws = efwi.workspace(max(efwi.workspace_size(efwi.WS_FORWARD, grid, [s]) for s in shots), dev)
    d_obs = torch.cat([efwi.model_forward(grid, shots[k], m_true, src[k], ws=fws) for k in range(ns)])
    del fws, m_true
    noise = T(np.stack([inputs.smooth_random_field((nz, nx), 20.0, 177 + k, 0.01) for k in range(3)]))
    m_ext = torch.stack([m_start * (1.0 + torch.roll(noise, shifts=(0, 41 * k), dims=(1, 2))) for k in range(ns)])
    del noise
    b_np, sink_np = inputs.hard_sinkholes(ns, nz, nx, [s.src_iz for s in w.shots], [s.src_ix for s in w.shots])
    b, sink = T(b_np), torch.tensor(sink_np, device=dev)
    del b_np, sink_np
    g_ext = torch.empty_like(m_ext)
    phi = torch.empty((ns,), dtype=torch.float64, device=dev)
    phi_reg = torch.empty((), dtype=torch.float64, device=dev)
    rws = efwi.workspace(efwi.workspace_size(efwi.WS_REGULARIZER, grid, []), dev)
    need = efwi.workspace_size(efwi.WS_BATCH, grid, shots)
    torch.cuda.synchronize()
    free = torch.cuda.mem_get_info(dev)[0]
    bws = efwi.workspace(min(need, int(free * 0.9)), dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    efwi.batch_gradient(grid, shots, m_ext, src, d_obs, g_ext=g_ext, phi=phi, ws=bws)
    efwi.extension_regularizer(grid, m_ext, b, sink, 1.0, g_ext, phi=phi_reg, ws=rws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert bool(torch.isfinite(phi).all()) and bool(torch.isfinite(phi_reg))
    cells = sum(s.wz * s.wx for s in shots)
    gcell = cells * nt / dt / 1e9
    out = {"shots_per_s": round(ns / dt, 4), "gcell_per_s": round(gcell, 4),
           "path_frac": round(path_bytes_per_cell_step(efwi.recompute_fraction(grid, 0)) * gcell / HBM_PEAK_GBS, 4),
           "ms_per_step": round(dt * 1e3, 2), "waves": len(efwi.batch_waves(grid, shots, bws.numel())), "shots": ns,
           "mean_cells_per_shot": int(cells / ns)}
    log(f"uneven batched form done: {out}")
    del bws, m_ext, g_ext, b, sink, d_obs, src, m_start
    torch.cuda.empty_cache()
    return out


def extension_ops(efwi, torch, grid, w, m_ext, src, dev, ph_steps=200):
    """The sources' zones of influence (eq.(10)) and the final model S_w W m~ (eq.(9)) on the
    full grid for the bench's shots, each timed with events on the current stream (median of
    5 calls), with their compulsory bytes (zones: write b and the sinkhole flag, 5 B per
    point and source; final model: read m~, b and the flags of every source, write m).
    Also the approximate inverse pseudo-Hessian of the comparison methods for one shot over
    ph_steps time steps (median of 3 calls): per step the forward state (read and write 5
    fields), the 3 staged parameters and the autocorrelation sum (read and write) are
    compulsory, 60 B per cell; the window sum and the inverse add 12 B per cell once. And the
    field-like DAS sampling of the first shot's recorded strains (1500 channels x 4000 steps,
    10-channel gauge, strain rate, every 4th sample; median of 5): reading the strains once
    and writing the field data are compulsory. And the cubic B-spline parameterization of the
    extended model's Vp and Vs planes (2 x shots planes, nodes every 50 m in x and every cell
    in z, as in the field example; median of 5 each): the model planes written by the
    expansion and read by the transpose are compulsory (the coefficients are 20 times
    fewer)."""
    ns, nz, nx = m_ext.shape[0], w.nz, w.nx
    zones = []
    for s in w.shots:
        xs = [s.src_ix] + list(s.ch_ix)
        zones.append(efwi.make_zone((s.src_iz * w.dz, 0.0, s.src_ix * w.dx),
                                    (1.0 / (20.0 ** 2), 0.0, 1.0 / (75.0 ** 2), 0.0, 0.0, 0.0),
                                    (0.0, (nz - 1) * w.dz, 0.0, 0.0, min(xs) * w.dx, max(xs) * w.dx), 200.0))
    b = torch.empty((ns, nz, nx), dtype=torch.float32, device=dev)
    sink = torch.empty((ns, nz, nx), dtype=torch.uint8, device=dev)
    m_out = torch.empty((3, nz, nx), dtype=torch.float32, device=dev)

    def med_ms(fn):
        times = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        return sorted(times)[2]

    zms = med_ms(lambda: efwi.zoi_weights(grid, zones, 2.0, 0.9, b=b, sink=sink))
    fms = med_ms(lambda: efwi.final_model(grid, m_ext, b, sink, m_out=m_out))
    zbytes, fbytes = 5 * nz * nx * ns, (17 * ns + 12) * nz * nx
    ph_grid = efwi.make_grid(nz, nx, w.dz, w.dx, w.dt, ph_steps, w.npml, w.pml_R, w.f0, w.vp_max)
    s0 = w.shots[0]
    ph_shot = [efwi.Shot(s0.src_iz, s0.src_ix, s0.ch_iz, s0.ch_ix)]
    ph_ws = efwi.workspace(efwi.workspace_size(efwi.WS_GRADIENT, ph_grid, ph_shot), dev)
    h = torch.empty((nz, nx), dtype=torch.float32, device=dev)
    pinv = torch.empty((nz, nx), dtype=torch.float32, device=dev)
    ph_src = src[:1, :, :ph_steps].contiguous()
    ph_times = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        efwi.pseudo_hessian(ph_grid, ph_shot, m_ext[:1], ph_src, 0.01, h=h, p=pinv, ws=ph_ws)
        e1.record()
        e1.synchronize()
        ph_times.append(e0.elapsed_time(e1))
    pms = sorted(ph_times)[1]
    pbytes = (60 * ph_steps + 12) * nz * nx
    fshot = efwi.Shot(s0.src_iz, s0.src_ix, s0.ch_iz, s0.ch_ix, gauge=10, decim=4, rate=True)
    e = torch.randn((len(s0.ch_ix), w.nt), dtype=torch.float32, device=dev)
    fout = torch.empty(fshot.data_shape(w.nt), dtype=torch.float32, device=dev)
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
    out = {"zoi_weights": {"sources": ns, "ms": round(zms, 3), "bytes": zbytes,
                           "GBs": round(zbytes / zms / 1e6, 1), "frac": round(zbytes / zms / 1e6 / HBM_PEAK_GBS, 4),
                           "sink_points": int(sink.sum().item())},
           "final_model": {"components": ns, "ms": round(fms, 3), "bytes": fbytes,
                           "GBs": round(fbytes / fms / 1e6, 1), "frac": round(fbytes / fms / 1e6 / HBM_PEAK_GBS, 4)},
           "pseudo_hessian": {"shots": 1, "steps": ph_steps, "ms": round(pms, 3), "bytes": pbytes,
                              "gcell_per_s": round(nz * nx * ph_steps / pms / 1e6, 2),
                              "GBs": round(pbytes / pms / 1e6, 1), "frac": round(pbytes / pms / 1e6 / HBM_PEAK_GBS, 4)},
           "das_field": {"channels": int(e.shape[0]), "steps": int(e.shape[1]), "gauge": 10, "decim": 4, "rate": True,
                         "ms": round(dms, 3), "bytes": dbytes, "GBs": round(dbytes / dms / 1e6, 1),
                         "frac": round(dbytes / dms / 1e6 / HBM_PEAK_GBS, 4)},
           "bspline_expand": {"planes": 2 * ns, "nodes": [int(coef.shape[2]), int(coef.shape[3])],
                              "ms": round(ems, 3), "bytes": bbytes, "GBs": round(bbytes / ems / 1e6, 1),
                              "frac": round(bbytes / ems / 1e6 / HBM_PEAK_GBS, 4)},
           "bspline_adjoint": {"planes": 2 * ns, "ms": round(ams, 3), "bytes": bbytes,
                               "GBs": round(bbytes / ams / 1e6, 1), "frac": round(bbytes / ams / 1e6 / HBM_PEAK_GBS, 4)}}
    del b, sink, m_out, h, pinv, ph_ws, e, fout, coef, planes, cbar
    return out


def vti_shot_form(efwi, inputs, torch, dev, w, m_start, src, d_obs_0):
    """One shot of the plain workload (1000 x 3000, nt = 4000, whole history) in a VTI medium
    (Thomsen eps 0.1 above the reservoir, 0.6 in it and 0.3 below, smoothed; delta = eps / 2),
    observed data those of the isotropic medium, timed once after one untimed call.
    path_frac: 200 B per cell-step (the isotropic 168 plus c11, c13 read in both steps and two
    more imaging sums read and written) over the time, against 8 TB/s."""
    from scipy.ndimage import gaussian_filter
    nz, nx = w.nz, w.nx
    i = np.arange(nz)
    col = np.where(i < nz // 2 - 3, 0.1, np.where(i < nz // 2 + 3, 0.6, 0.3))
    eps = torch.tensor(np.repeat(gaussian_filter(col, 2.0)[:, None], nx, axis=1).astype(np.float32), device=dev)
    vmax = 1.01 * float((m_start[0] * torch.sqrt(1.0 + 2.0 * eps)).max())   # horizontal P speed bound
    grid = efwi.make_grid(nz, nx, w.dz, w.dx, w.dt, w.nt, w.npml, w.pml_R, w.f0, vmax, eps=eps)
    s = w.shots[0]
    shot = efwi.Shot(s.src_iz, s.src_ix, s.ch_iz, s.ch_ix, ckpt_interval=w.nt)
    ws = efwi.workspace(efwi.workspace_size(efwi.WS_GRADIENT, grid, [shot]), dev)
    efwi.shot_gradient(grid, shot, m_start, src[0], d_obs_0, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g, _ = efwi.shot_gradient(grid, shot, m_start, src[0], d_obs_0, ws=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gcell = nz * nx * w.nt / dt / 1e9
    out = {"shots": 1, "ms": round(dt * 1e3, 1), "gcell_per_s": round(gcell, 3), "bytes_per_cell_step": 200,
           "path_frac": round(200.0 * gcell / HBM_PEAK_GBS, 4), "finite": bool(torch.isfinite(g).all())}
    del ws, g
    return out


def precision_3d_sample(efwi, inputs, torch, dev, nt=200):
    """One shot of the 3D precision workload on its full 300 x 400 x 400 grid (5 m, CPML 20,
    two DAS wells along x with a channel at every interior node, 356 each and 712 in all,
    six-component moment tensor), nt steps of the 3000 with
    sqrt(nt) FP16 checkpoints, d_obs = 0; timed once after one untimed call. path_frac: the
    algorithmic bytes per cell-step without the CPML memory variables (forward 140 B:
    velocity 60, stress 80; recomputed step with the history 176 B; transposed step with the
    imaging sums 240 B: velocity 124, stress 116) over the time, against 8 TB/s."""
    w = inputs.precision_3d(nt=nt, nshots=1, anomalies=False)
    s = w.shots[0]
    grid = efwi.make_grid3d(w.nz, w.ny, w.nx, w.h, w.h, w.h, w.dt, nt, w.npml, w.pml_R, w.f0, w.vp_max)
    shot = efwi.Shot(s.src_iz, s.src_ix, s.ch_iz, s.ch_ix, src_iy=s.src_iy, ch_iy=s.ch_iy, ckpt_mode=efwi.CKPT_FP16)
    m = torch.tensor(np.asarray(w.m_start, np.float32), device=dev)
    src = torch.tensor(np.asarray(np.outer(s.M, w.stf), np.float32), device=dev)
    d_obs = torch.zeros((len(s.ch_ix), nt), dtype=torch.float32, device=dev)
    ws = efwi.workspace(efwi.workspace_size(efwi.WS_GRADIENT, grid, [shot]), dev)
    efwi.shot_gradient(grid, shot, m, src, d_obs, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g, _ = efwi.shot_gradient(grid, shot, m, src, d_obs, ws=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    cells = w.nz * w.ny * w.nx
    rf = efwi.recompute_fraction(grid, 0)
    bpc = 140.0 + 176.0 * rf + 240.0
    gbs = bpc * cells * nt / dt / 1e9
    out = {"grid": [w.nz, w.ny, w.nx], "nt": nt, "checkpoints": "sqrt(nt), FP16",
           "recompute_fraction": round(rf, 4),
           "ms": round(dt * 1e3, 1), "gcell_per_s": round(cells * nt / dt / 1e9, 3),
           "bytes_per_cell_step": round(bpc, 1), "path_GBs": round(gbs, 1),
           "path_frac": round(gbs / HBM_PEAK_GBS, 4), "finite": bool(torch.isfinite(g).all())}
    del ws, m, g
    torch.cuda.empty_cache()
    return out


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():  # noqa: C901
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--shots", type=int, default=20, help="shots per step (profiling runs use fewer)")
    ap.add_argument("--nt", type=int, default=4000, help="time steps (profiling runs use fewer)")
    ap.add_argument("--sample-every", type=int, default=16, help="time every k-th launch of each kernel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-form measurement")
    ap.add_argument("--no-sqrt", action="store_true", help="skip the sqrt(nt)-checkpoint form")
    ap.add_argument("--no-compressed", action="store_true", help="skip the FP16/BF16-checkpoint forms")
    ap.add_argument("--no-uneven", action="store_true", help="skip the 64-shot uneven-window batched form")
    ap.add_argument("--no-vti", action="store_true", help="skip the one-shot VTI form")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default tile shape")
    ap.add_argument("--no-extension-ops", action="store_true", help="skip timing the ZOI and final-model kernels")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D precision-workload sample")
    ap.add_argument("--interval", type=int, default=-1,
                    help="checkpoint interval of the plain form (-1: largest that fits, 0: sqrt(nt))")
    ap.add_argument("--mem-fraction", type=float, default=0.92,
                    help="share of the free device memory the plain form's workspace may take")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="first run a plain device copy of this many MiB (scales HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: --gpus must be 1 (on several GPUs the shots would be "
                                   "sharded, one process per GPU; that path is not built)"}))
        sys.exit(2)

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
    w = inputs.plain_2d(nshots=args.shots, nt=args.nt)
    ns, nz, nx, nt = len(w.shots), w.nz, w.nx, w.nt
    grid = efwi.make_grid(nz, nx, w.dz, w.dx, w.dt, nt, w.npml, w.pml_R, w.f0, w.vp_max)
    shots = [efwi.Shot(s.src_iz, s.src_ix, s.ch_iz, s.ch_ix, ckpt_interval=0) for s in w.shots]
    T = lambda a: torch.tensor(np.asarray(a, np.float32), device=dev)

    # ---- untimed set-up: inputs resident in HBM ----
    m_start, m_true = T(w.m_start), T(w.m_true)
    src = T(np.stack([np.outer(s.M, w.stf) for s in w.shots]))
    fwd_ws = efwi.workspace(efwi.workspace_size(efwi.WS_FORWARD, grid, shots[:1]), dev)
    d_obs = torch.cat([efwi.model_forward(grid, shots[k], m_true, src[k], ws=fwd_ws) for k in range(ns)])
    del fwd_ws
    noise = T(np.stack([inputs.smooth_random_field((nz, nx), 20.0, 77 + k, 0.01) for k in range(3)]))
    m_ext = torch.stack([m_start * (1.0 + torch.roll(noise, shifts=(0, 37 * k), dims=(1, 2))) for k in range(ns)])
    b_np, sink_np = inputs.hard_sinkholes(ns, nz, nx, [s.src_iz for s in w.shots], [s.src_ix for s in w.shots])
    b, sink = T(b_np), torch.tensor(sink_np, device=dev)
    del b_np, sink_np
    g_ext = torch.empty_like(m_ext)
    phi = torch.empty((ns,), dtype=torch.float64, device=dev)
    phi_reg = torch.empty((), dtype=torch.float64, device=dev)
    rws = efwi.workspace(efwi.workspace_size(efwi.WS_REGULARIZER, grid, []), dev)
    nch = [s.nch for s in shots]
    obs = list(torch.split(d_obs, nch))
    torch.cuda.synchronize()
    # Tile shape of the fused time-step kernels, picked by the library's autotuner from a
    # short timed run of the first shot (results do not depend on it).
    tune_ms = {}
    tiles = efwi.autotune(grid, shots[0], m_ext[0], src[0], steps=64, times=tune_ms) if not args.no_autotune \
        else efwi.get_tile_rows()
    log(f"tile rows (forward, transposed): {tiles}; sweep ms by rows: {tune_ms}")
    # Checkpoint interval: the largest whose workspace fits in the free HBM (whole history
    # when it fits: nothing recomputed).
    budget = int(args.mem_fraction * torch.cuda.mem_get_info(dev)[0])
    L = efwi.plan_interval(grid, shots[0], budget) if args.interval < 0 else args.interval
    shots = [dataclasses.replace(s, ckpt_interval=L, _keep=[]) for s in shots]
    ws = efwi.workspace(efwi.workspace_size(efwi.WS_GRADIENT, grid, shots[:1]), dev)
    torch.cuda.synchronize()
    log(f"set-up done: checkpoint interval {L}, workspace {ws.numel() / 2**30:.1f} GiB")

    def plain_step(shot_list, wsp):
        """Plain per-shot form: one shot gradient after the other, one shot's workspace."""
        for k in range(ns):
            efwi.shot_gradient(grid, shot_list[k], m_ext[k], src[k], obs[k], g=g_ext[k], phi=phi[k], ws=wsp)
        efwi.extension_regularizer(grid, m_ext, b, sink, 1.0, g_ext, phi=phi_reg, ws=rws)

    for _ in range(args.warmup):
        plain_step(shots, ws)
    torch.cuda.synchronize()
    log("warm-up done")
    efwi.timing_reset()
    efwi.timing_enable(args.sample_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plain_step(shots, ws)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timing = efwi.timing_query()
    efwi.timing_enable(0)
    assert bool(torch.isfinite(phi).all()) and bool(torch.isfinite(phi_reg))
    g_plain = g_ext.clone()
    log(f"timed steps done: {elapsed:.2f} s")
    del ws
    torch.cuda.empty_cache()

    forms = {}

    rf_sqrt = efwi.recompute_fraction(grid, 0)

    def timed_once(fn):
        """One timed step of a checkpointed form; path_frac: its algorithmic bytes per
        cell-step (recomputed steps included) over the step time, against 8 TB/s."""
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        dt_ = time.perf_counter() - t1
        gcell = ns * nz * nx * nt / dt_ / 1e9
        return {"shots_per_s": round(ns / dt_, 4), "gcell_per_s": round(gcell, 4),
                "ms_per_step": round(dt_ * 1e3, 2), "identical_to_plain": bool(torch.equal(g_plain, g_ext)),
                "path_frac": round(path_bytes_per_cell_step(rf_sqrt) * gcell / HBM_PEAK_GBS, 4)}

    if not args.no_sqrt:
        # sqrt(nt)-checkpoint form: every segment but the last recomputed in the reverse sweep.
        sq = [dataclasses.replace(s, ckpt_interval=0, _keep=[]) for s in shots]
        sws = efwi.workspace(efwi.workspace_size(efwi.WS_GRADIENT, grid, sq[:1]), dev)
        g_ext.zero_()
        forms["sqrt_nt_checkpoints"] = timed_once(lambda: plain_step(sq, sws))
        forms["sqrt_nt_checkpoints"]["recompute_fraction"] = round(efwi.recompute_fraction(grid, 0), 4)
        log(f"sqrt(nt) form done: {forms['sqrt_nt_checkpoints']}")
        del sws
        torch.cuda.empty_cache()

    if not args.no_compressed:
        # Compressed-checkpoint forms: sqrt(nt) checkpoints stored as 16-bit codes with one
        # FP32 scale per field and snapshot. Accuracy (untimed): the data-term gradient of
        # the first two shots against the FP32-checkpoint one (bitwise equal to the plain form).
        acc_shots = range(min(2, ns))
        sq = [dataclasses.replace(s, ckpt_interval=0, _keep=[]) for s in shots]
        sws = efwi.workspace(efwi.workspace_size(efwi.WS_GRADIENT, grid, sq[:1]), dev)
        ref = [efwi.shot_gradient(grid, sq[k], m_ext[k], src[k], obs[k], ws=sws)[0].double() for k in acc_shots]
        del sws
        torch.cuda.empty_cache()
        for name, mode in (("fp16_checkpoints", efwi.CKPT_FP16), ("bf16_checkpoints", efwi.CKPT_BF16)):
            cs = [dataclasses.replace(s, ckpt_interval=0, ckpt_mode=mode, _keep=[]) for s in shots]
            cws = efwi.workspace(efwi.workspace_size(efwi.WS_GRADIENT, grid, cs[:1]), dev)
            f = timed_once(lambda: plain_step(cs, cws))
            f.pop("identical_to_plain")
            got = [efwi.shot_gradient(grid, cs[k], m_ext[k], src[k], obs[k], ws=cws)[0].double() for k in acc_shots]
            f["grad_rel_l2_vs_fp32"] = [
                max(float(torch.linalg.vector_norm(got[q][c] - ref[q][c]) / torch.linalg.vector_norm(ref[q][c]))
                    for q in range(len(ref))) for c in range(3)]
            f["workspace_GiB"] = round(cws.numel() / 2**30, 2)
            forms[name] = f
            log(f"{name} form done: {f}")
            del cws, got
            torch.cuda.empty_cache()
        del ref

    if not args.no_batched:
        # Batched form: every shot advanced together (one launch per half step covers all
        # shots' tiles), sqrt(nt) checkpoints, in as few waves as the free memory allows.
        bshots = [dataclasses.replace(s, ckpt_interval=0, _keep=[]) for s in shots]
        need = efwi.workspace_size(efwi.WS_BATCH, grid, bshots)
        free = torch.cuda.mem_get_info(dev)[0]
        bws = efwi.workspace(min(need, int(free * 0.9)), dev)
        g_ext.zero_()

        def batched_step():
            efwi.batch_gradient(grid, bshots, m_ext, src, d_obs, g_ext=g_ext, phi=phi, ws=bws)
            efwi.extension_regularizer(grid, m_ext, b, sink, 1.0, g_ext, phi=phi_reg, ws=rws)

        forms["batched"] = timed_once(batched_step)
        forms["batched"]["waves"] = len(efwi.batch_waves(grid, bshots, bws.numel()))
        log(f"batched form done: {forms['batched']}")
        del bws
        torch.cuda.empty_cache()

    ext_ops = None
    if not args.no_extension_ops:
        ext_ops = extension_ops(efwi, torch, grid, w, m_ext, src, dev)
        log(f"extension operators done: {ext_ops}")

    if not args.no_uneven:
        forms["batched_uneven_64"] = uneven_batched_form(efwi, inputs, torch, dev, grid, nt, log)

    if not args.no_vti:
        nch0 = len(w.shots[0].ch_ix)
        forms["vti_1shot"] = vti_shot_form(efwi, inputs, torch, dev, w, m_start, src, d_obs[:nch0].contiguous())
        log(f"VTI form done: {forms['vti_1shot']}")

    if not args.no_3d:
        forms["precision_3d_sample"] = precision_3d_sample(efwi, inputs, torch, dev)
        log(f"3D sample done: {forms['precision_3d_sample']}")

    cell_steps = ns * nz * nx * nt * args.steps
    value = cell_steps / elapsed / 1e9
    rf = efwi.recompute_fraction(grid, L)
    kern = {}
    for name, (launches, timed, ms) in timing.items():
        if launches:
            kern[name] = {"launches": launches, "timed": timed,
                          "mean_us": round(ms * 1e3, 2) if timed else None, "share": None}
    total_ms = sum(k["launches"] * k["mean_us"] / 1e3 for k in kern.values() if k["mean_us"])
    for k in kern.values():
        if k["mean_us"]:
            k["share"] = round(k["launches"] * k["mean_us"] / 1e3 / total_ms, 4)
    dominant = max((n for n in kern if n in KERNEL_BYTES and kern[n]["share"]), key=lambda n: kern[n]["share"])
    bytes_launch = kernel_bytes_per_launch(dominant, nz * nx, nt, L)
    achieved = bytes_launch / (kern[dominant]["mean_us"] * 1e-6) / 1e9
    rows = tiles[1] if dominant == "adj_step" else tiles[0]
    traffic = measured_traffic(dominant, nz * nx, rows) if rf == 0.0 else None
    pb = path_bytes_per_cell_step(rf)
    out = {
        "metric": "Gcell-updates/s fwd+adj+grad (and % HBM roofline); shots/s batched vs plain",
        "value": round(value, 4),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"plain per-shot 2D elastic, {nz}x{nx} dx=2.5m, nt={nt}, {ns} MT shots, "
                               f"{len(w.shots[0].ch_ix)} DAS channels, CPML {w.npml}, FP32 history "
                               f"(checkpoint interval {L}), + extension regularizer (hard sinkholes)",
                   "nz": nz, "nx": nx, "nt": nt, "shots": ns, "ckpt_interval": L,
                   "recompute_fraction": round(rf, 4), "form": "plain per-shot",
                   "tile_rows": {"forward": tiles[0], "transposed": tiles[1],
                                 "autotune_ms": {str(k): [round(x, 3) for x in v] for k, v in tune_ms.items()}}},
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "bytes_per_launch": int(bytes_launch), "mean_launch_us": kern[dominant]["mean_us"]},
        "path": {"bytes_per_cell_step": round(pb, 1),
                 "achieved_GBs": round(pb * cell_steps / elapsed / 1e9, 1),
                 "frac": round(pb * cell_steps / elapsed / 1e9 / HBM_PEAK_GBS, 4)},
        "shots_per_s": {"plain": round(ns * args.steps / elapsed, 4),
                        **{k: v["shots_per_s"] for k, v in forms.items() if "shots_per_s" in v}},
        "forms": forms,
        "extension_ops": ext_ops,
        "kernels": kern,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
