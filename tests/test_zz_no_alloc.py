"""The allocation-free entry point (efwi_shot_gradient_noalloc) against efwi_shot_gradient
with a caller workspace, through the C ABI: two calls in a row on the library's per-GPU
scratch, the second with a smaller input (fewer steps, a smaller window), each bitwise equal
to the workspace call (same kernels, same arithmetic per node)."""
import numpy as np
import pytest
import torch

from paper_2305_14130_amd import inputs

pytestmark = pytest.mark.gpu


def T(a):
    return torch.tensor(np.asarray(a, np.float32), device="cuda")


def _inputs(efwi, nt, window=None, interval=0):
    w = inputs.parity_2d(nt=nt, blob_amp=0.3)
    sh = w.shots[0]
    grid = efwi.make_grid(w.nz, w.nx, w.dz, w.dx, w.dt, nt, w.npml, w.pml_R, w.f0, w.vp_max)
    kw = dict(ckpt_interval=interval)
    chz, chx = sh.ch_iz, sh.ch_ix
    if window is not None:
        z0, x0, wz, wx = window
        keep = (chx >= x0 + w.npml + 2) & (chx < x0 + wx - w.npml - 2)
        chz, chx = chz[keep], chx[keep]
        kw.update(z0=z0, x0=x0, wz=wz, wx=wx)
    shot = efwi.Shot(sh.src_iz, sh.src_ix, chz, chx, **kw)
    m, src = T(w.m_start), T(np.outer(sh.M, w.stf))
    d_obs = efwi.model_forward(grid, shot, T(w.m_true), src)
    return grid, shot, m, src, d_obs


def _compare(efwi, grid, shot, m, src, d_obs):
    g_ref, phi_ref = efwi.shot_gradient(grid, shot, m, src, d_obs, d_out=(d_ref := torch.empty_like(d_obs)))
    g = torch.full_like(m, float("nan"))
    phi = torch.full((), float("nan"), dtype=torch.float64, device="cuda")
    d_out = torch.full_like(d_obs, float("nan"))
    efwi.shot_gradient_noalloc(grid, shot, m, src, d_obs, g, phi, d_out=d_out)
    torch.cuda.synchronize()
    assert torch.equal(d_out, d_ref)
    assert torch.equal(g, g_ref)
    assert phi.item() == phi_ref.item() and np.isfinite(phi.item())


def test_noalloc_two_calls_second_smaller(gpu_lib):
    efwi = gpu_lib
    print("noalloc: 100x200 nt=1000 sqrt(nt) checkpoints, then a 70x130 window nt=400, interval 37", flush=True)
    _compare(efwi, *_inputs(efwi, 1000))
    _compare(efwi, *_inputs(efwi, 400, window=(15, 0, 70, 130), interval=37))


def test_noalloc_refuses_oversize(gpu_lib):
    efwi = gpu_lib
    grid, shot, m, src, d_obs = _inputs(efwi, 400, interval=10**6)    # whole history: 175 MiB
    assert efwi.workspace_size(efwi.WS_GRADIENT, grid, [shot]) > efwi.noalloc_scratch_bytes()
    g = torch.empty_like(m)
    phi = torch.empty((), dtype=torch.float64, device="cuda")
    with pytest.raises(efwi.EfwiError) as ei:
        efwi.shot_gradient_noalloc(grid, shot, m, src, d_obs, g, phi)
    assert ei.value.status == efwi.E_WORKSPACE
