"""3D GPU (HIP, FP32) vs FP64 oracle parity through the C ABI.

A crop of the 3D precision workload (shale with a 3-cell reservoir, six-component
moment-tensor shots in the layer, two horizontal DAS wells): 36 x 40 x 72 cells at 5 m with
an 8-cell CPML, so the 64 x 16 tiles are ragged in x and y and several tiles touch the strips.
Same bars as 2D: data 1e-5, gradient and misfit 1e-5 * max(1, kappa).
"""
import numpy as np
import pytest
import torch

from oracle import elastic3d as E3
from paper_2305_14130_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-5


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def r32(x):
    return float(np.float32(x))


def T(a):
    return torch.tensor(np.asarray(a, np.float32), device="cuda")


@pytest.fixture(scope="module")
def case():
    w = inputs.precision_3d(nz=36, ny=40, nx=72, nt=200, nshots=2, nch_per_well=20, npml=8)
    c = type("C", (), {})()
    c.w = w
    c.sh = w.shots[0]
    c.g_o = E3.Grid3D(nz=w.nz, ny=w.ny, nx=w.nx, dz=r32(w.h), dy=r32(w.h), dx=r32(w.h), dt=r32(w.dt), nt=w.nt,
                      npml=w.npml, pml_R=r32(w.pml_R), pml_f0=r32(w.f0), vp_max=r32(w.vp_max))
    c.m = f32(w.m_start)
    c.mt = f32(w.m_true * np.array([1.1, 1.05, 1.0])[:, None, None, None])
    c.src = f32(np.outer(c.sh.M, w.stf))
    c.pos = (c.sh.src_iz, c.sh.src_iy, c.sh.src_ix)
    c.ch = (c.sh.ch_iz, c.sh.ch_iy, c.sh.ch_ix)
    c.d_obs = f32(E3.model_forward(c.g_o, c.mt, c.pos, c.src, c.ch))
    c.g_ref, c.phi_o, c.d_o = E3.shot_gradient(c.g_o, c.m, c.pos, c.src, c.ch, c.d_obs)
    c.kappa = max(1.0, float(np.linalg.norm(c.d_o) / np.linalg.norm(c.d_o - c.d_obs)))
    return c


def _grid(efwi, w):
    return efwi.make_grid3d(w.nz, w.ny, w.nx, w.h, w.h, w.h, w.dt, w.nt, w.npml, w.pml_R, w.f0, w.vp_max)


def _shot(efwi, sh, **kw):
    return efwi.Shot(sh.src_iz, sh.src_ix, sh.ch_iz, sh.ch_ix, src_iy=sh.src_iy, ch_iy=sh.ch_iy, **kw)


def test_forward_data_3d(gpu_lib, case):
    efwi = gpu_lib
    d = efwi.model_forward(_grid(efwi, case.w), _shot(efwi, case.sh), T(case.m), T(case.src))
    torch.cuda.synchronize()
    assert rel(d.cpu().numpy(), case.d_o) <= TOL


@pytest.mark.parametrize("interval", [0, 37, 10**6])
def test_gradient_3d(gpu_lib, case, interval):
    efwi = gpu_lib
    g, phi = efwi.shot_gradient(_grid(efwi, case.w), _shot(efwi, case.sh, ckpt_interval=interval), T(case.m),
                                T(case.src), T(case.d_obs))
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    bar = TOL * case.kappa
    for k in range(3):
        e = rel(g[k], case.g_ref[k])
        assert e <= bar, (interval, k, e, case.kappa)
    assert abs(phi.item() - case.phi_o) / case.phi_o <= 2 * bar


def test_adjoint_and_dot_product_3d(gpu_lib, case):
    efwi = gpu_lib
    w = case.w
    g_o = E3.Grid3D(**{**case.g_o.__dict__, "nt": 90})
    grid = efwi.make_grid3d(w.nz, w.ny, w.nx, w.h, w.h, w.h, w.dt, 90, w.npml, w.pml_R, w.f0, w.vp_max)
    rng = np.random.default_rng(3)
    f = f32(rng.standard_normal((6, 90)))
    r = f32(rng.standard_normal((len(case.sh.ch_ix), 90)))
    fb_o = E3.model_adjoint(g_o, case.m, case.pos, case.ch, r)
    shot = _shot(efwi, case.sh)
    fb = efwi.model_adjoint(grid, shot, T(case.m), T(r)).cpu().numpy()
    assert fb.shape == (6, 90)
    assert rel(fb, fb_o) <= TOL
    Lf = efwi.model_forward(grid, shot, T(case.m), T(f)).cpu().numpy().astype(np.float64)
    a, b = np.sum(Lf * r), np.sum(f * fb.astype(np.float64))
    assert abs(a - b) / abs(a) <= 1e-5


def test_fp16_checkpoints_3d(gpu_lib, case):
    """Stated bound of the FP16-compressed checkpoints against the exact gradient."""
    efwi = gpu_lib
    g, _ = efwi.shot_gradient(_grid(efwi, case.w), _shot(efwi, case.sh, ckpt_interval=20, ckpt_mode=efwi.CKPT_FP16),
                              T(case.m), T(case.src), T(case.d_obs))
    g = g.cpu().numpy()
    for k in range(3):
        assert rel(g[k], case.g_ref[k]) <= 1e-3


def test_batch_3d_equals_per_shot(gpu_lib, case):
    efwi = gpu_lib
    w = case.w
    grid = _grid(efwi, w)
    shots = [_shot(efwi, s, ckpt_interval=25) for s in w.shots]
    src = T(np.stack([np.outer(s.M, w.stf) for s in w.shots]))
    m_ext = T(np.stack([case.m, case.m * 1.01]))
    obs = [efwi.model_forward(grid, shots[k], T(case.mt), src[k]) for k in range(2)]
    g2, p2 = efwi.batch_gradient(grid, shots, m_ext, src, torch.cat(obs))
    for k in range(2):
        g1, p1 = efwi.shot_gradient(grid, shots[k], m_ext[k], src[k], obs[k])
        assert torch.equal(g1, g2[k]) and p1.item() == p2[k].item()
