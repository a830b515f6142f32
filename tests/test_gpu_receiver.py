"""GPU (HIP) vs FP64 oracle parity of the field-like DAS sampling K_r of eq.(3) (gauge-length
mean, strain rate, resampling) through the C ABI: the operator itself (efwi_das_field), the
forward data, the misfit and the gradient J^T K^T r in 2D and 3D, and the batch.

Bars: the operator on the same FP32 point strains within 2 FP32 ulps of the oracle's FP64
value (the kernel sums in FP64 and rounds once); data, gradient and misfit as for the point
strain (1e-5, 1e-5 * max(1, kappa)), which also covers the strain rate: it differences the
FP32 running strain, whose rounding (2^-24 of |e|) grows by |e| / (dt |de/dt|), a few tens
for these wavelets, to about 1e-6 of a sample.
"""
import numpy as np
import pytest
import torch

from oracle import elastic2d as E
from oracle import elastic3d as E3
from oracle import receiver as KR
from paper_2305_14130_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-5
SAMPLINGS = [(2, 4, 1), (10, 4, 1), (3, 3, 0), (1, 1, 1)]


def T(a):
    return torch.tensor(np.asarray(a, np.float32), device="cuda")


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def r32(x):
    return float(np.float32(x))


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("gauge,decim,rate", SAMPLINGS)
def test_das_field_operator(gpu_lib, gauge, decim, rate):
    efwi = gpu_lib
    nt = 203
    grid = efwi.make_grid(60, 120, 5.0, 5.0, 0.5e-3, nt, 8, 1e-3, 30.0, 4600.0)
    chx = np.arange(20, 100).astype(np.int32)
    shot = efwi.Shot(30, 60, np.full(len(chx), 31, np.int32), chx, gauge=gauge, decim=decim, rate=bool(rate))
    e = f32(np.cumsum(np.random.default_rng(gauge + 7 * decim).standard_normal((len(chx), nt)), axis=1) * 1e-9)
    out = efwi.das_field(grid, shot, T(e)).cpu().numpy()
    ref = KR.field_data(e, gauge, decim, rate, r32(0.5e-3))
    assert out.shape == ref.shape == shot.data_shape(nt)
    ref32 = np.asarray(ref, np.float32)
    assert np.all(np.abs(out - ref32) <= 2 * np.spacing(np.abs(ref32)))


class Case2D:
    def __init__(self, nt=600):
        w = inputs.parity_2d(nt=nt)
        self.w, self.sh = w, w.shots[0]
        self.g_o = E.Grid2D(nz=w.nz, nx=w.nx, dz=r32(w.dz), dx=r32(w.dx), dt=r32(w.dt), nt=nt, npml=20,
                            pml_R=r32(w.pml_R), pml_f0=r32(w.f0), vp_max=r32(w.vp_max))
        self.m = f32(w.m_start)
        self.src = f32(np.outer(self.sh.M, w.stf))
        self.e_true = E.model_forward(self.g_o, f32(w.m_true) * np.array([1.05, 1.03, 1.0])[:, None, None],
                                      self.sh.src_iz, self.sh.src_ix, self.src, self.sh.ch_iz, self.sh.ch_ix)

    def grid(self, efwi):
        w = self.w
        return efwi.make_grid(w.nz, w.nx, w.dz, w.dx, w.dt, self.g_o.nt, 20, w.pml_R, w.f0, w.vp_max)

    def shot(self, efwi, **kw):
        return efwi.Shot(self.sh.src_iz, self.sh.src_ix, self.sh.ch_iz, self.sh.ch_ix, **kw)


@pytest.fixture(scope="module")
def c2():
    return Case2D()


@pytest.mark.parametrize("gauge,decim,rate", SAMPLINGS[:3])
def test_field_gradient_2d(gpu_lib, c2, gauge, decim, rate):
    efwi = gpu_lib
    sh = c2.sh
    d_obs = f32(KR.field_data(c2.e_true, gauge, decim, rate, c2.g_o.dt))
    g_o, phi_o, y_o = KR.shot_gradient_field(c2.g_o, c2.m, sh.src_iz, sh.src_ix, c2.src, sh.ch_iz, sh.ch_ix, d_obs,
                                             gauge, decim, rate)
    kappa = max(1.0, float(np.linalg.norm(y_o) / np.linalg.norm(y_o - d_obs)))
    grid = c2.grid(efwi)
    shot = c2.shot(efwi, gauge=gauge, decim=decim, rate=bool(rate), ckpt_interval=37)
    d = efwi.model_forward(grid, shot, T(c2.m), T(c2.src)).cpu().numpy()
    assert d.shape == y_o.shape and rel(d, y_o) <= TOL
    d_out = torch.empty(y_o.shape, dtype=torch.float32, device="cuda")
    g, phi = efwi.shot_gradient(grid, shot, T(c2.m), T(c2.src), T(d_obs), d_out=d_out)
    g = g.cpu().numpy()
    assert torch.equal(d_out.cpu(), torch.tensor(d))
    for k in range(3):
        assert rel(g[k], g_o[k]) <= TOL * kappa, (k, rel(g[k], g_o[k]), kappa)
    assert abs(phi.item() - phi_o) / phi_o <= 2 * TOL * kappa
    # J^T v with a field-space v equals the gradient when v is the field residual
    v = T(d - d_obs)
    gj = efwi.shot_jt(grid, shot, T(c2.m), T(c2.src), v).cpu().numpy()
    for k in range(3):
        assert rel(gj[k], g[k]) <= 1e-6


def test_field_adjoint_dot_product(gpu_lib, c2):
    """<K L f, y> = <f, L^T K^T y> for the source components f through the library's forward
    and adjoint with a strain-rate gauge receiver (FP32 on both sides)."""
    efwi = gpu_lib
    grid = c2.grid(efwi)
    shot = c2.shot(efwi, gauge=4, decim=3, rate=True)
    rng = np.random.default_rng(3)
    f = T(c2.src * (1 + 0.2 * rng.standard_normal(c2.src.shape)))
    y = T(rng.standard_normal(shot.data_shape(c2.g_o.nt)) * 1e-6)
    d = efwi.model_forward(grid, shot, T(c2.m), f)
    fb = efwi.model_adjoint(grid, shot, T(c2.m), y)
    lhs = float(torch.sum(d.double() * y.double()))
    rhs = float(torch.sum(f.double() * fb.double()))
    assert lhs == pytest.approx(rhs, rel=1e-4)


def test_batch_with_field_sampling_equals_per_shot(gpu_lib, c2):
    efwi = gpu_lib
    grid = c2.grid(efwi)
    shots = [c2.shot(efwi, gauge=g, decim=dc, rate=r, ckpt_interval=29) for g, dc, r in ((2, 4, True), (1, 1, False),
                                                                                         (5, 2, False))]
    rng = np.random.default_rng(4)
    m_ext = T(np.stack([c2.m * (1 + 0.01 * rng.standard_normal(c2.m.shape)) for _ in shots]))
    src = T(np.stack([c2.src * (k + 1) for k in range(len(shots))]))
    d_obs = [efwi.model_forward(grid, s, T(c2.m), src[k]) * 0.5 for k, s in enumerate(shots)]
    d_cat = torch.cat([d.reshape(-1) for d in d_obs])
    g_ext, phi = efwi.batch_gradient(grid, shots, m_ext, src, d_cat)
    for k, s in enumerate(shots):
        g1, p1 = efwi.shot_gradient(grid, s, m_ext[k], src[k], d_obs[k])
        assert torch.equal(g_ext[k], g1) and phi[k].item() == p1.item()
    # the same batch in several waves, packed largest first (shot 2 ahead of the others), on
    # one lane and on two: the shots' data differ in length, so each shot's data, residual and
    # misfit slots must follow it through the reordering
    full = efwi.workspace_size(efwi.WS_BATCH, grid, shots)
    try:
        two = [c for c in (1 << e for e in range(12, 32)) if (efwi.set_wave_cache_bytes(c) or True) and
               efwi.batch_waves(grid, shots, full, with_lanes=True)[1] == 2]
        assert two
        for cache in sorted({1 << 16, two[0], two[-1]}):
            efwi.set_wave_cache_bytes(cache)
            assert len(efwi.batch_waves(grid, shots, full)) > 1
            g2, p2 = efwi.batch_gradient(grid, shots, m_ext, src, d_cat, ws=efwi.workspace(full))
            assert torch.equal(g_ext, g2) and torch.equal(phi, p2), cache
    finally:
        efwi.set_wave_cache_bytes(0)


def test_field_gradient_3d(gpu_lib):
    efwi = gpu_lib
    w = inputs.precision_3d(nz=36, ny=40, nx=72, nt=160, nshots=1, nch_per_well=20, npml=8)
    sh = w.shots[0]
    g_o = E3.Grid3D(nz=w.nz, ny=w.ny, nx=w.nx, dz=r32(w.h), dy=r32(w.h), dx=r32(w.h), dt=r32(w.dt), nt=w.nt,
                    npml=w.npml, pml_R=r32(w.pml_R), pml_f0=r32(w.f0), vp_max=r32(w.vp_max))
    m = f32(w.m_start)
    src = f32(np.outer(sh.M, w.stf))
    pos, ch = (sh.src_iz, sh.src_iy, sh.src_ix), (sh.ch_iz, sh.ch_iy, sh.ch_ix)
    gauge, decim, rate = 3, 2, 1
    e_obs = E3.model_forward(g_o, f32(w.m_true) * np.array([1.1, 1.05, 1.0])[:, None, None, None], pos, src, ch)
    d_obs = f32(KR.field_data(e_obs, gauge, decim, rate, g_o.dt))
    e, hist = E3.forward(g_o, m, pos, src, ch, store=True)
    y = KR.field_data(e, gauge, decim, rate, g_o.dt)
    phi_o, r = E.misfit(y, d_obs)
    _, grads = E3.adjoint(g_o, m, pos, ch, KR.field_data_T(r, e.shape[0], e.shape[1], gauge, decim, rate, g_o.dt),
                          hist=hist)
    g_ref = E3.chain_rule(m, grads)
    kappa = max(1.0, float(np.linalg.norm(y) / np.linalg.norm(y - d_obs)))
    grid = efwi.make_grid3d(w.nz, w.ny, w.nx, w.h, w.h, w.h, w.dt, w.nt, w.npml, w.pml_R, w.f0, w.vp_max)
    shot = efwi.Shot(sh.src_iz, sh.src_ix, sh.ch_iz, sh.ch_ix, src_iy=sh.src_iy, ch_iy=sh.ch_iy, gauge=gauge,
                     decim=decim, rate=True, ckpt_interval=17)
    g, phi = efwi.shot_gradient(grid, shot, T(m), T(src), T(d_obs))
    g = g.cpu().numpy()
    for k in range(3):
        assert rel(g[k], g_ref[k]) <= TOL * kappa, (k, rel(g[k], g_ref[k]), kappa)
    assert abs(phi.item() - phi_o) / phi_o <= 2 * TOL * kappa
