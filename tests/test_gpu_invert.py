"""The inversion driver on the library's objectives (GPU): the extended and conventional
objectives and gradients equal the library's pieces called directly, and a few l-BFGS
iterations on the guided-wave synthetic decrease both objectives."""
import numpy as np
import pytest
import torch

from paper_2305_14130_amd import efwi, inputs, invert

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup(gpu_lib):
    w = inputs.guided_wave_synthetic(nt=500)
    grid = efwi.make_grid(w.nz, w.nx, w.dz, w.dx, w.dt, w.nt, w.npml, w.pml_R, w.f0, w.vp_max)
    T = lambda a: torch.tensor(np.asarray(a, np.float32), device="cuda")
    d_obs = torch.cat([efwi.model_forward(grid, efwi.Shot(s.src_iz, s.src_ix, s.ch_iz, s.ch_ix), T(w.m_true),
                                          T(np.outer(s.M, w.stf))) for s in w.shots])
    zones = [efwi.make_zone((s.src_iz * w.dz, 0.0, s.src_ix * w.dx), (1 / 400.0, 0, 1e-4, 0, 0, 0),
                            (0.0, 500.0, 0, 0, 0.0, 2000.0), 0.0) for s in w.shots]
    b, sink = efwi.zoi_weights(grid, zones, 2.0, 0.9)
    return w, grid, d_obs, b, sink


def test_objectives_match_library(setup):
    w, grid, d_obs, b, sink = setup
    ext = invert.ExtendedFWI(w, d_obs, b, sink, 3e-4)
    rng = np.random.default_rng(1)
    x = torch.tensor(0.01 * rng.standard_normal((3, 2, w.nz, w.nx)), dtype=torch.float32, device="cuda")
    phi, gx = ext(x)
    m = ext.model(x)
    g, p = efwi.batch_gradient(ext.grid, ext.shots, m, ext.src, d_obs)
    pr = efwi.extension_regularizer(ext.grid, m, b, sink, 3e-4, g)
    assert phi == pytest.approx(float(p.sum()) + float(pr), rel=1e-12)
    assert torch.equal(gx, (g[:, :2] * ext.m0[:2]).contiguous())
    conv = invert.ConventionalFWI(w, d_obs)
    phi_c, gc = conv(x[0])
    gsum = torch.zeros_like(gc)
    psum = 0.0
    for k, s in enumerate(conv.shots):
        gk, pk = efwi.shot_gradient(conv.grid, s, conv.model(x[0]), conv.src[k], d_obs.split([sh.nch for sh in conv.shots])[k])
        gsum += gk[:2] * conv.m0[:2]
        psum += pk.item()
    assert phi_c == pytest.approx(psum, rel=1e-12)
    assert torch.allclose(gc, gsum, rtol=1e-5, atol=1e-6 * float(gsum.abs().max()))


def test_a_few_iterations_decrease_both(setup):
    w, grid, d_obs, b, sink = setup
    for prob in (invert.ConventionalFWI(w, d_obs), invert.ExtendedFWI(w, d_obs, b, sink, 3e-4)):
        x, rec = invert.lbfgs(prob, prob.x0(), max_iter=4, rate_tol=0.0, first_step=0.01)
        assert len(rec.phi) >= 2 and all(b_ <= a for a, b_ in zip(rec.phi, rec.phi[1:]))
        assert rec.phi[-1] < 0.9 * rec.phi[0]
        m = prob.final(x)
        assert m.shape == (3, w.nz, w.nx) and bool(torch.isfinite(m).all())


def test_alternative_methods_match_library(setup):
    """eq.(15): the preconditioned problem keeps the conventional objective and hands the
    solver S_w W of the per-shot gradients; the mute + pseudo-Hessian start is the library's
    operator at the starting model."""
    w, grid, d_obs, b, sink = setup
    rng = np.random.default_rng(2)
    x = torch.tensor(0.01 * rng.standard_normal((2, w.nz, w.nx)), dtype=torch.float32, device="cuda")
    pre = invert.PreconditionedFWI(w, d_obs, b, sink)
    phi, gx = pre(x)
    conv = invert.ConventionalFWI(w, d_obs)
    assert phi == conv(x)[0]
    m = pre.model(x)
    g, _ = efwi.batch_gradient(pre.grid, pre.shots, m.unsqueeze(0).repeat(pre.ns, 1, 1, 1).contiguous(), pre.src,
                               d_obs)
    assert torch.equal(gx, (efwi.final_model(pre.grid, g, b, sink)[:2] * pre.m0[:2]).contiguous())
    h0 = invert.inverse_pseudo_hessian(conv, 0.01)
    _, p = efwi.pseudo_hessian(conv.grid, conv.shots, conv.m0.unsqueeze(0).repeat(conv.ns, 1, 1, 1).contiguous(),
                               conv.src, 0.01)
    assert h0.shape == (2, w.nz, w.nx) and torch.equal(h0[0], p) and torch.equal(h0[1], p)
    assert float(p.min()) == pytest.approx(0.01, rel=1e-6) and float(p.max()) == 1.0
    x1, rec = invert.lbfgs(conv, conv.x0(), max_iter=3, rate_tol=0.0, first_step=0.01, h0=h0)
    assert rec.phi[-1] < 0.95 * rec.phi[0]
