"""Pins of the field-like DAS sampling oracle (K_r of eq.(3): gauge-length strain rate,
resampled): the transpose by the dot-product test, the identity case, closed forms on a
field linear in time and along the fiber, and the gradient with the field receiver against
a central finite difference of its own misfit."""
import numpy as np
import pytest

from oracle import elastic2d as E
from oracle import receiver as KR


@pytest.mark.parametrize("gauge,decim,rate", [(1, 1, 0), (1, 1, 1), (2, 4, 1), (10, 4, 1), (3, 3, 0), (5, 7, 1)])
def test_transpose_dot_product(gauge, decim, rate):
    rng = np.random.default_rng(gauge * 100 + decim * 10 + rate)
    nch, nt, dt = 23, 61, 5e-4
    x = rng.standard_normal((nch, nt))
    nf, ntf = KR.field_shape(nch, nt, gauge, decim)
    y = rng.standard_normal((nf, ntf))
    lhs = float(np.sum(KR.field_data(x, gauge, decim, rate, dt) * y))
    rhs = float(np.sum(x * KR.field_data_T(y, nch, nt, gauge, decim, rate, dt)))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_identity_case():
    x = np.random.default_rng(1).standard_normal((7, 13))
    assert np.array_equal(KR.field_data(x, 1, 1, 0, 1e-3), x)
    assert np.array_equal(KR.field_data_T(x, 7, 13, 1, 1, 0, 1e-3), x)


@pytest.mark.parametrize("gauge,decim", [(1, 2), (2, 4), (10, 4)])
def test_linear_field_closed_form(gauge, decim):
    """e_c(t_{n+1}) = a t_{n+1} + b c: the gauge mean is a t + b (f + (gauge - 1) / 2) at the
    resampled times, its strain rate a (from the second sample on)."""
    nch, nt, dt, a, b = 30, 40, 2e-3, 3.0, 0.25
    t = (np.arange(nt) + 1) * dt
    e = a * t[None, :] + b * np.arange(nch)[:, None]
    nf, ntf = KR.field_shape(nch, nt, gauge, decim)
    tk = (np.arange(ntf) + 1) * decim * dt
    f = np.arange(nf)[:, None]
    assert np.allclose(KR.field_data(e, gauge, decim, 0, dt), a * tk[None, :] + b * (f + (gauge - 1) / 2.0),
                       rtol=1e-13, atol=1e-13)
    assert np.allclose(KR.field_data(e, gauge, decim, 1, dt), a, rtol=1e-9)
    assert KR.field_data(e, gauge, decim, 1, dt).shape == (nch - gauge + 1, nt // decim)


def test_field_gradient_matches_finite_difference():
    nz, nx, nt = 30, 60, 120
    g = E.Grid2D(nz=nz, nx=nx, dz=5.0, dx=5.0, dt=5e-4, nt=nt, npml=6, pml_R=1e-3, pml_f0=30.0, vp_max=3400.0)
    rng = np.random.default_rng(5)
    m = np.stack([np.full((nz, nx), 3000.0), np.full((nz, nx), 1700.0), np.full((nz, nx), 2100.0)])
    m = m * (1 + 0.01 * rng.standard_normal(m.shape))
    t = np.arange(nt) * 5e-4
    stf = (1 - 2 * (np.pi * 40 * (t - 0.03)) ** 2) * np.exp(-(np.pi * 40 * (t - 0.03)) ** 2)
    src = np.outer([1e15, 0.6e15, 0.2e15], stf)
    chz = np.full(24, 12)
    chx = np.arange(16, 40)
    gauge, decim, rate = 3, 2, 1
    nf, ntf = KR.field_shape(24, nt, gauge, decim)
    d_obs = 0.3 * KR.field_data(E.model_forward(g, m * 1.02, 15, 30, src, chz, chx), gauge, decim, rate, g.dt)
    grad, phi, _ = KR.shot_gradient_field(g, m, 15, 30, src, chz, chx, d_obs, gauge, decim, rate)
    dm = np.zeros_like(m)
    dm[0, 14:18, 20:26] = 1.0
    dm[1, 10:13, 33:37] = -0.7
    dm[2, 16:19, 28:31] = 0.5
    h = 1e-3

    def f(mm):
        return KR.shot_gradient_field(g, mm, 15, 30, src, chz, chx, d_obs, gauge, decim, rate)[1]

    fd = (f(m + h * dm) - f(m - h * dm)) / (2 * h)
    assert float(np.sum(grad * dm)) == pytest.approx(fd, rel=1e-6)
