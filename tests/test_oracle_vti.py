"""Pins of the VTI oracle: Thomsen's definitions recovered from the staged stiffness
(epsilon, and delta = epsilon / 2), the isotropic oracle for epsilon = 0, the horizontal and
vertical P-wave speeds Vp0 sqrt(1 + 2 eps) and Vp0 measured on the simulated wavefield, the
transpose by the dot-product test, and the gradient (Vp0, Vs0, rho) against central finite
differences."""
import numpy as np
import pytest

from oracle import elastic2d as E
from oracle import vti2d as V


def ricker(nt, dt, f0, t0):
    a = (np.pi * f0 * (np.arange(nt) * dt - t0)) ** 2
    return (1 - 2 * a) * np.exp(-a)


def test_thomsen_parameters_recovered():
    rng = np.random.default_rng(0)
    vp, vs = rng.uniform(2500, 4500, (5, 7)), rng.uniform(1200, 2200, (5, 7))
    rho, eps = rng.uniform(2000, 2700, (5, 7)), rng.uniform(0.0, 0.6, (5, 7))
    m = V.stage_vti(vp, vs, rho, eps)
    c11, c13, c33, c55 = m["c11"], m["c13"], m["c33"], m["mu"]
    assert np.allclose(c33, rho * vp * vp, rtol=1e-15) and np.allclose(c55, rho * vs * vs, rtol=1e-15)
    assert np.allclose((c11 - c33) / (2 * c33), eps, rtol=1e-12, atol=1e-15)
    delta = ((c13 + c55) ** 2 - (c33 - c55) ** 2) / (2 * c33 * (c33 - c55))
    assert np.allclose(delta, eps / 2, rtol=1e-10, atol=1e-14)
    iso = V.stage_vti(vp, vs, rho, 0.0)
    assert np.allclose(iso["c13"], rho * vp * vp - 2 * rho * vs * vs, rtol=1e-12)


def small(nt=90):
    nz, nx = 40, 60
    rng = np.random.default_rng(1)
    m = np.stack([np.full((nz, nx), 3000.0), np.full((nz, nx), 1600.0), np.full((nz, nx), 2200.0)])
    m = m * (1 + 0.01 * rng.standard_normal(m.shape))
    eps = 0.2 + 0.1 * rng.uniform(size=(nz, nx))
    g = E.Grid2D(nz=nz, nx=nx, dz=5.0, dx=5.0, dt=4e-4, nt=nt, npml=8, pml_R=1e-3, pml_f0=30.0, vp_max=3800.0)
    src = np.outer([1e15, 0.7e15, 0.3e15], ricker(nt, 4e-4, 40.0, 0.025))
    chz, chx = np.full(20, 14), np.arange(18, 38)
    return g, m, eps, src, chz, chx


def test_isotropic_limit():
    g, m, _, src, chz, chx = small(60)
    d_iso = E.model_forward(g, m, 20, 30, src, chz, chx)
    d_vti = V.model_forward(g, m, 0.0, 20, 30, src, chz, chx)
    assert np.allclose(d_vti, d_iso, rtol=0, atol=1e-12 * np.abs(d_iso).max())
    d_obs = 0.5 * d_iso
    g_iso, p_iso, _ = E.shot_gradient(g, m, 20, 30, src, chz, chx, d_obs)
    g_vti, p_vti, _ = V.shot_gradient(g, m, 0.0, 20, 30, src, chz, chx, d_obs)
    assert p_vti == pytest.approx(p_iso, rel=1e-12)
    assert np.allclose(g_vti, g_iso, rtol=0, atol=1e-10 * np.abs(g_iso).max())


def test_p_wave_speeds_horizontal_and_vertical():
    """An explosion in a homogeneous VTI medium: the P pulse's travel time between two
    receivers on the x axis gives Vp0 sqrt(1 + 2 eps), on the z axis Vp0 (2%)."""
    n, h, dt, nt, eps, vp0 = 141, 5.0, 4e-4, 380, 0.25, 3000.0
    m = np.stack([np.full((n, n), vp0), np.full((n, n), 1500.0), np.full((n, n), 2000.0)])
    g = E.Grid2D(nz=n, nx=n, dz=h, dx=h, dt=dt, nt=nt, npml=15, pml_R=1e-4, pml_f0=25.0, vp_max=vp0 * 1.23)
    src = np.outer([1e15, 1e15, 0.0], ricker(nt, dt, 25.0, 0.05))
    c, r1, r2 = 70, 30, 55
    tr = {k: np.zeros(nt) for k in ("x1", "x2", "z1", "z2")}

    def probe(k, P):
        tr["x1"][k], tr["x2"][k] = P.vx[c, c + r1], P.vx[c, c + r2]
        tr["z1"][k], tr["z2"][k] = P.vz[c + r1, c], P.vz[c + r2, c]

    none = np.zeros(0, np.int64)
    V.forward(g, m, eps, c, c, src, none, none, probe=probe)

    def lag(a, b):
        cc = np.correlate(b, a, mode="full")
        k = int(np.argmax(cc))
        y0, y1, y2 = cc[k - 1], cc[k], cc[k + 1]
        return (k - (len(a) - 1) + 0.5 * (y0 - y2) / (y0 - 2 * y1 + y2)) * dt

    vx = (r2 - r1) * h / lag(tr["x1"], tr["x2"])
    vz = (r2 - r1) * h / lag(tr["z1"], tr["z2"])
    assert vx == pytest.approx(vp0 * np.sqrt(1 + 2 * eps), rel=0.02)
    assert vz == pytest.approx(vp0, rel=0.02)


def test_transpose_dot_product():
    g, m, eps, src, chz, chx = small(70)
    rng = np.random.default_rng(2)
    f = rng.standard_normal(src.shape) * 1e15
    r = rng.standard_normal((len(chz), g.nt))
    d = V.model_forward(g, m, eps, 20, 30, f, chz, chx)
    fb = V.adjoint(g, m, eps, 20, 30, chz, chx, r)
    assert float(np.sum(d * r)) == pytest.approx(float(np.sum(f * fb)), rel=1e-11)


def test_gradient_finite_difference():
    g, m, eps, src, chz, chx = small(90)
    d_obs = 0.3 * V.model_forward(g, m * 1.02, eps, 20, 30, src, chz, chx)
    grad, phi, _ = V.shot_gradient(g, m, eps, 20, 30, src, chz, chx, d_obs)
    dm = np.zeros_like(m)
    dm[0, 15:20, 20:27] = 1.0
    dm[1, 10:14, 33:38] = -0.8
    dm[2, 18:22, 26:31] = 0.6
    hstep = 1e-3

    def f(mm):
        return V.shot_gradient(g, mm, eps, 20, 30, src, chz, chx, d_obs)[1]

    fd = (f(m + hstep * dm) - f(m - hstep * dm)) / (2 * hstep)
    assert float(np.sum(grad * dm)) == pytest.approx(fd, rel=1e-6)
