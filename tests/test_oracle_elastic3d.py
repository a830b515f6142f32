"""Pins of the 3D FP64 oracle.

T1  analytic 3D explosion: v_r = M0/(4 pi rho a^2) [s(tau)/r^2 + s'(tau)/(a r)], tau = t - r/a
T2  exact leapfrog energy conservation with rigid walls
T3  source-receiver reciprocity (six-component MT source vs DAS e_xx receiver)
T4  dot product <L f, r> = <f, L^T r> with and without CPML, all six MT components
T5  central finite differences of the misfit vs the gradient (Vp, Vs, rho)
"""
import math

import numpy as np
import pytest

from oracle import elastic3d as E3
from paper_2305_14130_amd.inputs import ricker


def _medium(rng, shape):
    vp = 3000.0 * (1 + 0.05 * rng.standard_normal(shape))
    vs = vp / 1.7 * (1 + 0.03 * rng.standard_normal(shape))
    rho = 2300.0 * (1 + 0.04 * rng.standard_normal(shape))
    return np.stack([vp, vs, rho])


def test_t1_analytic_explosion_3d():
    h, dt, f0, a, rho0 = 5.0, 0.5e-3, 30.0, 3000.0, 2300.0
    n, nt = 56, 200
    g = E3.Grid3D(nz=n, ny=n, nx=n, dz=h, dy=h, dx=h, dt=dt, nt=nt, npml=10, pml_f0=f0, vp_max=a)
    vp = np.full((n, n, n), a)
    m = np.stack([vp, vp / 1.7, np.full_like(vp, rho0)])
    s0, jr = 28, 37
    M0 = 1e9
    stf = ricker(nt, dt, f0)
    tr = []
    E3.forward(g, m, (s0, s0, s0), E3.moment_tensor_series([M0, M0, M0, 0, 0, 0], stf), ([s0], [s0], [s0 + 5]),
               probe=lambda k, P: tr.append(P.vx[s0, s0, jr]))
    tr = np.array(tr)
    r = (jr + 0.5 - s0) * h
    t = (np.arange(nt) + 0.5) * dt - r / a - 1.5 / f0
    arg = (math.pi * f0 * t) ** 2
    s = (1 - 2 * arg) * np.exp(-arg)
    sdot = -2 * math.pi ** 2 * f0 ** 2 * t * (3 - 2 * arg) * np.exp(-arg)
    ana = M0 / (4 * math.pi * rho0 * a * a) * (s / r ** 2 + sdot / (a * r))
    err = np.linalg.norm(tr - ana) / np.linalg.norm(ana)
    assert err < 3e-2, err
    assert abs(np.argmax(np.abs(tr)) - np.argmax(np.abs(ana))) <= 1
    assert np.sign(tr[np.argmax(np.abs(tr))]) == np.sign(ana[np.argmax(np.abs(ana))])


def test_t2_energy_rigid():
    rng = np.random.default_rng(1)
    shape = (14, 16, 18)
    g = E3.Grid3D(*shape, 5.0, 5.0, 5.0, 0.35e-3, 420, npml=0, vp_max=3400.0)
    m = _medium(rng, shape)
    med = E3.stage(*m)
    lam, mu = med["lam"], med["mu"]
    stf = ricker(g.nt, g.dt, 40.0)
    stf[150:] = 0.0
    prev, energy = {}, []

    def probe(n, P):
        if prev:
            kin = 0.5 * sum(np.sum(prev[v] * getattr(P, v) / med["b" + v[1]]) for v in ("vx", "vy", "vz"))
            s = [prev["sxx"], prev["syy"], prev["szz"]]
            tr = s[0] + s[1] + s[2]
            # compliance of the normal block: (s_c - lam tr / (3 lam + 2 mu)) / (2 mu)
            pot = 0.5 * np.sum(sum(sc * (sc - lam * tr / (3 * lam + 2 * mu)) for sc in s) / (2 * mu))
            pot += 0.5 * sum(np.sum(prev[sn] ** 2 / med[E3.SHEAR_MU[sn]]) for sn in E3.SHEAR_TERMS)
            energy.append(kin + pot)
        prev.update({f: getattr(P, f).copy() for f in E3.FIELDS})

    E3.forward(g, m, (7, 8, 9), E3.moment_tensor_series([1e9, 0.8e9, 0.6e9, 0.3e9, -0.2e9, 0.1e9], stf),
               ([7], [8], [12]), probe=probe)
    e = np.array(energy[170:])
    assert np.max(np.abs(e - e[0])) / abs(e[0]) < 1e-9


@pytest.mark.parametrize("npml", [0, 4])
def test_t4_dot_product(npml):
    rng = np.random.default_rng(2 + npml)
    shape = (14, 15, 17)
    g = E3.Grid3D(*shape, 5.0, 5.0, 5.0, 0.35e-3, 70, npml=npml, pml_f0=30.0, vp_max=3400.0)
    m = _medium(rng, shape)
    ch = (np.array([7, 7, 9]), np.array([7, 8, 6]), np.array([5, 11, 9]))
    f = rng.standard_normal((6, g.nt))
    r = rng.standard_normal((3, g.nt))
    Lf = E3.model_forward(g, m, (7, 7, 8), f, ch)
    LTr = E3.model_adjoint(g, m, (7, 7, 8), ch, r)
    a, b = np.sum(Lf * r), np.sum(f * LTr)
    assert abs(a - b) / abs(a) < 1e-12


@pytest.mark.parametrize("which", [0, 1, 2])
def test_t5_fd_gradient(which):
    rng = np.random.default_rng(20 + which)
    shape = (14, 15, 18)
    g = E3.Grid3D(*shape, 5.0, 5.0, 5.0, 0.35e-3, 90, npml=4, pml_f0=30.0, vp_max=3400.0)
    m = _medium(rng, shape)
    mt = m * np.array([1.02, 0.99, 1.01])[:, None, None, None]
    src = E3.moment_tensor_series([1e16, 0.7e16, 0.5e16, 0.2e16, -0.3e16, 0.1e16], ricker(g.nt, g.dt, 40.0))
    ch = (np.full(6, 7), np.full(6, 7), np.arange(5, 11))
    d_obs = E3.model_forward(g, mt, (7, 7, 4), src, ch)
    G, phi, _ = E3.shot_gradient(g, m, (7, 7, 4), src, ch, d_obs)
    dm = np.zeros_like(m)
    dm[which] = rng.standard_normal(shape) * m[which]
    h = 1e-5
    pp, _ = E3.misfit(E3.model_forward(g, m + h * dm, (7, 7, 4), src, ch), d_obs)
    pm, _ = E3.misfit(E3.model_forward(g, m - h * dm, (7, 7, 4), src, ch), d_obs)
    fd = (pp - pm) / (2 * h)
    an = np.sum(G * dm)
    assert abs(fd - an) / abs(an) < 1e-6, (fd, an)


def test_t3_reciprocity_mt_source_das_receiver():
    """Rigid walls: e_xx at q from the six-component MT source at p equals
    -(M : strain)(p) from a unit stress-rate source in sxx at q, where each engineering shear
    strain at p is the mean over the four shear nodes around p, listed here directly:
    xy at (i, k-1..k, j-1..j), xz at (i-1..i, k, j-1..j), yz at (i-1..i, k-1..k, j)."""
    rng = np.random.default_rng(4)
    shape = (13, 14, 16)
    g = E3.Grid3D(*shape, 5.0, 5.0, 5.0, 0.35e-3, 150, npml=0, vp_max=3400.0)
    m = _medium(rng, shape)
    stf = ricker(g.nt, g.dt, 45.0)
    M = np.array([1.0, 0.6, -0.7, 0.4, -0.5, 0.3])
    p, q = (6, 7, 5), (7, 6, 11)
    d1 = E3.forward(g, m, p, E3.moment_tensor_series(M, stf), ([q[0]], [q[1]], [q[2]]))[0]
    i, k, j = p
    acc = np.zeros(6)
    rec = []

    def probe(n, P):
        D, Dp = E3.d_minus, E3.d_plus
        exx = D(P.vx, g.dx, E3.X)[p]
        eyy = D(P.vy, g.dy, E3.Y)[p]
        ezz = D(P.vz, g.dz, E3.Z)[p]
        gxy = Dp(P.vx, g.dy, E3.Y) + Dp(P.vy, g.dx, E3.X)
        gxz = Dp(P.vx, g.dz, E3.Z) + Dp(P.vz, g.dx, E3.X)
        gyz = Dp(P.vy, g.dz, E3.Z) + Dp(P.vz, g.dy, E3.Y)
        sxy = 0.25 * gxy[i, k - 1:k + 1, j - 1:j + 1].sum()
        sxz = 0.25 * gxz[i - 1:i + 1, k, j - 1:j + 1].sum()
        syz = 0.25 * gyz[i - 1:i + 1, k - 1:k + 1, j].sum()
        acc[:] += g.dt * np.array([exx, eyy, ezz, sxy, sxz, syz])
        rec.append(-(M @ acc))

    E3.forward(g, m, q, E3.moment_tensor_series([-1.0, 0, 0, 0, 0, 0], stf), ([q[0]], [q[1]], [q[2]]), probe=probe)
    d2 = np.array(rec)
    assert np.linalg.norm(d1 - d2) / np.linalg.norm(d1) < 1e-12
