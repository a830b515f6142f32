"""Pins of the comparison-method oracle (approximate inverse pseudo-Hessian, near-offset
mute; the eq.(15) preconditioning is the final-model operator, pinned with the regularizer).

What fixes the values, independently of the oracle's accumulation code:
* an impulsive source: after one step the stress is a single injected spike, so the
  velocities of the next half step, and with them H, follow in closed form from the
  staggered fourth-order stencil (9/8, -1/24) and the injection scaling dt/(dx dz);
* H is quadratic in the source amplitude (a sum of squares, not of magnitudes);
* the last step's increment of H equals |v|^2 of the final state of a forward run;
* the inverse operator's range, extremes and monotonicity;
* the mute keeps exactly the channels at or beyond the radius.
"""
import numpy as np
import pytest

from oracle import elastic2d as E
from oracle import precondition as PH

K1, K2 = 9.0 / 8.0, -1.0 / 24.0


def homogeneous(nz, nx, vp=3000.0, vs=1700.0, rho=2000.0):
    return np.full((nz, nx), vp), np.full((nz, nx), vs), np.full((nz, nx), rho)


@pytest.mark.parametrize("comp", [0, 1])
def test_impulse_closed_form(comp):
    nz, nx, dz, dx, dt, rho = 20, 30, 5.0, 4.0, 5e-4, 2000.0
    iz, ix = 9, 14
    vp, vs, r = homogeneous(nz, nx, rho=rho)
    src = np.zeros((3, 2))
    src[comp, 0] = 1.0e6                   # a spike of M_xx (comp 0) or M_zz (comp 1) at step 0
    A = -dt / (dx * dz) * 1.0e6            # the injected stress spike
    g1 = E.Grid2D(nz=nz, nx=nx, dz=dz, dx=dx, dt=dt, nt=1)
    assert np.all(PH.autocorrelation(g1, vp, vs, r, iz, ix, src[:, :1]) == 0.0)   # v^{1/2} = 0
    g2 = E.Grid2D(nz=nz, nx=nx, dz=dz, dx=dx, dt=dt, nt=2)
    H = PH.autocorrelation(g2, vp, vs, r, iz, ix, src)
    expect = np.zeros((nz, nx))
    h = dx if comp == 0 else dz
    for off, c in ((-2, K2), (-1, K1), (0, -K1), (1, -K2)):
        v = dt / rho * c * A / h           # v^{3/2} = dt b D+ sigma^1 at the spike's neighbours
        if comp == 0:
            expect[iz, ix + off] = v * v   # vx at (iz, j + 1/2) belongs to node (iz, j)
        else:
            expect[iz + off, ix] = v * v   # vz at (i + 1/2, ix) belongs to node (i, ix)
    assert np.allclose(H, expect, rtol=1e-12, atol=0.0)


def small_case(nt=80, amp=1.0):
    nz, nx = 40, 56
    vp, vs, r = homogeneous(nz, nx)
    vp[20:, :] = 3600.0
    g = E.Grid2D(nz=nz, nx=nx, dz=5.0, dx=5.0, dt=5e-4, nt=nt, npml=8, pml_R=1e-3, pml_f0=30.0, vp_max=3600.0)
    t = np.arange(nt) * 5e-4
    stf = (1 - 2 * (np.pi * 30 * (t - 0.04)) ** 2) * np.exp(-(np.pi * 30 * (t - 0.04)) ** 2)
    src = amp * np.outer([1e15, -0.4e15, 0.6e15], stf)
    return g, vp, vs, r, 18, 27, src


def test_quadratic_in_amplitude_and_nonnegative():
    g, vp, vs, r, iz, ix, src = small_case()
    H1 = PH.autocorrelation(g, vp, vs, r, iz, ix, src)
    H2 = PH.autocorrelation(g, vp, vs, r, iz, ix, 2.0 * src)
    assert np.all(H1 >= 0.0) and H1.max() > 0.0
    assert np.allclose(H2, 4.0 * H1, rtol=1e-12, atol=0.0)


def test_last_step_increment_is_final_state():
    g, vp, vs, r, iz, ix, src = small_case(nt=50)
    K = 50
    gk = E.Grid2D(**{**g.__dict__, "nt": K})
    gk1 = E.Grid2D(**{**g.__dict__, "nt": K - 1})
    Hk = PH.autocorrelation(gk, vp, vs, r, iz, ix, src[:, :K])
    Hk1 = PH.autocorrelation(gk1, vp, vs, r, iz, ix, src[:, :K - 1])
    none = np.zeros(0, np.int64)
    _, _, P = E.forward(gk, vp, vs, r, iz, ix, src[:, :K], none, none, store=True)
    assert np.allclose(Hk - Hk1, P.vx ** 2 + P.vz ** 2, rtol=1e-9, atol=1e-12 * Hk.max())


def test_sum_over_shots_places_windows():
    a = np.arange(6.0).reshape(2, 3)
    H = PH.sum_over_shots((4, 5), [(1, 2, a), (0, 0, np.ones((2, 2)))])
    expect = np.zeros((4, 5))
    expect[1:3, 2:5] += a
    expect[0:2, 0:2] += 1.0
    assert np.array_equal(H, expect)


def test_inverse_operator():
    rng = np.random.default_rng(3)
    H = rng.uniform(0.0, 1.0, (30, 40)) ** 4
    H[7, 9] = 5.0
    P = PH.inverse_operator(H, 0.01)
    assert P.max() == 1.0 and P[7, 9] == pytest.approx(0.01, rel=1e-15)
    assert np.all(P[H <= 0.05] == 1.0)                        # clipped: uniform weight far away
    o = np.argsort(H, axis=None)
    assert np.all(np.diff(P.ravel()[o]) <= 0.0)               # more energy, smaller weight
    assert np.all(PH.inverse_operator(np.zeros((3, 4)), 0.1) == 1.0)
    assert np.all(PH.inverse_operator(H, 1.0) == H.max() / np.maximum(H, H.max()))


def test_near_offset_keep():
    keep = PH.near_offset_keep(10, 20, [10, 10, 10, 13, 40], [20, 59, 60, 24, 20], 5.0, 5.0, 200.0)
    # distances 0, 195, 200, 25, 150 m
    assert keep.tolist() == [False, False, True, False, False]
