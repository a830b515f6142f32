"""Pins of the regularizer oracle (eq.(8) second term, eqs.(10)-(12)).

Checked against properties the paper states or that follow from the operators' definitions:
rows of W sum to one; W only changes sinkhole samples; a consistent extended model
S^T m is left unchanged by W, gives zero penalty and zero gradient; P = I - S^T S_w is a
projector; the hard-mask limit reduces to "each unmasked model against the mean of the
unmasked models"; finite differences of the penalty match the gradient.
"""
import numpy as np
import pytest

from oracle import regularizer as R


def zoi_1d(n, src, radius, nexp, nu):
    """eq.(10) weights for the 1D example: b = (cos^n(pi r / 2) - log nu) / (1 - log nu),
    r = 1 - |x - x_s| / radius inside the sinkhole (1 at the source, 0 at its edge)."""
    x = np.arange(n)
    b = np.ones((len(src), n))
    sink = np.zeros((len(src), n), bool)
    for s, xs in enumerate(src):
        dist = np.abs(x - xs) / radius
        inside = dist < 1.0
        r = 1.0 - dist[inside]
        b[s, inside] = (np.cos(0.5 * np.pi * r) ** nexp - np.log(nu)) / (1.0 - np.log(nu))
        sink[s] = inside
    return b, sink


@pytest.fixture
def example_31x3():
    """The paper's W illustration: a 1D model with 31 samples extended along 3 sources."""
    return zoi_1d(31, [6, 15, 24], 5.0, 2, 0.9)


def test_w_rows_sum_to_one_and_only_touch_sinkholes(example_31x3):
    b, sink = example_31x3
    assert np.isclose(b[sink].min(), -np.log(0.9) / (1 - np.log(0.9)))   # "small positive value"
    for p in range(31):
        W = R.w_matrix(b[:, p], sink[:, p])
        assert np.allclose(W.sum(axis=1), 1.0)
        for s in range(3):
            if not sink[s, p]:
                assert np.array_equal(W[s], np.eye(3)[s])
            else:
                assert W[s, s] < 1.0 and np.all(W[s] >= 0.0)


def test_consistent_model_is_fixed_point(example_31x3):
    b, sink = example_31x3
    rng = np.random.default_rng(0)
    m = rng.standard_normal((3, 31))                      # (Vp, Vs, rho)-like parameters
    m_ext = np.broadcast_to(m, (3, 3, 31)).copy()         # S^T m
    phi, g = R.regularizer(m_ext, b, sink, eta=2.0)
    assert abs(phi) < 1e-24 and np.max(np.abs(g)) < 1e-12
    assert np.allclose(R.final_model(m_ext, b, sink), m)  # eq.(9) recovers m


def test_projector_idempotent_and_sw_is_not_adjoint(example_31x3):
    b, sink = example_31x3
    for p in range(31):
        P = R.projector(b[:, p], sink[:, p])
        assert np.allclose(P @ P, P)
    # where the outer-taper weights differ, S^T S_w is not symmetric (S^T != S_w^T)
    P = R.projector(np.array([0.3, 1.0, 0.6]), np.zeros(3, bool))
    assert np.allclose(P @ P, P) and not np.allclose(P, P.T)


def test_hard_mask_closed_form():
    """b_s = 0 inside s's mask, 1 elsewhere: penalty = 1/2 eta^2 sum_x sum_{s in O(x)}
    (m_s - mean_O)^2 with O(x) the shots not masking x; gradient eta^2 (m_s - mean_O) on O."""
    rng = np.random.default_rng(1)
    ns, n = 5, 40
    sink = np.zeros((ns, n), bool)
    for s in range(ns):
        c = 4 + 8 * s
        sink[s, max(0, c - 3):c + 4] = True
    sink[1, 20:24] = True                                  # overlapping masks
    sink[3, 20:22] = True
    b = np.where(sink, 0.0, 1.0)
    m_ext = rng.standard_normal((ns, 3, n))
    eta = 1.5
    phi, g = R.regularizer(m_ext, b, sink, eta)
    phi_ref = 0.0
    g_ref = np.zeros_like(m_ext)
    for x in range(n):
        O = [s for s in range(ns) if not sink[s, x]]
        mu = m_ext[O, :, x].mean(axis=0)
        for s in O:
            phi_ref += 0.5 * eta ** 2 * np.sum((m_ext[s, :, x] - mu) ** 2)
            g_ref[s, :, x] = eta ** 2 * (m_ext[s, :, x] - mu)
    assert np.isclose(phi, phi_ref, rtol=1e-12)
    assert np.allclose(g, g_ref, rtol=1e-12, atol=1e-14)


def test_finite_difference_gradient(example_31x3):
    b, sink = example_31x3
    rng = np.random.default_rng(2)
    m_ext = rng.standard_normal((3, 3, 31))
    phi, g = R.regularizer(m_ext, b, sink, eta=0.7)
    for _ in range(4):
        dm = rng.standard_normal(m_ext.shape)
        h = 1e-6
        fp, _ = R.regularizer(m_ext + h * dm, b, sink, 0.7)
        fm, _ = R.regularizer(m_ext - h * dm, b, sink, 0.7)
        assert np.isclose((fp - fm) / (2 * h), np.sum(g * dm), rtol=1e-7)


def test_degenerate_points():
    # a sinkhole point where no other source has weight: W row is the identity
    W = R.w_matrix(np.array([0.2, 0.0, 0.0]), np.array([True, False, False]))
    assert np.array_equal(W, np.eye(3))
    # no useful source at the point: no penalty there
    phi, g = R.regularizer(np.ones((2, 3, 1)) * np.array([1.0, 2.0])[:, None, None],
                           np.zeros((2, 1)), np.zeros((2, 1), bool), 1.0)
    assert phi == 0.0 and np.all(g == 0.0)


def test_soft_weight_sinkhole_by_hand():
    """A point worked by hand from eqs.(9), (11) and (12) with soft weights inside a
    sinkhole: Ns = 3, b = (0.2, 0.5, 1.0), source 0's sinkhole covers the point, m = (1, 2, 4).

    eq.(11): (W m)_0 = 0.2 * 1 + 0.8 * (0.5 * 2 + 1.0 * 4) / 1.5 = 43/15; rows 1, 2 unchanged.
    eq.(12): b' = (1, 0.5, 1.0) (b'_0 = 1 inside source 0's sinkhole), sum 5/2, so
    S_w W m = (43/15 + 1 + 4) / (5/2) = 236/75 (b'_0 = b_0 would give 3.2784...).
    y = W m - S^T S_w W m = (-21, -86, 64) / 75; phi = 1/2 |y|^2 = 11933/11250 (eta = 1).
    z = y - (b'/sum b') sum(y) = (-19, -387, 406) / 375 and g = W^T z =
    (-19/1875, -5881/5625, 5938/5625)."""
    b = np.array([0.2, 0.5, 1.0])[:, None]
    sink = np.array([True, False, False])[:, None]
    m = np.array([1.0, 2.0, 4.0])
    scale = np.array([1.0, -3.0, 0.5])                      # Vp, Vs, rho: same weights
    m_ext = (m[:, None] * scale[None, :])[:, :, None]        # [3 shots][3 params][1 point]
    assert np.allclose(R.w_matrix(b[:, 0], sink[:, 0]) @ m, [43 / 15, 2.0, 4.0], rtol=0, atol=1e-14)
    assert np.allclose(R.sw_row(b[:, 0], sink[:, 0]), [0.4, 0.2, 0.4], rtol=0, atol=1e-15)
    assert np.allclose(R.final_model(m_ext, b, sink)[:, 0], 236 / 75 * scale, rtol=1e-14)
    phi, g = R.regularizer(m_ext, b, sink, eta=1.0)
    assert np.isclose(phi, 11933 / 11250 * float(np.sum(scale ** 2)), rtol=1e-13)
    g_hand = np.array([-19 / 1875, -5881 / 5625, 5938 / 5625])
    assert np.allclose(g[:, :, 0], g_hand[:, None] * scale[None, :], rtol=1e-13, atol=1e-15)
    # eta scales the value by eta^2 and the gradient by eta^2
    phi2, g2 = R.regularizer(m_ext, b, sink, eta=3.0)
    assert np.isclose(phi2, 9.0 * phi, rtol=1e-13) and np.allclose(g2, 9.0 * g, rtol=1e-13)
