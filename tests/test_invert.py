"""Host-side checks of the inversion driver: the l-BFGS loop with its strong-Wolfe line
search on functions with known minima, the convergence-rate stop of eq.(13) and the cosine
similarity of eq.(14). (The objectives of the FWI problems are the library's, covered by the
GPU parity tests; tests/test_gpu_invert.py runs the loop on them.)"""
import numpy as np
import pytest
import torch

from paper_2305_14130_amd.invert import convergence_rate, cosine_similarity, lbfgs, wolfe_search


def rosenbrock(x):
    x = x.double()
    a, b = x[:-1], x[1:]
    f = float(torch.sum(100.0 * (b - a * a) ** 2 + (1.0 - a) ** 2))
    g = torch.zeros_like(x)
    g[:-1] += -400.0 * a * (b - a * a) - 2.0 * (1.0 - a)
    g[1:] += 200.0 * (b - a * a)
    return f, g


def test_lbfgs_rosenbrock():
    x0 = torch.tensor([-1.2, 1.0, -1.2, 1.0, 0.5, -0.3], dtype=torch.float64)
    x, rec = lbfgs(rosenbrock, x0, max_iter=500, rate_tol=0.0)
    assert np.allclose(x.numpy(), 1.0, atol=1e-5)
    assert all(b <= a for a, b in zip(rec.phi, rec.phi[1:]))       # monotone decrease


def test_lbfgs_quadratic_and_rate_stop():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((20, 20))
    H = torch.tensor(A @ A.T + 20 * np.eye(20))
    xs = torch.tensor(rng.standard_normal(20))
    c = 3.0

    def quad(x):
        r = x - xs
        return float(0.5 * r @ H @ r) + c, H @ r

    x, rec = lbfgs(quad, torch.zeros(20, dtype=torch.float64), max_iter=200, rate_tol=0.0)
    assert np.allclose(x.numpy(), xs.numpy(), atol=1e-6)
    # the loop stops at the first iteration whose eq.(13) rate is below the threshold
    _, rec2 = lbfgs(quad, torch.zeros(20, dtype=torch.float64), max_iter=200, rate_tol=1e-3)
    assert rec2.rate[-1] < 1e-3 and all(r >= 1e-3 for r in rec2.rate[:-1])
    assert rec2.stop.startswith("convergence rate")


def test_wolfe_conditions_hold():
    x = torch.tensor([-1.2, 1.0], dtype=torch.float64)
    f0, g0 = rosenbrock(x)
    d = -g0
    for a0 in (1e-4, 1e-2, 1.0):
        a, f, g = wolfe_search(rosenbrock, x, f0, g0, d, a0)
        assert f <= f0 + 1e-4 * a * float(g0 @ d)
        assert abs(float(g @ d)) <= 0.9 * abs(float(g0 @ d))
    assert wolfe_search(rosenbrock, x, f0, g0, g0, 1.0) is None     # not a descent direction


def test_cosine_similarity_and_rate():
    v = np.array([1.0, -2.0, 3.0])
    assert cosine_similarity(v, 2.5 * v) == pytest.approx(1.0)
    assert cosine_similarity(v, -v) == pytest.approx(-1.0)
    assert cosine_similarity([1.0, 0.0], [0.0, 3.0]) == pytest.approx(0.0)
    assert cosine_similarity(torch.tensor([3.0, 4.0]), np.array([4.0, 3.0])) == pytest.approx(24.0 / 25.0)
    assert convergence_rate(10.0, 9.99) == pytest.approx(1e-3)


def test_line_search_backs_off_from_non_finite_values():
    def fg(x):
        if float(x[0]) > 0.5:
            return float("nan"), torch.full_like(x, float("nan"))
        return float((x[0] - 0.4) ** 2), 2 * (x - 0.4)
    x0 = torch.zeros(1, dtype=torch.float64)
    f0, g0 = fg(x0)
    a, f, g = wolfe_search(fg, x0, f0, g0, -g0, 10.0)
    assert np.isfinite(f) and f < f0


def test_lbfgs_diagonal_initial_inverse_hessian():
    """With h0 the exact inverse of a diagonal Hessian the first step lands on the minimum;
    the identity start on the same ill-conditioned quadratic does not; on a non-diagonal
    quadratic the scaled diagonal still converges."""
    a = torch.logspace(-2, 2, 50, dtype=torch.float64)
    x0 = torch.linspace(-1.0, 2.0, 50, dtype=torch.float64)

    def quad(x):
        return float(0.5 * torch.sum(a * x * x)), a * x

    f0 = quad(x0)[0]
    x1, rec1 = lbfgs(quad, x0, max_iter=1, rate_tol=0.0, h0=1.0 / a)
    assert rec1.phi[-1] <= 1e-20 * f0 and float(x1.abs().max()) <= 1e-10
    _, rec_id = lbfgs(quad, x0, max_iter=1, rate_tol=0.0)
    assert rec_id.phi[-1] > 1e-6 * f0
    rng = np.random.default_rng(4)
    B = rng.standard_normal((30, 30))
    H = torch.tensor(B @ B.T + np.diag(np.logspace(-1, 2, 30)))
    xs = torch.tensor(rng.standard_normal(30))

    def quad2(x):
        r = x - xs
        return float(0.5 * r @ H @ r), H @ r

    x, _ = lbfgs(quad2, torch.zeros(30, dtype=torch.float64), max_iter=300, rate_tol=0.0,
                 h0=1.0 / torch.diagonal(H))
    assert np.allclose(x.numpy(), xs.numpy(), atol=1e-6)
