"""Pins of the cubic B-spline parameterization oracle: the textbook values of the uniform
cubic B-spline (2/3 at its node, 1/6 one spacing away, 1/48 at 1.5 spacings, 0 beyond 2),
partition of unity and reproduction of linear functions on the grid (so constant and
linear coefficient sequences give constant and linear models), symmetry of the kernel, the
transpose by the dot-product test, and separability against a brute-force double sum."""
import numpy as np
import pytest

from oracle import bspline as BS


def test_kernel_values():
    assert BS.kernel(0.0) == pytest.approx(2.0 / 3.0, abs=1e-16)
    assert BS.kernel(1.0) == pytest.approx(1.0 / 6.0, abs=1e-16)
    assert BS.kernel(-1.0) == pytest.approx(1.0 / 6.0, abs=1e-16)
    assert BS.kernel(1.5) == pytest.approx(1.0 / 48.0, abs=1e-16)
    assert BS.kernel(0.5) == pytest.approx(23.0 / 48.0, abs=1e-16)
    assert BS.kernel(2.0) == 0.0 and BS.kernel(-2.5) == 0.0


@pytest.mark.parametrize("n,D", [(1, 1), (7, 1), (30, 4), (101, 10), (100, 10)])
def test_partition_of_unity_and_linear_reproduction(n, D):
    B = BS.basis(n, D)
    assert B.shape == (n, BS.nodes(n, D))
    assert np.allclose(B.sum(axis=1), 1.0, rtol=0, atol=1e-14)
    # coefficients at the node positions reproduce a linear function exactly
    pos = (np.arange(B.shape[1]) - 1.0) * D
    assert np.allclose(B @ (3.0 + 0.25 * pos), 3.0 + 0.25 * np.arange(n), rtol=0, atol=1e-12)
    # every node's support reaches the grid (no node is wasted)
    assert np.all(B.max(axis=0) > 0.0) or n < 2


def test_expand_brute_force_and_dot_product():
    rng = np.random.default_rng(2)
    nz, nx, Dz, Dx = 13, 47, 1, 10
    Nz, Nx = BS.nodes(nz, Dz), BS.nodes(nx, Dx)
    c = rng.standard_normal((2, Nz, Nx))
    m = BS.expand(c, nz, nx, Dz, Dx)
    i, j = 7, 23
    brute = sum(c[1, a, b] * BS.kernel((i - (a - 1) * Dz) / Dz) * BS.kernel((j - (b - 1) * Dx) / Dx)
                for a in range(Nz) for b in range(Nx))
    assert m[1, i, j] == pytest.approx(brute, rel=1e-13)
    g = rng.standard_normal((2, nz, nx))
    assert np.sum(m * g) == pytest.approx(np.sum(c * BS.adjoint(g, Dz, Dx)), rel=1e-12)
