"""FP64 oracle: the cubic B-spline model parameterization of the field example's smoothing
regularization (model described by cubic B-spline coefficients on a coarse node grid).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Definition (de Boor's uniform cubic B-spline, written out): along an axis with node spacing
D grid cells, node k (k = 0 .. N-1) sits at grid position (k - 1) D and carries the basis
function B((z - (k - 1) D) / D) with
    B(t) = 2/3 - t^2 + |t|^3 / 2        for |t| < 1,
    B(t) = (2 - |t|)^3 / 6              for 1 <= |t| < 2,
    B(t) = 0                            otherwise.
N = ceil((n - 1) / D) + 3 nodes cover grid points 0 .. n-1 with every node whose support
reaches them, so the basis sums to one on the grid. A 2D model plane is
m[i][j] = sum_a sum_b c[a][b] B_a(i) B_b(j) (Bz c Bx^T), and the gradient with respect to
the coefficients is Bz^T g Bx. Node spacings are whole numbers of cells (a reading: the
paper's 50 m by 1 m falls on its grid).
"""
from __future__ import annotations

import numpy as np


def kernel(t):
    a = np.abs(np.asarray(t, np.float64))
    return np.where(a < 1.0, 2.0 / 3.0 - a * a + 0.5 * a ** 3, np.where(a < 2.0, (2.0 - a) ** 3 / 6.0, 0.0))


def nodes(n, D):
    return int(-(-(n - 1) // D)) + 3


def basis(n, D):
    """[n][N] matrix of the axis: entry (i, k) = B((i - (k - 1) D) / D)."""
    N = nodes(n, D)
    i = np.arange(n, dtype=np.float64)[:, None]
    k = np.arange(N, dtype=np.float64)[None, :]
    return kernel((i - (k - 1.0) * D) / D)


def expand(c, nz, nx, Dz, Dx):
    """m = Bz c Bx^T for every plane of c [..][Nz][Nx]."""
    Bz, Bx = basis(nz, Dz), basis(nx, Dx)
    return np.einsum("ia,...ab,jb->...ij", Bz, np.asarray(c, np.float64), Bx)


def adjoint(g, Dz, Dx):
    """c_bar = Bz^T g Bx for every plane of g [..][nz][nx]."""
    g = np.asarray(g, np.float64)
    nz, nx = g.shape[-2:]
    Bz, Bx = basis(nz, Dz), basis(nx, Dx)
    return np.einsum("ia,...ij,jb->...ab", Bz, g, Bx)
