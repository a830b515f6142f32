"""GPU (HIP) vs FP64 oracle parity of the cubic B-spline model parameterization through the
C ABI (efwi_bspline_expand / efwi_bspline_adjoint), and the inversion driver's use of it with
a gradient mask. Bar: within 2 FP32 ulps of the oracle's FP64 value on the same FP32 inputs
(the kernels sum in FP64 in another order and round once)."""
import numpy as np
import pytest
import torch

from oracle import bspline as BS
from paper_2305_14130_amd import inputs, invert

pytestmark = pytest.mark.gpu


def close32(out, ref):
    ref32 = np.asarray(ref, np.float32)
    return bool(np.all(np.abs(out - ref32) <= 2 * np.spacing(np.abs(ref32)) + 1e-30))


# (30, 1100, 3, 1): rows longer than a workgroup's column segment and node group (every
# column a node); (40, 5000, 1, 1990): a spacing whose weight table leaves room for only a
# few hundred staged cells; (700, 60, 1, 5): enough coefficient rows (3 x 702) for the
# transpose to take four rows per workgroup
@pytest.mark.parametrize("nz,nx,Dz,Dx", [(37, 150, 1, 10), (64, 65, 4, 7), (5, 3, 2, 9), (100, 400, 1, 10),
                                         (30, 1100, 3, 1), (40, 5000, 1, 1990), (700, 60, 1, 5)])
def test_expand_and_adjoint_parity(gpu_lib, nz, nx, Dz, Dx):
    efwi = gpu_lib
    rng = np.random.default_rng(nz + nx)
    Nz, Nx = BS.nodes(nz, Dz), BS.nodes(nx, Dx)
    assert (efwi.bspline_nodes(nz, Dz), efwi.bspline_nodes(nx, Dx)) == (Nz, Nx)
    c = np.asarray(rng.standard_normal((3, Nz, Nx)), np.float32)
    m = efwi.bspline_expand(torch.tensor(c, device="cuda"), nz, nx, Dz, Dx).cpu().numpy()
    assert close32(m, BS.expand(c.astype(np.float64), nz, nx, Dz, Dx))
    g = np.asarray(rng.standard_normal((3, nz, nx)), np.float32)
    cb = efwi.bspline_adjoint(torch.tensor(g, device="cuda"), Dz, Dx).cpu().numpy()
    assert close32(cb, BS.adjoint(g.astype(np.float64), Dz, Dx))
    # constant coefficients give a constant model (partition of unity)
    one = efwi.bspline_expand(torch.ones((1, Nz, Nx), device="cuda"), nz, nx, Dz, Dx).cpu().numpy()
    assert np.allclose(one, 1.0, rtol=0, atol=2e-7)


def test_parameterized_objective(gpu_lib):
    """With B-spline unknowns and a mask, the conventional objective is the grid objective at
    the expanded model, and its gradient the B-spline transpose of the masked grid gradient."""
    efwi = gpu_lib
    w = inputs.guided_wave_synthetic(nt=300)
    grid = efwi.make_grid(w.nz, w.nx, w.dz, w.dx, w.dt, w.nt, w.npml, w.pml_R, w.f0, w.vp_max)
    T = lambda a: torch.tensor(np.asarray(a, np.float32), device="cuda")
    d_obs = torch.cat([efwi.model_forward(grid, efwi.Shot(s.src_iz, s.src_ix, s.ch_iz, s.ch_ix), T(w.m_true),
                                          T(np.outer(s.M, w.stf))) for s in w.shots])
    mask = torch.zeros((w.nz, w.nx), device="cuda")
    mask[40:60] = 1.0
    spl = invert.ConventionalFWI(w, d_obs, bspline=(1, 10), mask=mask)
    grd = invert.ConventionalFWI(w, d_obs)
    x = 0.01 * torch.randn(spl.x0().shape, device="cuda")
    phi, gx = spl(x)
    rel = efwi.bspline_expand(x, w.nz, w.nx, 1, 10)
    phi2, g2 = grd(rel)
    assert phi == phi2
    assert torch.equal(gx, efwi.bspline_adjoint((g2 * mask).contiguous(), 1, 10))
    assert gx.shape == (2, efwi.bspline_nodes(w.nz, 1), efwi.bspline_nodes(w.nx, 10))
