"""GPU (HIP) vs FP64 oracle parity of the model-extension operators through the C ABI:
the zones of influence of eq.(10) (efwi_zoi_weights) and the final model S_w W m~ of
eq.(9) (efwi_final_model).

Bars: sinkhole flags bit-exact (both sides decide d^2 < 1 in FP64 with the same summation
order, and the grids put nodes exactly on sinkhole edges); weights within one FP32 ulp of
the oracle's FP64 value rounded to FP32 (the kernel computes in FP64 and rounds once; the
libraries' cos, pow and log may differ in the last FP64 bit); final model within 2 FP32
ulps (FP64 sums in a different order, rounded once).
"""
import numpy as np
import pytest
import torch

from oracle import regularizer as R
from oracle import zoi as Z

pytestmark = pytest.mark.gpu


def f32(a):
    return np.asarray(a, np.float32)


def zones_2d():
    th = np.deg2rad(25.0)
    Rm = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    C = Rm @ np.diag([1 / 35.0**2, 1 / 80.0**2]) @ Rm.T
    return [
        # axis-aligned sinkhole 30 m x 60 m around node (60, 100): nodes on its edges
        {"src": (300.0, 0.0, 500.0), "icov": (1 / 900.0, 0.0, 1 / 3600.0, 0.0, 0.0, 0.0),
         "box": (200.0, 420.0, 0.0, 0.0, 150.0, 1100.0), "taper": 60.0},
        # rotated sinkhole (off-diagonal term), off-node centre
        {"src": (312.5, 0.0, 802.5), "icov": (C[0, 0], 0.0, C[1, 1], 0.0, C[0, 1], 0.0),
         "box": (150.0, 500.0, 0.0, 0.0, 400.0, 1200.0), "taper": 100.0},
        # step transition (taper 0), box touching the grid edge
        {"src": (100.0, 0.0, 50.0), "icov": (1 / 400.0, 0.0, 1 / 400.0, 0.0, 0.0, 0.0),
         "box": (0.0, 250.0, 0.0, 0.0, 0.0, 600.0), "taper": 0.0},
        # box outside the grid: the whole grid is in the transition
        {"src": (550.0, 0.0, 1250.0), "icov": (1 / 2500.0, 0.0, 1 / 2500.0, 0.0, 0.0, 0.0),
         "box": (700.0, 800.0, 0.0, 0.0, 1400.0, 1500.0), "taper": 300.0},
    ]


def to_c(efwi, zn):
    return efwi.make_zone(zn["src"], zn["icov"], zn["box"], zn["taper"])


def rounded(zn):
    """The oracle gets the same FP32-rounded zone parameters the C ABI carries."""
    return {k: (tuple(float(np.float32(v)) for v in zn[k]) if k != "taper" else float(np.float32(zn[k])))
            for k in zn}


def check_weights(b_gpu, s_gpu, b_ref, s_ref):
    assert np.array_equal(s_gpu.astype(bool), s_ref)
    ref32 = f32(b_ref)
    assert np.all(np.abs(b_gpu - ref32) <= np.spacing(ref32)), float(np.max(np.abs(b_gpu - ref32)))


@pytest.mark.parametrize("n,nu", [(2.0, 0.9), (3.5, 0.05)])
def test_zoi_weights_2d(gpu_lib, n, nu):
    efwi = gpu_lib
    nz, nx, h = 120, 261, 5.0
    grid = efwi.make_grid(nz, nx, h, h, 1e-4, 10, 0, 1e-3, 10.0, 4000.0)
    zs = zones_2d()
    b, sink = efwi.zoi_weights(grid, [to_c(efwi, z) for z in zs], n, nu)
    torch.cuda.synchronize()
    b_ref, s_ref = Z.zoi_weights((nz, nx), (h, h), [rounded(z) for z in zs], float(np.float32(n)),
                                 float(np.float32(nu)))
    assert s_ref[0].sum() > 50 and s_ref[0, 60, 100] and not s_ref[0, 66, 100] and not s_ref[0, 60, 112]
    check_weights(b.cpu().numpy(), sink.cpu().numpy(), b_ref, s_ref)


def test_zoi_weights_more_zones_than_a_launch(gpu_lib):
    """21 zones (the kernel takes up to 16 per launch): each zone's weights and flags land
    in its own slot, the second launch's too."""
    efwi = gpu_lib
    nz, nx, h = 60, 131, 5.0
    grid = efwi.make_grid(nz, nx, h, h, 1e-4, 10, 0, 1e-3, 10.0, 4000.0)
    zs = [{"src": (80.0 + 5.0 * (s % 7), 0.0, 30.0 * s), "icov": (1 / (400.0 + 50.0 * s), 0.0, 1 / 1600.0, 0.0, 0.0, 0.0),
           "box": (40.0, 220.0, 0.0, 0.0, max(0.0, 30.0 * s - 100.0), 30.0 * s + 100.0), "taper": 20.0 + 5.0 * s}
          for s in range(21)]
    b, sink = efwi.zoi_weights(grid, [to_c(efwi, z) for z in zs], 2.5, 0.7)
    torch.cuda.synchronize()
    b_ref, s_ref = Z.zoi_weights((nz, nx), (h, h), [rounded(z) for z in zs], 2.5, float(np.float32(0.7)))
    assert all(s_ref[s].any() for s in range(21))
    check_weights(b.cpu().numpy(), sink.cpu().numpy(), b_ref, s_ref)


def test_zoi_weights_3d(gpu_lib):
    efwi = gpu_lib
    nz, ny, nx, h = 20, 24, 28, 5.0
    grid = efwi.make_grid3d(nz, ny, nx, h, h, h, 1e-4, 10, 0, 1e-3, 10.0, 4000.0)
    A = np.array([[1 / 400.0, 1e-4, -2e-4], [1e-4, 1 / 900.0, 3e-4], [-2e-4, 3e-4, 1 / 1600.0]])
    zs = [{"src": (50.0, 60.0, 70.0), "icov": (A[0, 0], A[1, 1], A[2, 2], A[0, 1], A[0, 2], A[1, 2]),
           "box": (20.0, 80.0, 10.0, 100.0, 20.0, 120.0), "taper": 25.0},
          {"src": (40.0, 55.0, 65.0), "icov": (1 / 225.0, 1 / 400.0, 1 / 625.0, 0.0, 0.0, 0.0),
           "box": (0.0, 95.0, 0.0, 115.0, 0.0, 135.0), "taper": 0.0}]
    b, sink = efwi.zoi_weights(grid, [to_c(efwi, z) for z in zs], 2.0, 0.8)
    torch.cuda.synchronize()
    b_ref, s_ref = Z.zoi_weights((nz, ny, nx), (h, h, h), [rounded(z) for z in zs], 2.0, float(np.float32(0.8)))
    assert s_ref[1, 8, 11, 13]
    check_weights(b.cpu().numpy(), sink.cpu().numpy(), b_ref, s_ref)


def test_final_model_and_zoi_regularizer(gpu_lib):
    """eq.(9) on a random extension with the oracle's ZOI weights; a consistent extension
    S^T m returns m; the regularizer with these soft weights matches the oracle too."""
    efwi = gpu_lib
    nz, nx, h = 60, 130, 5.0
    grid = efwi.make_grid(nz, nx, h, h, 1e-4, 10, 0, 1e-3, 10.0, 4000.0)
    zs = [{"src": (150.0, 0.0, 100.0 + 110.0 * s), "icov": (1 / 400.0, 0.0, 1 / 1600.0, 0.0, 0.0, 0.0),
           "box": (50.0, 250.0, 0.0, 0.0, 40.0 + 100.0 * s, 300.0 + 100.0 * s), "taper": 80.0} for s in range(5)]
    b_ref, s_ref = Z.zoi_weights((nz, nx), (h, h), [rounded(z) for z in zs], 2.0, float(np.float32(0.9)))
    b32 = f32(b_ref)
    rng = np.random.default_rng(5)
    m = np.stack([np.full((nz, nx), 3000.0), np.full((nz, nx), 1700.0), np.full((nz, nx), 2400.0)])
    m_ext = f32(m[None] * (1 + 0.02 * rng.standard_normal((5, 3, nz, nx))))
    bt = torch.tensor(b32, device="cuda")
    st = torch.tensor(s_ref.astype(np.uint8), device="cuda")
    out = efwi.final_model(grid, torch.tensor(m_ext, device="cuda"), bt, st).cpu().numpy()
    ref = R.final_model(m_ext.astype(np.float64), b32.astype(np.float64), s_ref)
    ref32 = f32(ref)
    assert np.all(np.abs(out - ref32) <= 2 * np.spacing(np.abs(ref32)))
    cons = f32(np.broadcast_to(f32(m)[None], (5, 3, nz, nx)).copy())
    out_c = efwi.final_model(grid, torch.tensor(cons, device="cuda"), bt, st).cpu().numpy()
    assert np.all(np.abs(out_c - f32(m)) <= 2 * np.spacing(f32(m)))
    # regularizer with soft ZOI weights
    g = torch.zeros((5, 3, nz, nx), dtype=torch.float32, device="cuda")
    phi = efwi.extension_regularizer(grid, torch.tensor(m_ext, device="cuda"), bt, st, 0.7, g)
    phi_o, g_o = R.regularizer(m_ext.astype(np.float64), b32.astype(np.float64), s_ref, float(np.float32(0.7)))
    assert abs(phi.item() - phi_o) / phi_o <= 1e-6
    gg = g.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(gg - g_o) / np.linalg.norm(g_o) <= 1e-6
