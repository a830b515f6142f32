"""torch.autograd over the HIP kernels: gradients against central finite differences of the
GPU objective, and the two formulations (data map + loss, misfit) against each other.

FD protocol: relative step h = 1e-3 on smooth random perturbations of Vp, Vs and rho
(Gaussian-correlated, including the CPML strips), central differences of the FP64 misfit
of FP32 data. The FP32 forward's rounding noise in the misfit (~1e-6 relative, amplified by
kappa = ||d|| / ||r||) divided by the FD step sets the bar: 5e-3.
"""
import numpy as np
import pytest
import torch
from scipy.ndimage import gaussian_filter

from paper_2305_14130_amd import inputs

pytestmark = pytest.mark.gpu


def T(a):
    return torch.tensor(np.asarray(a, np.float32), device="cuda")


@pytest.fixture(scope="module")
def setup(gpu_lib):
    efwi = gpu_lib
    nt = 500
    w = inputs.parity_2d(nt=nt, blob_amp=0.3)
    sh = w.shots[0]
    grid = efwi.make_grid(w.nz, w.nx, w.dz, w.dx, w.dt, nt, w.npml, w.pml_R, w.f0, w.vp_max)
    shot = efwi.Shot(sh.src_iz, sh.src_ix, sh.ch_iz, sh.ch_ix)
    src = T(np.outer(sh.M, w.stf))
    m = T(w.m_start)
    d_obs = efwi.model_forward(grid, shot, T(w.m_true), src)
    return efwi, grid, shot, src, m, d_obs


def smooth_dirs(shape, n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        d = np.stack([gaussian_filter(rng.standard_normal(shape[1:]), 4.0) for _ in range(3)])
        out.append(d / np.abs(d).max())
    return out


def test_shot_misfit_matches_fd(setup):
    from paper_2305_14130_amd.autograd import ShotMisfit
    efwi, grid, shot, src, m, d_obs = setup
    mv = m.clone().requires_grad_(True)
    phi = ShotMisfit.apply(mv, src, d_obs, grid, shot)
    phi.backward()
    g = mv.grad.double()
    h = 1e-3
    for dm in smooth_dirs(m.shape, 4, 3):
        dmt = (m * T(dm)).double()
        pp = ShotMisfit.apply((m.double() + h * dmt).float(), src, d_obs, grid, shot).item()
        pm = ShotMisfit.apply((m.double() - h * dmt).float(), src, d_obs, grid, shot).item()
        fd = (pp - pm) / (2 * h)
        an = float((g * dmt).sum())
        assert abs(fd - an) / abs(an) < 5e-3, (fd, an)


def test_shot_data_with_custom_loss(setup):
    """m -> d through ShotData, then a non-L2 loss in torch: backward runs J^T on the loss's
    data-space gradient; checked by FD and, for the L2 loss, against ShotMisfit."""
    from paper_2305_14130_amd.autograd import ShotData, ShotMisfit
    efwi, grid, shot, src, m, d_obs = setup

    def l2(mm):
        d = ShotData.apply(mm, src, grid, shot)
        return 0.5 * ((d.double() - d_obs.double()) ** 2).sum()

    def corr(mm):  # 1 - normalized zero-lag correlation per trace
        d = ShotData.apply(mm, src, grid, shot).double()
        o = d_obs.double()
        return (1.0 - (d * o).sum(1) / (d.norm(dim=1) * o.norm(dim=1))).sum()

    mv = m.clone().requires_grad_(True)
    l2(mv).backward()
    g_data = mv.grad.clone()
    mv2 = m.clone().requires_grad_(True)
    ShotMisfit.apply(mv2, src, d_obs, grid, shot).backward()
    e = float((g_data - mv2.grad).norm() / mv2.grad.norm())
    assert e < 1e-4, e
    mv3 = m.clone().requires_grad_(True)
    corr(mv3).backward()
    g = mv3.grad.double()
    h = 1e-3
    for dm in smooth_dirs(m.shape, 2, 5):
        dmt = (m * T(dm)).double()
        fd = (corr((m.double() + h * dmt).float()).item() - corr((m.double() - h * dmt).float()).item()) / (2 * h)
        an = float((g * dmt).sum())
        assert abs(fd - an) / abs(an) < 5e-3, (fd, an)


def test_extended_misfit_fd(setup):
    """eq.(8) with three shots on their own components plus the consistency penalty."""
    from paper_2305_14130_amd.autograd import extended_misfit
    efwi, grid, shot, src, m, d_obs = setup
    ns = 3
    w = inputs.parity_2d(nt=grid.nt, blob_amp=0.3)
    shots = [efwi.Shot(50, 40 + 30 * k, shot.ch_iz, shot.ch_ix) for k in range(ns)]
    srcs = torch.stack([src * (1.0 + 0.2 * k) for k in range(ns)])
    obs = torch.cat([efwi.model_forward(grid, shots[k], T(w.m_true), srcs[k]) for k in range(ns)])
    rng = np.random.default_rng(9)
    m_ext = torch.stack([m * (1.0 + 0.005 * T(gaussian_filter(rng.standard_normal(m.shape), (0, 3, 3))))
                         for _ in range(ns)]).contiguous()
    b_np, sink_np = inputs.hard_sinkholes(ns, grid.nz, grid.nx, [50] * ns, [40 + 30 * k for k in range(ns)], 4, 10)
    b, sink = T(b_np), torch.tensor(sink_np, device="cuda")
    # eta balances the penalty against the data term at this scale
    eta = 1e-5
    mv = m_ext.clone().requires_grad_(True)
    f = extended_misfit(mv, srcs, obs, grid, shots, b, sink, eta)
    f.backward()
    g = mv.grad.double()
    h = 1e-3
    for k, dm in enumerate(smooth_dirs(m.shape, 2, 11)):
        dmt = torch.stack([(m * T(dm)).double() * (1 + 0.3 * q) for q in range(ns)])
        fp = extended_misfit((m_ext.double() + h * dmt).float(), srcs, obs, grid, shots, b, sink, eta).item()
        fm = extended_misfit((m_ext.double() - h * dmt).float(), srcs, obs, grid, shots, b, sink, eta).item()
        fd = (fp - fm) / (2 * h)
        an = float((g * dmt).sum())
        assert abs(fd - an) / abs(an) < 5e-3, (k, fd, an)


def test_checkpoint_interval_choice(setup):
    from paper_2305_14130_amd.autograd import checkpoint_interval
    efwi, grid, shot, src, m, d_obs = setup
    assert checkpoint_interval(grid, shot) == grid.nt          # small history fits
    assert checkpoint_interval(grid, shot, budget_fraction=1e-9) == 0


def test_full_size_differentiation(gpu_lib):
    """The differentiation workload at full size: 1200 x 4000 at 2 m, nt = 8000 at 0.2 ms,
    one of its 32 shots with the 2000 channels. ShotMisfit's gradient, with the default
    ceil(sqrt(nt)) = 90-step checkpoints and recomputation, is bitwise the gradient from the
    longest interval that fits half the free HBM (the whole history when it fits), and it
    agrees with central differences (h = 1e-3 relative) of the FP64 misfit of the FP32 data
    on 10 seeded smooth perturbations, to the bar stated above."""
    from paper_2305_14130_amd.autograd import ShotMisfit
    efwi = gpu_lib
    w = inputs.differentiation_2d(nshots=1)
    sh = w.shots[0]
    grid = efwi.make_grid(w.nz, w.nx, w.dz, w.dx, w.dt, w.nt, w.npml, w.pml_R, w.f0, w.vp_max)
    shot = efwi.Shot(sh.src_iz, sh.src_ix, sh.ch_iz, sh.ch_ix)
    src = T(np.outer(sh.M, w.stf))
    m = T(w.m_start)
    d_obs = efwi.model_forward(grid, shot, T(w.m_true), src)
    mv = m.clone().requires_grad_(True)
    ShotMisfit.apply(mv, src, d_obs, grid, shot).backward()
    g = mv.grad
    L = efwi.plan_interval(grid, shot, torch.cuda.mem_get_info()[0] // 2)
    assert L > 90
    long_shot = efwi.Shot(sh.src_iz, sh.src_ix, sh.ch_iz, sh.ch_ix, ckpt_interval=L)
    g_long, _ = efwi.shot_gradient(grid, long_shot, m, src, d_obs)
    assert torch.equal(g, g_long), L
    del g_long

    def phi(mm):
        d = efwi.model_forward(grid, shot, mm, src)
        return 0.5 * float(((d.double() - d_obs.double()) ** 2).sum())

    g = g.double()
    h = 1e-3
    for k, dm in enumerate(smooth_dirs(m.shape, 10, 17)):
        dmt = (m * T(dm)).double()
        fd = (phi((m.double() + h * dmt).float()) - phi((m.double() - h * dmt).float())) / (2 * h)
        an = float((g * dmt).sum())
        assert abs(fd - an) / abs(an) < 5e-3, (k, fd, an)
