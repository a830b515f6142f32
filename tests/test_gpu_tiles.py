"""Tile shape of the fused 2D time-step kernels: every node is computed by the same
arithmetic whichever tile (and halo) holds it, so gradients, misfits and data must be
bitwise identical for every tile height; the autotuner must pick valid heights."""
import numpy as np
import pytest
import torch

from paper_2305_14130_amd import inputs

pytestmark = pytest.mark.gpu


def T(a):
    return torch.tensor(np.asarray(a, np.float32), device="cuda")


@pytest.fixture(scope="module")
def case(gpu_lib):
    efwi = gpu_lib
    w = inputs.parity_2d(nt=300, blob_amp=0.3)
    grid = efwi.make_grid(w.nz, w.nx, w.dz, w.dx, w.dt, w.nt, w.npml, w.pml_R, w.f0, w.vp_max)
    sh = w.shots[0]
    shot = efwi.Shot(sh.src_iz, sh.src_ix, sh.ch_iz, sh.ch_ix, ckpt_interval=23)
    m, mt = T(w.m_start), T(w.m_true)
    src = T(np.outer(sh.M, w.stf))
    d_obs = efwi.model_forward(grid, shot, mt, src)
    return efwi, grid, shot, m, src, d_obs


def _run(case, rows):
    efwi, grid, shot, m, src, d_obs = case
    efwi.set_tile_rows(*rows)
    d = torch.empty_like(d_obs)
    g, phi = efwi.shot_gradient(grid, shot, m, src, d_obs, d_out=d)
    fb = efwi.model_adjoint(grid, shot, m, d_obs)
    torch.cuda.synchronize()
    return g.clone(), phi.item(), d.clone(), fb.clone()


def test_results_do_not_depend_on_tile_rows(case):
    efwi = case[0]
    saved = efwi.get_tile_rows()
    try:
        ref = _run(case, (8, 8))
        for rows in ((12, 16), (16, 12), (16, 16), (12, 8)):
            got = _run(case, rows)
            assert torch.equal(got[0], ref[0]), rows
            assert got[1] == ref[1], rows
            assert torch.equal(got[2], ref[2]), rows
            assert torch.equal(got[3], ref[3]), rows
    finally:
        efwi.set_tile_rows(*saved)


def test_autotune_picks_valid_rows(case):
    efwi, grid, shot, m, src, d_obs = case
    saved = efwi.get_tile_rows()
    try:
        ref = _run(case, (8, 8))
        f, a = efwi.autotune(grid, shot, m, src, steps=12)
        assert f in (8, 12, 16) and a in (8, 12, 16)
        assert efwi.get_tile_rows() == (f, a)
        g, phi = efwi.shot_gradient(grid, shot, m, src, d_obs)
        assert torch.equal(g, ref[0]) and phi.item() == ref[1]
    finally:
        efwi.set_tile_rows(*saved)
