"""Pins of the 16-bit checkpoint encodings and of the oracle's checkpointed gradient.

* The checkpointed schedule with exact snapshots reproduces the plain full-history gradient
  to round-off (pins the segment bookkeeping: boundaries, the kept last segment, restarts).
* Encodings: the largest magnitude maps to an exact code (FP16: 16384, BF16: 1.0), relative
  rounding error at most half a unit in the last place (2^-11 FP16, 2^-8 BF16) over the
  normal range, ties to even, zeros stay zeros.
* Compressed snapshots perturb the gradient by a small, nonzero amount.
"""
import numpy as np
import pytest

from oracle import checkpoint as C
from oracle import elastic2d as E
from paper_2305_14130_amd.inputs import parity_2d


@pytest.mark.parametrize("codec,ulp", [("fp16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
def test_roundtrip_error_bounds(codec, ulp):
    rng = np.random.default_rng(0)
    x = rng.standard_normal(20000) * 10.0 ** rng.uniform(-3, 3, 20000)
    y = C.roundtrip(x, codec)
    mx = np.abs(x).max()
    assert np.abs(y).max() == mx                       # the max-abs element is exact
    big = np.abs(x) > mx * 2.0 ** -12                  # normal range of both codes
    assert np.all(np.abs(y - x)[big] <= ulp * np.abs(x)[big] * (1 + 1e-12))
    assert np.all(C.roundtrip(np.zeros(7), codec) == 0.0)


def test_ties_round_to_even():
    # BF16 (scale = max = 2): codes 0.5 + 2^-9 and 0.5 + 3 2^-9 are ties between BF16
    # neighbours 2^-8 apart; they round to the even neighbours 0.5 and 0.5 + 2^-7
    x = np.array([2.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8])
    y = C.roundtrip(x, "bf16")
    assert y[1] == 1.0 and y[2] == 1.0 + 2.0 ** -6
    # FP16 (scale max/2^14 with max = 16384 here): 2 + 2^-10 is halfway between 2 and 2 + 2^-9
    x = np.array([16384.0, 2.0 + 2.0 ** -10, 2.0 + 3 * 2.0 ** -10])
    y = C.roundtrip(x, "fp16")
    assert y[1] == 2.0 and y[2] == 2.0 + 2.0 ** -8


def _case(nt=260):
    w = parity_2d(nt=nt, blob_amp=0.3)
    sh = w.shots[0]
    g = E.Grid2D(nz=w.nz, nx=w.nx, dz=w.dz, dx=w.dx, dt=w.dt, nt=nt, npml=w.npml, pml_R=w.pml_R,
                 pml_f0=w.f0, vp_max=w.vp_max)
    src = E.moment_tensor_series(sh.M, w.stf)
    d_obs = E.model_forward(g, w.m_true, sh.src_iz, sh.src_ix, src, sh.ch_iz, sh.ch_ix)
    return g, w.m_start, sh, src, d_obs


def test_checkpointed_schedule_equals_full_history():
    g, m, sh, src, d_obs = _case()
    g0, phi0, d0 = E.shot_gradient(g, m, sh.src_iz, sh.src_ix, src, sh.ch_iz, sh.ch_ix, d_obs)
    for L in (17, 64, 260):
        g1, phi1, d1 = E.shot_gradient_checkpointed(g, m, sh.src_iz, sh.src_ix, src, sh.ch_iz, sh.ch_ix, d_obs, L)
        assert np.array_equal(d0, d1) and phi0 == phi1
        assert np.max(np.abs(g1 - g0)) <= 1e-12 * np.max(np.abs(g0))


@pytest.mark.parametrize("codec,lo,hi", [("fp16", 1e-9, 1e-3), ("bf16", 1e-7, 3e-2)])
def test_compressed_snapshots_perturb_gradient_slightly(codec, lo, hi):
    g, m, sh, src, d_obs = _case()
    g0, _, _ = E.shot_gradient(g, m, sh.src_iz, sh.src_ix, src, sh.ch_iz, sh.ch_ix, d_obs)
    g1, _, _ = E.shot_gradient_checkpointed(g, m, sh.src_iz, sh.src_ix, src, sh.ch_iz, sh.ch_ix, d_obs, 17, codec)
    for k in range(3):
        e = np.linalg.norm(g1[k] - g0[k]) / np.linalg.norm(g0[k])
        assert lo < e < hi, (codec, k, e)


def _case3d(nt=48):
    from oracle import elastic3d as E3
    from paper_2305_14130_amd.inputs import ricker
    rng = np.random.default_rng(5)
    shape = (18, 20, 22)
    vp = 3000.0 * (1 + 0.05 * rng.standard_normal(shape))
    m = np.stack([vp, vp / 1.7, 2300.0 * (1 + 0.04 * rng.standard_normal(shape))])
    g = E3.Grid3D(*shape, 5.0, 5.0, 5.0, 0.4e-3, nt, npml=4, pml_f0=40.0, vp_max=3600.0)
    src = E3.moment_tensor_series([1.0, -0.4, 0.7, 0.3, -0.2, 0.5], ricker(nt, g.dt, 60.0) * 1e9)
    pos = (9, 10, 8)
    ch = (np.full(6, 9), np.full(6, 11), np.arange(7, 13))
    d_obs = E3.model_forward(g, m * np.array([1.05, 1.02, 1.0])[:, None, None, None], pos, src, ch)
    return E3, g, m, pos, src, ch, d_obs


def test_checkpointed_schedule_equals_full_history_3d():
    E3, g, m, pos, src, ch, d_obs = _case3d()
    g0, phi0, d0 = E3.shot_gradient(g, m, pos, src, ch, d_obs)
    for L in (7, 16, 48):
        g1, phi1, d1 = E3.shot_gradient_checkpointed(g, m, pos, src, ch, d_obs, L)
        assert np.array_equal(d0, d1) and phi0 == phi1
        assert np.max(np.abs(g1 - g0)) <= 1e-12 * np.max(np.abs(g0)), L


@pytest.mark.parametrize("codec,lo,hi", [("fp16", 1e-9, 1e-3), ("bf16", 1e-7, 3e-2)])
def test_compressed_snapshots_perturb_gradient_slightly_3d(codec, lo, hi):
    E3, g, m, pos, src, ch, d_obs = _case3d()
    g0, _, _ = E3.shot_gradient(g, m, pos, src, ch, d_obs)
    g1, _, d1 = E3.shot_gradient_checkpointed(g, m, pos, src, ch, d_obs, 7, codec)
    for k in range(3):
        e = np.linalg.norm(g1[k] - g0[k]) / np.linalg.norm(g0[k])
        assert lo < e < hi, (codec, k, e)
