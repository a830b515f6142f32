"""C ABI checks that need no GPU: the library loads, exports every function that
include/efwi.h declares, and validates arguments on the host before any HIP call."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "efwi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(efwi_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def efwi():
    from paper_2305_14130_amd import efwi as mod
    return mod


def test_every_declared_symbol_is_exported(efwi):
    names = _declared()
    assert len(names) >= 10
    lib = ctypes.CDLL(efwi.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(efwi.EXPORTED)


def test_version_and_status_strings(efwi):
    assert efwi.version().startswith("efwi-gfx950")
    assert efwi._lib.efwi_status_string(efwi.E_CFL) == b"EFWI_E_CFL"


def _ok_case(efwi):
    grid = efwi.make_grid(100, 200, 5.0, 5.0, 0.5e-3, 50, 20, 1e-3, 30.0, 4500.0)
    shot = efwi.Shot(50, 40, np.full(3, 50, np.int32), np.array([60, 63, 66], np.int32))
    return grid, shot


def test_validation_accepts_good_arguments(efwi):
    grid, shot = _ok_case(efwi)
    efwi.validate(grid, [shot])
    assert efwi.workspace_size(efwi.WS_GRADIENT, grid, [shot]) > 0


@pytest.mark.parametrize("mutate,status", [
    (lambda g, s: setattr(g, "dt", 1.0e-3), "E_CFL"),
    (lambda g, s: setattr(g, "nt", 0), "E_INVAL"),
    (lambda g, s: setattr(g, "dx", 0.0), "E_INVAL"),
    (lambda g, s: setattr(g, "ndim", 4), "E_INVAL"),
    (lambda g, s: (setattr(g, "ndim", 3), setattr(g, "dy", 5.0)), "E_RANGE"),   # ny = 1: no room for CPML
    (lambda g, s: setattr(s, "src_ix", 10), "E_RANGE"),            # inside the CPML strip
    (lambda g, s: setattr(s, "src_iz", 99), "E_RANGE"),
    (lambda g, s: setattr(s, "ch_ix", np.array([60, 63, 195], np.int32)), "E_RANGE"),
    (lambda g, s: setattr(s, "ch_ix", np.array([60, 63, 63], np.int32)), "E_INVAL"),   # duplicate node
    (lambda g, s: setattr(s, "wx", 230), "E_RANGE"),                # window beyond the model
    (lambda g, s: setattr(s, "ckpt_mode", 7), "E_INVAL"),
    (lambda g, s: setattr(s, "ckpt_interval", -1), "E_INVAL"),
])
def test_validation_errors(efwi, mutate, status):
    grid, shot = _ok_case(efwi)
    mutate(grid, shot)
    with pytest.raises(efwi.EfwiError) as ei:
        efwi.validate(grid, [shot])
    assert ei.value.status == getattr(efwi, status)
    assert efwi._lib.efwi_last_error()


def test_workspace_size_grows_with_checkpoint_interval(efwi):
    grid, shot = _ok_case(efwi)
    small = efwi.workspace_size(efwi.WS_GRADIENT, grid, [shot])
    shot.ckpt_interval = 10**6
    full = efwi.workspace_size(efwi.WS_GRADIENT, grid, [shot])
    assert full > small
    assert efwi.workspace_size(efwi.WS_FORWARD, grid, [shot]) < small


def test_plan_interval_fits_the_budget(efwi):
    grid, shot = _ok_case(efwi)
    nt = grid.nt

    def need(L):
        shot.ckpt_interval = L
        return efwi.workspace_size(efwi.WS_GRADIENT, grid, [shot])

    assert efwi.plan_interval(grid, shot, 1 << 40) == nt
    sq = int(np.ceil(np.sqrt(nt)))
    L = efwi.plan_interval(grid, shot, need(sq))   # fewer checkpoint slots may let a larger L fit
    assert L >= sq and need(L) <= need(sq)
    budget = (need(sq) + need(nt)) // 2
    L = efwi.plan_interval(grid, shot, budget)
    assert sq <= L < nt and need(L) <= budget < need(L + 1)
    with pytest.raises(efwi.EfwiError) as ei:
        efwi.plan_interval(grid, shot, need(sq) - 1)
    assert ei.value.status == efwi.E_WORKSPACE
    assert efwi.recompute_fraction(grid, nt) == 0.0
    assert efwi.recompute_fraction(grid, 10) == (5 - 1) * 10 / nt


def test_tile_rows_setting(efwi):
    f0, a0 = efwi.get_tile_rows()
    try:
        efwi.set_tile_rows(16, 12)
        assert efwi.get_tile_rows() == (16, 12)
        efwi.set_tile_rows(0, 8)            # 0 keeps the forward value
        assert efwi.get_tile_rows() == (16, 8)
        for bad in ((7, 0), (0, 32), (-8, 8)):
            with pytest.raises(efwi.EfwiError) as ei:
                efwi.set_tile_rows(*bad)
            assert ei.value.status == efwi.E_INVAL
        assert efwi.get_tile_rows() == (16, 8)
    finally:
        efwi.set_tile_rows(f0, a0)


def test_autotune_workspace_size(efwi):
    grid, shot = _ok_case(efwi)
    sc = shot.c_struct()
    assert efwi._lib.efwi_autotune_workspace_size(grid, sc, 16) > 0
    assert efwi._lib.efwi_autotune_workspace_size(grid, sc, 0) == 0
    grid.ndim = 3
    assert efwi._lib.efwi_autotune_workspace_size(grid, sc, 16) == 0


def test_batch_waves_follow_the_cache_budget(efwi):
    """Small windows share a wave; 1000 x 3000 shots, whose per-step state alone fills most
    of the 256 MB Infinity Cache, get one wave each; a small workspace splits waves too."""
    small = efwi.make_grid(100, 200, 5.0, 5.0, 0.5e-3, 50, 20, 1e-3, 30.0, 4500.0)
    shots = [efwi.Shot(50, 40 + 10 * k, np.full(3, 50, np.int32), np.array([60, 63, 66], np.int32))
             for k in range(6)]
    big_ws = efwi.workspace_size(efwi.WS_BATCH, small, shots)
    assert efwi.batch_waves(small, shots, big_ws) == [list(range(6))]
    one = efwi.workspace_size(efwi.WS_BATCH, small, shots[:1])
    assert efwi.batch_waves(small, shots, one) == [[k] for k in range(6)]
    with pytest.raises(efwi.EfwiError) as ei:
        efwi.batch_waves(small, shots, one // 2)
    assert ei.value.status == efwi.E_WORKSPACE
    large = efwi.make_grid(1000, 3000, 2.5, 2.5, 0.25e-3, 40, 40, 1e-3, 60.0, 3990.0)
    bshots = [efwi.Shot(500, 1000 + 100 * k, np.full(4, 500, np.int32), np.array([600, 610, 620, 630], np.int32))
              for k in range(3)]
    ws = efwi.workspace_size(efwi.WS_BATCH, large, bshots)
    assert efwi.batch_waves(large, bshots, ws) == [[0], [1], [2]]
    # the per-step bound can be lifted (waves sized by the workspace alone) and restored
    assert efwi.get_wave_cache_bytes() == 256 << 20
    try:
        efwi.set_wave_cache_bytes(-1)
        assert efwi.batch_waves(large, bshots, ws) == [[0, 1, 2]]
        efwi.set_wave_cache_bytes(1)                      # below one shot: still one shot per wave
        assert efwi.batch_waves(small, shots, big_ws) == [[k] for k in range(6)]
    finally:
        efwi.set_wave_cache_bytes(0)
    assert efwi.get_wave_cache_bytes() == 256 << 20


def test_batch_waves_pack_largest_first(efwi):
    """Uneven windows are packed first fit, largest first: windows of 600, 500, 400 and 500
    columns in a workspace that holds 600 + 400 or 500 + 500 but not 600 + 500 go into two
    waves (in order they would take three); each wave lists its shots ascending. Two lanes
    (the default) plan each half of the workspace when one lane would take several waves and
    every shot fits a half; other lane counts are refused."""
    grid = efwi.make_grid(120, 700, 5.0, 5.0, 0.5e-3, 200, 10, 1e-3, 30.0, 4500.0)

    def shot(wx, x0):
        return efwi.Shot(60, x0 + wx // 2, np.full(3, 60, np.int32), np.array([x0 + 20, x0 + 23, x0 + 26], np.int32),
                         z0=0, x0=x0, wz=120, wx=wx)

    sh = [shot(600, 0), shot(500, 100), shot(400, 200), shot(500, 50)]
    pair = lambda a, b: efwi.workspace_size(efwi.WS_BATCH, grid, [sh[a], sh[b]])
    ws = max(pair(0, 2), pair(1, 3))
    assert pair(0, 1) > ws and pair(1, 2) + efwi.workspace_size(efwi.WS_GRADIENT, grid, [sh[3]]) > ws
    assert efwi.get_wave_lanes() == 2                                    # the default
    assert efwi.batch_waves(grid, sh, ws) == [[0, 2], [1, 3]]            # a shot exceeds half: one lane
    try:
        efwi.set_wave_lanes(1)
        assert efwi.get_wave_lanes() == 1
        assert efwi.batch_waves(grid, sh, ws) == [[0, 2], [1, 3]]
        assert efwi.batch_waves(grid, sh, 2 * ws) == [[0, 1, 2, 3]]
        efwi.set_wave_lanes(2)
        assert efwi.get_wave_lanes() == 2
        assert efwi.batch_waves(grid, sh, 2 * ws) == [[0, 1, 2, 3]]     # one wave holds all: one lane
        assert efwi.batch_waves(grid, sh[:1], 2 * ws) == [[0]]
        assert efwi.batch_waves(grid, sh, 2 * ws, with_lanes=True)[1] == 1
        efwi.set_wave_cache_bytes(1)                # one shot per wave: the whole bound is exceeded, one lane
        assert efwi.batch_waves(grid, sh, 2 * ws, with_lanes=True) == ([[0], [1], [3], [2]], 1)
        # six equal shots with a bound of two shots' per-step state: one lane would take waves
        # of two, each lane takes waves of one (half the bound), so two lanes advance them
        small = efwi.make_grid(100, 200, 5.0, 5.0, 0.5e-3, 50, 20, 1e-3, 30.0, 4500.0)
        six = [efwi.Shot(50, 40 + 10 * k, np.full(3, 50, np.int32), np.array([60, 63, 66], np.int32))
               for k in range(6)]
        big_ws = efwi.workspace_size(efwi.WS_BATCH, small, six)
        efwi.set_wave_lanes(1)
        lo, hi = 1, 1 << 34                         # the least bound that pairs two shots in a wave
        while hi - lo > 1:
            mid = (lo + hi) // 2
            efwi.set_wave_cache_bytes(mid)
            lo, hi = (lo, mid) if len(efwi.batch_waves(small, six, big_ws)[0]) >= 2 else (mid, hi)
        efwi.set_wave_cache_bytes(hi)
        assert efwi.batch_waves(small, six, big_ws, with_lanes=True) == ([[0, 1], [2, 3], [4, 5]], 1)
        efwi.set_wave_lanes(2)
        assert efwi.batch_waves(small, six, big_ws, with_lanes=True) == ([[k] for k in range(6)], 2)
        efwi.set_wave_cache_bytes(0)
        for bad in (-1, 3):
            with pytest.raises(efwi.EfwiError) as ei:
                efwi.set_wave_lanes(bad)
            assert ei.value.status == efwi.E_INVAL
    finally:
        efwi.set_wave_lanes(0)
        efwi.set_wave_cache_bytes(0)
    assert efwi.get_wave_lanes() == 2


@pytest.mark.parametrize("change", [
    dict(nu=1.0), dict(nu=0.0), dict(n=0.0), dict(n=float("nan")),
    dict(taper=-1.0), dict(box=(10.0, 5.0, 0, 0, 0, 100.0)),
    dict(icov=(1e-3, 0.0, 1e-3, 0.0, 2e-3, 0.0)),          # |zx| > sqrt(zz xx): indefinite
    dict(icov=(-1e-3, 0.0, 1e-3, 0.0, 0.0, 0.0)),
    dict(src=(float("inf"), 0.0, 0.0)),
])
def test_zoi_argument_errors(efwi, change):
    """efwi_zoi_weights validates every zone on the host before any launch (the device
    pointers below are never used)."""
    grid = efwi.make_grid(100, 200, 5.0, 5.0, 0.5e-3, 50, 20, 1e-3, 30.0, 4500.0)
    z = dict(src=(250.0, 0.0, 500.0), icov=(1e-3, 0.0, 1e-3, 0.0, 0.0, 0.0), box=(100.0, 400.0, 0, 0, 100.0, 900.0),
             taper=50.0, n=2.0, nu=0.9)
    z.update(change)
    zone = efwi.make_zone(z["src"], z["icov"], z["box"], z["taper"])
    fake = ctypes.c_void_p(256)
    rc = efwi._lib.efwi_zoi_weights(ctypes.byref(grid), 1, ctypes.byref(zone), z["n"], z["nu"], fake, fake, None)
    assert rc == efwi.E_INVAL
    assert efwi._lib.efwi_last_error()


def test_final_model_argument_errors(efwi):
    grid = efwi.make_grid(100, 200, 5.0, 5.0, 0.5e-3, 50, 20, 1e-3, 30.0, 4500.0)
    fake = ctypes.c_void_p(256)
    assert efwi._lib.efwi_final_model(ctypes.byref(grid), 0, fake, fake, fake, fake, None) == efwi.E_INVAL
    assert efwi._lib.efwi_final_model(ctypes.byref(grid), 2, fake, None, fake, fake, None) == efwi.E_INVAL


@pytest.mark.parametrize("case", ["3d", "ns0", "clip0", "clip_big", "clip_nan", "null", "small_ws"])
def test_pseudo_hessian_argument_errors(efwi, case):
    """efwi_pseudo_hessian rejects bad arguments on the host before any launch (the device
    pointers below are never used)."""
    if case == "3d":
        grid = efwi.make_grid3d(40, 40, 40, 5.0, 5.0, 5.0, 0.5e-3, 50, 8, 1e-3, 30.0, 4500.0)
        shot = efwi.Shot(20, 20, [21], [25], src_iy=20, ch_iy=[20])
    else:
        grid = efwi.make_grid(100, 200, 5.0, 5.0, 0.5e-3, 50, 20, 1e-3, 30.0, 4500.0)
        shot = efwi.Shot(50, 100, [51, 51], [80, 120])
    arr = (efwi._ShotC * 1)(shot.c_struct())
    fake = ctypes.c_void_p(256)
    ns = 0 if case == "ns0" else 1
    clip = {"clip0": 0.0, "clip_big": 1.5, "clip_nan": float("nan")}.get(case, 0.01)
    h = None if case == "null" else fake
    ws_bytes = 64 if case == "small_ws" else 1 << 40
    rc = efwi._lib.efwi_pseudo_hessian(ctypes.byref(grid), ns, arr, fake, fake, clip, h, fake, fake, ws_bytes, None)
    assert rc == (efwi.E_WORKSPACE if case == "small_ws" else efwi.E_INVAL)
    assert efwi._lib.efwi_last_error()


@pytest.mark.parametrize("kw", [dict(gauge=-1), dict(decim=-2), dict(gauge=5), dict(decim=60), dict(rate=2)])
def test_das_sampling_validation(efwi, kw):
    """The shot's DAS sampling is checked on the host: gauge and decim >= 0, a gauge no
    longer than the channel list, decim <= nt, rate 0 or 1."""
    grid = efwi.make_grid(100, 200, 5.0, 5.0, 0.5e-3, 50, 20, 1e-3, 30.0, 4500.0)
    shot = efwi.Shot(50, 100, [51, 51, 51, 51], [80, 81, 82, 83])
    sc = shot.c_struct()
    for k, v in kw.items():
        setattr(sc, k, v)
    arr = (efwi._ShotC * 1)(sc)
    assert efwi._lib.efwi_validate(ctypes.byref(grid), 1, arr) == efwi.E_INVAL
    assert efwi._lib.efwi_last_error()


def test_das_sampling_sizes(efwi):
    """Field sampling needs the recorded strains and the field residual in the workspace;
    the default sampling keeps the sizes of the point-strain path."""
    grid = efwi.make_grid(100, 200, 5.0, 5.0, 0.5e-3, 50, 20, 1e-3, 30.0, 4500.0)
    point = efwi.Shot(50, 100, [51] * 8, list(range(80, 88)))
    field = efwi.Shot(50, 100, [51] * 8, list(range(80, 88)), gauge=3, decim=4, rate=True)
    assert field.data_shape(50) == (6, 12) and point.data_shape(50) == (8, 50)
    for kind in (efwi.WS_FORWARD, efwi.WS_GRADIENT):
        assert efwi.workspace_size(kind, grid, [field]) > efwi.workspace_size(kind, grid, [point])
    assert efwi.workspace_size(efwi.WS_ADJOINT, grid, [field]) == efwi.workspace_size(efwi.WS_ADJOINT, grid, [point])


def test_grouped_gradient_argument_errors(efwi):
    """Group indices outside [0, ng), ng < 1 and NULL arrays are rejected on the host."""
    grid = efwi.make_grid(100, 200, 5.0, 5.0, 0.5e-3, 50, 20, 1e-3, 30.0, 4500.0)
    shots = [efwi.Shot(50, 100, [51], [120]), efwi.Shot(50, 110, [51], [130])]
    arr = (efwi._ShotC * 2)(*[s.c_struct() for s in shots])
    fake = ctypes.c_void_p(256)
    ip = ctypes.POINTER(ctypes.c_int)
    for grp, ng in (([0, 2], 2), ([0, -1], 2), ([0, 0], 0)):
        g = np.asarray(grp, np.int32)
        rc = efwi._lib.efwi_batch_gradient_grouped(ctypes.byref(grid), 2, arr, g.ctypes.data_as(ip), ng, fake, fake,
                                                   fake, fake, fake, fake, 1 << 40, None)
        assert rc == efwi.E_INVAL
    rc = efwi._lib.efwi_batch_gradient_grouped(ctypes.byref(grid), 2, arr, None, 1, fake, fake, fake, fake, fake, fake,
                                               1 << 40, None)
    assert rc == efwi.E_INVAL


def test_bspline_arguments(efwi):
    """Node counts follow ceil((n - 1) / D) + 3; bad sizes, spacings and NULL arrays are
    rejected before any launch."""
    assert efwi._lib.efwi_bspline_nodes(100, 10) == 13 and efwi._lib.efwi_bspline_nodes(101, 10) == 13
    assert efwi._lib.efwi_bspline_nodes(102, 10) == 14 and efwi._lib.efwi_bspline_nodes(1, 1) == 3
    assert efwi._lib.efwi_bspline_nodes(0, 1) == 0 and efwi._lib.efwi_bspline_nodes(10, 0) == 0
    fake = ctypes.c_void_p(256)
    for args in ((0, 10, 1, 1, 1), (10, 10, 0, 1, 1), (10, 10, 1, 1, 0), (10, 10, 1000, 1001, 1)):
        assert efwi._lib.efwi_bspline_expand(*args, fake, fake, None) == efwi.E_INVAL
        assert efwi._lib.efwi_bspline_adjoint(*args, fake, fake, None) == efwi.E_INVAL
    assert efwi._lib.efwi_bspline_expand(10, 10, 1, 1, 1, None, fake, None) == efwi.E_INVAL


def test_vti_is_2d_only(efwi):
    """A VTI medium (grid.eps set) is refused on a 3D grid before any device access."""
    g3 = efwi.make_grid3d(40, 40, 40, 5.0, 5.0, 5.0, 0.5e-3, 50, 8, 1e-3, 30.0, 4500.0)
    g3.eps = 256
    shot = efwi.Shot(20, 20, [21], [25], src_iy=20, ch_iy=[20])
    arr = (efwi._ShotC * 1)(shot.c_struct())
    assert efwi._lib.efwi_validate(ctypes.byref(g3), 1, arr) == efwi.E_UNSUPPORTED
    g2 = efwi.make_grid(100, 200, 5.0, 5.0, 0.5e-3, 50, 20, 1e-3, 30.0, 4500.0)
    sh2 = efwi.Shot(50, 100, [51], [120])
    a2 = (efwi._ShotC * 1)(sh2.c_struct())
    iso = efwi._lib.efwi_workspace_size(efwi.WS_GRADIENT, ctypes.byref(g2), 1, a2)
    g2.eps = 256
    assert efwi._lib.efwi_workspace_size(efwi.WS_GRADIENT, ctypes.byref(g2), 1, a2) > iso


def test_3d_window_size_limit(efwi):
    """3D kernels address a shot's arrays with 32-bit byte offsets: a window whose padded
    arrays reach 2^30 elements is refused on the host."""
    g = efwi.make_grid3d(1100, 1100, 1000, 5.0, 5.0, 5.0, 0.4e-3, 10, 8, 1e-3, 30.0, 4500.0)
    shot = efwi.Shot(500, 500, [501], [520], src_iy=500, ch_iy=[500])
    arr = (efwi._ShotC * 1)(shot.c_struct())
    assert efwi._lib.efwi_validate(ctypes.byref(g), 1, arr) == efwi.E_RANGE
    small = efwi.Shot(500, 500, [501], [520], src_iy=500, ch_iy=[500], z0=300, y0=300, x0=300, wz=400, wy=400, wx=400)
    arr = (efwi._ShotC * 1)(small.c_struct())
    assert efwi._lib.efwi_validate(ctypes.byref(g), 1, arr) == efwi.OK


def test_2d_window_size_limit(efwi):
    """The 2D kernels address a shot's history slots and imaging sums with 32-bit byte
    offsets from one base: a window whose 5 * cells reaches 2^30 elements (about 2.1e8 cells)
    is refused on the host, before any launch; the largest workloads here pass."""
    g = efwi.make_grid(12000, 20000, 5.0, 5.0, 0.5e-3, 10, 20, 1e-3, 30.0, 4500.0)
    shot = efwi.Shot(6000, 10000, [6001], [10020])
    arr = (efwi._ShotC * 1)(shot.c_struct())
    assert efwi._lib.efwi_validate(ctypes.byref(g), 1, arr) == efwi.E_RANGE
    assert b"2^30" in efwi._lib.efwi_last_error()
    for wz, wx in ((1200, 4000), (6000, 6000)):   # 4.8e6 and 3.6e7 cells: accepted
        ok = efwi.Shot(6000, 10000, [6001], [10020], z0=6000 - wz // 2, x0=10000 - wx // 2, wz=wz, wx=wx)
        arr = (efwi._ShotC * 1)(ok.c_struct())
        assert efwi._lib.efwi_validate(ctypes.byref(g), 1, arr) == efwi.OK


def test_noalloc_scratch_limit_checked_on_host(efwi):
    """efwi_shot_gradient_noalloc refuses a shot whose gradient workspace exceeds its fixed
    scratch before any HIP call (the pointers are never dereferenced)."""
    grid, shot = _ok_case(efwi)
    grid.nt = 1000
    shot.ckpt_interval = 10**6                       # whole history: beyond 64 MiB
    assert efwi.noalloc_scratch_bytes() == 64 << 20
    sc = shot.c_struct()
    fake = ctypes.c_void_p(256)
    rc = efwi._lib.efwi_shot_gradient_noalloc(ctypes.byref(grid), ctypes.byref(sc), fake, fake, fake, fake, fake,
                                              None, None)
    assert rc == efwi.E_WORKSPACE
    assert b"scratch" in efwi._lib.efwi_last_error()
