"""Pins of the ZOI oracle (Source zone of influence, eq.(10)).

Checked against what eq.(10) and the geometry fix: weight 1 in the active part, the floor
value (-log nu)/(1 - log nu) at the source, the closed-form transition value at known
Mahalanobis and Euclidean distances (rotated ellipse, box taper), continuity at the
sinkhole edge, monotonicity along a ray, mirror symmetry, the 3D ellipsoid, and the paper's
1D illustration of W (31 samples, 3 sources).
"""
import numpy as np
import pytest

from oracle import zoi as Z

N, NU = 2.0, 0.9
FLOOR = -np.log(NU) / (1.0 - np.log(NU))


def zone(src, icov, box, taper):
    return {"src": src, "icov": icov, "box": box, "taper": taper}


def f(r):
    """eq.(10) written out once more for expected values at chosen r."""
    return (np.cos(np.pi * r / 2) ** N - np.log(NU)) / (1 - np.log(NU))


def test_active_part_is_one_and_source_is_the_floor():
    # 2D, 5 m cells; source at node (20, 40); sinkhole ellipse 30 m (z) x 60 m (x)
    zn = zone((100.0, 0.0, 200.0), (1 / 30.0**2, 0, 1 / 60.0**2, 0, 0, 0), (50.0, 150.0, 0, 0, 50.0, 350.0), 40.0)
    b, sink = Z.zoi_weights((41, 81), (5.0, 5.0), [zn], N, NU)
    assert b[0, 20, 40] == pytest.approx(FLOOR, abs=1e-15)
    assert sink[0, 20, 40]
    z = np.arange(41)[:, None] * 5.0
    x = np.arange(81)[None, :] * 5.0
    in_box = (z >= 50) & (z <= 150) & (x >= 50) & (x <= 350)
    d2 = ((z - 100) / 30) ** 2 + ((x - 200) / 60) ** 2
    assert np.all(b[0][in_box & (d2 >= 1)] == 1.0)
    assert np.array_equal(sink[0], d2 < 1)
    # on the sinkhole's principal axes (exact cell multiples): d = 1 is outside, b = 1
    assert not sink[0, 26, 40] and b[0, 26, 40] == 1.0     # 30 m below the source
    assert not sink[0, 20, 52] and b[0, 20, 52] == 1.0     # 60 m to the right
    # half way along an axis: r = 1/2
    assert b[0, 20, 46] == pytest.approx(f(0.5), rel=1e-14)
    assert b[0, 17, 40] == pytest.approx(f(0.5), rel=1e-14)


def test_rotated_ellipse_and_monotone_ray():
    th = np.deg2rad(30.0)
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    a, c = 40.0, 15.0                                     # semi-axes along the rotated (z', x')
    C = R @ np.diag([1 / a**2, 1 / c**2]) @ R.T           # inverse covariance in (z, x)
    icov = (C[0, 0], 0.0, C[1, 1], 0.0, C[0, 1], 0.0)
    # a 1-node grid at the origin and the source placed at -p: the node's offset is p
    for frac in (0.0, 0.25, 0.5, 0.9):
        pz, px = R @ np.array([frac * a, 0.0])
        zn = zone((-pz, 0.0, -px), icov, (-100, 100, 0, 0, -100, 100), 0.0)
        b, sink = Z.zoi_weights((1, 1), (1.0, 1.0), [zn], N, NU)
        assert sink[0, 0, 0]
        assert b[0, 0, 0] == pytest.approx(f(1.0 - frac), rel=1e-12, abs=1e-15)
    # along the minor axis beyond c the point is outside the sinkhole
    pz, px = R @ np.array([0.0, 1.2 * c])
    zn = zone((-pz, 0.0, -px), icov, (-100, 100, 0, 0, -100, 100), 0.0)
    b, sink = Z.zoi_weights((1, 1), (1.0, 1.0), [zn], N, NU)
    assert not sink[0, 0, 0] and b[0, 0, 0] == 1.0
    # weights rise monotonically from the source outwards inside the sinkhole
    zn = zone((100.0, 0.0, 100.0), icov, (0, 200, 0, 0, 0, 200), 0.0)
    b, sink = Z.zoi_weights((201, 201), (1.0, 1.0), [zn], N, NU)
    ray = b[0, 100, 100:160]
    assert np.all(np.diff(ray) >= 0.0) and ray[0] == pytest.approx(FLOOR, abs=1e-15) and ray[-1] == 1.0


def test_outer_taper():
    zn = zone((50.0, 0.0, 50.0), (1.0, 0, 1.0, 0, 0, 0), (20.0, 80.0, 0, 0, 20.0, 80.0), 10.0)
    b, sink = Z.zoi_weights((101, 101), (1.0, 1.0), [zn], N, NU)
    assert b[0, 50, 15] == pytest.approx(f(0.5), rel=1e-14)        # 5 m left of the box
    assert b[0, 50, 85] == pytest.approx(f(0.5), rel=1e-14)
    assert b[0, 10, 50] == pytest.approx(FLOOR, abs=1e-15)          # beyond the taper
    # corner: Euclidean distance sqrt(3^2 + 4^2) = 5 m
    assert b[0, 16, 17] == pytest.approx(f(0.5), rel=1e-14)
    assert np.all(b[0, 20:81, 20:81][~sink[0, 20:81, 20:81]] == 1.0)
    # taper 0: a step to the floor value just outside the box
    zn["taper"] = 0.0
    b, _ = Z.zoi_weights((101, 101), (1.0, 1.0), [zn], N, NU)
    assert b[0, 50, 19] == pytest.approx(FLOOR, abs=1e-15) and b[0, 50, 20] == 1.0


def test_mirror_symmetry_and_3d_ellipsoid():
    zn = zone((60.0, 0.0, 100.0), (1 / 25.0**2, 0, 1 / 45.0**2, 0, 0, 0), (10, 110, 0, 0, 10, 190), 20.0)
    b, sink = Z.zoi_weights((25, 41), (5.0, 5.0), [zn], N, NU)
    # mirror about the source row (12) and column (20)
    assert np.allclose(b[0, 12 - 5:12, :], b[0, 12 + 5:12:-1, :], rtol=0, atol=1e-15)
    assert np.allclose(b[0, :, 20 - 9:20], b[0, :, 20 + 9:20:-1], rtol=0, atol=1e-15)
    # 3D: an ellipsoid with semi-axes 10 (z), 20 (y), 30 (x) metres around node (10, 10, 10)
    zn3 = zone((10.0, 20.0, 30.0), (1 / 100.0, 1 / 400.0, 1 / 900.0, 0, 0, 0), (0, 50, 0, 50, 0, 50), 0.0)
    b3, s3 = Z.zoi_weights((21, 21, 21), (1.0, 2.0, 3.0), [zn3], N, NU)
    assert b3[0, 10, 10, 10] == pytest.approx(FLOOR, abs=1e-15)
    assert not s3[0, 20, 10, 10] and not s3[0, 10, 20, 10] and not s3[0, 10, 10, 20]
    assert b3[0, 15, 10, 10] == pytest.approx(f(0.5), rel=1e-14)    # 5 m of 10 along z
    assert b3[0, 10, 15, 10] == pytest.approx(f(0.5), rel=1e-14)    # 10 m of 20 along y
    assert b3[0, 10, 10, 15] == pytest.approx(f(0.5), rel=1e-14)    # 15 m of 30 along x


def test_paper_1d_illustration():
    """The W illustration: 31 samples, 3 sources (6, 15, 24), sinkhole radius 5 samples; the
    same weights as the explicit 1D formula of the regularizer pins."""
    zones = [zone((0.0, 0.0, float(xs)), (1.0, 0, 1 / 25.0, 0, 0, 0), (0, 0, 0, 0, 0, 30), 0.0) for xs in (6, 15, 24)]
    b, sink = Z.zoi_weights((1, 31), (1.0, 1.0), zones, N, NU)
    x = np.arange(31)
    for s, xs in enumerate((6, 15, 24)):
        dist = np.abs(x - xs) / 5.0
        inside = dist < 1
        expect = np.ones(31)
        expect[inside] = f(1 - dist[inside])
        assert np.array_equal(sink[s, 0], inside)
        assert np.allclose(b[s, 0], expect, rtol=1e-14, atol=0)
