"""FP64 oracle: the source zones of influence (ZOI) of the model extension.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Paper passages followed
-----------------------
* Source zone of influence, eq.(10): the ZOI of source s is a weight field b_s over the
  physical model, equal to 1 in the zone's active part and falling through a transition
  ``b = (cos^n(pi r / 2) - log nu) / (1 - log nu)`` where ``0 <= r <= 1`` is the
  normalized distance away from the active part; n sets the stiffness and nu (0 < nu < 1)
  the height of the transition. The outer transition uses the Euclidean distance, the
  sinkhole around the source the Mahalanobis distance (an ellipse or ellipsoid).
* The sinkhole of s (the region where the operator W of eq.(11) replaces m_s) is where
  the Mahalanobis distance to the source is below one.

Readings where the paper is silent
----------------------------------
* log is the natural logarithm.
* Active part: an axis-aligned box (z, [y,] x ranges in metres, covering the
  source-receiver spread); outer transition r = (Euclidean distance to the box) / taper,
  capped at 1 (a step to the floor value when the taper is 0).
* Sinkhole: d = sqrt(dp^T C^-1 dp) with dp the offset from the source and C^-1 a given
  symmetric positive definite matrix; inside (d < 1) r = 1 - d, so b is the floor value
  (-log nu)/(1 - log nu) at the source and rises to 1 at the sinkhole's edge.
* Where both transitions apply, the larger r (the smaller weight) is taken.
* Coordinates: node (i, [k,] j) sits at (i dz, [k dy,] j dx) metres.
"""
from __future__ import annotations

import numpy as np


def transition(r, n, nu):
    """eq.(10): weight at normalized distance r in [0, 1]."""
    ln = np.log(nu)
    return (np.cos(0.5 * np.pi * r) ** n - ln) / (1.0 - ln)


def mahalanobis2(dz, dy, dx, icov):
    """Squared Mahalanobis distance, summed in a fixed order (zz, xx, zx[, yy, zy, yx]) so that
    the sinkhole test is reproducible bit for bit. icov = (zz, yy, xx, zy, zx, yx); dy is None
    in 2D."""
    czz, cyy, cxx, czy, czx, cyx = (float(c) for c in icov)
    t = (czz * dz) * dz
    t = t + (cxx * dx) * dx
    t = t + ((2.0 * czx) * dz) * dx
    if dy is not None:
        t = t + (cyy * dy) * dy
        t = t + ((2.0 * czy) * dz) * dy
        t = t + ((2.0 * cyx) * dy) * dx
    return t


def zoi_weights(shape, spacing, zones, n, nu):
    """ZOI weights and sinkhole flags of every source.

    shape: (nz, nx) or (nz, ny, nx); spacing: (dz, dx) or (dz, dy, dx) in metres;
    zones: one dict per source with keys
      ``src``   (z, y, x) sinkhole centre in metres (y ignored in 2D),
      ``icov``  (zz, yy, xx, zy, zx, yx) inverse covariance of the sinkhole, 1/m^2,
      ``box``   (z0, z1, y0, y1, x0, x1) active part in metres (y ignored in 2D),
      ``taper`` width of the outer transition in metres.
    Returns (b [Ns][shape] FP64, sink [Ns][shape] bool)."""
    three = len(shape) == 3
    axes = [np.arange(s, dtype=np.float64) * float(h) for s, h in zip(shape, spacing)]
    grids = np.meshgrid(*axes, indexing="ij")
    z, x = grids[0], grids[-1]
    y = grids[1] if three else None
    b = np.empty((len(zones),) + tuple(shape))
    sink = np.zeros((len(zones),) + tuple(shape), bool)
    for s, zn in enumerate(zones):
        sz, sy, sx = (float(v) for v in zn["src"])
        z0, z1, y0, y1, x0, x1 = (float(v) for v in zn["box"])
        taper = float(zn["taper"])
        # outer transition: Euclidean distance to the active box
        ez = np.maximum(np.maximum(z0 - z, z - z1), 0.0)
        ex = np.maximum(np.maximum(x0 - x, x - x1), 0.0)
        e2 = ez * ez + ex * ex
        if three:
            ey = np.maximum(np.maximum(y0 - y, y - y1), 0.0)
            e2 = e2 + ey * ey
        e = np.sqrt(e2)
        if taper > 0.0:
            r_out = np.minimum(e / taper, 1.0)
        else:
            r_out = np.where(e > 0.0, 1.0, 0.0)
        # sinkhole: Mahalanobis distance to the source
        d2 = mahalanobis2(z - sz, (y - sy) if three else None, x - sx, zn["icov"])
        inside = d2 < 1.0
        r_sink = np.where(inside, 1.0 - np.sqrt(np.where(inside, d2, 0.0)), 0.0)
        b[s] = transition(np.maximum(r_out, r_sink), n, nu)
        sink[s] = inside
    return b, sink
