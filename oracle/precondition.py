"""FP64 oracle: the two alternative ways of reducing source footprints that the paper
compares extended FWI with (Synthetic example, comparison with alternative methods).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Paper passages followed
-----------------------
* Approximate inverse pseudo-Hessian: a diagonal operator built by autocorrelating the
  absolute particle-velocity wavefields in time, summing over shots, clipping and scaling;
  it is given to l-BFGS as the initial inverse Hessian at every iteration, together with a
  near-offset mute (channels closer than 200 m to the source are dropped).
* Gradient preconditioning, eq.(15): the per-shot gradients g_s of conventional FWI,
  stacked as an extended vector, are mapped by the footprint-removal operator S_w W of
  eq.(9) before the solver sees them. That operator is ``regularizer.final_model``; this
  module adds nothing to it.

Readings where the paper is silent
----------------------------------
* Zero-lag autocorrelation of |v| in time: H_s(x) = sum_n |v_s(x, t_{n+1/2})|^2 over every
  leapfrog step n = 0 .. nt-1 (the velocities of the step's first half step); no dt factor
  (the operator is scaled afterwards anyway).
* |v|^2 at normal node (i, j) uses the staggered components that carry the node's index,
  vx at (i, j+1/2) and vz at (i+1/2, j), without interpolation.
* A shot on a window contributes inside its window only; H = sum_s H_s.
* Clipping and scaling: P = c max(H) / max(H, c max(H)) with a clip fraction 0 < c <= 1,
  i.e. H is clipped from below at c times its maximum, inverted, and scaled so that the
  largest value of P is 1 (far from the sources) and P is smallest where the wavefield
  energy is largest (around the sources). A zero H gives P = 1 everywhere.
"""
from __future__ import annotations

import numpy as np

from . import elastic2d as E


def autocorrelation(grid: E.Grid2D, vp, vs, rho, src_iz, src_ix, src):
    """H_s of one shot on its own grid: sum over the nt steps of vx^2 + vz^2 at the normal
    nodes (readings above), from the oracle's forward propagation with the moment-tensor
    source ``src`` [3][nt]."""
    H = np.zeros((grid.nz, grid.nx))

    def probe(n, P):
        # after full step n the propagator holds v^{n+1/2}
        H[...] += P.vx * P.vx + P.vz * P.vz

    none = np.zeros(0, dtype=np.int64)
    E.forward(grid, vp, vs, rho, src_iz, src_ix, src, none, none, probe=probe)
    return H


def sum_over_shots(shape, parts):
    """H = sum_s H_s, each H_s placed at its window origin: parts = [(z0, x0, H_s), ...]."""
    H = np.zeros(shape)
    for z0, x0, Hs in parts:
        H[z0:z0 + Hs.shape[0], x0:x0 + Hs.shape[1]] += Hs
    return H


def inverse_operator(H, clip):
    """P = c max(H) / max(H, c max(H)) (reading above); 1 everywhere when H is all zero."""
    H = np.asarray(H, np.float64)
    top = float(H.max()) if H.size else 0.0
    if top <= 0.0:
        return np.ones_like(H)
    floor = clip * top
    return floor / np.maximum(H, floor)


def near_offset_keep(src_iz, src_ix, ch_iz, ch_ix, dz, dx, radius):
    """Channels kept by the near-offset mute: Euclidean source-channel distance (between
    normal nodes, in metres) not below ``radius``."""
    dist = np.hypot((np.asarray(ch_iz) - src_iz) * dz, (np.asarray(ch_ix) - src_ix) * dx)
    return dist >= radius
