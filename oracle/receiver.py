"""FP64 oracle: the field-like DAS sampling operator K_r of eq.(3) (the data of a shot are
a spatio-temporal sampling of its wavefield) for the acquisition of the field example: a
fiber that measures strain rate over a gauge length, its data resampled in time.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Readings where the paper is silent
----------------------------------
* The point measurement is the one of the synthetic path: e_c(t_{n+1}), the x-x strain at
  the channel's normal node (the time integral of the 4th-order D-x vx), for the shot's
  channels in fiber order, one node apart.
* Gauge length: field channel f is the mean of the point measurements of the ``gauge``
  consecutive channels f .. f + gauge - 1 (the strain integrated over the gauge divided by
  its length, sampled at the gauge's nodes); nch - gauge + 1 field channels.
* Strain rate: the first difference in time at the simulation step,
  (e(t_{n+1}) - e(t_n)) / dt with e(t_0) = 0, taken before the resampling.
* Resampling: every ``decim``-th sample, those at t_{n+1} = k decim dt (k = 1, 2, ...):
  floor(nt / decim) samples; no anti-alias filter (the sources' band lies far below the
  resampled Nyquist frequency).
* The misfit compares K d with field-shaped observed data; its gradient is J^T K^T r.
"""
from __future__ import annotations

import numpy as np

from . import elastic2d as E


def field_shape(nch, nt, gauge, decim):
    return nch - gauge + 1, nt // decim


def field_data(e, gauge, decim, rate, dt):
    """K e: [nch][nt] point strain -> [nch - gauge + 1][nt // decim] field data."""
    e = np.asarray(e, np.float64)
    nch, nt = e.shape
    nf, ntf = field_shape(nch, nt, gauge, decim)
    x = e
    if rate:
        prev = np.concatenate([np.zeros((nch, 1)), e[:, :-1]], axis=1)
        x = (e - prev) / dt
    avg = np.stack([x[f:f + gauge].mean(axis=0) for f in range(nf)]) if nf > 0 else np.zeros((0, nt))
    return avg[:, decim - 1::decim][:, :ntf]


def field_data_T(y, nch, nt, gauge, decim, rate, dt):
    """K^T y: [nch - gauge + 1][nt // decim] -> [nch][nt], each step of field_data transposed
    in reverse order (resampling, gauge mean, time difference)."""
    y = np.asarray(y, np.float64)
    nf, ntf = field_shape(nch, nt, gauge, decim)
    z = np.zeros((nf, nt))
    z[:, decim - 1::decim][:, :ntf] = y
    x = np.zeros((nch, nt))
    for f in range(nf):
        x[f:f + gauge] += z[f] / gauge
    if rate:
        nxt = np.concatenate([x[:, 1:], np.zeros((nch, 1))], axis=1)
        x = (x - nxt) / dt
    return x


def shot_gradient_field(grid, m, src_iz, src_ix, src, ch_iz, ch_ix, d_obs, gauge, decim, rate):
    """Misfit 1/2 ||K d - d_obs||^2 of one shot with field-shaped d_obs, its gradient
    J^T K^T (K d - d_obs) w.r.t. (Vp, Vs, rho), and K d. Returns (g, phi, K d)."""
    d, hist, _ = E.forward(grid, m[0], m[1], m[2], src_iz, src_ix, src, ch_iz, ch_ix, store=True)
    y = field_data(d, gauge, decim, rate, grid.dt)
    phi, r = E.misfit(y, d_obs)
    rv = field_data_T(r, d.shape[0], d.shape[1], gauge, decim, rate, grid.dt)
    _, gpar = E.adjoint(grid, m[0], m[1], m[2], src_iz, src_ix, ch_iz, ch_ix, rv, hist=hist)
    return E.chain_rule(m[0], m[1], m[2], *gpar), phi, y
