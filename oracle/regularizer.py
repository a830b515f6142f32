"""FP64 oracle: the consistency regularizer of the extended misfit.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Paper passages followed
-----------------------
* eq.(8), second term: ``1/2 eta^2 || (I - S^T S_w) W m~ ||^2`` with m~ = (m_1..m_Ns).
* W (Model extension along sources, and eq.(11)): block matrix of diagonal blocks; for
  model m_s it replaces the values inside s's sinkhole by
  ``b_s m_s + (1 - b_s) / (sum_{i!=s} b_i) * sum_{i!=s} b_i m_i`` and leaves the rest;
  each row sums to one.
* S_w (eq.(12)): weighted sum ``sum_s b'_s m_s / sum_s b'_s`` with b'_s = b_s outside s's
  sinkhole and b'_s = 1 inside.
* S^T: spreading (copy along sources); not the adjoint of S_w.

Because every block of W and S_w is diagonal, the operators act independently at each
spatial point (and, with the same weights, on each of Vp, Vs, rho). This module builds the
Ns x Ns matrices of W and S^T S_w at each point explicitly and applies them with matrix
products, so each line can be checked against the equations by eye.

Readings where the paper is silent
----------------------------------
* If the other sources' weights sum to zero at a sinkhole point (eq.(11) divides by zero),
  that row of W is the identity.
* If sum_s b'_s = 0 at a point, no source is useful there and the point contributes nothing
  (its (I - S^T S_w) block is taken as zero).
"""
from __future__ import annotations

import numpy as np


def w_matrix(b, sink):
    """Dense Ns x Ns block of W at one point (b: [Ns] weights, sink: [Ns] bool)."""
    ns = len(b)
    W = np.eye(ns)
    for s in range(ns):
        if not sink[s]:
            continue
        others = [i for i in range(ns) if i != s]
        B = float(sum(b[i] for i in others))
        if B <= 0.0:
            continue
        W[s, :] = 0.0
        W[s, s] = b[s]
        for i in others:
            W[s, i] = (1.0 - b[s]) * b[i] / B
    return W


def sw_row(b, sink):
    """Row vector of S_w at one point: b'_s / sum b' (None if sum b' = 0)."""
    bp = np.where(np.asarray(sink, bool), 1.0, np.asarray(b, np.float64))
    tot = bp.sum()
    if tot <= 0.0:
        return None
    return bp / tot


def projector(b, sink):
    """I - S^T S_w at one point (Ns x Ns); zero block if S_w is undefined there."""
    ns = len(b)
    row = sw_row(b, sink)
    if row is None:
        return np.zeros((ns, ns))
    return np.eye(ns) - np.outer(np.ones(ns), row)


def regularizer(m_ext, b, sink, eta):
    """Value and gradient of 1/2 eta^2 ||(I - S^T S_w) W m~||^2.

    m_ext: [Ns][3][...] extended model; b: [Ns][...] ZOI weights; sink: [Ns][...] sinkhole
    indicator. Returns (phi_reg, grad [Ns][3][...]) with grad = eta^2 W^T P^T P W m~,
    P = I - S^T S_w."""
    m_ext = np.asarray(m_ext, np.float64)
    ns, npar = m_ext.shape[:2]
    space = m_ext.shape[2:]
    mflat = m_ext.reshape(ns, npar, -1)
    bflat = np.asarray(b, np.float64).reshape(ns, -1)
    sflat = np.asarray(sink).reshape(ns, -1).astype(bool)
    grad = np.zeros_like(mflat)
    phi = 0.0
    for p in range(mflat.shape[2]):
        W = w_matrix(bflat[:, p], sflat[:, p])
        P = projector(bflat[:, p], sflat[:, p])
        A = P @ W
        y = A @ mflat[:, :, p]               # [Ns][3]
        phi += 0.5 * eta * eta * float(np.sum(y * y))
        grad[:, :, p] = eta * eta * (A.T @ y)
    return phi, grad.reshape((ns, npar) + space)


def final_model(m_ext, b, sink):
    """eq.(9): m^ = S_w W m~ (zero where S_w is undefined)."""
    m_ext = np.asarray(m_ext, np.float64)
    ns, npar = m_ext.shape[:2]
    space = m_ext.shape[2:]
    mflat = m_ext.reshape(ns, npar, -1)
    bflat = np.asarray(b, np.float64).reshape(ns, -1)
    sflat = np.asarray(sink).reshape(ns, -1).astype(bool)
    out = np.zeros((npar, mflat.shape[2]))
    for p in range(mflat.shape[2]):
        row = sw_row(bflat[:, p], sflat[:, p])
        if row is None:
            continue
        out[:, p] = row @ (w_matrix(bflat[:, p], sflat[:, p]) @ mflat[:, :, p])
    return out.reshape((npar,) + space)
