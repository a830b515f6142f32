"""PyTorch autograd over the HIP library: the per-shot gradient of eq.(6) and the extended
objective of eq.(8) as differentiable functions of the (extended) model.

* ``ShotData``        m_s -> d_s (DAS data); backward J_s^T v through the hand-written
                      transposed kernels (any data-space loss on top).
* ``ShotMisfit``      m_s -> phi_s = 1/2 ||d_s - d_obs||^2; forward also runs the adjoint
                      (one forward + one reverse sweep), backward scales the stored gradient.
* ``BatchMisfit``     m~ -> sum_s phi_s(m_s), all shots advanced together.
* ``ExtensionPenalty`` m~ -> 1/2 eta^2 ||(I - S^T S_w) W m~||^2.
* ``extended_misfit`` the sum of the two, eq.(8).

Checkpointing: ``checkpoint_interval`` picks the largest checkpoint interval whose workspace
fits in a fraction of the free device memory (the whole forward history when it fits, so
nothing is recomputed; sqrt(nt) checkpoints, the library's default, at the least).
"""
from __future__ import annotations


import torch

from . import efwi


def checkpoint_interval(grid, shot, device=None, budget_fraction=0.6) -> int:
    """Largest checkpoint interval whose workspace fits in a fraction of the free device
    memory (nt: whole history, no recomputation); 0 (sqrt(nt)) if even that does not fit,
    and the call then needs the memory it needs."""
    budget = int(budget_fraction * torch.cuda.mem_get_info(device)[0])
    try:
        return efwi.plan_interval(grid, shot, budget)
    except efwi.EfwiError as e:
        if e.status != efwi.E_WORKSPACE:
            raise
        return 0


class ShotData(torch.autograd.Function):
    """d = K u(m) for one shot; backward: J^T applied to the incoming data-space gradient."""

    @staticmethod
    def forward(ctx, m, src, grid, shot):
        m = m.contiguous()
        d = efwi.model_forward(grid, shot, m, src)
        ctx.save_for_backward(m, src)
        ctx.grid, ctx.shot = grid, shot
        return d

    @staticmethod
    def backward(ctx, gd):
        m, src = ctx.saved_tensors
        g = efwi.shot_jt(ctx.grid, ctx.shot, m, src, gd.contiguous().to(torch.float32))
        return g, None, None, None


class ShotMisfit(torch.autograd.Function):
    """phi_s(m) = 1/2 ||d_s(m) - d_obs||^2 (FP64 scalar); ``ws`` an optional workspace (one
    is allocated per call otherwise)."""

    @staticmethod
    def forward(ctx, m, src, d_obs, grid, shot, ws=None):
        g, phi = efwi.shot_gradient(grid, shot, m.contiguous(), src, d_obs, ws=ws)
        ctx.save_for_backward(g)
        return phi

    @staticmethod
    def backward(ctx, gphi):
        (g,) = ctx.saved_tensors
        return gphi.to(g.dtype) * g, None, None, None, None, None


class BatchMisfit(torch.autograd.Function):
    """sum_s phi_s(m_s) over an extended model m~ [ns][3][nz][nx] (data term of eq.(8))."""

    @staticmethod
    def forward(ctx, m_ext, src, d_obs, grid, shots, ws):
        g, phi = efwi.batch_gradient(grid, shots, m_ext.contiguous(), src, d_obs, ws=ws)
        ctx.save_for_backward(g)
        return phi.sum()

    @staticmethod
    def backward(ctx, gphi):
        (g,) = ctx.saved_tensors
        return gphi.to(g.dtype) * g, None, None, None, None, None


class ExtensionPenalty(torch.autograd.Function):
    """1/2 eta^2 ||(I - S^T S_w) W m~||^2 (second term of eq.(8))."""

    @staticmethod
    def forward(ctx, m_ext, b, sink, eta, grid):
        g = torch.zeros_like(m_ext)
        phi = efwi.extension_regularizer(grid, m_ext.contiguous(), b, sink, eta, g)
        ctx.save_for_backward(g)
        return phi

    @staticmethod
    def backward(ctx, gphi):
        (g,) = ctx.saved_tensors
        return gphi.to(g.dtype) * g, None, None, None, None


def extended_misfit(m_ext, src, d_obs, grid, shots, b, sink, eta, ws=None):
    """eq.(8): data misfit of every shot on its own component plus the consistency term."""
    return BatchMisfit.apply(m_ext, src, d_obs, grid, list(shots), ws) + \
        ExtensionPenalty.apply(m_ext, b, sink, eta, grid)
