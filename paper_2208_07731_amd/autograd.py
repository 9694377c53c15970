"""torch.autograd.Function wrappers around the fit and its hand-written adjoint.

ISDFFit:  Theta = ISDFFit.apply(phi, psi, idx[, prec, rblock]).  Backward
          calls isdf_fit_backward with the upstream gradient of Theta.
ISDFLoss: L = ISDFLoss.apply(phi, psi, idx, g[, prec, rblock]) with
          L = sum_r g_r sum_mu |Theta_r,mu|^2.  The forward runs the fused
          adjoint once (loss and gradients in one pass over the grid, Theta
          recomputed per r-block, never stored); backward scales the stored
          gradients by the upstream scalar.
Passing the same tensor as phi and psi selects the aliased (real Theta)
path; its gradient then flows into that tensor through both arguments.
The interpolation points idx are constants (no gradient).
"""
from __future__ import annotations

import torch

from . import api


class ISDFFit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi, psi, idx, prec: str = "fp64", rblock: int | None = None):
        aliased = psi is phi
        theta, minv, _ = api.fit(phi, None if aliased else psi, idx, prec=prec, rblock=rblock)
        ctx.save_for_backward(phi, psi, idx, minv)
        ctx.aliased, ctx.prec, ctx.rblock = aliased, prec, rblock
        ctx.mark_non_differentiable(minv)
        return theta

    @staticmethod
    def backward(ctx, gtheta):
        phi, psi, idx, minv = ctx.saved_tensors
        dphi, dpsi, _, _ = api.fit_backward(phi, None if ctx.aliased else psi, idx, minv,
                                            theta_bar=gtheta.contiguous(), prec=ctx.prec, rblock=ctx.rblock)
        return dphi, dpsi, None, None, None


class ISDFLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi, psi, idx, g, prec: str = "fp64", rblock: int | None = None):
        aliased = psi is phi
        p2 = None if aliased else psi
        _, minv, _ = api.fit(phi, p2, idx, prec=prec, nrows=0)
        dphi, dpsi, loss, _ = api.fit_backward(phi, p2, idx, minv, g=g.contiguous(), prec=prec, rblock=rblock)
        ctx.save_for_backward(dphi, dpsi)
        return loss

    @staticmethod
    def backward(ctx, gl):
        dphi, dpsi = ctx.saved_tensors
        return dphi * gl, dpsi * gl, None, None, None, None
