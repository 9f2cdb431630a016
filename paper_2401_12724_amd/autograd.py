"""torch.autograd.Function around the BYSDF and its hand-written adjoint.

BYSDFEval.apply(theta, types, q, offsets) returns E (n x 3, RGB) for the
queries q grouped by type (offsets: int64 CSR on the device) at the per-type
parameters theta (n_types x 8: albedo r g b, beta, ply twist, fiber twist,
ply density, fiber density).  The forward pass writes theta into the handle
(bysdf_types_set_theta) and runs bysdf_eval; the backward pass writes the
same theta back (another forward on the handle may have replaced it) and
runs bysdf_eval_backward, which recomputes the model (shadowing included)
with forward-mode tangents, so nothing but the inputs is kept between the
passes.  The handle clamps theta to its valid ranges (albedo >= 0, beta in
[1e-4, 10], twists in [-1.5, 1.5] rad, densities in [0, 1]); where a
component lies strictly outside its range the value does not depend on it
and its gradient is zero.
"""
from __future__ import annotations

import torch

from . import bysdf

# valid ranges of theta's columns (albedo rgb, beta, ply twist, fiber twist,
# ply density, fiber density), as the handle clamps them
_LO = (0.0, 0.0, 0.0, 1e-4, -1.5, -1.5, 0.0, 0.0)
_HI = (float("inf"), float("inf"), float("inf"), 10.0, 1.5, 1.5, 1.0, 1.0)


class BYSDFEval(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, types, q, offsets):
        assert theta.is_cuda and theta.dtype == torch.float32
        th = theta.detach().contiguous()
        bysdf.bysdf_types_set_theta(types, th)
        vals, _ = bysdf.bysdf_eval(types, q)
        ctx.types, ctx.q, ctx.offsets = types, q, offsets
        ctx.theta = th  # this forward's theta (and alive until the handle's copy has run)
        return vals[0:3].t().contiguous()

    @staticmethod
    def backward(ctx, grad_E):
        th = ctx.theta
        bysdf.bysdf_types_set_theta(ctx.types, th)
        g, _ = bysdf.bysdf_eval_backward(ctx.types, ctx.q, ctx.offsets, grad_E.contiguous())
        lo = torch.tensor(_LO, dtype=th.dtype, device=th.device)
        hi = torch.tensor(_HI, dtype=th.dtype, device=th.device)
        inside = (th >= lo) & (th <= hi)
        return g * inside, None, None, None


def project_(theta):
    """Clamp theta (n_types x 8) into the ranges the handle accepts, in place:
    a step that leaves a range would otherwise park the component where the
    value, and with it the gradient, no longer depends on it."""
    with torch.no_grad():
        lo = torch.tensor(_LO, dtype=theta.dtype, device=theta.device)
        hi = torch.tensor(_HI, dtype=theta.dtype, device=theta.device)
        theta.copy_(torch.maximum(torch.minimum(theta, hi), lo))
    return theta


def bysdf_fit_step(theta, types, q, offsets, target, opt):
    """One step of the least-squares fit sum (E - target)^2 with optimiser
    opt, projected back into the valid parameter ranges."""
    opt.zero_grad(set_to_none=True)
    E = BYSDFEval.apply(theta, types, q, offsets)
    loss = ((E - target) ** 2).sum()
    loss.backward()
    opt.step()
    project_(theta)
    return loss.detach()
