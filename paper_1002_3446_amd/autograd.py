"""torch.autograd.Function over the event path: log w_int as a function of the RAMBO
uniforms and the parton fractions x1, x2.

forward  = bg_generate with caller-supplied uniforms, x1, x2, helicities and orderings,
           returning the log integrand weight (no cut step function, no sampling density);
backward = bg_amp2_grad, the hand-written adjoint, which recomputes the forward inside its
           kernel (only the inputs are saved).
"""
from __future__ import annotations

import torch

from . import bg


class LogWeight(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, x12, cfg, hel, order):
        N = u.shape[0]
        ins = dict(uniforms=u.detach().contiguous(), x12=x12.detach().contiguous(), hel=hel, order=order)
        lw = bg.generate(cfg, N, inputs=ins, outputs=("logw",))["logw"]
        ctx.save_for_backward(u, x12, hel, order)
        ctx.cfg = cfg
        return lw

    @staticmethod
    def backward(ctx, g):
        u, x12, hel, order = ctx.saved_tensors
        gu, gx, _ = bg.amp2_grad(ctx.cfg, u.detach().contiguous(), x12.detach().contiguous(), hel, order,
                                 gout=g.contiguous().to(torch.float64), want_logw=False)
        return gu, gx, None, None, None


def log_weight(u, x12, cfg, hel, order):
    """log w_int [N] (differentiable in u [N, 4(n-2)] and x12 [N, 2])."""
    return LogWeight.apply(u, x12, cfg, hel, order)
