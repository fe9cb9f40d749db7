"""torch.autograd.Function over K unrolled UPN steps (the differentiated form).

Forward: x^(K) = UPN_K(b, alpha) from x^(0) = 0 through tvreg_upn_unrolled_fwd.
Backward: tvreg_upn_unrolled_bwd, the hand-written reverse pass (segments of
``ckpt_every`` steps recomputed from checkpoints), giving dl/db and
dl/dlog(alpha) for whatever loss autograd puts on x^(K).  The step sizes L_j
are decisions of the line search and are held fixed in the derivative;
passing ``L_replay`` freezes them in the forward pass too, which makes the
map differentiable in the ordinary sense around the given inputs.
"""
from __future__ import annotations

import math

import torch

from . import Geometry, upn_unrolled_bwd, upn_unrolled_fwd


class UnrolledUPN(torch.autograd.Function):
    @staticmethod
    def forward(ctx, b, log_alpha, geom: Geometry, K: int, tau: float, ckpt_every: int,
                L_replay, L_bar: float):
        alpha = math.exp(float(log_alpha.detach().item()))
        bd = b.detach().contiguous()
        xK, tape, L = upn_unrolled_fwd(geom, bd, K, alpha, tau=tau, ckpt_every=ckpt_every,
                                       L_replay=L_replay, L_bar=L_bar)
        ctx.geom = geom
        ctx.tape = tape
        ctx.L = L
        ctx.save_for_backward(bd, log_alpha)
        return xK

    @staticmethod
    def backward(ctx, gx):
        bd, log_alpha = ctx.saved_tensors
        da, db = upn_unrolled_bwd(ctx.geom, bd, ctx.tape, gx.to(bd.dtype).contiguous())
        ga = torch.tensor(da, dtype=log_alpha.dtype, device=log_alpha.device)
        return db, ga, None, None, None, None, None, None


def unrolled_upn(geom: Geometry, b: torch.Tensor, log_alpha: torch.Tensor, K: int = 30,
                 tau: float = 1e-4, ckpt_every: int = 5, L_replay=None,
                 L_bar: float = 1.0) -> torch.Tensor:
    """x^(K) of K UPN steps from 0, differentiable in b and log_alpha."""
    return UnrolledUPN.apply(b, log_alpha, geom, int(K), float(tau), int(ckpt_every), L_replay,
                             float(L_bar))
