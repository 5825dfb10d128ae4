"""torch.autograd.Function for exact top-K scores.

Forward: the exact top-K of every user (any screen precision; the result is
the same).  The returned scores are the float64 keys cast to float32, and the
gradient flows to U and I through them with the top-K indices held fixed:
dU = sum_k G I[idx], dI[i] = sum of G U over the (u, k) that picked item i
(hand-written HIP gather and atomic scatter-add kernels).
"""
from __future__ import annotations

import torch

from . import mips


class TopKScores(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, I, K, precision="bf16", recompute_idx=False):
        idx, score = mips.bmm_topk(U.detach(), I.detach(), K, precision)
        ctx.K = K
        ctx.precision = precision
        ctx.recompute = bool(recompute_idx)
        if ctx.recompute:
            ctx.save_for_backward(U, I)
        else:
            ctx.save_for_backward(U, I, idx)
        ctx.mark_non_differentiable(idx)
        return score.to(torch.float32), idx

    @staticmethod
    def backward(ctx, grad_scores, grad_idx):
        if ctx.recompute:
            U, I = ctx.saved_tensors
            idx, _ = mips.bmm_topk(U.detach(), I.detach(), ctx.K, ctx.precision)
        else:
            U, I, idx = ctx.saved_tensors
        if grad_scores is None:
            return None, None, None, None, None
        dU, dI = mips.topk_backward(U.detach(), I.detach(), idx, grad_scores)
        return dU, dI, None, None, None


def topk_scores(U, I, K, precision="bf16", recompute_idx=False):
    """(scores float32 [n_u, K] differentiable w.r.t. U and I, idx int32 [n_u, K])."""
    return TopKScores.apply(U, I, K, precision, recompute_idx)
