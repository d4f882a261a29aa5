"""Learned normalised min-sum as a torch.autograd.Function.

The forward and the gradient run in the library's kernels (ldpc_nms_fwd and
its hand-written adjoint ldpc_nms_bwd, with per-iteration checkpoints);
PyTorch provides device memory, the stream and the optimiser.
"""
from __future__ import annotations

import numpy as np
import torch

from . import ldpc_nms_bwd, ldpc_nms_fwd, ldpc_quantize_weights


class NMSLoss(torch.autograd.Function):
    """loss[t] for t < T (their sum is the mean per-bit BCE over iterations)
    of the learned decoder with weights w [T][Mb][Nb] on frames llr [F][N]
    with transmitted codewords cw [F][N]."""

    @staticmethod
    def forward(ctx, w, llr, cw, hbm, Z):
        w = w.detach().contiguous()
        loss, ckpt, _ = ldpc_nms_fwd(hbm, Z, llr, cw, w)
        ctx.hbm, ctx.Z = np.asarray(hbm, dtype=np.int16), Z
        ctx.save_for_backward(w, cw, ckpt)
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        w, cw, ckpt = ctx.saved_tensors
        grad_w = ldpc_nms_bwd(ctx.hbm, ctx.Z, cw, w, ckpt, grad_loss.contiguous().float())
        return grad_w, None, None, None, None


def nms_loss(w, llr, cw, hbm, Z):
    """Per-iteration losses [T]; differentiable with respect to w."""
    return NMSLoss.apply(w, llr, cw, hbm, Z)


def quantize_weights(w):
    """1/16-step weights for the int8 decoder, wq = clamp(rint(16 w), 0, 31),
    computed by the library (ldpc_quantize_weights)."""
    return ldpc_quantize_weights(w.detach().float().contiguous())
