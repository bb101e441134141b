"""``torch.autograd.Function`` for the sampled-entry tensor-ring loss

    L = 1/(2B) * sum_b (Trace(G_1(i_1^b) ... G_N(i_N^b)) - x_b)^2,

forward and backward both in the library's HIP kernels (tr_entry_fwd,
tr_entry_bwd).  The backward recomputes each core's environment from the
cores; only the residuals are saved.  Cores are FP32 tensors in the
G_{k(2)} layout (I_k x R_k R_{k+1})."""
from __future__ import annotations

import torch

from . import api


class TRContract(torch.autograd.Function):
    @staticmethod
    def forward(ctx, desc, idx, x, *cores):
        B = idx.shape[0]
        resid, loss = api.tr_entry_fwd(desc, list(cores), idx, x, B)
        ctx.desc = desc
        ctx.save_for_backward(idx, resid, *cores)
        return loss

    @staticmethod
    def backward(ctx, gloss):
        idx, resid, *cores = ctx.saved_tensors
        B = idx.shape[0]
        g = gloss.detach().to(torch.float64).contiguous()
        grads = api.tr_entry_bwd(ctx.desc, cores, idx, resid, B, scale_dev=g)
        return (None, None, None, *grads)


def tr_entry_loss(desc, idx, x, cores):
    """Differentiable sampled-entry loss (FP64 scalar tensor)."""
    return TRContract.apply(desc, idx, x, *cores)
