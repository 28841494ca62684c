"""Autograd glue for the unrolled decoder: forward and backward are the HIP
kernels behind pbp_unrolled_forward / pbp_unrolled_backward; this module
only keeps the per-iteration checkpoints between the two calls."""

import torch

from .binding import pbp_unrolled_backward, pbp_unrolled_forward


class UnrolledBP(torch.autograd.Function):
    """out = R^T at column m+1 of T unrolled BP iterations with scales
    alpha (T, m, 2); differentiable in llr (B, N) and alpha."""

    @staticmethod
    def forward(ctx, llr, alpha, code):
        llr = llr.detach().contiguous()
        alpha = alpha.detach().contiguous()
        out, ckpt = pbp_unrolled_forward(code, llr, alpha, ckpt=True)
        ctx.code = code
        ctx.save_for_backward(llr, alpha, ckpt)
        return out

    @staticmethod
    def backward(ctx, dout):
        llr, alpha, ckpt = ctx.saved_tensors
        dalpha, dllr, _ = pbp_unrolled_backward(
            ctx.code, llr, alpha, ckpt, dout.contiguous(),
            dllr=ctx.needs_input_grad[0])
        return (dllr if ctx.needs_input_grad[0] else None,
                dalpha if ctx.needs_input_grad[1] else None, None)


def unrolled_bp(llr, alpha, code):
    return UnrolledBP.apply(llr, alpha, code)


def info_bce(out, u_info, info_pos):
    """Mean binary cross-entropy of the information bits under the output
    LLRs (P(u = 1) = sigmoid(-LLR)): softplus(-(1 - 2u) LLR)."""
    z = out[:, info_pos]
    return torch.nn.functional.softplus(-(1.0 - 2.0 * u_info) * z).mean()
