"""torch.autograd.Function for C = A B through a fast-multiplication plan.

Forward: fastmm_gemm with the plan's rule.  Backward: fastmm_gemm_backward, which computes
dA = G B^T and dB = A^T G with rules derived from the same rule by the symmetries of section 3.1
(the transpose of the rotation [V,W,U] for the <M0,N0,K0> product G B^T, the transpose of
[W,U,V] for the <K0,M0,N0> product A^T G), at the plan's depth, cutoff, scaling and precision,
reading B^T and A^T through transpose flags.  Argument marshalling only; the arithmetic runs in
libfastmm.so.
"""
from __future__ import annotations

import torch

from .fastmm import Plan, fastmm_gemm, fastmm_gemm_backward


class FastMatmulFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, B, plan: Plan):
        ctx.plan = plan
        ctx.save_for_backward(A, B)
        return fastmm_gemm(plan, A.contiguous(), B.contiguous())

    @staticmethod
    def backward(ctx, G):
        A, B = ctx.saved_tensors
        need_a, need_b = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_a or need_b):
            return None, None, None
        dA, dB = fastmm_gemm_backward(ctx.plan, A, B, G.contiguous(), need_a, need_b)
        return dA, dB, None


def fast_matmul(A, B, plan: Plan):
    """Differentiable C = A B computed by `plan` (forward and backward on the GPU)."""
    return FastMatmulFn.apply(A, B, plan)
