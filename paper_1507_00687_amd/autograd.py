"""torch.autograd.Function for C = A B through a fast-multiplication plan.

Forward: fastmm_gemm with the plan's rule.  Backward: fastmm_gemm_backward, which computes
dA = G B^T and dB = A^T G with the cyclic rotations of the same rule ([V,W,U] for the
<K0,N0,M0> product B G^T and [W,U,V] for the <N0,M0,K0> product G^T A), at the plan's depth,
cutoff, scaling and precision.  Argument marshalling only; the arithmetic runs in libfastmm.so.
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
