"""torch.autograd.Function for y = A(values) x with a hand-written backward.

Forward: csr_spmv / csr_spmm.  Backward (both on the GPU through the C ABI):
  d values[p] = dY[row(p), :] . X[colind[p], :]   (csr_sddmm, sampled dot)
  d X         = A^T dY                            (csr_spmv_t: CSC-index gather,
                                                   or atomic scatter)
y is bilinear in (values, x), so these are the exact gradients.
"""
from __future__ import annotations

import torch

from .ops import CSR, Plan, default_opts, sddmm, spmm, spmv, spmv_t, transpose_index


class GradContext:
    """Per-pattern state reused across calls: forward plan, CSC index and the
    plan of the CSC pattern (for the deterministic transpose)."""

    def __init__(self, A: CSR, mode: int = 0, plans: bool = True, k: int = 1):
        self.A = A
        self.mode = mode
        self.plan = Plan.for_matrix(A, default_opts(k, A.values.dtype)) if plans else None
        self.index = transpose_index(A) if mode == 0 else None
        self.plan_t = None
        if plans and mode == 0:
            self.plan_t = Plan(self.index.colptr, A.n, A.m, A.nnz, default_opts(k, A.values.dtype))


class SpMVFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values: torch.Tensor, x: torch.Tensor, gctx: GradContext):
        A = gctx.A.with_values(values)
        y = spmv(A, x, plan=gctx.plan) if x.dim() == 1 else spmm(A, x, plan=gctx.plan)
        ctx.save_for_backward(values, x)
        ctx.gctx = gctx
        return y

    @staticmethod
    def backward(ctx, dy: torch.Tensor):
        values, x = ctx.saved_tensors
        g = ctx.gctx
        A = g.A.with_values(values)
        dy = dy.contiguous()
        dvalues = dx = None
        if ctx.needs_input_grad[0]:
            dvalues = sddmm(A, dy, x, plan=g.plan)
        if ctx.needs_input_grad[1]:
            if g.mode == 0:
                dx = spmv_t(A, dy, mode=0, index=g.index, plan=g.plan_t)
            else:
                dx = spmv_t(A, dy, mode=1, plan=g.plan)
        return dvalues, dx, None


def spmv_autograd(values: torch.Tensor, x: torch.Tensor, gctx: GradContext) -> torch.Tensor:
    return SpMVFunction.apply(values, x, gctx)
