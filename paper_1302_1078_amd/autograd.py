"""torch.autograd.Function for y = A(values) x with a hand-written backward.

Forward: csr_spmv / csr_spmm.  Backward (both on the GPU through the C ABI):
  d values[p] = dY[row(p), :] . X[colind[p], :]   (csr_sddmm, sampled dot)
  d X         = A^T dY                            (csr_spmv_t: CSC-index gather,
                                                   or atomic scatter)
With the CSC index (mode 0) and csc_values, the values are first moved to CSC
order by the two-pass block transposition (csr_values_to_csc), so the gather
reads them in sequence instead of through perm; the result is bitwise the
same.
y is bilinear in (values, x), so these are the exact gradients.
"""
from __future__ import annotations

import torch

from .ops import (CSCIndex, CSR, Plan, csc_value_map, default_opts, sddmm, spmm, spmv, spmv_t, transpose_index,
                  values_to_csc)


class GradContext:
    """Per-pattern state reused across calls: forward plan, CSC index and the
    plan of the CSC pattern (for the deterministic transpose)."""

    def __init__(self, A: CSR, mode: int = 0, plans: bool = True, k: int = 1, csc_values: bool = True):
        self.A = A
        self.mode = mode
        self.plan = Plan.for_matrix(A, default_opts(k, A.values.dtype)) if plans else None
        self.index = transpose_index(A) if mode == 0 else None
        self.plan_t = None
        if plans and mode == 0:
            self.plan_t = Plan(self.index.colptr, A.n, A.m, A.nnz, default_opts(k, A.values.dtype))
        self.vmap = csc_value_map(self.index) if (mode == 0 and csc_values) else None
        self.index_v = CSCIndex(self.index.colptr, self.index.rowind, None) if self.vmap is not None else None

    def transpose(self, A: CSR, dy: torch.Tensor) -> torch.Tensor:
        """A^T dy by this context's mode."""
        if self.mode != 0:
            return spmv_t(A, dy, mode=1, plan=self.plan)
        if self.vmap is None:
            return spmv_t(A, dy, mode=0, index=self.index, plan=self.plan_t)
        vcsc = values_to_csc(A.values, self.vmap)
        return spmv_t(A.with_values(vcsc), dy, mode=0, index=self.index_v, plan=self.plan_t)


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
            dx = g.transpose(A, dy)
        return dvalues, dx, None


def spmv_autograd(values: torch.Tensor, x: torch.Tensor, gctx: GradContext) -> torch.Tensor:
    return SpMVFunction.apply(values, x, gctx)
