"""torch.autograd.Function for y = A(values) x with a hand-written backward.

Forward: csr_spmv / csr_spmm.  Backward (both on the GPU through the C ABI):
  d values[p] = dY[row(p), :] . X[colind[p], :]   (csr_sddmm, sampled dot)
When the values need a gradient and x is a vector, the forward runs
csr_spmv_save, which also stores every gathered x[colind[p]]; the sampled dot
then streams that copy (csr_sddmm_saved, bitwise the same result) instead of
gathering x a second time, for nnz more elements written and kept.
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

from .ops import (CSCIndex, CSR, Plan, csc_value_map, default_opts, sddmm, sddmm_saved, spmm, spmv, spmv_save,
                  spmv_t, transpose_index, values_to_csc)


class GradContext:
    """Per-pattern state reused across calls: forward plans, CSC index and the
    plans of the CSC pattern (for the deterministic transpose).  Plans are
    kept per number of right-hand sides k (a plan with split rows serves
    products up to its max_k), so a 2-D X of any width gets a plan built for
    it on first use; `k` only picks the plans built up front.  `save_gather`
    lets a vector forward keep its gathered operand for the sampled dot."""

    def __init__(self, A: CSR, mode: int = 0, plans: bool = True, k: int = 1, csc_values: bool = True,
                 save_gather: bool = True):
        self.A = A
        self.mode = mode
        self.save_gather = save_gather
        self.plans = plans
        self._fwd = {}
        self._csc = {}
        self.index = transpose_index(A) if mode == 0 else None
        self.vmap = csc_value_map(self.index) if (mode == 0 and csc_values) else None
        self.index_v = CSCIndex(self.index.colptr, self.index.rowind, None) if self.vmap is not None else None
        self.plan = self.plan_for(k)
        self.plan_t = self.plan_t_for(k)

    def plan_for(self, k: int):
        """Plan of the CSR pattern for products with k right-hand sides."""
        if not self.plans:
            return None
        if k not in self._fwd:
            self._fwd[k] = Plan.for_matrix(self.A, default_opts(k, self.A.values.dtype))
        return self._fwd[k]

    def plan_t_for(self, k: int):
        """Plan of the CSC pattern (n rows) for the mode-0 transpose with k columns."""
        if not self.plans or self.mode != 0:
            return None
        if k not in self._csc:
            A = self.A
            self._csc[k] = Plan(self.index.colptr, A.n, A.m, A.nnz, default_opts(k, A.values.dtype))
        return self._csc[k]

    def transpose(self, A: CSR, dy: torch.Tensor) -> torch.Tensor:
        """A^T dy by this context's mode."""
        k = 1 if dy.dim() == 1 else dy.shape[1]
        if self.mode != 0:
            return spmv_t(A, dy, mode=1, plan=self.plan)
        plan_t = self.plan_t_for(k)
        if self.vmap is None:
            return spmv_t(A, dy, mode=0, index=self.index, plan=plan_t)
        vcsc = values_to_csc(A.values, self.vmap)
        return spmv_t(A.with_values(vcsc), dy, mode=0, index=self.index_v, plan=plan_t)


class SpMVFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values: torch.Tensor, x: torch.Tensor, gctx: GradContext):
        A = gctx.A.with_values(values)
        ctx.xsave = None
        if x.dim() == 1 and gctx.save_gather and ctx.needs_input_grad[0]:
            y, ctx.xsave = spmv_save(A, x, plan=gctx.plan_for(1))
        elif x.dim() == 1:
            y = spmv(A, x, plan=gctx.plan_for(1))
        else:
            y = spmm(A, x, plan=gctx.plan_for(x.shape[1]))
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
        if ctx.needs_input_grad[0] and ctx.xsave is not None:
            dvalues = sddmm_saved(A, dy, ctx.xsave, plan=g.plan_for(1))
            ctx.xsave = None
        elif ctx.needs_input_grad[0]:
            dvalues = sddmm(A, dy, x, plan=g.plan)
        if ctx.needs_input_grad[1]:
            dx = g.transpose(A, dy)
        return dvalues, dx, None


def spmv_autograd(values: torch.Tensor, x: torch.Tensor, gctx: GradContext) -> torch.Tensor:
    return SpMVFunction.apply(values, x, gctx)
