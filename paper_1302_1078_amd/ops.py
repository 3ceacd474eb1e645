"""Python binding of the CSR library: argument marshalling only.

Every operation here calls one C entry point of libspx.so on the caller's
current torch stream; all arithmetic runs in the library's HIP kernels.
PyTorch provides device memory (tensors) and streams.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import PlanOpts, check

_DT = {torch.float64: _lib.SPX_F64, torch.float32: _lib.SPX_F32, torch.bfloat16: _lib.SPX_BF16}


def dtype_code(t: torch.Tensor) -> int:
    try:
        return _DT[t.dtype]
    except KeyError:
        raise TypeError(f"unsupported dtype {t.dtype}") from None


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("tensors must live on the GPU (no CPU path)")


def _contig(*ts):
    for t in ts:
        if t is not None and not t.is_contiguous():
            raise ValueError("tensors must be contiguous")


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


@dataclass
class CSR:
    """CSR matrix on the device: rowptr int32[m+1], colind int32[nnz], values[nnz]."""
    rowptr: torch.Tensor
    colind: torch.Tensor
    values: torch.Tensor
    shape: tuple

    @property
    def m(self) -> int:
        return int(self.shape[0])

    @property
    def n(self) -> int:
        return int(self.shape[1])

    @property
    def nnz(self) -> int:
        return int(self.colind.numel())

    @property
    def device(self):
        return self.rowptr.device

    def with_values(self, values: torch.Tensor) -> "CSR":
        if values.numel() != self.nnz:
            raise ValueError("values length differs from nnz")
        return CSR(self.rowptr, self.colind, values, self.shape)


def version() -> str:
    return _lib.load().spx_version().decode()


def default_opts(k: int = 1, vtype=torch.float64) -> PlanOpts:
    o = PlanOpts()
    code = vtype if isinstance(vtype, int) else _DT[vtype]
    check(_lib.load().spx_plan_default_opts(k, code, ctypes.byref(o)), "spx_plan_default_opts")
    return o


# ---------------------------------------------------------------- assembly and validation

def from_coo(m: int, n: int, r: torch.Tensor, c: torch.Tensor, v: torch.Tensor) -> CSR:
    """Canonical CSR from triplets (device int32 r, c and float64 v)."""
    L = _lib.load()
    _dev(r, c, v)
    _contig(r, c, v)
    if r.dtype != torch.int32 or c.dtype != torch.int32 or v.dtype != torch.float64:
        raise TypeError("r, c must be int32 and v float64")
    nnz_in = int(r.numel())
    dev = r.device
    ws_bytes = ctypes.c_size_t()
    check(L.csr_from_coo_workspace_bytes(m, n, nnz_in, ctypes.byref(ws_bytes)), "csr_from_coo")
    ws = _workspace(ws_bytes.value, dev)
    rowptr = torch.empty(m + 1, dtype=torch.int32, device=dev)
    colind = torch.empty(max(nnz_in, 1), dtype=torch.int32, device=dev)
    values = torch.empty(max(nnz_in, 1), dtype=torch.float64, device=dev)
    nnz_out = torch.empty(1, dtype=torch.int32, device=dev)
    check(L.csr_from_coo(m, n, nnz_in, _ptr(r), _ptr(c), _ptr(v), _ptr(rowptr), _ptr(colind),
                         _ptr(values), _ptr(nnz_out), _ptr(ws), ws_bytes.value, _stream()),
          "csr_from_coo")
    t = int(nnz_out.item())
    if t < 0:
        raise ValueError("csr_from_coo: a triplet index is out of range")
    return CSR(rowptr, colind[:t], values[:t], (m, n))


def from_coo_host(m: int, n: int, r, c, v):
    """Canonical CSR from host triplets (numpy int32 r, c and float64 v), on
    the host through csr_from_coo_host; returns numpy (rowptr, colind, values)."""
    import numpy as np
    L = _lib.load()
    r = np.ascontiguousarray(r, dtype=np.int32)
    c = np.ascontiguousarray(c, dtype=np.int32)
    v = np.ascontiguousarray(v, dtype=np.float64)
    if not (r.shape == c.shape == v.shape) or r.ndim != 1:
        raise ValueError("r, c and v must be 1-D arrays of one length")
    nnz_in = int(r.size)
    rowptr = np.empty(m + 1, dtype=np.int32)
    colind = np.empty(max(nnz_in, 1), dtype=np.int32)
    values = np.empty(max(nnz_in, 1), dtype=np.float64)
    nnz_out = ctypes.c_int32()
    check(L.csr_from_coo_host(m, n, nnz_in, r.ctypes.data, c.ctypes.data, v.ctypes.data, rowptr.ctypes.data,
                              colind.ctypes.data, values.ctypes.data, ctypes.byref(nnz_out)),
          "csr_from_coo_host")
    t = nnz_out.value
    return rowptr, colind[:t].copy(), values[:t].copy()


def validate_host(m: int, n: int, rowptr, colind) -> None:
    """Raise SpxError unless the host CSR arrays are structurally valid."""
    import numpy as np
    L = _lib.load()
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    colind = np.ascontiguousarray(colind, dtype=np.int32)
    if rowptr.size != m + 1:
        raise ValueError("rowptr must have m + 1 entries")
    check(L.csr_validate_host(m, n, int(colind.size), rowptr.ctypes.data, colind.ctypes.data),
          "csr_validate_host")


def validate(A: CSR, check_sorted: bool = True) -> int:
    L = _lib.load()
    status = torch.empty(1, dtype=torch.int32, device=A.device)
    check(L.csr_validate(A.m, A.n, A.nnz, _ptr(A.rowptr), _ptr(A.colind), int(check_sorted),
                         _ptr(status), _stream()), "csr_validate")
    return int(status.item())


# ---------------------------------------------------------------- plans

class Plan:
    """Row-binning plan of one sparsity pattern; owns its device workspace."""

    def __init__(self, rowptr: torch.Tensor, m: int, n: int, nnz: int, opts: PlanOpts | None = None):
        L = _lib.load()
        _dev(rowptr)
        self.opts = opts if opts is not None else default_opts(1)
        self.m, self.n, self.nnz = m, n, nnz
        nb = ctypes.c_size_t()
        check(L.csr_plan_workspace_bytes(m, nnz, ctypes.byref(self.opts), ctypes.byref(nb)),
              "csr_plan_workspace_bytes")
        self.workspace = _workspace(nb.value, rowptr.device)
        h = ctypes.c_void_p()
        check(L.csr_plan_create(m, n, nnz, _ptr(rowptr), ctypes.byref(self.opts), _ptr(self.workspace),
                                nb.value, _stream(), ctypes.byref(h)), "csr_plan_create")
        self.handle = h

    @classmethod
    def for_matrix(cls, A: CSR, opts: PlanOpts | None = None, k: int = 1) -> "Plan":
        return cls(A.rowptr, A.m, A.n, A.nnz, opts if opts is not None else default_opts(k, A.values.dtype))

    @classmethod
    def staged(cls, A: CSR, k: int, xdtype=torch.float64, pipelined: bool = False) -> "Plan":
        """Staged plan (csr_plan_create_staged): tiles of consecutive rows whose
        X windows are copied into LDS, for SpMM with exactly this k and X type.
        pipelined: run the persistent double-buffered kernel
        (csr_plan_staged_pipeline)."""
        L = _lib.load()
        _dev(A.rowptr, A.colind)
        xt = _lib.SPX_F64 if xdtype == torch.float64 else _lib.SPX_F32
        self = cls.__new__(cls)
        self.opts = default_opts(k, A.values.dtype)
        self.m, self.n, self.nnz = A.m, A.n, A.nnz
        nb = ctypes.c_size_t()
        check(L.csr_plan_staged_workspace_bytes(A.m, A.n, A.nnz, k, xt, ctypes.byref(nb)),
              "csr_plan_staged_workspace_bytes")
        self.workspace = _workspace(nb.value, A.device)
        h = ctypes.c_void_p()
        check(L.csr_plan_create_staged(A.m, A.n, A.nnz, _ptr(A.rowptr), _ptr(A.colind), k, xt,
                                       _ptr(self.workspace), nb.value, _stream(), ctypes.byref(h)),
              "csr_plan_create_staged")
        self.handle = h
        if pipelined:
            check(L.csr_plan_staged_pipeline(h, 1), "csr_plan_staged_pipeline")
        return self

    def attach_hot_x(self, A: CSR, hot: int, xdtype=torch.float64) -> "Plan":
        """Keep the x entries of the `hot` most-used columns in LDS for SpMV
        through this plan (csr_plan_attach_hot_x).  Returns self."""
        L = _lib.load()
        _dev(A.rowptr, A.colind)
        xt = _lib.SPX_F64 if xdtype == torch.float64 else _lib.SPX_F32
        nb = ctypes.c_size_t()
        check(L.csr_plan_hot_x_workspace_bytes(A.n, A.nnz, hot, ctypes.byref(nb)), "csr_plan_hot_x_workspace_bytes")
        self.hot_workspace = _workspace(nb.value, A.device)
        check(L.csr_plan_attach_hot_x(self.handle, A.n, A.nnz, _ptr(A.colind), hot, xt, _ptr(self.hot_workspace),
                                      nb.value, _stream()), "csr_plan_attach_hot_x")
        return self

    def staged_info(self) -> dict:
        a, b, c, d = (ctypes.c_int32() for _ in range(4))
        check(_lib.load().csr_plan_staged_info(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                               ctypes.byref(d)), "csr_plan_staged_info")
        return {"tile_rows": a.value, "tiles": b.value, "staged_tiles": c.value, "max_window_rows": d.value}

    def export_bins(self):
        import numpy as np
        nb = self.opts.nbins
        perm = np.empty(max(self.m, 1), dtype=np.int32)
        off = np.empty(nb + 1, dtype=np.int32)
        check(_lib.load().csr_plan_export_bins(self.handle, perm.ctypes.data_as(ctypes.c_void_p),
                                               off.ctypes.data_as(ctypes.c_void_p)), "export_bins")
        return perm[:self.m], off

    def info(self) -> dict:
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(_lib.load().csr_plan_info(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
              "csr_plan_info")
        return {"nbins": a.value, "split_rows": b.value, "segments": c.value}

    @property
    def ptr(self):
        return self.handle

    def __del__(self):
        # at interpreter exit the module globals may already be gone
        h = getattr(self, "handle", None)
        lib = getattr(_lib, "_lib", None) if _lib is not None else None
        if h is not None and h.value and lib is not None:
            lib.csr_plan_destroy(h)
            self.handle = None


def _plan_ptr(plan):
    return plan.handle if plan is not None else ctypes.c_void_p(0)


# ---------------------------------------------------------------- products

def spmv(A: CSR, x: torch.Tensor, y: torch.Tensor | None = None, plan: Plan | None = None) -> torch.Tensor:
    """y <- A x."""
    L = _lib.load()
    _dev(A.rowptr, x)
    _contig(x)
    if x.numel() < A.n:
        raise ValueError(f"x has {x.numel()} entries, A has {A.n} columns")
    if y is None:
        y = torch.empty(A.m, dtype=x.dtype, device=x.device)
    _contig(y)
    if y.numel() < A.m or y.dtype != x.dtype:
        raise ValueError("y must hold m entries of x's dtype")
    check(L.csr_spmv(A.m, A.n, A.nnz, _ptr(A.rowptr), _ptr(A.colind), _ptr(A.values),
                     dtype_code(A.values), _ptr(x), _ptr(y), dtype_code(x), _plan_ptr(plan), _stream()),
          "csr_spmv")
    return y


def spmv_save(A: CSR, x: torch.Tensor, y: torch.Tensor | None = None, xsave: torch.Tensor | None = None,
              plan: Plan | None = None) -> tuple[torch.Tensor, torch.Tensor]:
    """y <- A x, keeping xsave[p] = x[colind[p]] (nnz entries of x's dtype)
    for sddmm_saved.  Returns (y, xsave)."""
    L = _lib.load()
    _dev(A.rowptr, x)
    _contig(x)
    if x.numel() < A.n:
        raise ValueError(f"x has {x.numel()} entries, A has {A.n} columns")
    if y is None:
        y = torch.empty(A.m, dtype=x.dtype, device=x.device)
    if xsave is None:
        xsave = torch.empty(A.nnz, dtype=x.dtype, device=x.device)
    _contig(y)
    _contig(xsave)
    if y.numel() < A.m or y.dtype != x.dtype:
        raise ValueError("y must hold m entries of x's dtype")
    if xsave.numel() < A.nnz or xsave.dtype != x.dtype:
        raise ValueError("xsave must hold nnz entries of x's dtype")
    check(L.csr_spmv_save(A.m, A.n, A.nnz, _ptr(A.rowptr), _ptr(A.colind), _ptr(A.values),
                          dtype_code(A.values), _ptr(x), _ptr(y), dtype_code(x), _ptr(xsave), _plan_ptr(plan),
                          _stream()), "csr_spmv_save")
    return y, xsave


def spmm(A: CSR, X: torch.Tensor, Y: torch.Tensor | None = None, plan: Plan | None = None) -> torch.Tensor:
    """Y <- A X with X (n x k) and Y (m x k) row-major (unit column stride)."""
    L = _lib.load()
    _dev(A.rowptr, X)
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be 2-D with unit column stride")
    k = X.shape[1]
    if X.shape[0] < A.n:
        raise ValueError(f"X has {X.shape[0]} rows, A has {A.n} columns")
    if Y is None:
        Y = torch.empty((A.m, k), dtype=X.dtype, device=X.device)
    if Y.dim() != 2 or Y.stride(1) != 1 or Y.shape[0] < A.m or Y.shape[1] != k or Y.dtype != X.dtype:
        raise ValueError("Y must be m x k with unit column stride and X's dtype")
    check(L.csr_spmm(A.m, A.n, A.nnz, _ptr(A.rowptr), _ptr(A.colind), _ptr(A.values),
                     dtype_code(A.values), k, _ptr(X), X.stride(0), _ptr(Y), Y.stride(0), dtype_code(X),
                     _plan_ptr(plan), _stream()), "csr_spmm")
    return Y


# ---------------------------------------------------------------- transpose and gradients

@dataclass
class CSCIndex:
    colptr: torch.Tensor
    rowind: torch.Tensor
    perm: torch.Tensor


def transpose_index(A: CSR) -> CSCIndex:
    L = _lib.load()
    dev = A.device
    nb = ctypes.c_size_t()
    check(L.csr_transpose_index_workspace_bytes(A.m, A.n, A.nnz, ctypes.byref(nb)), "transpose_index")
    ws = _workspace(nb.value, dev)
    colptr = torch.empty(A.n + 1, dtype=torch.int32, device=dev)
    rowind = torch.empty(max(A.nnz, 1), dtype=torch.int32, device=dev)
    perm = torch.empty(max(A.nnz, 1), dtype=torch.int32, device=dev)
    check(L.csr_transpose_index(A.m, A.n, A.nnz, _ptr(A.rowptr), _ptr(A.colind), _ptr(colptr),
                                _ptr(rowind), _ptr(perm), _ptr(ws), nb.value, _stream()),
          "csr_transpose_index")
    return CSCIndex(colptr, rowind[:A.nnz], perm[:A.nnz])


@dataclass
class CSCValueMap:
    """One-time map of a pattern for csr_values_to_csc (dest int32[nnz],
    local uint16[nnz] stored as int16)."""
    dest: torch.Tensor
    local: torch.Tensor


def csc_value_map(index: CSCIndex) -> CSCValueMap:
    L = _lib.load()
    perm = index.perm
    nnz = perm.numel()
    nb = ctypes.c_size_t()
    check(L.csr_csc_value_map_workspace_bytes(nnz, ctypes.byref(nb)), "csr_csc_value_map")
    ws = _workspace(nb.value, perm.device)
    dest = torch.empty(max(nnz, 1), dtype=torch.int32, device=perm.device)
    local = torch.empty(max(nnz, 1), dtype=torch.int16, device=perm.device)
    check(L.csr_csc_value_map(nnz, _ptr(perm), _ptr(dest), _ptr(local), _ptr(ws), nb.value, _stream()),
          "csr_csc_value_map")
    return CSCValueMap(dest[:nnz], local[:nnz])


def values_to_csc(values: torch.Tensor, vmap: CSCValueMap, staging: torch.Tensor | None = None,
                  out: torch.Tensor | None = None) -> torch.Tensor:
    """values[perm] in CSC order through the two-pass block transposition
    (csr_values_to_csc)."""
    _dev(values)
    _contig(values)
    nnz = values.numel()
    if vmap.dest.numel() != nnz:
        raise ValueError("values_to_csc: map and values differ in size")
    staging = torch.empty_like(values) if staging is None else staging
    out = torch.empty_like(values) if out is None else out
    check(_lib.load().csr_values_to_csc(nnz, _ptr(vmap.dest), _ptr(vmap.local), _ptr(values), dtype_code(values),
                                        _ptr(staging), _ptr(out), _stream()), "csr_values_to_csc")
    return out


def spmv_t(A: CSR, dY: torch.Tensor, mode: int = 0, index: CSCIndex | None = None,
           plan: Plan | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
    """dX <- A^T dY.  mode 0: deterministic gather over the CSC index (plan, if
    given, is a plan of the CSC pattern; an index whose perm is None means
    A.values are already in CSC order); mode 1: atomic scatter (plan of the
    CSR pattern)."""
    L = _lib.load()
    _dev(A.rowptr, dY)
    vec = dY.dim() == 1
    k = 1 if vec else dY.shape[1]
    if dY.shape[0] < A.m or (not vec and dY.stride(1) != 1) or (vec and not dY.is_contiguous()):
        raise ValueError("dY must have m rows and unit column stride")
    if out is None:
        out = torch.empty((A.n,) if vec else (A.n, k), dtype=dY.dtype, device=dY.device)
    if out.shape[0] < A.n or out.dim() != dY.dim() or (not vec and out.stride(1) != 1):
        raise ValueError("out must have n rows and unit column stride")
    lddy = 1 if vec else dY.stride(0)
    lddx = 1 if vec else out.stride(0)
    if mode == 0 and index is None:
        index = transpose_index(A)
    cp, ri, pm = (index.colptr, index.rowind, index.perm) if index is not None else (None, None, None)
    check(L.csr_spmv_t(A.m, A.n, A.nnz, _ptr(A.rowptr), _ptr(A.colind), _ptr(cp), _ptr(ri), _ptr(pm),
                       _ptr(A.values), dtype_code(A.values), k, _ptr(dY), lddy, _ptr(out), lddx,
                       dtype_code(dY), mode, _plan_ptr(plan), _stream()), "csr_spmv_t")
    return out


def sddmm(A: CSR, dY: torch.Tensor, X: torch.Tensor, plan: Plan | None = None,
          out: torch.Tensor | None = None) -> torch.Tensor:
    """out[p] = dY[row(p), :] . X[colind[p], :] for each stored nonzero p."""
    L = _lib.load()
    _dev(A.rowptr, dY, X)
    vec = dY.dim() == 1
    k = 1 if vec else dY.shape[1]
    if dY.shape[0] < A.m or X.shape[0] < A.n or X.dim() != dY.dim() or X.dtype != dY.dtype:
        raise ValueError("dY must have m rows and X n rows, same rank and dtype")
    if not vec and (X.shape[1] != k or dY.stride(1) != 1 or X.stride(1) != 1):
        raise ValueError("dY and X must be k wide with unit column stride")
    if out is None:
        out = torch.empty(A.nnz, dtype=dY.dtype, device=dY.device)
    if out.numel() < A.nnz or not out.is_contiguous():
        raise ValueError("out must hold nnz entries")
    check(L.csr_sddmm(A.m, A.n, A.nnz, _ptr(A.rowptr), _ptr(A.colind), k, _ptr(dY),
                      1 if vec else dY.stride(0), _ptr(X), 1 if vec else X.stride(0), _ptr(out),
                      dtype_code(dY), _plan_ptr(plan), _stream()), "csr_sddmm")
    return out


def sddmm_saved(A: CSR, dy: torch.Tensor, xsave: torch.Tensor, plan: Plan | None = None,
                out: torch.Tensor | None = None) -> torch.Tensor:
    """out[p] = dy[row(p)] * xsave[p], with xsave from spmv_save (k = 1):
    bitwise sddmm(A, dy, x) for the x that was saved."""
    L = _lib.load()
    _dev(A.rowptr, dy, xsave)
    _contig(dy)
    _contig(xsave)
    if dy.dim() != 1 or dy.numel() < A.m or xsave.numel() < A.nnz or xsave.dtype != dy.dtype:
        raise ValueError("dy must be a vector of m entries and xsave hold nnz entries of its dtype")
    if out is None:
        out = torch.empty(A.nnz, dtype=dy.dtype, device=dy.device)
    if out.numel() < A.nnz or not out.is_contiguous():
        raise ValueError("out must hold nnz entries")
    check(L.csr_sddmm_saved(A.m, A.nnz, _ptr(A.rowptr), _ptr(dy), _ptr(xsave), _ptr(out), dtype_code(dy),
                            _plan_ptr(plan), _stream()), "csr_sddmm_saved")
    return out


# ---------------------------------------------------------------- ordering and metrics

def _host_pattern(A: CSR):
    rp = A.rowptr.detach().to("cpu", torch.int32).contiguous()
    ci = A.colind.detach().to("cpu", torch.int32).contiguous()
    return rp, ci


def rcm(A: CSR) -> torch.Tensor:
    """Reverse Cuthill-McKee order (csr_rcm, host): device int32 perm, perm[new] = old."""
    rp, ci = _host_pattern(A)
    perm = torch.empty(A.m, dtype=torch.int32)
    check(_lib.load().csr_rcm(A.m, A.n, A.nnz, _ptr(rp), _ptr(ci), _ptr(perm)), "csr_rcm")
    return perm.to(A.device)


def degree_order(A: CSR) -> torch.Tensor:
    """Columns by descending nonzero count, ties ascending (csr_degree_order,
    device): int32 perm, perm[new] = old, for permute()."""
    L = _lib.load()
    _dev(A.colind)
    nb = ctypes.c_size_t()
    check(L.csr_degree_order_workspace_bytes(A.n, A.nnz, ctypes.byref(nb)), "csr_degree_order")
    ws = _workspace(nb.value, A.device)
    perm = torch.empty(max(A.n, 1), dtype=torch.int32, device=A.device)
    check(L.csr_degree_order(A.n, A.nnz, _ptr(A.colind), _ptr(perm), _ptr(ws), nb.value, _stream()),
          "csr_degree_order")
    return perm[:A.n]


def bandwidth(A: CSR) -> int:
    """Largest |colind[p] - row| over the nonzeros (csr_bandwidth, device, Sec. 4.4)."""
    L = _lib.load()
    _dev(A.rowptr, A.colind)
    out = torch.empty(1, dtype=torch.int32, device=A.device)
    check(L.csr_bandwidth(A.m, A.nnz, _ptr(A.rowptr), _ptr(A.colind), _ptr(out), _stream()), "csr_bandwidth")
    return int(out.item())


def banded_opts(A: CSR, k: int = 1, vtype=torch.float64) -> PlanOpts:
    """Default plan options with rows ordered band by band of the matrix's
    bandwidth (spx_plan_opts.row_period): each XCD sweeps its own band."""
    o = default_opts(k, vtype)
    o.row_period = bandwidth(A)
    return o


def permute(A: CSR, perm: torch.Tensor) -> CSR:
    """P A P^T for a device permutation perm[new] = old (csr_permute; FP64 values)."""
    L = _lib.load()
    _dev(perm, A.values)
    _contig(perm)
    if A.m != A.n:
        raise ValueError("permute needs a square matrix")
    if perm.dtype != torch.int32 or perm.numel() != A.m:
        raise ValueError("perm must be int32 with m entries")
    if A.values.dtype != torch.float64:
        raise TypeError("permute takes FP64 values")
    nb = ctypes.c_size_t()
    check(L.csr_permute_workspace_bytes(A.m, A.nnz, ctypes.byref(nb)), "csr_permute")
    ws = _workspace(nb.value, A.device)
    rowptr = torch.empty(A.m + 1, dtype=torch.int32, device=A.device)
    colind = torch.empty(max(A.nnz, 1), dtype=torch.int32, device=A.device)
    values = torch.empty(max(A.nnz, 1), dtype=torch.float64, device=A.device)
    nnz_out = torch.empty(1, dtype=torch.int32, device=A.device)
    check(L.csr_permute(A.m, A.nnz, _ptr(A.rowptr), _ptr(A.colind), _ptr(A.values), _ptr(perm),
                        _ptr(rowptr), _ptr(colind), _ptr(values), _ptr(nnz_out), _ptr(ws), nb.value,
                        _stream()), "csr_permute")
    t = int(nnz_out.item())
    if t < 0:
        raise ValueError("csr_permute: perm is not a permutation")
    return CSR(rowptr, colind[:t], values[:t], (A.m, A.n))


def vector_access(A: CSR, line: int = 16, parts: int = 8, chunk: int = 64) -> float:
    """Expected number of times x is moved from memory (csr_vector_access, host)."""
    rp, ci = _host_pattern(A)
    out = ctypes.c_double()
    check(_lib.load().csr_vector_access(A.m, A.n, A.nnz, _ptr(rp), _ptr(ci), line, parts, chunk,
                                        ctypes.byref(out)), "csr_vector_access")
    return out.value


def tile_lines(A: CSR, line: int = 16, tile: int = 256) -> int:
    """Distinct (tile, x line) pairs over tiles of `tile` consecutive rows
    (csr_tile_lines, host): the x lines a workgroup serving those rows gathers."""
    rp, ci = _host_pattern(A)
    out = ctypes.c_int64()
    check(_lib.load().csr_tile_lines(A.m, A.n, A.nnz, _ptr(rp), _ptr(ci), line, tile, ctypes.byref(out)),
          "csr_tile_lines")
    return out.value


def ucld(A: CSR, line: int = 16) -> float:
    """Useful cacheline density (csr_ucld, host)."""
    rp, ci = _host_pattern(A)
    out = ctypes.c_double()
    check(_lib.load().csr_ucld(A.m, A.nnz, _ptr(rp), _ptr(ci), line, ctypes.byref(out)), "csr_ucld")
    return out.value


# ---------------------------------------------------------------- register blocking

@dataclass
class BCSR:
    """Register-blocked matrix on the device (see csr_to_bcsr in include/spx.h)."""
    m: int
    n: int
    a: int
    b: int
    bitmap: bool
    browptr: torch.Tensor
    bcol: torch.Tensor
    bvals: torch.Tensor
    bmask: torch.Tensor | None
    boff: torch.Tensor | None

    @property
    def nblocks(self) -> int:
        return int(self.bcol.numel()) if self.bcol is not None else 0

    @staticmethod
    def from_csr(A: CSR, a: int, b: int, bitmap: bool = False) -> "BCSR":
        L = _lib.load()
        _dev(A.rowptr, A.colind, A.values)
        if A.values.dtype != torch.float64:
            raise TypeError("register blocking takes FP64 values")
        nb = ctypes.c_size_t()
        check(L.bcsr_workspace_bytes(A.m, A.n, A.nnz, ctypes.byref(nb)), "bcsr_workspace_bytes")
        ws = _workspace(nb.value, A.device)
        cnt = torch.empty(1, dtype=torch.int32, device=A.device)
        check(L.csr_bcsr_count(A.m, A.n, A.nnz, _ptr(A.rowptr), _ptr(A.colind), a, b, _ptr(cnt), _ptr(ws),
                               nb.value, _stream()), "csr_bcsr_count")
        nblocks = int(cnt.item())
        dev = A.device
        mb = -(-A.m // a)
        browptr = torch.empty(mb + 1, dtype=torch.int32, device=dev)
        bcol = torch.empty(max(nblocks, 1), dtype=torch.int32, device=dev)
        bvals = torch.empty(max(A.nnz if bitmap else nblocks * a * b, 1), dtype=torch.float64, device=dev)
        bmask = torch.empty(max(nblocks, 1), dtype=torch.int64, device=dev) if bitmap else None
        boff = torch.empty(max(nblocks, 1), dtype=torch.int32, device=dev) if bitmap else None
        check(L.csr_to_bcsr(A.m, A.n, A.nnz, _ptr(A.rowptr), _ptr(A.colind), _ptr(A.values), a, b, int(bitmap),
                            _ptr(browptr), _ptr(bcol), _ptr(bvals), _ptr(bmask), _ptr(boff), _ptr(ws), nb.value,
                            _stream()), "csr_to_bcsr")
        keep = nblocks
        return BCSR(A.m, A.n, a, b, bitmap, browptr, bcol[:keep],
                    bvals[:A.nnz] if bitmap else bvals[:nblocks * a * b],
                    bmask[:keep] if bitmap else None, boff[:keep] if bitmap else None)

    def stored_bytes(self) -> int:
        """Values, one column index per block, block-row pointers (+ mask and
        offset per block in bitmap form)."""
        extra = 12 * self.nblocks if self.bitmap else 0
        return 8 * int(self.bvals.numel()) + 4 * self.nblocks + 4 * int(self.browptr.numel()) + extra


def bcsr_spmv(B: BCSR, x: torch.Tensor, y: torch.Tensor | None = None, lanes: int = 0) -> torch.Tensor:
    """y <- A x for a register-blocked A (bcsr_spmv), FP64."""
    _dev(x)
    _contig(x)
    if x.dtype != torch.float64 or x.numel() != B.n:
        raise ValueError("x must be float64 with n entries")
    if y is None:
        y = torch.empty(B.m, dtype=torch.float64, device=x.device)
    check(_lib.load().bcsr_spmv(B.m, B.n, B.a, B.b, int(B.bitmap), B.nblocks, _ptr(B.browptr), _ptr(B.bcol),
                                _ptr(B.bvals), _ptr(B.bmask), _ptr(B.boff), _ptr(x), _ptr(y), lanes, _stream()),
          "bcsr_spmv")
    return y


def bcsr_spmm(B: BCSR, X: torch.Tensor, Y: torch.Tensor | None = None, slots: int = 0,
              row_period: int = 0, values: torch.Tensor | None = None) -> torch.Tensor:
    """Y <- A X for a register-blocked A of a x 1 dense blocks (bcsr_spmm); X n x k
    and Y m x k row-major (row strides taken from the tensors).  values: the
    blocks' values in another type (B.bvals converted to float32 or bfloat16,
    with float32 X and Y); default B.bvals, FP64.  row_period: 0, or the rows of
    a period whose bands the XCDs sweep (the matrix's bandwidth for a banded
    matrix; bitwise the same result)."""
    _dev(X)
    vals = B.bvals if values is None else values
    if vals.numel() != B.bvals.numel():
        raise ValueError("values must hold one entry per stored block value")
    xt = torch.float64 if vals.dtype == torch.float64 else torch.float32
    if X.dtype != xt or X.dim() != 2 or X.shape[0] != B.n or X.stride(1) != 1:
        raise ValueError(f"X must be {xt}, n x k, unit column stride")
    if B.bitmap:
        raise ValueError("bcsr_spmm takes the dense block form")
    k = X.shape[1]
    if Y is None:
        Y = torch.empty((B.m, k), dtype=xt, device=X.device)
    if Y.dtype != xt or Y.dim() != 2 or tuple(Y.shape) != (B.m, k) or Y.stride(1) != 1:
        raise ValueError(f"Y must be {xt}, m x k, unit column stride")
    check(_lib.load().bcsr_spmm(B.m, B.n, B.a, B.b, B.nblocks, _ptr(B.browptr), _ptr(B.bcol), _ptr(vals),
                                dtype_code(vals), k, _ptr(X), X.stride(0), _ptr(Y), Y.stride(0), dtype_code(Y),
                                slots, row_period, _stream()), "bcsr_spmm")
    return Y


# ---------------------------------------------------------------- probes

PROBE_KINDS = {"read": 0, "write": 1, "write_nt": 2, "copy": 3, "flush": 4, "gather_rows": 5,
               "gather_elems": 6}
GATHER_ROUNDS = 256  # rounds per wavefront of the gather probes


def probe(kind: str, buf: torch.Tensor, buf2: torch.Tensor | None = None, blocks: int = 0) -> None:
    """Launch one memory probe over buf (see spx_probe in include/spx.h)."""
    _dev(buf, buf2)
    check(_lib.load().spx_probe(PROBE_KINDS[kind], _ptr(buf), _ptr(buf2), buf.numel() * buf.element_size(),
                                blocks, _stream()), "spx_probe")


def probe_index_gather(idx: torch.Tensor, x: torch.Tensor | None, gather: bool = True,
                       blocks: int = 4096, sink: torch.Tensor | None = None) -> torch.Tensor:
    """Stream idx and (gather=True) read x[idx[p]] (spx_probe_index_gather);
    returns the per-workgroup sums, f64[blocks]."""
    _dev(idx, x)
    if idx.dtype != torch.int32 or (x is not None and x.dtype != torch.float64):
        raise TypeError("probe_index_gather: idx int32, x float64")
    _contig(idx)
    if sink is None:
        sink = torch.zeros(blocks, dtype=torch.float64, device=idx.device)
    n = x.numel() if x is not None else 0
    check(_lib.load().spx_probe_index_gather(_ptr(idx), idx.numel(), _ptr(x), n, int(gather), _ptr(sink),
                                             blocks, _stream()), "spx_probe_index_gather")
    return sink


def chase_cycle(n: int, device, seed: int = 0, stride: int = 32) -> torch.Tensor:
    """next int32[n]: one random cycle through the n / stride slots that are
    multiples of `stride` (one per 128-byte line at the default), built on
    the device; the other slots hold 0 and are never visited from a slot of
    the cycle."""
    if n % stride:
        raise ValueError("chase_cycle: n must be a multiple of stride")
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    perm = torch.randperm(n // stride, generator=g, device=device, dtype=torch.int64) * stride
    nxt = torch.zeros(n, dtype=torch.int32, device=device)
    nxt[perm] = torch.roll(perm, -1).to(torch.int32)
    return nxt


def probe_chase(nxt: torch.Tensor, start: torch.Tensor, hops: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """Follow nxt from start[l] for `hops` dependent loads per lane
    (spx_probe_chase); returns the 64 final indices."""
    _dev(nxt, start)
    if nxt.dtype != torch.int32 or start.dtype != torch.int32 or start.numel() < 64:
        raise TypeError("probe_chase: nxt int32[n], start int32[64]")
    _contig(nxt)
    _contig(start)
    if out is None:
        out = torch.empty(64, dtype=torch.int32, device=nxt.device)
    check(_lib.load().spx_probe_chase(_ptr(nxt), nxt.numel(), _ptr(start), hops, _ptr(out), _stream()),
          "spx_probe_chase")
    return out
