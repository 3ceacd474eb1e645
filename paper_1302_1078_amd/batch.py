"""Batched products: many (A_b, X_b) -> Y_b in one launch per lane layout.

csr_batch_create bins every matrix with its own plan options (from
``autotune`` or the defaults) and builds a tile list grouped by layout and
ordered by cost (heaviest first); each ``run()`` launches one workgroup per
tile of each layout on the current stream, so it can be captured into a HIP
graph (``capture()``) and replayed.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import CsrDesc, PlanOpts, check
from .ops import CSR, _ptr, _stream, default_opts, dtype_code


class Batched:
    def __init__(self, mats: list, Xs: list, Ys: list | None = None, opts: list | None = None):
        L = _lib.load()
        if len(mats) != len(Xs) or not mats:
            raise ValueError("need one X per matrix and at least one matrix")
        self.mats, self.Xs = list(mats), list(Xs)
        self.Ys = []
        descs = (CsrDesc * len(mats))()
        for i, (A, X) in enumerate(zip(mats, Xs)):
            vec = X.dim() == 1
            k = 1 if vec else X.shape[1]
            if X.shape[0] < A.n or (not vec and X.stride(1) != 1):
                raise ValueError(f"matrix {i}: X must have n rows and unit column stride")
            if Ys is not None:
                Y = Ys[i]
            else:
                Y = torch.empty((A.m,) if vec else (A.m, k), dtype=X.dtype, device=X.device)
            self.Ys.append(Y)
            o = opts[i] if opts is not None else default_opts(k, A.values.dtype)
            d = descs[i]
            d.m, d.n, d.nnz, d.k = A.m, A.n, A.nnz, k
            d.rowptr, d.colind, d.values = A.rowptr.data_ptr(), A.colind.data_ptr(), A.values.data_ptr()
            d.X, d.Y = X.data_ptr(), Y.data_ptr()
            d.ldx = 1 if vec else X.stride(0)
            d.ldy = 1 if vec else Y.stride(0)
            d.vtype, d.xytype = dtype_code(A.values), dtype_code(X)
            d.opts = o
        self._descs = descs
        nb = ctypes.c_size_t()
        check(L.csr_batch_workspace_bytes(len(mats), descs, ctypes.byref(nb)), "csr_batch_workspace_bytes")
        self.workspace = torch.empty(max(nb.value, 1), dtype=torch.uint8, device=mats[0].device)
        h = ctypes.c_void_p()
        check(L.csr_batch_create(len(mats), descs, _ptr(self.workspace), nb.value, _stream(), ctypes.byref(h)),
              "csr_batch_create")
        self.handle = h
        self.graph = None

    def run(self):
        check(_lib.load().csr_batch_run(self.handle, _stream()), "csr_batch_run")
        return self.Ys

    def capture(self) -> torch.cuda.CUDAGraph:
        """Capture one run() into a HIP graph; replay with self.graph.replay()."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run()  # warm-up outside the graph
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g
        return g

    def info(self) -> dict:
        a, b, c = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
        check(_lib.load().csr_batch_info(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
              "csr_batch_info")
        return {"tiles": a.value, "grid": b.value, "segments": c.value}

    def __del__(self):
        # at interpreter exit the module globals may already be gone
        h = getattr(self, "handle", None)
        lib = getattr(_lib, "_lib", None) if _lib is not None else None
        if h is not None and h.value and lib is not None:
            lib.csr_batch_destroy(h)
            self.handle = None
