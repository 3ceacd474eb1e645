"""ctypes view of libspx.so (the C ABI declared in include/spx.h).

Loading fails loudly when the library has not been built: there is no CPU or
PyTorch fallback for any operation of this package.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# SPX_LIB may point at another build of the same library (for comparisons)
LIB_PATH = os.environ.get("SPX_LIB") or os.path.join(_PKG, "libspx.so")

SPX_OK, SPX_ERR_INVALID, SPX_ERR_UNSUPPORTED, SPX_ERR_WORKSPACE, SPX_ERR_HIP = range(5)
SPX_F64, SPX_F32, SPX_BF16 = 0, 1, 2
SPX_MAX_BINS = 12
SPX_NOALLOC_SCRATCH_BYTES = 50331648
SPX_FLAG_NO_NT_STORE = 1
SPX_FLAG_SCALAR_X = 2
SPX_FLAG_NO_XCD_MAP = 4
SPX_FLAG_ONE_ROW = 8
SPX_FLAG_KEEP_STREAM = 16

STATUS_NAMES = {0: "SPX_OK", 1: "SPX_ERR_INVALID", 2: "SPX_ERR_UNSUPPORTED",
                3: "SPX_ERR_WORKSPACE", 4: "SPX_ERR_HIP"}


class PlanOpts(ctypes.Structure):
    _fields_ = [
        ("nbins", ctypes.c_int32),
        ("upper", ctypes.c_int32 * SPX_MAX_BINS),
        ("lanes", ctypes.c_int32 * SPX_MAX_BINS),
        ("split_chunk", ctypes.c_int32),
        ("kahan_len", ctypes.c_int32),
        ("max_k", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("occupancy", ctypes.c_int32),
        ("row_period", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 2),
    ]

    def to_dict(self) -> dict:
        nb = self.nbins
        return {"nbins": nb, "upper": list(self.upper[:nb - 1]), "lanes": list(self.lanes[:nb]),
                "split_chunk": self.split_chunk, "kahan_len": self.kahan_len,
                "max_k": self.max_k, "flags": self.flags, "occupancy": self.occupancy,
                "row_period": self.row_period}

    @classmethod
    def from_dict(cls, d: dict) -> "PlanOpts":
        o = cls()
        o.nbins = int(d["nbins"])
        for i, u in enumerate(d["upper"]):
            o.upper[i] = int(u)
        for i, l in enumerate(d["lanes"]):
            o.lanes[i] = int(l)
        o.split_chunk = int(d.get("split_chunk", 4096))
        o.kahan_len = int(d.get("kahan_len", 256))
        o.max_k = int(d.get("max_k", 1))
        o.flags = int(d.get("flags", 0))
        o.occupancy = int(d.get("occupancy", 0))
        o.row_period = int(d.get("row_period", 0))
        return o


class CsrDesc(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int32), ("n", ctypes.c_int32), ("nnz", ctypes.c_int32), ("k", ctypes.c_int32),
        ("rowptr", ctypes.c_void_p), ("colind", ctypes.c_void_p), ("values", ctypes.c_void_p),
        ("X", ctypes.c_void_p), ("Y", ctypes.c_void_p),
        ("ldx", ctypes.c_int64), ("ldy", ctypes.c_int64),
        ("vtype", ctypes.c_int), ("xytype", ctypes.c_int),
        ("opts", PlanOpts),
    ]


P = ctypes.c_void_p
i32, i64, u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
PP = ctypes.POINTER(ctypes.c_void_p)
SZ = ctypes.POINTER(ctypes.c_size_t)

# name -> (restype, argtypes); every function declared in include/spx.h
SIGNATURES = {
    "spx_last_error": (ctypes.c_char_p, []),
    "spx_version": (ctypes.c_char_p, []),
    "spx_plan_default_opts": (ctypes.c_int, [i32, ctypes.c_int, ctypes.POINTER(PlanOpts)]),
    "csr_from_coo_workspace_bytes": (ctypes.c_int, [i32, i32, i64, SZ]),
    "csr_from_coo": (ctypes.c_int, [i32, i32, i64, P, P, P, P, P, P, P, P, ctypes.c_size_t, P]),
    "csr_validate": (ctypes.c_int, [i32, i32, i32, P, P, i32, P, P]),
    "csr_from_coo_host": (ctypes.c_int, [i32, i32, i64, P, P, P, P, P, P, P]),
    "csr_validate_host": (ctypes.c_int, [i32, i32, i32, P, P]),
    "csr_plan_workspace_bytes": (ctypes.c_int, [i32, i32, ctypes.POINTER(PlanOpts), SZ]),
    "csr_plan_create": (ctypes.c_int, [i32, i32, i32, P, ctypes.POINTER(PlanOpts), P,
                                       ctypes.c_size_t, P, PP]),
    "csr_plan_export_bins": (ctypes.c_int, [P, P, P]),
    "csr_plan_info": (ctypes.c_int, [P, P, P, P]),
    "csr_plan_staged_workspace_bytes": (ctypes.c_int, [i32, i32, i32, i32, ctypes.c_int, SZ]),
    "csr_plan_create_staged": (ctypes.c_int, [i32, i32, i32, P, P, i32, ctypes.c_int, P, ctypes.c_size_t, P, PP]),
    "csr_plan_staged_info": (ctypes.c_int, [P, P, P, P, P]),
    "csr_plan_staged_pipeline": (ctypes.c_int, [P, i32]),
    "csr_plan_hot_x_workspace_bytes": (ctypes.c_int, [i32, i32, i32, SZ]),
    "csr_plan_attach_hot_x": (ctypes.c_int, [P, i32, i32, P, i32, ctypes.c_int, P, ctypes.c_size_t, P]),
    "csr_plan_destroy": (None, [P]),
    "csr_spmv": (ctypes.c_int, [i32, i32, i32, P, P, P, ctypes.c_int, P, P, ctypes.c_int, P, P]),
    "csr_spmm": (ctypes.c_int, [i32, i32, i32, P, P, P, ctypes.c_int, i32, P, i64, P, i64,
                                ctypes.c_int, P, P]),
    "csr_transpose_index_workspace_bytes": (ctypes.c_int, [i32, i32, i32, SZ]),
    "csr_transpose_index": (ctypes.c_int, [i32, i32, i32, P, P, P, P, P, P, ctypes.c_size_t, P]),
    "csr_csc_value_map_workspace_bytes": (ctypes.c_int, [i32, SZ]),
    "csr_csc_value_map": (ctypes.c_int, [i32, P, P, P, P, ctypes.c_size_t, P]),
    "csr_values_to_csc": (ctypes.c_int, [i32, P, P, P, ctypes.c_int, P, P, P]),
    "csr_values_to_csc_noalloc": (ctypes.c_int, [i32, P, P, P, ctypes.c_int, P, P]),
    "csr_spmv_t": (ctypes.c_int, [i32, i32, i32, P, P, P, P, P, P, ctypes.c_int, i32, P, i64, P, i64,
                                  ctypes.c_int, i32, P, P]),
    "csr_sddmm": (ctypes.c_int, [i32, i32, i32, P, P, i32, P, i64, P, i64, P, ctypes.c_int, P, P]),
    "csr_spmv_save": (ctypes.c_int, [i32, i32, i32, P, P, P, ctypes.c_int, P, P, ctypes.c_int, P, P, P]),
    "csr_sddmm_saved": (ctypes.c_int, [i32, i32, P, P, P, P, ctypes.c_int, P, P]),
    "csr_batch_workspace_bytes": (ctypes.c_int, [i32, ctypes.POINTER(CsrDesc), SZ]),
    "csr_batch_create": (ctypes.c_int, [i32, ctypes.POINTER(CsrDesc), P, ctypes.c_size_t, P, PP]),
    "csr_batch_run": (ctypes.c_int, [P, P]),
    "csr_batch_info": (ctypes.c_int, [P, P, P, P]),
    "csr_batch_destroy": (None, [P]),
    "csr_rcm": (ctypes.c_int, [i32, i32, i32, P, P, P]),
    "csr_degree_order_workspace_bytes": (ctypes.c_int, [i32, i32, SZ]),
    "csr_degree_order": (ctypes.c_int, [i32, i32, P, P, P, ctypes.c_size_t, P]),
    "csr_bandwidth": (ctypes.c_int, [i32, i32, P, P, P, P]),
    "csr_permute_workspace_bytes": (ctypes.c_int, [i32, i32, SZ]),
    "csr_permute": (ctypes.c_int, [i32, i32, P, P, P, P, P, P, P, P, P, ctypes.c_size_t, P]),
    "csr_vector_access": (ctypes.c_int, [i32, i32, i32, P, P, i32, i32, i32, ctypes.POINTER(ctypes.c_double)]),
    "csr_ucld": (ctypes.c_int, [i32, i32, P, P, i32, ctypes.POINTER(ctypes.c_double)]),
    "csr_tile_lines": (ctypes.c_int, [i32, i32, i32, P, P, i32, i32, ctypes.POINTER(ctypes.c_int64)]),
    "bcsr_workspace_bytes": (ctypes.c_int, [i32, i32, i32, SZ]),
    "csr_bcsr_count": (ctypes.c_int, [i32, i32, i32, P, P, i32, i32, P, P, ctypes.c_size_t, P]),
    "csr_to_bcsr": (ctypes.c_int, [i32, i32, i32, P, P, P, i32, i32, i32, P, P, P, P, P, P, ctypes.c_size_t, P]),
    "bcsr_spmv": (ctypes.c_int, [i32, i32, i32, i32, i32, i32, P, P, P, P, P, P, P, i32, P]),
    "bcsr_spmm": (ctypes.c_int, [i32, i32, i32, i32, i32, P, P, P, ctypes.c_int, i32, P, ctypes.c_int64, P,
                                 ctypes.c_int64, ctypes.c_int, i32, i32, P]),
    "spx_probe": (ctypes.c_int, [i32, P, P, ctypes.c_size_t, i32, P]),
    "spx_probe_index_gather": (ctypes.c_int, [P, i64, P, i32, i32, P, i32, P]),
    "spx_probe_chase": (ctypes.c_int, [P, i64, P, i64, P, P]),
}

_lib = None


class SpxError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = last_error()
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def load():
    """Load libspx.so; raise if it is missing (build with paper_1302_1078_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m "
                          "paper_1302_1078_amd.build` (hipcc, gfx950); there is no fallback")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name, None)
        if fn is None:
            continue  # reported by missing_symbols()
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def missing_symbols() -> list:
    L = load()
    return [name for name in SIGNATURES if getattr(L, name, None) is None]


def last_error() -> str:
    L = _lib
    if L is None:
        return ""
    s = L.spx_last_error()
    return s.decode() if s else ""


def check(status: int, where: str) -> None:
    if status != SPX_OK:
        raise SpxError(status, where)
