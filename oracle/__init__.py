"""FP64 CPU oracle for the CSR SpMV / SpMM path -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library and never calls
it.  The arithmetic lives in ``oracle.c`` (plain C, FP64, no FMA contraction);
this module marshals numpy arrays and holds the paper's counting formulas.

Functions and the passages they follow:

* ``csr_from_coo``   -- CRS arrays rptrs/cids/val (Sec. 3).
* ``bin_rows``       -- row binning by length, the GPU analogue of the paper's
  dynamic row chunks (Sec. 4.1).
* ``spmv``           -- y <- A x (Sec. 1, Sec. 3).
* ``spmm``           -- Y <- A X with a zeroed per-row temporary (Sec. 5).
* ``spmv_t``         -- A^T dY, the CCS dual (Sec. 3).
* ``sddmm``          -- sampled dot dY[row] . X[col] (gradient w.r.t. values).
* ``flops`` / ``app_bytes`` -- 2 tau k flops (Sec. 3) and the application
  byte count (Sec. 4.2 for SpMV, Sec. 5 for SpMM), generalised to element
  sizes and non-square shapes.
* ``spmv_abs``       -- sum_p |a_p x_{c_p}| per row, the scale of the
  floating-point error bounds of a row's dot product.
* ``rel2``           -- ||y_hat - y||_2 / ||y||_2 in FP64, the absolute norm of
  the difference when ||y|| = 0.
* ``ucld``           -- useful cacheline density (Sec. 4.1).
* ``tile_lines``     -- distinct x cachelines per tile of consecutive rows
  (Sec. 4.1 and 4.2's cacheline counting, per workgroup tile).
* ``degree_order``   -- columns by descending nonzero count, ties ascending
  (a locality ordering set beside the paper's RCM step, Sec. 4.4).

Parity: each function is pinned in ``tests/test_oracle.py`` against brute
force, invariants or closed forms (``sddmm`` by exact central differences of
``spmv``/``spmm``, ``rel2`` by hand-computed vectors, ``spmv_abs`` by a dense
brute force); none is "parity unpinned".
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.orc_csr_from_coo.restype = ctypes.c_int
        L.orc_csr_from_coo.argtypes = [i32, i32, i64, P, P, P, P, P, P, P]
        L.orc_bin_rows.argtypes = [i32, P, i32, P, P, P]
        L.orc_spmv.argtypes = [i32, P, P, P, P, P, ctypes.c_int]
        L.orc_spmm.argtypes = [i32, i32, P, P, P, P, i64, P, i64, ctypes.c_int]
        L.orc_spmv_t.argtypes = [i32, i32, i32, P, P, P, P, i64, P, i64]
        L.orc_sddmm.argtypes = [i32, i32, P, P, P, i64, P, i64, P]
        L.orc_spmv_abs.argtypes = [i32, P, P, P, P, P]
        L.orc_ucld.restype = f64
        L.orc_ucld.argtypes = [i32, P, P, i32, P]
        L.orc_vector_access.restype = f64
        L.orc_vector_access.argtypes = [i32, i32, P, P, i32, i32, i32]
        L.orc_tile_lines.restype = ctypes.c_int64
        L.orc_tile_lines.argtypes = [i32, i32, P, P, i32, i32]
        L.orc_rcm.restype = ctypes.c_int
        L.orc_rcm.argtypes = [i32, i32, P, P, P]
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


@dataclass
class CSR:
    m: int
    n: int
    rowptr: np.ndarray
    colind: np.ndarray
    values: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.rowptr)

    def row_of(self) -> np.ndarray:
        return np.repeat(np.arange(self.m, dtype=np.int32), self.row_lengths())


def csr_from_coo(m: int, n: int, r, c, v) -> CSR:
    r, c, v = _i32(r), _i32(c), _f64(v)
    nnz_in = r.shape[0]
    rowptr = np.zeros(m + 1, dtype=np.int32)
    colind = np.empty(max(nnz_in, 1), dtype=np.int32)
    values = np.empty(max(nnz_in, 1), dtype=np.float64)
    out = np.zeros(1, dtype=np.int64)
    rc = lib().orc_csr_from_coo(m, n, nnz_in, _p(r), _p(c), _p(v), _p(rowptr), _p(colind),
                                _p(values), _p(out))
    if rc != 0:
        raise ValueError("triplet index out of range")
    t = int(out[0])
    return CSR(m, n, rowptr, colind[:t].copy(), values[:t].copy())


def bin_rows(rowptr, upper) -> tuple:
    rowptr = _i32(rowptr)
    m = rowptr.shape[0] - 1
    upper = _i32(upper)
    nbins = upper.shape[0]
    perm = np.empty(max(m, 1), dtype=np.int32)
    off = np.empty(nbins + 1, dtype=np.int32)
    lib().orc_bin_rows(m, _p(rowptr), nbins, _p(upper), _p(perm), _p(off))
    return perm[:m].copy(), off


def spmv(A: CSR, x, nthreads: int = 0) -> np.ndarray:
    x = _f64(x)
    assert x.shape[0] >= A.n
    y = np.empty(A.m, dtype=np.float64)
    lib().orc_spmv(A.m, _p(A.rowptr), _p(_i32(A.colind)), _p(_f64(A.values)), _p(x), _p(y), nthreads)
    return y


def spmm(A: CSR, X, nthreads: int = 0) -> np.ndarray:
    X = _f64(X)
    assert X.ndim == 2 and X.shape[0] >= A.n
    k = X.shape[1]
    Y = np.empty((A.m, k), dtype=np.float64)
    lib().orc_spmm(A.m, k, _p(A.rowptr), _p(_i32(A.colind)), _p(_f64(A.values)), _p(X), k, _p(Y),
                   k, nthreads)
    return Y


def spmv_t(A: CSR, dY) -> np.ndarray:
    dY = _f64(dY)
    squeeze = dY.ndim == 1
    if squeeze:
        dY = dY[:, None]
    k = dY.shape[1]
    dX = np.empty((A.n, k), dtype=np.float64)
    lib().orc_spmv_t(A.m, A.n, k, _p(A.rowptr), _p(_i32(A.colind)), _p(_f64(A.values)), _p(dY), k,
                     _p(dX), k)
    return dX[:, 0] if squeeze else dX


def sddmm(A: CSR, dY, X) -> np.ndarray:
    dY, X = _f64(dY), _f64(X)
    if dY.ndim == 1:
        dY = dY[:, None]
        X = X[:, None]
    k = dY.shape[1]
    out = np.empty(max(A.nnz, 1), dtype=np.float64)
    lib().orc_sddmm(A.m, k, _p(A.rowptr), _p(_i32(A.colind)), _p(dY), k, _p(X), k, _p(out))
    return out[:A.nnz].copy()


def spmv_abs(A: CSR, x) -> np.ndarray:
    x = _f64(x)
    out = np.empty(A.m, dtype=np.float64)
    lib().orc_spmv_abs(A.m, _p(A.rowptr), _p(_i32(A.colind)), _p(_f64(A.values)), _p(x), _p(out))
    return out


def ucld(A: CSR, line: int = 8) -> float:
    used = np.zeros(1, dtype=np.int64)
    return float(lib().orc_ucld(A.m, _p(A.rowptr), _p(_i32(A.colind)), line, _p(used)))


def vector_access(A: CSR, line: int = 16, parts: int = 8, chunk: int = 64) -> float:
    """Expected number of times x is moved from memory (Sec. 4.2): rows dealt
    round-robin to `parts` infinite caches in chunks of `chunk` rows."""
    return float(lib().orc_vector_access(A.m, A.n, _p(A.rowptr), _p(_i32(A.colind)), line, parts, chunk))


def tile_lines(A: CSR, line: int = 16, tile: int = 256) -> int:
    """Distinct (tile, x line) pairs over tiles of `tile` consecutive rows
    (x line = column // line): the x lines a row tile gathers, summed over
    tiles (the per-tile form of Sec. 4.1's cacheline counting)."""
    return int(lib().orc_tile_lines(A.m, A.n, _p(A.rowptr), _p(_i32(A.colind)), line, tile))


def rcm(A: CSR) -> np.ndarray:
    """Reverse Cuthill-McKee order of the pattern of A + A^T (Sec. 4.4);
    perm[new] = old."""
    perm = np.empty(A.m, dtype=np.int32)
    if lib().orc_rcm(A.m, A.n, _p(A.rowptr), _p(_i32(A.colind)), _p(perm)) != 0:
        raise ValueError("rcm needs a square matrix")
    return perm


def degree_order(A: CSR) -> np.ndarray:
    """Columns listed by descending number of nonzeros, equal counts in
    ascending column index; perm[new] = old (n entries)."""
    count = [0] * A.n
    for c in np.asarray(A.colind).tolist():
        count[c] += 1
    return np.array(sorted(range(A.n), key=lambda j: (-count[j], j)), dtype=np.int32)


def permute(A: CSR, perm) -> CSR:
    """P A P^T for perm[new] = old (rows and columns renumbered), assembled
    canonically."""
    perm = np.asarray(perm, dtype=np.int64)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    rows = np.repeat(np.arange(A.m, dtype=np.int64), np.diff(A.rowptr))
    return csr_from_coo(A.m, A.n, inv[rows].astype(np.int32), inv[A.colind].astype(np.int32), A.values)


@dataclass
class BCSR:
    """Register-blocked CRS (Sec. 4.5): A cut into a x b blocks; every block
    holding a nonzero is kept.  Block rows ascend, block columns ascend inside
    a block row.  Dense form: `values` holds a*b entries per block, row-major
    inside the block, zeros explicit.  Bitmap form: `mask[q]` has bit
    (r*b + c) set for each nonzero at (r, c) of block q, and `values` holds
    only the nonzeros, block after block, in bit order (`offset[q]` = index
    of block q's first value)."""
    m: int
    n: int
    a: int
    b: int
    browptr: np.ndarray
    bcol: np.ndarray
    values: np.ndarray
    mask: np.ndarray = None
    offset: np.ndarray = None

    @property
    def nblocks(self) -> int:
        return int(self.browptr[-1])


def to_bcsr(A: CSR, a: int, b: int, bitmap: bool = False) -> BCSR:
    """Block the matrix, from the definition: block (I, J) holds the entries
    (I*a + r, J*b + c), 0 <= r < a, 0 <= c < b."""
    mb = -(-A.m // a)
    rows = A.row_of().astype(np.int64)
    cols = A.colind.astype(np.int64)
    key = (rows // a) * (-(-A.n // b) + 1) + cols // b
    pos = (rows % a) * b + cols % b
    order = np.lexsort((pos, key))  # blocks in (block row, block column) order, entries by position
    key, pos, vals = key[order], pos[order], A.values[order]
    uniq, first = np.unique(key, return_index=True)
    nb = uniq.size
    brow = uniq // (-(-A.n // b) + 1)
    bcol = (uniq % (-(-A.n // b) + 1)).astype(np.int32)
    browptr = np.searchsorted(brow, np.arange(mb + 1), side="left").astype(np.int32)
    blk = np.repeat(np.arange(nb), np.diff(np.append(first, key.size)))
    if not bitmap:
        dense = np.zeros(nb * a * b, dtype=np.float64)
        dense[blk * a * b + pos] = vals
        return BCSR(A.m, A.n, a, b, browptr, bcol, dense)
    mask = np.zeros(nb, dtype=np.uint64)
    np.bitwise_or.at(mask, blk, np.left_shift(np.uint64(1), pos.astype(np.uint64)))
    return BCSR(A.m, A.n, a, b, browptr, bcol, vals.copy(), mask, first.astype(np.int32))


def bcsr_dense(B: BCSR) -> np.ndarray:
    """The m x n matrix a BCSR holds (explicit zeros and padding dropped)."""
    mb = B.browptr.size - 1
    D = np.zeros((mb * B.a, (-(-B.n // B.b)) * B.b), dtype=np.float64)
    for I in range(mb):
        for q in range(B.browptr[I], B.browptr[I + 1]):
            J = int(B.bcol[q])
            if B.mask is None:
                blk = B.values[q * B.a * B.b:(q + 1) * B.a * B.b].reshape(B.a, B.b)
            else:
                blk = np.zeros(B.a * B.b)
                bits = [t for t in range(B.a * B.b) if (int(B.mask[q]) >> t) & 1]
                blk[bits] = B.values[B.offset[q]:B.offset[q] + len(bits)]
                blk = blk.reshape(B.a, B.b)
            D[I * B.a:(I + 1) * B.a, J * B.b:(J + 1) * B.b] = blk
    return D[:B.m, :B.n]


def bcsr_bytes(B: BCSR) -> int:
    """Bytes the blocked matrix occupies: values, one 4-byte column per block
    and the block-row pointers (+ the 8-byte mask and 4-byte offset per block
    in bitmap form).  A dense 8 x 8 block is 8*64 + 4 = 516 B (Sec. 4.5)."""
    nb = B.nblocks
    extra = 12 * nb if B.mask is not None else 0
    return 8 * int(B.values.size if B.mask is None else B.values.size) + 4 * nb + 4 * B.browptr.size + extra


def max_threads() -> int:
    return int(lib().orc_max_threads())


# ---------------------------------------------------------------- counting formulas

def flops(nnz: int, k: int = 1) -> int:
    """One multiply and one add per nonzero and right-hand side (Sec. 3)."""
    return 2 * nnz * k


def app_bytes(m: int, n: int, nnz: int, k: int = 1, s_val: int = 8, s_x: int = 8, s_y: int = 8,
              s_idx: int = 4) -> int:
    """Application bytes: every array moved exactly once (Sec. 4.2, Sec. 5).

    values + column ids per nonzero, x (n x k) read, y (m x k) written, and
    the m+1 row pointers.  For a square FP64 SpMV this is 4 + 20 n + 12 tau.
    """
    return (s_val + s_idx) * nnz + s_x * k * n + s_y * k * m + s_idx * (m + 1)


def rel2(y_hat, y_ref) -> float:
    """||y_hat - y_ref||_2 / ||y_ref||_2 in FP64 (0 if both vanish)."""
    y_hat = np.asarray(y_hat, dtype=np.float64).ravel()
    y_ref = np.asarray(y_ref, dtype=np.float64).ravel()
    den = float(np.linalg.norm(y_ref))
    num = float(np.linalg.norm(y_hat - y_ref))
    if den == 0.0:
        return num
    return num / den
