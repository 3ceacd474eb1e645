"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

Only input drawing lives here: COO triplets, dense vectors, and the rounding
of FP64 draws to the stored FP32/BF16 formats.  Nothing in this module
assembles CSR or computes a product; the oracle (``oracle/``) and the GPU
library (``paper_1302_1078_amd``) each do that independently from what this
module returns.

The matrices stand in for the paper's workloads (Table 1 of the paper: 22
matrices from the UFL collection, which are not available here):

* ``uniform``: fixed nonzeros per row at uniformly random distinct columns.
* ``powerlaw``: Zipf-Mandelbrot row lengths with hot columns drawn from the
  same law (shaped like webbase-1M, scircuit, torso1 in Table 1).
* ``stencil5`` / ``stencil7`` / ``stencil27``: 2D and 3D grid stencils
  (mesh_2048 in Table 1 is the 2D 5-point stencil on 2048 x 2048; atmosmodd's
  counts match a 3D 7-point stencil on 148 x 148 x 58).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spgen.c")
_LIB = os.path.join(_HERE, "libspgen.so")

# stream tags (arbitrary fixed constants)
TAG_ROWLEN = 0x524F574C454E0001
TAG_COLW = 0x434F4C5700000002
TAG_COLS = 0x434F4C5300000003
TAG_VALUES = 0x56414C5500000004
TAG_X = 0x5800000000000005
TAG_DY = 0x4459000000000006
TAG_BATCH = 0x4241544348000007
TAG_PERM = 0x5045524D00000008


def build(force: bool = True) -> str:
    """Compile libspgen.so with gcc (OpenMP; generation is thread-count independent)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-D_GNU_SOURCE", "-o", tmp, _SRC, "-lm"])
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
        i32, i64, u64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        L.spgen_key.restype = u64
        L.spgen_key.argtypes = [u64, u64]
        L.spgen_uniform.argtypes = [u64, i64, f64, f64, P]
        L.spgen_normal.argtypes = [u64, i64, P]
        L.spgen_small_ints.argtypes = [u64, i64, i32, i32, P]
        L.spgen_zm_mean.restype = f64
        L.spgen_zm_mean.argtypes = [f64, f64, i32]
        L.spgen_zm_shift.restype = f64
        L.spgen_zm_shift.argtypes = [f64, i32, f64]
        L.spgen_zm_lengths.argtypes = [u64, i64, f64, f64, i32, P]
        L.spgen_uniform_rows.restype = ctypes.c_int
        L.spgen_uniform_rows.argtypes = [u64, i32, i32, i32, P, P]
        L.spgen_weighted_rows.restype = i64
        L.spgen_weighted_rows.argtypes = [u64, i32, i32, P, P, P, P, P, P]
        L.spgen_stencil5.restype = i64
        L.spgen_stencil5.argtypes = [i32, i32, P, P]
        L.spgen_stencil3d.restype = i64
        L.spgen_stencil3d.argtypes = [i32, i32, i32, i32, P, P]
        L.spgen_values_by_row.argtypes = [u64, i64, P, P, i32, f64, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def key(seed: int, tag: int) -> int:
    return int(lib().spgen_key(ctypes.c_uint64(seed & (2**64 - 1)), ctypes.c_uint64(tag)))


# ---------------------------------------------------------------- vectors

def uniform(n: int, seed: int, tag: int = TAG_X, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    lib().spgen_uniform(key(seed, tag), n, lo, hi, _p(out))
    return out


def normal(n: int, seed: int, tag: int = TAG_DY) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    lib().spgen_normal(key(seed, tag), n, _p(out))
    return out


def small_ints(n: int, seed: int, tag: int = TAG_X, lo: int = -8, hi: int = 8) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    lib().spgen_small_ints(key(seed, tag), n, lo, hi, _p(out))
    return out


# ---------------------------------------------------------------- rounding of stored formats

def to_f32(a: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even FP64 -> FP32 (IEEE conversion)."""
    return np.asarray(a, dtype=np.float64).astype(np.float32)


def to_bf16_bits(a: np.ndarray) -> np.ndarray:
    """FP64 -> FP32 (RNE) -> BF16 (RNE on the FP32 bit pattern); returns uint16 bits.
    NaN keeps a quiet-NaN payload."""
    f = to_f32(a).view(np.uint32).astype(np.uint64)
    lsb = (f >> 16) & 1
    rounded = ((f + 0x7FFF + lsb) >> 16).astype(np.uint16)
    nan = np.isnan(to_f32(a))
    if nan.any():
        rounded = rounded.copy()
        rounded[nan] = ((f[nan] >> 16) | 0x40).astype(np.uint16)
    return rounded


def bf16_bits_to_f64(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------- Zipf-Mandelbrot law

def zm_mean(alpha: float, q: float, lmax: int) -> float:
    return float(lib().spgen_zm_mean(alpha, q, lmax))


def zm_shift(alpha: float, lmax: int, mean: float) -> float:
    q = float(lib().spgen_zm_shift(alpha, lmax, mean))
    if math.isnan(q):
        raise ValueError(f"mean {mean} unreachable for alpha={alpha}, lmax={lmax}")
    return q


def zm_lengths(count: int, alpha: float, q: float, lmax: int, seed: int, tag: int) -> np.ndarray:
    out = np.empty(count, dtype=np.int32)
    lib().spgen_zm_lengths(key(seed, tag), count, alpha, q, lmax, _p(out))
    return out


# ---------------------------------------------------------------- COO structures

@dataclass
class COO:
    """Triplets in emission order: rows grouped and ascending, columns in draw order."""
    m: int
    n: int
    r: np.ndarray  # int32
    c: np.ndarray  # int32
    v: np.ndarray  # float64
    info: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.r.shape[0])


def _values(r, c, seed, kind, diag):
    v = np.empty(r.shape[0], dtype=np.float64)
    kinds = {"uniform": 0, "ints": 1, "laplacian": 2}
    lib().spgen_values_by_row(key(seed, TAG_VALUES), r.shape[0], _p(r), _p(c), kinds[kind],
                              float(diag), _p(v))
    return v


def uniform_rows(m: int, n: int, per_row: int, seed: int = 0, values: str = "uniform") -> COO:
    if per_row > n:
        raise ValueError("per_row > n")
    r = np.empty(m * per_row, dtype=np.int32)
    c = np.empty(m * per_row, dtype=np.int32)
    lib().spgen_uniform_rows(key(seed, TAG_COLS), m, n, per_row, _p(r), _p(c))
    return COO(m, n, r, c, _values(r, c, seed, values, 0.0), {"kind": "uniform", "per_row": per_row})


def powerlaw(m: int, n: int, alpha: float, lmax: int, mean: float, seed: int = 0,
             values: str = "uniform", col_alpha: float | None = None) -> COO:
    """Zipf-Mandelbrot row lengths (mean `mean`, max `lmax`) with hot columns of
    the same law, or of exponent `col_alpha` (same mean and maximum) when given:
    that changes how skewed the column use is and leaves the row lengths as
    they are."""
    lmax = int(min(lmax, n))
    q = zm_shift(alpha, lmax, mean)
    lens = zm_lengths(m, alpha, q, lmax, seed, TAG_ROWLEN)
    if col_alpha is None or col_alpha == alpha:
        w = zm_lengths(n, alpha, q, lmax, seed, TAG_COLW)
    else:
        w = zm_lengths(n, col_alpha, zm_shift(col_alpha, lmax, mean), lmax, seed, TAG_COLW)
    off = np.zeros(m, dtype=np.int64)
    if m > 1:
        np.cumsum(lens[:-1], out=off[1:])
    wcum = np.cumsum(w.astype(np.int64))
    nnz = int(lens.astype(np.int64).sum())
    r = np.empty(nnz, dtype=np.int32)
    c = np.empty(nnz, dtype=np.int32)
    draws = lib().spgen_weighted_rows(key(seed, TAG_COLS), m, n, _p(lens), _p(off), _p(wcum),
                                      _p(w), _p(r), _p(c))
    return COO(m, n, r, c, _values(r, c, seed, values, 0.0),
               {"kind": "powerlaw", "alpha": alpha, "lmax": lmax, "mean": mean, "q": q,
                "col_alpha": alpha if col_alpha is None else col_alpha, "draws": int(draws)})


def stencil5(nx: int, ny: int, seed: int = 0, values: str = "uniform") -> COO:
    m = nx * ny
    cap = 5 * m
    r = np.empty(cap, dtype=np.int32)
    c = np.empty(cap, dtype=np.int32)
    t = int(lib().spgen_stencil5(nx, ny, _p(r), _p(c)))
    r, c = r[:t].copy(), c[:t].copy()
    return COO(m, m, r, c, _values(r, c, seed, values, 4.0), {"kind": "stencil5", "grid": (nx, ny)})


def stencil3d(nx: int, ny: int, nz: int, pts: int, seed: int = 0, values: str = "uniform") -> COO:
    m = nx * ny * nz
    cap = pts * m
    r = np.empty(cap, dtype=np.int32)
    c = np.empty(cap, dtype=np.int32)
    t = int(lib().spgen_stencil3d(nx, ny, nz, pts, _p(r), _p(c)))
    if t < 0:
        raise ValueError("pts must be 7 or 27")
    r, c = r[:t].copy(), c[:t].copy()
    return COO(m, m, r, c, _values(r, c, seed, values, float(pts - 1)),
               {"kind": f"stencil{pts}", "grid": (nx, ny, nz)})


def shuffled(coo: COO, seed: int) -> COO:
    """Same triplets in a seeded random order (exercises COO -> CSR assembly)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = rng.permutation(coo.nnz)
    return COO(coo.m, coo.n, coo.r[p].copy(), coo.c[p].copy(), coo.v[p].copy(), dict(coo.info))


# ---------------------------------------------------------------- named workloads

def relabeled(coo: COO, seed: int, fraction: float = 1.0) -> COO:
    """Rows and columns renumbered by one seeded random permutation (P A P^T,
    square matrices): a banded matrix loses its band.  Old vertex i becomes
    label[i].  With fraction < 1 only a seeded random subset of
    round(fraction * m) vertices is shuffled among its own labels; the others
    keep theirs."""
    if coo.m != coo.n:
        raise ValueError("relabeling needs a square matrix")
    rng = np.random.Generator(np.random.PCG64(seed))
    if fraction >= 1.0:
        label = rng.permutation(coo.m).astype(np.int32)
    else:
        label = np.arange(coo.m, dtype=np.int32)
        moved = np.sort(rng.choice(coo.m, int(round(fraction * coo.m)), replace=False))
        label[moved] = moved[rng.permutation(moved.size)]
    return COO(coo.m, coo.n, label[coo.r], label[coo.c], coo.v.copy(),
               dict(coo.info, relabeled=seed, relabeled_fraction=fraction))


def workload_c0(seed: int = 0) -> COO:
    """10,000 x 10,000, 10 distinct uniform columns per row, values U[-1,1)."""
    return uniform_rows(10_000, 10_000, 10, seed)


def workload_c1(seed: int = 0, m: int = 1 << 20) -> COO:
    """1,048,576 square, Zipf(2.0) rows with mean 16 and max 20,000, hot columns."""
    return powerlaw(m, m, 2.0, 20_000, 16.0, seed)


def workload_c2_stencil(seed: int = 0, N: int = 128) -> COO:
    """3D 27-point stencil on N^3 (128^3: 2,097,152 rows, 55,742,968 nonzeros)."""
    return stencil3d(N, N, N, 27, seed)


def workload_c3(seed: int = 0, m: int = 1 << 19) -> COO:
    """524,288 square, Zipf(2.0) rows with mean 20 (max 20,000), hot columns."""
    return powerlaw(m, m, 2.0, 20_000, 20.0, seed)


@dataclass
class BatchSpec:
    kind: str
    rows: int
    k: int
    mean: float = 0.0
    grid: tuple = ()


def batch_specs(count: int = 256, seed: int = 0, rmin: int = 1_000, rmax: int = 200_000,
                ks=(1, 4, 16)) -> list:
    """Recipe of the batched workload: row counts log-uniform in [rmin, rmax];
    a quarter 2D 5-point, a quarter 3D 7-point, half Zipf(2.2) power law with
    mean U[8, 32]; SpMM width drawn uniformly from `ks`."""
    u = uniform(4 * count, seed, TAG_BATCH, 0.0, 1.0)
    kinds = ["stencil5"] * (count // 4) + ["stencil7"] * (count // 4)
    kinds += ["powerlaw"] * (count - len(kinds))
    # seeded Fisher-Yates with the batch stream
    order = list(range(count))
    for i in range(count - 1, 0, -1):
        j = int(u[3 * count + i] * (i + 1))
        order[i], order[j] = order[j], order[i]
    specs = []
    for b in range(count):
        rows = int(round(math.exp(math.log(rmin) + u[b] * (math.log(rmax) - math.log(rmin)))))
        kind = kinds[order[b]]
        k = ks[min(int(u[count + b] * len(ks)), len(ks) - 1)]
        if kind == "stencil5":
            s = max(2, int(round(math.sqrt(rows))))
            specs.append(BatchSpec(kind, s * s, k, grid=(s, s)))
        elif kind == "stencil7":
            s = max(2, int(round(rows ** (1.0 / 3.0))))
            specs.append(BatchSpec(kind, s * s * s, k, grid=(s, s, s)))
        else:
            mean = 8.0 + 24.0 * u[2 * count + b]
            specs.append(BatchSpec(kind, rows, k, mean=mean))
    return specs


def batch_matrix(spec: BatchSpec, seed: int, index: int) -> COO:
    s = (seed * 1_000_003 + index * 7919 + 1) & (2**63 - 1)
    if spec.kind == "stencil5":
        return stencil5(spec.grid[0], spec.grid[1], s)
    if spec.kind == "stencil7":
        return stencil3d(spec.grid[0], spec.grid[1], spec.grid[2], 7, s)
    return powerlaw(spec.rows, spec.rows, 2.2, 20_000, spec.mean, s)
