"""Seeded test matrices built from the generators and assembled by the oracle,
plus helpers that move them to the GPU for the parity tests."""
from __future__ import annotations

import numpy as np

import oracle
import spgen


def matrix(kind: str, seed: int = 0):
    """Small/medium matrices that cover every bin, ragged tails and empty rows."""
    if kind == "uniform":
        coo = spgen.uniform_rows(3000, 2500, 10, seed)
    elif kind == "powerlaw":
        coo = spgen.powerlaw(20_000, 18_000, 2.0, 6_000, 16.0, seed)
    elif kind == "powerlaw_sq":
        coo = spgen.powerlaw(30_000, 30_000, 2.0, 12_000, 16.0, seed)
    elif kind == "stencil27":
        coo = spgen.stencil3d(17, 13, 11, 27, seed)
    elif kind == "stencil5":
        coo = spgen.stencil5(77, 61, seed)
    elif kind == "empty_rows":
        base = spgen.powerlaw(5000, 4000, 2.0, 2_000, 12.0, seed)
        keep = (base.r % 3) != 1
        coo = spgen.COO(base.m, base.n, base.r[keep], base.c[keep], base.v[keep])
    elif kind == "one_long_row":
        # one dense row of 50,000 entries plus a diagonal: exercises split rows
        n = 60_000
        r = np.concatenate([np.zeros(50_000, np.int32), np.arange(1, 1000, dtype=np.int32)])
        c = np.concatenate([np.arange(50_000, dtype=np.int32), np.arange(1, 1000, dtype=np.int32)])
        coo = spgen.COO(1000, n, r, c, spgen.uniform(r.size, seed, spgen.TAG_VALUES))
    elif kind == "tall":
        coo = spgen.powerlaw(9_000, 700, 2.0, 700, 9.0, seed)
    elif kind == "wide":
        coo = spgen.powerlaw(700, 9_000, 2.0, 3_000, 40.0, seed)
    else:
        raise KeyError(kind)
    return oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)


KINDS = ["uniform", "powerlaw", "stencil27", "stencil5", "empty_rows", "one_long_row", "tall", "wide"]


def int_valued(A: oracle.CSR, seed: int = 0) -> oracle.CSR:
    """Same pattern with small-integer values: every partial sum is exact."""
    v = spgen.small_ints(A.nnz, seed, spgen.TAG_VALUES)
    return oracle.CSR(A.m, A.n, A.rowptr, A.colind, v)


def to_gpu(A: oracle.CSR, vdtype=None):
    import torch
    import paper_1302_1078_amd as spx
    dev = torch.device("cuda", 0)
    vals = torch.from_numpy(np.ascontiguousarray(A.values))
    if vdtype is not None:
        vals = vals.to(vdtype)
    return spx.CSR(torch.from_numpy(A.rowptr).to(dev), torch.from_numpy(A.colind).to(dev),
                   vals.to(dev), (A.m, A.n))


def single_bin_opts(lanes: int, k: int = 1, chunk: int = 512, kahan: int = 256):
    """Plan options with every row in one bin served by `lanes` threads (0 = split)."""
    import paper_1302_1078_amd as spx
    o = spx.PlanOpts()
    o.nbins = 1
    o.lanes[0] = lanes
    o.split_chunk = chunk
    o.kahan_len = kahan
    o.max_k = k
    return o


def keep_stream(o):
    """Serve stream bins as 256-row tiles even on matrices too small to fill
    the device (test matrices are)."""
    from paper_1302_1078_amd._lib import SPX_FLAG_KEEP_STREAM
    o.flags |= SPX_FLAG_KEEP_STREAM
    return o


def two_bin_opts(split_above: int, lanes: int, k: int = 1, chunk: int = 512, kahan: int = 256):
    import paper_1302_1078_amd as spx
    o = spx.PlanOpts()
    o.nbins = 2
    o.upper[0] = split_above
    o.lanes[0] = lanes
    o.lanes[1] = 0
    o.split_chunk = chunk
    o.kahan_len = kahan
    o.max_k = k
    return o


def gamma(n, u):
    n = np.asarray(n, dtype=np.float64)
    return n * u / (1.0 - n * u)


def stream_mm_opts(k: int, upper: int = 32, chunk: int = 256, kahan: int = 256):
    """Rows up to `upper` in a stream bin (row groups of KL lanes when k > 1), a
    wavefront bin up to 256, split rows above."""
    import paper_1302_1078_amd as spx
    return spx.PlanOpts.from_dict({"nbins": 3, "upper": [upper, 256], "lanes": [512, 64, 0],
                                   "split_chunk": chunk, "kahan_len": kahan, "max_k": k})


U32 = 2.0 ** -24


def quantised(A, vdtype, torch):
    """(GPU CSR with stored values, FP64 widening of the stored values)."""
    def dev(torch, a):
        return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    if vdtype == "f32":
        q = spgen.to_f32(A.values)
        vals = dev(torch, q)
        wide = q.astype(np.float64)
    else:
        bits = spgen.to_bf16_bits(A.values)
        vals = dev(torch, bits.view(np.int16)).view(torch.bfloat16)
        wide = spgen.bf16_bits_to_f64(bits)
    import paper_1302_1078_amd as spx
    G = spx.CSR(dev(torch, A.rowptr), dev(torch, A.colind), vals, (A.m, A.n))
    return G, oracle.CSR(A.m, A.n, A.rowptr, A.colind, wide)


def check_bound(y, y5, S, L, kahan_len, what):
    err = np.abs(y.astype(np.float64) - y5)
    comp = L > kahan_len
    plain_bound = gamma(L + 8, U32) * S
    comp_bound = U32 * np.abs(y5) + gamma(L, U32) ** 2 * S + 2.0 ** -45 * S
    assert (err[~comp] <= plain_bound[~comp]).all(), (what, "plain rows")
    assert (err[comp] <= comp_bound[comp]).all(), (what, "compensated rows")


def c3_submatrix(rows: int = 2000, longest: int = 10, seed: int = 0) -> oracle.CSR:
    """The gradient-check submatrix of the differentiation workload (the
    524,288 x 524,288 power-law matrix, Zipf(2.0) rows of mean 20): its
    `longest` longest rows plus rows - longest rows drawn with a seeded
    generator, in ascending row order, and the columns compacted to the ones
    those rows touch (values as generated, FP64)."""
    coo = spgen.workload_c3(0)
    B = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    del coo
    L = B.row_lengths()
    top = np.argsort(-L, kind="stable")[:longest]
    rest = np.setdiff1d(np.arange(B.m), top)
    pick = np.sort(np.concatenate([top, np.random.default_rng(seed).choice(rest, rows - longest,
                                                                            replace=False)]))
    row_of = B.row_of()
    keep = np.isin(row_of, pick)
    r = np.searchsorted(pick, row_of[keep]).astype(np.int32)
    cols, c = np.unique(B.colind[keep], return_inverse=True)
    return oracle.csr_from_coo(pick.size, cols.size, r, c.astype(np.int32), B.values[keep])
