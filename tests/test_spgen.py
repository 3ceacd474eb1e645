"""Pins of the seeded input generators (closed forms, the paper's Table 1, laws)."""
import math

import numpy as np
import pytest

import spgen
from _golden import table


def _trunc(x: float, digits: int) -> str:
    f = 10 ** digits
    return f"{math.floor(x * f) / f:.{digits}f}"


def _sci_trunc(x: float) -> str:
    e = math.floor(math.log10(x))
    mant = math.floor(x / 10 ** e * 100) / 100
    return f"{mant:.2f}e-{-e:02d}"


@pytest.mark.parametrize("row", table("table1_stencils.txt"), ids=lambda r: r["name"])
def test_table1_stencil_counts(row):
    dims = [int(d) for d in row["grid"].split("x")]
    if row["kind"] == "5pt":
        coo = spgen.stencil5(*dims)
        closed = 5 * dims[0] * dims[1] - 2 * (dims[0] + dims[1])
    else:
        coo = spgen.stencil3d(*dims, 7)
        a, b, c = dims
        closed = 7 * a * b * c - 2 * (a * b + b * c + a * c)
    assert coo.m == int(row["rows"])
    assert coo.nnz == int(row["nonzeros"]) == closed
    lens = np.bincount(coo.r, minlength=coo.m)
    cols = np.bincount(coo.c, minlength=coo.n)
    assert lens.max() == int(row["max_nnz_r"]) and cols.max() == int(row["max_nnz_c"])
    assert _trunc(coo.nnz / coo.m, 2) == row["nnz_per_row"]
    assert _sci_trunc(coo.nnz / coo.m ** 2) == row["density"]


def test_stencil27_histogram_and_closed_form():
    for N in (3, 5, 16):
        coo = spgen.stencil3d(N, N, N, 27)
        assert coo.nnz == (3 * N - 2) ** 3
    coo = spgen.stencil3d(128, 128, 128, 27)
    assert coo.nnz == 55_742_968
    L, cnt = np.unique(np.bincount(coo.r), return_counts=True)
    assert dict(zip(L.tolist(), cnt.tolist())) == {8: 8, 12: 1512, 18: 95256, 27: 2000376}


def test_stencil7_closed_form():
    for (a, b, c) in [(2, 3, 4), (7, 7, 7), (10, 3, 1)]:
        coo = spgen.stencil3d(a, b, c, 7)
        assert coo.nnz == 7 * a * b * c - 2 * (a * b + b * c + a * c)


def test_stencil_columns_valid_and_symmetric():
    coo = spgen.stencil3d(6, 5, 4, 27)
    A = np.zeros((coo.m, coo.n), dtype=np.int8)
    A[coo.r, coo.c] = 1
    assert (A == A.T).all() and A.sum() == coo.nnz


def test_uniform_rows_distinct_exact_count():
    coo = spgen.workload_c0()
    assert coo.m == coo.n == 10_000 and coo.nnz == 100_000
    pairs = coo.r.astype(np.int64) * coo.n + coo.c
    assert np.unique(pairs).size == coo.nnz
    assert (np.bincount(coo.r) == 10).all()
    assert coo.c.min() >= 0 and coo.c.max() < coo.n
    assert coo.v.min() >= -1.0 and coo.v.max() < 1.0


def test_zipf_mean_within_one_percent():
    q = spgen.zm_shift(2.0, 20_000, 16.0)
    assert abs(spgen.zm_mean(2.0, q, 20_000) - 16.0) < 1e-9
    lens = spgen.zm_lengths(1_000_000, 2.0, q, 20_000, seed=0, tag=spgen.TAG_ROWLEN)
    assert abs(lens.mean() - 16.0) / 16.0 < 0.01
    assert lens.min() >= 1 and lens.max() <= 20_000
    # pure Zipf(2) truncated at 20,000 has a mean far below 16: the shift is needed
    assert spgen.zm_mean(2.0, 0.0, 20_000) < 7.0


def test_powerlaw_rows_distinct_and_as_drawn():
    coo = spgen.powerlaw(20_000, 20_000, 2.0, 2_000, 16.0, seed=3)
    q = coo.info["q"]
    lens = spgen.zm_lengths(20_000, 2.0, q, 2_000, seed=3, tag=spgen.TAG_ROWLEN)
    assert (np.bincount(coo.r, minlength=coo.m) == lens).all()
    pairs = coo.r.astype(np.int64) * coo.n + coo.c
    assert np.unique(pairs).size == coo.nnz


def test_powerlaw_dense_rows_small_n():
    # rows longer than n/4 use weighted keys; a row may take every column
    coo = spgen.powerlaw(300, 40, 2.2, 20_000, 12.0, seed=1)
    lens = np.bincount(coo.r, minlength=coo.m)
    assert lens.max() <= 40
    pairs = coo.r.astype(np.int64) * coo.n + coo.c
    assert np.unique(pairs).size == coo.nnz


def test_determinism():
    a = spgen.powerlaw(5_000, 5_000, 2.0, 1_000, 16.0, seed=7)
    b = spgen.powerlaw(5_000, 5_000, 2.0, 1_000, 16.0, seed=7)
    c = spgen.powerlaw(5_000, 5_000, 2.0, 1_000, 16.0, seed=8)
    assert (a.r == b.r).all() and (a.c == b.c).all() and (a.v.view(np.uint64) == b.v.view(np.uint64)).all()
    assert a.nnz != c.nnz or (a.c != c.c).any()
    x1, x2 = spgen.uniform(1000, 0), spgen.uniform(1000, 0)
    assert (x1 == x2).all() and x1.min() >= -1 and x1.max() < 1


def test_normal_moments():
    z = spgen.normal(200_000, seed=0)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01


def test_bf16_rounding_rne():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 0.0, 1.0 + 2 ** -7], dtype=np.float64)
    bits = spgen.to_bf16_bits(vals)
    back = spgen.bf16_bits_to_f64(bits)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa (1.0) wins
    assert back.tolist() == [1.0, 1.0, 1.0 + 2 ** -6, -2.5, 0.0, 1.0 + 2 ** -7]


def test_batch_specs_recipe():
    specs = spgen.batch_specs(256, seed=0)
    kinds = [s.kind for s in specs]
    assert kinds.count("stencil5") == 64 and kinds.count("stencil7") == 64
    assert kinds.count("powerlaw") == 128
    assert all(s.k in (1, 4, 16) for s in specs)
    rows = np.array([s.rows for s in specs])
    assert rows.min() >= 900 and rows.max() <= 210_000


def test_partial_relabel_and_column_law():
    st = spgen.stencil5(40, 30, 1)
    half = spgen.relabeled(st, 3, fraction=0.5)
    full = spgen.relabeled(st, 3)
    # a relabelling is a bijection of the vertices: the set of (r, c) pairs
    # maps one to one, so the pair count is unchanged and no pair repeats
    for h in (half, full):
        assert np.unique(h.r.astype(np.int64) * h.n + h.c).size == st.nnz
    # half of the vertices are candidates to move; the rest keep their labels
    fixed = np.flatnonzero(half.r == st.r)  # entries whose row label did not change
    assert 0.4 < np.unique(st.r[fixed]).size / st.m < 0.7
    assert np.array_equal(spgen.relabeled(st, 3, 0.5).r, half.r)  # seeded
    # the column law changes the column degrees, not the row lengths
    a = spgen.powerlaw(20_000, 20_000, 2.0, 2_000, 16.0, seed=4)
    b = spgen.powerlaw(20_000, 20_000, 2.0, 2_000, 16.0, seed=4, col_alpha=1.6)
    la = np.bincount(a.r, minlength=a.m)
    lb = np.bincount(b.r, minlength=b.m)
    assert np.array_equal(la, lb)
    da = np.sort(np.bincount(a.c, minlength=a.n))[::-1]
    db = np.sort(np.bincount(b.c, minlength=b.n))[::-1]
    top = a.n // 100
    assert db[:top].sum() > da[:top].sum()  # a heavier column tail concentrates more accesses
