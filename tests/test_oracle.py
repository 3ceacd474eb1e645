"""Pins of the FP64 oracle against brute force, invariants and the paper's numbers.

Each test is chosen so that a plausible slip in the oracle (a dropped term, a
transposed operand, a wrong row/column index, summation in the wrong order,
a missing zero-initialisation) fails at least one of them.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import spgen
from _golden import kv


def rand_coo(rng, m, n, nnz, dup=True, ints=True):
    r = rng.integers(0, m, nnz).astype(np.int32) if m else np.zeros(0, np.int32)
    c = rng.integers(0, n, nnz).astype(np.int32) if n else np.zeros(0, np.int32)
    if not dup:
        key = np.unique(r.astype(np.int64) * max(n, 1) + c)
        r, c = (key // max(n, 1)).astype(np.int32), (key % max(n, 1)).astype(np.int32)
        p = rng.permutation(r.size)
        r, c = r[p], c[p]
    v = rng.integers(-8, 9, r.size).astype(np.float64) if ints else rng.uniform(-1, 1, r.size)
    return r, c, v


def dense_from_coo(m, n, r, c, v):
    D = np.zeros((m, n), dtype=np.float64)
    for a, b, x in zip(r, c, v):
        D[a, b] += x
    return D


def dense(A):
    D = np.zeros((A.m, A.n), dtype=np.float64)
    D[A.row_of(), A.colind] = A.values
    return D


SHAPES = [(1, 1), (5, 7), (7, 5), (16, 16), (33, 17), (64, 64), (3, 0), (0, 4)]


# ---------------------------------------------------------------- CSR assembly

@pytest.mark.parametrize("m,n", SHAPES)
def test_csr_from_coo_brute_force(m, n):
    rng = np.random.default_rng(m * 100 + n)
    nnz = 0 if m == 0 or n == 0 else 3 * (m + n)
    r, c, v = rand_coo(rng, m, n, nnz)
    A = oracle.csr_from_coo(m, n, r, c, v)
    # canonical structure (Sec. 3): rptrs[0]=0, rptrs[m]=tau, cids sorted per row
    assert A.rowptr[0] == 0 and A.rowptr[-1] == A.nnz == A.colind.size
    assert (np.diff(A.rowptr) >= 0).all()
    for i in range(m):
        cols = A.colind[A.rowptr[i]:A.rowptr[i + 1]]
        assert (np.diff(cols) > 0).all()
    # the stored set of (i, j) is exactly the set of input positions, and
    # values equal the dense accumulation (integers: exact in any order)
    D = dense_from_coo(m, n, r, c, v)
    assert (dense(A) == D).all()
    assert A.nnz == np.unique(r.astype(np.int64) * max(n, 1) + c).size


def test_csr_from_coo_scipy_third_opinion():
    rng = np.random.default_rng(11)
    r, c, v = rand_coo(rng, 50, 40, 600)
    A = oracle.csr_from_coo(50, 40, r, c, v)
    S = sp.coo_matrix((v, (r, c)), shape=(50, 40)).tocsr()
    S.sum_duplicates()
    S.sort_indices()
    assert (S.indptr == A.rowptr).all() and (S.indices == A.colind).all()
    assert (S.data == A.values).all()


def test_duplicates_summed_in_input_order():
    # (1e16 + 1) rounds to 1e16, so input order gives 0; any reordering that
    # adds the cancelling pair first gives 1.
    r = np.array([0, 0, 0], np.int32)
    c = np.array([2, 2, 2], np.int32)
    v = np.array([1e16, 1.0, -1e16])
    A = oracle.csr_from_coo(1, 3, r, c, v)
    assert A.nnz == 1 and A.values[0] == 0.0
    A2 = oracle.csr_from_coo(1, 3, r, c, v[[0, 2, 1]])
    assert A2.values[0] == 1.0


def test_round_trip_identity():
    coo = spgen.powerlaw(3_000, 2_500, 2.0, 400, 12.0, seed=5)
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    sh = spgen.shuffled(spgen.COO(A.m, A.n, A.row_of(), A.colind, A.values), seed=9)
    B = oracle.csr_from_coo(sh.m, sh.n, sh.r, sh.c, sh.v)
    assert (A.rowptr == B.rowptr).all() and (A.colind == B.colind).all()
    assert (A.values.view(np.uint64) == B.values.view(np.uint64)).all()


def test_out_of_range_rejected():
    with pytest.raises(ValueError):
        oracle.csr_from_coo(2, 2, np.array([0, 2]), np.array([0, 0]), np.array([1.0, 1.0]))
    with pytest.raises(ValueError):
        oracle.csr_from_coo(2, 2, np.array([0, 1]), np.array([0, -1]), np.array([1.0, 1.0]))


# ---------------------------------------------------------------- binning

@pytest.mark.parametrize("upper", [[4, 64, 1024], [0, 1, 2, 8, 32], [1_000_000]])
def test_bin_rows_partition(upper):
    coo = spgen.powerlaw(4_000, 4_000, 2.0, 2_000, 16.0, seed=2)
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    perm, off = oracle.bin_rows(A.rowptr, upper)
    L = A.row_lengths()
    assert off[0] == 0 and off[-1] == A.m and (np.diff(off) >= 0).all()
    assert np.array_equal(np.sort(perm), np.arange(A.m))
    # brute force: bin index = number of thresholds strictly below L, capped
    nb = len(upper)
    b = np.minimum(np.searchsorted(np.asarray(upper), L, side="left"), nb - 1)
    expect = np.argsort(b, kind="stable")
    assert np.array_equal(perm, expect)
    for k in range(nb):
        rows = perm[off[k]:off[k + 1]]
        assert (np.diff(rows) > 0).all()
        Lk = L[rows]
        if k < nb - 1:
            assert (Lk <= upper[k]).all()
        if k > 0:
            assert (Lk > upper[k - 1]).all()


# ---------------------------------------------------------------- SpMV

@pytest.mark.parametrize("m,n", SHAPES)
def test_spmv_dense_brute_force_exact(m, n):
    rng = np.random.default_rng(m * 7 + n)
    nnz = 0 if m == 0 or n == 0 else 4 * (m + n)
    r, c, v = rand_coo(rng, m, n, nnz)
    A = oracle.csr_from_coo(m, n, r, c, v)
    x = rng.integers(-8, 9, n).astype(np.float64)
    y = oracle.spmv(A, x)
    # integer inputs: every partial sum is exact, so any order agrees exactly
    Di = dense_from_coo(m, n, r, c, v).astype(np.int64)
    assert (y == (Di @ x.astype(np.int64)).astype(np.float64)).all()


def test_spmv_float_matches_dense_and_scipy():
    rng = np.random.default_rng(1)
    r, c, v = rand_coo(rng, 64, 48, 900, ints=False)
    A = oracle.csr_from_coo(64, 48, r, c, v)
    x = rng.uniform(-1, 1, 48)
    y = oracle.spmv(A, x)
    yd = dense(A) @ x
    ys = sp.csr_matrix((A.values, A.colind, A.rowptr), shape=(64, 48)) @ x
    assert oracle.rel2(y, yd) < 1e-14 and oracle.rel2(y, ys) < 1e-14
    # sequential ascending-p order, checked by an explicit loop
    for i in (0, 17, 63):
        s = 0.0
        for p in range(A.rowptr[i], A.rowptr[i + 1]):
            s = s + A.values[p] * x[A.colind[p]]
        assert y[i] == s


def test_spmv_identity_and_permutation():
    n = 1000
    x = spgen.uniform(n, 0)
    I = oracle.csr_from_coo(n, n, np.arange(n), np.arange(n), np.ones(n))
    assert (oracle.spmv(I, x) == x).all()
    perm = np.random.default_rng(4).permutation(n)
    P = oracle.csr_from_coo(n, n, np.arange(n), perm, np.ones(n))
    assert (oracle.spmv(P, x) == x[perm]).all()


def test_spmv_unit_vectors_give_columns():
    coo = spgen.powerlaw(300, 200, 2.0, 100, 8.0, seed=3)
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    D = dense(A)
    for j in (0, 5, 199):
        e = np.zeros(A.n)
        e[j] = 1.0
        assert (oracle.spmv(A, e) == D[:, j]).all()


def test_spmv_ones_gives_row_sums_and_empty_rows_positive_zero():
    coo = spgen.powerlaw(2000, 2000, 2.0, 300, 4.0, seed=8)
    # drop every third row to create empty rows
    keep = coo.r % 3 != 0
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r[keep], coo.c[keep], coo.v[keep])
    y = oracle.spmv(A, np.ones(A.n))
    for i in range(A.m):
        s = 0.0
        for p in range(A.rowptr[i], A.rowptr[i + 1]):
            s = s + A.values[p]
        assert y[i] == s
    empty = A.row_lengths() == 0
    assert empty.sum() > 0 and (y[empty] == 0).all() and not np.signbit(y[empty]).any()


def test_spmv_linearity():
    coo = spgen.workload_c0()
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    x, z = spgen.uniform(A.n, 1), spgen.uniform(A.n, 2)
    a, b = 0.75, -1.5
    lhs = oracle.spmv(A, a * x + b * z)
    rhs = a * oracle.spmv(A, x) + b * oracle.spmv(A, z)
    scale = oracle.spmv_abs(A, np.abs(a * x) + np.abs(b * z))
    assert (np.abs(lhs - rhs) <= 1e-14 * scale + 1e-300).all()


def test_spmv_laplacian27_exact():
    N = 9
    coo = spgen.stencil3d(N, N, N, 27, values="laplacian")
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    y = oracle.spmv(A, np.ones(A.n))
    L = A.row_lengths()
    # row sum = 26 - (L - 1): zero on interior rows
    assert (y == 26.0 - (L - 1)).all() and (y[L == 27] == 0).all()


def test_spmv_thread_count_invariant():
    coo = spgen.powerlaw(20_000, 20_000, 2.0, 2_000, 16.0, seed=1)
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    x = spgen.uniform(A.n, 3)
    y1 = oracle.spmv(A, x, nthreads=1)
    y4 = oracle.spmv(A, x, nthreads=4)
    assert (y1.view(np.uint64) == y4.view(np.uint64)).all()


# ---------------------------------------------------------------- SpMM

@pytest.mark.parametrize("k", [1, 3, 16])
def test_spmm_columns_are_spmv(k):
    coo = spgen.powerlaw(1500, 1200, 2.0, 300, 10.0, seed=4)
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    X = spgen.uniform(A.n * k, 5).reshape(A.n, k)
    Y = oracle.spmm(A, X)
    for j in range(k):
        assert (Y[:, j].view(np.uint64) == oracle.spmv(A, X[:, j].copy()).view(np.uint64)).all()


def test_spmm_dense_brute_force_exact():
    rng = np.random.default_rng(21)
    m, n, k = 40, 30, 5
    r, c, v = rand_coo(rng, m, n, 300)
    A = oracle.csr_from_coo(m, n, r, c, v)
    X = rng.integers(-8, 9, (n, k)).astype(np.float64)
    Y = oracle.spmm(A, X)
    Di = dense_from_coo(m, n, r, c, v).astype(np.int64)
    assert (Y == (Di @ X.astype(np.int64))).all()


# ---------------------------------------------------------------- transpose / sampled dot

def test_spmv_t_dense_exact_and_untouched_columns():
    rng = np.random.default_rng(31)
    m, n = 50, 70
    r, c, v = rand_coo(rng, m, n, 200)
    c = np.where(c >= 60, c - 10, c).astype(np.int32)  # columns 60..69 untouched
    A = oracle.csr_from_coo(m, n, r, c, v)
    dy = rng.integers(-8, 9, m).astype(np.float64)
    dx = oracle.spmv_t(A, dy)
    Di = dense_from_coo(m, n, r, c, v).astype(np.int64)
    assert (dx == (Di.T @ dy.astype(np.int64))).all()
    assert (dx[60:] == 0).all() and not np.signbit(dx[60:]).any()
    dY = rng.integers(-8, 9, (m, 3)).astype(np.float64)
    assert (oracle.spmv_t(A, dY) == Di.T @ dY.astype(np.int64)).all()


def test_adjoint_identity():
    coo = spgen.powerlaw(5_000, 4_000, 2.0, 500, 20.0, seed=6)
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    x, dy = spgen.uniform(A.n, 1), spgen.normal(A.m, 2)
    lhs = float(np.dot(oracle.spmv_t(A, dy), x))
    rhs = float(np.dot(dy, oracle.spmv(A, x)))
    scale = float(np.dot(np.abs(dy), oracle.spmv_abs(A, np.abs(x))))
    assert abs(lhs - rhs) <= 1e-13 * scale


@pytest.mark.parametrize("k", [1, 3])
def test_sddmm_is_the_central_difference_of_spmv(k):
    """Independent pin of the sampled dot: f(values) = <dY, A(values) X> is
    linear in the values, so the central difference (f(v + e_p) - f(v - e_p)) / 2
    with h = 1 has no truncation error, and with small-integer values, X and
    dY every sum is exact.  f is evaluated through the oracle's SpMM / SpMV
    only, so a wrong row or column index, a transposed operand or a dropped
    term in sddmm shows up as an exact mismatch."""
    rng = np.random.default_rng(40 + k)
    m, n = 37, 29
    r, c, v = rand_coo(rng, m, n, 160, dup=False)
    A = oracle.csr_from_coo(m, n, r, c, v)
    X = rng.integers(-8, 9, (n, k)).astype(np.float64)
    dY = rng.integers(-8, 9, (m, k)).astype(np.float64)

    def f(vals):
        Av = oracle.CSR(A.m, A.n, A.rowptr, A.colind, vals)
        Y = oracle.spmm(Av, X) if k > 1 else oracle.spmv(Av, X[:, 0].copy())[:, None]
        return float((dY * Y).sum())

    fd = np.empty(A.nnz)
    for p in range(A.nnz):
        e = np.zeros(A.nnz)
        e[p] = 1.0
        fd[p] = (f(A.values + e) - f(A.values - e)) / 2.0
    got = oracle.sddmm(A, dY[:, 0].copy(), X[:, 0].copy()) if k == 1 else oracle.sddmm(A, dY, X)
    assert (got == fd).all()


def test_rel2_hand_computed():
    """rel2 = ||y_hat - y_ref||_2 / ||y_ref||_2 on hand-computed vectors: a
    swapped argument order, a max-norm or a 1-norm each give another number."""
    # ||[3, 4]|| = 5 and the difference [0, 1] has norm 1
    assert oracle.rel2([3.0, 5.0], [3.0, 4.0]) == 0.2
    # swapped: 1 / ||[3, 5]|| = 1 / sqrt(34)
    assert oracle.rel2([3.0, 4.0], [3.0, 5.0]) == 1.0 / np.sqrt(34.0)
    # difference [1, 1]: 2-norm sqrt(2) (max-norm would give 1, 1-norm 2)
    assert oracle.rel2([4.0, 5.0], [3.0, 4.0]) == np.sqrt(2.0) / 5.0
    # [1, 2, 2] has norm 3; difference [2, -1, 2] has norm 3
    assert oracle.rel2([3.0, 1.0, 4.0], [1.0, 2.0, 2.0]) == 1.0
    # matrices are measured as one flattened vector (Frobenius norm)
    assert oracle.rel2([[3.0], [5.0]], [[3.0], [4.0]]) == 0.2
    # a vanishing reference falls back to the absolute norm of the difference
    assert oracle.rel2([3.0, 4.0], [0.0, 0.0]) == 5.0
    assert oracle.rel2([0.0, 0.0], [0.0, 0.0]) == 0.0
    # equal inputs
    assert oracle.rel2([1e-300, -7.0], [1e-300, -7.0]) == 0.0


def test_spmv_abs_brute_force():
    """spmv_abs(A, x)_i = sum_p |a_p x_{c_p}| = (|A| |x|)_i, checked exactly on
    integers against a dense brute force; x has mixed signs so that taking
    the absolute value after the sum (|A x|) would fail."""
    rng = np.random.default_rng(51)
    m, n = 45, 38
    r, c, v = rand_coo(rng, m, n, 300)
    A = oracle.csr_from_coo(m, n, r, c, v)
    x = rng.integers(-8, 9, n).astype(np.float64)
    Di = np.abs(dense(A)).astype(np.int64)
    S = oracle.spmv_abs(A, x)
    assert (S == (Di @ np.abs(x).astype(np.int64))).all()
    assert (S > np.abs(oracle.spmv(A, x))).any()
    # an empty row gives +0.0
    B = oracle.csr_from_coo(3, 4, [0, 2], [1, 3], [2.0, -5.0])
    assert list(oracle.spmv_abs(B, np.array([1.0, -3.0, 7.0, 2.0]))) == [6.0, 0.0, 10.0]
    # floats: within rounding of the dense |A| |x|, and never below |A x|
    rf, cf, vf = rand_coo(rng, m, n, 300, ints=False)
    F = oracle.csr_from_coo(m, n, rf, cf, vf)
    xf = rng.uniform(-1, 1, n)
    Sf = oracle.spmv_abs(F, xf)
    assert np.allclose(Sf, np.abs(dense(F)) @ np.abs(xf), rtol=1e-14, atol=0)
    assert (Sf >= np.abs(oracle.spmv(F, xf)) * (1 - 1e-15)).all()


def test_sddmm_closed_form():
    coo = spgen.powerlaw(800, 900, 2.0, 200, 10.0, seed=7)
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    x, dy = spgen.uniform(A.n, 1), spgen.normal(A.m, 2)
    dv = oracle.sddmm(A, dy, x)
    assert (dv == dy[A.row_of()] * x[A.colind]).all()
    X, dY = spgen.uniform(A.n * 4, 3).reshape(-1, 4), spgen.normal(A.m * 4, 4).reshape(-1, 4)
    dv4 = oracle.sddmm(A, dY, X)
    rows = A.row_of()
    for p in (0, 17, A.nnz - 1):
        s = 0.0
        for t in range(4):
            s = s + dY[rows[p], t] * X[A.colind[p], t]
        assert dv4[p] == s


# ---------------------------------------------------------------- counting formulas and UCLD

def test_byte_and_flop_model_matches_paper():
    g = kv("worked_examples.txt")
    assert int(g["bytes_per_nonzero"]) == 8 + 4
    assert abs(2 / 12 - float(g["flop_per_byte"])) < 1e-15
    assert float(g["sustained_gbs"]) * 2 / 12 == float(g["spmv_cap_gflops"])
    for n, tau in [(1, 1), (10_000, 100_000), (1 << 20, 16_777_216)]:
        expect = int(g["app_bytes_const"]) + int(g["app_bytes_per_row"]) * n + \
            int(g["app_bytes_per_nonzero"]) * tau
        assert oracle.app_bytes(n, n, tau) == expect
    # Sec. 5: 8 m k + 8 n k + (n + 1) 4 + tau (8 + 4)
    m = n = 1 << 20
    tau, k = 16_777_216, 16
    assert oracle.app_bytes(m, n, tau, k) == 8 * m * k + 8 * n * k + (n + 1) * 4 + tau * 12
    assert oracle.flops(tau, k) == 2 * tau * k


def test_ucld_worked_example():
    g = kv("worked_examples.txt")
    cols = [int(t) for t in g["ucld_row_columns"].split()]
    line = int(g["ucld_line_doubles"])
    A = oracle.csr_from_coo(1, 64, np.zeros(len(cols)), cols, np.ones(len(cols)))
    assert oracle.ucld(A, line) == float(g["ucld_value"])
    worst = oracle.csr_from_coo(1, 64, np.zeros(4), [0, 8, 16, 24], np.ones(4))
    best = oracle.csr_from_coo(1, 64, np.zeros(8), list(range(8, 16)), np.ones(8))
    assert oracle.ucld(worst, line) == float(g["ucld_worst"])
    assert oracle.ucld(best, line) == float(g["ucld_best"])


def test_dense_block_bytes_example():
    g = kv("worked_examples.txt")
    # 64 nonzeros of one dense 8 x 8 region: CRS stores value + column id each
    assert 64 * (8 + 4) == int(g["dense_block_crs_bytes"])
    assert 64 * 8 + 4 == int(g["dense_block_blocked_bytes"])


def test_compensated_sum_pin_values():
    # 1.0 followed by 4096 copies of 2^-25: plain FP32 accumulation stays at 1.0
    # (each addend is below half an ulp of 1), the exact sum is 1 + 2^-13.
    terms = np.array([1.0] + [2.0 ** -25] * 4096)
    s32 = np.float32(0)
    for t in terms.astype(np.float32):
        s32 = np.float32(s32 + t)
    assert s32 == np.float32(1.0)
    A = oracle.csr_from_coo(1, terms.size, np.zeros(terms.size), np.arange(terms.size), terms)
    assert oracle.spmv(A, np.ones(terms.size))[0] == 1.0001220703125 == 1 + 2.0 ** -13


# ---------------------------------------------------------------- RCM and vector access (Sec. 4.4, Sec. 4.2)

def sym_adj(A):
    """Neighbour sets of the pattern of A + A^T without the diagonal (brute force)."""
    nb = [set() for _ in range(A.n)]
    for i in range(A.m):
        for p in range(A.rowptr[i], A.rowptr[i + 1]):
            j = int(A.colind[p])
            if j != i:
                nb[i].add(j)
                nb[j].add(i)
    return nb


def bandwidth(A):
    if A.nnz == 0:
        return 0
    return int(np.abs(A.row_of().astype(np.int64) - A.colind).max())


def check_cm_order(nb, order):
    """Breadth-first numbering invariants of Cuthill-McKee: every vertex but a
    component's first has an earlier neighbour; the position of the earliest
    such neighbour (its parent) never decreases; siblings come in ascending
    (degree, index); a component is numbered before the next one starts."""
    pos = {v: t for t, v in enumerate(order)}
    deg = [len(s) for s in nb]
    last_parent = -1
    prev = None
    for t, v in enumerate(order):
        earlier = [pos[w] for w in nb[v] if pos[w] < t]
        if not earlier:  # a new component: everything before it is closed
            assert all(pos[w] < t for u in order[:t] for w in nb[u]), t
            last_parent, prev = -1, None
            continue
        par = min(earlier)
        assert par >= last_parent, (t, par, last_parent)
        if par == last_parent:
            assert (deg[prev], prev) < (deg[v], v), (prev, v)
        last_parent, prev = par, v


def test_rcm_is_a_permutation_and_cm_order():
    rng = np.random.default_rng(40)
    for n, nnz in [(1, 1), (7, 12), (60, 150), (300, 900)]:
        r, c, v = rand_coo(rng, n, n, nnz)
        A = oracle.csr_from_coo(n, n, r, c, v)
        perm = oracle.rcm(A)
        assert np.array_equal(np.sort(perm), np.arange(n))
        check_cm_order(sym_adj(A), list(perm[::-1]))


def test_rcm_diagonal_and_empty():
    n = 9
    A = oracle.csr_from_coo(n, n, np.arange(n, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))
    # every vertex is its own component, taken in (degree 0, index) order, then reversed
    assert np.array_equal(oracle.rcm(A), np.arange(n)[::-1])
    E = oracle.csr_from_coo(0, 0, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0))
    assert oracle.rcm(E).size == 0
    with pytest.raises(ValueError):
        oracle.rcm(oracle.csr_from_coo(2, 3, np.zeros(1, np.int32), np.ones(1, np.int32), np.ones(1)))


def test_rcm_recovers_relabeled_path_and_stencils():
    """A relabeled path regains bandwidth 1; relabeled 2D / 3D stencils come
    back within the breadth-first bound 2w - 1 (w = widest level), far below
    the relabeled bandwidth (Sec. 4.4: RCM narrows the band)."""
    n = 500
    i = np.arange(n - 1, dtype=np.int32)
    path = spgen.COO(n, n, np.concatenate([i, i + 1]), np.concatenate([i + 1, i]), np.ones(2 * (n - 1)), {})
    for coo, w_max in [(path, 1), (spgen.stencil5(30, 20, 1), 20), (spgen.stencil3d(8, 7, 6, 7, 2), None)]:
        R = spgen.relabeled(coo, 5)
        A = oracle.csr_from_coo(R.m, R.n, R.r, R.c, R.v)
        perm = oracle.rcm(A)
        B = oracle.permute(A, perm)
        nb = sym_adj(A)
        order = list(perm[::-1])
        check_cm_order(nb, order)
        # level widths of the breadth-first structure from the first vertex
        level = {order[0]: 0}
        frontier = [order[0]]
        while frontier:
            nxt = []
            for u in frontier:
                for w in nb[u]:
                    if w not in level:
                        level[w] = level[u] + 1
                        nxt.append(w)
            frontier = nxt
        widths = np.bincount(list(level.values()))
        bw = bandwidth(B)
        assert bw <= 2 * widths.max() - 1
        assert bw < bandwidth(A) / 4
        if w_max is not None:
            assert widths.max() <= w_max
    # the path: a peripheral start and bandwidth exactly 1
    Rp = spgen.relabeled(path, 5)
    Ap = oracle.csr_from_coo(n, n, Rp.r, Rp.c, Rp.v)
    assert bandwidth(oracle.permute(Ap, oracle.rcm(Ap))) == 1


def test_rcm_components_contiguous():
    # two relabeled paths of 40 and 25 vertices plus 3 isolated vertices
    a = np.arange(39, dtype=np.int32)
    b = np.arange(40, 64, dtype=np.int32)
    r = np.concatenate([a, a + 1, b, b + 1])
    c = np.concatenate([a + 1, a, b + 1, b])
    n = 68
    R = spgen.relabeled(spgen.COO(n, n, r, c, np.ones(r.size), {}), 3)
    A = oracle.csr_from_coo(n, n, R.r, R.c, R.v)
    perm = oracle.rcm(A)
    nb = sym_adj(A)
    comp = np.full(n, -1)
    for s0 in range(n):
        if comp[s0] < 0:
            stack = [s0]
            comp[s0] = s0
            while stack:
                u = stack.pop()
                for w in nb[u]:
                    if comp[w] < 0:
                        comp[w] = s0
                        stack.append(w)
    labels = comp[perm]
    runs = [labels[0]] + [labels[t] for t in range(1, n) if labels[t] != labels[t - 1]]
    assert len(runs) == len(set(runs)) == 5  # each component in one run
    assert bandwidth(oracle.permute(A, perm)) == 1


def test_degree_order_pins():
    """Hand-worked case, then invariants: a permutation whose counts never
    increase, equal counts in ascending index, and the identity when every
    column has the same count."""
    # columns used 2, 0, 3, 2, 1 times
    r = np.array([0, 0, 1, 1, 2, 2, 3, 3], dtype=np.int32)
    c = np.array([0, 2, 2, 3, 0, 4, 2, 3], dtype=np.int32)
    A = oracle.csr_from_coo(4, 5, r, c, np.ones(8))
    assert np.array_equal(oracle.degree_order(A), [2, 0, 3, 4, 1])
    rng = np.random.default_rng(41)
    for n, nnz in [(1, 0), (9, 30), (200, 1500)]:
        rr, cc, vv = rand_coo(rng, n, n, nnz)
        B = oracle.csr_from_coo(n, n, rr, cc, vv)
        perm = oracle.degree_order(B)
        cnt = np.bincount(B.colind, minlength=n)
        assert np.array_equal(np.sort(perm), np.arange(n))
        seq = cnt[perm]
        assert (np.diff(seq) <= 0).all()
        same = np.diff(seq) == 0
        assert (np.diff(perm)[same] > 0).all()
    I = oracle.csr_from_coo(6, 6, np.arange(6, dtype=np.int32), np.arange(6, dtype=np.int32), np.ones(6))
    assert np.array_equal(oracle.degree_order(I), np.arange(6))


def test_vector_access_brute_force_and_closed_forms():
    rng = np.random.default_rng(41)
    for m, n, nnz, line, parts, chunk in [(50, 70, 300, 4, 3, 5), (200, 130, 900, 16, 8, 7), (10, 10, 0, 4, 2, 3)]:
        r, c, v = rand_coo(rng, m, n, nnz)
        A = oracle.csr_from_coo(m, n, r, c, v)
        pairs = set()
        for i in range(m):
            q = (i // chunk) % parts
            for p in range(A.rowptr[i], A.rowptr[i + 1]):
                pairs.add((q, int(A.colind[p]) // line))
        expect = len(pairs) / -(-n // line)
        assert oracle.vector_access(A, line, parts, chunk) == expect
    # a diagonal matrix moves x once; a dense one once per part
    n = 512
    D = oracle.csr_from_coo(n, n, np.arange(n, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))
    assert oracle.vector_access(D, 16, 8, 64) == 1.0
    rr, cc = np.meshgrid(np.arange(64, dtype=np.int32), np.arange(48, dtype=np.int32), indexing="ij")
    F = oracle.csr_from_coo(64, 48, rr.ravel(), cc.ravel(), np.ones(rr.size))
    assert oracle.vector_access(F, 16, 8, 8) == 8.0
    assert oracle.vector_access(F, 16, 8, 64) == 1.0


# ---------------------------------------------------------------- register blocking (Sec. 4.5)

@pytest.mark.parametrize("a,b", [(1, 1), (8, 1), (1, 8), (2, 4), (8, 8), (4, 2), (3, 5)])
def test_bcsr_roundtrip_and_block_count(a, b):
    rng = np.random.default_rng(60 + a * 10 + b)
    for m, n, nnz in [(1, 1, 1), (13, 29, 40), (70, 55, 600), (64, 64, 4096)]:
        r, c, v = rand_coo(rng, m, n, nnz, dup=False)
        A = oracle.csr_from_coo(m, n, r, c, v)
        blocks = {(int(i) // a, int(j) // b) for i, j in zip(A.row_of(), A.colind)}
        for bitmap in (False, True):
            B = oracle.to_bcsr(A, a, b, bitmap)
            assert B.nblocks == len(blocks)
            assert np.array_equal(oracle.bcsr_dense(B), dense(A))
            for I in range(B.browptr.size - 1):
                cols = B.bcol[B.browptr[I]:B.browptr[I + 1]]
                assert np.all(np.diff(cols) > 0)
                assert {(I, int(J)) for J in cols} == {blk for blk in blocks if blk[0] == I}
            if bitmap:
                counts = np.array([bin(int(x)).count("1") for x in B.mask])
                assert counts.sum() == A.nnz
                assert np.array_equal(B.offset, np.concatenate([[0], np.cumsum(counts)[:-1]]))


def test_bcsr_bytes_match_the_paper():
    """A dense 8 x 8 region: 768 B in CRS (64 x 8 + 64 x 4) and 516 B blocked
    (64 x 8 + one 4-byte offset), Sec. 4.5; blocking saves memory only above
    (8ab + 4) / 12 nonzeros per block, 43 of 64 (67 %, the paper's "70 %")."""
    rr, cc = np.meshgrid(np.arange(8, dtype=np.int32), np.arange(8, dtype=np.int32), indexing="ij")
    A = oracle.csr_from_coo(8, 8, rr.ravel(), cc.ravel(), np.ones(64))
    B = oracle.to_bcsr(A, 8, 8)
    rowptr_bytes = 4 * B.browptr.size
    assert oracle.bcsr_bytes(B) - rowptr_bytes == 516
    assert 12 * A.nnz == 768
    rng = np.random.default_rng(61)
    for t, relation in [(42, -1), (43, 0), (44, 1)]:
        pick = rng.choice(64, t, replace=False)
        S = oracle.csr_from_coo(8, 8, rr.ravel()[pick], cc.ravel()[pick], np.ones(t))
        blocked = oracle.bcsr_bytes(oracle.to_bcsr(S, 8, 8)) - rowptr_bytes
        assert np.sign(12 * t - blocked) == relation, t


def test_tile_lines_brute_force_and_closed_forms():
    """Distinct (tile, x line) pairs: Python sets on random matrices; equal to
    vector_access with one part per tile (an independent oracle function, so
    a wrong tile bound or line index in either shows); closed forms for a
    diagonal and a dense matrix."""
    rng = np.random.default_rng(61)
    for m, n, nnz in [(1, 1, 1), (37, 50, 200), (300, 128, 2000), (1000, 5000, 6000)]:
        r, c, v = rand_coo(rng, m, n, nnz)
        A = oracle.csr_from_coo(m, n, r, c, v)
        rows = A.row_of()
        for line, tile in [(16, 256), (8, 7), (1, 1), (4, 1000)]:
            expect = len({(int(i) // tile, int(j) // line) for i, j in zip(rows, A.colind)})
            assert oracle.tile_lines(A, line, tile) == expect
            tiles = -(-m // tile)
            nlines = -(-n // line)
            assert oracle.vector_access(A, line, tiles, tile) * nlines == pytest.approx(expect, rel=1e-15)
    # diagonal n x n: a tile of T rows (T a multiple of the line L) touches T / L lines
    n = 4096
    D = oracle.csr_from_coo(n, n, np.arange(n), np.arange(n), np.ones(n))
    assert oracle.tile_lines(D, 16, 256) == (n // 256) * (256 // 16)
    # dense m x n: every tile touches every line
    F = oracle.csr_from_coo(10, 40, np.repeat(np.arange(10), 40), np.tile(np.arange(40), 10), np.ones(400))
    assert oracle.tile_lines(F, 16, 3) == 4 * 3
    assert oracle.tile_lines(oracle.csr_from_coo(0, 5, [], [], []), 16, 4) == 0
