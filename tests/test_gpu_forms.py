"""GPU parity of the precision and differentiation forms against the oracle.

Precision: FP32/BF16 values with FP32 vectors.  The accumulation error is
measured against the oracle on the stored (quantised) inputs widened exactly
to FP64; every row must satisfy a floating-point error bound
(Higham, Accuracy and Stability of Numerical Algorithms, 2nd ed., Ch. 3-4;
Ogita, Rump and Oishi, SIAM J. Sci. Comput. 26(6), 2005, for the compensated
dot product):
  plain FP32 rows:        |e_i| <= gamma_{L+8}(2^-24) * sum_p |a_p x_p|
  compensated long rows:  |e_i| <= 2^-24 |y_i| + (gamma_L(2^-24))^2 * S_i + 2^-45 S_i
The total error against the original FP64 data is reported (rel2).

Differentiation: transpose products, sampled dot and the autograd Function.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import spgen
from _cases import (U32, c3_submatrix, check_bound, gamma, int_valued, keep_stream, matrix, quantised,
                    single_bin_opts, stream_mm_opts, to_gpu, two_bin_opts)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spx():
    import paper_1302_1078_amd as m
    return m


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("kind", ["powerlaw", "one_long_row", "stencil27", "empty_rows"])
@pytest.mark.parametrize("vdtype", ["f32", "bf16"])
def test_precision_spmv_bounds(spx, torch, kind, vdtype):
    A = matrix(kind, seed=21)
    x = spgen.uniform(A.n, 22)
    xq = spgen.to_f32(x)
    G, A5 = quantised(A, vdtype, torch)
    y5 = oracle.spmv(A5, xq.astype(np.float64))
    S = oracle.spmv_abs(A5, xq.astype(np.float64))
    y3 = oracle.spmv(A, x)
    L = A.row_lengths()
    for name, opts in [("default", spx.default_opts(1, torch.float32)),
                       ("default-stream", keep_stream(spx.default_opts(1, torch.float32))),
                       ("block", single_bin_opts(256)), ("split", single_bin_opts(0, chunk=256)),
                       ("wave+split", two_bin_opts(300, 64, chunk=512))]:
        plan = spx.Plan.for_matrix(G, opts)
        y = spx.spmv(G, dev(torch, xq), plan=plan).cpu().numpy()
        check_bound(y, y5, S, L, opts.kahan_len, (kind, vdtype, name))
        total = oracle.rel2(y.astype(np.float64), y3)
        assert total <= (2e-6 if vdtype == "f32" else 2e-2), (kind, vdtype, name, total)


@pytest.mark.parametrize("vdtype", ["f32", "bf16"])
@pytest.mark.parametrize("k", [8, 32])
def test_precision_spmm_bounds(spx, torch, vdtype, k):
    A = matrix("powerlaw", seed=23)
    X = spgen.uniform(A.n * k, 24).reshape(A.n, k)
    Xq = spgen.to_f32(X)
    G, A5 = quantised(A, vdtype, torch)
    Y5 = oracle.spmm(A5, Xq.astype(np.float64))
    L = A.row_lengths()
    # default plan; and a plan with kahan_len 4, so that most rows take the
    # compensated path
    for kahan, opts in [(256, spx.default_opts(k, torch.float32)), (4, stream_mm_opts(k, kahan=4))]:
        plan = spx.Plan.for_matrix(G, opts)
        Y = spx.spmm(G, dev(torch, Xq), plan=plan).cpu().numpy()
        for j in (0, k // 2, k - 1):
            S = oracle.spmv_abs(A5, Xq[:, j].astype(np.float64))
            check_bound(Y[:, j], Y5[:, j], S, L, kahan, (vdtype, k, j, kahan))


def test_compensated_sum_pin(spx, torch):
    # 1.0 followed by 4096 copies of 2^-25 (exact sum 1 + 2^-13 = 1.0001220703125).
    # With compensation the FP32 result is exact; without it the lane that holds
    # 1.0 drops its small addends.
    vals = np.array([1.0] + [2.0 ** -25] * 4096)
    A = oracle.csr_from_coo(1, vals.size, np.zeros(vals.size), np.arange(vals.size), vals)
    G = spx.CSR(dev(torch, A.rowptr), dev(torch, A.colind), dev(torch, vals.astype(np.float32)), (1, vals.size))
    ones = torch.ones(vals.size, dtype=torch.float32, device="cuda:0")
    exact = np.float32(1.0001220703125)
    for opts in (single_bin_opts(256), single_bin_opts(0, chunk=1024), single_bin_opts(64)):
        y = spx.spmv(G, ones, plan=spx.Plan.for_matrix(G, opts)).cpu().numpy()
        assert y[0] == exact
    opts = single_bin_opts(256, kahan=1_000_000)  # compensation off
    y = spx.spmv(G, ones, plan=spx.Plan.for_matrix(G, opts)).cpu().numpy()
    assert y[0] != exact and abs(float(y[0]) - 1.0001220703125) < 1e-6


def test_bf16_exact_values(spx, torch):
    # integers in [-8, 8] are exact in BF16; with integer x every sum is exact
    A = int_valued(matrix("powerlaw", 25), 3)
    x = spgen.small_ints(A.n, 4)
    G, _ = quantised(A, "bf16", torch)
    y = spx.spmv(G, dev(torch, x.astype(np.float32)), plan=spx.Plan.for_matrix(G)).cpu().numpy()
    assert np.array_equal(y.astype(np.float64), oracle.spmv(A, x))


# ---------------------------------------------------------------- transpose index and products

@pytest.mark.parametrize("kind", ["powerlaw", "empty_rows", "tall", "wide"])
def test_transpose_index_bit_exact(spx, torch, kind):
    A = matrix(kind, 31)
    G = to_gpu(A)
    idx = spx.transpose_index(G)
    perm = np.argsort(A.colind, kind="stable")
    colptr = np.concatenate([[0], np.cumsum(np.bincount(A.colind, minlength=A.n))])
    assert np.array_equal(idx.perm.cpu().numpy(), perm)
    assert np.array_equal(idx.rowind.cpu().numpy(), A.row_of()[perm])
    assert np.array_equal(idx.colptr.cpu().numpy(), colptr)


@pytest.mark.parametrize("kind", ["powerlaw", "empty_rows", "tall", "wide", "one_long_row"])
@pytest.mark.parametrize("k", [1, 4, 16])
def test_spmv_t_parity(spx, torch, kind, k):
    A = matrix(kind, 32)
    G = to_gpu(A)
    dY = spgen.normal(A.m * k, 33).reshape(A.m, k)
    ref = oracle.spmv_t(A, dY)
    idx = spx.transpose_index(G)
    plan_t = spx.Plan(idx.colptr, A.n, A.m, A.nnz, spx.default_opts(k))
    plan = spx.Plan.for_matrix(G, spx.default_opts(1))
    dYd = dev(torch, dY if k > 1 else dY[:, 0])
    outs = []
    for mode, pl in ((0, None), (0, plan_t), (1, None), (1, plan)):
        dX = spx.spmv_t(G, dYd, mode=mode, index=idx, plan=pl).cpu().numpy().reshape(A.n, k)
        for j in range(k):
            assert oracle.rel2(dX[:, j], ref[:, j]) <= 1e-12, (kind, k, mode, j)
        outs.append(dX)
    again = spx.spmv_t(G, dYd, mode=0, index=idx, plan=plan_t).cpu().numpy().reshape(A.n, k)
    assert np.array_equal(outs[1].view(np.uint64), again.view(np.uint64))  # deterministic


@pytest.mark.parametrize("dtype,nnz", [(d, n) for d in ("f64", "f32", "bf16")
                                       for n in (0, 1, 8191, 8192, 3 * 8192 + 77, 300_001)]
                         + [("f32", 4096 * 8192 + 5)])
def test_values_to_csc_is_the_permutation(spx, torch, dtype, nnz):
    """The two-pass block transposition returns values[perm] bit for bit:
    empty, one element, one block minus one, exactly one block, several
    blocks with a ragged last one, and (f32) just past the 4,096 blocks that
    the workgroup-sorted first pass handles, so the plain pass runs (perm: a
    random permutation)."""
    from paper_1302_1078_amd.ops import CSCIndex
    rng = np.random.default_rng(nnz)
    perm = rng.permutation(nnz).astype(np.int32)
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dtype]
    vals = torch.from_numpy(spgen.uniform(max(nnz, 1), 3)[:nnz]).to("cuda:0").to(tdt)
    pm = dev(torch, perm)
    vmap = spx.csc_value_map(CSCIndex(None, None, pm))
    got = spx.values_to_csc(vals, vmap)
    want = vals[pm.long()]
    assert torch.equal(got.view(torch.int16) if dtype == "bf16" else got,
                       want.view(torch.int16) if dtype == "bf16" else want)


@pytest.mark.parametrize("kind", ["powerlaw", "wide", "one_long_row"])
@pytest.mark.parametrize("k", [1, 3])
def test_spmv_t_csc_values_bitwise(spx, torch, kind, k):
    """A^T dY with values moved to CSC order (perm = NULL) is bitwise the
    transpose that reads them through perm, with and without a plan."""
    from paper_1302_1078_amd.ops import CSCIndex
    A = matrix(kind, 36)
    G = to_gpu(A)
    dY = spgen.normal(A.m * k, 37).reshape(A.m, k)
    dYd = dev(torch, dY if k > 1 else dY[:, 0])
    idx = spx.transpose_index(G)
    vcsc = spx.values_to_csc(G.values, spx.csc_value_map(idx))
    nop = CSCIndex(idx.colptr, idx.rowind, None)
    plan_t = spx.Plan(idx.colptr, A.n, A.m, A.nnz, spx.default_opts(k))
    for pl in (None, plan_t):
        a = spx.spmv_t(G, dYd, mode=0, index=idx, plan=pl).cpu().numpy()
        b = spx.spmv_t(G.with_values(vcsc), dYd, mode=0, index=nop, plan=pl).cpu().numpy()
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_spmv_t_exact_inputs_and_adjoint(spx, torch):
    A = int_valued(matrix("powerlaw", 34), 1)
    G = to_gpu(A)
    dy = spgen.small_ints(A.m, 5)
    ref = oracle.spmv_t(A, dy)
    for mode in (0, 1):
        assert np.array_equal(spx.spmv_t(G, dev(torch, dy), mode=mode).cpu().numpy(), ref)
    B = matrix("powerlaw", 35)
    G = to_gpu(B)
    x, dy = spgen.uniform(B.n, 1), spgen.normal(B.m, 2)
    atdy = spx.spmv_t(G, dev(torch, dy), mode=0).cpu().numpy()
    ax = spx.spmv(G, dev(torch, x)).cpu().numpy()
    scale = float(np.dot(np.abs(dy), oracle.spmv_abs(B, np.abs(x))))
    assert abs(float(np.dot(atdy, x)) - float(np.dot(dy, ax))) <= 1e-12 * scale


@pytest.mark.parametrize("k", [1, 4])
def test_sddmm_parity(spx, torch, k):
    A = matrix("powerlaw", 36)
    G = to_gpu(A)
    dY = spgen.normal(A.m * k, 37).reshape(A.m, k)
    X = spgen.uniform(A.n * k, 38).reshape(A.n, k)
    ref = oracle.sddmm(A, dY, X)
    for plan in (None, spx.Plan.for_matrix(G, spx.default_opts(1))):
        if k == 1:
            out = spx.sddmm(G, dev(torch, dY[:, 0]), dev(torch, X[:, 0]), plan=plan).cpu().numpy()
            assert np.array_equal(out.view(np.uint64), ref.view(np.uint64))  # one rounded product
        else:
            out = spx.sddmm(G, dev(torch, dY), dev(torch, X), plan=plan).cpu().numpy()
            scale = oracle.sddmm(A, np.abs(dY), np.abs(X))
            assert (np.abs(out - ref) <= gamma(k + 1, 2.0 ** -53) * scale).all()
    out32 = spx.sddmm(G, dev(torch, dY.astype(np.float32)), dev(torch, X.astype(np.float32))).cpu().numpy()
    ref32 = oracle.sddmm(A, spgen.to_f32(dY).astype(np.float64), spgen.to_f32(X).astype(np.float64))
    scale = oracle.sddmm(A, np.abs(dY), np.abs(X))
    assert (np.abs(out32 - ref32) <= gamma(k + 1, U32) * scale * 1.01).all()


# ---------------------------------------------------------------- autograd

def test_autograd_gradcheck_f64(spx, torch):
    coo = spgen.powerlaw(60, 50, 2.0, 40, 5.0, seed=3)
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    G = to_gpu(A)
    for mode in (0, 1):
        g = spx.GradContext(G, mode=mode)
        v = G.values.clone().requires_grad_(True)
        x = dev(torch, spgen.uniform(A.n, 4)).requires_grad_(True)
        assert torch.autograd.gradcheck(lambda vv, xx: spx.spmv_autograd(vv, xx, g), (v, x),
                                        eps=1e-6, atol=1e-9, rtol=1e-7)
        X = dev(torch, spgen.uniform(A.n * 3, 5).reshape(A.n, 3)).requires_grad_(True)
        g3 = spx.GradContext(G, mode=mode, k=3)
        assert torch.autograd.gradcheck(lambda vv, xx: spx.spmv_autograd(vv, xx, g3), (v, X),
                                        eps=1e-6, atol=1e-9, rtol=1e-7)


def test_autograd_c3_submatrix_reference_and_fd_f32(spx, torch):
    # the 2,000-row submatrix of the differentiation workload: its 10 longest
    # rows (18k-19k nonzeros, split rows) plus 1,990 seeded rows
    A = c3_submatrix()
    A32 = spx.CSR(dev(torch, A.rowptr), dev(torch, A.colind), dev(torch, spgen.to_f32(A.values)), (A.m, A.n))
    x = spgen.to_f32(spgen.uniform(A.n, 7))
    dy = spgen.to_f32(spgen.normal(A.m, 8))
    g = spx.GradContext(A32, mode=0)
    v = A32.values.clone().requires_grad_(True)
    xt = dev(torch, x).requires_grad_(True)
    y = spx.spmv_autograd(v, xt, g)
    y.backward(dev(torch, dy))
    # reference gradients in FP64 on the host: scipy's sparse transpose product
    # and the closed form of the sampled dot
    S = sp.csr_matrix((spgen.to_f32(A.values).astype(np.float64), A.colind, A.rowptr), shape=(A.m, A.n))
    assert np.allclose(xt.grad.cpu().numpy(), S.T @ dy.astype(np.float64), rtol=1e-5, atol=1e-5)
    dv_ref = dy.astype(np.float64)[A.row_of()] * x.astype(np.float64)[A.colind]
    assert np.allclose(v.grad.cpu().numpy(), dv_ref, rtol=1e-6, atol=1e-7)
    # central differences with h = 1: y is bilinear, so there is no truncation error
    f = lambda vv, xx: float(torch.dot(spx.spmv_autograd(vv, xx, g).double(), dev(torch, dy).double()))  # noqa: E731
    rng = np.random.default_rng(1)
    L = A.row_lengths()
    long_rows = np.flatnonzero(L > 2048)
    picks = list(rng.choice(A.nnz, 20, replace=False)) + [int(A.rowptr[A.m] - 1)]
    picks += [int(A.rowptr[i]) + int(rng.integers(L[i])) for i in long_rows[:5]]  # nonzeros of split rows
    with torch.no_grad():
        for p in picks:
            e = torch.zeros_like(v)
            e[p] = 1.0
            fd = (f(v + e, xt) - f(v - e, xt)) / 2.0
            assert abs(fd - float(v.grad[p])) <= 1e-4 * (1 + abs(fd))
        for j in rng.choice(A.n, 20, replace=False):
            e = torch.zeros_like(xt)
            e[j] = 1.0
            fd = (f(v, xt + e) - f(v, xt - e)) / 2.0
            assert abs(fd - float(xt.grad[j])) <= 1e-4 * (1 + abs(fd))


@pytest.mark.parametrize("mode", [0, 1])
def test_autograd_c3_submatrix_gradcheck_f64(spx, torch, mode):
    """torch.autograd.gradcheck (fast mode) in FP64 on the differentiation
    workload's 2,000-row submatrix, for x and for a 3-column X through a
    context built for k = 1 (its plans for k = 3 are made on first use).  y is
    bilinear in (values, x), so the difference step can be 1: the numerical
    Jacobian then carries rounding error only."""
    A = c3_submatrix()
    G = to_gpu(A)
    g = spx.GradContext(G, mode=mode)
    v = G.values.clone().requires_grad_(True)
    x = dev(torch, spgen.uniform(A.n, 4)).requires_grad_(True)
    X = dev(torch, spgen.uniform(A.n * 3, 5).reshape(A.n, 3)).requires_grad_(True)
    # mode 0 (CSC gather) is deterministic, so two backward passes must agree
    # bit for bit; mode 1 adds into dx with atomics in no fixed order, so two
    # passes may differ by reordering: at most about 2 (deg + 1) 2^-53 times
    # sum |a| |dy| per column, far below 1e-10 at these degrees and magnitudes
    nondet = 0.0 if mode == 0 else 1e-10
    for inp in (x, X):
        assert torch.autograd.gradcheck(lambda vv, xx: spx.spmv_autograd(vv, xx, g), (v, inp),
                                        eps=1.0, atol=1e-8, rtol=1e-8, fast_mode=True, nondet_tol=nondet)


# ---------------------------------------------------------------- saved gather

def save_plans(spx, torch, vdtype):
    """Plans that reach every SpMV traversal the save variant stores from:
    none (unbinned row groups), the default binning, kept stream tiles,
    multi-row groups (rows of at most 4 nonzeros, 4 per 4-lane group), one
    workgroup per row, and split rows."""
    t = torch.float64 if vdtype == "f64" else torch.float32
    return [("none", None),
            ("default", spx.default_opts(1, t)),
            ("default-stream", keep_stream(spx.default_opts(1, t))),
            ("multi-row", spx.PlanOpts.from_dict({"nbins": 3, "upper": [4, 64], "lanes": [4, 64, 0],
                                                  "split_chunk": 256, "kahan_len": 256, "max_k": 1})),
            ("block", single_bin_opts(256)),
            ("split", single_bin_opts(0, chunk=256)),
            ("wave+split", two_bin_opts(300, 64, chunk=512))]


@pytest.mark.parametrize("kind", ["uniform", "powerlaw", "stencil27", "empty_rows", "one_long_row", "tall",
                                  "wide"])
@pytest.mark.parametrize("vdtype", ["f64", "f32", "bf16"])
def test_spmv_save_and_sddmm_saved(spx, torch, kind, vdtype):
    """The save variant gives bitwise the product of csr_spmv and stores
    exactly x[colind[p]]; the sampled dot read from it is bitwise the gathering
    one and the oracle's single rounded product dy[row(p)] x[colind[p]]."""
    A = matrix(kind, seed=41)
    x = spgen.uniform(A.n, 42)
    dy = spgen.normal(A.m, 43)
    if vdtype == "f64":
        G = to_gpu(A)
        xs, dys = x, dy
        ref = oracle.sddmm(A, dy[:, None], x[:, None])
    else:
        G, _ = quantised(A, vdtype, torch)
        xs, dys = spgen.to_f32(x), spgen.to_f32(dy)
        # the product of two FP32 numbers is exact in FP64, so rounding it once
        # to FP32 is the kernel's single FP32 multiplication
        ref = oracle.sddmm(A, dys.astype(np.float64)[:, None], xs.astype(np.float64)[:, None]).astype(np.float32)
    xd, dyd = dev(torch, xs), dev(torch, dys)
    gathered = xs[A.colind]
    for name, opts in save_plans(spx, torch, vdtype):
        plan = None if opts is None else spx.Plan.for_matrix(G, opts)
        y, xsave = spx.spmv_save(G, xd, plan=plan)
        y0 = spx.spmv(G, xd, plan=plan)
        assert torch.equal(y.view(torch.int8), y0.view(torch.int8)), (kind, vdtype, name)
        assert np.array_equal(xsave.cpu().numpy().view(np.uint8), gathered.view(np.uint8)), (kind, vdtype, name)
        out = spx.sddmm_saved(G, dyd, xsave, plan=plan)
        out0 = spx.sddmm(G, dyd, xd, plan=plan)
        assert torch.equal(out.view(torch.int8), out0.view(torch.int8)), (kind, vdtype, name)
        assert np.array_equal(out.cpu().numpy().view(np.uint8), ref.view(np.uint8)), (kind, vdtype, name)


def test_saved_gather_edges_and_misuse(spx, torch):
    from paper_1302_1078_amd import _lib
    L = _lib.load()
    # empty matrix, and rows without nonzeros only
    for m, n in [(0, 4), (5, 3)]:
        A = oracle.csr_from_coo(m, n, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0))
        G = to_gpu(A)
        y, xsave = spx.spmv_save(G, dev(torch, spgen.uniform(n, 1)))
        assert xsave.numel() == 0 and (y.cpu().numpy() == 0).all()
        assert spx.sddmm_saved(G, dev(torch, spgen.uniform(m, 2)), xsave).numel() == 0
    A = matrix("powerlaw", seed=44)
    G = to_gpu(A)
    x = dev(torch, spgen.uniform(A.n, 45))
    y = torch.empty(A.m, dtype=torch.float64, device="cuda:0")
    # null xsave with nonzeros present
    st = L.csr_spmv_save(A.m, A.n, A.nnz, G.rowptr.data_ptr(), G.colind.data_ptr(), G.values.data_ptr(),
                         _lib.SPX_F64, x.data_ptr(), y.data_ptr(), _lib.SPX_F64, None, None, None)
    assert st == _lib.SPX_ERR_INVALID
    # a staged plan has no saved-gather variant
    S = to_gpu(matrix("stencil27", seed=2))
    with pytest.raises(spx.SpxError):
        spx.spmv_save(S, dev(torch, spgen.uniform(S.n, 1)), plan=spx.Plan.staged(S, 8))
    # dtype rules of the sampled dot
    _, xsave = spx.spmv_save(G, x)
    out = torch.empty(A.nnz, dtype=torch.float64, device="cuda:0")
    dy = dev(torch, spgen.normal(A.m, 46))
    st = L.csr_sddmm_saved(A.m, A.nnz, G.rowptr.data_ptr(), dy.data_ptr(), xsave.data_ptr(), out.data_ptr(),
                           _lib.SPX_BF16, None, None)
    assert st == _lib.SPX_ERR_UNSUPPORTED
    st = L.csr_sddmm_saved(A.m, A.nnz, G.rowptr.data_ptr(), dy.data_ptr(), None, out.data_ptr(),
                           _lib.SPX_F64, None, None)
    assert st == _lib.SPX_ERR_INVALID
    with pytest.raises(ValueError):
        spx.sddmm_saved(G, dy.float(), xsave)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_autograd_saved_gather_bitwise(spx, torch, dtype):
    """Gradients with and without the saved gather agree bit for bit on the
    differentiation workload's 2,000-row submatrix (mode 0, deterministic)."""
    A = c3_submatrix()
    t = torch.float64 if dtype == "f64" else torch.float32
    G = spx.CSR(dev(torch, A.rowptr), dev(torch, A.colind), dev(torch, A.values).to(t), (A.m, A.n))
    x = dev(torch, spgen.uniform(A.n, 7)).to(t)
    dy = dev(torch, spgen.normal(A.m, 8)).to(t)
    grads = []
    for save in (True, False):
        g = spx.GradContext(G, mode=0, save_gather=save)
        v = G.values.clone().requires_grad_(True)
        xt = x.clone().requires_grad_(True)
        y = spx.spmv_autograd(v, xt, g)
        y.backward(dy)
        grads.append((y.detach(), v.grad, xt.grad))
    for a, b in zip(*grads):
        assert torch.equal(a.view(torch.int8), b.view(torch.int8))


def test_saved_gather_graph_replay(spx, torch):
    """The saved-gather forward and its sampled dot captured in a HIP graph:
    every replay (x and dy changed eagerly in between) equals eager calls."""
    A = matrix("powerlaw", seed=47)
    G = to_gpu(A)
    plan = spx.Plan.for_matrix(G, spx.default_opts(1))
    x = dev(torch, spgen.uniform(A.n, 48))
    dy = dev(torch, spgen.normal(A.m, 49))
    y = torch.empty(A.m, dtype=torch.float64, device="cuda:0")
    xg = torch.empty(A.nnz, dtype=torch.float64, device="cuda:0")
    out = torch.empty(A.nnz, dtype=torch.float64, device="cuda:0")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up on a side stream before capture
        spx.spmv_save(G, x, y=y, xsave=xg, plan=plan)
        spx.sddmm_saved(G, dy, xg, plan=plan, out=out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        spx.spmv_save(G, x, y=y, xsave=xg, plan=plan)
        spx.sddmm_saved(G, dy, xg, plan=plan, out=out)
    for r in range(3):
        x.mul_(-0.5)
        dy.add_(1.0)
        y_ref = spx.spmv(G, x, plan=plan)
        out_ref = spx.sddmm(G, dy, x, plan=plan)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y.view(torch.int64), y_ref.view(torch.int64)), r
        assert torch.equal(out.view(torch.int64), out_ref.view(torch.int64)), r


def scatter_case(name: str) -> oracle.CSR:
    """Patterns for the atomic transpose's per-workgroup merging: "hot" puts
    most nonzeros in four columns, so every workgroup adds many contributions
    into few table slots; "distinct" gives long rows of distinct columns, so a
    workgroup meets more columns than its table holds and the rest go straight
    to memory; "mixed" interleaves the two."""
    rng = np.random.default_rng(sum(map(ord, name)))
    if name == "hot":
        m, n = 20000, 5000
        L = rng.integers(1, 9, m)
        cols = [np.unique(np.where(rng.random(l) < 0.8, rng.integers(0, 4, l), rng.integers(0, n, l)))
                for l in L]
    elif name == "distinct":
        m, n = 6, 300_000
        cols = [np.sort(rng.choice(n, 90_000, replace=False)) for _ in range(m)]
    else:
        m, n = 3000, 60_000
        cols = []
        for i in range(m):
            l = int(rng.integers(0, 200)) if i % 3 else int(rng.integers(0, 6))
            c = rng.integers(0, n, l)
            c[: l // 4] = rng.integers(0, 8, l // 4)
            cols.append(np.unique(c))
    rowptr = np.zeros(m + 1, dtype=np.int32)
    rowptr[1:] = np.cumsum([len(c) for c in cols])
    colind = np.concatenate(cols).astype(np.int32)
    return oracle.CSR(m, n, rowptr, colind, spgen.small_ints(len(colind), 3).astype(np.float64))


@pytest.mark.parametrize("name", ["hot", "distinct", "mixed"])
@pytest.mark.parametrize("vname", ["f64", "f32", "bf16"])
def test_spmv_t_atomic_merging_exact(spx, torch, name, vname):
    """Small-integer values and dy: every partial sum is exact in FP32 and
    FP64, so the atomic scatter, in whatever order its additions land, gives
    the oracle's A^T dy bit for bit, through its default traversal and a
    stream-bin plan."""
    A = scatter_case(name)
    vt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[vname]
    xt = torch.float64 if vname == "f64" else torch.float32
    G = to_gpu(A, vt)
    dy = spgen.small_ints(A.m, 4)
    ref = oracle.spmv_t(A, dy)
    assert np.abs(ref).max() < 2 ** 24
    dyd = dev(torch, dy).to(xt)
    for pl in (None, spx.Plan.for_matrix(G, keep_stream(spx.default_opts(1, vt)))):
        got = spx.spmv_t(G, dyd, mode=1, plan=pl).double().cpu().numpy()
        assert np.array_equal(got, ref), (name, vname)


@pytest.mark.parametrize("mode", [0, 1])
def test_spmv_t_single_column_strided(spx, torch, mode):
    """k = 1 given as m x 1 and n x 1 column views of wider arrays
    (lddy = 3, lddx = 5): the result lands in the viewed column only, and
    the other columns keep their contents."""
    A = matrix("powerlaw", 38)
    G = to_gpu(A)
    dy = spgen.normal(A.m, 39)
    ref = oracle.spmv_t(A, dy)
    wide_dy = torch.zeros(A.m, 3, dtype=torch.float64, device="cuda:0")
    wide_dy[:, 1] = dev(torch, dy)
    wide_dx = torch.full((A.n, 5), 7.0, dtype=torch.float64, device="cuda:0")
    spx.spmv_t(G, wide_dy[:, 1:2], mode=mode, out=wide_dx[:, 2:3])
    got = wide_dx.cpu().numpy()
    assert oracle.rel2(got[:, 2], ref) <= 1e-12
    assert np.all(np.delete(got, 2, axis=1) == 7.0)


def test_sddmm_single_column_strided(spx, torch):
    """k = 1 given as m x 1 and n x 1 column views of wider arrays
    (lddy = 3, ldx = 4): the sampled dot reads the viewed columns only and
    equals the vector call bit for bit (and the oracle within 1e-12)."""
    A = matrix("powerlaw", 40)
    G = to_gpu(A)
    dy, x = spgen.normal(A.m, 41), spgen.uniform(A.n, 42)
    wide_dy = torch.full((A.m, 3), 5.0, dtype=torch.float64, device="cuda:0")
    wide_x = torch.full((A.n, 4), -3.0, dtype=torch.float64, device="cuda:0")
    wide_dy[:, 2] = dev(torch, dy)
    wide_x[:, 1] = dev(torch, x)
    got = spx.sddmm(G, wide_dy[:, 2:3], wide_x[:, 1:2])
    want = spx.sddmm(G, dev(torch, dy), dev(torch, x))
    assert torch.equal(got, want)
    ref = oracle.sddmm(A, dy.reshape(-1, 1), x.reshape(-1, 1))
    assert oracle.rel2(got.cpu().numpy(), ref) <= 1e-12


def test_spmv_t_atomic_graph_replay(spx, torch):
    """The atomic transpose (zeroing kernel, then the merged scatter) captured
    in a HIP graph and replayed four times with eager work between replays:
    on small-integer inputs every replay gives the eager result exactly."""
    A = scatter_case("mixed")
    G = to_gpu(A, torch.float32)
    plan = spx.Plan.for_matrix(G, spx.default_opts(1, torch.float32))
    dy = dev(torch, spgen.small_ints(A.m, 6)).float()
    eager = spx.spmv_t(G, dy, mode=1, plan=plan).clone()
    assert np.array_equal(eager.double().cpu().numpy(), oracle.spmv_t(A, dy.double().cpu().numpy()))
    out = torch.empty_like(eager)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        spx.spmv_t(G, dy, mode=1, plan=plan, out=out)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        spx.spmv_t(G, dy, mode=1, plan=plan, out=out)
    for i in range(4):
        out.fill_(float(i + 1))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), i
