"""Full-size parity, in the launch configuration the benchmark times (default
plans, or the autotuned batch), against the FP64 oracle run on the host over
every output element.  The oracle's inputs are the generators' triplets
assembled by the oracle itself; nothing it reads comes from the GPU.

  C1  power-law 1,048,576 rows, 16.8 M nonzeros: CSR assembly bit-exact;
      FP64 SpMV (default plan and the benchmark's plan with hot x) and SpMM
      (k = 16).
  C2  27-point stencil on 128^3 (55.7 M nonzeros) and the C1 power-law
      matrix: SpMV (k = 1) and SpMM (k = 8, 32) with FP64, FP32 and BF16
      values, every element against the oracle; the stencil's SpMM also
      through the staged plan the benchmark reports beside the default.
  C3  power-law 524,288 rows, FP32: one autograd forward and backward
      (y, dx = A^T dy, dvalues).
  C4  the 256-matrix batch with autotuned plans (autotune.tune_batch), replayed
      from a HIP graph.
  C0  uniform 10,000 rows: SpMV.

FP64 results: every row within 2(L + 2) 2^-53 sum_p |a_p x_p| and rel2 <=
1e-12.  FP32 / BF16 results: the per-row error bounds of the precision form
against the oracle on the quantised inputs (U32 = 2^-24; compensated rows
above kahan_len), and their total error against the FP64 oracle on the
original data."""
import numpy as np
import pytest

import oracle
import spgen
from _cases import U32, check_bound, gamma

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

U64 = 2.0 ** -53


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


def upload(spx, torch, coo):
    return spx.from_coo(coo.m, coo.n, dev(torch, coo.r), dev(torch, coo.c), dev(torch, coo.v))


def check_f64(y, A, X, what):
    """y (m x k) against the oracle: per-row bound and rel2."""
    X = X.reshape(A.n, -1)
    y = y.reshape(A.m, -1)
    L = A.row_lengths().astype(np.float64)
    absA = oracle.CSR(A.m, A.n, A.rowptr, A.colind, np.abs(A.values))
    ref = oracle.spmm(A, X) if X.shape[1] > 1 else oracle.spmv(A, X[:, 0])[:, None]
    S = oracle.spmm(absA, np.abs(X)) if X.shape[1] > 1 else oracle.spmv(absA, np.abs(X[:, 0]))[:, None]
    err = np.abs(y - ref)
    assert (err <= 2.0 * (L[:, None] + 2.0) * U64 * S).all(), (what, "per-row bound")
    for j in range(X.shape[1]):
        assert oracle.rel2(y[:, j], ref[:, j]) <= 1e-12, (what, j)


@pytest.fixture(scope="module")
def c2_stencil(spx, torch):
    coo = spgen.workload_c2_stencil(0)
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    return A, upload(spx, torch, coo)


@pytest.fixture(scope="module")
def c1_matrix(spx, torch):
    coo = spgen.workload_c1(0)
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    return A, upload(spx, torch, coo)


def test_c1_assembly_spmv_spmm(spx, torch, c1_matrix):
    A, G = c1_matrix  # G assembled on the device from the generator's triplets
    assert np.array_equal(G.rowptr.cpu().numpy(), A.rowptr)
    assert np.array_equal(G.colind.cpu().numpy(), A.colind)
    assert np.array_equal(G.values.cpu().numpy(), A.values)
    x = spgen.uniform(A.n, 1)
    y = spx.spmv(G, dev(torch, x), plan=spx.Plan.for_matrix(G, spx.default_opts(1))).cpu().numpy()
    check_f64(y, A, x, "C1 SpMV")
    # the benchmark's SpMV plan: the default bins with the 65,536 most-used
    # columns' x entries packed (bitwise the plain plan's y)
    import bench
    hot = spx.Plan.for_matrix(G, spx.default_opts(1)).attach_hot_x(G, bench.HOT_X_COLUMNS)
    yh = spx.spmv(G, dev(torch, x), plan=hot).cpu().numpy()
    assert np.array_equal(yh.view(np.uint64), y.view(np.uint64))
    check_f64(yh, A, x, "C1 SpMV, hot x plan")
    k = 16
    X = spgen.uniform(A.n * k, 2).reshape(A.n, k)
    Y = spx.spmm(G, dev(torch, X), plan=spx.Plan.for_matrix(G, spx.default_opts(k))).cpu().numpy()
    check_f64(Y, A, X, "C1 SpMM k=16")


def oracle_product(A, X):
    """FP64 oracle product for X of shape n x k (k = 1 uses the SpMV)."""
    return oracle.spmm(A, X) if X.shape[1] > 1 else oracle.spmv(A, X[:, 0].copy())[:, None]


# unit roundoff of the stored values: BF16 is the round-to-nearest-even of the
# FP32-rounded value, so it carries both roundings
U_VALUE = {"f32": U32, "bf16": 2.0 ** -8 + U32 + 2.0 ** -8 * U32}


def check_precision_form(spx, torch, A, G, k, what, staged=False):
    """The precision form in the benchmark's launch configuration (default
    plan of each value type) against the oracle, every output element:
      f64          per-row bound and rel2 <= 1e-12 against the FP64 oracle;
      f32 / bf16   per-row accumulation bound against the oracle on the
                   quantised inputs widened exactly (plain rows gamma_{L+8},
                   compensated rows above kahan_len near one rounding), and
                   the total error against the FP64 oracle on the original
                   data: (u_v + u_x + u_v u_x) S + gamma_{L+8} (1 + u_v)(1 + u_x) S,
                   S = sum_p |a_p x_p|."""
    L = A.row_lengths()
    X64 = spgen.uniform(A.n * k, 7, spgen.TAG_X).reshape(A.n, k)
    Xq = spgen.to_f32(X64)
    absA = oracle.CSR(A.m, A.n, A.rowptr, A.colind, np.abs(A.values))
    ref64 = oracle_product(A, X64)
    S64 = oracle_product(absA, np.abs(X64))
    for vname in ("f64", "f32", "bf16"):
        if vname == "f64":
            Gv, Xd, wide = G, dev(torch, X64), None
        elif vname == "f32":
            Gv, Xd = G.with_values(G.values.float()), dev(torch, Xq)
            wide = spgen.to_f32(A.values).astype(np.float64)
        else:
            Gv, Xd = G.with_values(G.values.to(torch.bfloat16)), dev(torch, Xq)
            wide = spgen.bf16_bits_to_f64(spgen.to_bf16_bits(A.values))
        opts = spx.default_opts(k, Gv.values.dtype)
        plan = spx.Plan.staged(Gv, k, Xd.dtype) if staged else spx.Plan.for_matrix(Gv, opts)
        if k == 1:
            y = spx.spmv(Gv, Xd[:, 0].contiguous(), plan=plan).double().cpu().numpy()[:, None]
        else:
            y = spx.spmm(Gv, Xd, plan=plan).double().cpu().numpy()
        del Xd, plan
        if vname == "f64":
            check_f64(y, A, X64, f"{what} k={k} f64")
            continue
        A5 = oracle.CSR(A.m, A.n, A.rowptr, A.colind, wide)
        absA5 = oracle.CSR(A.m, A.n, A.rowptr, A.colind, np.abs(wide))
        Xq64 = Xq.astype(np.float64)
        y5 = oracle_product(A5, Xq64)
        S5 = oracle_product(absA5, np.abs(Xq64))
        uv = U_VALUE[vname]
        tot = (uv + U32 + uv * U32) + gamma(L + 8, U32)[:, None] * (1 + uv) * (1 + U32)
        assert (np.abs(y - ref64) <= tot * S64).all(), (what, k, vname, "total error vs FP64 oracle")
        for j in range(k):
            check_bound(y[:, j], y5[:, j], S5[:, j], L, opts.kahan_len, (what, k, vname, j))


@pytest.mark.parametrize("k", [1, 8, 32])
def test_c2_stencil_precisions(spx, torch, c2_stencil, k):
    A, G = c2_stencil
    check_precision_form(spx, torch, A, G, k, "C2 27-point 128^3")


@pytest.mark.parametrize("k", [8, 32])
def test_c2_stencil_precisions_staged(spx, torch, c2_stencil, k):
    A, G = c2_stencil
    check_precision_form(spx, torch, A, G, k, "C2 27-point 128^3, staged plan", staged=True)


@pytest.mark.parametrize("k", [1, 8, 32])
def test_c2_powerlaw_precisions(spx, torch, c1_matrix, k):
    A, G = c1_matrix
    check_precision_form(spx, torch, A, G, k, "C2 power-law 1M")


def test_c3_autograd_step(spx, torch):
    coo = spgen.workload_c3(0)
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    G = upload(spx, torch, coo)
    del coo
    q = spgen.to_f32(A.values)
    A32 = oracle.CSR(A.m, A.n, A.rowptr, A.colind, q.astype(np.float64))
    G32 = G.with_values(G.values.float())
    x = spgen.to_f32(spgen.uniform(A.n, 3))
    dy = spgen.to_f32(spgen.normal(A.m, 4, spgen.TAG_DY))
    g = spx.GradContext(G32)
    v = G32.values.clone().requires_grad_(True)
    xt = dev(torch, x).requires_grad_(True)
    y = spx.spmv_autograd(v, xt, g)
    y.backward(dev(torch, dy))
    L = A.row_lengths()
    absA = oracle.CSR(A.m, A.n, A.rowptr, A.colind, np.abs(A32.values))
    xd, dyd = x.astype(np.float64), dy.astype(np.float64)
    check_bound(y.detach().double().cpu().numpy(), oracle.spmv(A32, xd), oracle.spmv(absA, np.abs(xd)), L,
                g.plan.opts.kahan_len, "C3 forward")
    # dx = A^T dy: column j sums its column's products (CSC traversal, plan of the CSC pattern)
    Lc = np.bincount(A.colind, minlength=A.n)
    dx5 = oracle.spmv_t(A32, dyd)
    Sc = oracle.spmv_t(absA, np.abs(dyd))
    check_bound(xt.grad.double().cpu().numpy(), dx5, Sc, Lc, g.plan_t.opts.kahan_len, "C3 dx")
    # dvalues[p] = dy[row] * x[col]: one FP32 product, correctly rounded
    dv5 = oracle.sddmm(A, dyd, xd)
    dv = v.grad.double().cpu().numpy()
    assert (np.abs(dv - dv5) <= U32 * np.abs(dv5)).all()


def test_c4_batch(spx, torch):
    from paper_1302_1078_amd import autotune
    from paper_1302_1078_amd.batch import Batched
    specs = spgen.batch_specs(256, seed=0)
    mats, Xs, refs = [], [], []
    for i, s in enumerate(specs):
        coo = spgen.batch_matrix(s, 0, i)
        A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
        G = upload(spx, torch, coo)
        X = spgen.to_f32(spgen.uniform(A.n * s.k, 1000 + i, spgen.TAG_X).reshape(A.n, s.k))
        mats.append(G.with_values(G.values.float()))
        Xs.append(dev(torch, X[:, 0] if s.k == 1 else X))
        refs.append((A, X))
    opts, rep = autotune.tune_batch(mats, Xs, reps=3)
    assert len(opts) == len(mats) and rep["accepted_matrices"] <= rep["changed_per_matrix"]
    B = Batched(mats, Xs, opts=opts)
    g = B.capture()
    g.replay()
    torch.cuda.synchronize()
    for i, ((A, X), Y, o) in enumerate(zip(refs, B.Ys, opts)):
        A5 = oracle.CSR(A.m, A.n, A.rowptr, A.colind, spgen.to_f32(A.values).astype(np.float64))
        absA5 = oracle.CSR(A.m, A.n, A.rowptr, A.colind, np.abs(A5.values))
        Yh = Y.double().cpu().numpy().reshape(A.m, -1)
        L = A.row_lengths()
        for j in range(X.shape[1]):
            xq = X[:, j].astype(np.float64)
            check_bound(Yh[:, j], oracle.spmv(A5, xq), oracle.spmv(absA5, np.abs(xq)), L, o.kahan_len,
                        ("C4", i, j))


def test_c0(spx, torch):
    coo = spgen.workload_c0(0)
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    G = upload(spx, torch, coo)
    x = spgen.uniform(A.n, 5)
    y = spx.spmv(G, dev(torch, x), plan=spx.Plan.for_matrix(G)).cpu().numpy()
    check_f64(y, A, x, "C0 SpMV")


@pytest.mark.parametrize("k", [8, 32])
def test_c2_stencil_banded_and_blocked_spmm(spx, torch, c2_stencil, k):
    """The two SpMM variants the benchmark reports beside the default on the
    27-point stencil, in its launch configuration (FP64): the plan with a row
    period equal to the bandwidth (bitwise the default plan's Y) and the 2 x 1
    blocked SpMM in the same banded order, each against the oracle over every
    element (per-row bound and rel2)."""
    A, G = c2_stencil
    X = spgen.uniform(A.n * k, 11, spgen.TAG_X).reshape(A.n, k)
    Xd = dev(torch, X)
    bw = spx.bandwidth(G)
    assert bw == 128 * 128 + 128 + 1
    Y0 = spx.spmm(G, Xd, plan=spx.Plan.for_matrix(G, spx.default_opts(k)))
    Y1 = spx.spmm(G, Xd, plan=spx.Plan.for_matrix(G, spx.banded_opts(G, k)))
    assert torch.equal(Y0, Y1)
    del Y0
    check_f64(Y1.cpu().numpy(), A, X, f"C2 27-point banded k={k}")
    del Y1
    B = spx.BCSR.from_csr(G, 2, 1)
    Yb = spx.bcsr_spmm(B, Xd, row_period=bw).cpu().numpy()
    del B
    check_f64(Yb, A, X, f"C2 27-point 2x1 blocks banded k={k}")


def test_c1_row_shards(spx, torch, c1_matrix):
    """The headline matrix cut into the 8 row blocks balanced by nonzeros that
    the benchmark's shard form times: each block's SpMV and SpMM (k = 16)
    through its own default plan, against the full x and X; the blocks'
    results stacked are checked against the oracle over every element."""
    import bench
    A, G = c1_matrix
    cuts = bench.row_shards(A.rowptr, 8)
    x = spgen.uniform(A.n, 1)
    k = 16
    X = spgen.uniform(A.n * k, 2).reshape(A.n, k)
    xd, Xd = dev(torch, x), dev(torch, X)
    ys, Ys = [], []
    for g in range(8):
        S = bench.shard_of(torch, spx, G, cuts[g], cuts[g + 1])
        ys.append(spx.spmv(S, xd, plan=spx.Plan.for_matrix(S, spx.default_opts(1))).cpu().numpy())
        Ys.append(spx.spmm(S, Xd, plan=spx.Plan.for_matrix(S, spx.default_opts(k))).cpu().numpy())
    check_f64(np.concatenate(ys), A, x, "C1 SpMV, 8 row blocks")
    check_f64(np.concatenate(Ys), A, X, "C1 SpMM k=16, 8 row blocks")
