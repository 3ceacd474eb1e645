"""Seeded random configurations against the oracle: plan options (bins,
thresholds, lane widths, stream and split bins, split chunk, compensation
threshold, flags, row period), SpMM width, value type and matrix kind are drawn from a
fixed seed per case, so every run checks the same combinations (60
products, 24 backward cases, 8 batches).  Each
product must meet the per-row error bound: FP64 2(L + 2) 2^-53 sum |a x|;
FP32 / BF16 the precision-form bounds against the quantised inputs."""
import numpy as np
import pytest

import oracle
import spgen
from _cases import check_bound, matrix, quantised

pytestmark = pytest.mark.gpu

LANES = [1, 2, 4, 8, 16, 32, 64, 256, 512]
FLAGS = [1, 2, 4, 8, 16]  # NO_NT_STORE, SCALAR_X, NO_XCD_MAP, ONE_ROW, KEEP_STREAM
KINDS = ["powerlaw", "stencil27", "stencil5", "empty_rows", "one_long_row", "tall", "wide", "uniform"]


@pytest.fixture(scope="module")
def spx():
    import paper_1302_1078_amd as m
    return m


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def random_opts(spx, rng, k):
    nb = int(rng.integers(1, 7))
    upper = sorted(rng.choice(np.arange(1, 3000), nb - 1, replace=False).tolist())
    lanes = [int(rng.choice(LANES)) for _ in range(nb)]
    if nb > 1 and rng.random() < 0.6:
        lanes[-1] = 0  # split bin
    flags = 0
    for f in FLAGS:
        if rng.random() < 0.25:
            flags |= f
    return spx.PlanOpts.from_dict({
        "nbins": nb, "upper": upper, "lanes": lanes,
        "split_chunk": int(rng.choice([256, 300, 1024, 4096])),
        "kahan_len": int(rng.choice([4, 64, 256, 100000])),
        "max_k": k, "flags": flags,
        "row_period": int(rng.choice([0, 0, 0, 1, 7, 100, 5000]))})


@pytest.mark.parametrize("case", range(60))
def test_random_configuration(spx, torch, case):
    rng = np.random.default_rng(1000 + case)
    kind = KINDS[int(rng.integers(len(KINDS)))]
    A = matrix(kind, seed=int(rng.integers(1 << 16)))
    k = int(rng.choice([1, 1, 2, 3, 4, 8, 16, 33]))
    vname = str(rng.choice(["f64", "f32", "bf16"]))
    opts = random_opts(spx, rng, k)
    X = spgen.uniform(A.n * k, int(rng.integers(1 << 16))).reshape(A.n, k)
    what = (case, kind, k, vname, opts.to_dict())
    if vname == "f64":
        G = spx.CSR(*(torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
                      for a in (A.rowptr, A.colind, A.values)), (A.m, A.n))
        Xd = torch.from_numpy(X).to("cuda:0")
        wideA, Xw = A, X
    else:
        G, wideA = quantised(A, vname, torch)
        Xw = spgen.to_f32(X).astype(np.float64)
        Xd = torch.from_numpy(spgen.to_f32(X)).to("cuda:0")
    plan = spx.Plan.for_matrix(G, opts)
    if k == 1:
        y = spx.spmv(G, Xd[:, 0].contiguous(), plan=plan).double().cpu().numpy()[:, None]
    else:
        y = spx.spmm(G, Xd, plan=plan).double().cpu().numpy()
    L = A.row_lengths()
    absA = oracle.CSR(A.m, A.n, A.rowptr, A.colind, np.abs(wideA.values))
    for j in range(k):
        ref = oracle.spmv(wideA, Xw[:, j])
        S = oracle.spmv(absA, np.abs(Xw[:, j]))
        if vname == "f64":
            assert (np.abs(y[:, j] - ref) <= 2.0 * (L + 2.0) * 2.0 ** -53 * S).all(), (what, j)
        else:
            check_bound(y[:, j], ref, S, L, opts.kahan_len, (what, j))


@pytest.mark.parametrize("case", range(24))
def test_random_backward(spx, torch, case):
    """A^T dY by the three transpose paths and the sampled dot, random plans
    and widths: FP64 within 2(L + 2) 2^-53 sum |a dy| per column (L = column
    length); the CSC-values path bitwise equal to the path through perm."""
    from paper_1302_1078_amd.ops import CSCIndex
    rng = np.random.default_rng(5000 + case)
    kind = KINDS[int(rng.integers(len(KINDS)))]
    A = matrix(kind, seed=int(rng.integers(1 << 16)))
    k = int(rng.choice([1, 1, 2, 3, 8]))
    G = spx.CSR(*(torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
                  for a in (A.rowptr, A.colind, A.values)), (A.m, A.n))
    dY = spgen.normal(A.m * k, int(rng.integers(1 << 16))).reshape(A.m, k)
    X = spgen.uniform(A.n * k, int(rng.integers(1 << 16))).reshape(A.n, k)
    dYd = torch.from_numpy(dY if k > 1 else dY[:, 0].copy()).to("cuda:0")
    Xd = torch.from_numpy(X if k > 1 else X[:, 0].copy()).to("cuda:0")
    idx = spx.transpose_index(G)
    plan_t = spx.Plan(idx.colptr, A.n, A.m, A.nnz, random_opts(spx, rng, k))
    plan = spx.Plan.for_matrix(G, random_opts(spx, rng, k))
    vcsc = spx.values_to_csc(G.values, spx.csc_value_map(idx))
    d_perm = spx.spmv_t(G, dYd, mode=0, index=idx, plan=plan_t).cpu().numpy().reshape(A.n, k)
    d_csc = spx.spmv_t(G.with_values(vcsc), dYd, mode=0, index=CSCIndex(idx.colptr, idx.rowind, None),
                       plan=plan_t).cpu().numpy().reshape(A.n, k)
    d_atom = spx.spmv_t(G, dYd, mode=1, plan=plan).cpu().numpy().reshape(A.n, k)
    assert np.array_equal(d_perm.view(np.uint64), d_csc.view(np.uint64)), case
    Lc = np.bincount(A.colind, minlength=A.n).astype(np.float64)
    absA = oracle.CSR(A.m, A.n, A.rowptr, A.colind, np.abs(A.values))
    ref = oracle.spmv_t(A, dY)
    S = oracle.spmv_t(absA, np.abs(dY))
    for d in (d_perm, d_atom):
        assert (np.abs(d - ref) <= 2.0 * (Lc[:, None] + 2.0) * 2.0 ** -53 * S).all(), case
    dv = spx.sddmm(G, dYd, Xd, plan=plan).cpu().numpy()
    dv_ref = oracle.sddmm(A, dY, X)
    assert (np.abs(dv - dv_ref) <= (k + 1) * 2.0 ** -53 * oracle.sddmm(A, np.abs(dY), np.abs(X))).all(), case


@pytest.mark.parametrize("case", range(8))
def test_random_batch(spx, torch, case):
    """A batch of random matrices, widths and plans: every result bitwise
    equal to its single launch with stream bins kept as tiles."""
    from paper_1302_1078_amd._lib import SPX_FLAG_KEEP_STREAM
    from paper_1302_1078_amd.batch import Batched
    rng = np.random.default_rng(9000 + case)
    dt = torch.float32 if rng.random() < 0.5 else torch.float64
    mats, Xs, opts = [], [], []
    for i in range(int(rng.integers(1, 12))):
        A = matrix(KINDS[int(rng.integers(len(KINDS)))], seed=int(rng.integers(1 << 16)))
        k = int(rng.choice([1, 1, 4, 16]))
        G = spx.CSR(*(torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
                      for a in (A.rowptr, A.colind, A.values)), (A.m, A.n))
        X = torch.from_numpy(spgen.uniform(A.n * k, int(rng.integers(1 << 16))).reshape(A.n, k)).to("cuda:0")
        mats.append(G.with_values(G.values.to(dt)))
        Xs.append((X[:, 0].contiguous() if k == 1 else X).to(dt))
        o = random_opts(spx, rng, k)
        o.flags &= ~2  # the batch serves only the vector X layouts
        opts.append(o)
    B = Batched(mats, Xs, opts=opts)
    Ys = [Y.clone() for Y in B.run()]
    for G, X, o, Y in zip(mats, Xs, opts, Ys):
        ko = spx.PlanOpts.from_dict(o.to_dict())
        ko.flags |= SPX_FLAG_KEEP_STREAM
        p = spx.Plan.for_matrix(G, ko)
        want = spx.spmv(G, X, plan=p) if X.dim() == 1 else spx.spmm(G, X, plan=p)
        assert torch.equal(want, Y), case
