"""Batched launches: each matrix's result must be bit-identical to the
single-matrix launch with the same plan options (identical per-row
arithmetic), within the FP bound of the oracle, and stable under HIP-graph
replay."""
import numpy as np
import pytest

import oracle
import spgen
from _cases import gamma, keep_stream, single_bin_opts, two_bin_opts

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


def build_set(torch, dtype, count=24, seed=0, rmax=30_000):
    specs = spgen.batch_specs(count, seed=seed, rmin=500, rmax=rmax)
    mats, Xs, refs = [], [], []
    for i, s in enumerate(specs):
        coo = spgen.batch_matrix(s, seed, i)
        A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
        X = spgen.uniform(A.n * s.k, 100 + i).reshape(A.n, s.k)
        if dtype == torch.float32:
            vals, Xq = spgen.to_f32(A.values), spgen.to_f32(X)
        else:
            vals, Xq = A.values, X
        import paper_1302_1078_amd as spx
        G = spx.CSR(dev(torch, A.rowptr), dev(torch, A.colind), dev(torch, vals), (A.m, A.n))
        Xd = dev(torch, Xq[:, 0] if s.k == 1 else Xq)
        mats.append(G)
        Xs.append(Xd)
        refs.append((oracle.CSR(A.m, A.n, A.rowptr, A.colind, vals.astype(np.float64)), Xq.astype(np.float64)))
    return specs, mats, Xs, refs


def single(spx, A, X, opts):
    plan = spx.Plan.for_matrix(A, opts)
    return spx.spmv(A, X, plan=plan) if X.dim() == 1 else spx.spmm(A, X, plan=plan)


@pytest.mark.parametrize("dtype_name", ["f32", "f64"])
def test_batch_bit_identical_to_single(spx, torch, dtype_name):
    from paper_1302_1078_amd.batch import Batched
    dtype = torch.float32 if dtype_name == "f32" else torch.float64
    specs, mats, Xs, refs = build_set(torch, dtype)
    opts = []
    for i, (A, X) in enumerate(zip(mats, Xs)):
        k = 1 if X.dim() == 1 else X.shape[1]
        if i % 3 == 0:
            opts.append(spx.default_opts(k, dtype))
        elif i % 3 == 1:
            opts.append(two_bin_opts(40, 16, k, chunk=256))
        else:
            opts.append(single_bin_opts(0 if i % 2 else 64, k, chunk=512))
    B = Batched(mats, Xs, opts=opts)
    Ys = B.run()
    info = B.info()
    assert info["tiles"] > 0 and info["grid"] > 0
    for i, (A, X) in enumerate(zip(mats, Xs)):
        # the batch keeps stream bins as stream tiles whatever the matrix size
        want = single(spx, A, X, keep_stream(spx.PlanOpts.from_dict(opts[i].to_dict()))).cpu().numpy()
        got = Ys[i].cpu().numpy()
        u = np.uint32 if dtype == torch.float32 else np.uint64
        assert np.array_equal(got.view(u), want.view(u)), (i, specs[i])
        Ar, Xr = refs[i]
        ref = oracle.spmm(Ar, Xr.reshape(Ar.n, -1))
        S = oracle.spmm(oracle.CSR(Ar.m, Ar.n, Ar.rowptr, Ar.colind, np.abs(Ar.values)), np.abs(Xr.reshape(Ar.n, -1)))
        u_ = 2.0 ** -24 if dtype == torch.float32 else 2.0 ** -53
        L = Ar.row_lengths()[:, None]
        assert (np.abs(got.reshape(ref.shape) - ref) <= gamma(L + 8, u_) * S + 1e-300).all(), i


def test_batch_graph_replay(spx, torch):
    from paper_1302_1078_amd.batch import Batched
    specs, mats, Xs, refs = build_set(torch, torch.float32, count=16, seed=3)
    B = Batched(mats, Xs)
    g = B.capture()
    for rep in range(3):
        for X in Xs:  # eager work between replays: new right-hand sides
            X.uniform_(-1.0, 1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [Y.clone() for Y in B.Ys]
        B.run()  # eager result for the same inputs
        torch.cuda.synchronize()
        for i in range(len(mats)):
            assert torch.equal(got[i], B.Ys[i]), (rep, i)


def test_batch_rejects_mixed_dtypes(spx, torch):
    from paper_1302_1078_amd.batch import Batched
    specs, mats, Xs, _ = build_set(torch, torch.float32, count=2, seed=5)
    A64 = spx.CSR(mats[1].rowptr, mats[1].colind, mats[1].values.double(), mats[1].shape)
    with pytest.raises(spx.SpxError):
        Batched([mats[0], A64], [Xs[0], Xs[1].double()])


def test_autotune_choice_is_correct_and_cached(spx, torch, tmp_path):
    from paper_1302_1078_amd import autotune
    coo = spgen.powerlaw(40_000, 40_000, 2.2, 8_000, 20.0, seed=2)
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    G = spx.CSR(dev(torch, A.rowptr), dev(torch, A.colind), dev(torch, A.values), (A.m, A.n))
    for k in (1, 16):
        X = spgen.uniform(A.n * k, 9).reshape(A.n, k)
        Xd = dev(torch, X[:, 0] if k == 1 else X)
        cache = str(tmp_path / "tune.json")
        o, rep = autotune.tune(G, Xd, reps=3, cache_path=cache)
        assert not rep["cached"] and len(rep["all_ms"]) == len(autotune.candidates(k))
        o2, rep2 = autotune.tune(G, Xd, reps=3, cache_path=cache)
        assert rep2["cached"] and o2.to_dict() == o.to_dict()
        Y = single(spx, G, Xd, o).cpu().numpy().reshape(A.m, k)
        ref = oracle.spmm(A, X)
        for j in range(k):
            assert oracle.rel2(Y[:, j], ref[:, j]) <= 1e-12
    with open(cache, "w") as f:
        f.write("{not json")
    o3, rep3 = autotune.tune(G, Xd, reps=2, cache_path=cache)  # corrupt cache: tuned again
    assert not rep3["cached"]


def test_tune_batch_options_and_time_in_batch(spx, torch):
    """tune_batch on a mixed batch: one option set per matrix, each a default
    or that matrix's own pick; the batch through them is bitwise equal to the
    single launches with the same options; time_in_batch gives a positive
    time per copy, also for a matrix too small to fill the chip alone."""
    from paper_1302_1078_amd import autotune
    from paper_1302_1078_amd.batch import Batched
    specs, mats, Xs, refs = build_set(torch, torch.float32, count=12, seed=7)
    opts, rep = autotune.tune_batch(mats, Xs, reps=2, rounds=1)
    assert len(opts) == len(mats)
    assert set(rep["groups"]) <= {1, 4, 16}
    assert 0 <= rep["accepted_matrices"] <= rep["changed_per_matrix"] <= len(mats)
    B = Batched(mats, Xs, opts=opts)
    Ys = B.run()
    for i, (A, X) in enumerate(zip(mats, Xs)):
        want = single(spx, A, X, keep_stream(spx.PlanOpts.from_dict(opts[i].to_dict())))
        assert torch.equal(Ys[i].view(torch.int32), want.view(torch.int32)), i
    small = min(range(len(mats)), key=lambda i: mats[i].nnz)
    k = 1 if Xs[small].dim() == 1 else Xs[small].shape[1]
    t = autotune.time_in_batch(mats[small], Xs[small], spx.default_opts(k, torch.float32), reps=2)
    assert t > 0
