"""GPU parity of the HIP path against the FP64 oracle (through the C ABI).

Bars: integer/index work bit-exact; FP64 products rel2 <= 1e-12 (2-norm,
per column); exact-arithmetic inputs bit-exact under any summation order;
every plan variant (each lane width, split rows) deterministic run to run.
"""
import numpy as np
import pytest

import oracle
import spgen
from _cases import KINDS, int_valued, keep_stream, matrix, single_bin_opts, stream_mm_opts, to_gpu, two_bin_opts

pytestmark = pytest.mark.gpu

TOL_F64 = 1e-12


@pytest.fixture(scope="module")
def spx():
    import paper_1302_1078_amd as m
    return m


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def dev_vec(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    return t.to(dtype) if dtype is not None else t


def plan_variants(spx, A, k=1):
    """(name, plan) pairs: none, default (its stream bin served by row groups,
    as on any matrix this small, and kept as stream tiles), and one plan per
    lane width."""
    G = to_gpu(A)
    out = [("none", None), ("default", spx.Plan.for_matrix(G, spx.default_opts(k))),
           ("default-stream", spx.Plan.for_matrix(G, keep_stream(spx.default_opts(k))))]
    for lanes in (1, 2, 4, 8, 16, 32, 64, 256, 512):
        out.append((f"lanes{lanes}", spx.Plan.for_matrix(G, keep_stream(single_bin_opts(lanes, k)))))
    out.append(("sub-bins", spx.Plan.for_matrix(G, spx.PlanOpts.from_dict(
        {"nbins": 7, "upper": [1, 2, 4, 8, 16, 32], "lanes": [1, 2, 4, 8, 16, 32, 256],
         "max_k": k}))))
    out.append(("stream+split", spx.Plan.for_matrix(G, keep_stream(spx.PlanOpts.from_dict(
        {"nbins": 2, "upper": [40], "lanes": [512, 0], "split_chunk": 256, "max_k": k})))))
    out.append(("split", spx.Plan.for_matrix(G, single_bin_opts(0, k, chunk=256))))
    out.append(("lanes8+split", spx.Plan.for_matrix(G, two_bin_opts(300, 8, k, chunk=256))))
    return G, out


# ---------------------------------------------------------------- assembly and validation

@pytest.mark.parametrize("kind", ["powerlaw", "stencil27", "empty_rows", "tall", "wide"])
def test_from_coo_bit_exact(spx, torch, kind):
    A = matrix(kind, seed=1)
    coo = spgen.COO(A.m, A.n, A.row_of(), A.colind, A.values)
    # add duplicates of a random tenth of the entries, then shuffle
    rng = np.random.default_rng(3)
    d = rng.choice(A.nnz, A.nnz // 10, replace=False)
    coo = spgen.COO(A.m, A.n, np.concatenate([coo.r, coo.r[d]]), np.concatenate([coo.c, coo.c[d]]),
                    np.concatenate([coo.v, rng.uniform(-1, 1, d.size)]))
    coo = spgen.shuffled(coo, seed=5)
    ref = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    G = spx.from_coo(coo.m, coo.n, dev_vec(torch, coo.r), dev_vec(torch, coo.c), dev_vec(torch, coo.v))
    assert np.array_equal(G.rowptr.cpu().numpy(), ref.rowptr)
    assert np.array_equal(G.colind.cpu().numpy(), ref.colind)
    assert np.array_equal(G.values.cpu().numpy().view(np.uint64), ref.values.view(np.uint64))


def test_from_coo_edge_cases(spx, torch):
    e = lambda a, dt: dev_vec(torch, np.asarray(a, dtype=dt))  # noqa: E731
    G = spx.from_coo(4, 3, e([], np.int32), e([], np.int32), e([], np.float64))
    assert G.nnz == 0 and G.rowptr.cpu().tolist() == [0, 0, 0, 0, 0]
    G = spx.from_coo(1, 1, e([0, 0], np.int32), e([0, 0], np.int32), e([2.0, 3.0], np.float64))
    assert G.rowptr.cpu().tolist() == [0, 1] and G.values.cpu().tolist() == [5.0]
    # input-order duplicate sum: (1e16 + 1) - 1e16 = 0 in FP64
    G = spx.from_coo(1, 3, e([0, 0, 0], np.int32), e([2, 2, 2], np.int32), e([1e16, 1.0, -1e16], np.float64))
    assert G.values.cpu().tolist() == [0.0]
    with pytest.raises(ValueError):
        spx.from_coo(2, 2, e([0, 2], np.int32), e([0, 0], np.int32), e([1.0, 1.0], np.float64))


def test_validate_codes(spx, torch):
    A = matrix("powerlaw", 2)
    G = to_gpu(A)
    assert spx.validate(G) == 0
    rp = A.rowptr.copy()
    rp[-1] += 1
    assert spx.validate(spx.CSR(dev_vec(torch, rp), G.colind, G.values, G.shape)) != 0
    rp = A.rowptr.copy()
    rp[5], rp[6] = rp[6] + 3, rp[5]
    assert spx.validate(spx.CSR(dev_vec(torch, rp), G.colind, G.values, G.shape)) == 3
    ci = A.colind.copy()
    ci[7] = A.n
    assert spx.validate(spx.CSR(G.rowptr, dev_vec(torch, ci), G.values, G.shape)) == 2
    L = A.row_lengths()
    i = int(np.argmax(L))
    ci = A.colind.copy()
    ci[A.rowptr[i]], ci[A.rowptr[i] + 1] = ci[A.rowptr[i] + 1], ci[A.rowptr[i]]
    bad = spx.CSR(G.rowptr, dev_vec(torch, ci), G.values, G.shape)
    assert spx.validate(bad, check_sorted=True) == 1 and spx.validate(bad, check_sorted=False) == 0


# ---------------------------------------------------------------- plans

@pytest.mark.parametrize("kind", ["powerlaw", "stencil27", "empty_rows", "one_long_row"])
@pytest.mark.parametrize("which", ["spmv", "spmm16", "custom"])
def test_plan_bins_bit_exact(spx, kind, which):
    A = matrix(kind, seed=4)
    G = to_gpu(A)
    if which == "spmv":
        o = spx.default_opts(1)
    elif which == "spmm16":
        o = spx.default_opts(16)
    else:
        o = two_bin_opts(5, 4, chunk=300)
    plan = spx.Plan.for_matrix(G, o)
    perm, off = plan.export_bins()
    nb = o.nbins
    ref_perm, ref_off = oracle.bin_rows(A.rowptr, list(o.upper[:nb]))
    assert np.array_equal(perm, ref_perm) and np.array_equal(off, ref_off)
    info = plan.info()
    if o.lanes[nb - 1] == 0:
        rows = ref_perm[ref_off[nb - 1]:ref_off[nb]]
        L = A.row_lengths()[rows]
        assert info["split_rows"] == rows.size
        assert info["segments"] == int(np.maximum(1, -(-L // o.split_chunk)).sum())


# ---------------------------------------------------------------- SpMV FP64

@pytest.mark.parametrize("kind", KINDS)
def test_spmv_f64_parity_all_plans(spx, torch, kind):
    A = matrix(kind, seed=7)
    x = spgen.uniform(A.n, 11)
    ref = oracle.spmv(A, x)
    G, plans = plan_variants(spx, A)
    xd = dev_vec(torch, x)
    for name, plan in plans:
        y = spx.spmv(G, xd, plan=plan).cpu().numpy()
        assert oracle.rel2(y, ref) <= TOL_F64, (kind, name)
        # per-row bound: any summation order of L products, FMA or not
        bound = 2 * (A.row_lengths() + 2) * 2.0 ** -53 * oracle.spmv_abs(A, x)
        assert (np.abs(y - ref) <= bound).all(), (kind, name)
        empty = A.row_lengths() == 0
        assert not np.signbit(y[empty]).any()


@pytest.mark.parametrize("kind", KINDS)
def test_spmv_exact_inputs_bit_exact(spx, torch, kind):
    A = int_valued(matrix(kind, seed=8), seed=2)
    x = spgen.small_ints(A.n, 3)
    ref = oracle.spmv(A, x)
    G, plans = plan_variants(spx, A)
    xd = dev_vec(torch, x)
    for name, plan in plans:
        y = spx.spmv(G, xd, plan=plan).cpu().numpy()
        assert np.array_equal(y, ref), (kind, name)


def gapped_matrix(gap: str, m: int = 3001, n: int = 500):
    """Rows of length 20 (even rows) separated by rows outside the stream bin:
    'empty' gaps keep the nonzeros of the length-20 rows one contiguous run,
    'short' gaps (length 2) break every tile's run, 'mixed' keeps the first
    half contiguous and breaks the second half in a few places only."""
    rng = np.random.default_rng(31)
    L = np.zeros(m, dtype=np.int64)
    L[0::2] = 20
    if gap == "short":
        L[1::2] = 2
    elif gap == "mixed":
        odd = np.arange(1, m, 2)
        L[odd[(odd > m // 2) & (odd % 194 == 1)]] = 2
    rowptr = np.zeros(m + 1, dtype=np.int32)
    rowptr[1:] = np.cumsum(L)
    colind = np.concatenate([np.sort(rng.choice(n, int(l), replace=False)) for l in L]).astype(np.int32)
    A = oracle.CSR(m, n, rowptr, colind, np.zeros(len(colind)))
    return int_valued(A, seed=5)


@pytest.mark.parametrize("gap", ["empty", "short", "mixed"])
@pytest.mark.parametrize("vname", ["f64", "f32"])
def test_stream_tiles_contiguous_or_not(spx, torch, gap, vname):
    """A stream tile whose rows form one contiguous run of nonzeros takes an
    element's position directly; any other tile searches for its row.  Both
    kinds of tile, and a matrix holding both, give the oracle's exact sums
    (small-integer inputs, stream bin for rows longer than 2)."""
    A = gapped_matrix(gap)
    x = spgen.small_ints(A.n, 4)
    ref = oracle.spmv(A, x)
    vt = torch.float64 if vname == "f64" else torch.float32
    G = to_gpu(A, vt)
    opts = keep_stream(spx.PlanOpts.from_dict({"nbins": 2, "upper": [2], "lanes": [1, 512], "max_k": 1}))
    plan = spx.Plan.for_matrix(G, opts)
    y = spx.spmv(G, dev_vec(torch, x, vt), plan=plan).double().cpu().numpy()
    assert np.array_equal(y, ref), (gap, vname)


def test_spmv_identity_permutation_laplacian(spx, torch):
    n = 5000
    x = spgen.uniform(n, 1)
    perm = np.random.default_rng(0).permutation(n)
    P = oracle.csr_from_coo(n, n, np.arange(n), perm, np.ones(n))
    G = to_gpu(P)
    y = spx.spmv(G, dev_vec(torch, x), plan=spx.Plan.for_matrix(G)).cpu().numpy()
    assert np.array_equal(y, x[perm])
    coo = spgen.stencil3d(20, 20, 20, 27, values="laplacian")
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    G = to_gpu(A)
    y = spx.spmv(G, dev_vec(torch, np.ones(A.n)), plan=spx.Plan.for_matrix(G)).cpu().numpy()
    assert np.array_equal(y, 26.0 - (A.row_lengths() - 1))


def test_spmv_deterministic(spx, torch):
    A = matrix("powerlaw_sq", seed=9)
    G = to_gpu(A)
    xd = dev_vec(torch, spgen.uniform(A.n, 2))
    for o in (spx.default_opts(1), keep_stream(spx.default_opts(1)), single_bin_opts(0, chunk=256)):
        plan = spx.Plan.for_matrix(G, o)
        ys = [spx.spmv(G, xd, plan=plan).cpu().numpy().view(np.uint64) for _ in range(4)]
        assert all(np.array_equal(ys[0], y) for y in ys[1:])


def test_degenerate_shapes(spx, torch):
    # m == 0: no-op; n == 0 / nnz == 0: y = +0
    Z = oracle.csr_from_coo(0, 5, [], [], [])
    G = to_gpu(Z)
    y = spx.spmv(G, dev_vec(torch, np.ones(5)))
    assert y.numel() == 0
    E = oracle.csr_from_coo(7, 0, [], [], [])
    G = to_gpu(E)
    for plan in (None, spx.Plan.for_matrix(G)):
        y = torch.full((7,), float("nan"), dtype=torch.float64, device="cuda:0")
        spx.spmv(G, torch.empty(0, dtype=torch.float64, device="cuda:0"), y=y, plan=plan)
        yc = y.cpu().numpy()
        assert (yc == 0).all() and not np.signbit(yc).any()
        Y = torch.full((7, 4), float("nan"), dtype=torch.float64, device="cuda:0")
        spx.spmm(G, torch.empty((0, 4), dtype=torch.float64, device="cuda:0"), Y=Y, plan=None)
        assert (Y.cpu().numpy() == 0).all()


def test_argument_errors(spx, torch):
    A = matrix("uniform", 1)
    G = to_gpu(A)
    x = dev_vec(torch, np.ones(A.n))
    with pytest.raises(spx.SpxError):
        spx.spmv(G, x.float())  # (F64 values, F32 vectors) is not a supported pair
    with pytest.raises(spx.SpxError):
        spx.spmm(G, torch.ones((A.n, 0), dtype=torch.float64, device="cuda:0"))
    other = spx.Plan.for_matrix(to_gpu(matrix("stencil5", 1)))
    with pytest.raises(spx.SpxError):
        spx.spmv(G, x, plan=other)
    plan16 = spx.Plan.for_matrix(G, single_bin_opts(0, k=4, chunk=256))
    with pytest.raises(spx.SpxError):
        spx.spmm(G, torch.ones((A.n, 8), dtype=torch.float64, device="cuda:0"), plan=plan16)


# ---------------------------------------------------------------- SpMM FP64

@pytest.mark.parametrize("kind", ["powerlaw", "stencil27", "empty_rows", "one_long_row", "wide"])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 8, 16, 32, 40, 100])
def test_spmm_f64_parity(spx, torch, kind, k):
    A = matrix(kind, seed=12)
    X = spgen.uniform(A.n * k, 13).reshape(A.n, k)
    ref = oracle.spmm(A, X)
    G = to_gpu(A)
    plans = [None, spx.Plan.for_matrix(G, spx.default_opts(k)),
             spx.Plan.for_matrix(G, two_bin_opts(64, 64, k, chunk=256)),
             spx.Plan.for_matrix(G, stream_mm_opts(k))]
    for ld_pad in (0, 3):
        Xd = torch.zeros((A.n, k + ld_pad), dtype=torch.float64, device="cuda:0")
        Xd[:, :k] = dev_vec(torch, X)
        Xv = Xd[:, :k]
        for plan in plans:
            Yd = torch.full((A.m, k + ld_pad), 7.0, dtype=torch.float64, device="cuda:0")
            spx.spmm(G, Xv, Y=Yd[:, :k], plan=plan)
            Y = Yd.cpu().numpy()
            for j in range(k):
                assert oracle.rel2(Y[:, j], ref[:, j]) <= TOL_F64, (kind, k, ld_pad, j)
            if ld_pad:
                assert (Y[:, k:] == 7.0).all()  # padding untouched


@pytest.mark.parametrize("k", [4, 16])
def test_spmm_exact_inputs_bit_exact(spx, torch, k):
    A = int_valued(matrix("powerlaw", 5), 1)
    X = spgen.small_ints(A.n * k, 6).reshape(A.n, k)
    ref = oracle.spmm(A, X)
    G = to_gpu(A)
    for plan in (None, spx.Plan.for_matrix(G, spx.default_opts(k)),
                 spx.Plan.for_matrix(G, single_bin_opts(0, k, chunk=256)),
                 spx.Plan.for_matrix(G, stream_mm_opts(k))):
        Y = spx.spmm(G, dev_vec(torch, X), plan=plan).cpu().numpy()
        assert np.array_equal(Y, ref)


def test_spmm_k1_equals_spmv_bitwise(spx, torch):
    A = matrix("powerlaw_sq", 3)
    G = to_gpu(A)
    x = spgen.uniform(A.n, 4)
    plan = spx.Plan.for_matrix(G, spx.default_opts(1))
    y = spx.spmv(G, dev_vec(torch, x), plan=plan).cpu().numpy()
    Y = spx.spmm(G, dev_vec(torch, x.reshape(-1, 1)), plan=plan).cpu().numpy()
    assert np.array_equal(y.view(np.uint64), Y[:, 0].view(np.uint64))


def test_spmm_deterministic_split(spx, torch):
    A = matrix("one_long_row", 3)
    G = to_gpu(A)
    X = dev_vec(torch, spgen.uniform(A.n * 16, 4).reshape(A.n, 16))
    plan = spx.Plan.for_matrix(G, spx.default_opts(16))
    assert plan.info()["segments"] > 1
    Ys = [spx.spmm(G, X, plan=plan).cpu().numpy().view(np.uint64) for _ in range(4)]
    assert all(np.array_equal(Ys[0], Y) for Y in Ys[1:])


@pytest.mark.parametrize("per_row", [1, 7, 31, 32])
@pytest.mark.parametrize("k", [2, 3, 8, 16, 100])
def test_spmm_equal_rows_stream_plan(spx, torch, per_row, k):
    """SpMM through a plan whose short-row bin is a stream bin (served by row
    groups of KL lanes when k > 1): rows of one length, so every slot count
    ends in a masked partial round at some row; a ragged last tile; bit-exact
    on integer inputs and within the FP64 bar on uniform ones."""
    coo = spgen.uniform_rows(1000, 700, per_row, 31)
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    G = to_gpu(A)
    plan = spx.Plan.for_matrix(G, stream_mm_opts(k))
    _, off = plan.export_bins()
    assert off[1] - off[0] == A.m  # every row in the short-row bin
    X = spgen.uniform(A.n * k, 32).reshape(A.n, k)
    Y = spx.spmm(G, dev_vec(torch, X), plan=plan).cpu().numpy()
    ref = oracle.spmm(A, X)
    for j in range(k):
        assert oracle.rel2(Y[:, j], ref[:, j]) <= TOL_F64, (per_row, k, j)
    Ai = int_valued(A, 33)
    Gi = to_gpu(Ai)
    Xi = spgen.small_ints(A.n * k, 34).reshape(A.n, k)
    Yi = spx.spmm(Gi, dev_vec(torch, Xi), plan=spx.Plan.for_matrix(Gi, stream_mm_opts(k))).cpu().numpy()
    assert np.array_equal(Yi, oracle.spmm(Ai, Xi))


def test_spmm_stream_deterministic_and_empty_rows(spx, torch):
    A = matrix("empty_rows", 7)
    G = to_gpu(A)
    k = 16
    X = dev_vec(torch, spgen.uniform(A.n * k, 8).reshape(A.n, k))
    plan = spx.Plan.for_matrix(G, stream_mm_opts(k))
    Y0 = torch.full((A.m, k), float("nan"), dtype=torch.float64, device="cuda:0")
    spx.spmm(G, X, Y=Y0, plan=plan)
    ref = oracle.spmm(A, X.cpu().numpy())
    Yn = Y0.cpu().numpy()
    assert np.isfinite(Yn).all()  # empty rows written as zeros
    assert (Yn[A.row_lengths() == 0] == 0.0).all()
    for j in range(k):
        assert oracle.rel2(Yn[:, j], ref[:, j]) <= TOL_F64
    Ys = [spx.spmm(G, X, plan=plan).cpu().numpy().view(np.uint64) for _ in range(4)]
    assert all(np.array_equal(Ys[0], y) for y in Ys[1:])


@pytest.mark.parametrize("k", [1, 16])
def test_occupancy_cap_same_result(spx, torch, k):
    """The occupancy cap (LDS padding) changes scheduling only: results are
    bitwise those of the uncapped launch."""
    A = matrix("powerlaw_sq", 9)
    G = to_gpu(A)
    X = spgen.uniform(A.n * k, 10).reshape(A.n, k)
    Xd = dev_vec(torch, X if k > 1 else X[:, 0])
    outs = []
    for occ in (0, 1, 2, 4, 8):
        o = spx.default_opts(k)
        o.occupancy = occ
        plan = spx.Plan.for_matrix(G, o)
        Y = (spx.spmm(G, Xd, plan=plan) if k > 1 else spx.spmv(G, Xd, plan=plan)).cpu().numpy()
        outs.append(Y.view(np.uint64))
    assert all(np.array_equal(outs[0], y) for y in outs[1:])
    ref = oracle.spmm(A, X) if k > 1 else oracle.spmv(A, X[:, 0])
    assert oracle.rel2(outs[0].view(np.float64).ravel(), ref.ravel()) <= TOL_F64


def test_memory_probes_run_and_keep_data(spx, torch):
    """Every probe kind launches and finishes; the read-only kinds leave the
    buffer unchanged, write / copy / flush change it as documented."""
    a = torch.arange(1 << 16, dtype=torch.float64, device="cuda:0")
    keep = a.clone()
    sink = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    for kind in ("read", "gather_rows", "gather_elems"):
        spx.probe(kind, a, sink, 64)
    torch.cuda.synchronize()
    assert torch.equal(a, keep)
    b = torch.empty_like(a)
    spx.probe("copy", a, b, 64)
    assert torch.equal(a, b)
    spx.probe("flush", b, None, 64)
    assert torch.equal(b, a + 1.0)
    spx.probe("write", b, None, 64)
    assert torch.equal(b, torch.ones_like(b))
    with pytest.raises(spx.SpxError):
        spx.probe("gather_rows", a[:8], None, 64)


@pytest.mark.parametrize("nidx", [0, 1, 999, 70_001])
def test_index_gather_probe_sums(spx, torch, nidx):
    """The index-gather probe reads exactly idx (and x[idx]) once each: the
    per-workgroup sums match the host's over the same contiguous ranges
    (exact for the index stream; FP64 rounding for the gather)."""
    from paper_1302_1078_amd.ops import probe_index_gather
    n = 5_000
    rng = np.random.default_rng(nidx)
    idx = rng.integers(0, n, nidx).astype(np.int32)
    x = spgen.uniform(n, 3)
    blocks = 64
    per = -(-nidx // blocks) if nidx else 0
    want_i = np.array([idx[t * per:(t + 1) * per].astype(np.float64).sum() for t in range(blocks)])
    want_x = np.array([x[idx[t * per:(t + 1) * per]].sum() for t in range(blocks)])
    idx_d, x_d = dev_vec(torch, idx), dev_vec(torch, x)
    got_i = probe_index_gather(idx_d, x_d, gather=False, blocks=blocks).cpu().numpy()
    got_x = probe_index_gather(idx_d, x_d, gather=True, blocks=blocks).cpu().numpy()
    assert np.array_equal(got_i, want_i)
    assert np.allclose(got_x, want_x, rtol=1e-12, atol=1e-12)
    with pytest.raises(spx.SpxError):
        probe_index_gather(idx_d, x_d, blocks=12)  # not a multiple of 8


def test_chase_probe_follows_the_cycle(spx, torch):
    """The chase probe's 64 lanes end where the host walk of the same cycle
    ends, from one shared start and from 64 distinct starts."""
    from paper_1302_1078_amd.ops import chase_cycle, probe_chase
    n, hops = 1 << 12, 1_000
    nxt = chase_cycle(n, "cuda:0", seed=5, stride=4)
    h = nxt.cpu().numpy()
    seen, i = 1, int(h[0])
    while i != 0:  # one cycle through every 4th slot
        assert i % 4 == 0
        i, seen = int(h[i]), seen + 1
    assert seen == n // 4
    for starts in (np.zeros(64, np.int32), (np.arange(64) * 61).astype(np.int32)):
        want = starts.copy()
        for _ in range(hops):
            want = h[want]
        out = probe_chase(nxt, dev_vec(torch, starts), hops).cpu().numpy()
        assert np.array_equal(out, want)
    with pytest.raises(spx.SpxError):
        probe_chase(nxt[:1000], dev_vec(torch, np.zeros(64, np.int32)), 10)  # n not a power of two


@pytest.mark.parametrize("k", [1, 16])
def test_nan_inf_stay_in_their_rows(spx, torch, k):
    """IEEE propagation: a NaN value poisons only its own row; an infinite x
    entry reaches exactly the rows that reference its column (Inf, or NaN
    where +Inf and -Inf meet); every other row stays exact.  Checked for each
    plan variant, including stream bins whose spare slots reload elements."""
    A = int_valued(matrix("powerlaw", 31), 32)
    vals = A.values.copy()
    bad_row = int(np.argmax(np.diff(A.rowptr) == 5))
    vals[A.rowptr[bad_row] + 2] = np.nan
    A2 = oracle.CSR(A.m, A.n, A.rowptr, A.colind, vals)
    X = spgen.small_ints(A.n * k, 33).reshape(A.n, k)
    hot = int(np.bincount(A.colind, minlength=A.n).argmax())
    X[hot, :] = np.inf
    ref = oracle.spmm(A2, X)
    G = to_gpu(A2)
    _, plans = plan_variants(spx, A2, k)
    for name, plan in plans:
        Xd = dev_vec(torch, X if k > 1 else X[:, 0])
        Y = spx.spmm(G, Xd, plan=plan) if k > 1 else spx.spmv(G, Xd, plan=plan)
        Y = Y.cpu().numpy().reshape(A.m, k)
        assert np.array_equal(Y, ref, equal_nan=True), name


def test_products_graph_replay(spx, torch):
    """Single products captured in one HIP graph (SpMV with split rows, SpMM,
    values to CSC order, the CSC transpose, the sampled dot) give on every
    replay, with new inputs written eagerly between replays, bitwise the
    results of the same calls made eagerly."""
    from paper_1302_1078_amd.ops import CSCIndex
    A = matrix("one_long_row", 41)
    G = to_gpu(A)
    dev = "cuda:0"
    k = 16
    plan_v = spx.Plan.for_matrix(G, spx.default_opts(1))
    assert plan_v.info()["segments"] > 1  # the 50,000-entry row is cut into split segments
    plan_m = spx.Plan.for_matrix(G, spx.default_opts(k))
    idx = spx.transpose_index(G)
    vmap = spx.csc_value_map(idx)
    nop = CSCIndex(idx.colptr, idx.rowind, None)
    plan_t = spx.Plan(idx.colptr, A.n, A.m, A.nnz, spx.default_opts(1))
    x = torch.empty(A.n, dtype=torch.float64, device=dev)
    X = torch.empty((A.n, k), dtype=torch.float64, device=dev)
    dy = torch.empty(A.m, dtype=torch.float64, device=dev)
    y = torch.empty(A.m, dtype=torch.float64, device=dev)
    Y = torch.empty((A.m, k), dtype=torch.float64, device=dev)
    stage = torch.empty_like(G.values)
    vcsc = torch.empty_like(G.values)
    dx = torch.empty(A.n, dtype=torch.float64, device=dev)
    dv = torch.empty(A.nnz, dtype=torch.float64, device=dev)
    Gc = G.with_values(vcsc)

    def calls():
        spx.spmv(G, x, y=y, plan=plan_v)
        spx.spmm(G, X, Y=Y, plan=plan_m)
        spx.values_to_csc(G.values, vmap, staging=stage, out=vcsc)
        spx.spmv_t(Gc, dy, mode=0, index=nop, plan=plan_t, out=dx)
        spx.sddmm(G, dy, x, out=dv)

    outs = (y, Y, vcsc, dx, dv)
    for t_ in (x, X, dy):
        t_.uniform_(-1.0, 1.0)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        calls()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        calls()
    for rep in range(3):
        for t_ in (x, X, dy):
            t_.uniform_(-1.0, 1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [t_.clone() for t_ in outs]
        calls()
        torch.cuda.synchronize()
        for name, a, b in zip(("spmv", "spmm", "values_to_csc", "spmv_t", "sddmm"), got, outs):
            assert torch.equal(a, b), (rep, name)
    ref = oracle.spmv(A, x.cpu().numpy())
    assert oracle.rel2(y.cpu().numpy(), ref) <= TOL_F64
