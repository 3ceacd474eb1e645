"""GPU parity of the staged SpMM (each row tile's X window copied into LDS)
against the FP64 oracle, through the C ABI.

Bars: FP64 per-row bound 2(L + 2) 2^-53 sum_p |a_p x_p| and rel2 <= 1e-12;
exact-arithmetic inputs bit-exact; FP32 / BF16 per-row bounds against the
oracle on the quantised inputs; tiles that fall back to direct gathers (too
many nonzeros, or a window above the LDS budget) within the same bars."""
import numpy as np
import pytest

import oracle
import spgen
from _cases import KINDS, U32, check_bound, int_valued, matrix, quantised, to_gpu

pytestmark = pytest.mark.gpu

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


def product(spx, G, Xd, plan):
    return spx.spmv(G, Xd[:, 0].contiguous(), plan=plan) if Xd.shape[1] == 1 else spx.spmm(G, Xd, plan=plan)


def check_f64(y, A, X, what):
    L = A.row_lengths().astype(np.float64)
    absA = oracle.CSR(A.m, A.n, A.rowptr, A.colind, np.abs(A.values))
    ref = oracle.spmm(A, X)
    S = oracle.spmm(absA, np.abs(X))
    assert (np.abs(y - ref) <= 2.0 * (L[:, None] + 2.0) * U64 * S).all(), what
    for j in range(X.shape[1]):
        assert oracle.rel2(y[:, j], ref[:, j]) <= 1e-12, (what, j)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("k", [2, 4, 8, 16, 32, 100])
def test_staged_f64_parity(spx, torch, kind, k):
    A = matrix(kind, seed=5)
    G = to_gpu(A)
    X = spgen.uniform(A.n * k, 6).reshape(A.n, k)
    plan = spx.Plan.staged(G, k)
    info = plan.staged_info()
    assert info["tiles"] == -(-A.m // info["tile_rows"])
    y = product(spx, G, dev(torch, X), plan).cpu().numpy().reshape(A.m, k)
    check_f64(y, A, X, (kind, k, info))


@pytest.mark.parametrize("kind", ["stencil27", "powerlaw", "one_long_row", "empty_rows"])
@pytest.mark.parametrize("k", [4, 16, 32])
def test_staged_exact_inputs_bit_exact(spx, torch, kind, k):
    A = int_valued(matrix(kind, seed=7), 2)
    G = to_gpu(A)
    X = spgen.small_ints(A.n * k, 8).reshape(A.n, k)
    y = spx.spmm(G, dev(torch, X), plan=spx.Plan.staged(G, k)).cpu().numpy()
    assert np.array_equal(y, oracle.spmm(A, X))


def test_staged_tiles_and_fallback(spx, torch):
    # every tile of a stencil is staged; the tile holding a 50,000-nonzero row
    # exceeds the 2,048 staged nonzeros and gathers directly, as do all tiles
    # whose window is above the 32 KB budget (k = 128 FP64: 1 KB rows, so at
    # most 32)
    S = to_gpu(matrix("stencil27", seed=1))
    info = spx.Plan.staged(S, 16).staged_info()
    assert info["staged_tiles"] == info["tiles"] and info["tile_rows"] == 16
    assert 0 < info["max_window_rows"] <= 32768 // 128
    L = to_gpu(matrix("one_long_row", seed=1))
    info = spx.Plan.staged(L, 16).staged_info()
    assert info["staged_tiles"] == info["tiles"] - 1
    big = spx.Plan.staged(S, 128).staged_info()
    assert big["staged_tiles"] < big["tiles"] and big["max_window_rows"] <= 32
    A = matrix("stencil27", seed=1)
    X = spgen.uniform(A.n * 128, 3).reshape(A.n, 128)
    y = spx.spmm(S, dev(torch, X), plan=spx.Plan.staged(S, 128)).cpu().numpy()
    check_f64(y, A, X, "k=128 mixed staged and direct tiles")


@pytest.mark.parametrize("vname", ["f32", "bf16"])
@pytest.mark.parametrize("kind", ["stencil27", "powerlaw", "one_long_row"])
@pytest.mark.parametrize("k", [8, 32])
def test_staged_precision_form(spx, torch, vname, kind, k):
    A = matrix(kind, seed=9)
    vdtype = "f32" if vname == "f32" else "bf16"
    G, A5 = quantised(A, vdtype, torch)
    Xq = spgen.to_f32(spgen.uniform(A.n * k, 10).reshape(A.n, k))
    plan = spx.Plan.staged(G, k, torch.float32)
    y = spx.spmm(G, dev(torch, Xq), plan=plan).double().cpu().numpy()
    absA5 = oracle.CSR(A.m, A.n, A.rowptr, A.colind, np.abs(A5.values))
    X5 = Xq.astype(np.float64)
    y5 = oracle.spmm(A5, X5)
    S5 = oracle.spmm(absA5, np.abs(X5))
    L = A.row_lengths()
    for j in range(k):
        check_bound(y[:, j], y5[:, j], S5[:, j], L, 256, (vname, kind, k, j))


def test_staged_deterministic_and_graph(spx, torch):
    A = matrix("stencil5", seed=3)
    G = to_gpu(A)
    k = 16
    X = dev(torch, spgen.uniform(A.n * k, 4).reshape(A.n, k))
    plan = spx.Plan.staged(G, k)
    Y0 = spx.spmm(G, X, plan=plan)
    Y = torch.empty_like(Y0)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        spx.spmm(G, X, Y=Y, plan=plan)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        spx.spmm(G, X, Y=Y, plan=plan)
    for r in range(3):
        X.mul_(-1.0)
        ref = spx.spmm(G, X, plan=plan)  # eager call between replays
        Y.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Y.view(torch.int64), ref.view(torch.int64)), r
    assert torch.equal(spx.spmm(G, X, plan=plan).view(torch.int64), spx.spmm(G, X, plan=plan).view(torch.int64))


def test_staged_plan_misuse(spx, torch):
    A = matrix("stencil27", seed=2)
    G = to_gpu(A)
    plan = spx.Plan.staged(G, 16)
    X8 = dev(torch, spgen.uniform(A.n * 8, 1).reshape(A.n, 8))
    with pytest.raises(spx.SpxError):
        spx.spmm(G, X8, plan=plan)                       # k differs from the plan's
    X17 = dev(torch, spgen.uniform(A.n * 17, 1).reshape(A.n, 17))[:, :16]
    with pytest.raises(spx.SpxError):
        spx.spmm(G, X17, plan=plan)                      # odd ld: no 16-byte loads, another lane layout
    X20 = dev(torch, spgen.uniform(A.n * 20, 1).reshape(A.n, 20))
    y20 = spx.spmm(G, X20[:, :16], plan=plan).cpu().numpy()  # ld 20 keeps the layout: served
    check_f64(y20, A, X20.cpu().numpy()[:, :16].copy(), "ld 20")
    Xf = dev(torch, spgen.uniform(A.n * 16, 1).reshape(A.n, 16)).float()
    with pytest.raises(spx.SpxError):
        spx.spmm(G.with_values(G.values.float()), Xf, plan=plan)  # X type differs
    dy = dev(torch, spgen.uniform(A.m, 1))
    with pytest.raises(spx.SpxError):
        spx.sddmm(G, dy, dev(torch, spgen.uniform(A.n, 2)), plan=plan)
    with pytest.raises(spx.SpxError):
        plan.export_bins()
    from paper_1302_1078_amd import _lib
    import ctypes
    nb = ctypes.c_size_t()
    L = _lib.load()
    assert L.csr_plan_staged_workspace_bytes(10, 10, 10, 0, 0, ctypes.byref(nb)) == _lib.SPX_ERR_UNSUPPORTED
    assert L.csr_plan_staged_workspace_bytes(10, 10, 10, 129, 0, ctypes.byref(nb)) == _lib.SPX_ERR_UNSUPPORTED
    assert L.csr_plan_staged_workspace_bytes(10, 10, 10, 4, 2, ctypes.byref(nb)) == _lib.SPX_ERR_UNSUPPORTED
    # k must be a multiple of the 16-byte vector: 2 FP64 or 4 FP32 elements
    assert L.csr_plan_staged_workspace_bytes(10, 10, 10, 3, 0, ctypes.byref(nb)) == _lib.SPX_ERR_UNSUPPORTED
    assert L.csr_plan_staged_workspace_bytes(10, 10, 10, 6, 1, ctypes.byref(nb)) == _lib.SPX_ERR_UNSUPPORTED
    assert L.csr_plan_staged_workspace_bytes(10, 10, 10, 2, 0, ctypes.byref(nb)) == _lib.SPX_OK


def test_staged_empty_and_tiny(spx, torch):
    for m, n, r, c in [(0, 5, [], []), (1, 1, [0], [0]), (300, 7, [299], [6])]:
        A = oracle.csr_from_coo(m, n, np.array(r, np.int32), np.array(c, np.int32), np.ones(len(r)))
        G = to_gpu(A)
        X = spgen.uniform(max(n, 1) * 8, 1).reshape(max(n, 1), 8)[:n]
        plan = spx.Plan.staged(G, 8)
        y = spx.spmm(G, dev(torch, np.ascontiguousarray(X)), plan=plan).cpu().numpy()
        assert np.array_equal(y, oracle.spmm(A, X)) if m else y.size == 0


# ---------------------------------------------------------------- pipelined kernel

@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("k", [2, 8, 16, 100])
def test_pipelined_equals_one_round_f64(spx, torch, kind, k):
    """The persistent double-buffered kernel does each row's arithmetic in the
    same order as the one-workgroup-per-tile kernel: bitwise the same Y, and
    within the FP64 bars of the oracle."""
    A = matrix(kind, seed=11)
    G = to_gpu(A)
    X = spgen.uniform(A.n * k, 12).reshape(A.n, k)
    Xd = dev(torch, X)
    y1 = spx.spmm(G, Xd, plan=spx.Plan.staged(G, k))
    y2 = spx.spmm(G, Xd, plan=spx.Plan.staged(G, k, pipelined=True))
    assert torch.equal(y1.view(torch.int64), y2.view(torch.int64)), (kind, k)
    check_f64(y2.cpu().numpy(), A, X, (kind, k, "pipelined"))


@pytest.mark.parametrize("vname", ["f32", "bf16"])
@pytest.mark.parametrize("kind", ["stencil27", "powerlaw", "one_long_row", "empty_rows"])
@pytest.mark.parametrize("k", [4, 16, 32])
def test_pipelined_equals_one_round_precision(spx, torch, vname, kind, k):
    A = matrix(kind, seed=13)
    G, _ = quantised(A, vname, torch)
    Xq = dev(torch, spgen.to_f32(spgen.uniform(A.n * k, 14).reshape(A.n, k)))
    y1 = spx.spmm(G, Xq, plan=spx.Plan.staged(G, k, torch.float32))
    y2 = spx.spmm(G, Xq, plan=spx.Plan.staged(G, k, torch.float32, pipelined=True))
    assert torch.equal(y1.view(torch.int32), y2.view(torch.int32)), (vname, kind, k)


def test_pipelined_graph_and_edges(spx, torch):
    A = matrix("stencil27", seed=15)
    G = to_gpu(A)
    k = 16
    X = dev(torch, spgen.uniform(A.n * k, 16).reshape(A.n, k))
    plan = spx.Plan.staged(G, k, pipelined=True)
    Y = torch.empty((A.m, k), dtype=torch.float64, device="cuda:0")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        spx.spmm(G, X, Y=Y, plan=plan)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        spx.spmm(G, X, Y=Y, plan=plan)
    for r in range(3):
        X.mul_(-1.0)
        ref = spx.spmm(G, X, plan=spx.Plan.staged(G, k))  # one-round kernel, eager, between replays
        Y.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Y.view(torch.int64), ref.view(torch.int64)), r
    # empty and tiny matrices, a single tile, and a plan that is not staged
    for m, n, r_, c_ in [(0, 5, [], []), (1, 1, [0], [0]), (300, 7, [299], [6])]:
        B = oracle.csr_from_coo(m, n, np.array(r_, np.int32), np.array(c_, np.int32), np.ones(len(r_)))
        H = to_gpu(B)
        Xs = spgen.uniform(max(n, 1) * 8, 1).reshape(max(n, 1), 8)[:n]
        y = spx.spmm(H, dev(torch, np.ascontiguousarray(Xs)), plan=spx.Plan.staged(H, 8, pipelined=True)).cpu().numpy()
        assert np.array_equal(y, oracle.spmm(B, Xs)) if m else y.size == 0
    from paper_1302_1078_amd import _lib
    binned = spx.Plan.for_matrix(G, spx.default_opts(k))
    assert _lib.load().csr_plan_staged_pipeline(binned.handle, 1) == _lib.SPX_ERR_INVALID
