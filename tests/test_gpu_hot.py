"""GPU checks of hot x (csr_plan_attach_hot_x): SpMV through a plan whose
most-used columns' x entries are read from a compact copy is bitwise the
product through the same plan without it (same products, same order), for
every matrix kind, value type and number of hot columns; SpMM and the
transpose ignore it; misuse is rejected."""
import numpy as np
import pytest

import oracle
import spgen
from _cases import KINDS, matrix, quantised, to_gpu

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


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("vname", ["f64", "f32", "bf16"])
def test_hot_x_bitwise(spx, torch, kind, vname):
    A = matrix(kind, seed=51)
    if vname == "f64":
        G = to_gpu(A)
        x = dev(torch, spgen.uniform(A.n, 52))
        t = torch.float64
    else:
        G, _ = quantised(A, vname, torch)
        x = dev(torch, spgen.to_f32(spgen.uniform(A.n, 52)))
        t = torch.float32
    opts = spx.default_opts(1, t)
    y0 = spx.spmv(G, x, plan=spx.Plan.for_matrix(G, opts))
    for hot in (1, 7, 256, A.n + 5):  # past n: every column is hot
        p = spx.Plan.for_matrix(G, opts).attach_hot_x(G, hot, x.dtype)
        y = spx.spmv(G, x, plan=p)
        assert torch.equal(y.view(torch.int8), y0.view(torch.int8)), (kind, vname, hot)
    if vname == "f64":
        ref = oracle.spmv(A, x.cpu().numpy())
        assert oracle.rel2(y.cpu().numpy(), ref) <= 1e-12


def test_hot_x_ranking_and_other_products(spx, torch):
    """The hot columns are the most used: with exact small-integer inputs the
    result equals the oracle exactly, whichever columns are hot; SpMM and the
    CSC transpose through a hot plan equal the plain plan's."""
    A = oracle.csr_from_coo(6, 5, np.array([0, 1, 2, 3, 4, 5, 5, 0], np.int32),
                            np.array([3, 3, 3, 1, 3, 1, 4, 0], np.int32), np.arange(1.0, 9.0))
    G = to_gpu(A)
    x = dev(torch, np.array([1.0, -2.0, 3.0, 4.0, -5.0]))
    p = spx.Plan.for_matrix(G, spx.default_opts(1)).attach_hot_x(G, 2)
    assert np.array_equal(spx.spmv(G, x, plan=p).cpu().numpy(), oracle.spmv(A, x.cpu().numpy()))
    B = matrix("powerlaw", seed=53)
    H = to_gpu(B)
    k = 8
    X = dev(torch, spgen.uniform(B.n * k, 54).reshape(B.n, k))
    ph = spx.Plan.for_matrix(H, spx.default_opts(k)).attach_hot_x(H, 64)
    p0 = spx.Plan.for_matrix(H, spx.default_opts(k))
    assert torch.equal(spx.spmm(H, X, plan=ph).view(torch.int64), spx.spmm(H, X, plan=p0).view(torch.int64))
    dy = dev(torch, spgen.normal(B.m, 55))
    xv = dev(torch, spgen.uniform(B.n, 56))
    p1 = spx.Plan.for_matrix(H, spx.default_opts(1)).attach_hot_x(H, 64)
    assert torch.equal(spx.sddmm(H, dy, xv, plan=p1).view(torch.int64),
                       spx.sddmm(H, dy, xv).view(torch.int64))
    _, xs = spx.spmv_save(H, xv, plan=p1)  # the saved gather reads the pattern's own colind
    assert np.array_equal(xs.cpu().numpy(), xv.cpu().numpy()[B.colind])


def test_hot_x_graph_replay(spx, torch):
    A = matrix("powerlaw", seed=57)
    G = to_gpu(A)
    x = dev(torch, spgen.uniform(A.n, 58))
    p = spx.Plan.for_matrix(G, spx.default_opts(1)).attach_hot_x(G, 128)
    p0 = spx.Plan.for_matrix(G, spx.default_opts(1))
    y = torch.empty(A.m, dtype=torch.float64, device="cuda:0")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        spx.spmv(G, x, y=y, plan=p)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        spx.spmv(G, x, y=y, plan=p)
    for r in range(3):
        x.mul_(-1.5)
        ref = spx.spmv(G, x, plan=p0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y.view(torch.int64), ref.view(torch.int64)), r


def test_hot_x_misuse(spx, torch):
    from paper_1302_1078_amd import _lib
    import ctypes
    L = _lib.load()
    A = matrix("powerlaw", seed=59)
    G = to_gpu(A)
    nb = ctypes.c_size_t()
    assert L.csr_plan_hot_x_workspace_bytes(A.n, A.nnz, 0, ctypes.byref(nb)) == _lib.SPX_ERR_UNSUPPORTED
    assert L.csr_plan_hot_x_workspace_bytes(A.n, A.nnz, (1 << 20) + 1, ctypes.byref(nb)) == _lib.SPX_ERR_UNSUPPORTED
    assert L.csr_plan_hot_x_workspace_bytes(A.n, A.nnz, 16, ctypes.byref(nb)) == _lib.SPX_OK
    p = spx.Plan.for_matrix(G, spx.default_opts(1)).attach_hot_x(G, 16)
    with pytest.raises(spx.SpxError):  # attached for FP64 x, called with FP32
        spx.spmv(G.with_values(G.values.float()), dev(torch, spgen.to_f32(spgen.uniform(A.n, 1))), plan=p)
    S = to_gpu(matrix("stencil27", seed=2))
    with pytest.raises(spx.SpxError):
        spx.Plan.staged(S, 8).attach_hot_x(S, 16)
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda:0")
    q = spx.Plan.for_matrix(G, spx.default_opts(1))
    assert L.csr_plan_attach_hot_x(q.handle, A.n + 1, A.nnz, G.colind.data_ptr(), 16, _lib.SPX_F64,
                                   ws.data_ptr(), nb.value, None) == _lib.SPX_ERR_INVALID
    assert L.csr_plan_attach_hot_x(q.handle, A.n, A.nnz, G.colind.data_ptr(), 16, _lib.SPX_F64,
                                   ws.data_ptr(), 16, None) == _lib.SPX_ERR_WORKSPACE
