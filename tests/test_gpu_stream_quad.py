"""Stream tiles whose nonzeros form one contiguous run load them four at a
time (16-byte index and value loads from an aligned position before the
tile's first nonzero); any other tile, and every tile of a matrix whose colind
or values are not 16-byte aligned, loads element by element.

Row-length patterns put the tiles' first nonzero at every position modulo 4
and their element counts below, at and across the 1,024 (FP64) and 2,048
(FP32 / BF16 values) element chunks.  Bars: small-integer inputs give the
oracle's exact sums; general inputs give bitwise the same y through the
four-at-a-time loads as through element loads (both sum each row's products
in ascending position), and FP64 within 1e-12 (2-norm) of the oracle.
"""
import numpy as np
import pytest

import oracle
import spgen
from _cases import int_valued, keep_stream

pytestmark = pytest.mark.gpu

VT = {"f64": "float64", "f32": "float32", "bf16": "bfloat16"}


@pytest.fixture(scope="module")
def spx():
    import paper_1302_1078_amd as m
    return m


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def lengths(pattern: str) -> np.ndarray:
    rng = np.random.default_rng(sum(map(ord, pattern)))
    if pattern == "rand1_7":        # tiles near 1,024 nonzeros
        return rng.integers(1, 8, 3000)
    if pattern == "rand1_15":       # near 2,048
        return rng.integers(1, 16, 3000)
    if pattern == "rand0_60":       # many chunks per tile, empty rows
        L = rng.integers(0, 61, 2000)
        L[rng.random(2000) < 0.2] = 0
        return L
    if pattern == "const3":         # one partial chunk per tile, ragged last tile
        return np.full(1000, 3)
    if pattern == "const4":         # exactly one FP64 chunk per tile
        return np.full(256 * 4 + 5, 4)
    if pattern == "const8":         # exactly one FP32 chunk per tile
        return np.full(256 * 4 + 9, 8)
    if pattern == "shift1":         # every later tile starts 1 past a multiple of 4
        L = np.full(256 * 5, 4)
        L[0] = 1
        return L
    if pattern == "shift3":         # ... 3 past
        L = np.full(256 * 5, 8)
        L[0] = 3
        return L
    if pattern == "tiny":
        return np.array([1, 5, 2, 0, 3])
    raise ValueError(pattern)


PATTERNS = ["rand1_7", "rand1_15", "rand0_60", "const3", "const4", "const8", "shift1", "shift3", "tiny"]


def pattern_matrix(pattern: str, n: int = 4000) -> oracle.CSR:
    L = lengths(pattern).astype(np.int64)
    rng = np.random.default_rng(7)
    rowptr = np.zeros(len(L) + 1, dtype=np.int32)
    rowptr[1:] = np.cumsum(L)
    cols = [np.sort(rng.choice(n, int(l), replace=False)) for l in L]
    colind = np.concatenate(cols).astype(np.int32) if len(cols) else np.zeros(0, np.int32)
    vals = spgen.uniform(len(colind), 3, spgen.TAG_VALUES)
    return oracle.CSR(len(L), n, rowptr, colind, vals)


def upload(spx, torch, A: oracle.CSR, vname: str, misalign: bool):
    """A on the device; with misalign, colind and values sit one element past
    a 16-byte boundary (views into one-longer buffers)."""
    dev = torch.device("cuda", 0)
    vt = getattr(torch, VT[vname])
    ci = torch.from_numpy(A.colind)
    va = torch.from_numpy(np.ascontiguousarray(A.values)).to(vt)
    if misalign:
        cbuf = torch.zeros(A.nnz + 1, dtype=torch.int32, device=dev)
        vbuf = torch.zeros(A.nnz + 1, dtype=vt, device=dev)
        cbuf[1:] = ci.to(dev)
        vbuf[1:] = va.to(dev)
        ci_d, va_d = cbuf[1:], vbuf[1:]
        assert ci_d.data_ptr() % 16 != 0 and va_d.data_ptr() % 16 != 0
    else:
        ci_d, va_d = ci.to(dev), va.to(dev)
        assert ci_d.data_ptr() % 16 == 0 and va_d.data_ptr() % 16 == 0
    return spx.CSR(torch.from_numpy(A.rowptr).to(dev), ci_d, va_d, (A.m, A.n))


def run(spx, torch, G, x_np, vname):
    xt = torch.float64 if vname == "f64" else torch.float32
    x = torch.from_numpy(x_np).to("cuda:0").to(xt)
    plan = spx.Plan.for_matrix(G, keep_stream(spx.default_opts(1, getattr(torch, VT[vname]))))
    y = spx.spmv(G, x, plan=plan)
    torch.cuda.synchronize()
    return y


@pytest.mark.parametrize("pattern", PATTERNS)
@pytest.mark.parametrize("vname", ["f64", "f32", "bf16"])
def test_stream_quads_exact(spx, torch, pattern, vname):
    """Small-integer values and x: the oracle's sums exactly, with and without
    the four-at-a-time loads."""
    A = int_valued(pattern_matrix(pattern), seed=9)
    x = spgen.small_ints(A.n, 2)
    ref = oracle.spmv(A, x)
    for misalign in (False, True):
        y = run(spx, torch, upload(spx, torch, A, vname, misalign), x, vname)
        assert np.array_equal(y.double().cpu().numpy(), ref), (pattern, vname, misalign)


@pytest.mark.parametrize("pattern", PATTERNS)
@pytest.mark.parametrize("vname", ["f64", "f32", "bf16"])
def test_stream_quads_bitwise_element_loads(spx, torch, pattern, vname):
    """General values: the same bits through both load paths; FP64 also
    within 1e-12 of the oracle."""
    A = pattern_matrix(pattern)
    x = spgen.uniform(A.n, 4)
    y_q = run(spx, torch, upload(spx, torch, A, vname, False), x, vname)
    y_e = run(spx, torch, upload(spx, torch, A, vname, True), x, vname)
    assert torch.equal(y_q.view(torch.uint8), y_e.view(torch.uint8)), (pattern, vname)
    if vname == "f64":
        ref = oracle.spmv(A, x)
        assert oracle.rel2(y_q.cpu().numpy(), ref) <= 1e-12


def test_stream_quads_graph_replay(spx, torch):
    """Captured in a HIP graph and replayed with eager work between the
    replays, the four-at-a-time path gives the eager result every time."""
    A = pattern_matrix("rand0_60")
    G = upload(spx, torch, A, "f64", False)
    x = torch.from_numpy(spgen.uniform(A.n, 4)).to("cuda:0")
    plan = spx.Plan.for_matrix(G, keep_stream(spx.default_opts(1)))
    y_eager = spx.spmv(G, x, plan=plan).clone()
    y = torch.empty_like(y_eager)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        spx.spmv(G, x, y=y, plan=plan)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        spx.spmv(G, x, y=y, plan=plan)
    for i in range(4):
        y.fill_(float(i))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, y_eager), i
