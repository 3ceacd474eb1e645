"""Plans with a row period (spx_plan_opts.row_period) and csr_bandwidth.

A row period P lists each bin's rows band by band, band = floor(8 (r mod P) / P),
ascending inside a band.  The order of rows never changes a row's arithmetic,
so every product through such a plan is bitwise the product through the same
plan without a period; the bins hold the same rows; csr_bandwidth is exact
integer work, compared with a host computation.
"""
import numpy as np
import pytest

import oracle
import spgen
from _cases import KINDS, keep_stream, matrix, to_gpu, two_bin_opts

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spx():
    import paper_1302_1078_amd as m
    return m


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def host_bandwidth(A: oracle.CSR) -> int:
    rows = np.repeat(np.arange(A.m, dtype=np.int64), np.diff(A.rowptr))
    return int(np.abs(A.colind.astype(np.int64) - rows).max()) if A.nnz else 0


def grid27(n: int) -> oracle.CSR:
    C = spgen.stencil3d(n, n, n, 27, 0)
    return oracle.csr_from_coo(C.m, C.n, C.r, C.c, C.v)


def cases():
    out = [(k, matrix(k)) for k in KINDS]
    out.append(("grid27_12", grid27(12)))
    return out


@pytest.mark.parametrize("name,A", cases(), ids=[c[0] for c in cases()])
def test_bandwidth_exact(spx, torch, name, A):
    assert spx.bandwidth(to_gpu(A)) == host_bandwidth(A), name


def test_bandwidth_degenerate(spx, torch):
    import paper_1302_1078_amd._lib as L
    dev = torch.device("cuda", 0)
    empty = spx.CSR(torch.zeros(4, dtype=torch.int32, device=dev), torch.zeros(0, dtype=torch.int32, device=dev),
                    torch.zeros(0, dtype=torch.float64, device=dev), (3, 5))
    assert spx.bandwidth(empty) == 0
    diag = spx.CSR(torch.arange(6, dtype=torch.int32, device=dev), torch.arange(5, dtype=torch.int32, device=dev),
                   torch.ones(5, dtype=torch.float64, device=dev), (5, 5))
    assert spx.bandwidth(diag) == 0
    corner = spx.CSR(torch.tensor([0, 1, 1, 2], dtype=torch.int32, device=dev),
                     torch.tensor([7, 0], dtype=torch.int32, device=dev),
                     torch.ones(2, dtype=torch.float64, device=dev), (3, 8))
    assert spx.bandwidth(corner) == 7
    lib = L.load()
    assert lib.csr_bandwidth(-1, 0, None, None, None, None) != 0


def band_of(rows, P):
    return (rows.astype(np.int64) % P) * 8 // P


PERIODS = [1, 3, 7, 100, "bw", "m", "10m"]


def period_value(P, A):
    if P == "bw":
        return max(host_bandwidth(A), 1)
    if P == "m":
        return A.m
    if P == "10m":
        return 10 * A.m
    return P


def plan_pair(spx, G, o):
    d = o.to_dict()
    p0 = spx.Plan.for_matrix(G, spx.PlanOpts.from_dict(dict(d, row_period=0)))
    return p0, d


@pytest.mark.parametrize("name,A", cases(), ids=[c[0] for c in cases()])
@pytest.mark.parametrize("P", PERIODS)
def test_row_period_bins(spx, torch, name, A, P):
    """Same rows per bin as without a period; inside a bin ordered by (band, row)."""
    G = to_gpu(A)
    Pv = period_value(P, A)
    for o in (spx.default_opts(1), spx.default_opts(16), two_bin_opts(40, 8, 4, chunk=256)):
        p0, d = plan_pair(spx, G, o)
        p1 = spx.Plan.for_matrix(G, spx.PlanOpts.from_dict(dict(d, row_period=Pv)))
        perm0, off0 = p0.export_bins()
        perm1, off1 = p1.export_bins()
        assert np.array_equal(off0, off1)
        assert np.array_equal(np.sort(perm1), np.arange(A.m))
        for b in range(len(off0) - 1):
            s0, s1 = perm0[off0[b]:off0[b + 1]], perm1[off1[b]:off1[b + 1]]
            assert np.array_equal(np.sort(s1), s0), (name, P, b)
            key = band_of(s1, Pv) * (A.m + 1) + s1
            assert np.all(np.diff(key) > 0), (name, P, b)


@pytest.mark.parametrize("name,A", cases(), ids=[c[0] for c in cases()])
@pytest.mark.parametrize("vname", ["f64", "f32", "bf16"])
def test_row_period_products_bitwise(spx, torch, name, A, vname):
    """SpMV and SpMM (k = 4, 16) through plans with each period equal the
    plan without one, bit for bit; FP64 also within 1e-12 of the oracle."""
    vt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[vname]
    xt = torch.float64 if vname == "f64" else torch.float32
    G = to_gpu(A, vt)
    for k in (1, 4, 16):
        X = torch.from_numpy(spgen.uniform(A.n * k, 6).reshape(A.n, k)).to("cuda:0").to(xt)
        for o in (keep_stream(spx.default_opts(k, vt)), two_bin_opts(40, 8, k, chunk=256)):
            p0, d = plan_pair(spx, G, o)
            y0 = spx.spmv(G, X[:, 0].contiguous(), plan=p0) if k == 1 else spx.spmm(G, X, plan=p0)
            for P in PERIODS:
                p1 = spx.Plan.for_matrix(G, spx.PlanOpts.from_dict(dict(d, row_period=period_value(P, A))))
                y1 = spx.spmv(G, X[:, 0].contiguous(), plan=p1) if k == 1 else spx.spmm(G, X, plan=p1)
                assert torch.equal(y0.view(torch.uint8), y1.view(torch.uint8)), (name, vname, k, P)
            if vname == "f64":
                ref = oracle.spmv(A, X[:, 0].cpu().numpy()) if k == 1 else oracle.spmm(A, X.cpu().numpy())
                assert oracle.rel2(y0.cpu().numpy(), ref) <= 1e-12


def test_banded_opts_on_a_grid(spx, torch):
    """banded_opts takes the matrix's bandwidth as the period: n^2 + n + 1 for
    the 27-point stencil on n^3; the banded SpMM equals the default one."""
    n = 16
    A = grid27(n)
    G = to_gpu(A)
    o = spx.banded_opts(G, 16)
    assert o.row_period == n * n + n + 1
    X = torch.from_numpy(spgen.uniform(A.n * 16, 2).reshape(A.n, 16)).to("cuda:0")
    y0 = spx.spmm(G, X, plan=spx.Plan.for_matrix(G, spx.default_opts(16)))
    y1 = spx.spmm(G, X, plan=spx.Plan.for_matrix(G, o))
    assert torch.equal(y0, y1)
