"""csr_permute on the device against the oracle, and products on RCM-ordered
matrices (Sec. 4.4): P A P^T applied to P x gives P (A x)."""
import numpy as np
import pytest

import oracle
import spgen
from _cases import int_valued, to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spx():
    import paper_1302_1078_amd as m
    return m


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def relabeled_cases():
    return [("stencil27", spgen.relabeled(spgen.stencil3d(17, 13, 11, 27, 1), 2)),
            ("stencil5", spgen.relabeled(spgen.stencil5(77, 61, 3), 4)),
            ("powerlaw", spgen.powerlaw(20_000, 20_000, 2.0, 6_000, 16.0, 5))]


@pytest.mark.parametrize("name,coo", relabeled_cases(), ids=[c[0] for c in relabeled_cases()])
def test_permute_bit_exact_and_products(spx, torch, name, coo):
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    G = to_gpu(A)
    perm = spx.rcm(G)
    ph = perm.cpu().numpy()
    assert np.array_equal(ph, oracle.rcm(A))
    B = spx.permute(G, perm)
    ref = oracle.permute(A, ph)
    assert np.array_equal(B.rowptr.cpu().numpy(), ref.rowptr)
    assert np.array_equal(B.colind.cpu().numpy(), ref.colind)
    assert np.array_equal(B.values.cpu().numpy(), ref.values)
    # products: (P A P^T)(P x) = P (A x), exactly on integer inputs
    Ai = int_valued(A, 6)
    Bi = spx.permute(to_gpu(Ai), perm)
    x = spgen.small_ints(A.n, 7)
    y = oracle.spmv(Ai, x)
    xp = torch.from_numpy(x[ph]).to("cuda:0")
    for opts in (spx.default_opts(1), None):
        plan = spx.Plan.for_matrix(Bi, opts) if opts is not None else None
        yp = spx.spmv(Bi, xp, plan=plan).cpu().numpy()
        assert np.array_equal(yp, y[ph])
    k = 16
    X = spgen.small_ints(A.n * k, 8).reshape(A.n, k)
    Y = oracle.spmm(Ai, X)
    Yp = spx.spmm(Bi, torch.from_numpy(np.ascontiguousarray(X[ph])).to("cuda:0"),
                  plan=spx.Plan.for_matrix(Bi, spx.default_opts(k))).cpu().numpy()
    assert np.array_equal(Yp, Y[ph])


def test_permute_identity_and_errors(spx, torch):
    coo = spgen.powerlaw(3000, 3000, 2.0, 1000, 10.0, 9)
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    G = to_gpu(A)
    ident = torch.arange(A.m, dtype=torch.int32, device="cuda:0")
    B = spx.permute(G, ident)
    assert np.array_equal(B.rowptr.cpu().numpy(), A.rowptr)
    assert np.array_equal(B.colind.cpu().numpy(), A.colind)
    assert np.array_equal(B.values.cpu().numpy(), A.values)
    rev = torch.flip(ident, [0]).contiguous()
    assert np.array_equal(spx.permute(G, rev).colind.cpu().numpy(), oracle.permute(A, rev.cpu().numpy()).colind)
    dup = ident.clone()
    dup[5] = 7  # not a permutation: vertex 5 gets no new label
    with pytest.raises(ValueError):
        spx.permute(G, dup)
    with pytest.raises(ValueError):
        spx.permute(G, ident[:-1].contiguous())


@pytest.mark.parametrize("name", ["powerlaw", "stencil5", "empty_cols", "empty"])
def test_degree_order_bit_exact_and_products(spx, torch, name):
    """csr_degree_order equals the oracle's order exactly (ties included);
    the symmetric relabelling it drives keeps (P A P^T)(P x) = P (A x)."""
    if name == "powerlaw":
        coo = spgen.powerlaw(30_000, 30_000, 2.0, 6_000, 16.0, 9)
    elif name == "stencil5":
        coo = spgen.stencil5(90, 70, 2)
    elif name == "empty_cols":  # only even columns used
        rng = np.random.default_rng(3)
        r = rng.integers(0, 500, 3000).astype(np.int32)
        c = (2 * rng.integers(0, 250, 3000)).astype(np.int32)
        coo = spgen.COO(500, 500, r, c, np.ones(3000), {})
    else:
        coo = spgen.COO(0, 0, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0), {})
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    G = to_gpu(A)
    perm = spx.degree_order(G)
    ph = perm.cpu().numpy()
    assert np.array_equal(ph, oracle.degree_order(A))
    if A.m == 0:
        return
    Ai = int_valued(A, 11)
    Bi = spx.permute(to_gpu(Ai), perm)
    x = spgen.small_ints(A.n, 12)
    y = oracle.spmv(Ai, x)
    yp = spx.spmv(Bi, torch.from_numpy(x[ph]).to("cuda:0"),
                  plan=spx.Plan.for_matrix(Bi, spx.default_opts(1))).cpu().numpy()
    assert np.array_equal(yp, y[ph])


@pytest.mark.parametrize("name,nx,ny,nz,pts,tag", [("stencil27", 14, 12, 10, 27, 2), ("stencil7", 20, 16, 12, 7, 3)])
def test_rcm_recovers_the_band_on_the_device(spx, torch, name, nx, ny, nz, pts, tag):
    """A 3D stencil with its rows and columns relabeled at random loses its
    band; the library's RCM order applied on the device (csr_permute)
    narrows it below a quarter of the relabeled one (Sec. 4.4), and
    csr_bandwidth reads the same value as the oracle's permuted matrix."""
    coo = spgen.relabeled(spgen.stencil3d(nx, ny, nz, pts, 1), tag)
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    G = to_gpu(A)
    perm = spx.rcm(G)
    P = spx.permute(G, perm)
    B = oracle.permute(A, perm.cpu().numpy())
    rows = np.repeat(np.arange(B.m), np.diff(B.rowptr))
    bw_host = int(np.abs(B.colind.astype(np.int64) - rows).max())
    bw_relabeled = spx.bandwidth(G)
    bw = spx.bandwidth(P)
    assert bw == bw_host, name
    assert bw < bw_relabeled / 4, (name, bw, bw_relabeled)
