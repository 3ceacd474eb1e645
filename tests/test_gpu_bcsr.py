"""Register-blocked CRS (Sec. 4.5) on the device: conversion bit-exact against
the oracle's blocking, products against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import spgen
from _cases import int_valued, matrix, to_gpu

pytestmark = pytest.mark.gpu

SHAPES = [(a, b) for a in (1, 2, 4, 8) for b in (1, 2, 4, 8)]


@pytest.fixture(scope="module")
def spx():
    import paper_1302_1078_amd as m
    return m


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


@pytest.fixture(scope="module")
def mats():
    # m and n not multiples of 8: ragged last block row and column
    return {"powerlaw": matrix("powerlaw", 21), "stencil27": matrix("stencil27", 22),
            "empty_rows": matrix("empty_rows", 23)}


@pytest.mark.parametrize("a,b", SHAPES)
@pytest.mark.parametrize("bitmap", [False, True])
def test_bcsr_conversion_and_spmv(spx, torch, mats, a, b, bitmap):
    for name, A in mats.items():
        G = to_gpu(A)
        B = spx.BCSR.from_csr(G, a, b, bitmap)
        R = oracle.to_bcsr(A, a, b, bitmap)
        assert B.nblocks == R.nblocks, name
        assert np.array_equal(B.browptr.cpu().numpy(), R.browptr), name
        assert np.array_equal(B.bcol.cpu().numpy(), R.bcol), name
        assert np.array_equal(B.bvals.cpu().numpy(), R.values), name
        if bitmap:
            assert np.array_equal(B.bmask.cpu().numpy().view(np.uint64), R.mask), name
            assert np.array_equal(B.boff.cpu().numpy(), R.offset), name
        x = spgen.uniform(A.n, 24)
        ref = oracle.spmv(A, x)
        xd = torch.from_numpy(x).to("cuda:0")
        for lanes in (0, 1, 8, 64):
            y = spx.bcsr_spmv(B, xd, lanes=lanes).cpu().numpy()
            assert oracle.rel2(y, ref) <= 1e-12, (name, lanes)
    # exact on integer inputs
    Ai = int_valued(mats["powerlaw"], 25)
    Bi = spx.BCSR.from_csr(to_gpu(Ai), a, b, bitmap)
    xi = spgen.small_ints(Ai.n, 26)
    y = spx.bcsr_spmv(Bi, torch.from_numpy(xi).to("cuda:0")).cpu().numpy()
    assert np.array_equal(y, oracle.spmv(Ai, xi))


def test_bcsr_edges_and_errors(spx, torch):
    # a matrix with no nonzeros, and one with a single dense 8 x 8 block
    E = oracle.csr_from_coo(10, 7, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0))
    BE = spx.BCSR.from_csr(to_gpu(E), 4, 2)
    assert BE.nblocks == 0
    y = spx.bcsr_spmv(BE, torch.ones(7, dtype=torch.float64, device="cuda:0")).cpu().numpy()
    assert np.array_equal(y, np.zeros(10))
    rr, cc = np.meshgrid(np.arange(8, dtype=np.int32), np.arange(8, dtype=np.int32), indexing="ij")
    D = oracle.csr_from_coo(8, 8, rr.ravel(), cc.ravel(), np.arange(64, dtype=np.float64))
    BD = spx.BCSR.from_csr(to_gpu(D), 8, 8)
    assert BD.nblocks == 1 and BD.stored_bytes() - 4 * 2 == 516  # the paper's 516 B block
    y = spx.bcsr_spmv(BD, torch.ones(8, dtype=torch.float64, device="cuda:0")).cpu().numpy()
    assert np.array_equal(y, np.arange(64, dtype=np.float64).reshape(8, 8).sum(1))
    with pytest.raises(spx.SpxError):
        spx.BCSR.from_csr(to_gpu(D), 3, 2)
    with pytest.raises(spx.SpxError):
        spx.bcsr_spmv(BD, torch.ones(8, dtype=torch.float64, device="cuda:0"), lanes=3)


# ---------------------------------------------------------------- multi-vector product (a x 1 blocks)

MM_KS = [1, 2, 3, 8, 16, 17, 32, 64, 65, 100]


@pytest.mark.parametrize("a", [2, 4, 8])
def test_bcsr_spmm_parity(spx, torch, mats, a):
    """Y = A X through a x 1 dense blocks against the FP64 oracle (rel2 <= 1e-12
    per column) for k from 1 to 100 (one and two column slabs, odd k, vector
    and scalar X loads), every slot count, on ragged matrices."""
    for name, A in mats.items():
        B = spx.BCSR.from_csr(to_gpu(A), a, 1)
        for k in MM_KS:
            X = spgen.uniform(A.n * k, 27 + k).reshape(A.n, k)
            ref = oracle.spmm(A, X)
            Xd = torch.from_numpy(X).to("cuda:0")
            kl = 1
            while kl * (2 if k % 2 == 0 else 1) < min(k, 64 if k % 2 == 0 else 32):
                kl <<= 1
            for slots in sorted({0, 1, max(1, 64 // kl)}):
                Y = spx.bcsr_spmm(B, Xd, slots=slots).cpu().numpy()
                for j in range(k):
                    assert oracle.rel2(Y[:, j], ref[:, j]) <= 1e-12, (name, a, k, slots, j)


@pytest.mark.parametrize("a", [2, 4, 8])
def test_bcsr_spmm_exact_and_strides(spx, torch, mats, a):
    """Small-integer inputs: the oracle's sums exactly, also with padded row
    strides (ldx, ldy > k), a misaligned X (scalar loads) and a stencil."""
    for name in ("powerlaw", "stencil27"):
        Ai = int_valued(mats[name], 28)
        B = spx.BCSR.from_csr(to_gpu(Ai), a, 1)
        for k in (4, 16, 24):
            X = spgen.small_ints(Ai.n * k, 29).reshape(Ai.n, k)
            ref = oracle.spmm(Ai, X)
            Xd = torch.from_numpy(X).to("cuda:0")
            assert np.array_equal(spx.bcsr_spmm(B, Xd).cpu().numpy(), ref), (name, a, k)
            Xp = torch.zeros((Ai.n, k + 6), dtype=torch.float64, device="cuda:0")
            Xp[:, :k] = Xd
            Yp = torch.full((Ai.m, k + 2), 7.0, dtype=torch.float64, device="cuda:0")
            spx.bcsr_spmm(B, Xp[:, :k], Y=Yp[:, :k])
            assert np.array_equal(Yp[:, :k].cpu().numpy(), ref), (name, a, k, "ld")
            assert bool((Yp[:, k:] == 7.0).all()), "columns past k untouched"
            Xm = torch.zeros(Ai.n * k + 1, dtype=torch.float64, device="cuda:0")
            Xm[1:] = Xd.reshape(-1)
            Xmis = Xm[1:].view(Ai.n, k)
            assert Xmis.data_ptr() % 16 != 0
            assert np.array_equal(spx.bcsr_spmm(B, Xmis).cpu().numpy(), ref), (name, a, k, "misaligned")


def test_bcsr_spmm_deterministic_and_errors(spx, torch, mats):
    A = mats["stencil27"]
    B = spx.BCSR.from_csr(to_gpu(A), 4, 1)
    X = torch.from_numpy(spgen.uniform(A.n * 16, 30).reshape(A.n, 16)).to("cuda:0")
    Y0 = spx.bcsr_spmm(B, X)
    for _ in range(3):
        assert torch.equal(spx.bcsr_spmm(B, X), Y0)
    E = oracle.csr_from_coo(10, 7, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0))
    BE = spx.BCSR.from_csr(to_gpu(E), 4, 1)
    Y = spx.bcsr_spmm(BE, torch.ones((7, 5), dtype=torch.float64, device="cuda:0"))
    assert np.array_equal(Y.cpu().numpy(), np.zeros((10, 5)))
    with pytest.raises(spx.SpxError):   # only a x 1 blocks
        spx.bcsr_spmm(spx.BCSR.from_csr(to_gpu(A), 4, 2), X)
    with pytest.raises(spx.SpxError):   # a = 1 is the CSR product
        spx.bcsr_spmm(spx.BCSR.from_csr(to_gpu(A), 1, 1), X)
    with pytest.raises(ValueError):     # bitmap form
        spx.bcsr_spmm(spx.BCSR.from_csr(to_gpu(A), 4, 1, True), X)
    with pytest.raises(spx.SpxError):   # slots not a power of two
        spx.bcsr_spmm(B, X, slots=3)
    with pytest.raises(spx.SpxError):   # 16 slots x 8 lanes > 64
        spx.bcsr_spmm(B, X, slots=16)


@pytest.mark.parametrize("a", [2, 4, 8])
def test_bcsr_spmm_row_period_bitwise(spx, torch, mats, a):
    """Block rows swept band by band of a row period give the same bits as the
    ascending order (each block row's sums are unchanged), for periods below,
    at and above the number of rows."""
    for name, A in mats.items():
        G = to_gpu(A)
        B = spx.BCSR.from_csr(G, a, 1)
        bw = spx.bandwidth(G)
        for k in (3, 16, 70):
            X = torch.from_numpy(spgen.uniform(A.n * k, 32 + k).reshape(A.n, k)).to("cuda:0")
            Y0 = spx.bcsr_spmm(B, X)
            for P in (1, 3, 7, 100, max(bw, 1), A.m, 10 * A.m):
                for slots in (0, 1):
                    Y1 = spx.bcsr_spmm(B, X, slots=slots, row_period=P)
                    if slots == 0:
                        assert torch.equal(Y0.view(torch.uint8), Y1.view(torch.uint8)), (name, a, k, P)
                    else:
                        ref = oracle.spmm(A, X.cpu().numpy())
                        assert oracle.rel2(Y1.cpu().numpy(), ref) <= 1e-12, (name, a, k, P, slots)
    with pytest.raises(spx.SpxError):
        spx.bcsr_spmm(B, X, row_period=-1)


@pytest.mark.parametrize("vdtype", ["f32", "bf16"])
@pytest.mark.parametrize("a", [2, 4])
def test_bcsr_spmm_precision(spx, torch, mats, vdtype, a):
    """FP32 / BF16 block values with FP32 X: every output within the FP32
    bound gamma_(L+8) sum |a||x| of the FP64 oracle on the stored (quantised)
    values; exact on small integers; the same bits with a row period."""
    from _cases import check_bound, quantised
    vt = torch.float32 if vdtype == "f32" else torch.bfloat16
    for name, A in mats.items():
        _, A5 = quantised(A, vdtype, torch)         # oracle matrix: the stored values, widened exactly
        B = spx.BCSR.from_csr(to_gpu(A5), a, 1)
        vals = B.bvals.to(vt)                        # exact: the values are representable
        assert torch.equal(vals.double(), B.bvals)
        L = A5.row_lengths()
        for k in (3, 8, 16, 40):
            Xq = spgen.to_f32(spgen.uniform(A.n * k, 33 + k).reshape(A.n, k))
            Xd = torch.from_numpy(Xq).to("cuda:0")
            Y5 = oracle.spmm(A5, Xq.astype(np.float64))
            Y = spx.bcsr_spmm(B, Xd, values=vals)
            Yh = Y.cpu().numpy()
            for j in (0, k // 2, k - 1):
                S = oracle.spmv_abs(A5, Xq[:, j].astype(np.float64))
                check_bound(Yh[:, j], Y5[:, j], S, L, 1 << 30, (name, vdtype, a, k, j))
            Yp = spx.bcsr_spmm(B, Xd, values=vals, row_period=max(spx.bandwidth(to_gpu(A5)), 1))
            assert torch.equal(Y.view(torch.uint8), Yp.view(torch.uint8)), (name, vdtype, a, k)
    Ai = int_valued(mats["stencil27"], 34)
    Bi = spx.BCSR.from_csr(to_gpu(Ai), a, 1)
    Xi = spgen.small_ints(Ai.n * 8, 35).reshape(Ai.n, 8)
    Y = spx.bcsr_spmm(Bi, torch.from_numpy(Xi.astype(np.float32)).to("cuda:0"), values=Bi.bvals.to(vt))
    assert np.array_equal(Y.double().cpu().numpy(), oracle.spmm(Ai, Xi))
    with pytest.raises(ValueError):   # FP32 values take FP32 X
        spx.bcsr_spmm(Bi, torch.from_numpy(Xi).to("cuda:0"), values=Bi.bvals.float())
