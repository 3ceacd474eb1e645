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
