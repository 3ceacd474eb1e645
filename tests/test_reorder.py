"""Ordering and structure metrics of the library (host functions of the C ABI:
csr_rcm, csr_vector_access, csr_ucld) against the pinned oracle.

These entry points run on the host, so they are checked here without a GPU;
csr_permute (device) is checked in test_gpu_reorder.py.
"""
import numpy as np
import pytest
import torch

import oracle
import spgen


@pytest.fixture(scope="module")
def spx():
    import paper_1302_1078_amd as m
    return m


def host_csr(spx, A):
    return spx.CSR(torch.from_numpy(A.rowptr), torch.from_numpy(A.colind),
                   torch.from_numpy(A.values), (A.m, A.n))


def cases():
    rng = np.random.default_rng(50)
    out = []
    for n, nnz in [(1, 1), (5, 3), (60, 150), (400, 1500)]:
        r = rng.integers(0, n, nnz).astype(np.int32)
        c = rng.integers(0, n, nnz).astype(np.int32)
        out.append(("random%d" % n, spgen.COO(n, n, r, c, np.ones(nnz), {})))
    out.append(("stencil5", spgen.relabeled(spgen.stencil5(40, 31, 1), 2)))
    out.append(("stencil27", spgen.relabeled(spgen.stencil3d(9, 8, 7, 27, 3), 4)))
    out.append(("powerlaw", spgen.powerlaw(6000, 6000, 2.0, 2000, 12.0, 5)))
    n = 50
    out.append(("isolated", spgen.COO(n, n, np.arange(n, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n), {})))
    return out


@pytest.mark.parametrize("name,coo", cases(), ids=[c[0] for c in cases()])
def test_rcm_matches_oracle(spx, name, coo):
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    perm = spx.rcm(host_csr(spx, A)).numpy()
    assert np.array_equal(perm, oracle.rcm(A)), name


def test_rcm_rejects_bad_input(spx):
    A = oracle.csr_from_coo(3, 4, np.array([0, 1], np.int32), np.array([1, 3], np.int32), np.ones(2))
    with pytest.raises(spx.SpxError):
        spx.rcm(host_csr(spx, A))
    B = oracle.csr_from_coo(4, 4, np.array([0, 1], np.int32), np.array([1, 3], np.int32), np.ones(2))
    bad = spx.CSR(torch.from_numpy(B.rowptr), torch.tensor([1, 9], dtype=torch.int32),
                  torch.from_numpy(B.values), (4, 4))
    with pytest.raises(spx.SpxError):
        spx.rcm(bad)


@pytest.mark.parametrize("name,coo", cases(), ids=[c[0] for c in cases()])
def test_metrics_match_oracle(spx, name, coo):
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    H = host_csr(spx, A)
    for line, parts, chunk in [(16, 8, 64), (8, 61, 64), (4, 3, 1)]:
        assert spx.vector_access(H, line, parts, chunk) == oracle.vector_access(A, line, parts, chunk)
    for line in (8, 16):
        assert spx.ucld(H, line) == oracle.ucld(A, line)
    for line, tile in [(16, 256), (8, 7), (1, 1), (4, 5000)]:
        assert spx.tile_lines(H, line, tile) == oracle.tile_lines(A, line, tile)
