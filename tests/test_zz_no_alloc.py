"""csr_values_to_csc_noalloc (staging in the library's fixed device array)
against csr_values_to_csc (staging from the caller), called through the C ABI:
the same bits, on two calls in a row with the second on a smaller matrix
(the array keeps the first call's contents), for every value type; both
equal values[perm] element by element.  Sizes above the array are refused
before any launch."""
import ctypes

import numpy as np
import pytest

import spgen
from _cases import to_gpu
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def spx():
    import paper_1302_1078_amd as m
    return m


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def matrix_and_map(spx, m, n, mean, seed):
    coo = spgen.powerlaw(m, n, 2.0, min(n, 4000), mean, seed)
    A = oracle.csr_from_coo(coo.m, coo.n, coo.r, coo.c, coo.v)
    G = to_gpu(A)
    idx = spx.transpose_index(G)
    return A, G, idx, spx.csc_value_map(idx)


@pytest.mark.parametrize("vname", ["f64", "f32", "bf16"])
def test_noalloc_matches_values_to_csc(spx, torch, vname):
    from paper_1302_1078_amd import _lib
    L = _lib.load()
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[vname]
    code = {"f64": _lib.SPX_F64, "f32": _lib.SPX_F32, "bf16": _lib.SPX_BF16}[vname]
    # the second call is smaller, so stale staging from the first call lies
    # beyond its range and must not leak into its result
    for m, n, mean, seed in ((60_000, 50_000, 20.0, 1), (9_000, 7_000, 6.0, 2)):
        A, G, idx, vmap = matrix_and_map(spx, m, n, mean, seed)
        vals = G.values.to(tdt)
        nnz = A.nnz
        staging = torch.empty(nnz, dtype=tdt, device="cuda:0")
        ref = torch.empty(nnz, dtype=tdt, device="cuda:0")
        out = torch.full((nnz,), 7.0, dtype=tdt, device="cuda:0")
        st = _stream(torch)
        assert L.csr_values_to_csc(nnz, _ptr(vmap.dest), _ptr(vmap.local), _ptr(vals), code, _ptr(staging),
                                   _ptr(ref), st) == 0, _lib.last_error()
        assert L.csr_values_to_csc_noalloc(nnz, _ptr(vmap.dest), _ptr(vmap.local), _ptr(vals), code,
                                           _ptr(out), st) == 0, _lib.last_error()
        torch.cuda.synchronize()
        bits = torch.int64 if vname == "f64" else (torch.int32 if vname == "f32" else torch.int16)
        assert torch.equal(out.view(bits), ref.view(bits)), (vname, m)
        # both are values[perm]: the CSC order of the transpose index
        perm = idx.perm.long()
        assert torch.equal(out.view(bits), vals[perm].view(bits)), (vname, m)


def test_noalloc_size_limit(spx, torch):
    from paper_1302_1078_amd import _lib
    L = _lib.load()
    cap = _lib.SPX_NOALLOC_SCRATCH_BYTES
    dummy = torch.zeros(16, dtype=torch.int32, device="cuda:0")
    for code, size in ((_lib.SPX_F64, 8), (_lib.SPX_F32, 4), (_lib.SPX_BF16, 2)):
        over = cap // size + 1  # one value more than the array holds; refused before any launch
        s = L.csr_values_to_csc_noalloc(over, _ptr(dummy), _ptr(dummy), _ptr(dummy), code, _ptr(dummy),
                                        _stream(torch))
        assert s == _lib.SPX_ERR_UNSUPPORTED and "SPX_NOALLOC_SCRATCH_BYTES" in _lib.last_error()
    assert L.csr_values_to_csc_noalloc(-1, None, None, None, _lib.SPX_F32, None, None) == _lib.SPX_ERR_INVALID
    assert L.csr_values_to_csc_noalloc(0, None, None, None, _lib.SPX_F32, None, None) == _lib.SPX_OK
