"""The library driven from plain C (tests/c_client/spx_client.c): include/spx.h
and the HIP runtime's C API only, no Python binding and no torch in the
process.  The client assembles the CRS arrays (Sec. 3) on the host and on the
device and compares them byte for byte, validates them, runs SpMV, SpMM
(Sec. 5), the CSC-index and atomic transposes and the sampled dot, and checks
two error returns; this test compares what it writes with the oracle."""
import importlib.util
import os
import subprocess

import numpy as np
import pytest

import oracle
import spgen

HERE = os.path.dirname(os.path.abspath(__file__))


def _load_builder():
    spec = importlib.util.spec_from_file_location("spx_c_client_build", os.path.join(HERE, "c_client", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


client_build = _load_builder()


@pytest.fixture(scope="module")
def client():
    return client_build.build()


def test_client_version_without_gpu(client):
    """The C client links libspx.so and reads its version with no HIP call."""
    r = subprocess.run([client, "--version"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    assert "gfx950" in r.stdout


def write_input(path, m, n, r, c, v, x, X, dy):
    k = X.shape[1]
    with open(path, "wb") as f:
        np.array([m, n, len(r), k], dtype="<i4").tofile(f)
        r.astype("<i4").tofile(f)
        c.astype("<i4").tofile(f)
        v.astype("<f8").tofile(f)
        x.astype("<f8").tofile(f)
        np.ascontiguousarray(X).astype("<f8").tofile(f)
        dy.astype("<f8").tofile(f)


def read_output(path, m, n, k):
    raw = open(path, "rb").read()
    off = 0

    def take(dtype, count):
        nonlocal off
        a = np.frombuffer(raw, dtype=dtype, count=count, offset=off)
        off += a.nbytes
        return a

    nnz = int(take("<i4", 1)[0])
    out = {"nnz": nnz, "rowptr": take("<i4", m + 1), "colind": take("<i4", nnz), "values": take("<f8", nnz),
           "y": take("<f8", m), "Y": take("<f8", m * k).reshape(m, k), "dx": take("<f8", n),
           "dx_atomic": take("<f8", n), "dvalues": take("<f8", nnz)}
    assert off == len(raw)
    return out


@pytest.mark.gpu
@pytest.mark.parametrize("shape", ["powerlaw", "duplicates"])
def test_client_products_against_oracle(client, tmp_path, shape):
    """Assembly bit-exact; FP64 SpMV, SpMM (k = 16), both transposes and the
    sampled dot within rel2 1e-12 of the oracle."""
    if shape == "powerlaw":
        coo = spgen.powerlaw(30_000, 20_000, 2.0, 4_000, 12.0, seed=3)
        m, n, r, c, v = coo.m, coo.n, coo.r, coo.c, coo.v
    else:  # every triplet three times, shuffled: duplicates summed in input order
        rng = np.random.default_rng(4)
        m, n, t = 5_000, 7_000, 40_000
        r0, c0 = rng.integers(0, m, t), rng.integers(0, n, t)
        idx = rng.permutation(3 * t)
        r, c = np.tile(r0, 3)[idx].astype(np.int32), np.tile(c0, 3)[idx].astype(np.int32)
        v = spgen.uniform(3 * t, 5)
    k = 16
    x = spgen.uniform(n, 6)
    X = spgen.uniform(n * k, 7).reshape(n, k)
    dy = spgen.normal(m, 8)
    fin, fout = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    write_input(fin, m, n, r, c, v, x, X, dy)
    print(f"spx_client {shape}: m={m} n={n} triplets={len(r)}", flush=True)
    p = subprocess.run([client, fin, fout], capture_output=True, text=True, timeout=120)
    assert p.returncode == 0, (p.returncode, p.stdout, p.stderr)
    got = read_output(fout, m, n, k)
    A = oracle.csr_from_coo(m, n, r, c, v)
    assert got["nnz"] == A.nnz
    assert np.array_equal(got["rowptr"], A.rowptr)
    assert np.array_equal(got["colind"], A.colind)
    assert np.array_equal(got["values"].view(np.uint64), A.values.view(np.uint64))
    assert oracle.rel2(got["y"], oracle.spmv(A, x)) <= 1e-12
    Yr = oracle.spmm(A, X)
    for j in range(k):
        assert oracle.rel2(got["Y"][:, j], Yr[:, j]) <= 1e-12, j
    dxr = oracle.spmv_t(A, dy)
    assert oracle.rel2(got["dx"], dxr) <= 1e-12
    assert oracle.rel2(got["dx_atomic"], dxr) <= 1e-12
    assert oracle.rel2(got["dvalues"], oracle.sddmm(A, dy, x)) <= 1e-12
