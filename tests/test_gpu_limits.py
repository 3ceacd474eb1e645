"""Products at the largest supported size: nnz = SPX_MAX_NNZ (2^31 - 2^25),
so the last rows' nonzeros sit at the top of the int32 position range that
the kernels' look-ahead and split segments must not overflow.

The matrix is built on the device (about 17 GB in FP32): rows of 1,024
nonzeros (a 256-lane bin), then a short row (stream bin), a 100,000-nonzero
row (split segments) and a short last row, with colind[p] = p mod n and every
value 1.  With small-integer x each y_i is an exact integer sum, checked on
sampled rows (first, middle, the last four) against the host's sum of the
same x entries; the rows in between are checked by their closed form where x
is all ones.  The SpMV runs through the default plan, no plan, and the default
plan with hot x (65,536 columns; its copy of the column indices spans the
same int32 positions)."""
import numpy as np
import pytest

import spgen

pytestmark = pytest.mark.gpu

MAX_NNZ = 2**31 - 2**25
N = 1 << 20


@pytest.fixture(scope="module")
def big():
    import torch

    import paper_1302_1078_amd as spx
    free, _ = torch.cuda.mem_get_info(0)
    if free < 40 * 2**30:
        pytest.skip(f"needs 40 GiB of free device memory ({free / 2**30:.0f} GiB free)")
    tail = [17, 100_000, 33]
    body = MAX_NNZ - sum(tail)
    rows_body = body // 1024
    lens = [1024] * rows_body
    rem = body - 1024 * rows_body
    if rem:
        lens.append(rem)
    lens += tail
    lens = np.array(lens, dtype=np.int64)
    assert lens.sum() == MAX_NNZ
    m = lens.size
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lens, out=rowptr[1:])
    dev = torch.device("cuda", 0)
    print(f"building m={m} nnz={MAX_NNZ} on the device", flush=True)
    colind = torch.arange(0, MAX_NNZ, dtype=torch.int32, device=dev)
    colind.remainder_(N)
    values = torch.ones(MAX_NNZ, dtype=torch.float32, device=dev)
    A = spx.CSR(torch.from_numpy(rowptr.astype(np.int32)).to(dev), colind, values, (m, N))
    yield spx, torch, A, rowptr
    del A, colind, values
    torch.cuda.empty_cache()


def expected(rowptr, rows, x):
    out = []
    for i in rows:
        p = np.arange(rowptr[i], rowptr[i + 1], dtype=np.int64) % N
        out.append(x[p].astype(np.float64).sum())
    return np.array(out)


def test_spmv_at_max_nnz(big):
    spx, torch, A, rowptr = big
    m = A.m
    x = spgen.small_ints(N, 21).astype(np.float32)
    xd = torch.from_numpy(x).to("cuda:0")
    sample = [0, 1, m // 2, m - 4, m - 3, m - 2, m - 1]
    want = expected(rowptr, sample, x)
    ones = torch.ones(N, dtype=torch.float32, device="cuda:0")
    hot = spx.Plan.for_matrix(A).attach_hot_x(A, 65536, xdtype=torch.float32)   # the benchmark's SpMV plan form
    for name, plan in (("default", spx.Plan.for_matrix(A)), ("none", None), ("hot_x", hot)):
        print(f"spmv plan={name}", flush=True)
        y = spx.spmv(A, xd, plan=plan).cpu().numpy()
        assert np.array_equal(y[sample].astype(np.float64), want), name
        y1 = spx.spmv(A, ones, plan=plan).cpu().numpy()
        assert np.array_equal(y1.astype(np.int64), np.diff(rowptr)), name


def test_spmm_at_max_nnz(big):
    spx, torch, A, rowptr = big
    m, k = A.m, 4
    X = spgen.small_ints(N * k, 22).reshape(N, k).astype(np.float32)
    Xd = torch.from_numpy(X).to("cuda:0")
    sample = [0, m // 2, m - 3, m - 2, m - 1]
    print("spmm k=4 default plan", flush=True)
    Y = spx.spmm(A, Xd, plan=spx.Plan.for_matrix(A, k=k)).cpu().numpy()
    for j in range(k):
        assert np.array_equal(Y[sample, j].astype(np.float64), expected(rowptr, sample, X[:, j])), j
