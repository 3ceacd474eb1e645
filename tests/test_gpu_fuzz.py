"""Seeded random configurations against the oracle: plan options (bins,
thresholds, lane widths, stream and split bins, split chunk, compensation
threshold, flags), SpMM width, value type and matrix kind are drawn from a
fixed seed per case, so every run checks the same 60 combinations.  Each
product must meet the per-row error bound: FP64 2(L + 2) 2^-53 sum |a x|;
FP32 / BF16 the precision-form bounds against the quantised inputs."""
import numpy as np
import pytest

import oracle
import spgen
from _cases import check_bound, matrix, quantised

pytestmark = pytest.mark.gpu

LANES = [1, 2, 4, 8, 16, 32, 64, 256, 512]
FLAGS = [1, 2, 4, 8, 16]  # NO_NT_STORE, SCALAR_X, NO_XCD_MAP, ONE_ROW, KEEP_STREAM
KINDS = ["powerlaw", "stencil27", "stencil5", "empty_rows", "one_long_row", "tall", "wide", "uniform"]


@pytest.fixture(scope="module")
def spx():
    import paper_1302_1078_amd as m
    return m


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def random_opts(spx, rng, k):
    nb = int(rng.integers(1, 7))
    upper = sorted(rng.choice(np.arange(1, 3000), nb - 1, replace=False).tolist())
    lanes = [int(rng.choice(LANES)) for _ in range(nb)]
    if nb > 1 and rng.random() < 0.6:
        lanes[-1] = 0  # split bin
    flags = 0
    for f in FLAGS:
        if rng.random() < 0.25:
            flags |= f
    return spx.PlanOpts.from_dict({
        "nbins": nb, "upper": upper, "lanes": lanes,
        "split_chunk": int(rng.choice([256, 300, 1024, 4096])),
        "kahan_len": int(rng.choice([4, 64, 256, 100000])),
        "max_k": k, "flags": flags})


@pytest.mark.parametrize("case", range(60))
def test_random_configuration(spx, torch, case):
    rng = np.random.default_rng(1000 + case)
    kind = KINDS[int(rng.integers(len(KINDS)))]
    A = matrix(kind, seed=int(rng.integers(1 << 16)))
    k = int(rng.choice([1, 1, 2, 3, 4, 8, 16, 33]))
    vname = str(rng.choice(["f64", "f32", "bf16"]))
    opts = random_opts(spx, rng, k)
    X = spgen.uniform(A.n * k, int(rng.integers(1 << 16))).reshape(A.n, k)
    what = (case, kind, k, vname, opts.to_dict())
    if vname == "f64":
        G = spx.CSR(*(torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
                      for a in (A.rowptr, A.colind, A.values)), (A.m, A.n))
        Xd = torch.from_numpy(X).to("cuda:0")
        wideA, Xw = A, X
    else:
        G, wideA = quantised(A, vname, torch)
        Xw = spgen.to_f32(X).astype(np.float64)
        Xd = torch.from_numpy(spgen.to_f32(X)).to("cuda:0")
    plan = spx.Plan.for_matrix(G, opts)
    if k == 1:
        y = spx.spmv(G, Xd[:, 0].contiguous(), plan=plan).double().cpu().numpy()[:, None]
    else:
        y = spx.spmm(G, Xd, plan=plan).double().cpu().numpy()
    L = A.row_lengths()
    absA = oracle.CSR(A.m, A.n, A.rowptr, A.colind, np.abs(wideA.values))
    for j in range(k):
        ref = oracle.spmv(wideA, Xw[:, j])
        S = oracle.spmv(absA, np.abs(Xw[:, j]))
        if vname == "f64":
            assert (np.abs(y[:, j] - ref) <= 2.0 * (L + 2.0) * 2.0 ** -53 * S).all(), (what, j)
        else:
            check_bound(y[:, j], ref, S, L, opts.kahan_len, (what, j))
