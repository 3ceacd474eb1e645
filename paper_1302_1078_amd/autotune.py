"""Per-matrix autotuner for plan options (bin thresholds, lanes per row,
split chunk, and for single SpMM products of banded matrices the row order).

Candidates are timed on the GPU with HIP events: each sample brackets `calls`
back-to-back launches of csr_spmv / csr_spmm on the current stream (so the
launch overhead of a small matrix does not decide), and the median of `reps`
samples counts.  With batch=True (the default; the batch is what the tuner
serves) the candidates are timed as a batch runs them, stream bins kept as
256-row tiles (SPX_FLAG_KEEP_STREAM).  The default plan (the first candidate)
is kept unless another is faster by at least `margin`: measured on the
256-matrix batch, picking the bare fastest single launch made the batch 5 %
slower than the defaults.  Decisions are cached in a JSON file keyed by a
hash of the sparsity structure, k, the value dtype and the tuner's settings;
an unreadable or mismatched cache entry is ignored (the matrix is tuned
again, or the default heuristic is used when tuning is off).
"""
from __future__ import annotations

import hashlib
import json
import os

import torch

from ._lib import SPX_FLAG_KEEP_STREAM, PlanOpts
from .ops import CSR, Plan, bandwidth, default_opts, spmm, spmv

STREAM = 512  # SPX_LANES_STREAM


TUNER_VERSION = 3  # part of the cache key: decisions of other tuner versions are not reused


def structure_key(A: CSR, k: int, setting: str = "") -> str:
    h = hashlib.sha1()
    h.update(f"v{TUNER_VERSION}:{setting}:{A.m}x{A.n}:{A.nnz}:k{k}:{A.values.dtype}".encode())
    h.update(A.rowptr.cpu().numpy().tobytes())
    if A.nnz:
        step = max(1, A.nnz // 65536)
        h.update(A.colind[::step].cpu().numpy().tobytes())
    return h.hexdigest()


def _copy(o: PlanOpts) -> PlanOpts:
    return PlanOpts.from_dict(o.to_dict())


def candidates(k: int, vdtype=torch.float64) -> list:
    """A small family around the defaults: lane widths halved / doubled,
    split chunk halved / doubled, split disabled, and a coarse 3-bin plan."""
    base = default_opts(k, vdtype)
    out = [base]
    half = _copy(base)
    dbl = _copy(base)
    for b in range(base.nbins):
        l = base.lanes[b]
        if l and l != STREAM:
            half.lanes[b] = max(1, l // 2) if l != 256 else 64
            dbl.lanes[b] = min(64, l * 2) if l < 64 else 256
    out += [half, dbl]
    if base.lanes[base.nbins - 1] == 0:
        for f in (0.5, 2.0):
            c = _copy(base)
            c.split_chunk = max(256, int(base.split_chunk * f))
            out.append(c)
        nosplit = _copy(base)
        nosplit.lanes[base.nbins - 1] = 256
        out.append(nosplit)
    if k == 1:
        # row groups of 1..32 lanes for the short rows instead of a stream bin
        sub = PlanOpts.from_dict({"nbins": 9, "upper": [1, 2, 4, 8, 16, 32, 128, 2048],
                                  "lanes": [1, 2, 4, 8, 16, 32, 64, 256, 0],
                                  "split_chunk": base.split_chunk, "kahan_len": base.kahan_len,
                                  "max_k": k, "flags": 0})
        out.append(sub)
    coarse = PlanOpts.from_dict({"nbins": 3, "upper": [8, 256], "lanes": [1 if k > 1 else STREAM, 64, 0],
                                 "split_chunk": base.split_chunk, "kahan_len": base.kahan_len,
                                 "max_k": k, "flags": 0})
    out.append(coarse)
    return out


def banded_candidate(A: CSR, base: PlanOpts) -> PlanOpts | None:
    """base with rows ordered band by band of A's bandwidth (row_period), or
    None when the bandwidth is 0 or leaves the rows ascending (>= m)."""
    P = bandwidth(A)
    if P <= 0 or P >= A.m:
        return None
    c = _copy(base)
    c.row_period = P
    return c


def load_cache(path: str | None) -> dict:
    if not path or not os.path.exists(path):
        return {}
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def _valid(entry) -> PlanOpts | None:
    try:
        o = PlanOpts.from_dict(entry["opts"])
        if not (1 <= o.nbins <= 12) or len(entry["opts"]["lanes"]) != o.nbins:
            return None
        return o
    except (KeyError, TypeError, ValueError):
        return None


def time_opts(A: CSR, X: torch.Tensor, opts: PlanOpts, reps: int = 5, calls: int = 8) -> float:
    """Median over `reps` samples of the time per call, each sample timing
    `calls` back-to-back launches (ms)."""
    plan = Plan.for_matrix(A, opts)
    vec = X.dim() == 1
    out = torch.empty((A.m,) if vec else (A.m, X.shape[1]), dtype=X.dtype, device=X.device)
    call = (lambda: spmv(A, X, y=out, plan=plan)) if vec else (lambda: spmm(A, X, Y=out, plan=plan))
    call()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(calls):
            call()
        e1.record()
        ts.append((e0, e1))
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) / calls for a, b in ts)
    return ms[len(ms) // 2]


def tune(A: CSR, X: torch.Tensor, reps: int = 5, cache_path: str | None = None,
         cands: list | None = None, batch: bool = True, margin: float = 0.05) -> tuple:
    """Return (best PlanOpts, report dict).  X is x (1-D) or X (n x k).  The
    first candidate is the baseline that another must beat by `margin`."""
    k = 1 if X.dim() == 1 else X.shape[1]
    key = structure_key(A, k, f"batch={int(batch)}:margin={margin}")
    cache = load_cache(cache_path)
    if key in cache:
        o = _valid(cache[key])
        if o is not None:
            return o, {"cached": True, "ms": cache[key].get("ms")}
    if cands is None:
        cands = candidates(k, A.values.dtype)
        if not batch and k > 1:
            # a batch deals tiles across matrices, so the per-XCD bands of a
            # row period only apply to single products
            b = banded_candidate(A, cands[0])
            if b is not None:
                cands.append(b)
    timed = []
    for o in cands:
        c = _copy(o)
        if batch:
            c.flags |= SPX_FLAG_KEEP_STREAM
        timed.append(c)
    times = [time_opts(A, X, o, reps) for o in timed]
    best = min(range(len(cands)), key=lambda i: times[i])
    if times[best] > times[0] * (1.0 - margin):
        best = 0
    report = {"cached": False, "ms": times[best], "all_ms": times, "choice": best}
    if cache_path:
        cache[key] = {"opts": cands[best].to_dict(), "ms": times[best]}
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f)
        os.replace(tmp, cache_path)
    return cands[best], report
