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


TUNER_VERSION = 4  # part of the cache key: decisions of other tuner versions are not reused


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


def time_in_batch(A: CSR, X: torch.Tensor, opts: PlanOpts, reps: int = 5, calls: int = 8,
                  fill_tiles: int = 4096, max_copies: int = 64) -> float:
    """Time per copy (ms) of `opts` inside a batch that fills the chip: the
    matrix alone when its tiles already do, otherwise enough copies of it
    (same A and X, separate outputs) to reach about `fill_tiles` tiles.  In
    a batch of many matrices the grid is full, so what a plan costs there is
    its throughput, not the latency of its own few tiles; timing a small
    matrix alone would reward plans that only add parallelism."""
    from .batch import Batched
    one = Batched([A], [X], opts=[opts])
    tiles = max(1, one.info()["tiles"])
    copies = max(1, min(max_copies, -(-fill_tiles // tiles)))
    B = one if copies == 1 else Batched([A] * copies, [X] * copies, opts=[opts] * copies)
    B.run()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(calls):
            B.run()
        e1.record()
        ts.append((e0, e1))
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) / calls for a, b in ts)
    return ms[len(ms) // 2] / copies


def tune(A: CSR, X: torch.Tensor, reps: int = 5, cache_path: str | None = None,
         cands: list | None = None, batch: bool = True, margin: float = 0.05) -> tuple:
    """Return (best PlanOpts, report dict).  X is x (1-D) or X (n x k).  The
    first candidate is the baseline that another must beat by `margin`.
    With batch=True each candidate is timed as the batch runs it, inside a
    batch that fills the chip (time_in_batch); otherwise as a single
    product (time_opts)."""
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
    times = [time_in_batch(A, X, o, reps) if batch else time_opts(A, X, o, reps) for o in timed]
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


def time_batch(mats: list, Xs: list, opts: list, reps: int = 5, calls: int = 4) -> float:
    """Median time (ms) of one run of the whole batch with these options,
    over `reps` samples of `calls` back-to-back runs."""
    from .batch import Batched
    B = Batched(mats, Xs, opts=opts)
    B.run()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(calls):
            B.run()
        e1.record()
        ts.append((e0, e1))
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) / calls for a, b in ts)
    return ms[len(ms) // 2]


def tune_batch(mats: list, Xs: list, reps: int = 3, margin: float = 0.01, rounds: int = 3,
               cache_path: str | None = None) -> tuple:
    """Plan options for a batch: each matrix's own choice (tune with
    batch=True), accepted for a group of matrices only if the whole batch
    gets faster with it.  A group is the matrices of one SpMM width (they
    share a launch).  Per-matrix timings cannot see how the choices combine
    in one launch ordered heaviest tile first (a plan with fewer, heavier
    tiles can lengthen the launch's tail), so every group's change is
    checked on the batch as it runs: the current and the trial options are
    timed alternately `rounds` times, and the trial is kept only if its
    median is faster by `margin`.  Returns (options per matrix, report)."""
    ks = [1 if X.dim() == 1 else X.shape[1] for X in Xs]
    picks = [tune(A, X, reps=reps, cache_path=cache_path)[0] for A, X in zip(mats, Xs)]
    chosen = [default_opts(k, A.values.dtype) for A, k in zip(mats, ks)]
    report = {"changed_per_matrix": sum(p.to_dict() != c.to_dict() for p, c in zip(picks, chosen)), "groups": {}}
    for kk in sorted(set(ks)):
        idx = [i for i, k in enumerate(ks) if k == kk and picks[i].to_dict() != chosen[i].to_dict()]
        if not idx:
            continue
        trial = list(chosen)
        for i in idx:
            trial[i] = picks[i]
        cur_t, new_t = [], []
        for _ in range(rounds):
            cur_t.append(time_batch(mats, Xs, chosen))
            new_t.append(time_batch(mats, Xs, trial))
        cur, new = sorted(cur_t)[rounds // 2], sorted(new_t)[rounds // 2]
        keep = new < cur * (1.0 - margin)
        report["groups"][kk] = {"matrices_changed": len(idx), "batch_ms": cur, "trial_ms": new, "accepted": keep}
        if keep:
            chosen = trial
    report["accepted_matrices"] = sum(c.to_dict() != default_opts(k, A.values.dtype).to_dict()
                                      for A, k, c in zip(mats, ks, chosen))
    return chosen, report
