"""Host logic of the autotuner, with the GPU timing replaced by fixed times:
the default plan (first candidate) is kept unless another is faster by the
margin; with batch=True candidates are timed inside a batch, with stream
bins kept as tiles, and returned without that flag; decisions are cached
under a key that carries the tuner's settings."""
import json
from types import SimpleNamespace

import pytest
import torch


@pytest.fixture()
def fake_matrix():
    rowptr = torch.tensor([0, 2, 3, 5], dtype=torch.int32)
    colind = torch.tensor([0, 2, 1, 0, 2], dtype=torch.int32)
    values = torch.ones(5, dtype=torch.float64)
    return SimpleNamespace(m=3, n=3, nnz=5, rowptr=rowptr, colind=colind, values=values)


def run_tune(monkeypatch, A, rel_times, **kw):
    from paper_1302_1078_amd import autotune
    seen = []

    def fake_time(A_, X_, opts, reps=5, calls=8):
        i = len(seen)
        seen.append(opts)
        return 1.0 * rel_times[i] if i < len(rel_times) else 1.0

    monkeypatch.setattr(autotune, "time_opts", fake_time)
    monkeypatch.setattr(autotune, "time_in_batch", fake_time)
    x = torch.ones(3, dtype=torch.float64)
    best, rep = autotune.tune(A, x, **kw)
    return best, rep, seen


def test_default_kept_unless_clearly_faster(monkeypatch, fake_matrix):
    from paper_1302_1078_amd import autotune
    n = len(autotune.candidates(1))
    best, rep, _ = run_tune(monkeypatch, fake_matrix, [1.0] * n)
    assert rep["choice"] == 0
    times = [1.0] * n
    times[2] = 0.97  # 3 % faster: within the 5 % margin, the default stays
    assert run_tune(monkeypatch, fake_matrix, times)[1]["choice"] == 0
    times[2] = 0.90  # 10 % faster: chosen
    best, rep, _ = run_tune(monkeypatch, fake_matrix, times)
    assert rep["choice"] == 2
    assert best.to_dict() == autotune.candidates(1)[2].to_dict()
    assert run_tune(monkeypatch, fake_matrix, times, margin=0.2)[1]["choice"] == 0


def test_batch_timing_keeps_stream_tiles(monkeypatch, fake_matrix):
    from paper_1302_1078_amd._lib import SPX_FLAG_KEEP_STREAM
    best, _, seen = run_tune(monkeypatch, fake_matrix, [], batch=True)
    assert seen and all(o.flags & SPX_FLAG_KEEP_STREAM for o in seen)
    assert not (best.flags & SPX_FLAG_KEEP_STREAM)
    _, _, seen = run_tune(monkeypatch, fake_matrix, [], batch=False)
    assert not any(o.flags & SPX_FLAG_KEEP_STREAM for o in seen)


def test_cache_key_carries_settings(monkeypatch, fake_matrix, tmp_path):
    from paper_1302_1078_amd import autotune
    cache = str(tmp_path / "tune.json")
    n = len(autotune.candidates(1))
    times = [1.0] * n
    times[1] = 0.5
    best, rep, _ = run_tune(monkeypatch, fake_matrix, times, cache_path=cache)
    assert rep["choice"] == 1 and not rep["cached"]
    _, rep2, seen = run_tune(monkeypatch, fake_matrix, times, cache_path=cache)
    assert rep2["cached"] and not seen  # reused, nothing timed
    _, rep3, seen = run_tune(monkeypatch, fake_matrix, times, cache_path=cache, margin=0.01)
    assert not rep3["cached"] and seen  # other settings: tuned again
    assert len(json.load(open(cache))) == 2


def test_banded_candidate_for_single_spmm(monkeypatch, fake_matrix):
    """Single SpMM products (batch=False, k > 1) also time the default plan with
    rows ordered by the matrix's bandwidth; batches and SpMV do not, nor does a
    bandwidth that leaves the order ascending."""
    from paper_1302_1078_amd import autotune
    seen = []
    monkeypatch.setattr(autotune, "time_opts", lambda A_, X_, o, reps=5, calls=8: seen.append(o) or 1.0)
    monkeypatch.setattr(autotune, "time_in_batch", lambda A_, X_, o, reps=5, calls=8: seen.append(o) or 1.0)
    monkeypatch.setattr(autotune, "bandwidth", lambda A_: 1)
    X = torch.ones((3, 4), dtype=torch.float64)
    n = len(autotune.candidates(4))
    autotune.tune(fake_matrix, X, batch=False)
    assert len(seen) == n + 1 and seen[-1].row_period == 1 and all(o.row_period == 0 for o in seen[:-1])
    seen.clear()
    autotune.tune(fake_matrix, X, batch=True)
    assert len(seen) == n and all(o.row_period == 0 for o in seen)
    seen.clear()
    autotune.tune(fake_matrix, torch.ones(3, dtype=torch.float64), batch=False)
    assert all(o.row_period == 0 for o in seen)
    seen.clear()
    monkeypatch.setattr(autotune, "bandwidth", lambda A_: 3)   # >= m: ascending anyway
    autotune.tune(fake_matrix, X, batch=False)
    assert len(seen) == n


def test_batch_and_single_timing_paths(monkeypatch, fake_matrix):
    """batch=True times candidates inside a batch (time_in_batch), batch=False
    as single products (time_opts); neither calls the other."""
    from paper_1302_1078_amd import autotune
    calls = {"batch": 0, "single": 0}

    def tb(A_, X_, o, reps=5, calls_=8):
        calls["batch"] += 1
        return 1.0

    def ts(A_, X_, o, reps=5, calls_=8):
        calls["single"] += 1
        return 1.0

    monkeypatch.setattr(autotune, "time_in_batch", tb)
    monkeypatch.setattr(autotune, "time_opts", ts)
    x = torch.ones(3, dtype=torch.float64)
    autotune.tune(fake_matrix, x, batch=True)
    assert calls["batch"] == len(autotune.candidates(1)) and calls["single"] == 0
    autotune.tune(fake_matrix, x, batch=False)
    assert calls["single"] == len(autotune.candidates(1))


def test_tune_batch_accepts_a_group_only_if_the_batch_gets_faster(monkeypatch):
    """Per-matrix picks are kept per SpMM width only when the whole batch's
    time drops by the margin; otherwise that group keeps its defaults."""
    from paper_1302_1078_amd import autotune
    from paper_1302_1078_amd._lib import PlanOpts
    mats = [SimpleNamespace(m=3, n=3, nnz=5, values=torch.ones(5, dtype=torch.float32)) for _ in range(4)]
    Xs = [torch.ones(3), torch.ones(3, 4), torch.ones(3), torch.ones(3, 4)]

    def pick(A, X, reps=3, cache_path=None):
        k = 1 if X.dim() == 1 else X.shape[1]
        d = autotune.default_opts(k, torch.float32).to_dict()
        d["split_chunk"] = 1024
        return PlanOpts.from_dict(d), {}

    monkeypatch.setattr(autotune, "tune", pick)

    def fake_batch(ms, xs, opts, reps=5, calls=4):
        # the k = 1 picks make the batch 10 % faster, the k = 4 picks 10 % slower
        t = 1.0
        for X, o in zip(xs, opts):
            if o.split_chunk == 1024:
                t *= 0.95 if X.dim() == 1 else 1.05
        return t

    monkeypatch.setattr(autotune, "time_batch", fake_batch)
    chosen, rep = autotune.tune_batch(mats, Xs)
    assert [o.split_chunk for o in chosen] == [1024, autotune.default_opts(4).split_chunk,
                                               1024, autotune.default_opts(4).split_chunk]
    assert rep["groups"][1]["accepted"] and not rep["groups"][4]["accepted"]
    assert rep["changed_per_matrix"] == 4 and rep["accepted_matrices"] == 2
