"""Host logic of bench.py, no GPU needed: the one-GPU rule, the algorithmic
byte count of a product (the paper's application bandwidth, Sec. 4.2: every
matrix, vector and row-pointer byte touched once) and the rule that the
counter-measured traffic is reported only for the kernel sources it was
taken with."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_app_bytes_hand_count():
    # 3 x 4 matrix, 5 nonzeros, k = 2, FP64 values and vectors:
    # values 5 x 8 + colind 5 x 4 + rowptr 4 x 4 + X 4 x 2 x 8 + Y 3 x 2 x 8
    assert bench.app_bytes(3, 4, 5, k=2) == 40 + 20 + 16 + 64 + 48
    # BF16 values, FP32 vectors, k = 1
    assert bench.app_bytes(3, 4, 5, k=1, sv=2, sx=4) == 10 + 20 + 16 + 16 + 12
    # the headline matrix: 1,048,576 square, 16,776,698 nonzeros
    m = 1 << 20
    assert bench.app_bytes(m, m, 16776698) == 12 * 16776698 + 16 * m + 4 * (m + 1)


def test_traffic_only_for_matching_sources(monkeypatch, tmp_path):
    (tmp_path / "profiles").mkdir()
    with open(tmp_path / "profiles" / "traffic.json", "w") as f:
        json.dump({"k_product_spmm_c1": {"bytes_per_launch": 1234, "source_hash": "aaaa"}}, f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_hash", lambda: "aaaa")
    assert bench.traffic_for("k_product_spmm_c1") == 1234.0
    assert bench.traffic_for("k_product_spmv_c1") is None
    monkeypatch.setattr(bench, "source_hash", lambda: "bbbb")
    assert bench.traffic_for("k_product_spmm_c1") is None
    os.remove(tmp_path / "profiles" / "traffic.json")
    assert bench.traffic_for("k_product_spmm_c1") is None


def test_source_hash_covers_the_product_sources(monkeypatch, tmp_path):
    """Changing any of the product kernel sources changes the hash."""
    csrc = tmp_path / "paper_1302_1078_amd" / "csrc"
    csrc.mkdir(parents=True)
    names = ("product.hip", "product_impl.hpp", "device.hpp", "plan.hip")
    for n in names:
        (csrc / n).write_text(n)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.source_hash()
    for n in names:
        (csrc / n).write_text(n + " changed")
        assert bench.source_hash() != h0, n
        (csrc / n).write_text(n)
    assert bench.source_hash() == h0


def test_host_llc_bytes_reads_sysfs(monkeypatch):
    """Every distinct L3 (one per shared_cpu_list) is counted once."""
    files = {
        "/sys/devices/system/cpu/cpu0/cache/index3/size": "32768K",
        "/sys/devices/system/cpu/cpu0/cache/index3/shared_cpu_list": "0-1",
        "/sys/devices/system/cpu/cpu1/cache/index3/size": "32768K",
        "/sys/devices/system/cpu/cpu1/cache/index3/shared_cpu_list": "0-1",
        "/sys/devices/system/cpu/cpu2/cache/index3/size": "96M",
        "/sys/devices/system/cpu/cpu2/cache/index3/shared_cpu_list": "2",
    }
    import builtins
    import io
    real_open = builtins.open

    def fake_open(path, *a, **kw):
        if path in files:
            return io.StringIO(files[path])
        if str(path).startswith("/sys/devices/system/cpu/"):
            raise OSError(path)
        return real_open(path, *a, **kw)

    monkeypatch.setattr(bench.os, "sched_getaffinity", lambda pid: {0, 1, 2, 3})
    monkeypatch.setattr(builtins, "open", fake_open)
    assert bench.host_llc_bytes() == (32 << 20) + (96 << 20)


def test_cpu_baseline_protocol_small():
    """The CPU-baseline leg on a small matrix: 2 warm-up + reps timed calls on
    all threads and on one thread, LLC flushed, and the figures it reports
    consistent with its own timings."""
    import spgen
    coo = spgen.powerlaw(4000, 4000, 2.0, 500, 16.0, seed=0)
    x = spgen.uniform(coo.n, 0)
    X = spgen.uniform(coo.n * 4, 1).reshape(coo.n, 4)
    out = bench.cpu_baseline(coo, x, X, 4, 2 * 1000, 2 * 4000, 2)
    assert out["kind"] == "oracle" and out["llc_flushed"] is True
    assert out["repetitions"] == 2 and out["warmup"] == 2
    assert out["cores"] >= 1 and out["one_thread"]["threads"] == 1
    for r in (out, out["one_thread"]):
        assert r["spmv_gflops"] > 0 and r["spmm_gflops"] > 0
    one = out["one_thread"]
    assert abs(one["gflops"] - (2000 + 8000) / (one["spmv_ms"] + one["spmm_ms"]) / 1e6) < 1e-9 * one["gflops"]


def test_row_shards_balance_by_nonzeros():
    """The row-block partition: contiguous blocks covering every row once, each
    within one row's length of nnz/parts (a block boundary can only fall
    between rows), and degenerate inputs (fewer rows than parts, no
    nonzeros, one dominating row) still give parts + 1 ordered cuts."""
    import numpy as np
    rng = np.random.default_rng(3)
    for m, parts in ((1000, 8), (37, 8), (5, 8), (1, 8), (20000, 3)):
        L = rng.integers(0, 50, m)
        L[rng.integers(0, m)] = 5000   # one long row
        rowptr = np.concatenate([[0], np.cumsum(L)])
        cuts = bench.row_shards(rowptr, parts)
        assert len(cuts) == parts + 1 and cuts[0] == 0 and cuts[-1] == m
        assert all(a <= b for a, b in zip(cuts, cuts[1:]))
        nnz = int(rowptr[-1])
        for g in range(parts):
            # each cut is the first row boundary at or past g * nnz / parts
            if 0 < g:
                c = cuts[g]
                target = nnz * g // parts
                assert rowptr[c] >= target or c == m
                assert c == 0 or rowptr[c - 1] < target or cuts[g - 1] == c
        per = [int(rowptr[cuts[g + 1]] - rowptr[cuts[g]]) for g in range(parts)]
        assert sum(per) == nnz
        assert max(per) <= nnz / parts + L.max() + 1
    assert bench.row_shards(np.zeros(11, dtype=np.int64), 4) == [0, 0, 0, 0, 10]
