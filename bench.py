#!/usr/bin/env python3
"""Throughput of the CSR SpMV / SpMM hot path on one MI355X.

Workload (default): the power-law matrix, 1,048,576 x 1,048,576 with
Zipf(2.0) row lengths (mean 16, max 20,000) and hot columns of the same law,
FP64 values, x and X uniform[-1, 1); one step = one SpMV y <- A x plus one
SpMM Y <- A X with k = 16 (X, Y row-major).  CSR assembly and row binning run
once before timing (the paper also leaves transformation time out).

Protocol (the paper's Sec. 4): every timed run is preceded by a cache flush
(a 1 GiB read-modify-write, outside the timed region, so A, x and X come from
HBM and not from L2 or the 256 MB Infinity Cache); with the defaults
(--warmup 10 --steps 60) that is 70 runs with the mean of the last 60.
Kernel time is measured with HIP events on the stream the kernels run on.

Prints ONE JSON line.  `value` is GFLOP/s of the step (2 tau (1 + k) flops
per step); the dominant kernel's effective HBM bandwidth (the paper's
application bytes, Sec. 4.2 / Sec. 5) is reported against 8 TB/s.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
METRIC = "SpMV/SpMM GFLOP/s + effective HBM GB/s (% of peak), FP64 vs FP32/BF16-value"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--k", type=int, default=16)
    ap.add_argument("--rows", type=int, default=1 << 20)
    ap.add_argument("--no-flush", action="store_true")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--forms", action="store_true", help="also time the FP32/BF16 forms on this matrix")
    return ap.parse_args()


def source_hash() -> str:
    h = hashlib.sha256()
    for name in ("product.hip", "device.hpp", "plan.hip"):
        with open(os.path.join(ROOT, "paper_1302_1078_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(kernel_key: str, launches_per_step: float):
    """HBM bytes per launch from committed rocprofv3 counter summaries, or None
    when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
        e = d.get(kernel_key)
        if not e or e.get("source_hash") != source_hash():
            return None
        return float(e["bytes_per_launch"])
    except Exception:
        return None


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only; --gpus {args.gpus} is not supported "
              "(the sharded design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1302_1078_amd as spx
    import spgen

    dev = torch.device("cuda", 0)
    k = args.k
    t0 = time.time()
    coo = spgen.workload_c1(seed=0, m=args.rows)
    m, n = coo.m, coo.n
    r = torch.from_numpy(coo.r).to(dev)
    c = torch.from_numpy(coo.c).to(dev)
    v = torch.from_numpy(coo.v).to(dev)
    A = spx.from_coo(m, n, r, c, v)  # step a1 (device, one-time)
    del r, c, v
    nnz = A.nnz
    plan_v = spx.Plan.for_matrix(A, spx.default_opts(1))  # step a2 (device, one-time)
    plan_m = spx.Plan.for_matrix(A, spx.default_opts(k))
    x = torch.from_numpy(spgen.uniform(n, 0, spgen.TAG_X)).to(dev)
    X = torch.from_numpy(spgen.uniform(n * k, 0, spgen.TAG_X + 1).reshape(n, k)).to(dev)
    y = torch.empty(m, dtype=torch.float64, device=dev)
    Y = torch.empty((m, k), dtype=torch.float64, device=dev)
    flush = torch.zeros(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
    torch.cuda.synchronize()
    setup_s = time.time() - t0

    def app_bytes(kk, sv=8, sx=8):
        return (sv + 4) * nnz + sx * kk * n + sx * kk * m + 4 * (m + 1)

    flops_v, flops_m = 2 * nnz, 2 * nnz * k
    bytes_v, bytes_m = app_bytes(1), app_bytes(k)

    def run(steps, flush_each):
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
        for s in range(steps):
            if flush_each:
                flush.add_(1.0)
            e = ev[s]
            e[0].record()
            spx.spmv(A, x, y=y, plan=plan_v)
            e[1].record()
            spx.spmm(A, X, Y=Y, plan=plan_m)
            e[2].record()
        return ev

    flush_each = not args.no_flush
    run(args.warmup, flush_each)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev = run(args.steps, flush_each)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    tv = np.array([e[0].elapsed_time(e[1]) for e in ev]) * 1e-3
    tm = np.array([e[1].elapsed_time(e[2]) for e in ev]) * 1e-3
    t_step = float(tv.mean() + tm.mean())

    # secondary: warm (no flush) back-to-back
    evw = run(20, False)
    torch.cuda.synchronize()
    tvw = float(np.mean([e[0].elapsed_time(e[1]) for e in evw])) * 1e-3
    tmw = float(np.mean([e[1].elapsed_time(e[2]) for e in evw])) * 1e-3

    detail = {
        "spmv": {"ms": tv.mean() * 1e3, "ms_median": float(np.median(tv)) * 1e3,
                 "ms_min": float(tv.min()) * 1e3, "gflops": flops_v / tv.mean() / 1e9,
                 "eff_gbs": bytes_v / tv.mean() / 1e9, "frac_hbm": bytes_v / tv.mean() / 1e9 / PEAK_HBM_GBS,
                 "bytes": bytes_v, "warm_ms": tvw * 1e3, "warm_eff_gbs": bytes_v / tvw / 1e9},
        "spmm": {"k": k, "ms": tm.mean() * 1e3, "ms_median": float(np.median(tm)) * 1e3,
                 "ms_min": float(tm.min()) * 1e3, "gflops": flops_m / tm.mean() / 1e9,
                 "eff_gbs": bytes_m / tm.mean() / 1e9, "frac_hbm": bytes_m / tm.mean() / 1e9 / PEAK_HBM_GBS,
                 "bytes": bytes_m, "warm_ms": tmw * 1e3, "warm_eff_gbs": bytes_m / tmw / 1e9},
        "plans": {"spmv": plan_v.info(), "spmm": plan_m.info()},
        "flushed": flush_each, "setup_s": round(setup_s, 2), "wall_s_timed": round(wall, 4),
        "source_hash": source_hash(),
    }

    if args.forms:
        forms = {}
        xf = x.float()
        Xf = X.float()
        for name, vals in (("f32", A.values.float()), ("bf16", A.values.to(torch.bfloat16))):
            Aq = A.with_values(vals)
            pv = spx.Plan.for_matrix(Aq, spx.default_opts(1, torch.float32))
            pm = spx.Plan.for_matrix(Aq, spx.default_opts(k, torch.float32))
            yq = torch.empty(m, dtype=torch.float32, device=dev)
            Yq = torch.empty((m, k), dtype=torch.float32, device=dev)
            tq = []
            for s in range(args.warmup + args.steps):
                if flush_each:
                    flush.add_(1.0)
                e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
                e[0].record()
                spx.spmv(Aq, xf, y=yq, plan=pv)
                e[1].record()
                spx.spmm(Aq, Xf, Y=Yq, plan=pm)
                e[2].record()
                tq.append(e)
            torch.cuda.synchronize()
            tq = tq[args.warmup:]
            a = np.mean([e[0].elapsed_time(e[1]) for e in tq]) * 1e-3
            b = np.mean([e[1].elapsed_time(e[2]) for e in tq]) * 1e-3
            sv = 4 if name == "f32" else 2
            forms[name] = {"spmv_ms": a * 1e3, "spmm_ms": b * 1e3,
                           "spmv_eff_gbs": app_bytes(1, sv, 4) / a / 1e9,
                           "spmm_eff_gbs": app_bytes(k, sv, 4) / b / 1e9,
                           "speedup_spmv_vs_f64": float(tv.mean() / a),
                           "speedup_spmm_vs_f64": float(tm.mean() / b)}
        detail["forms"] = forms

    cpu = None
    if not args.no_cpu:
        import oracle
        ro = oracle.CSR(m, n, A.rowptr.cpu().numpy(), A.colind.cpu().numpy(), A.values.cpu().numpy())
        xh = x.cpu().numpy()
        Xh = X.cpu().numpy()
        oracle.spmv(ro, xh)  # warm-up
        reps, spent, c0 = 0, 0.0, time.perf_counter()
        tv_c, tm_c = 0.0, 0.0
        while spent < args.cpu_seconds and reps < 50:
            a0 = time.perf_counter()
            oracle.spmv(ro, xh)
            a1 = time.perf_counter()
            oracle.spmm(ro, Xh)
            a2 = time.perf_counter()
            tv_c += a1 - a0
            tm_c += a2 - a1
            reps += 1
            spent = time.perf_counter() - c0
        cpu = {"value": (flops_v + flops_m) * reps / (tv_c + tm_c) / 1e9, "unit": "GFLOP/s",
               "cores": oracle.max_threads(), "kind": "oracle",
               "sample": f"full matrix, {reps} x (SpMV + SpMM k={k}) in FP64, OpenMP dynamic,64; "
                         f"{spent:.1f} s; host caches not flushed",
               "spmv_gflops": flops_v * reps / tv_c / 1e9, "spmm_gflops": flops_m * reps / tm_c / 1e9}

    dom = "spmm" if tm.mean() >= tv.mean() else "spmv"
    t_dom = float(tm.mean() if dom == "spmm" else tv.mean())
    b_dom = bytes_m if dom == "spmm" else bytes_v
    traffic = traffic_for(f"k_product_{dom}_c1", 1.0)
    roofline = {"bound": "hbm", "achieved": b_dom / t_dom / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": b_dom / t_dom / 1e9 / PEAK_HBM_GBS, "traffic": traffic,
                "kernel": f"k_product ({'SpMM k=%d' % k if dom == 'spmm' else 'SpMV'}, FP64)",
                "algorithmic_bytes_per_launch": b_dom}

    out = {
        "metric": METRIC,
        "value": (flops_v + flops_m) / t_step / 1e9,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"power-law {m:,} x {n:,}, Zipf(2.0) row lengths mean 16 max 20,000, "
                               f"hot columns; FP64 SpMV + SpMM k={k}",
                   "m": m, "n": n, "nnz": nnz, "k": k, "index": "int32", "seed": 0},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": detail,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
