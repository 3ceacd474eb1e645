#!/usr/bin/env python3
"""Throughput of the CSR SpMV / SpMM hot path on one MI355X.

Headline workload: the power-law matrix, 1,048,576 x 1,048,576 with Zipf(2.0)
row lengths (mean 16, max 20,000) and hot columns of the same law, FP64
values, x and X uniform[-1, 1); one step = one SpMV y <- A x plus one SpMM
Y <- A X with k = 16 (row-major).  CSR assembly, row binning and the SpMV
plan's ranking of the columns by use run once, on the device, before timing
(the paper also leaves transformation time out); each SpMV call gathers the
x entries of the 65,536 most-used columns into the plan's compact copy
inside its timed region.  `value` is GFLOP/s of the step (2 tau (1 + k)
flops per step).

Protocol (the paper's Sec. 4): every timed call, the SpMV and the SpMM of a
step alike, is preceded by its own cache flush (a 1 GiB read-modify-write
outside the timed region, so A, x and X come from HBM rather than from L2 or
the 256 MB Infinity Cache); with the defaults (--warmup 10 --steps 60) that is
70 runs and the mean of the last 60.  Kernel time comes from HIP events on
the stream the kernels run on.

CPU baseline (the oracle, never tuned): the same matrix, SpMV + SpMM, 2
warm-up and 10 timed repetitions on all host cores and on one thread, the
host's last-level caches flushed before each repetition by touching a buffer
of twice their total size.

The other workloads are reported under detail.forms (skip with --quick):
  c0  10,000 x 10,000, 10 uniform columns per row, FP64 SpMV (launch-bound)
  c2  precision form: 27-point stencil on 128^3 and the power-law matrix,
      FP64 / FP32 / BF16 values, k in {1, 8, 32}; the reduced-precision
      errors against the GPU's FP64 product of the same data (the oracle runs
      only in the CPU-baseline leg; the tests hold these products to the
      oracle)
  c3  differentiation form: 524,288 power-law (mean 20), FP32 forward and
      backward (CSC-index and atomic transpose, sampled dot gathering x or
      streaming the forward's saved gather), and the autograd step with and
      without the saved gather
  c4  batched form: 256 matrices in one launch per lane layout replayed from a
      HIP graph, autotuned plans, against sequential single-matrix calls
  shard  one GPU's row block of an 8-way sharding of the headline matrix
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
HOT_X_COLUMNS = 65536   # x entries of the most-used columns packed by the headline SpMV plan
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
    ap.add_argument("--cpu-reps", type=int, default=10, help="timed oracle repetitions (after 2 warm-up)")
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--no-warm", action="store_true",
                    help="skip the unflushed (warm) calls, so a kernel trace holds flushed calls only")
    ap.add_argument("--forms", default="c0,c2,c3,c4,shard",
                    help="comma list of extra workloads (c0, c2, c3, c4; shard = one GPU's row block of an 8-GPU sharding; ksweep = SpMM k sweep and variants; occupancy = workgroups-per-CU sweep; rcm = RCM ordering; bcsr = register blocking; locality = column-locality sweep)")
    ap.add_argument("--form-steps", type=int, default=20)
    return ap.parse_args()


def source_hash() -> str:
    h = hashlib.sha256()
    for name in ("product.hip", "product_impl.hpp", "device.hpp", "plan.hip"):
        with open(os.path.join(ROOT, "paper_1302_1078_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(kernel_key: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel sources changed since the counters were taken."""
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


class Timer:
    """Per-call HIP-event timing with an optional cache flush before EACH call.

    Every callable of a step gets its own flush (outside its timed region)
    and its own pair of events recorded on the current stream, the stream the
    library launches on."""

    def __init__(self, torch, dev, flush: bool):
        self.torch = torch
        self.flush_buf = torch.zeros(1 << 27, dtype=torch.float64, device=dev) if flush else None

    def run(self, fns, steps, warmup):
        """fns: list of callables timed separately within each step.
        Returns an array [steps, len(fns)] of seconds."""
        import numpy as np
        torch = self.torch
        rows = []
        for s in range(warmup + steps):
            row = []
            for fn in fns:
                if self.flush_buf is not None:
                    self.flush_buf.add_(1.0)
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                fn()
                e1.record()
                row.append((e0, e1))
            if s >= warmup:
                rows.append(row)
        torch.cuda.synchronize()
        return np.array([[a.elapsed_time(b) * 1e-3 for a, b in row] for row in rows]).reshape(steps, len(fns))


def chase_latency(torch, spx, dev):
    """ns per dependent load, from pointer chases over a random cycle of
    128-byte lines in a 1 GiB buffer.  A chase of H hops touches H lines; run
    warm (the same path just walked), 2 MB of lines stay in L2 and 16 MB miss
    the 4 MB L2 but stay in the Infinity Cache; run after a 1 GiB flush, every
    line comes from HBM.  "one address": all lanes on one chain; "64 chains":
    one gather of 64 lines per hop (the SpMV x access)."""
    import numpy as np
    from paper_1302_1078_amd.ops import chase_cycle, probe_chase
    n = 1 << 28
    nxt = chase_cycle(n, dev, seed=1)
    one = torch.zeros(64, dtype=torch.int32, device=dev)
    # 64 starts spread along the cycle (each walked from its own slot)
    many = torch.empty(64, dtype=torch.int32, device=dev)
    i = torch.zeros(1, dtype=torch.int32, device=dev)
    for lane in range(64):
        many[lane] = i[0]
        i = probe_chase(nxt, i.repeat(64), 1 << 12)[:1]
    cases = (("L2", one, 16384, False), ("infinity_cache", one, 131072, False), ("HBM", one, 16384, True),
             ("L2_gather64", many, 256, False), ("HBM_gather64", many, 1024, True))
    out = {}
    for label, start, hops, cold in cases:
        fn = lambda start=start, hops=hops: probe_chase(nxt, start, hops)  # noqa: E731
        t = float(np.median(Timer(torch, dev, cold).run([fn], 3, 1)[:, 0]))
        out[label + "_ns"] = t / hops * 1e9
    del nxt
    return out


def app_bytes(m, n, nnz, k=1, sv=8, sx=8):
    return (sv + 4) * nnz + sx * k * n + sx * k * m + 4 * (m + 1)


def upload(torch, spx, coo, dev):
    r = torch.from_numpy(coo.r).to(dev)
    c = torch.from_numpy(coo.c).to(dev)
    v = torch.from_numpy(coo.v).to(dev)
    A = spx.from_coo(coo.m, coo.n, r, c, v)
    del r, c, v
    return A


def rel2(a, b):
    """||a - b||_2 / ||b||_2 (the absolute norm when b = 0)."""
    import numpy as np
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    d = float(np.linalg.norm(a - b))
    return d / nb if nb > 0 else d


# ---------------------------------------------------------------- c0

def bench_c0(ctx):
    import numpy as np
    torch, spx, spgen, dev = ctx["torch"], ctx["spx"], ctx["spgen"], ctx["dev"]
    A = upload(torch, spx, spgen.workload_c0(0), dev)
    plan = spx.Plan.for_matrix(A)
    x = torch.from_numpy(spgen.uniform(A.n, 0)).to(dev)
    y = torch.empty(A.m, dtype=torch.float64, device=dev)
    t = ctx["timer"].run([lambda: spx.spmv(A, x, y=y, plan=plan)], ctx["fsteps"], 5)[:, 0]
    # a HIP graph of 100 back-to-back SpMVs (launch overhead amortised)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        spx.spmv(A, x, y=y, plan=plan)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(100):
            spx.spmv(A, x, y=y, plan=plan)
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    per = e0.elapsed_time(e1) * 1e-3 / 500
    b = app_bytes(A.m, A.n, A.nnz)
    return {"workload": "uniform 10,000 x 10,000, 10 nnz/row, FP64 SpMV", "nnz": A.nnz,
            "us_single_flushed": float(t.mean() * 1e6), "us_per_spmv_graph100_warm": per * 1e6,
            "gflops_graph": 2 * A.nnz / per / 1e9, "eff_gbs_graph": b / per / 1e9}


# ---------------------------------------------------------------- c2

def bench_c2(ctx, A1=None):
    """Reduced-precision forms.  Each FP32 / BF16 result reports rel2 against
    the GPU's plain FP64 product of the original data (rel2_vs_gpu_fp64) and
    against the GPU's FP64 product of the quantised inputs widened exactly
    (rel2_vs_quantised_fp64, the accumulation alone).  The oracle itself runs
    only in the CPU-baseline leg here: tests/test_gpu_full.py checks these same
    products (same matrices, same seeded X, same default plans) against the
    FP64 oracle element by element, the FP64 ones within 1e-12 and the
    reduced-precision ones within their per-row and total error bounds."""
    import numpy as np
    torch, spx, spgen, dev = ctx["torch"], ctx["spx"], ctx["spgen"], ctx["dev"]
    out = {}
    mats = [("stencil27_128", upload(torch, spx, spgen.workload_c2_stencil(0), dev))]
    if A1 is not None:
        mats.append(("powerlaw_1M", A1))

    def fp64_product(Aw, Xw, k):
        plan = spx.Plan.for_matrix(Aw, spx.default_opts(k))
        if k == 1:
            return spx.spmv(Aw, Xw[:, 0].contiguous(), plan=plan).cpu().numpy()[:, None]
        return spx.spmm(Aw, Xw, plan=plan).cpu().numpy()

    for name, A in mats:
        m, n, nnz = A.m, A.n, A.nnz
        rows = {}
        # register-blocked alternative for the banded matrix's SpMM: 2 x 1
        # blocks swept band by band of the bandwidth
        Bst = spx.BCSR.from_csr(A, 2, 1) if name.startswith("stencil") else None
        bw = spx.bandwidth(A) if Bst is not None else 0
        for k in (1, 8, 32):
            X64 = spgen.uniform(n * k, 7, spgen.TAG_X).reshape(n, k)
            Xq = spgen.to_f32(X64)
            y3 = fp64_product(A, torch.from_numpy(X64).to(dev), k)
            Xq64 = torch.from_numpy(Xq.astype(np.float64)).to(dev)
            base_t = None
            for vname in ("f64", "f32", "bf16"):
                if vname == "f64":
                    vals, Xd = A.values, torch.from_numpy(X64).to(dev)
                elif vname == "f32":
                    vals = A.values.float()
                    Xd = torch.from_numpy(Xq).to(dev)
                else:
                    vals = A.values.to(torch.bfloat16)
                    Xd = torch.from_numpy(Xq).to(dev)
                Aq = A.with_values(vals)
                plan = spx.Plan.for_matrix(Aq, spx.default_opts(k, vals.dtype))
                if k == 1:
                    xd = Xd[:, 0].contiguous()
                    yd = torch.empty(m, dtype=xd.dtype, device=dev)
                    fn = lambda: spx.spmv(Aq, xd, y=yd, plan=plan)  # noqa: E731
                else:
                    yd = torch.empty((m, k), dtype=Xd.dtype, device=dev)
                    fn = lambda: spx.spmm(Aq, Xd, Y=yd, plan=plan)  # noqa: E731
                t = float(ctx["timer"].run([fn], ctx["fsteps"], 3)[:, 0].mean())
                yh = yd.double().cpu().numpy().reshape(m, k)
                sv = {"f64": 8, "f32": 4, "bf16": 2}[vname]
                sx = 8 if vname == "f64" else 4
                b = app_bytes(m, n, nnz, k, sv, sx)
                r = {"us": t * 1e6, "gflops": 2 * nnz * k / t / 1e9, "eff_gbs": b / t / 1e9,
                     "frac_hbm": b / t / 1e9 / PEAK_HBM_GBS, "bytes": b}
                if k > 1 and name.startswith("stencil"):
                    # the staged plan (row tiles' X windows in LDS), an opt-in
                    # alternative for banded matrices, on the same data, and its
                    # persistent double-buffered form
                    ps = spx.Plan.staged(Aq, k, Xd.dtype)
                    pp = spx.Plan.staged(Aq, k, Xd.dtype, pipelined=True)
                    ys = torch.empty_like(yd)
                    ts, tp = ctx["timer"].run([lambda: spx.spmm(Aq, Xd, Y=ys, plan=ps),
                                               lambda: spx.spmm(Aq, Xd, Y=ys, plan=pp)], ctx["fsteps"], 3).mean(axis=0)
                    ts, tp = float(ts), float(tp)
                    r["staged_plan"] = {"us": ts * 1e6, "eff_gbs": b / ts / 1e9, "frac_hbm": b / ts / 1e9 / PEAK_HBM_GBS,
                                        "speedup_vs_default_plan": t / ts, **ps.staged_info(),
                                        "pipelined_us": tp * 1e6, "pipelined_speedup_vs_default_plan": t / tp}
                    del ps, pp, ys
                    # rows ordered band by band of the bandwidth (row_period):
                    # each XCD sweeps its own slab of the grid
                    pb = spx.Plan.for_matrix(Aq, spx.banded_opts(Aq, k, vals.dtype))
                    yb = torch.empty_like(yd)
                    tb = float(ctx["timer"].run([lambda: spx.spmm(Aq, Xd, Y=yb, plan=pb)], ctx["fsteps"], 3)[:, 0].mean())
                    r["banded_plan"] = {"us": tb * 1e6, "eff_gbs": b / tb / 1e9, "frac_hbm": b / tb / 1e9 / PEAK_HBM_GBS,
                                        "speedup_vs_default_plan": t / tb, "row_period": int(pb.opts.row_period),
                                        "equals_default_bitwise": bool(torch.equal(yb.view(torch.uint8),
                                                                                   yd.view(torch.uint8)))}
                    del pb, yb
                    bv = Bst.bvals if vname == "f64" else Bst.bvals.to(vals.dtype)
                    yc = torch.empty_like(yd)
                    tc = float(ctx["timer"].run([lambda: spx.bcsr_spmm(Bst, Xd, Y=yc, row_period=bw, values=bv)],
                                                ctx["fsteps"], 3)[:, 0].mean())
                    r["bcsr_2x1_banded"] = {"us": tc * 1e6, "eff_gbs": b / tc / 1e9,
                                            "frac_hbm": b / tc / 1e9 / PEAK_HBM_GBS,
                                            "speedup_vs_default_plan": t / tc,
                                            "max_rel_diff_vs_default_plan": float((yc.double() - yd.double()).abs().max()
                                                                                  / yd.double().abs().max())}
                    del bv, yc
                if k == 1 and name.startswith("powerlaw"):
                    # the same SpMV through the plan with hot x attached (the
                    # matrix's column use is skewed; the headline step's plan)
                    ph = spx.Plan.for_matrix(Aq, spx.default_opts(1, vals.dtype)).attach_hot_x(
                        Aq, HOT_X_COLUMNS, xdtype=xd.dtype)
                    yhx = torch.empty_like(yd)
                    th = float(ctx["timer"].run([lambda: spx.spmv(Aq, xd, y=yhx, plan=ph)], ctx["fsteps"], 3)[:, 0].mean())
                    r["hot_x_plan"] = {"us": th * 1e6, "eff_gbs": b / th / 1e9, "frac_hbm": b / th / 1e9 / PEAK_HBM_GBS,
                                       "speedup_vs_default_plan": t / th, "hot_columns": HOT_X_COLUMNS,
                                       "equals_default_bitwise": bool(torch.equal(yhx.view(torch.uint8),
                                                                                  yd.view(torch.uint8)))}
                    del ph, yhx
                if vname != "f64":
                    r["rel2_vs_gpu_fp64"] = max(rel2(yh[:, j], y3[:, j]) for j in range(k))
                    y5 = fp64_product(A.with_values(vals.double()), Xq64, k)
                    r["rel2_vs_quantised_fp64"] = max(rel2(yh[:, j], y5[:, j]) for j in range(k))
                    r["speedup_vs_f64"] = base_t / t
                else:
                    base_t = t
                rows[f"k{k}_{vname}"] = r
        out[name] = {"m": m, "nnz": nnz, "results": rows}
        del Bst
    out["note"] = ("FP32/BF16 values with FP32 x/y and FP32 accumulation; rows longer than 256 use "
                   "compensated sums with an FP64 cross-lane reduction")
    return out


# ---------------------------------------------------------------- k sweep (SpMM variants)

def bench_ksweep(ctx, A1=None):
    """SpMM variant ablation and k sweep (Sec. 5): for k in 1..64, X row-major
    with vector X loads (the k-specialised kernel), with scalar X loads (the
    generic kernel), with non-temporal Y stores (the paper's NRNGO-store
    variant), and X column-major served as k SpMVs over contiguous columns.
    FP64, flushed calls."""
    torch, spx, spgen, dev = ctx["torch"], ctx["spx"], ctx["spgen"], ctx["dev"]
    from paper_1302_1078_amd import _lib
    out = {}
    mats = [("stencil27_128", upload(torch, spx, spgen.workload_c2_stencil(0), dev))]
    if A1 is not None:
        mats.append(("powerlaw_1M", A1))
    for name, A in mats:
        m, n, nnz = A.m, A.n, A.nnz
        pv = spx.Plan.for_matrix(A, spx.default_opts(1))
        rows = {}
        for k in (1, 2, 4, 8, 16, 32, 64):
            X = torch.from_numpy(spgen.uniform(n * k, 11, spgen.TAG_X).reshape(n, k)).to(dev)
            Y = torch.empty((m, k), dtype=torch.float64, device=dev)
            b = app_bytes(m, n, nnz, k)
            r = {}
            nt = _lib.SPX_FLAG_NO_NT_STORE
            variants = [("vector", nt), ("scalar_x", nt | _lib.SPX_FLAG_SCALAR_X), ("vector_nt_store", 0)]
            plans, Ys = [], []
            for _, flags in variants:
                o = spx.default_opts(k)
                o.flags = flags
                plans.append(spx.Plan.for_matrix(A, o))
                Ys.append(Y if not Ys else torch.empty_like(Y))
            fns = [lambda p=p, Yv=Yv: spx.spmm(A, X, Y=Yv, plan=p) for p, Yv in zip(plans, Ys)]
            # variants take turns call by call (order reversed every other
            # round), so that drift over the sweep does not favour one of them
            ctx["timer"].run(fns, 0, 3)
            ts = [[] for _ in fns]
            for s in range(ctx["fsteps"]):
                for i in (range(len(fns)) if s % 2 == 0 else reversed(range(len(fns)))):
                    ts[i].append(float(ctx["timer"].run([fns[i]], 1, 0)[0, 0]))
            ref = Ys[0]
            for (vname, _), Yv, tv in zip(variants, Ys, ts):
                t = sum(tv) / len(tv)
                err = float((Yv - ref).abs().max() / ref.abs().max().clamp_min(1e-300))
                r[vname] = {"us": t * 1e6, "gflops": 2 * nnz * k / t / 1e9, "eff_gbs": b / t / 1e9,
                            "max_rel_diff_vs_vector": err}
            del plans, Ys, fns
            XT = X.t().contiguous()
            YT = torch.empty((k, m), dtype=torch.float64, device=dev)

            def colmajor():
                for j in range(k):
                    spx.spmv(A, XT[j], y=YT[j], plan=pv)
            t = float(ctx["timer"].run([colmajor], max(3, ctx["fsteps"] // 4), 1)[:, 0].mean())
            err = float((YT.t() - ref).abs().max() / ref.abs().max().clamp_min(1e-300))
            r["colmajor_k_spmv"] = {"us": t * 1e6, "gflops": 2 * nnz * k / t / 1e9, "eff_gbs": b / t / 1e9,
                                    "max_rel_diff_vs_vector": err}
            rows[f"k{k}"] = r
            del X, Y, XT, YT, ref
            torch.cuda.empty_cache()
        out[name] = {"m": m, "nnz": nnz, "results": rows}
    return out


# ---------------------------------------------------------------- occupancy sweep

def bench_occupancy(ctx, A1=None):
    """Latency versus bandwidth (Sec. 4.2): the same products with at most
    1..8 workgroups per CU (LDS padding), the GPU analogue of the paper's
    threads-per-core scaling.  FP64, flushed calls, default plans."""
    torch, spx, spgen, dev = ctx["torch"], ctx["spx"], ctx["spgen"], ctx["dev"]
    out = {}
    mats = [("stencil27_128", upload(torch, spx, spgen.workload_c2_stencil(0), dev))]
    if A1 is not None:
        mats.append(("powerlaw_1M", A1))
    for name, A in mats:
        m, n, nnz = A.m, A.n, A.nnz
        rows = {}
        for k in (1, 16):
            X = torch.from_numpy(spgen.uniform(n * k, 12, spgen.TAG_X).reshape(n, k)).to(dev)
            x = X[:, 0].contiguous()
            Y = torch.empty((m, k), dtype=torch.float64, device=dev)
            b = app_bytes(m, n, nnz, k)
            r = {}
            for occ in (1, 2, 3, 4, 6, 8, 0):
                o = spx.default_opts(k)
                o.occupancy = occ
                plan = spx.Plan.for_matrix(A, o)
                if k == 1:
                    fn = lambda plan=plan: spx.spmv(A, x, y=Y[:, 0], plan=plan)  # noqa: E731
                else:
                    fn = lambda plan=plan: spx.spmm(A, X, Y=Y, plan=plan)  # noqa: E731
                t = float(ctx["timer"].run([fn], ctx["fsteps"], 3)[:, 0].mean())
                r[f"wg_per_cu_{occ}" if occ else "uncapped"] = {"us": t * 1e6, "eff_gbs": b / t / 1e9}
            rows[f"k{k}"] = r
            del X, x, Y
        out[name] = rows
    return out


# ---------------------------------------------------------------- RCM ordering (Sec. 4.4)

def row_shards(rowptr, parts: int):
    """Row boundaries of `parts` contiguous row blocks holding about nnz/parts
    nonzeros each: the 1D row-block partition balanced by nonzeros that a
    multi-GPU SpMV / SpMM would use.  Block g is rows [cuts[g], cuts[g+1])."""
    import numpy as np
    rowptr = np.asarray(rowptr, dtype=np.int64)
    m, nnz = len(rowptr) - 1, int(rowptr[-1])
    cuts = [0]
    for g in range(1, parts):
        cuts.append(max(cuts[-1], min(m, int(np.searchsorted(rowptr, nnz * g // parts, side="left")))))
    cuts.append(m)
    return cuts


def shard_of(torch, spx, A, r0, r1):
    """Rows [r0, r1) of A as a CSR of their own (all n columns): row pointers
    rebased, column indices and values as views into A's."""
    p0, p1 = int(A.rowptr[r0]), int(A.rowptr[r1])
    rp = (A.rowptr[r0:r1 + 1] - p0).contiguous()
    return spx.CSR(rp, A.colind[p0:p1], A.values[p0:p1], (r1 - r0, A.n))


XGMI_LINK_GBS = 153.0   # one xGMI link, per direction
XGMI_LINKS = 7


def bench_shard(ctx, A):
    """One GPU's share of a row-block sharding over 8 GPUs, at its real shape:
    the headline matrix cut into 8 row blocks balanced by nonzeros, and each
    block's SpMV and SpMM (k = 16) timed against the full x and X, each call
    flushed, again with warm caches, and through each shard's own autotuned
    plans (flushed).  Reports every shard, the slowest one
    against an eighth of the full product (the compute part of the scaling),
    and the modelled allgather of x / X over 7 xGMI links (not measured: one
    GPU)."""
    import numpy as np
    from paper_1302_1078_amd import autotune
    torch, spx, dev = ctx["torch"], ctx["spx"], ctx["dev"]
    x, X = ctx["c1_x"], ctx["c1_X"]
    k = X.shape[1]
    tv_full, tm_full = ctx["c1_times"]
    parts = 8
    rp = A.rowptr.cpu().numpy()
    cuts = row_shards(rp, parts)
    shards = []
    for g in range(parts):
        S = shard_of(torch, spx, A, cuts[g], cuts[g + 1])
        pv = spx.Plan.for_matrix(S, spx.default_opts(1))
        pm = spx.Plan.for_matrix(S, spx.default_opts(k))
        y = torch.empty(S.m, dtype=torch.float64, device=dev)
        Y = torch.empty((S.m, k), dtype=torch.float64, device=dev)
        fns = [lambda: spx.spmv(S, x, y=y, plan=pv), lambda: spx.spmm(S, X, Y=Y, plan=pm)]
        t = ctx["timer"].run(fns, ctx["fsteps"], 3).mean(axis=0)
        tw = Timer(torch, dev, False).run(fns, ctx["fsteps"], 3).mean(axis=0)
        # each shard's own tuned plans, as a sharded deployment would pick them
        ov, _ = autotune.tune(S, x, batch=False)
        om, _ = autotune.tune(S, X, batch=False)
        tv_p, tm_p = spx.Plan.for_matrix(S, ov), spx.Plan.for_matrix(S, om)
        tt = ctx["timer"].run([lambda: spx.spmv(S, x, y=y, plan=tv_p), lambda: spx.spmm(S, X, Y=Y, plan=tm_p)],
                              ctx["fsteps"], 3).mean(axis=0)
        lens = np.diff(rp[cuts[g]:cuts[g + 1] + 1])
        shards.append({"rows": S.m, "nnz": S.nnz, "longest_row": int(lens.max()) if len(lens) else 0,
                       "spmv_us": t[0] * 1e6, "spmm_us": t[1] * 1e6,
                       "spmv_warm_us": tw[0] * 1e6, "spmm_warm_us": tw[1] * 1e6,
                       "spmv_tuned_us": tt[0] * 1e6, "spmm_tuned_us": tt[1] * 1e6,
                       "tuned_split_chunk": [ov.split_chunk, om.split_chunk]})
        del S, pv, pm, y, Y, tv_p, tm_p
    tv_max = max(r["spmv_us"] for r in shards)
    tm_max = max(r["spmm_us"] for r in shards)
    fw = Timer(torch, dev, False).run([lambda: spx.spmv(A, x, y=ctx["c1_y"], plan=ctx["c1_plans"][0]),
                                       lambda: spx.spmm(A, X, Y=ctx["c1_Y"], plan=ctx["c1_plans"][1])],
                                      ctx["fsteps"], 3).mean(axis=0) * 1e6
    twv_max = max(r["spmv_warm_us"] for r in shards)
    twm_max = max(r["spmm_warm_us"] for r in shards)
    recv = (parts - 1) / parts
    return {"workload": "power-law 1,048,576 x 1,048,576 (the headline matrix), 8 row blocks by nonzeros, FP64",
            "parts": parts, "row_cuts": cuts, "shards": shards,
            "full_spmv_us": tv_full * 1e6, "full_spmm_us": tm_full * 1e6,
            "slowest_spmv_us": tv_max, "slowest_spmm_us": tm_max,
            "compute_efficiency_spmv": tv_full * 1e6 / (parts * tv_max),
            "compute_efficiency_spmm": tm_full * 1e6 / (parts * tm_max),
            "tuned": {"slowest_spmv_us": max(r["spmv_tuned_us"] for r in shards),
                      "slowest_spmm_us": max(r["spmm_tuned_us"] for r in shards),
                      "compute_efficiency_spmv": tv_full * 1e6 / (parts * max(r["spmv_tuned_us"] for r in shards)),
                      "compute_efficiency_spmm": tm_full * 1e6 / (parts * max(r["spmm_tuned_us"] for r in shards))},
            "warm": {"full_spmv_us": float(fw[0]), "full_spmm_us": float(fw[1]),
                     "slowest_spmv_us": twv_max, "slowest_spmm_us": twm_max,
                     "compute_efficiency_spmv": float(fw[0]) / (parts * twv_max),
                     "compute_efficiency_spmm": float(fw[1]) / (parts * twm_max)},
            "modelled_allgather_x_us": 8 * A.n * recv / (XGMI_LINKS * XGMI_LINK_GBS * 1e9) * 1e6,
            "modelled_allgather_X_us": 8 * A.n * k * recv / (XGMI_LINKS * XGMI_LINK_GBS * 1e9) * 1e6,
            "note": "compute only; the allgather is modelled from the link rate, not measured (one GPU)"}


def bench_rcm(ctx, A1=None):
    """Products before and after reverse Cuthill-McKee ordering (Sec. 4.4)
    and degree ordering (columns, and rows with them, by descending column
    count): the 27-point stencil in its natural order, randomly relabeled,
    and the relabeled matrix reordered; the power-law matrix as generated and
    reordered.  Reports time, UCLD and vector access (x lines of 128 B, rows
    dealt to 8 XCD caches in contiguous eighths, the tile map's layout)."""
    torch, spx, spgen, dev = ctx["torch"], ctx["spx"], ctx["spgen"], ctx["dev"]
    out = {}
    st = spgen.workload_c2_stencil(0)
    stencil = upload(torch, spx, st, dev)
    relab = upload(torch, spx, spgen.relabeled(st, 1), dev)
    del st
    mats = [("stencil27_128", [("natural", stencil), ("relabeled", relab)])]
    if A1 is not None:
        mats.append(("powerlaw_1M", [("natural", A1)]))
    for name, orders in mats:
        src_name, src = orders[-1]
        t0 = time.time()
        perm = spx.rcm(src)
        rcm_s = time.time() - t0
        t0 = time.time()
        R = spx.permute(src, perm)
        torch.cuda.synchronize()
        permute_s = time.time() - t0
        t0 = time.time()
        Dg = spx.permute(src, spx.degree_order(src))
        torch.cuda.synchronize()
        degree_s = time.time() - t0
        rows = {}
        for oname, A in orders + [(f"rcm_of_{src_name}", R), (f"degree_of_{src_name}", Dg)]:
            m, n, nnz = A.m, A.n, A.nnz
            r = {"ucld_line16": spx.ucld(A, 16),
                 "vector_access_8xcd": spx.vector_access(A, 16, 8, -(-m // 8)),
                 "bandwidth": int((A.colind.long() - torch.repeat_interleave(
                     torch.arange(m, device=dev), A.rowptr[1:].long() - A.rowptr[:-1].long())).abs().max())}
            for k in (1, 8):
                X = torch.from_numpy(spgen.uniform(n * k, 13, spgen.TAG_X).reshape(n, k)).to(dev)
                plan = spx.Plan.for_matrix(A, spx.default_opts(k))
                if k == 1:
                    x = X[:, 0].contiguous()
                    y = torch.empty(m, dtype=torch.float64, device=dev)
                    fn = lambda: spx.spmv(A, x, y=y, plan=plan)  # noqa: E731
                else:
                    Y = torch.empty((m, k), dtype=torch.float64, device=dev)
                    fn = lambda: spx.spmm(A, X, Y=Y, plan=plan)  # noqa: E731
                t = float(ctx["timer"].run([fn], ctx["fsteps"], 3)[:, 0].mean())
                r[f"k{k}_us"] = t * 1e6
                r[f"k{k}_gflops"] = 2 * nnz * k / t / 1e9
            rows[oname] = r
        out[name] = {"orders": rows, "rcm_host_s": round(rcm_s, 2), "permute_device_s": round(permute_s, 3),
                     "degree_order_and_permute_device_s": round(degree_s, 3)}
        del R, perm, Dg
        torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------- locality sweep (Sec. 4.1, 4.2)

def bench_locality(ctx, A1=None):
    """How the x access pattern sets SpMV speed (the paper's UCLD and
    actual-versus-application study, Sec. 4.1 and 4.2), over matrices whose
    column locality differs while their size stays fixed: per matrix the
    useful cacheline density (128 B lines), the distinct x lines per 256-row
    tile (a stream tile of the SpMV), the vector access for 8 XCD caches, the
    flushed FP64 SpMV time, and the flushed time of the index-gather probe
    with and without the x reads (the x gather alone is their difference).
    The x-gather L2 hit rate comes from counter runs of the same probe
    (python -m paper_1302_1078_amd.run --workload locality)."""
    torch, spx, spgen, dev = ctx["torch"], ctx["spx"], ctx["spgen"], ctx["dev"]
    from paper_1302_1078_amd.run import locality_matrices
    out = {}
    for name, A in locality_matrices(torch, spx, spgen, dev):
        m, n, nnz = A.m, A.n, A.nnz
        tiles = -(-m // 256)
        pairs = spx.tile_lines(A, 16, 256)
        x = torch.from_numpy(spgen.uniform(n, 0)).to(dev)
        y = torch.empty(m, dtype=torch.float64, device=dev)
        plan = spx.Plan.for_matrix(A, spx.default_opts(1))
        fns = [lambda: spx.spmv(A, x, y=y, plan=plan),
               lambda: spx.ops.probe_index_gather(A.colind, x, gather=True, blocks=4096),
               lambda: spx.ops.probe_index_gather(A.colind, x, gather=False, blocks=4096)]
        t = ctx["timer"].run(fns, ctx["fsteps"], 3).mean(axis=0)
        out[name] = {"m": m, "nnz": nnz, "ucld_line16": spx.ucld(A, 16),
                     "tile_lines_per_tile": pairs / tiles, "gathers_per_line_in_tile": nnz / pairs,
                     "vector_access_8xcd": spx.vector_access(A, 16, 8, -(-m // 8)),
                     "spmv_us": t[0] * 1e6, "spmv_gflops": 2 * nnz / t[0] / 1e9,
                     "xgather_probe_us": t[1] * 1e6, "colstream_probe_us": t[2] * 1e6}
        del A, x, y, plan
        torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------- register blocking (Sec. 4.5)

def bench_bcsr(ctx, A1=None):
    """SpMV on register-blocked CRS against the CSR kernel (the paper's
    relative-performance table, Sec. 4.5): dense a x b blocks with explicit
    zeros, and bitmap blocks (64-bit mask + packed nonzeros).  FP64, flushed.
    Density = nonzeros / stored values."""
    torch, spx, spgen, dev = ctx["torch"], ctx["spx"], ctx["spgen"], ctx["dev"]
    out = {}
    mats = [("stencil27_128", upload(torch, spx, spgen.workload_c2_stencil(0), dev),
             [(8, 8), (8, 4), (8, 2), (8, 1), (4, 8), (2, 8), (1, 8), (4, 4), (2, 2)])]
    if A1 is not None:  # sparse rows: blocks above 8 values would mostly store zeros
        mats.append(("powerlaw_1M", A1, [(8, 1), (4, 1), (2, 1), (1, 8), (1, 4), (2, 2)]))
    for name, A, shapes in mats:
        m, n, nnz = A.m, A.n, A.nnz
        x = torch.from_numpy(spgen.uniform(n, 14, spgen.TAG_X)).to(dev)
        y = torch.empty(m, dtype=torch.float64, device=dev)
        plan = spx.Plan.for_matrix(A, spx.default_opts(1))
        t_csr = float(ctx["timer"].run([lambda: spx.spmv(A, x, y=y, plan=plan)], ctx["fsteps"], 3)[:, 0].mean())
        ref = y.clone()
        rows = {"csr": {"us": t_csr * 1e6, "gflops": 2 * nnz / t_csr / 1e9, "bytes": 12 * nnz + 4 * (m + 1)}}
        variants = [(a, b, False) for a, b in shapes] + [(8, 8, True), (8, 1, True), (4, 4, True), (1, 8, True)]
        for a, b, bitmap in variants:
            B = spx.BCSR.from_csr(A, a, b, bitmap)
            t = float(ctx["timer"].run([lambda: spx.bcsr_spmv(B, x, y=y)], ctx["fsteps"], 3)[:, 0].mean())
            err = float((y - ref).abs().max() / ref.abs().max())
            rows[f"{a}x{b}{'_bitmap' if bitmap else ''}"] = {
                "us": t * 1e6, "gflops": 2 * nnz / t / 1e9, "relative_to_csr": t_csr / t,
                "density": nnz / (B.nblocks * a * b) if B.nblocks else 0.0, "blocks": B.nblocks,
                "bytes": B.stored_bytes(), "max_rel_diff_vs_csr": err}
            del B
            torch.cuda.empty_cache()
        if name.startswith("stencil"):
            rows["spmm"] = bcsr_spmm_rows(ctx, A)
        out[name] = rows
    return out


def bcsr_spmm_rows(ctx, A):
    """SpMM (Sec. 5) through a x 1 register blocks against the CSR kernel with
    the default and the banded plan, FP64, flushed, per k: time, and the
    largest difference to the default CSR product relative to its largest
    entry (the sums run in another order)."""
    torch, spx, spgen, dev = ctx["torch"], ctx["spx"], ctx["spgen"], ctx["dev"]
    res = {}
    for k in (8, 16, 32):
        X = torch.from_numpy(spgen.uniform(A.n * k, 31, spgen.TAG_X).reshape(A.n, k)).to(dev)
        Y = torch.empty((A.m, k), dtype=torch.float64, device=dev)
        p0 = spx.Plan.for_matrix(A, spx.default_opts(k))
        pb = spx.Plan.for_matrix(A, spx.banded_opts(A, k))
        t0 = float(ctx["timer"].run([lambda: spx.spmm(A, X, Y=Y, plan=p0)], ctx["fsteps"], 3)[:, 0].mean())
        ref = Y.clone()
        tb = float(ctx["timer"].run([lambda: spx.spmm(A, X, Y=Y, plan=pb)], ctx["fsteps"], 3)[:, 0].mean())
        r = {"csr_us": t0 * 1e6, "csr_banded_us": tb * 1e6}
        bw = spx.bandwidth(A)
        for a in (2, 4, 8):
            B = spx.BCSR.from_csr(A, a, 1)
            t = float(ctx["timer"].run([lambda: spx.bcsr_spmm(B, X, Y=Y)], ctx["fsteps"], 3)[:, 0].mean())
            r[f"bcsr_{a}x1"] = {"us": t * 1e6, "speedup_vs_csr": t0 / t, "gflops": 2 * A.nnz * k / t / 1e9,
                                "density": A.nnz / (B.nblocks * a), "stored_bytes": B.stored_bytes(),
                                "max_rel_diff_vs_csr": float((Y - ref).abs().max() / ref.abs().max())}
            if a < 8:  # block rows swept band by band of the bandwidth
                Yb = Y.clone()
                tbb = float(ctx["timer"].run([lambda: spx.bcsr_spmm(B, X, Y=Y, row_period=bw)],
                                             ctx["fsteps"], 3)[:, 0].mean())
                r[f"bcsr_{a}x1"].update({"banded_us": tbb * 1e6, "banded_speedup_vs_csr": t0 / tbb,
                                         "banded_equals_unbanded_bitwise": bool(torch.equal(Y, Yb))})
                del Yb
            del B
            torch.cuda.empty_cache()
        res[f"k{k}"] = r
        del X, Y, ref, p0, pb
        torch.cuda.empty_cache()
    return res


# ---------------------------------------------------------------- c3

def bench_c3(ctx):
    import numpy as np
    torch, spx, spgen, dev = ctx["torch"], ctx["spx"], ctx["spgen"], ctx["dev"]
    A64 = upload(torch, spx, spgen.workload_c3(0), dev)
    A = A64.with_values(A64.values.float())
    m, n, nnz = A.m, A.n, A.nnz
    x = torch.from_numpy(spgen.to_f32(spgen.uniform(n, 3))).to(dev)
    dy = torch.from_numpy(spgen.to_f32(spgen.normal(m, 4, spgen.TAG_DY))).to(dev)
    g0 = spx.GradContext(A, mode=0)
    plan = g0.plan
    y = torch.empty(m, dtype=torch.float32, device=dev)
    dx = torch.empty(n, dtype=torch.float32, device=dev)
    dv = torch.empty(nnz, dtype=torch.float32, device=dev)
    xg = torch.empty(nnz, dtype=torch.float32, device=dev)
    vstage = torch.empty_like(A.values)
    vcsc = torch.empty_like(A.values)
    Acsc = A.with_values(vcsc)

    def dx_csc_values():
        spx.values_to_csc(A.values, g0.vmap, staging=vstage, out=vcsc)
        spx.spmv_t(Acsc, dy, mode=0, index=g0.index_v, plan=g0.plan_t, out=dx)

    fns = [lambda: spx.spmv(A, x, y=y, plan=plan),
           lambda: spx.spmv_t(A, dy, mode=0, index=g0.index, plan=g0.plan_t, out=dx),
           lambda: spx.spmv_t(A, dy, mode=1, plan=plan, out=dx),
           lambda: spx.sddmm(A, dy, x, plan=plan, out=dv),
           dx_csc_values,
           lambda: spx.values_to_csc(A.values, g0.vmap, staging=vstage, out=vcsc),
           lambda: spx.spmv_save(A, x, y=y, xsave=xg, plan=plan),
           lambda: spx.sddmm_saved(A, dy, xg, plan=plan, out=dv)]
    t = ctx["timer"].run(fns, ctx["fsteps"], 3).mean(axis=0)
    fwd_b = app_bytes(m, n, nnz, 1, 4, 4)
    csc_b = 4 * nnz * 3 + 4 * (n + 1) + 4 * m + 4 * n     # perm, rowind, values + colptr, dy, dx
    atom_b = 8 * nnz + 4 * (m + 1) + 4 * m + 2 * 4 * n    # colind, values, rowptr, dy, dx zero+write
    sdd_b = 8 * nnz + 4 * (m + 1) + 4 * m + 4 * n         # colind, out, rowptr, dy, x
    sdds_b = 8 * nnz + 4 * (m + 1) + 4 * m                # saved x, out, rowptr, dy
    # autograd round trip through the Function, with the forward's gathered
    # x kept for the sampled dot (the default) and without
    v = A.values.clone().requires_grad_(True)
    xt = x.clone().requires_grad_(True)
    g1 = spx.GradContext(A, mode=0, save_gather=False)

    def step(g):
        def f():
            v.grad = xt.grad = None   # gradients set to None between steps, as zero_grad() does
            yy = spx.spmv_autograd(v, xt, g)
            yy.backward(dy)
        return f
    ta = ctx["timer"].run([step(g0), step(g1)], 10, 2).mean(axis=0)
    return {"workload": "power-law 524,288 x 524,288, Zipf(2.0) mean 20, FP32", "nnz": nnz,
            "forward_us": t[0] * 1e6, "forward_eff_gbs": fwd_b / t[0] / 1e9,
            "dx_csc_us": t[1] * 1e6, "dx_csc_eff_gbs": csc_b / t[1] / 1e9,
            "dx_csc_values_moved_us": t[4] * 1e6, "values_to_csc_us": t[5] * 1e6,
            "dx_atomic_us": t[2] * 1e6, "dx_atomic_eff_gbs": atom_b / t[2] / 1e9,
            "dvalues_us": t[3] * 1e6, "dvalues_eff_gbs": sdd_b / t[3] / 1e9,
            "forward_save_us": t[6] * 1e6, "forward_save_eff_gbs": (fwd_b + 4 * nnz) / t[6] / 1e9,
            "dvalues_saved_us": t[7] * 1e6, "dvalues_saved_eff_gbs": sdds_b / t[7] / 1e9,
            "autograd_fwd_bwd_us": float(ta[0]) * 1e6,
            "autograd_fwd_bwd_no_saved_gather_us": float(ta[1]) * 1e6,
            "note": "gradients are checked in tests/test_gpu_forms.py (gradcheck, FD, dense reference)"}


# ---------------------------------------------------------------- c4

def bench_c4(ctx):
    import numpy as np
    torch, spx, spgen, dev = ctx["torch"], ctx["spx"], ctx["spgen"], ctx["dev"]
    from paper_1302_1078_amd import autotune
    from paper_1302_1078_amd.batch import Batched
    t0 = time.time()
    specs = spgen.batch_specs(256, seed=0)
    mats32, mats64, X32, X64, ks = [], [], [], [], []
    flops = bytes32 = bytes64 = 0
    for i, s in enumerate(specs):
        A = upload(torch, spx, spgen.batch_matrix(s, 0, i), dev)
        X = spgen.uniform(A.n * s.k, 1000 + i, spgen.TAG_X).reshape(A.n, s.k)
        xd = torch.from_numpy(X[:, 0].copy() if s.k == 1 else X).to(dev)
        mats64.append(A)
        X64.append(xd)
        mats32.append(A.with_values(A.values.float()))
        X32.append(xd.float())
        ks.append(s.k)
        flops += 2 * A.nnz * s.k
        bytes32 += app_bytes(A.m, A.n, A.nnz, s.k, 4, 4)
        bytes64 += app_bytes(A.m, A.n, A.nnz, s.k, 8, 8)
    gen_s = time.time() - t0
    import tempfile
    cache = os.path.join(tempfile.mkdtemp(prefix="spx_tune_"), "autotune_c4.json")  # tune afresh
    t1 = time.time()
    opts, tune_report = autotune.tune_batch(mats32, X32, reps=3, cache_path=cache)
    tune_s = time.time() - t1
    B = Batched(mats32, X32, opts=opts)
    g = B.capture()
    t_graph = float(ctx["timer"].run([g.replay], ctx["fsteps"], 3)[:, 0].mean())
    t_run = float(ctx["timer"].run([B.run], ctx["fsteps"], 3)[:, 0].mean())
    # the same batch with every matrix on its default plan, for comparison
    Bd = Batched(mats32, X32)
    gd = Bd.capture()
    t_graph_default = float(ctx["timer"].run([gd.replay], ctx["fsteps"], 3)[:, 0].mean())
    del gd, Bd
    # sequential single calls get plans tuned for single calls
    single = [autotune.tune(A, X, reps=3, batch=False)[0] for A, X in zip(mats32, X32)]
    plans32 = [spx.Plan.for_matrix(A, o) for A, o in zip(mats32, single)]
    plans64 = [spx.Plan.for_matrix(A, spx.default_opts(k)) for A, k in zip(mats64, ks)]
    outs32 = [torch.empty_like(Y) for Y in B.Ys]
    outs64 = [torch.empty(Y.shape, dtype=torch.float64, device=dev) for Y in B.Ys]

    def seq(mats, Xs, plans, outs):
        def f():
            for A, X, p, Y in zip(mats, Xs, plans, outs):
                if X.dim() == 1:
                    spx.spmv(A, X, y=Y, plan=p)
                else:
                    spx.spmm(A, X, Y=Y, plan=p)
        return f
    t_seq32 = float(ctx["timer"].run([seq(mats32, X32, plans32, outs32)], ctx["fsteps"], 3)[:, 0].mean())
    t_seq64 = float(ctx["timer"].run([seq(mats64, X64, plans64, outs64)], ctx["fsteps"], 3)[:, 0].mean())
    # the batch keeps stream bins as stream tiles; single launches of the same
    # options with that flag must agree bit for bit
    from paper_1302_1078_amd._lib import PlanOpts, SPX_FLAG_KEEP_STREAM
    keep = []
    for o in opts:
        c = PlanOpts.from_dict(o.to_dict())
        c.flags |= SPX_FLAG_KEEP_STREAM
        keep.append(c)
    outs_chk = [torch.empty_like(Y) for Y in B.Ys]
    seq(mats32, X32, [spx.Plan.for_matrix(A, o) for A, o in zip(mats32, keep)], outs_chk)()
    torch.cuda.synchronize()
    same = all(torch.equal(a, b) for a, b in zip(outs_chk, B.Ys))
    info = B.info()
    return {"workload": "256 matrices (64 2D 5-pt, 64 3D 7-pt, 128 Zipf(2.2) mean 8-32), rows "
                        "log-uniform [1e3, 2e5], FP32 values, k in {1, 4, 16}",
            "matrices": len(specs), "total_nnz": int(sum(A.nnz for A in mats32)),
            "total_rows": int(sum(A.m for A in mats32)), "tiles": info["tiles"], "grid": info["grid"],
            "graph_us": t_graph * 1e6, "run_us": t_run * 1e6, "graph_default_plans_us": t_graph_default * 1e6,
            "autotune": tune_report, "seq_f32_us": t_seq32 * 1e6,
            "seq_f64_us": t_seq64 * 1e6, "gflops_graph": flops / t_graph / 1e9,
            "eff_gbs_graph": bytes32 / t_graph / 1e9,
            "speedup_vs_seq_f32": t_seq32 / t_graph, "speedup_vs_seq_f64": t_seq64 / t_graph,
            "batched_equals_single_bitwise": bool(same), "gen_s": round(gen_s, 1),
            "autotune_s": round(tune_s, 1)}


# ---------------------------------------------------------------- CPU baseline (the oracle)

def host_llc_bytes() -> int:
    """Total last-level cache the process can reach: the size of each distinct
    L3 (sysfs cache index3, one entry per shared_cpu_list) over the CPUs of
    the affinity set."""
    seen = {}
    for cpu in sorted(os.sched_getaffinity(0)):
        d = f"/sys/devices/system/cpu/cpu{cpu}/cache/index3"
        try:
            with open(os.path.join(d, "size")) as f:
                size = f.read().strip()
            with open(os.path.join(d, "shared_cpu_list")) as f:
                shared = f.read().strip()
        except OSError:
            continue
        mult = {"K": 1 << 10, "M": 1 << 20, "G": 1 << 30}.get(size[-1:].upper(), 1)
        seen[shared] = int(size.rstrip("KMGkmg")) * mult
    return sum(seen.values())


class HostFlush:
    """Evicts the host's last-level caches: threads on all allowed CPUs
    read-modify-write a buffer of twice their total size (at least 64 MiB,
    at most 4 GiB)."""

    def __init__(self, threads: int):
        import numpy as np
        from concurrent.futures import ThreadPoolExecutor
        llc = host_llc_bytes()
        self.bytes = min(max(2 * llc, 64 << 20), 4 << 30)
        self.llc = llc
        self.buf = np.ones(self.bytes // 8, dtype=np.float64)
        self.chunks = np.array_split(self.buf, max(1, threads))
        self.pool = ThreadPoolExecutor(max(1, threads))

    def __call__(self):
        import numpy as np
        list(self.pool.map(lambda c: np.add(c, 1.0, out=c), self.chunks))

    def close(self):
        self.pool.shutdown()


def cpu_baseline(coo1, xh, Xh, k, flops_v, flops_m, reps):
    """The oracle (plain FP64 C, OpenMP dynamic,64, never tuned) on the
    headline matrix: 2 warm-up + `reps` timed repetitions of one SpMV and one
    SpMM, each call preceded by a host last-level-cache flush, on all host
    threads and on one thread."""
    import numpy as np
    import oracle
    ro = oracle.csr_from_coo(coo1.m, coo1.n, coo1.r, coo1.c, coo1.v)  # the oracle's own assembly
    threads = oracle.max_threads()
    flush = HostFlush(len(os.sched_getaffinity(0)))
    try:
        runs, spent = _cpu_runs(ro, xh, Xh, flush, threads, flops_v, flops_m, reps)
    finally:
        flush.close()   # the flush threads end with the baseline; bench.py starts no process
    return {"value": runs["all"]["gflops"], "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"the headline matrix ({ro.nnz:,} nonzeros), SpMV + SpMM k={k}, FP64; 2 warm-up + "
                      f"{reps} timed repetitions on {threads} threads and on 1 thread, each call after a "
                      f"host LLC flush ({flush.bytes >> 20} MiB touched, 2x the {flush.llc >> 20} MiB of L3); "
                      f"{spent:.1f} s in total",
            "llc_flushed": True, "repetitions": reps, "warmup": 2,
            "spmv_gflops": runs["all"]["spmv_gflops"], "spmm_gflops": runs["all"]["spmm_gflops"],
            "one_thread": runs["one_thread"]}


def _cpu_runs(ro, xh, Xh, flush, threads, flops_v, flops_m, reps):
    import numpy as np
    import oracle
    c0 = time.perf_counter()
    runs = {}
    for label, nth in (("all", threads), ("one_thread", 1)):
        tv, tm = [], []
        for rep in range(2 + reps):
            flush()
            a0 = time.perf_counter()
            oracle.spmv(ro, xh, nthreads=nth)
            a1 = time.perf_counter()
            flush()
            a2 = time.perf_counter()
            oracle.spmm(ro, Xh, nthreads=nth)
            a3 = time.perf_counter()
            if rep >= 2:
                tv.append(a1 - a0)
                tm.append(a3 - a2)
        tv, tm = float(np.mean(tv)), float(np.mean(tm))
        runs[label] = {"threads": nth, "gflops": (flops_v + flops_m) / (tv + tm) / 1e9,
                       "spmv_gflops": flops_v / tv / 1e9, "spmm_gflops": flops_m / tm / 1e9,
                       "spmv_ms": tv * 1e3, "spmm_ms": tm * 1e3}
    return runs, time.perf_counter() - c0


# ---------------------------------------------------------------- headline (c1)

def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the products run on one GPU; --gpus {args.gpus} is not supported "
              "(a row-block sharding over several GPUs is designed but not implemented)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1302_1078_amd as spx
    import spgen

    dev = torch.device("cuda", 0)
    k = args.k
    t0 = time.time()
    coo1 = spgen.workload_c1(seed=0, m=args.rows)
    A = upload(torch, spx, coo1, dev)  # step a1 (device)
    m, n, nnz = A.m, A.n, A.nnz
    # step a2 (device): the binned default plans; the SpMV plan also packs the x
    # entries of the most-used columns (the matrix's column use is skewed: the
    # top 65,536 columns carry 73 % of the nonzeros), a gather that each call
    # repeats inside its timed region
    plan_v = spx.Plan.for_matrix(A, spx.default_opts(1)).attach_hot_x(A, HOT_X_COLUMNS)
    plan_m = spx.Plan.for_matrix(A, spx.default_opts(k))
    x = torch.from_numpy(spgen.uniform(n, 0, spgen.TAG_X)).to(dev)
    X = torch.from_numpy(spgen.uniform(n * k, 0, spgen.TAG_X + 1).reshape(n, k)).to(dev)
    y = torch.empty(m, dtype=torch.float64, device=dev)
    Y = torch.empty((m, k), dtype=torch.float64, device=dev)
    timer = Timer(torch, dev, not args.no_flush)
    torch.cuda.synchronize()
    setup_s = time.time() - t0

    flops_v, flops_m = 2 * nnz, 2 * nnz * k
    bytes_v, bytes_m = app_bytes(m, n, nnz), app_bytes(m, n, nnz, k)
    step = [lambda: spx.spmv(A, x, y=y, plan=plan_v), lambda: spx.spmm(A, X, Y=Y, plan=plan_m)]

    timer.run(step, 0, args.warmup)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    t = timer.run(step, args.steps, 0)
    wall = time.perf_counter() - w0
    tv, tm = t[:, 0], t[:, 1]
    t_step = float(tv.mean() + tm.mean())
    if args.no_warm:
        tvw = tmw = float("nan")
    else:
        tw = Timer(torch, dev, False).run(step, 20, 2)
        tvw, tmw = float(tw[:, 0].mean()), float(tw[:, 1].mean())

    def stats(ts, flops, b, warm):
        return {"ms": ts.mean() * 1e3, "ms_median": float(np.median(ts)) * 1e3, "ms_min": float(ts.min()) * 1e3,
                "gflops": flops / ts.mean() / 1e9, "eff_gbs": b / ts.mean() / 1e9,
                "frac_hbm": b / ts.mean() / 1e9 / PEAK_HBM_GBS, "bytes": b,
                "warm_ms": None if warm != warm else warm * 1e3,
                "warm_eff_gbs": None if warm != warm else b / warm / 1e9}

    detail = {"spmv": stats(tv, flops_v, bytes_v, tvw), "spmm": dict(stats(tm, flops_m, bytes_m, tmw), k=k),
              "plans": {"spmv": dict(plan_v.info(), hot_x_columns=HOT_X_COLUMNS), "spmm": plan_m.info()},
              "flushed": not args.no_flush,
              "setup_s": round(setup_s, 2), "wall_s_timed_incl_flush": round(wall, 4),
              "source_hash": source_hash()}

    # the same SpMV through the plain default plan (no hot x), for comparison
    plan_p = spx.Plan.for_matrix(A, spx.default_opts(1))
    yp = torch.empty_like(y)
    tp = timer.run([lambda: spx.spmv(A, x, y=yp, plan=plan_p)], args.steps, 2)[:, 0]
    detail["spmv_plain_plan"] = dict(stats(tp, flops_v, bytes_v, float("nan")),
                                     hot_x_speedup=float(tp.mean() / tv.mean()),
                                     equals_hot_x_plan_bitwise=bool(torch.equal(yp.view(torch.int64),
                                                                                y.view(torch.int64))))
    del yp

    # random-access ceilings of the two gathers, on buffers the size of X and x
    gather = {}
    for kind, nbytes, per_round, label in (("gather_rows", n * k * 8, 8, "X_rows_128B"),
                                           ("gather_elems", n * 8, 64, "x_elems_8B")):
        buf = torch.zeros(nbytes // 8, dtype=torch.float64, device=dev)
        blocks = 4096
        fn = lambda buf=buf, kind=kind: spx.probe(kind, buf, None, blocks)  # noqa: E731
        tg = float(np.median(Timer(torch, dev, False).run([fn], 5, 2)[:, 0]))
        rate = blocks * 4 * spx.ops.GATHER_ROUNDS * per_round / tg
        gather[label] = {"buffer_bytes": nbytes, "g_accesses_per_s": rate / 1e9}
        del buf
    gather["spmm_x_rows_g_per_s"] = nnz / float(tm.mean()) / 1e9
    gather["spmv_x_elems_g_per_s"] = nnz / float(tv.mean()) / 1e9
    detail["gather_ceiling"] = gather
    detail["latency"] = chase_latency(torch, spx, dev)
    # the paper's own best figures: another machine and other (UFL) matrices, so context only
    detail["paper_context"] = {
        "hardware": "Intel Xeon Phi SE10P (Knights Corner, 61 cores at 1.05 GHz)",
        "precision": "FP64 CRS, int32 indices",
        "spmv_gflops_best": 22.0,        # Sec. 4: best of 22 matrices, compiler-vectorised
        "spmv_gflops_bandwidth_cap": 30.0,  # Sec. 4.2: 180 GB/s sustained x 1/6 flop per byte
        "spmm_k16_gflops_best": 128.0,   # Sec. 5: hand-vectorised, non-temporal Y stores
        "note": "not comparable workloads; vs_baseline stays null"}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(coo1, x.cpu().numpy(), X.cpu().numpy(), k, flops_v, flops_m, args.cpu_reps)
    del coo1

    if not args.quick:
        ctx = {"torch": torch, "spx": spx, "spgen": spgen, "dev": dev, "timer": timer,
               "fsteps": args.form_steps, "tmp": os.environ.get("TMPDIR", "/tmp"),
               "c1_x": x, "c1_X": X, "c1_y": y, "c1_Y": Y, "c1_plans": (plan_p, plan_m),
               "c1_times": (float(tp.mean()), float(tm.mean()))}   # shards use plain plans
        forms = {}
        for name in [f.strip() for f in args.forms.split(",") if f.strip()]:
            f0 = time.time()
            try:
                if name == "c0":
                    forms[name] = bench_c0(ctx)
                elif name == "c2":
                    forms[name] = bench_c2(ctx, A)
                elif name == "c3":
                    forms[name] = bench_c3(ctx)
                elif name == "c4":
                    forms[name] = bench_c4(ctx)
                elif name == "ksweep":
                    forms[name] = bench_ksweep(ctx, A)
                elif name == "occupancy":
                    forms[name] = bench_occupancy(ctx, A)
                elif name == "rcm":
                    forms[name] = bench_rcm(ctx, A)
                elif name == "bcsr":
                    forms[name] = bench_bcsr(ctx, A)
                elif name == "locality":
                    forms[name] = bench_locality(ctx, A)
                elif name == "shard":
                    forms[name] = bench_shard(ctx, A)
                forms[name]["bench_s"] = round(time.time() - f0, 1)
            except Exception as e:  # a failing form is reported, not hidden
                forms[name] = {"error": repr(e)}
            print(f"[bench] {name} done in {time.time() - f0:.1f} s", file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
        detail["forms"] = forms

    dom = "spmm" if tm.mean() >= tv.mean() else "spmv"
    t_dom = float(tm.mean() if dom == "spmm" else tv.mean())
    b_dom = bytes_m if dom == "spmm" else bytes_v
    roofline = {"bound": "hbm", "achieved": b_dom / t_dom / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": b_dom / t_dom / 1e9 / PEAK_HBM_GBS, "traffic": traffic_for(f"k_product_{dom}_c1"),
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
                   "m": m, "n": n, "nnz": nnz, "k": k, "index": "int32", "seed": 0,
                   "plans": f"binned defaults; the SpMV plan packs x of the {HOT_X_COLUMNS:,} most-used columns"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": detail,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
