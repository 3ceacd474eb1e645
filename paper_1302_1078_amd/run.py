"""Run one product on one synthetic workload a few times (for profilers).

    python -m paper_1302_1078_amd.run --workload c1 --op spmm --k 16 --reps 5

Workloads (seed 0): c1 power-law 1,048,576 square (Zipf 2.0, mean 16, max
20,000, hot columns); stencil27 (27-point stencil on 128^3); c3 power-law
524,288 (mean 20); c0 uniform 10,000 x 10,000.  --probe-copy-mib N first
runs a non-temporal copy of N MiB (a known-size kernel that calibrates the
profiler's traffic counters).  Each product call is preceded by a cache flush
unless --no-flush.
"""
from __future__ import annotations

import argparse
import os
import sys


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c1", choices=["c0", "c1", "c3", "stencil27", "c4", "locality"],
                    help="c4: the 256-matrix batch (FP32 values, k in {1, 4, 16}); runs the batch "
                         "and then the same products launched one by one, --reps times each.  "
                         "locality: the locality sweep's matrices in turn (locality_matrices), --op "
                         "xgather / colstream / spmv --reps times on each")
    ap.add_argument("--op", default="spmv", choices=["spmv", "spmm", "xgather", "colstream", "autograd",
                                                     "transpose_atomic"],
                    help="xgather / colstream: the index-gather probe over the matrix's colind "
                         "(with / without the x reads); autograd: forward + backward through the "
                         "autograd Function (values and x both require gradients); transpose_atomic: "
                         "dx = A^T dy by the atomic scatter")
    ap.add_argument("--hot-x", type=int, default=0,
                    help="SpMV through a plan with the x entries of this many most-used columns packed")
    ap.add_argument("--k", type=int, default=16)
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32", "bf16"])
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--lanes", default="", help="comma list: single-bin plans to run after the default")
    ap.add_argument("--staged", action="store_true",
                    help="SpMM through a staged plan (each row tile's X window in LDS) instead of the default")
    ap.add_argument("--pipelined", action="store_true",
                    help="with --staged: the persistent double-buffered staged kernel")
    ap.add_argument("--banded", action="store_true",
                    help="rows ordered band by band of the matrix's bandwidth (plan row_period)")
    ap.add_argument("--bcsr", type=int, default=0,
                    help="SpMM through a x 1 register blocks (a = 2, 4 or 8; FP64), with --banded swept by band")
    ap.add_argument("--probe-copy-mib", type=int, default=0)
    ap.add_argument("--no-flush", action="store_true")
    ap.add_argument("--bandwidth", action="store_true",
                    help="only time the memory probes (read / write / copy of 1 GiB) and exit")
    args = ap.parse_args(argv)

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import torch

    import spgen
    from . import autograd as ops_autograd
    from . import ops
    from ._lib import PlanOpts

    dev = torch.device("cuda", 0)
    if args.bandwidth:
        bandwidth(torch, ops, dev)
        return
    if args.probe_copy_mib:
        a = torch.zeros(args.probe_copy_mib << 17, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        ops.probe("copy", a, b)
        torch.cuda.synchronize()
        del a, b
    if args.workload == "c4":
        batch_vs_single(torch, ops, spgen, dev, args.reps)
        return
    if args.workload == "locality":
        locality_run(torch, ops, spgen, dev, args.op, args.reps, not args.no_flush)
        return
    coo = {"c0": lambda: spgen.workload_c0(0), "c1": lambda: spgen.workload_c1(0),
           "c3": lambda: spgen.workload_c3(0), "stencil27": lambda: spgen.workload_c2_stencil(0)}[args.workload]()
    A = ops.from_coo(coo.m, coo.n, torch.from_numpy(coo.r).to(dev), torch.from_numpy(coo.c).to(dev),
                     torch.from_numpy(coo.v).to(dev))
    vt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[args.dtype]
    xt = torch.float64 if args.dtype == "f64" else torch.float32
    A = A.with_values(A.values.to(vt))
    k = args.k if args.op == "spmm" else 1
    X = torch.from_numpy(spgen.uniform(A.n * k, 0)).to(dev).to(xt)
    X = X if k > 1 else X.reshape(-1)
    X = X.reshape(A.n, k) if k > 1 else X
    Y = torch.empty((A.m, k) if k > 1 else (A.m,), dtype=xt, device=dev)
    flush = None if args.no_flush else torch.zeros(1 << 27, dtype=torch.float64, device=dev)
    if args.op == "autograd":
        g = ops_autograd.GradContext(A)
        v = A.values.clone().requires_grad_(True)
        x = torch.from_numpy(spgen.uniform(A.n, 0)).to(dev).to(xt).requires_grad_(True)
        dy = torch.from_numpy(spgen.normal(A.m, 1)).to(dev).to(xt)
        for _ in range(args.reps):
            if flush is not None:
                ops.probe("flush", flush)
            v.grad = x.grad = None
            ops_autograd.spmv_autograd(v, x, g).backward(dy)
        torch.cuda.synchronize()
        print(f"ran autograd forward + backward on {args.workload} ({A.nnz} nnz, {args.dtype}) x{args.reps}",
              flush=True)
        return
    if args.op == "transpose_atomic":
        # dx = A^T dy by the atomic scatter (mode 1) through the CSR plan
        plan = ops.Plan.for_matrix(A, ops.default_opts(1, vt))
        dy = torch.from_numpy(spgen.normal(A.m, 1)).to(dev).to(xt)
        dx = torch.empty(A.n, dtype=xt, device=dev)
        for _ in range(args.reps):
            if flush is not None:
                ops.probe("flush", flush)
            ops.spmv_t(A, dy, mode=1, plan=plan, out=dx)
        torch.cuda.synchronize()
        print(f"ran atomic transpose on {args.workload} ({A.nnz} nnz, {args.dtype}) x{args.reps}", flush=True)
        return
    if args.op in ("xgather", "colstream"):
        x = torch.from_numpy(spgen.uniform(A.n, 0)).to(dev)
        for _ in range(args.reps):
            if flush is not None:
                ops.probe("flush", flush)
            ops.probe_index_gather(A.colind, x, gather=args.op == "xgather", blocks=4096)
        torch.cuda.synchronize()
        print(f"ran {args.op} on {args.workload} ({A.nnz} indices) x{args.reps}", flush=True)
        return
    if args.bcsr:
        if k == 1 or args.dtype != "f64":
            raise SystemExit("--bcsr serves the FP64 SpMM (k > 1)")
        B = ops.BCSR.from_csr(A, args.bcsr, 1)
        period = ops.bandwidth(A) if args.banded else 0
        for _ in range(args.reps):
            if flush is not None:
                ops.probe("flush", flush)
            ops.bcsr_spmm(B, X, Y=Y, row_period=period)
        torch.cuda.synchronize()
        print(f"ran bcsr_spmm {args.bcsr}x1 on {args.workload} ({B.nblocks} blocks, k={k}) x{args.reps}", flush=True)
        return
    plans = [ops.Plan.staged(A, k, xt, pipelined=args.pipelined) if args.staged
             else ops.Plan.for_matrix(A, ops.banded_opts(A, k, vt) if args.banded else ops.default_opts(k, vt))]
    if args.hot_x:
        if k != 1:
            raise SystemExit("--hot-x serves the SpMV (--op spmv)")
        plans[0].attach_hot_x(A, args.hot_x, xdtype=xt)
    for l in [int(s) for s in args.lanes.split(",") if s.strip()]:
        plans.append(ops.Plan.for_matrix(A, PlanOpts.from_dict({"nbins": 1, "upper": [], "lanes": [l],
                                                                 "split_chunk": 4096, "max_k": k})))
    for plan in plans:
        for _ in range(args.reps):
            if flush is not None:
                ops.probe("flush", flush)
            if k == 1:
                ops.spmv(A, X, y=Y, plan=plan)
            else:
                ops.spmm(A, X, Y=Y, plan=plan)
    torch.cuda.synchronize()
    print(f"ran {args.op} on {args.workload} ({A.m} rows, {A.nnz} nnz, k={k}, {args.dtype}) "
          f"x{args.reps} per plan, {len(plans)} plan(s)", flush=True)


LOCALITY = ("powerlaw_col1.6", "powerlaw_col2.0", "powerlaw_col2.0_degree", "powerlaw_col2.4",
            "stencil27_natural", "stencil27_half_relabeled", "stencil27_relabeled")


def locality_matrices(torch, ops, spgen, dev):
    """The locality sweep (the paper's Sec. 4.1-4.2 study of how the x access
    pattern sets SpMV speed), one matrix at a time as (name, device CSR), in
    LOCALITY order: the headline power-law row lengths (1,048,576 square,
    Zipf 2.0, mean 16) with column laws of exponent 1.6, 2.0 and 2.4, the 2.0
    matrix in degree order, and the 27-point stencil on 128^3 in natural
    order, with half of its vertices relabelled at random, and fully
    relabelled.  FP64 values."""
    def up(coo):
        return ops.from_coo(coo.m, coo.n, torch.from_numpy(coo.r).to(dev), torch.from_numpy(coo.c).to(dev),
                            torch.from_numpy(coo.v).to(dev))
    for ca in (1.6, 2.0, 2.4):
        A = up(spgen.powerlaw(1 << 20, 1 << 20, 2.0, 20_000, 16.0, 0, col_alpha=ca))
        yield f"powerlaw_col{ca}", A
        if ca == 2.0:
            yield "powerlaw_col2.0_degree", ops.permute(A, ops.degree_order(A))
        del A
    st = spgen.workload_c2_stencil(0)
    yield "stencil27_natural", up(st)
    yield "stencil27_half_relabeled", up(spgen.relabeled(st, 1, 0.5))
    yield "stencil27_relabeled", up(spgen.relabeled(st, 1))


def locality_run(torch, ops, spgen, dev, op: str, reps: int, flush: bool):
    """For counter runs: `op` (xgather, colstream or spmv with the default
    plan) `reps` times on each locality matrix, in LOCALITY order, each call
    after a 1 GiB flush."""
    fb = torch.zeros(1 << 27, dtype=torch.float64, device=dev) if flush else None
    for name, A in locality_matrices(torch, ops, spgen, dev):
        x = torch.from_numpy(spgen.uniform(A.n, 0)).to(dev)
        plan = ops.Plan.for_matrix(A, ops.default_opts(1)) if op == "spmv" else None
        y = torch.empty(A.m, dtype=torch.float64, device=dev)
        for _ in range(reps):
            if fb is not None:
                ops.probe("flush", fb)
            if op == "spmv":
                ops.spmv(A, x, y=y, plan=plan)
            else:
                ops.probe_index_gather(A.colind, x, gather=op == "xgather", blocks=4096)
        torch.cuda.synchronize()
        print(f"locality {name}: {op} x{reps} ({A.m} rows, {A.nnz} nnz)", flush=True)


def batch_vs_single(torch, ops, spgen, dev, reps: int):
    """The 256-matrix batch (default plans, stream bins kept as tiles, as a
    batch runs them) and the same products as single launches."""
    from ._lib import SPX_FLAG_KEEP_STREAM
    from .batch import Batched
    mats, Xs, opts = [], [], []
    for i, s in enumerate(spgen.batch_specs(256, seed=0)):
        coo = spgen.batch_matrix(s, 0, i)
        A = ops.from_coo(coo.m, coo.n, torch.from_numpy(coo.r).to(dev), torch.from_numpy(coo.c).to(dev),
                         torch.from_numpy(coo.v).to(dev))
        A = A.with_values(A.values.float())
        X = torch.from_numpy(spgen.uniform(A.n * s.k, 1000 + i, spgen.TAG_X)).to(dev).float()
        Xs.append(X if s.k == 1 else X.reshape(A.n, s.k))
        o = ops.default_opts(s.k, torch.float32)
        o.flags |= SPX_FLAG_KEEP_STREAM
        mats.append(A)
        opts.append(o)
    plans = [ops.Plan.for_matrix(A, o) for A, o in zip(mats, opts)]
    outs = [torch.empty((A.m,) if X.dim() == 1 else (A.m, X.shape[1]), device=dev) for A, X in zip(mats, Xs)]
    B = Batched(mats, Xs, opts=opts)
    for _ in range(reps):
        B.run()
        torch.cuda.synchronize()
        for A, X, p, Y in zip(mats, Xs, plans, outs):
            if X.dim() == 1:
                ops.spmv(A, X, y=Y, plan=p)
            else:
                ops.spmm(A, X, Y=Y, plan=p)
        torch.cuda.synchronize()
    same = all(torch.equal(a, b) for a, b in zip(outs, B.Ys))
    print(f"ran the 256-matrix batch and its single launches x{reps}; bitwise equal: {same}", flush=True)


def bandwidth(torch, ops, dev, reps: int = 20):
    """Median GB/s of the streaming probes over 1 GiB buffers (HIP events)."""
    import statistics
    a = torch.zeros(1 << 27, dtype=torch.float64, device=dev)
    b = torch.zeros_like(a)
    sink = torch.zeros(1, dtype=torch.float64, device=dev)
    nbytes = a.numel() * 8
    cases = {"read": (lambda: ops.probe("read", a, sink, 16384), nbytes),
             "write": (lambda: ops.probe("write", a, None, 16384), nbytes),
             "write_nt": (lambda: ops.probe("write_nt", a, None, 16384), nbytes),
             "copy": (lambda: ops.probe("copy", a, b, 16384), 2 * nbytes)}
    for name, (fn, moved) in cases.items():
        fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            ts.append((e0, e1))
        torch.cuda.synchronize()
        ms = statistics.median(x.elapsed_time(y) for x, y in ts)
        print(f"{name:9s} {moved / 2**30:.0f} GiB moved  {ms * 1e3:8.1f} us  {moved / ms / 1e6:7.0f} GB/s", flush=True)


if __name__ == "__main__":
    main()
