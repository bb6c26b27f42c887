"""Micro-benchmark of one operator kind on resident fields (for profiling).

  python -m paper_1711_03836_amd.kernel_bench --dims 32,32,32,64 --prec f32 --nrhs 12 --kind K1 --reps 20

Prints one JSON line: mean launch time from HIP events on the stream the
kernels run on, the algorithmic bytes of one launch and the resulting GB/s.
--copy-mib N first runs a plain device-to-device copy of N MiB (torch), whose
hardware counters calibrate FETCH_SIZE / WRITE_SIZE readings.
"""
import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PREC = {"f64": 0, "f32": 1, "f16": 2}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dims", default="32,32,32,64")
    ap.add_argument("--prec", choices=list(PREC), default="f32")
    ap.add_argument("--nrhs", type=int, default=12)
    ap.add_argument("--kind", default="K1", help="an operator kind (K1, MHAT, ...) or SOLVE")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--tune", default="auto", help="'auto' or recon,R,bs[,march[,lds[,order]]]")
    ap.add_argument("--eps", type=float, default=0.2)
    ap.add_argument("--kappa", type=float, default=0.124)
    ap.add_argument("--csw", type=float, default=1.5)
    ap.add_argument("--mu", type=float, default=0.1)
    ap.add_argument("--tune64", default="auto", help="SOLVE: stencil configuration of the FP64 reliable updates")
    ap.add_argument("--copy-mib", type=int, default=0)
    ap.add_argument("--stream-mib", type=int, default=0, help="measure read / write / copy bandwidth of plain "
                    "torch kernels on N MiB and exit")
    args = ap.parse_args()

    import torch
    from paper_1711_03836_amd import bqhip as bq
    from paper_1711_03836_amd import inputs

    if args.stream_mib:
        n = args.stream_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        c = torch.empty_like(a)
        res = {}
        for name, fn, nbytes in (("read_sum", lambda: a.sum(), n * 4), ("write_fill", lambda: c.fill_(1.0), n * 4),
                                 ("copy", lambda: c.copy_(a), 2 * n * 4),
                                 ("triad", lambda: torch.add(a, c, alpha=2.0, out=c), 3 * n * 4)):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(10):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 10
            res[name] = {"ms": ms, "gbs": nbytes / ms / 1e6}
        print(json.dumps({"stream_mib": args.stream_mib, **res}), flush=True)
        return

    if args.copy_mib:
        n = args.copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        c = torch.empty_like(a)
        c.copy_(a)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        c.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        print(json.dumps({"copy_mib": args.copy_mib, "ms": ms, "gbs": 2 * n * 4 / ms / 1e6}), flush=True)
        del a, c

    dims = tuple(int(v) for v in args.dims.split(","))
    prec = PREC[args.prec]
    U = inputs.gauge_field(dims, args.eps, seed=20171110)
    ctx = bq.Context(0)
    G = bq.Gauge(ctx, dims, U, t_bc=-1)
    op = bq.Op(G, args.kappa, args.csw, args.mu)
    if args.tune == "auto":
        op.autotune(prec, args.nrhs)
    else:
        ctx.tune_set(prec, args.nrhs, *(int(v) for v in args.tune.split(",")))
    if args.kind == "SOLVE":
        # one solve of M x = b for the 12 point sources (inner precision --prec, FP64 reliable updates),
        # so that per-dispatch counters cover the CG iteration's kernels (K2 with the residual update,
        # the vector updates, the reductions)
        b = inputs.point_sources(dims)
        if prec != bq.BQ_F64:
            if args.tune64 == "auto":
                op.autotune(bq.BQ_F64, b.shape[0])
            else:
                ctx.tune_set(bq.BQ_F64, b.shape[0], *(int(v) for v in args.tune64.split(",")))
        fb = bq.Field(ctx, dims, bq.BQ_FULL, bq.BQ_F64, b.shape[0])
        fx = bq.Field(ctx, dims, bq.BQ_FULL, bq.BQ_F64, b.shape[0])
        fb.put(b)
        rc, info = op.solve(fb, fx, 1e-10, system=bq.BQ_SYS_M, inner_prec=prec)
        st = op.stats()
        print(json.dumps({"kind": "SOLVE", "dims": dims, "prec": args.prec, "nrhs": b.shape[0],
                          "tune": ctx.tune_get(prec, b.shape[0]), "tune64": ctx.tune_get(bq.BQ_F64, b.shape[0]),
                          "ms": st["seconds"] * 1e3,
                          "iters": max(i["iters"] for i in info), "launches": st["launches"],
                          "true_rel_resid": max(i["true_rel_resid"] for i in info)}), flush=True)
        return
    kind = getattr(bq, "BQ_OP_" + args.kind)
    si, so = bq.OP_SUBSETS[kind]
    fi = bq.Field(ctx, dims, si, prec, args.nrhs)
    fo = bq.Field(ctx, dims, so, prec, args.nrhs)
    fi.put(inputs.gaussian_spinor(dims, args.nrhs, seed=5))
    stream = torch.cuda.Stream()
    ms, by = op.time_apply(kind, fi, fo, reps=args.reps, stream=stream)
    print(json.dumps({"kind": args.kind, "dims": dims, "prec": args.prec, "nrhs": args.nrhs,
                      "tune": ctx.tune_get(prec, args.nrhs), "ms": ms, "bytes": by, "gbs": by / ms / 1e6,
                      "frac_of_8TBs": by / ms / 1e6 / 8000.0, "launches": args.reps + 1}), flush=True)


if __name__ == "__main__":
    main()
