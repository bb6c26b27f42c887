"""The solver workloads besides the 12-point-source benchmark, each printing one JSON line.

  python -m paper_1711_03836_amd.workloads solve16
      16^3x32, U = exp(0.2 i H), kappa = 0.125, c_SW = 1.7, mu = 0, one complex Gaussian source,
      M x = b through the odd-site Schur system to a relative residual of 1e-10: plain FP64 CG
      against FP32-inner and FP16-inner CG with FP64 reliable updates, on the same GPU.
  python -m paper_1711_03836_amd.workloads trace48 [--inner f32|f16] [--nnoise 64] [--block 16]
      48^3x96, U = exp(0.15 i H), kappa = 0.1235, c_SW = 1.9, mu = 0: Tr M^-1 and Tr M^-2 from
      complex Z2 noise vectors solved in blocks, mixed precision, residual 1e-8, autotuned stencil.

Inputs are resident on the device before the timed solves; times are device times of the solve
calls (HIP events) and the host wall clock around them.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PREC = {"f64": 0, "f32": 1, "f16": 2}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def solve16(args):
    import torch
    from paper_1711_03836_amd import bqhip as bq
    from paper_1711_03836_amd import inputs
    dims, eps, kappa, csw, tol = (16, 16, 16, 32), 0.2, 0.125, 1.7, 1e-10
    U = inputs.gauge_field(dims, eps, seed=1711)
    b = inputs.gaussian_spinor(dims, 1, seed=3836)
    ctx = bq.Context(0)
    G = bq.Gauge(ctx, dims, U, t_bc=-1)
    op = bq.Op(G, kappa, csw, 0.0)
    fb = bq.Field(ctx, dims, bq.BQ_FULL, bq.BQ_F64, 1)
    fx = bq.Field(ctx, dims, bq.BQ_FULL, bq.BQ_F64, 1)
    fb.put(b)
    for p in (0, 1, 2):
        op.autotune(p, 1)
    out = {"workload": "16^3x32 EO-clover CG, 1 Gaussian source, U=exp(0.2 i H), kappa 0.125, c_SW 1.7, mu 0, "
                       "tol 1e-10 (M x = b through Mhat^dag Mhat)", "plaquette": G.plaquette(), "runs": {}}
    for name in ("f64", "f32", "f16"):
        p = PREC[name]
        op.solve(fb, fx, tol, system=bq.BQ_SYS_M, inner_prec=p, chunk=args.chunk)  # warm-up
        torch.cuda.synchronize()
        best = None
        for _ in range(args.reps):
            t0 = time.perf_counter()
            rc, info = op.solve(fb, fx, tol, system=bq.BQ_SYS_M, inner_prec=p, chunk=args.chunk)
            wall = time.perf_counter() - t0
            st = op.stats()
            if best is None or st["seconds"] < best[1]["seconds"]:
                best = (info[0], st, wall)
        info, st, wall = best
        out["runs"][name] = {"device_ms": st["seconds"] * 1e3, "wall_ms": wall * 1e3, "iters": info["iters"],
                             "reliable_updates": info["reliable_updates"],
                             "true_rel_resid": info["true_rel_resid"], "full_rel_resid": info["full_rel_resid"],
                             "gbs": st["bytes"] / st["seconds"] / 1e9, "tune": ctx.tune_get(p, 1)}
        log(f"[solve16] {name}: {st['seconds'] * 1e3:.1f} ms, {info['iters']} iterations, "
            f"{info['reliable_updates']} reliable updates, true residual {info['true_rel_resid']:.2e}")
    r = out["runs"]
    out["speedup_f32_vs_f64"] = r["f64"]["device_ms"] / r["f32"]["device_ms"]
    out["speedup_f16_vs_f64"] = r["f64"]["device_ms"] / r["f16"]["device_ms"]
    print(json.dumps(out), flush=True)


def trace48(args):
    import torch
    from paper_1711_03836_amd import bqhip as bq
    from paper_1711_03836_amd import inputs
    dims = tuple(int(v) for v in args.dims.split(","))
    eps, kappa, csw, tol = 0.15, 0.1235, 1.9, 1e-8
    V = int(np.prod(dims))
    log(f"[trace] generating U = exp(i*{eps}*H) on {dims} ...")
    t0 = time.time()
    U = inputs.gauge_field(dims, eps, seed=48096)
    log(f"[trace] links ready in {time.time() - t0:.1f}s")
    ctx = bq.Context(0)
    G = bq.Gauge(ctx, dims, U, t_bc=-1)
    del U
    op = bq.Op(G, kappa, csw, 0.0)
    inner = PREC[args.inner]
    for p in {inner, 0}:
        op.autotune(p, args.block)
        log(f"[trace] tune prec {p} x{args.block}: {ctx.tune_get(p, args.block)}")
    torch.cuda.synchronize()
    # one library call per block (noise seeds seed, seed+1, ...), so that progress is visible
    t1, t2, info1, info2 = [], [], [], []
    dev, nbytes = 0.0, 0.0
    t0 = time.perf_counter()
    for k in range(args.nnoise // args.block):
        a, b, inf = op.trace(seed=args.seed + k, nnoise=args.block, block=args.block, tol=tol, inner_prec=inner,
                             chunk=args.chunk)
        st = op.stats()
        dev += st["seconds"]
        nbytes += st["bytes"]
        t1.append(a)
        t2.append(b)
        info1 += inf[:args.block]
        info2 += inf[args.block:]
        log(f"[trace] block {k}: {st['seconds']:.1f}s device, iterations {max(c['iters'] for c in inf)}")
    wall = time.perf_counter() - t0
    t1, t2, info = np.concatenate(t1), np.concatenate(t2), info1 + info2
    st = {"seconds": dev, "bytes": nbytes}
    n = len(t1)

    def est(t):
        m = t.mean()
        se = t.real.std(ddof=1) / np.sqrt(n) if n > 1 else float("nan")
        return {"re": float(m.real), "im": float(m.imag), "stderr": float(se), "per_site_component": float(m.real / (12 * V))}

    first, second = info[:n], info[n:]
    out = {"workload": f"{'x'.join(map(str, dims))} stochastic traces, U=exp({eps} i H), kappa {kappa}, c_SW {csw}, "
                       f"mu 0, {n} complex Z2 noises in blocks of {args.block}, tol {tol:g}, {args.inner} inner + "
                       "f64 reliable updates",
           "tr_Minv": est(t1), "tr_Minv2": est(t2), "wall_s": wall, "device_s": st["seconds"],
           "s_per_noise": wall / n, "gbs": st["bytes"] / st["seconds"] / 1e9,
           "iters_first": [int(min(c["iters"] for c in first)), int(max(c["iters"] for c in first))],
           "iters_second": [int(min(c["iters"] for c in second)), int(max(c["iters"] for c in second))],
           "worst_true_rel_resid": max(c["true_rel_resid"] for c in info),
           "worst_full_rel_resid": max(c["full_rel_resid"] for c in info),
           "tune": {args.inner: ctx.tune_get(inner, args.block), "f64": ctx.tune_get(0, args.block)}}
    log(f"[trace] Tr M^-1 = {out['tr_Minv']['re']:.6e} +- {out['tr_Minv']['stderr']:.2e}, "
        f"Tr M^-2 = {out['tr_Minv2']['re']:.6e} +- {out['tr_Minv2']['stderr']:.2e}; {wall:.1f}s")
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("solve16")
    a.add_argument("--reps", type=int, default=2)
    a.add_argument("--chunk", type=int, default=4)
    b = sub.add_parser("trace48")
    b.add_argument("--dims", default="48,48,48,96")
    b.add_argument("--inner", choices=["f32", "f16"], default="f32")
    b.add_argument("--nnoise", type=int, default=64)
    b.add_argument("--block", type=int, default=16)
    b.add_argument("--seed", type=int, default=20171110, help="noise seed of the first block (block k: seed + k)")
    b.add_argument("--chunk", type=int, default=4)
    args = ap.parse_args()
    {"solve16": solve16, "trace48": trace48}[args.cmd](args)


if __name__ == "__main__":
    main()
