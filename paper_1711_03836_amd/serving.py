"""Serving workload: many solve requests of mixed lattice sizes and kappa, Poisson arrivals.

  python -m paper_1711_03836_amd.serving --requests 2000 --load 0.8

Gauge fields U = exp(0.2 i H) on 8^4, 16^3x32, 24^3x48 and 32^3x64 stay resident on
the device.  Each request draws its lattice uniformly from those four, kappa uniform
in [0.118, 0.124] (c_SW = 1.5, mu = 0), 1-12 right-hand sides and a relative residual
of 1e-10, and is served by the continuous-batching server of the C library.

Sources: a pool of seeded complex Gaussian fields per lattice is generated once and kept
on the device; the sources of a request are pool fields shifted cyclically along x by
request-dependent offsets (on the device), so every request has its own Gaussian sources
and neither sources nor solutions cross PCIe.

Latency = completion - arrival (queueing included), on the host clock.  --load L runs
Poisson arrivals at L x the saturated throughput, measured first as a closed loop that
keeps --saturation-outstanding requests submitted at all times (--saturation-requests of
them); --qps sets the rate directly.  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

# Every server session runs on a stream of its own.  HIP maps a process's streams onto a fixed
# number of hardware queues (4 unless set), and streams that share a queue run in submission
# order: a small lattice's chunk would then wait behind a large lattice's kernels.  Four
# sessions, the context stream and torch's stream need 8.  Effective only when set before the
# HIP runtime starts; a smaller value already in the environment is raised.
if int(os.environ.get("GPU_MAX_HW_QUEUES") or 0) < 8:
    os.environ["GPU_MAX_HW_QUEUES"] = "8"

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SIZES = [(8, 8, 8, 8), (16, 16, 16, 32), (24, 24, 24, 48), (32, 32, 32, 64)]
POOL = 3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class World:
    """Resident gauge fields and source pools for the serving lattices."""

    def __init__(self, bq, ctx, sizes=SIZES, eps=0.2, seed=4, pool=POOL):
        import torch
        from paper_1711_03836_amd import inputs
        self.bq, self.ctx, self.sizes = bq, ctx, [tuple(s) for s in sizes]
        self.gauges, self.pools = {}, {}
        for k, d in enumerate(self.sizes):
            U = inputs.gauge_field(d, eps, seed=seed + k)
            self.gauges[d] = bq.Gauge(ctx, d, U, t_bc=-1)
            del U
            self.pools[d] = torch.from_numpy(inputs.gaussian_spinor(d, pool, seed=100 + k)).to("cuda")

    def sources(self, dims, nrhs, rseed):
        """nrhs sources for one request (a device tensor): pool fields rolled along x by
        request-dependent amounts."""
        import torch
        pool = self.pools[dims]
        V = int(np.prod(dims))
        shp = (dims[3], dims[2], dims[1], dims[0], 4, 3)
        cols = [torch.roll(pool[(rseed + k) % pool.shape[0]].reshape(shp), 2 * ((rseed * 7 + k) % (dims[0] // 2)),
                           dims=3).reshape(V, 4, 3) for k in range(nrhs)]
        return torch.stack(cols).contiguous()


def make_requests(n, seed, sizes=SIZES, kappa=(0.118, 0.124), nrhs=(1, 12)):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        out.append({"id": i, "dims": tuple(sizes[rng.integers(len(sizes))]),
                    "kappa": float(rng.uniform(*kappa)), "nrhs": int(rng.integers(nrhs[0], nrhs[1] + 1)),
                    "rseed": int(rng.integers(1 << 30))})
    return out


def run(bq, world, server, reqs, qps=None, seed=0, csw=1.5, tol=1e-10, inner_prec=1, progress=50, outstanding=8):
    """Serve `reqs`: Poisson arrivals with rate qps, or (qps None) a closed loop that keeps
    `outstanding` requests submitted.  Returns a summary dict."""
    rng = np.random.default_rng(seed)
    if qps:
        arrivals = np.cumsum(rng.exponential(1.0 / qps, size=len(reqs)))
        arrivals -= arrivals[0]
    else:
        arrivals = np.zeros(len(reqs))
    t0 = time.perf_counter()
    nxt, pending, lat, info_worst, ncols = 0, {}, [], 0.0, 0
    by_dims = {}
    done_count = 0
    while done_count < len(reqs):
        now = time.perf_counter() - t0
        while nxt < len(reqs) and arrivals[nxt] <= now and (qps or len(pending) < outstanding):
            r = reqs[nxt]
            b = world.sources(r["dims"], r["nrhs"], r["rseed"])
            tk = server.submit(world.gauges[r["dims"]], b, r["kappa"], csw, 0.0, tol, inner_prec)
            pending[tk] = (nxt, t0 + arrivals[nxt] if qps else time.perf_counter())
            nxt += 1
        if not pending:
            time.sleep(max(0.0, min(0.01, arrivals[nxt] - now)))
            continue
        done = server.step()
        tdone = time.perf_counter()
        for tk in done:
            i, tarr = pending.pop(tk)
            rc, info, _ = server.result(tk)
            if rc != bq.BQ_OK:
                raise RuntimeError(f"request {i} failed: {rc} {info}")
            lat.append(tdone - tarr)
            by_dims.setdefault(reqs[i]["dims"], []).append((tdone - tarr, len(info)))
            info_worst = max(info_worst, max(c["true_rel_resid"] for c in info))
            ncols += len(info)
            done_count += 1
            if progress and done_count % progress == 0:
                log(f"[serve] {done_count}/{len(reqs)} done, p50 so far {np.percentile(lat, 50):.3f}s")
    span = time.perf_counter() - t0
    lat = np.array(lat)
    per = {}
    for d, v in sorted(by_dims.items()):
        lv = np.array([a for a, _ in v])
        per["x".join(map(str, d))] = {"requests": len(v), "rhs": int(sum(n for _, n in v)),
                                      "p50_s": float(np.percentile(lv, 50)), "p99_s": float(np.percentile(lv, 99)),
                                      "mean_s": float(lv.mean())}
    return {"requests": len(reqs), "rhs": ncols, "seconds": span, "solves_per_s": len(reqs) / span,
            "rhs_per_s": ncols / span, "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "qps": qps, "worst_true_rel_resid": info_worst, "per_lattice": per}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--saturation-requests", type=int, default=200)
    ap.add_argument("--saturation-outstanding", type=int, default=8)
    ap.add_argument("--load", type=float, nargs="*", default=[0.5, 0.8])
    ap.add_argument("--qps", type=float, default=None)
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--chunk", type=int, default=16)
    ap.add_argument("--sessions", type=int, default=1, help="server sessions per gauge field (bq_server_set_sessions)")
    ap.add_argument("--inner", choices=["f64", "f32", "f16"], default="f32")
    ap.add_argument("--seed", type=int, default=2017)
    ap.add_argument("--out", default=None, help="also write the JSON line to this file")
    args = ap.parse_args()

    from paper_1711_03836_amd import bqhip as bq
    prec = {"f64": 0, "f32": 1, "f16": 2}[args.inner]
    ctx = bq.Context(0)
    log("[serve] building gauge fields and source pools ...")
    world = World(bq, ctx)
    out = {"workload": "serving mix: lattices {8^4, 16^3x32, 24^3x48, 32^3x64}, kappa U[0.118,0.124], c_SW 1.5, "
                       "1-12 Gaussian RHS, tol 1e-10, U=exp(0.2 i H)", "slots": args.slots, "chunk": args.chunk,
           "sessions": args.sessions, "inner_prec": args.inner, "runs": []}
    sat = None
    if args.qps is None:
        server = bq.Server(ctx, args.slots, args.chunk)
        server.set_sessions(args.sessions)
        r = run(bq, world, server, make_requests(args.saturation_requests, args.seed + 1), None, inner_prec=prec,
                outstanding=args.saturation_outstanding)
        server.close()
        sat = r["solves_per_s"]
        out["saturation"] = r
        log(f"[serve] saturated throughput {sat:.2f} requests/s")
    rates = [args.qps] if args.qps else [f * sat for f in args.load]
    for q in rates:
        server = bq.Server(ctx, args.slots, args.chunk)
        server.set_sessions(args.sessions)
        r = run(bq, world, server, make_requests(args.requests, args.seed), q, seed=args.seed, inner_prec=prec)
        server.close()
        r["load"] = q / sat if sat else None
        out["runs"].append(r)
        log(f"[serve] qps {q:.2f}: p50 {r['p50_s']:.3f}s p99 {r['p99_s']:.3f}s, {r['solves_per_s']:.2f} solves/s")
        for d, v in r["per_lattice"].items():
            log(f"[serve]   {d}: {v['requests']} requests, p50 {v['p50_s']:.3f}s p99 {v['p99_s']:.3f}s")
    print(json.dumps(out), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(json.dumps(out) + "\n")


if __name__ == "__main__":
    main()
