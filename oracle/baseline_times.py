"""Wall time of the CPU oracle on the benchmark's workloads (test infrastructure: runs the oracle only).

  python -m oracle.baseline_times [--out FILE.json] [--skip-full32] [--skip-48]

Prints one JSON line with the host's CPU model, the OpenMP threads the oracle uses, and
  - apply: per lattice of the workloads (4^4, 16^3x32, 32^3x64, 48^3x96) the time of one
    application of M, of D_eo (the hopping term from odd to even sites) and of Mhat, and the
    operator set-up (clover field and its inverse);
  - plain4: FP64 CG on M^dag M over the full 4^4 lattice (no preconditioning), kappa 0.12,
    c_SW 1.0, mu 0, U = exp(0.3 i H), one complex Gaussian source, tol 1e-12;
  - eo16: M x = b on 16^3x32 through the odd-site Schur system (preparation, CG on
    Mhat^dag Mhat to 1e-10, reconstruction), kappa 0.125, c_SW 1.7, U = exp(0.2 i H), one
    Gaussian source;
  - eo32: the same for the first of the 12 point sources on 32^3x64 (kappa 0.124, c_SW 1.5,
    mu 0.1), and the time of all 12 EXTRAPOLATED as 12 x that solve;
  - trace48: the 48^3x96 trace workload (64 noises, two solves each) EXTRAPOLATED from the
    oracle's CG iteration time there and the iteration counts of the GPU run (--trace-iters).
The oracle is plain C over full-lattice arrays (odd-site systems keep even sites at zero), so
its per-site work is not the GPU's; its times are a reported baseline.
"""
import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from paper_1711_03836_amd import inputs  # noqa: E402


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def timed(fn, *a):
    t0 = time.perf_counter()
    out = fn(*a)
    return out, time.perf_counter() - t0


def log(msg):
    print(f"[oracle] {msg}", file=sys.stderr, flush=True)


# (name, dims, link roughness eps, kappa, c_SW, mu)
LATTICES = [("4^4", (4, 4, 4, 4), 0.3, 0.12, 1.0, 0.0),
            ("16^3x32", (16, 16, 16, 32), 0.2, 0.125, 1.7, 0.0),
            ("32^3x64", (32, 32, 32, 64), 0.2, 0.124, 1.5, 0.1),
            ("48^3x96", (48, 48, 48, 96), 0.15, 0.1235, 1.9, 0.0)]


def applies(ref, seed):
    psi = inputs.gaussian_spinor(ref.dims, 1, seed=seed)[0]
    po = ref.odd(psi)
    _, tM = timed(ref.M, psi)
    _, tD = timed(lambda v: ref.even(ref.hop(v)), po)
    _, tMh = timed(ref.Mhat, po)
    return {"M_seconds": tM, "Deo_seconds": tD, "Mhat_seconds": tMh}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--skip-full32", action="store_true", help="no full 32^3x64 solve")
    ap.add_argument("--skip-48", action="store_true", help="no 48^3x96 lattice")
    ap.add_argument("--trace-iters", type=int, default=250, help="CG iterations per noise of the GPU trace run")
    args = ap.parse_args()
    out = {"cpu_model": cpu_model(), "threads": orc.num_threads(), "logical_cpus": os.cpu_count(), "apply": {}}
    ops = {}
    for k, (name, dims, eps, kappa, csw, mu) in enumerate(LATTICES):
        if name == "48^3x96" and args.skip_48:
            continue
        U = inputs.gauge_field(dims, eps, seed=20171110 if name == "32^3x64" else 11 + k)
        ref, tset = timed(orc.Operator, dims, U, kappa, csw, mu)
        a = applies(ref, 31 + k)
        a["setup_seconds"] = tset
        out["apply"][name] = a
        log(f"{name}: set-up {tset:.1f}s, M {a['M_seconds']:.3f}s, D_eo {a['Deo_seconds']:.3f}s, "
            f"Mhat {a['Mhat_seconds']:.3f}s")
        if name == "48^3x96":
            po = ref.odd(inputs.gaussian_spinor(dims, 1, seed=41)[0])
            _, tcg = timed(ref.cg, po, 1, 1e-30, 2)
            out["trace48"] = {"cg_iteration_seconds": tcg / 2, "iters_per_noise": args.trace_iters,
                              "extrapolated_64_noises_seconds": 64 * args.trace_iters * tcg / 2}
            log(f"48^3x96: CG iteration {tcg / 2:.2f}s")
        else:
            ops[name] = (ref, dims)
        del U

    # 4^4, plain FP64 CG on M^dag M
    ref, dims = ops["4^4"]
    b = inputs.gaussian_spinor(dims, 1, seed=12)[0]
    (x, it), dt = timed(ref.cg, ref.M(b, dagger=True), 0, 1e-12)
    out["plain4"] = {"seconds": dt, "iters": it,
                     "rel_resid_M": float(np.linalg.norm(b - ref.M(x)) / np.linalg.norm(b))}
    log(f"4^4 plain CG: {dt:.3f}s, {it} iterations")

    # 16^3x32, even-odd solve of M x = b
    ref, dims = ops["16^3x32"]
    b = inputs.gaussian_spinor(dims, 1, seed=22)[0]
    (x, it), dt = timed(ref.solve_M, b, 1e-10)
    out["eo16"] = {"seconds": dt, "iters": it,
                   "rel_resid_M": float(np.linalg.norm(b - ref.M(x)) / np.linalg.norm(b))}
    log(f"16^3x32 EO solve: {dt:.1f}s, {it} iterations")

    # 32^3x64, one of the 12 point sources
    ref, dims = ops["32^3x64"]
    if not args.skip_full32:
        b = inputs.point_sources(dims)[0]
        (x, it), dt = timed(ref.solve_M, b, 1e-10)
        out["eo32"] = {"seconds": dt, "iters": it,
                       "rel_resid_M": float(np.linalg.norm(b - ref.M(x)) / np.linalg.norm(b)),
                       "extrapolated_12_sources_seconds": 12 * dt}
        log(f"32^3x64 point-source solve: {dt:.1f}s, {it} iterations")
    line = json.dumps(out)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
