"""Build the HIP library libbqhip.so (gfx950) in-tree with hipcc.

Each translation unit under csrc/ is compiled to an object in parallel (the
stencil once per storage precision and columns per thread), then linked into
paper_1711_03836_amd/libbqhip.so.  Every build recompiles.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbqhip.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("BQ_OFFLOAD_ARCH", "gfx950")
FLAGS = [
    "-O3", f"--offload-arch={ARCH}", "-fPIC", "-std=c++17",
    "-ffp-contract=on",                    # contraction only inside a source expression
    "-mcode-object-version=5",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",   # no packed FP32 instructions
    "-Wall", "-Wno-unused-function",
    "-I", CSRC, "-I", os.path.join(ROOT, "include"),
]

# (source, object, extra defines): the stencil is compiled once per (storage precision, columns
# per thread) so that its variants build in parallel
STENCIL_R = {0: (1, 2), 1: (1, 2, 3, 4), 2: (1, 2, 3, 4)}
UNITS = [("bq_dslash_inst.hip", f"bq_dslash_p{p}_r{r}.o", [f"-DBQ_INST_PREC={p}", f"-DBQ_INST_R={r}"])
         for p, rs in STENCIL_R.items() for r in rs]
UNITS += [(s, s.replace(".hip", ".o"), []) for s in ("bq_clover.hip", "bq_blas.hip", "bq_krylov.hip", "bq_block.hip", "bq_api.hip")]


def _compile(unit, verbose: bool) -> str:
    src, objname, defs = unit
    obj = os.path.join(BUILD, objname)
    cmd = [HIPCC, *FLAGS, *defs, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{msgs}")
    if msgs.strip() and verbose:
        print(msgs, flush=True)
    return obj


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(UNITS), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, verbose), UNITS))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
           "-Wl,-rpath,/opt/rocm/lib", "-Wl,--no-undefined"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
