"""The C ABI library loads and exports every function include/bqhip.h declares (no GPU needed)."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bqhip.h")
LIB = os.path.join(ROOT, "paper_1711_03836_amd", "libbqhip.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(bq_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_api():
    names = declared()
    for n in ("bq_context_create", "bq_gauge_upload", "bq_op_create", "bq_apply", "bq_solve", "bq_trace"):
        assert n in names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libbqhip.so is not built (run paper_1711_03836_amd/build.py)")
    return C.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (bq_\w+)$", out, flags=re.M))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    for n in declared():
        getattr(lib, n)


def test_binding_covers_header():
    from paper_1711_03836_amd import bqhip
    assert sorted(bqhip.EXPORTED) == declared()


def test_argument_validation_without_device(lib):
    from paper_1711_03836_amd import bqhip as b
    assert b.bq_version() >= 10000
    assert b.bq_context_create(0, 0, b.ALLOC_FN(), b.DEALLOC_FN(), None, None) == b.BQ_ERR_INVALID
    assert b"NULL" in b.bq_last_error()
    assert b.bq_gauge_upload(None, None, None, 0, -1, None) == b.BQ_ERR_INVALID
    assert b.bq_field_create(None, None, 0, 0, 1, None) == b.BQ_ERR_INVALID
    assert b.bq_solve(None, None, None, None, None, None) == b.BQ_ERR_INVALID
    assert b.bq_apply(None, 0, None, None, None) == b.BQ_ERR_INVALID
    # freeing NULL handles is a no-op
    for f in (b.bq_context_destroy, b.bq_gauge_free, b.bq_op_free, b.bq_field_free):
        assert f(None) == b.BQ_OK


def test_solve_parameters_validated_before_any_handle_use(lib):
    """bq_trace and bq_solve reject out-of-range precisions, solvers and tolerances before they touch
    the operator, so a placeholder handle (never dereferenced) suffices on a host without a GPU."""
    from paper_1711_03836_amd import bqhip as b
    dummy = C.create_string_buffer(64)
    h = C.cast(dummy, C.c_void_p)
    t = (C.c_double * 2)()
    for bad in ({"inner_prec": 3}, {"inner_prec": -1}, {"solver": 7}, {"tol": 0.0}, {"tol": float("nan")}):
        kw = {"tol": 1e-10, "maxiter": 100, "inner_prec": b.BQ_F32, "delta": 0.0, "system": b.BQ_SYS_M, "chunk": 4,
              "use_graph": 0, "solver": b.BQ_SOLVER_CG}
        kw.update(bad)
        prm = b.bq_solve_params(kw["tol"], kw["maxiter"], kw["inner_prec"], kw["delta"], kw["system"], kw["chunk"],
                                kw["use_graph"], kw["solver"])
        assert b.bq_trace(h, 1, 1, 1, C.byref(prm), t, t, None) == b.BQ_ERR_INVALID, bad
        assert b.bq_solve(h, h, h, C.byref(prm), None, None) == b.BQ_ERR_INVALID, bad
