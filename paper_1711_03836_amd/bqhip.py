"""ctypes binding of the C ABI in include/bqhip.h (argument marshalling only).

Every function of the header is exposed under the same name; non-zero return
codes raise BqError with the library's message.  Small classes (Context,
Gauge, Op, Field) own the handles and convert numpy arrays (host) or torch
tensors (device) in the canonical layout:

  links  (4, V, 3, 3) complex128      spinors (nrhs, V, 4, 3) complex128

torch is imported before the library is loaded so that both share one HIP
runtime in the process.  There is no fallback: without the built library
this module raises ImportError.
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np

try:  # share torch's HIP runtime when torch is present (device buffers, streams)
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is part of the environment
    torch = None

HERE = os.path.dirname(os.path.abspath(__file__))
# BQHIP_LIBRARY selects another build of the same library (e.g. a variant under test)
LIB_PATH = os.environ.get("BQHIP_LIBRARY") or os.path.join(HERE, "libbqhip.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python paper_1711_03836_amd/build.py` "
                      "(or __graft_entry__.build()) first")

_lib = C.CDLL(LIB_PATH)

BQ_OK = 0
BQ_PENDING = 1
ERRORS = {-1: "BQ_ERR_INVALID", -2: "BQ_ERR_OOM", -3: "BQ_ERR_NOT_CONVERGED", -4: "BQ_ERR_NONFINITE",
          -5: "BQ_ERR_CLOVER_NOT_HPD", -6: "BQ_ERR_BUSY", -7: "BQ_ERR_DEVICE", -8: "BQ_ERR_UNSUPPORTED"}
BQ_ERR_INVALID, BQ_ERR_OOM, BQ_ERR_NOT_CONVERGED, BQ_ERR_NONFINITE = -1, -2, -3, -4
BQ_ERR_CLOVER_NOT_HPD, BQ_ERR_BUSY, BQ_ERR_DEVICE, BQ_ERR_UNSUPPORTED = -5, -6, -7, -8
BQ_NOALLOC_SCRATCH_BYTES = 64 << 20  # static per-device work array of bq_apply_noalloc

BQ_F64, BQ_F32, BQ_F16 = 0, 1, 2
BQ_EVEN, BQ_ODD, BQ_FULL = 0, 1, 2
(BQ_OP_M, BQ_OP_MDAG, BQ_OP_MHAT, BQ_OP_MHATDAG, BQ_OP_MHATDAG_MHAT, BQ_OP_DEO, BQ_OP_DOE, BQ_OP_DEO_DAG,
 BQ_OP_DOE_DAG, BQ_OP_K1, BQ_OP_K1_DAG, BQ_OP_CLOVER, BQ_OP_CLOVER_INV, BQ_OP_MDAGM) = range(14)
BQ_SYS_NORMAL, BQ_SYS_M, BQ_SYS_FULL_NORMAL, BQ_SYS_MHAT = 0, 1, 2, 3
BQ_SOLVER_CG, BQ_SOLVER_BICGSTAB, BQ_SOLVER_BLOCK_CG = 0, 1, 2
TRACE_TERMS = ("Minv", "Minv2", "g5Minv", "MdagMinv", "dkappa", "dcsw", "dmu")  # BQ_TR_* order
BQ_TR_COUNT = len(TRACE_TERMS)

OP_SUBSETS = {BQ_OP_M: (BQ_FULL, BQ_FULL), BQ_OP_MDAG: (BQ_FULL, BQ_FULL), BQ_OP_MDAGM: (BQ_FULL, BQ_FULL),
              BQ_OP_CLOVER: (BQ_FULL, BQ_FULL), BQ_OP_MHAT: (BQ_ODD, BQ_ODD), BQ_OP_MHATDAG: (BQ_ODD, BQ_ODD),
              BQ_OP_MHATDAG_MHAT: (BQ_ODD, BQ_ODD), BQ_OP_DEO: (BQ_ODD, BQ_EVEN), BQ_OP_DEO_DAG: (BQ_ODD, BQ_EVEN),
              BQ_OP_K1: (BQ_ODD, BQ_EVEN), BQ_OP_K1_DAG: (BQ_ODD, BQ_EVEN), BQ_OP_DOE: (BQ_EVEN, BQ_ODD),
              BQ_OP_DOE_DAG: (BQ_EVEN, BQ_ODD), BQ_OP_CLOVER_INV: (BQ_EVEN, BQ_EVEN)}


class bq_solve_params(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxiter", C.c_int), ("inner_prec", C.c_int), ("delta", C.c_double),
                ("system", C.c_int), ("chunk", C.c_int), ("use_graph", C.c_int), ("solver", C.c_int)]


class bq_solve_info(C.Structure):
    _fields_ = [("iters", C.c_int), ("reliable_updates", C.c_int), ("true_rel_resid", C.c_double),
                ("full_rel_resid", C.c_double), ("converged", C.c_int), ("status", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class bq_solve_stats(C.Structure):
    _fields_ = [("bytes", C.c_double), ("seconds", C.c_double), ("launches", C.c_longlong), ("chunks", C.c_int),
                ("iterations", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class BqError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_h = C.c_void_p
_P = C.POINTER
# caller device allocator: void* alloc(size_t bytes, void* ctx); void dealloc(void* ptr, void* ctx)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
DEALLOC_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
_sig = {
    "bq_version": (C.c_int, []),
    "bq_last_error": (C.c_char_p, []),
    "bq_context_create": (C.c_int, [C.c_int, C.c_uint64, ALLOC_FN, DEALLOC_FN, C.c_void_p, _P(_h)]),
    "bq_context_destroy": (C.c_int, [_h]),
    "bq_context_hbm_used": (C.c_int, [_h, _P(C.c_uint64)]),
    "bq_gauge_upload": (C.c_int, [_h, _P(C.c_int), C.c_void_p, C.c_int, C.c_int, _P(_h)]),
    "bq_gauge_plaquette": (C.c_int, [_h, _P(C.c_double)]),
    "bq_gauge_su3_deviation": (C.c_int, [_h, _P(C.c_double)]),
    "bq_gauge_free": (C.c_int, [_h]),
    "bq_op_create": (C.c_int, [_h, C.c_double, C.c_double, C.c_double, _P(_h)]),
    "bq_op_free": (C.c_int, [_h]),
    "bq_field_create": (C.c_int, [_h, _P(C.c_int), C.c_int, C.c_int, C.c_int, _P(_h)]),
    "bq_field_free": (C.c_int, [_h]),
    "bq_field_put": (C.c_int, [_h, C.c_void_p, C.c_int, C.c_void_p]),
    "bq_field_get": (C.c_int, [_h, C.c_void_p, C.c_int, C.c_void_p]),
    "bq_apply": (C.c_int, [_h, C.c_int, _h, _h, C.c_void_p]),
    "bq_apply_noalloc": (C.c_int, [_h, C.c_int, _h, _h, C.c_void_p]),
    "bq_solve": (C.c_int, [_h, _h, _h, _P(bq_solve_params), _P(bq_solve_info), C.c_void_p]),
    "bq_trace": (C.c_int, [_h, C.c_uint64, C.c_int, C.c_int, _P(bq_solve_params), _P(C.c_double), _P(C.c_double),
                           _P(bq_solve_info)]),
    "bq_solve_multishift": (C.c_int, [_h, _h, C.c_int, _P(C.c_double), _P(_h), _P(bq_solve_params),
                                      _P(bq_solve_info), C.c_void_p]),
    "bq_trace_estimators": (C.c_int, [_h, C.c_uint64, C.c_int, C.c_int, _P(bq_solve_params), _P(C.c_double),
                                      _P(bq_solve_info)]),
    "bq_solve_stats_get": (C.c_int, [_h, _P(bq_solve_stats)]),
    "bq_time_apply": (C.c_int, [_h, C.c_int, _h, _h, C.c_int, C.c_void_p, _P(C.c_double), _P(C.c_double)]),
    "bq_time_copy": (C.c_int, [_h, C.c_uint64, C.c_int, C.c_void_p, _P(C.c_double)]),
    "bq_tune_get": (C.c_int, [_h, C.c_int, C.c_int, _P(C.c_int), _P(C.c_int), _P(C.c_int), _P(C.c_int), _P(C.c_int),
                              _P(C.c_int)]),
    "bq_tune_set": (C.c_int, [_h, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]),
    "bq_autotune": (C.c_int, [_h, C.c_int, C.c_int]),
    "bq_server_create": (C.c_int, [_h, C.c_int, C.c_int, _P(_h)]),
    "bq_server_set_backfill": (C.c_int, [_h, C.c_int]),
    "bq_server_set_sessions": (C.c_int, [_h, C.c_int]),
    "bq_server_release": (C.c_int, [_h, _h]),
    "bq_server_submit": (C.c_int, [_h, _h, C.c_double, C.c_double, C.c_double, C.c_void_p, C.c_void_p, C.c_int,
                                   C.c_double, C.c_int, C.c_int, _P(C.c_uint64)]),
    "bq_server_step": (C.c_int, [_h, _P(C.c_uint64), C.c_int, _P(C.c_int)]),
    "bq_server_result": (C.c_int, [_h, C.c_uint64, _P(bq_solve_info)]),
    "bq_server_pending": (C.c_int, [_h, _P(C.c_int), _P(C.c_int)]),
    "bq_server_free": (C.c_int, [_h]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f

EXPORTED = tuple(_sig)


def check(rc):
    if rc != BQ_OK:
        raise BqError(rc, _lib.bq_last_error().decode())
    return rc


def _dims(dims):
    return (C.c_int * 4)(*[int(d) for d in dims])


def _ptr_of(a):
    """(pointer, on_device) for a numpy array or a torch tensor."""
    if torch is not None and isinstance(a, torch.Tensor):
        return C.c_void_p(a.data_ptr()), int(a.is_cuda)
    return a.ctypes.data_as(C.c_void_p), 0


def _order_after_torch(a, stream):
    """For a torch device tensor and no explicit stream: order the library's work after the kernels that
    produced (or are still to overwrite) `a` on torch's current stream.  The library orders itself
    after a stream it is handed; torch's default stream has the handle 0, which the library reads as
    "no stream", so that one is synchronized from the host instead."""
    if stream is None and torch is not None and isinstance(a, torch.Tensor) and a.is_cuda:
        cur = torch.cuda.current_stream(a.device)
        if cur.cuda_stream == 0:
            cur.synchronize()
            return None
        return cur
    return stream


def _check_tensor(a):
    if torch is not None and isinstance(a, torch.Tensor):
        if a.dtype != torch.complex128 or not a.is_contiguous():
            raise ValueError("torch tensors in the canonical layout must be contiguous complex128")


def _stream(stream):
    if stream is None:
        return None
    if torch is not None and isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


# ---------------------------------------------------------------------------
# owning wrappers
# ---------------------------------------------------------------------------

class Context:
    def __init__(self, device=0, hbm_budget=0, alloc=None, dealloc=None):
        """alloc(nbytes) -> device pointer (int) and dealloc(ptr): an optional device allocator of the
        caller (e.g. torch.cuda.caching_allocator_alloc / caching_allocator_delete) through which the
        context takes all of its device memory."""
        h = _h()
        if (alloc is None) != (dealloc is None):
            raise ValueError("give both alloc and dealloc, or neither")
        if alloc is not None:
            # the ctypes callbacks must live as long as the context
            self._afn = ALLOC_FN(lambda n, _ctx: int(alloc(int(n))) or None)
            self._dfn = DEALLOC_FN(lambda p, _ctx: dealloc(int(p)))
        else:
            self._afn, self._dfn = ALLOC_FN(), DEALLOC_FN()
        check(bq_context_create(int(device), int(hbm_budget), self._afn, self._dfn, None, C.byref(h)))
        self.h = h

    def hbm_used(self):
        v = C.c_uint64()
        check(bq_context_hbm_used(self.h, C.byref(v)))
        return v.value

    def time_copy(self, nbytes, reps=10, stream=None):
        """Mean time (ms) of a plain device copy of nbytes (moving 2 * nbytes), HIP events on stream."""
        ms = C.c_double()
        check(bq_time_copy(self.h, int(nbytes), int(reps), _stream(stream), C.byref(ms)))
        return ms.value

    def tune_get(self, prec, nrhs):
        """(recon, R, bs, march, lds, order) of the stencil for this precision and column count."""
        r, R, bs, m, l, o = C.c_int(), C.c_int(), C.c_int(), C.c_int(), C.c_int(), C.c_int()
        check(bq_tune_get(self.h, prec, nrhs, C.byref(r), C.byref(R), C.byref(bs), C.byref(m), C.byref(l),
                          C.byref(o)))
        return r.value, R.value, bs.value, m.value, l.value, o.value

    def tune_set(self, prec, nrhs, recon, R, bs, march=0, lds=0, order=0):
        check(bq_tune_set(self.h, prec, nrhs, recon, R, bs, march, lds, order))

    def save_tuning(self, path, keys, lattice=None):
        """Write the stencil configurations of the (prec, nrhs) pairs in `keys` to a JSON file,
        with the lattice they were tuned on (informational), for load_tuning in a later process."""
        entries = [{"prec": int(p), "nrhs": int(n), "config": list(self.tune_get(p, n))} for p, n in keys]
        with open(path, "w") as f:
            json.dump({"lattice": list(lattice) if lattice else None, "entries": entries}, f, indent=1)

    def load_tuning(self, path):
        """Apply the configurations a save_tuning file holds; returns the (prec, nrhs) pairs set."""
        with open(path) as f:
            doc = json.load(f)
        keys = []
        for e in doc["entries"]:
            self.tune_set(e["prec"], e["nrhs"], *e["config"])
            keys.append((e["prec"], e["nrhs"]))
        return keys

    def close(self):
        if self.h:
            check(bq_context_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Gauge:
    def __init__(self, ctx: Context, dims, links, t_bc=-1):
        self.ctx, self.dims = ctx, tuple(int(d) for d in dims)
        if not (torch is not None and isinstance(links, torch.Tensor)):
            links = np.ascontiguousarray(links, dtype=np.complex128)
        _check_tensor(links)
        if torch is not None and isinstance(links, torch.Tensor) and links.is_cuda:
            torch.cuda.current_stream(links.device).synchronize()  # the upload reads on the library's stream
        p, dev = _ptr_of(links)
        h = _h()
        check(bq_gauge_upload(ctx.h, _dims(dims), p, dev, int(t_bc), C.byref(h)))
        self.h = h
        self._close_pending = False

    def plaquette(self):
        v = C.c_double()
        check(bq_gauge_plaquette(self.h, C.byref(v)))
        return v.value

    def su3_deviation(self):
        v = C.c_double()
        check(bq_gauge_su3_deviation(self.h, C.byref(v)))
        return v.value

    def close(self):
        if self.h:
            check(bq_gauge_free(self.h))
            self.h = None

    def _retry_close(self):
        """Called when an operator or server that used this field lets go of it."""
        if getattr(self, "_close_pending", False) and self.h:
            try:
                self.close()
            except BqError:
                pass

    def __del__(self):
        # finalized while operators or server sessions still use the field (a reference cycle
        # collected in arbitrary order): those free it when they close
        try:
            self.close()
        except Exception as e:  # (module globals may already be gone at interpreter exit)
            self._close_pending = getattr(e, "code", None) == -6  # BQ_ERR_BUSY


class Op:
    def __init__(self, gauge: Gauge, kappa, csw, mu=0.0):
        self.gauge, self.ctx, self.dims = gauge, gauge.ctx, gauge.dims
        self.kappa, self.csw, self.mu = float(kappa), float(csw), float(mu)
        h = _h()
        check(bq_op_create(gauge.h, self.kappa, self.csw, self.mu, C.byref(h)))
        self.h = h

    def apply(self, kind, fin, fout, stream=None):
        check(bq_apply(self.h, kind, fin.h, fout.h, _stream(stream)))

    def apply_noalloc(self, kind, fin, fout, stream=None):
        check(bq_apply_noalloc(self.h, kind, fin.h, fout.h, _stream(stream)))

    def time_apply(self, kind, fin, fout, reps=20, stream=None):
        ms, by = C.c_double(), C.c_double()
        check(bq_time_apply(self.h, kind, fin.h, fout.h, int(reps), _stream(stream), C.byref(ms), C.byref(by)))
        return ms.value, by.value

    def solve(self, b, x, tol, system=BQ_SYS_NORMAL, inner_prec=BQ_F64, maxiter=100000, delta=0.0, chunk=4,
              use_graph=False, stream=None, raise_on_error=True, solver=BQ_SOLVER_CG):
        prm = bq_solve_params(float(tol), int(maxiter), int(inner_prec), float(delta), int(system), int(chunk),
                              int(bool(use_graph)), int(solver))
        info = (bq_solve_info * b.nrhs)()
        rc = bq_solve(self.h, b.h, x.h, C.byref(prm), info, _stream(stream))
        if raise_on_error and rc != BQ_OK:
            check(rc)
        return rc, [i.as_dict() for i in info]

    def trace(self, seed, nnoise, block, tol, inner_prec=BQ_F32, maxiter=100000, chunk=4, use_graph=False):
        prm = bq_solve_params(float(tol), int(maxiter), int(inner_prec), 0.0, BQ_SYS_M, int(chunk),
                              int(bool(use_graph)))
        t1 = (C.c_double * (2 * nnoise))()
        t2 = (C.c_double * (2 * nnoise))()
        info = (bq_solve_info * (2 * nnoise))()
        check(bq_trace(self.h, C.c_uint64(seed & (2**64 - 1)), int(nnoise), int(block), C.byref(prm), t1, t2, info))
        a1 = np.frombuffer(t1, dtype=np.float64).copy()
        a2 = np.frombuffer(t2, dtype=np.float64).copy()
        return a1[0::2] + 1j * a1[1::2], a2[0::2] + 1j * a2[1::2], [i.as_dict() for i in info]

    def solve_multishift(self, b, xs, shifts, tol, maxiter=100000, chunk=8, stream=None, raise_on_error=True,
                         solver=BQ_SOLVER_CG):
        """(A + shifts[k]) xs[k] = b, A = Mhat^dag Mhat on odd sites; returns (rc, info[k][col]).
        solver=BQ_SOLVER_BLOCK_CG: block multishift CG (all columns in one block Krylov space)."""
        n = len(shifts)
        if len(xs) != n:
            raise ValueError("one solution field per shift")
        prm = bq_solve_params(float(tol), int(maxiter), BQ_F64, 0.0, BQ_SYS_NORMAL, int(chunk), 0, int(solver))
        sh = (C.c_double * n)(*[float(v) for v in shifts])
        hx = (_h * n)(*[f.h for f in xs])
        info = (bq_solve_info * (n * b.nrhs))()
        rc = bq_solve_multishift(self.h, b.h, n, sh, hx, C.byref(prm), info, _stream(stream))
        if raise_on_error and rc != BQ_OK:
            check(rc)
        flat = [i.as_dict() for i in info]
        return rc, [flat[k * b.nrhs:(k + 1) * b.nrhs] for k in range(n)]

    def trace_estimators(self, seed, nnoise, block, tol, inner_prec=BQ_F32, maxiter=100000, chunk=4):
        """Per-noise terms of every BQ_TR_* estimator: dict name -> complex array (nnoise,), and info."""
        prm = bq_solve_params(float(tol), int(maxiter), int(inner_prec), 0.0, BQ_SYS_M, int(chunk), 0)
        est = (C.c_double * (2 * BQ_TR_COUNT * nnoise))()
        info = (bq_solve_info * (2 * nnoise))()
        check(bq_trace_estimators(self.h, C.c_uint64(seed & (2**64 - 1)), int(nnoise), int(block), C.byref(prm),
                                  est, info))
        a = np.frombuffer(est, dtype=np.float64).reshape(nnoise, BQ_TR_COUNT, 2)
        z = a[..., 0] + 1j * a[..., 1]
        return {name: z[:, k].copy() for k, name in enumerate(TRACE_TERMS)}, [i.as_dict() for i in info]

    def stats(self):
        st = bq_solve_stats()
        check(bq_solve_stats_get(self.h, C.byref(st)))
        return st.as_dict()

    def autotune(self, prec, nrhs):
        check(bq_autotune(self.h, prec, nrhs))

    def close(self):
        if self.h:
            check(bq_op_free(self.h))
            self.h = None
            self.gauge._retry_close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Field:
    def __init__(self, ctx: Context, dims, subset=BQ_FULL, prec=BQ_F64, nrhs=1):
        self.ctx, self.dims = ctx, tuple(int(d) for d in dims)
        self.subset, self.prec, self.nrhs = subset, prec, nrhs
        self.V = int(np.prod(self.dims))
        h = _h()
        check(bq_field_create(ctx.h, _dims(dims), subset, prec, nrhs, C.byref(h)))
        self.h = h

    def put(self, a, stream=None):
        """a: (nrhs, V, 4, 3) complex128 numpy array or torch tensor (host or device)."""
        if not (torch is not None and isinstance(a, torch.Tensor)):
            a = np.ascontiguousarray(a, dtype=np.complex128)
        if tuple(a.shape) != (self.nrhs, self.V, 4, 3):
            raise ValueError(f"expected shape {(self.nrhs, self.V, 4, 3)}, got {tuple(a.shape)}")
        _check_tensor(a)
        p, dev = _ptr_of(a)
        check(bq_field_put(self.h, p, dev, _stream(_order_after_torch(a, stream))))

    def get(self, out=None, stream=None):
        """Return (nrhs, V, 4, 3) complex128; sites outside the field's subset are zero (or kept from `out`)."""
        if out is None:
            out = np.zeros((self.nrhs, self.V, 4, 3), dtype=np.complex128)
        if tuple(out.shape) != (self.nrhs, self.V, 4, 3):
            raise ValueError(f"expected shape {(self.nrhs, self.V, 4, 3)}, got {tuple(out.shape)}")
        _check_tensor(out)
        p, dev = _ptr_of(out)
        check(bq_field_get(self.h, p, dev, _stream(_order_after_torch(out, stream))))
        return out

    def close(self):
        if self.h:
            check(bq_field_free(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching solve server (see bq_server_* in bqhip.h)."""

    def __init__(self, ctx: Context, slots=16, chunk=16):
        self.ctx = ctx
        h = _h()
        check(bq_server_create(ctx.h, int(slots), int(chunk), C.byref(h)))
        self.h = h
        self._keep = {}  # ticket -> (gauge, b, x): kept alive until retirement
        self._gauges = {}  # gauge fields the server's sessions may hold

    def submit(self, gauge: Gauge, b, kappa, csw, mu=0.0, tol=1e-10, inner_prec=BQ_F32, maxiter=100000):
        """b: (nrhs, V, 4, 3) complex128, numpy (host) or a contiguous torch tensor (host or device);
        the solution x is returned by result() in the same kind of array."""
        if torch is not None and isinstance(b, torch.Tensor):
            if b.dtype != torch.complex128 or not b.is_contiguous():
                raise ValueError("torch sources must be contiguous complex128")
            x = torch.zeros_like(b)
            if b.is_cuda:  # the server reads b on its own stream: finish the work that produced it
                torch.cuda.current_stream(b.device).synchronize()
            bp, xp = C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr())
        else:
            b = np.ascontiguousarray(b, dtype=np.complex128)
            x = np.zeros_like(b)
            bp, xp = b.ctypes.data_as(C.c_void_p), x.ctypes.data_as(C.c_void_p)
        t = C.c_uint64()
        check(bq_server_submit(self.h, gauge.h, float(kappa), float(csw), float(mu), bp, xp, b.shape[0], float(tol),
                               int(inner_prec), int(maxiter), C.byref(t)))
        self._keep[t.value] = (gauge, b, x)
        self._gauges[id(gauge)] = gauge
        return t.value

    def step(self, max_done=4096):
        """Tickets completed in one scheduling step; returns once a session's chunk has finished
        (at once when nothing is in flight)."""
        done = (C.c_uint64 * max_done)()
        n = C.c_int()
        check(bq_server_step(self.h, done, max_done, C.byref(n)))
        return [done[i] for i in range(min(n.value, max_done))]

    def result(self, ticket):
        """(rc, info list, x) once retired; None while pending."""
        g, b, x = self._keep[ticket]
        info = (bq_solve_info * b.shape[0])()
        rc = bq_server_result(self.h, C.c_uint64(ticket), info)
        if rc == BQ_PENDING:
            return None
        del self._keep[ticket]
        return rc, [i.as_dict() for i in info], x

    def pending(self):
        q, r = C.c_int(), C.c_int()
        check(bq_server_pending(self.h, C.byref(q), C.byref(r)))
        return q.value, r.value

    def set_backfill(self, steps):
        check(bq_server_set_backfill(self.h, int(steps)))

    def set_sessions(self, per_key):
        """Sessions per (gauge field, mu, inner precision); see bq_server_set_sessions."""
        check(bq_server_set_sessions(self.h, int(per_key)))

    def release(self, gauge: Gauge):
        check(bq_server_release(self.h, gauge.h))
        self._gauges.pop(id(gauge), None)

    def close(self):
        if self.h:
            check(bq_server_free(self.h))
            self.h = None
            for g in self._gauges.values():
                g._retry_close()
            self._gauges = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
