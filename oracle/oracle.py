"""Python face of the FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It wraps `bq_oracle.c` (plain C, double complex, full
lattice) with numpy arrays in the canonical host layout:

  links   U[mu, i, a, b]  shape (4, V, 3, 3) complex128
  spinor  psi[i, s, c]    shape (V, 4, 3)    complex128
  clover  T[i, k, l]      shape (V, 12, 12)  complex128, k = 3*s + c

Every operator follows the paper's definitions: the hopping term with
chemical potential (Eq. 1), the clover term (Eq. 2), the checkerboard
(volume/2) Schur system of the section on SIMD data layout, and the cg solver
of the solver list and Tables 1-2.  The conventions the paper leaves open are
listed at the top of bq_oracle.c.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# BQ_ORACLE_LIB lets the mutation test load a deliberately broken build of the same source.
LIB_PATH = os.environ.get("BQ_ORACLE_LIB") or os.path.join(HERE, "libbqoracle.so")

_lib = None

_cp = C.c_void_p
_i4 = C.POINTER(C.c_int)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.environ.get("BQ_ORACLE_LIB") and (not os.path.exists(LIB_PATH) or os.path.getmtime(
            LIB_PATH) < os.path.getmtime(os.path.join(HERE, "bq_oracle.c"))):
        from . import build as _b
        _b.build()
    lib = C.CDLL(LIB_PATH)
    L4, d, i, l = _i4, C.c_double, C.c_int, C.c_long
    sig = {
        "or_hop": (None, [L4, _cp, i, d, i, _cp, _cp]),
        "or_hop_site": (None, [L4, _cp, i, d, i, _cp, l, _cp]),
        "or_clover": (None, [L4, _cp, d, d, _cp]),
        "or_clover_site": (None, [L4, _cp, d, d, l, _cp]),
        "or_field_strength_site": (None, [L4, _cp, l, i, i, _cp]),
        "or_invert12": (i, [_cp, _cp]),
        "or_clover_invert": (i, [L4, _cp, _cp]),
        "or_clover_apply": (None, [L4, _cp, i, i, _cp, _cp]),
        "or_M_site": (None, [L4, _cp, _cp, d, i, d, i, _cp, l, _cp]),
        "or_apply_M": (None, [L4, _cp, _cp, d, i, d, i, _cp, _cp]),
        "or_apply_Mhat": (None, [L4, _cp, _cp, _cp, d, i, d, i, _cp, _cp, _cp]),
        "or_eo_prepare": (None, [L4, _cp, _cp, d, i, d, _cp, _cp, _cp]),
        "or_eo_reconstruct": (None, [L4, _cp, _cp, d, i, d, _cp, _cp, _cp]),
        "or_cg": (i, [L4, _cp, _cp, _cp, d, i, d, i, _cp, _cp, d, i]),
        "or_plaquette": (d, [L4, _cp]),
        "or_z2_noise": (None, [L4, C.c_uint64, l, _cp]),
        "or_Mhat_sites": (None, [L4, _cp, d, d, i, d, i, _cp, l, _cp, _cp]),
        "or_M_sites": (None, [L4, _cp, d, d, i, d, i, _cp, l, _cp, _cp]),
        "or_clover_sites": (None, [L4, _cp, d, d, l, _cp, _cp]),
        "or_num_threads": (i, []),
        "or_sigma_F": (None, [L4, _cp, _cp]),
        "or_hop_dmu": (None, [L4, _cp, i, d, _cp, _cp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _dims(dims):
    a = (C.c_int * 4)(*[int(x) for x in dims])
    return a


def _c(a, dtype=np.complex128):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def volume(dims):
    return int(np.prod(dims))


def site_parity(dims):
    """Parity (x1+x2+x3+x4) mod 2 of every site, shape (V,)."""
    V = volume(dims)
    i = np.arange(V)
    s = np.zeros(V, dtype=np.int64)
    for L in dims:
        s += i % L
        i = i // L
    return s & 1


def num_threads() -> int:
    return _load().or_num_threads()


# ---------------------------------------------------------------------------
# operators on whole fields
# ---------------------------------------------------------------------------

def hop(dims, U, psi, t_bc=-1, mu=0.0, dagger=False):
    """D psi (Eq. 1 without the mass and kappa), or D^dag psi."""
    lib = _load()
    U = _c(U); psi = _c(psi)
    out = np.empty_like(psi)
    lib.or_hop(_dims(dims), _p(U), int(t_bc), float(mu), int(bool(dagger)), _p(psi), _p(out))
    return out


def clover(dims, U, kappa, csw):
    """T(x) = 1 + kappa c_SW sum_{mu<nu} sigma_{mu nu} F_{mu nu}(x) (Eq. 2), shape (V,12,12)."""
    lib = _load()
    U = _c(U)
    T = np.empty((volume(dims), 12, 12), dtype=np.complex128)
    lib.or_clover(_dims(dims), _p(U), float(kappa), float(csw), _p(T))
    return T


def field_strength_site(dims, U, i, mu, nu):
    lib = _load()
    U = _c(U)
    F = np.empty((3, 3), dtype=np.complex128)
    lib.or_field_strength_site(_dims(dims), _p(U), int(i), int(mu), int(nu), _p(F))
    return F


def clover_invert(dims, T):
    lib = _load()
    T = _c(T)
    Ti = np.empty_like(T)
    if lib.or_clover_invert(_dims(dims), _p(T), _p(Ti)) != 0:
        raise np.linalg.LinAlgError("singular clover block")
    return Ti


def clover_apply(dims, T, psi, adj=False, parity_mask=3):
    lib = _load()
    T = _c(T); psi = _c(psi)
    out = np.empty_like(psi)
    lib.or_clover_apply(_dims(dims), _p(T), int(bool(adj)), int(parity_mask), _p(psi), _p(out))
    return out


def apply_M(dims, U, T, kappa, psi, t_bc=-1, mu=0.0, dagger=False):
    """M psi = T psi - kappa D psi, or M^dag psi."""
    lib = _load()
    U = _c(U); T = _c(T); psi = _c(psi)
    out = np.empty_like(psi)
    lib.or_apply_M(_dims(dims), _p(U), _p(T), float(kappa), int(t_bc), float(mu), int(bool(dagger)),
                   _p(psi), _p(out))
    return out


def apply_Mhat(dims, U, T, Tinv, kappa, psi, t_bc=-1, mu=0.0, dagger=False):
    """Odd-site Schur operator T_oo - kappa^2 D_oe T_ee^-1 D_eo (or its adjoint) on a full-size array."""
    lib = _load()
    U = _c(U); T = _c(T); Tinv = _c(Tinv); psi = _c(psi)
    out = np.empty_like(psi)
    work = np.empty((2,) + psi.shape, dtype=np.complex128)
    lib.or_apply_Mhat(_dims(dims), _p(U), _p(T), _p(Tinv), float(kappa), int(t_bc), float(mu),
                      int(bool(dagger)), _p(psi), _p(out), _p(work))
    return out


def eo_prepare(dims, U, Tinv, kappa, b, t_bc=-1, mu=0.0):
    lib = _load()
    U = _c(U); Tinv = _c(Tinv); b = _c(b)
    out = np.empty_like(b)
    work = np.empty((2,) + b.shape, dtype=np.complex128)
    lib.or_eo_prepare(_dims(dims), _p(U), _p(Tinv), float(kappa), int(t_bc), float(mu), _p(b), _p(out),
                      _p(work))
    return out


def eo_reconstruct(dims, U, Tinv, kappa, b, x_odd, t_bc=-1, mu=0.0):
    lib = _load()
    U = _c(U); Tinv = _c(Tinv); b = _c(b)
    x = np.array(x_odd, dtype=np.complex128, copy=True, order="C")
    work = np.empty((2,) + b.shape, dtype=np.complex128)
    lib.or_eo_reconstruct(_dims(dims), _p(U), _p(Tinv), float(kappa), int(t_bc), float(mu), _p(b), _p(x),
                          _p(work))
    return x


def cg(dims, U, T, Tinv, kappa, b, system, tol, maxiter, t_bc=-1, mu=0.0):
    """Plain CG on M^dag M (system 0, full lattice) or Mhat^dag Mhat (system 1, odd sites)."""
    lib = _load()
    U = _c(U); T = _c(T); b = _c(b)
    Tinv = _c(Tinv) if Tinv is not None else T
    x = np.empty_like(b)
    it = lib.or_cg(_dims(dims), _p(U), _p(T), _p(Tinv), float(kappa), int(t_bc), float(mu), int(system),
                   _p(b), _p(x), float(tol), int(maxiter))
    return x, it


def sigma_F(dims, U):
    """S(x) = sum_{mu<nu} sigma_{mu nu} F_{mu nu}(x), the clover term of Eq. 2 without kappa c_SW,
    shape (V, 12, 12): T = 1 + kappa c_SW S."""
    lib = _load()
    U = _c(U)
    S = np.empty((volume(dims), 12, 12), dtype=np.complex128)
    lib.or_sigma_F(_dims(dims), _p(U), _p(S))
    return S


def hop_dmu(dims, U, psi, t_bc=-1, mu=0.0):
    """(dD/dmu) psi: the time hops of Eq. 1 with e^{+mu} -> +e^{+mu} (forward), e^{-mu} -> -e^{-mu} (backward)."""
    lib = _load()
    U = _c(U); psi = _c(psi)
    out = np.empty_like(psi)
    lib.or_hop_dmu(_dims(dims), _p(U), int(t_bc), float(mu), _p(psi), _p(out))
    return out


def plaquette(dims, U):
    return _load().or_plaquette(_dims(dims), _p(_c(U)))


def z2_noise(dims, seed, n):
    """Complex Z2 noise vector n of the counter-based stream `seed`, shape (V, 4, 3)."""
    eta = np.empty((volume(dims), 4, 3), dtype=np.complex128)
    _load().or_z2_noise(_dims(dims), C.c_uint64(seed & (2**64 - 1)), int(n), _p(eta))
    return eta


# ---------------------------------------------------------------------------
# sampled outputs (large lattices)
# ---------------------------------------------------------------------------

def Mhat_sites(dims, U, kappa, csw, psi, sites, t_bc=-1, mu=0.0, dagger=False):
    lib = _load()
    U = _c(U); psi = _c(psi)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty((len(sites), 4, 3), dtype=np.complex128)
    lib.or_Mhat_sites(_dims(dims), _p(U), float(kappa), float(csw), int(t_bc), float(mu), int(bool(dagger)),
                      _p(psi), len(sites), _p(sites), _p(out))
    return out


def M_sites(dims, U, kappa, csw, psi, sites, t_bc=-1, mu=0.0, dagger=False):
    lib = _load()
    U = _c(U); psi = _c(psi)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty((len(sites), 4, 3), dtype=np.complex128)
    lib.or_M_sites(_dims(dims), _p(U), float(kappa), float(csw), int(t_bc), float(mu), int(bool(dagger)),
                   _p(psi), len(sites), _p(sites), _p(out))
    return out


def clover_sites(dims, U, kappa, csw, sites):
    lib = _load()
    U = _c(U)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    out = np.empty((len(sites), 12, 12), dtype=np.complex128)
    lib.or_clover_sites(_dims(dims), _p(U), float(kappa), float(csw), len(sites), _p(sites), _p(out))
    return out


# ---------------------------------------------------------------------------
# a bundled operator and the solves built on it
# ---------------------------------------------------------------------------

class Operator:
    """M(U; kappa, c_SW, mu) with its clover field and inverse built once."""

    def __init__(self, dims, U, kappa, csw, mu=0.0, t_bc=-1):
        self.dims = tuple(int(d) for d in dims)
        self.V = volume(dims)
        self.U = _c(U)
        self.kappa, self.csw, self.mu, self.t_bc = float(kappa), float(csw), float(mu), int(t_bc)
        self.T = clover(dims, self.U, kappa, csw)
        self.Tinv = clover_invert(dims, self.T)
        self.parity = site_parity(dims)

    def M(self, psi, dagger=False):
        return apply_M(self.dims, self.U, self.T, self.kappa, psi, self.t_bc, self.mu, dagger)

    def Mhat(self, psi, dagger=False):
        return apply_Mhat(self.dims, self.U, self.T, self.Tinv, self.kappa, psi, self.t_bc, self.mu, dagger)

    def hop(self, psi, dagger=False):
        return hop(self.dims, self.U, psi, self.t_bc, self.mu, dagger)

    def odd(self, psi):
        out = np.array(psi, copy=True)
        out[self.parity == 0] = 0
        return out

    def even(self, psi):
        out = np.array(psi, copy=True)
        out[self.parity == 1] = 0
        return out

    def prepare(self, b):
        return eo_prepare(self.dims, self.U, self.Tinv, self.kappa, b, self.t_bc, self.mu)

    def reconstruct(self, b, x_odd):
        return eo_reconstruct(self.dims, self.U, self.Tinv, self.kappa, b, x_odd, self.t_bc, self.mu)

    def cg(self, b, system, tol, maxiter=100000):
        return cg(self.dims, self.U, self.T, self.Tinv, self.kappa, b, system, tol, maxiter, self.t_bc, self.mu)

    def dM(self, psi, param):
        """(dM/dp) psi for p = 'kappa', 'csw' or 'mu', with M = T - kappa D, T = 1 + kappa c_SW S:
        dM/dkappa = c_SW S - D, dM/dc_SW = kappa S, dM/dmu = -kappa dD/dmu."""
        if param == "mu":
            return -self.kappa * hop_dmu(self.dims, self.U, psi, self.t_bc, self.mu)
        if not hasattr(self, "_S"):
            self._S = sigma_F(self.dims, self.U)
        Spsi = np.einsum("ikl,il->ik", self._S, psi.reshape(self.V, 12)).reshape(psi.shape)
        if param == "kappa":
            return self.csw * Spsi - self.hop(psi)
        if param == "csw":
            return self.kappa * Spsi
        raise ValueError(param)

    def solve_M(self, b, tol, maxiter=100000):
        """x = M^-1 b through the odd-site Schur system: bhat, CG on Mhat^dag Mhat, reconstruction."""
        bhat = self.prepare(b)
        bp = self.Mhat(bhat, dagger=True)
        xo, it = self.cg(bp, 1, tol, maxiter)
        return self.reconstruct(b, xo), it


def dense_matrix(apply, n_sites):
    """Dense matrix of a linear map on (n_sites, 4, 3) fields, built column by column from unit vectors."""
    n = n_sites * 12
    A = np.empty((n, n), dtype=np.complex128)
    e = np.zeros((n_sites, 4, 3), dtype=np.complex128)
    flat = e.reshape(-1)
    for k in range(n):
        flat[:] = 0
        flat[k] = 1.0
        A[:, k] = apply(e).reshape(-1)
    return A
