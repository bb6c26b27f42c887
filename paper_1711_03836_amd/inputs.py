"""Seeded synthetic inputs for the Wilson-clover hot path.

This module is the only code shared by the HIP path and the CPU oracle.  It
draws random numbers and lays them out in the canonical host layout; it holds
none of the fermion matrix's arithmetic.

Canonical host layout (C order, complex128):
  * site index  i = x1 + L1*(x2 + L2*(x3 + L3*x4)), directions 0..3 = x,y,z,t
  * gauge links U[mu, i, a, b]   -> shape (4, V, 3, 3)
  * spinors     psi[rhs, i, s, c] -> shape (nrhs, V, 4, 3)

The paper's production runs used QCD gauge ensembles that are not available;
near-unit random SU(3) fields U = exp(i*eps*H) stand in for them, with H a
seeded random traceless Hermitian 3x3 matrix per link.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "volume", "check_dims", "gauge_field", "unit_gauge", "gaussian_spinor",
    "point_sources", "random_gauge_transform", "coords",
]

_CHUNK = 1 << 20  # links generated per numpy batch


def volume(dims) -> int:
    v = 1
    for d in dims:
        v *= int(d)
    return v


def check_dims(dims) -> tuple:
    dims = tuple(int(d) for d in dims)
    if len(dims) != 4 or any(d < 2 or d % 2 for d in dims):
        raise ValueError(f"lattice extents must be 4 even numbers >= 2, got {dims}")
    return dims


def coords(dims):
    """Integer coordinates (V, 4) of every site in canonical order."""
    dims = check_dims(dims)
    V = volume(dims)
    i = np.arange(V, dtype=np.int64)
    x = np.empty((V, 4), dtype=np.int64)
    for mu in range(4):
        x[:, mu] = i % dims[mu]
        i = i // dims[mu]
    return x


def _traceless_hermitian(X):
    """X: (n, 3, 3, 2) iid normals -> traceless Hermitian H = (A + A^dag)/2 - tr/3."""
    A = X[..., 0] + 1j * X[..., 1]
    H = 0.5 * (A + np.conj(np.swapaxes(A, 1, 2)))
    tr = np.trace(H, axis1=1, axis2=2).real / 3.0
    H -= tr[:, None, None] * np.eye(3)
    return H


def _expi(H, eps):
    """exp(i*eps*H) for Hermitian H through its eigendecomposition (unitary)."""
    w, Q = np.linalg.eigh(H)
    return (Q * np.exp(1j * eps * w)[:, None, :]) @ np.conj(np.swapaxes(Q, 1, 2))


def gauge_field(dims, eps: float, seed: int) -> np.ndarray:
    """Links U_mu(x) = exp(i*eps*H_mu(x)), shape (4, V, 3, 3) complex128.

    The generator is numpy's PCG64 seeded with `seed`; each link consumes 18
    standard normals in the order (row, col, re/im), links in the order
    (mu, site).  Generation is chunked but the stream is the same for any
    chunk size.
    """
    dims = check_dims(dims)
    V = volume(dims)
    rng = np.random.default_rng(seed)
    n = 4 * V
    U = np.empty((n, 3, 3), dtype=np.complex128)
    for s in range(0, n, _CHUNK):
        m = min(_CHUNK, n - s)
        X = rng.standard_normal((m, 3, 3, 2))
        U[s:s + m] = _expi(_traceless_hermitian(X), eps)
    return U.reshape(4, V, 3, 3)


def unit_gauge(dims) -> np.ndarray:
    dims = check_dims(dims)
    V = volume(dims)
    U = np.zeros((4, V, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def gaussian_spinor(dims, nrhs: int, seed: int) -> np.ndarray:
    """Complex Gaussian sources: Re, Im iid N(0,1); shape (nrhs, V, 4, 3)."""
    dims = check_dims(dims)
    V = volume(dims)
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((nrhs, V, 4, 3, 2))
    return X[..., 0] + 1j * X[..., 1]


def point_sources(dims) -> np.ndarray:
    """The 12 spin-colour point sources at the origin; column k = 3*s + c."""
    dims = check_dims(dims)
    V = volume(dims)
    b = np.zeros((12, V, 4, 3), dtype=np.complex128)
    for s in range(4):
        for c in range(3):
            b[3 * s + c, 0, s, c] = 1.0
    return b


def random_gauge_transform(dims, seed: int, eps: float = 1.0) -> np.ndarray:
    """Random SU(3) matrix per site, shape (V, 3, 3)."""
    dims = check_dims(dims)
    V = volume(dims)
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((V, 3, 3, 2))
    return _expi(_traceless_hermitian(X), eps)
