"""Plain solver and estimator definitions of the CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this
module.  Each function is the textbook algorithm in numpy, on top of the operators of
oracle.py (full-lattice arrays (V, 4, 3); odd-site systems keep even sites at zero), in
FP64, without blocking, fusion or reordering:

  - shifted_cg      the definition behind the "multishift cg" of the solver list (section
                    "Algorithms"; RHMC's rational functions need (W^dag W + b_k)^-1 for all
                    shifts b_k): one plain CG per shift on (Mhat^dag Mhat + sigma_k) x_k = b.
  - bicgstab        BiCGstab of the solver list, in van der Vorst's form, on Mhat x = b.
  - block_cg        the block part of the solver list's "block multishift cg": O'Leary's block CG
                    on Mhat^dag Mhat X = B with the N x N step matrices solved densely.
  - block_multishift_cg
                    the solver list's "block multishift cg": block CG on the base system
                    A + sigma_0 (sigma_0 the smallest shift) whose block residuals serve every
                    shift, R_k^sigma = R_k xi_k^sigma with N x N matrices xi (the block form of
                    the shifted-CG collinearity); each shift gets its own step matrices from the
                    base ones.
  - trace_terms     the per-noise terms of the traces of section "Measurements"
                    (Tr M^-1, Tr gamma_5 M^-1, Tr (M^dag M)^-1) and of the abstract's
                    reweighting traces Tr(M^-1 dM/dp) for p = kappa, c_SW, mu.
"""
from __future__ import annotations

import numpy as np

from . import oracle as orc

# gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 in the chiral basis of bq_oracle.c
GAMMA5_DIAG = np.array([1.0, 1.0, -1.0, -1.0])


def _dot(a, b):
    """<a, b> = sum conj(a) b over all components."""
    return np.vdot(a.reshape(-1), b.reshape(-1))


def _norm(a):
    return float(np.sqrt(np.real(_dot(a, a))))


def normal_op(op):
    """A v = Mhat^dag Mhat v on odd sites."""
    return lambda v: op.Mhat(op.Mhat(v), dagger=True)


def shifted_cg(op, b, sigma, tol, maxiter=100000):
    """x = (Mhat^dag Mhat + sigma)^-1 b by plain CG from x = 0, stopping when |r| <= tol |b|
    (recursive residual).  Returns (x, iterations); iterations = -1 if maxiter was reached."""
    A = normal_op(op)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rho = np.real(_dot(r, r))
    bn = _norm(b)
    if np.sqrt(rho) <= tol * bn:
        return x, 0
    for it in range(1, maxiter + 1):
        Ap = A(p) + sigma * p
        alpha = rho / np.real(_dot(p, Ap))
        x = x + alpha * p
        r = r - alpha * Ap
        rho_new = np.real(_dot(r, r))
        if np.sqrt(rho_new) <= tol * bn:
            return x, it
        p = r + (rho_new / rho) * p
        rho = rho_new
    return x, -1


def multishift(op, b, shifts, tol, maxiter=100000):
    """Every shift's solution of (Mhat^dag Mhat + sigma_k) x_k = b, each by its own CG."""
    return [shifted_cg(op, b, s, tol, maxiter) for s in shifts]


def bicgstab(op, b, tol, maxiter=100000):
    """BiCGstab (van der Vorst 1992) on Mhat x = b (odd sites), x0 = 0, shadow residual r0^ = b.
    Stops when the recursive residual |r| <= tol |b|.  Returns (x, iterations); -1 if maxiter was
    reached or the method broke down."""
    A = op.Mhat
    x = np.zeros_like(b)
    r = b.copy()
    rhat = r.copy()
    rho = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    bn = _norm(b)
    if bn == 0:
        return x, 0
    for it in range(1, maxiter + 1):
        rho_new = _dot(rhat, r)
        if rho_new == 0:
            return x, -1
        beta = (rho_new / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = A(p)
        alpha = rho_new / _dot(rhat, v)
        s = r - alpha * v
        t = A(s)
        tt = np.real(_dot(t, t))
        omega = _dot(t, s) / tt if tt > 0 else 0.0
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho = rho_new
        if _norm(r) <= tol * bn:
            return x, it
        if omega == 0:
            return x, -1
    return x, -1


def block_cg(op, B, tol, maxiter=100000):
    """O'Leary's block CG on A X = B, A = Mhat^dag Mhat, for the N columns of B (shape (N, V, 4, 3))
    at once: with the N x N matrices of inner products taken between all columns,
        Q = A P;  alpha = (P^dag Q)^-1 (R^dag R);  X += P alpha;  R' = R - Q alpha;
        beta = (R^dag R)^-1 (R'^dag R');  P = R' + P beta.
    Stops when every column's recursive residual |r_c| <= tol |b_c|.  Returns (X, iterations)."""
    A = normal_op(op)
    N = B.shape[0]
    shape = B.shape[1:]

    def gram(Xs, Ys):  # G[i, j] = <X_i, Y_j>
        return np.array([[_dot(Xs[i], Ys[j]) for j in range(N)] for i in range(N)])

    def comb(Ps, m):  # column j of the result = sum_i Ps[i] m[i, j]
        return np.einsum("i...,ij->j...", Ps, m)

    X = np.zeros_like(B)
    R = B.copy()
    P = R.copy()
    bn = np.array([_norm(B[c]) for c in range(N)])
    RR = gram(R, R)
    for it in range(1, maxiter + 1):
        Q = np.stack([A(P[c]) for c in range(N)])
        alpha = np.linalg.solve(gram(P, Q), RR)
        X = X + comb(P, alpha)
        R = R - comb(Q, alpha)
        rn = np.array([_norm(R[c]) for c in range(N)])
        if np.all(rn <= tol * bn):
            return X, it
        RR_new = gram(R, R)
        beta = np.linalg.solve(RR, RR_new)
        P = R + comb(P, beta)
        RR = RR_new
    assert X.shape[1:] == shape
    return X, -1


def block_multishift_cg(op, B, shifts, tol, maxiter=100000):
    """Block CG for (Mhat^dag Mhat + sigma_s) X_s = B, all shifts s and the N columns of B
    (shape (N, V, 4, 3)) in one block Krylov space.

    The base system A' = A + sigma_0 (sigma_0 = min shifts) runs O'Leary's block CG,
        alpha_k = (P^dag A' P)^-1 (R^dag R),  X += P alpha_k,  R' = R - A' P alpha_k,
        beta_k = (R^dag R)^-1 (R'^dag R'),  P = R' + P beta_k.
    Its residual blocks satisfy the three-term relation
        A' R_k = -R_{k+1} alpha_k^-1 + R_k (alpha_k^-1 + C_k) - R_{k-1} C_k,  C_k = alpha_{k-1}^-1 beta_{k-1},
    and for a shift d = sigma_s - sigma_0 the block-CG residuals of A' + d are R_k xi_k (the same
    Galerkin conditions).  Matching the two three-term relations column block by column block gives
        (alpha^d_k)^-1 = xi_k^-1 (alpha_k^-1 + C_k + d) xi_k - xi_{k-1}^-1 C_k xi_k   (k = 0: alpha_0^-1 + d),
        beta^d_{k-1} = alpha^d_{k-1} xi_{k-1}^-1 C_k xi_k,
        P^d_k = R_k xi_k + P^d_{k-1} beta^d_{k-1},  X^d += P^d_k alpha^d_k,
        xi_{k+1} = alpha_k^-1 xi_k alpha^d_k,        xi_0 = 1.
    Stops when every shift's every column has |R xi e_c| <= tol |b_c| (the base, the smallest shift,
    is last).  Returns ([X_s for s in shifts], iterations); iterations = -1 if maxiter was reached."""
    A = normal_op(op)
    N = B.shape[0]
    s0 = min(shifts)
    inv = np.linalg.inv
    eye = np.eye(N, dtype=complex)

    def gram(Xs, Ys):  # G[i, j] = <X_i, Y_j>
        return np.array([[_dot(Xs[i], Ys[j]) for j in range(N)] for i in range(N)])

    def comb(Ps, m):  # column j of the result = sum_i Ps[i] m[i, j]
        return np.einsum("i...,ij->j...", Ps, m)

    bn2 = np.array([np.real(_dot(B[c], B[c])) for c in range(N)])
    R = B.copy()
    P = R.copy()
    RR = gram(R, R)
    Xs = [np.zeros_like(B) for _ in shifts]
    Ps = [B.copy() for _ in shifts]
    xi = [eye.copy() for _ in shifts]
    xi_prev = [None] * len(shifts)
    a_prev_s = [None] * len(shifts)
    a_prev = b_prev = None
    for it in range(1, maxiter + 1):
        Q = np.stack([A(P[c]) for c in range(N)]) + s0 * P
        a = np.linalg.solve(gram(P, Q), RR)
        for s, sig in enumerate(shifts):
            d = sig - s0
            if it == 1:
                a_s = inv(inv(a) + d * eye)
            else:
                C = inv(a_prev) @ b_prev
                a_s = inv(inv(xi[s]) @ (inv(a) + C + d * eye) @ xi[s] - inv(xi_prev[s]) @ C @ xi[s])
                b_s = a_prev_s[s] @ inv(xi_prev[s]) @ C @ xi[s]
                Ps[s] = comb(R, xi[s]) + comb(Ps[s], b_s)
            Xs[s] = Xs[s] + comb(Ps[s], a_s)
            xi_prev[s], a_prev_s[s] = xi[s], a_s
            xi[s] = inv(a) @ xi[s] @ a_s
        R = R - comb(Q, a)
        RR_new = gram(R, R)
        done = True
        for s in range(len(shifts)):
            for c in range(N):
                v = xi[s][:, c]
                if np.real(np.vdot(v, RR_new @ v)) > tol * tol * bn2[c]:
                    done = False
        if done:
            return Xs, it
        b = np.linalg.solve(RR, RR_new)
        P = R + comb(P, b)
        a_prev, b_prev, RR = a, b, RR_new
    return Xs, -1


TRACE_TERMS = ("Minv", "Minv2", "g5Minv", "MdagMinv", "dkappa", "dcsw", "dmu")


def trace_terms(op, eta, tol=1e-12):
    """Per-noise terms whose noise averages estimate the traces (E[eta eta^dag] = 1):
        Minv     eta^dag M^-1 eta            -> Tr M^-1
        Minv2    eta^dag M^-2 eta            -> Tr M^-2
        g5Minv   eta^dag gamma_5 M^-1 eta    -> Tr gamma_5 M^-1
        MdagMinv |M^-1 eta|^2                -> Tr (M M^dag)^-1 = Tr (M^dag M)^-1
        dkappa   eta^dag (dM/dkappa) M^-1 eta -> Tr (M^-1 dM/dkappa) = d ln det M / d kappa
        dcsw, dmu likewise for c_SW and mu.
    The solves are the oracle's EO solve to `tol`.  Returns a dict of complex numbers."""
    x1, _ = op.solve_M(eta, tol)
    x2, _ = op.solve_M(x1, tol)
    g5x1 = x1 * GAMMA5_DIAG[None, :, None]
    return {
        "Minv": _dot(eta, x1),
        "Minv2": _dot(eta, x2),
        "g5Minv": _dot(eta, g5x1),
        "MdagMinv": _dot(x1, x1),
        "dkappa": _dot(eta, op.dM(x1, "kappa")),
        "dcsw": _dot(eta, op.dM(x1, "csw")),
        "dmu": _dot(eta, op.dM(x1, "mu")),
    }
