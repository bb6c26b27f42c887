"""Pins of the oracle's solvers and trace estimators (oracle/solvers.py) against dense linear
algebra, finite differences and closed forms on tiny lattices.

  - shifted CG (the multishift cg of the solver list, section "Algorithms"): numpy's dense solve
    of (Mhat^dag Mhat + sigma) x = b for several shifts;
  - BiCGstab (solver list) on the non-Hermitian Mhat (mu != 0): dense solve of Mhat x = b;
  - block CG (solver list): dense solve for 3 right-hand sides, and with one right-hand side it is
    plain CG (same iterations, same iterate);
  - block multishift CG (solver list): every shift's solution against the dense solve of
    (Mhat^dag Mhat + sigma) X = B, with and without a zero shift; with one shift it is block CG (same
    iterations, same iterate); with one column it takes the iterations of CG on the smallest shift;
    planted mistakes in its shift recurrences (source mutations of the oracle function) fail the pins;
  - trace terms (section "Measurements", the abstract's reweighting traces): per noise equal to
    eta^dag A eta with the dense A; the dM/dp operators equal the derivative of the oracle's own
    M (central differences of dense M(p)), so Tr(M^-1 dM/dp) is the derivative of ln det M;
    Tr gamma_5 M^-1 = 0 in the free field; noise averages within 4 standard errors of the exact
    traces.
Each group also plants a plausible mistake in a copy of the algorithm and checks that its pin
fails.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from oracle import solvers as sv
from paper_1711_03836_amd import inputs


def rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


@pytest.fixture(scope="module", params=[((2, 2, 2, 2), 0.1), ((2, 4, 2, 4), -0.15)])
def tiny(request):
    dims, mu = request.param
    U = inputs.gauge_field(dims, 0.3, seed=70)
    op = orc.Operator(dims, U, 0.12, 1.1, mu=mu)
    V = op.V
    par = np.repeat(op.parity, 12)
    o = np.where(par == 1)[0]
    Mhat = orc.dense_matrix(op.Mhat, V)[np.ix_(o, o)]
    b = np.stack([op.odd(v) for v in inputs.gaussian_spinor(dims, 3, seed=71)])
    return dims, op, o, Mhat, b


def _odd_vec(b, o):
    return b.reshape(-1)[o]


# --- shifted CG ---------------------------------------------------------------------

def _check_shifted(solve, op, o, Mhat, b, shifts):
    A = Mhat.conj().T @ Mhat
    for s in shifts:
        x, it = solve(op, b[0], s, 1e-13)
        want = np.linalg.solve(A + s * np.eye(len(o)), _odd_vec(b[0], o))
        if it <= 0 or rel(_odd_vec(x, o), want) > 1e-10:
            return False
        if np.abs(x.reshape(-1)[np.setdiff1d(np.arange(x.size), o)]).max() != 0:
            return False
    return True


def test_shifted_cg_dense(tiny):
    dims, op, o, Mhat, b = tiny
    assert _check_shifted(sv.shifted_cg, op, o, Mhat, b, (0.0, 0.05, 0.7))
    xs = sv.multishift(op, b[1], (0.0, 0.2), 1e-13)
    A = Mhat.conj().T @ Mhat
    for (x, it), s in zip(xs, (0.0, 0.2)):
        assert rel(_odd_vec(x, o), np.linalg.solve(A + s * np.eye(len(o)), _odd_vec(b[1], o))) < 1e-10


def test_shifted_cg_planted_mistake(tiny):
    dims, op, o, Mhat, b = tiny

    def wrong_sign(op_, bb, sigma, tol, maxiter=100000):  # (A - sigma) instead of (A + sigma)
        return sv.shifted_cg(op_, bb, -sigma, tol, maxiter)
    assert not _check_shifted(wrong_sign, op, o, Mhat, b, (0.05,))


# --- BiCGstab -------------------------------------------------------------------------

def test_bicgstab_dense(tiny):
    dims, op, o, Mhat, b = tiny
    assert np.abs(Mhat - Mhat.conj().T).max() > 1e-3  # non-Hermitian at mu != 0
    for c in range(2):
        x, it = sv.bicgstab(op, b[c], 1e-13)
        assert it > 0
        assert rel(_odd_vec(x, o), np.linalg.solve(Mhat, _odd_vec(b[c], o))) < 1e-10


def test_bicgstab_planted_mistake(tiny):
    dims, op, o, Mhat, b = tiny

    class Adjoint:  # solving with Mhat^dag instead of Mhat
        Mhat = staticmethod(lambda v: op.Mhat(v, dagger=True))
    x, it = sv.bicgstab(Adjoint, b[0], 1e-13)
    assert rel(_odd_vec(x, o), np.linalg.solve(Mhat, _odd_vec(b[0], o))) > 1e-3


# --- block CG -------------------------------------------------------------------------

def test_block_cg_dense(tiny):
    dims, op, o, Mhat, b = tiny
    A = Mhat.conj().T @ Mhat
    X, it = sv.block_cg(op, b, 1e-13)
    assert it > 0
    for c in range(3):
        assert rel(_odd_vec(X[c], o), np.linalg.solve(A, _odd_vec(b[c], o))) < 1e-10
    # the block method needs fewer iterations than one CG per column
    its = [sv.shifted_cg(op, b[c], 0.0, 1e-13)[1] for c in range(3)]
    assert it < max(its)


def test_block_cg_one_column_is_cg(tiny):
    dims, op, o, Mhat, b = tiny
    X, it = sv.block_cg(op, b[:1], 1e-12)
    x, it2 = sv.shifted_cg(op, b[0], 0.0, 1e-12)
    assert it == it2
    assert rel(X[0], x) < 1e-12


def test_block_cg_planted_mistake(tiny, monkeypatch):
    dims, op, o, Mhat, b = tiny
    A = Mhat.conj().T @ Mhat
    real_solve = np.linalg.solve
    # beta from R'^dag R' alone (a dropped inverse of R^dag R): no longer A-conjugate directions
    calls = {"n": 0}

    def bad_solve(M, rhs):
        calls["n"] += 1
        return rhs if calls["n"] % 2 == 0 else real_solve(M, rhs)
    monkeypatch.setattr(sv.np.linalg, "solve", bad_solve)
    X, it = sv.block_cg(op, b, 1e-13, maxiter=60)
    monkeypatch.setattr(sv.np.linalg, "solve", real_solve)
    assert it == -1 or rel(_odd_vec(X[0], o), real_solve(A, _odd_vec(b[0], o))) > 1e-6


# --- block multishift CG ------------------------------------------------------------------

def _check_block_multishift(fn, op, o, Mhat, b, shifts):
    A = Mhat.conj().T @ Mhat
    Xs, it = fn(op, b, shifts, 1e-13)
    if it <= 0:
        return False
    for X, s in zip(Xs, shifts):
        for c in range(b.shape[0]):
            want = np.linalg.solve(A + s * np.eye(len(o)), _odd_vec(b[c], o))
            if rel(_odd_vec(X[c], o), want) > 1e-10:
                return False
    return True


@pytest.mark.parametrize("shifts", [(0.0, 0.05, 0.7), (0.02, 0.3, 1.5, 4.0)])
def test_block_multishift_dense(tiny, shifts):
    dims, op, o, Mhat, b = tiny
    assert _check_block_multishift(sv.block_multishift_cg, op, o, Mhat, b, shifts)


def test_block_multishift_reduces_to_block_cg_and_cg(tiny):
    dims, op, o, Mhat, b = tiny
    Xs, it = sv.block_multishift_cg(op, b, (0.0,), 1e-12)
    X, it2 = sv.block_cg(op, b, 1e-12)
    assert it == it2 and rel(Xs[0], X) < 1e-12
    # one column: the block recurrences are the scalar ones; the base (smallest shift) sets the count
    Xs, it = sv.block_multishift_cg(op, b[:1], (0.1, 0.5), 1e-12)
    x, it3 = sv.shifted_cg(op, b[0], 0.1, 1e-12)
    assert it == it3 and rel(Xs[0][0], x) < 1e-10


BMS_MUTATIONS = {
    "beta of a shift with xi_k for xi_k-1": ("b_s = a_prev_s[s] @ inv(xi_prev[s]) @ C @ xi[s]",
                                             "b_s = a_prev_s[s] @ inv(xi[s]) @ C @ xi[s]"),
    "xi update multiplied on the wrong side": ("xi[s] = inv(a) @ xi[s] @ a_s", "xi[s] = a_s @ xi[s] @ inv(a)"),
    "shift added to alpha instead of its inverse": ("a_s = inv(inv(a) + d * eye)", "a_s = a + d * eye"),
    "shifted direction from the new residual": ("R = R - comb(Q, a)\n", "R -= comb(Q, a)\n"),
}


@pytest.mark.parametrize("name", sorted(BMS_MUTATIONS))
def test_block_multishift_planted_mistakes(tiny, name):
    import inspect
    import textwrap
    dims, op, o, Mhat, b = tiny
    old, new = BMS_MUTATIONS[name]
    src = textwrap.dedent(inspect.getsource(sv.block_multishift_cg))
    assert src.count(old) == 1, old
    if name == "shifted direction from the new residual":
        # update R before the shifts read it (they need R_k, not R_k+1)
        src = src.replace("        R = R - comb(Q, a)\n", "", 1)
        src = src.replace("        a = np.linalg.solve(gram(P, Q), RR)\n",
                          "        a = np.linalg.solve(gram(P, Q), RR)\n        R_old = R\n        R = R - comb(Q, a)\n", 1)
    else:
        src = src.replace(old, new, 1)
    ns = dict(vars(sv))
    exec(compile(src, "<mutant>", "exec"), ns)
    mutant = ns["block_multishift_cg"]
    try:
        ok = _check_block_multishift(lambda *a: mutant(*a, maxiter=400), op, o, Mhat, b, (0.0, 0.05, 0.7))
    except np.linalg.LinAlgError:
        ok = False
    assert not ok, name


# --- trace terms ------------------------------------------------------------------------

@pytest.fixture(scope="module")
def trace_world():
    dims = (2, 2, 2, 2)
    U = inputs.gauge_field(dims, 0.3, seed=80)
    kappa, csw, mu = 0.12, 1.3, 0.1
    op = orc.Operator(dims, U, kappa, csw, mu=mu)
    M = orc.dense_matrix(op.M, op.V)
    return dims, U, kappa, csw, mu, op, M


def _dense_dM(dims, U, kappa, csw, mu, param, h=1e-5):
    """Central difference of the oracle's dense M in one parameter."""
    p = {"kappa": kappa, "csw": csw, "mu": mu}

    def Md(d):
        q = dict(p)
        q[param] += d
        o = orc.Operator(dims, U, q["kappa"], q["csw"], mu=q["mu"])
        return orc.dense_matrix(o.M, o.V)
    return (Md(h) - Md(-h)) / (2 * h)


@pytest.mark.parametrize("param", ["kappa", "csw", "mu"])
def test_dM_is_derivative_of_M(trace_world, param):
    dims, U, kappa, csw, mu, op, M = trace_world
    exact = orc.dense_matrix(lambda v: op.dM(v, param), op.V)
    fd = _dense_dM(dims, U, kappa, csw, mu, param)
    assert np.abs(exact - fd).max() < 1e-8 * np.abs(exact).max()
    # hence Tr(M^-1 dM/dp) = d ln det M / dp
    Minv = np.linalg.inv(M)
    tr = np.trace(Minv @ exact)
    h = 1e-5
    q = {"kappa": kappa, "csw": csw, "mu": mu}
    ld = []
    for d in (h, -h):
        qq = dict(q)
        qq[param] += d
        o = orc.Operator(dims, U, qq["kappa"], qq["csw"], mu=qq["mu"])
        sgn, logabs = np.linalg.slogdet(orc.dense_matrix(o.M, o.V))
        ld.append(np.log(sgn) + logabs)
    dlogdet = (ld[0] - ld[1]) / (2 * h)
    assert abs(tr - dlogdet) < 1e-6 * max(abs(tr), 1.0)


def test_dmu_planted_mistake(trace_world, monkeypatch):
    """A backward time hop differentiated with the wrong sign fails the derivative pin."""
    dims, U, kappa, csw, mu, op, M = trace_world
    fd = _dense_dM(dims, U, kappa, csw, mu, "mu")

    Us = U.copy()
    Us[3] = 0  # links of the time direction removed: the hopping term's spatial part only

    def wrong(psi):  # d/dmu of e^{-mu} taken as +e^{-mu}: both time hops with a positive factor
        return -kappa * (orc.hop(dims, U, psi, op.t_bc, mu) - orc.hop(dims, Us, psi, op.t_bc, mu))
    wrong_dense = orc.dense_matrix(wrong, op.V)
    assert np.abs(wrong_dense - fd).max() > 1e-3


def test_trace_terms_dense_and_free_field(trace_world):
    dims, U, kappa, csw, mu, op, M = trace_world
    Minv = np.linalg.inv(M)
    n = M.shape[0]
    g5 = np.kron(np.eye(op.V), np.kron(np.diag([1, 1, -1, -1]), np.eye(3)))
    dense = {
        "Minv": Minv, "Minv2": Minv @ Minv, "g5Minv": g5 @ Minv,
        "MdagMinv": np.linalg.inv(M @ M.conj().T),
        "dkappa": orc.dense_matrix(lambda v: op.dM(v, "kappa"), op.V) @ Minv,
        "dcsw": orc.dense_matrix(lambda v: op.dM(v, "csw"), op.V) @ Minv,
        "dmu": orc.dense_matrix(lambda v: op.dM(v, "mu"), op.V) @ Minv,
    }
    # per noise: the terms are eta^dag A eta with the dense A
    for k in range(2):
        eta = orc.z2_noise(dims, 5, k)
        terms = sv.trace_terms(op, eta, tol=1e-13)
        e = eta.reshape(-1)
        for name in sv.TRACE_TERMS:
            want = np.vdot(e, dense[name] @ e)
            assert abs(terms[name] - want) < 1e-9 * max(abs(want), 1.0), name
    # noise averages estimate the traces
    est = {k: [] for k in sv.TRACE_TERMS}
    for k in range(120):
        t = sv.trace_terms(op, orc.z2_noise(dims, 6, k), tol=1e-11)
        for name in sv.TRACE_TERMS:
            est[name].append(t[name])
    for name in sv.TRACE_TERMS:
        a = np.array(est[name])
        exact = np.trace(dense[name])
        for part in (np.real, np.imag):
            se = part(a).std(ddof=1) / np.sqrt(len(a))
            assert abs(part(a).mean() - part(exact)) <= 4 * se + 1e-9 * n, (name, part)
    # free field: tr(gamma_5 (a + i b.gamma)^-1) = 0 at every momentum
    free = orc.Operator(dims, inputs.unit_gauge(dims), kappa, csw, mu=mu)
    Mf = orc.dense_matrix(free.M, free.V)
    assert abs(np.trace(g5 @ np.linalg.inv(Mf))) < 1e-12
