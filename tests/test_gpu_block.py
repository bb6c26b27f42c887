"""Block CG and block multishift CG (the solver list's "block multishift cg", section "Algorithms")
on the GPU, through the C ABI, against the oracle (oracle/solvers.py):

  - block CG takes the oracle's block-CG iteration count (to one iteration: the stopping test
    compares rounded sums) and fewer iterations than CG per column; its solutions agree with the
    oracle's CG solutions to cond * tol;
  - block CG on the M and Mhat systems and block multishift CG on 2^4 against numpy's dense solve
    of the oracle's matrices;
  - one column is CG (same iteration count);
  - a repeated column is numerically dependent: it waits for a second run and is solved there; a
    zero column gets x = 0;
  - block multishift CG: every shift's solution against the oracle's CG on (A + sigma) x = b, the
    iteration count of the oracle's block multishift CG, the FP64 residuals the oracle recomputes;
  - unsupported combinations are refused.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from oracle import solvers as sv
from paper_1711_03836_amd import inputs

pytestmark = pytest.mark.gpu

DIMS = (6, 4, 4, 6)
KAPPA, CSW, MU = 0.124, 1.5, 0.1


@pytest.fixture(scope="module")
def bq():
    from paper_1711_03836_amd import bqhip
    return bqhip


@pytest.fixture(scope="module")
def world(bq):
    ctx = bq.Context(0)
    U = inputs.gauge_field(DIMS, 0.3, seed=501)
    G = bq.Gauge(ctx, DIMS, U, t_bc=-1)
    op = bq.Op(G, KAPPA, CSW, MU)
    ref = orc.Operator(DIMS, U, KAPPA, CSW, mu=MU, t_bc=-1)
    return ctx, G, op, ref, U


def _odd_sources(ref, n, seed):
    return np.stack([ref.odd(v) for v in inputs.gaussian_spinor(ref.dims, n, seed=seed)])


def _solve(bq, ctx, dims, op, b, tol, system, solver, subset, **kw):
    fb = bq.Field(ctx, dims, subset, bq.BQ_F64, b.shape[0])
    fx = bq.Field(ctx, dims, subset, bq.BQ_F64, b.shape[0])
    fb.put(b)
    rc, info = op.solve(fb, fx, tol, system=system, inner_prec=bq.BQ_F64, solver=solver, **kw)
    return rc, info, fx.get()


def test_block_cg_against_oracle(bq, world):
    ctx, G, op, ref, U = world
    b = _odd_sources(ref, 4, 511)
    tol = 1e-11
    rc, info, x = _solve(bq, ctx, DIMS, op, b, tol, bq.BQ_SYS_NORMAL, bq.BQ_SOLVER_BLOCK_CG, bq.BQ_ODD)
    assert rc == bq.BQ_OK
    Xo, it_o = sv.block_cg(ref, b, tol)
    A = sv.normal_op(ref)
    rc2, info_cg, _ = _solve(bq, ctx, DIMS, op, b, tol, bq.BQ_SYS_NORMAL, bq.BQ_SOLVER_CG, bq.BQ_ODD)
    its = [i["iters"] for i in info]
    print(f"block CG iterations {its} (oracle block CG {it_o}); CG {[i['iters'] for i in info_cg]}", flush=True)
    assert max(abs(i - it_o) for i in its) <= 1
    assert max(its) < max(i["iters"] for i in info_cg)
    for c in range(4):
        want, _ = sv.shifted_cg(ref, b[c], 0.0, 1e-13)
        err = np.linalg.norm(x[c] - want) / np.linalg.norm(want)
        res = np.linalg.norm(b[c] - A(x[c])) / np.linalg.norm(b[c])
        print(f"col {c}: rel diff {err:.2e}, oracle residual {res:.2e}, reported {info[c]['true_rel_resid']:.2e}",
              flush=True)
        assert info[c]["converged"] and info[c]["reliable_updates"] == 0
        assert res < 1.5 * tol and abs(res - info[c]["true_rel_resid"]) <= 0.01 * res + 1e-16
        assert err < 1e-8
        assert np.all(x[c][ref.parity == 0] == 0)
        # the block solution equals the oracle's block CG iterate to the same accuracy
        assert np.linalg.norm(x[c] - Xo[c]) / np.linalg.norm(Xo[c]) < 1e-8


@pytest.mark.parametrize("system", ["BQ_SYS_M", "BQ_SYS_MHAT"])
def test_block_cg_dense_2222(bq, system):
    dims = (2, 2, 2, 2)
    U = inputs.gauge_field(dims, 0.3, seed=512)
    ctx = bq.Context(0)
    G = bq.Gauge(ctx, dims, U, t_bc=+1)
    op = bq.Op(G, 0.12, 1.0, -0.1)
    ref = orc.Operator(dims, U, 0.12, 1.0, mu=-0.1, t_bc=+1)
    sys_ = getattr(bq, system)
    if sys_ == bq.BQ_SYS_M:
        b = inputs.gaussian_spinor(dims, 3, seed=513)
        Md = orc.dense_matrix(ref.M, ref.V)
        rc, info, x = _solve(bq, ctx, dims, op, b, 1e-13, sys_, bq.BQ_SOLVER_BLOCK_CG, bq.BQ_FULL)
        for c in range(3):
            want = np.linalg.solve(Md, b[c].reshape(-1))
            assert np.linalg.norm(x[c].reshape(-1) - want) / np.linalg.norm(want) < 1e-10
            assert info[c]["full_rel_resid"] < 1e-11
    else:
        o = np.where(np.repeat(ref.parity, 12) == 1)[0]
        Mh = orc.dense_matrix(ref.Mhat, ref.V)[np.ix_(o, o)]
        b = _odd_sources(ref, 3, 514)
        rc, info, x = _solve(bq, ctx, dims, op, b, 1e-13, sys_, bq.BQ_SOLVER_BLOCK_CG, bq.BQ_ODD)
        for c in range(3):
            want = np.linalg.solve(Mh, b[c].reshape(-1)[o])
            assert np.linalg.norm(x[c].reshape(-1)[o] - want) / np.linalg.norm(want) < 1e-10
    assert rc == bq.BQ_OK


def test_block_cg_one_column_is_cg(bq, world):
    ctx, G, op, ref, U = world
    b = _odd_sources(ref, 1, 515)
    rc, info, x = _solve(bq, ctx, DIMS, op, b, 1e-10, bq.BQ_SYS_NORMAL, bq.BQ_SOLVER_BLOCK_CG, bq.BQ_ODD)
    rc2, info2, x2 = _solve(bq, ctx, DIMS, op, b, 1e-10, bq.BQ_SYS_NORMAL, bq.BQ_SOLVER_CG, bq.BQ_ODD)
    assert rc == rc2 == bq.BQ_OK
    assert abs(info[0]["iters"] - info2[0]["iters"]) <= 1
    assert np.linalg.norm(x[0] - x2[0]) / np.linalg.norm(x2[0]) < 1e-8


def test_block_cg_dependent_and_zero_columns(bq, world):
    ctx, G, op, ref, U = world
    b0 = _odd_sources(ref, 2, 516)
    b = np.stack([b0[0], b0[0], np.zeros_like(b0[0]), b0[1]])
    rc, info, x = _solve(bq, ctx, DIMS, op, b, 1e-10, bq.BQ_SYS_NORMAL, bq.BQ_SOLVER_BLOCK_CG, bq.BQ_ODD)
    print([(i["iters"], i["reliable_updates"], i["true_rel_resid"]) for i in info], flush=True)
    assert rc == bq.BQ_OK and all(i["converged"] for i in info)
    assert info[1]["reliable_updates"] >= 1  # the repeated column is solved in a later run
    assert np.linalg.norm(x[1] - x[0]) / np.linalg.norm(x[0]) < 1e-8
    assert np.all(x[2] == 0) and info[2]["true_rel_resid"] == 0


def test_block_multishift_against_oracle(bq, world):
    ctx, G, op, ref, U = world
    shifts = [0.5, 0.0, 0.02, 3.0]  # the smallest shift carries the block Krylov space
    b = _odd_sources(ref, 3, 517)
    tol = 1e-11
    fb = bq.Field(ctx, DIMS, bq.BQ_ODD, bq.BQ_F64, 3)
    fb.put(b)
    xs = [bq.Field(ctx, DIMS, bq.BQ_ODD, bq.BQ_F64, 3) for _ in shifts]
    rc, info = op.solve_multishift(fb, xs, shifts, tol, solver=bq.BQ_SOLVER_BLOCK_CG)
    assert rc == bq.BQ_OK
    xs = [f.get() for f in xs]
    _, it_o = sv.block_multishift_cg(ref, b, shifts, tol)
    it_gpu = max(i["iters"] for row in info for i in row)
    _, info_ms = op.solve_multishift(fb, [bq.Field(ctx, DIMS, bq.BQ_ODD, bq.BQ_F64, 3) for _ in shifts], shifts, tol)
    print(f"block multishift iterations {it_gpu} (oracle {it_o}); multishift CG "
          f"{max(i['iters'] for row in info_ms for i in row)}", flush=True)
    assert abs(it_gpu - it_o) <= 1
    assert it_gpu < max(i["iters"] for row in info_ms for i in row)
    A = sv.normal_op(ref)
    for k, s in enumerate(shifts):
        for c in range(3):
            want, _ = sv.shifted_cg(ref, b[c], s, 1e-13)
            got = xs[k][c]
            err = np.linalg.norm(got - want) / np.linalg.norm(want)
            res = np.linalg.norm(b[c] - A(got) - s * got) / np.linalg.norm(b[c])
            print(f"shift {s}: col {c} iters {info[k][c]['iters']}, rel diff {err:.2e}, residual {res:.2e}, "
                  f"reported {info[k][c]['true_rel_resid']:.2e}", flush=True)
            assert info[k][c]["converged"]
            assert res < 1e-10 and abs(res - info[k][c]["true_rel_resid"]) <= 0.01 * res + 1e-16
            assert err < 1e-8
        if s > 0.0:  # shifted systems are better conditioned and stop earlier
            assert max(i["iters"] for i in info[k]) <= max(i["iters"] for i in info[1])


def test_block_multishift_dense_2222(bq):
    dims = (2, 2, 2, 2)
    U = inputs.gauge_field(dims, 0.3, seed=518)
    ctx = bq.Context(0)
    G = bq.Gauge(ctx, dims, U, t_bc=-1)
    op = bq.Op(G, 0.12, 1.2, 0.1)
    ref = orc.Operator(dims, U, 0.12, 1.2, mu=0.1, t_bc=-1)
    o = np.where(np.repeat(ref.parity, 12) == 1)[0]
    Mh = orc.dense_matrix(ref.Mhat, ref.V)[np.ix_(o, o)]
    A = Mh.conj().T @ Mh
    b = _odd_sources(ref, 4, 519)
    shifts = [0.01, 0.1, 1.0]
    fb = bq.Field(ctx, dims, bq.BQ_ODD, bq.BQ_F64, 4)
    fb.put(b)
    xs = [bq.Field(ctx, dims, bq.BQ_ODD, bq.BQ_F64, 4) for _ in shifts]
    rc, info = op.solve_multishift(fb, xs, shifts, 1e-13, solver=bq.BQ_SOLVER_BLOCK_CG)
    assert rc == bq.BQ_OK
    for k, s in enumerate(shifts):
        xk = xs[k].get()
        for c in range(4):
            want = np.linalg.solve(A + s * np.eye(len(o)), b[c].reshape(-1)[o])
            assert np.linalg.norm(xk[c].reshape(-1)[o] - want) / np.linalg.norm(want) < 1e-10


def test_block_unsupported(bq, world):
    ctx, G, op, ref, U = world
    b = _odd_sources(ref, 2, 520)
    fb = bq.Field(ctx, DIMS, bq.BQ_ODD, bq.BQ_F64, 2)
    fx = bq.Field(ctx, DIMS, bq.BQ_ODD, bq.BQ_F64, 2)
    fb.put(b)
    with pytest.raises(bq.BqError) as e:
        op.solve(fb, fx, 1e-10, inner_prec=bq.BQ_F32, solver=bq.BQ_SOLVER_BLOCK_CG)
    assert e.value.code == bq.BQ_ERR_UNSUPPORTED
    big = bq.Field(ctx, DIMS, bq.BQ_ODD, bq.BQ_F64, 17)
    bigx = bq.Field(ctx, DIMS, bq.BQ_ODD, bq.BQ_F64, 17)
    with pytest.raises(bq.BqError) as e:
        op.solve(big, bigx, 1e-10, inner_prec=bq.BQ_F64, solver=bq.BQ_SOLVER_BLOCK_CG)
    assert e.value.code == bq.BQ_ERR_UNSUPPORTED
    ff = bq.Field(ctx, DIMS, bq.BQ_FULL, bq.BQ_F64, 2)
    ffx = bq.Field(ctx, DIMS, bq.BQ_FULL, bq.BQ_F64, 2)
    with pytest.raises(bq.BqError) as e:
        op.solve(ff, ffx, 1e-10, system=bq.BQ_SYS_FULL_NORMAL, inner_prec=bq.BQ_F64, solver=bq.BQ_SOLVER_BLOCK_CG)
    assert e.value.code == bq.BQ_ERR_UNSUPPORTED
    # maxiter reached: not converged, x holds the last iterate
    rc, info, _ = _solve(bq, ctx, DIMS, op, b, 1e-12, bq.BQ_SYS_NORMAL, bq.BQ_SOLVER_BLOCK_CG, bq.BQ_ODD,
                         maxiter=8, raise_on_error=False)
    assert rc == bq.BQ_ERR_NOT_CONVERGED and not info[0]["converged"]
