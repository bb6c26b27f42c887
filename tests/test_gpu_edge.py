"""The method's edge cases on the GPU, through the C ABI, against the CPU oracle.

Every operator kind in FP64, FP32 and FP16 (same bars as test_gpu_parity: 1e-12, 1e-5, 4e-3
relative to the largest reference element) for the settings Eq. 1 and Eq. 2 allow beyond the
default workload:
  - periodic time boundary (t_bc = +1);
  - lattices with an extent of 2, where the forward and backward neighbours of a site coincide
    (x + mu = x - mu) and the stencil must add both hops: 2^4, 2x4x2x4, 4x2x4x2;
  - kappa = 0, where M, M^dag, Mhat and the clover are the identity (bitwise in FP64 and FP32);
  - c_SW = 0 (plain Wilson hopping term, T = 1);
  - a negative chemical potential mu = -0.2.
Also on 2^4: FP64 solves of M x = b and M^dag M x = b against numpy's dense solve of the oracle's
matrix, links that are not SU(3) (the two-row form must not be used), and a caller's device
allocator routed through bq_context_create.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1711_03836_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5, 2: 4e-3}
KINDS = ["BQ_OP_M", "BQ_OP_MDAG", "BQ_OP_MDAGM", "BQ_OP_MHAT", "BQ_OP_MHATDAG", "BQ_OP_MHATDAG_MHAT", "BQ_OP_DEO",
         "BQ_OP_DOE", "BQ_OP_DEO_DAG", "BQ_OP_DOE_DAG", "BQ_OP_K1", "BQ_OP_K1_DAG", "BQ_OP_CLOVER",
         "BQ_OP_CLOVER_INV"]
# (name, dims, kappa, c_SW, mu, t_bc, link roughness)
CASES = [
    ("periodic_t", (6, 4, 4, 6), 0.124, 1.5, 0.1, +1, 0.3),
    ("extent2_2222", (2, 2, 2, 2), 0.12, 1.0, 0.1, -1, 0.3),
    ("extent2_2424", (2, 4, 2, 4), 0.12, 1.2, 0.1, -1, 0.3),
    ("extent2_4242", (4, 2, 4, 2), 0.12, 1.2, -0.1, +1, 0.3),
    ("kappa0", (6, 4, 4, 6), 0.0, 1.5, 0.1, -1, 0.3),
    ("csw0", (6, 4, 4, 6), 0.124, 0.0, 0.1, -1, 0.3),
    ("mu_negative", (6, 4, 4, 6), 0.124, 1.5, -0.2, -1, 0.3),
]
IDENTITY_KINDS = ("BQ_OP_M", "BQ_OP_MDAG", "BQ_OP_MDAGM", "BQ_OP_MHAT", "BQ_OP_MHATDAG", "BQ_OP_MHATDAG_MHAT",
                  "BQ_OP_CLOVER", "BQ_OP_CLOVER_INV")


@pytest.fixture(scope="module")
def bq():
    from paper_1711_03836_amd import bqhip
    return bqhip


@pytest.fixture(scope="module")
def ctx(bq):
    return bq.Context(0)


def maxrel(got, want):
    return np.abs(got - want).max() / np.abs(want).max()


def oracle_apply(ref, K, kind, psi):
    if kind == K.BQ_OP_M:
        return ref.M(psi)
    if kind == K.BQ_OP_MDAG:
        return ref.M(psi, dagger=True)
    if kind == K.BQ_OP_MDAGM:
        return ref.M(ref.M(psi), dagger=True)
    if kind == K.BQ_OP_MHAT:
        return ref.Mhat(ref.odd(psi))
    if kind == K.BQ_OP_MHATDAG:
        return ref.Mhat(ref.odd(psi), dagger=True)
    if kind == K.BQ_OP_MHATDAG_MHAT:
        return ref.Mhat(ref.Mhat(ref.odd(psi)), dagger=True)
    if kind in (K.BQ_OP_DEO, K.BQ_OP_DEO_DAG):
        return ref.even(ref.hop(ref.odd(psi), dagger=kind == K.BQ_OP_DEO_DAG))
    if kind in (K.BQ_OP_DOE, K.BQ_OP_DOE_DAG):
        return ref.odd(ref.hop(ref.even(psi), dagger=kind == K.BQ_OP_DOE_DAG))
    if kind in (K.BQ_OP_K1, K.BQ_OP_K1_DAG):
        h = ref.even(ref.hop(ref.odd(psi), dagger=kind == K.BQ_OP_K1_DAG))
        return orc.clover_apply(ref.dims, ref.Tinv, h, parity_mask=1)
    if kind == K.BQ_OP_CLOVER:
        return orc.clover_apply(ref.dims, ref.T, psi)
    if kind == K.BQ_OP_CLOVER_INV:
        return orc.clover_apply(ref.dims, ref.Tinv, ref.even(psi), parity_mask=1)
    raise ValueError(kind)


@pytest.fixture(scope="module")
def worlds(bq, ctx):
    cache = {}

    def get(name):
        if name not in cache:
            _, dims, kappa, csw, mu, tbc, eps = next(c for c in CASES if c[0] == name)
            U = inputs.gauge_field(dims, eps, seed=900 + len(cache))
            G = bq.Gauge(ctx, dims, U, t_bc=tbc)
            op = bq.Op(G, kappa, csw, mu)
            ref = orc.Operator(dims, U, kappa, csw, mu=mu, t_bc=tbc)
            cache[name] = (dims, G, op, ref, U)
        return cache[name]
    return get


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("case", [c[0] for c in CASES])
def test_edge_operator_parity(bq, ctx, worlds, case, prec):
    dims, G, op, ref, U = worlds(case)
    nrhs = 2
    psi = inputs.gaussian_spinor(dims, nrhs, seed=17 + prec)
    for kind_name in KINDS:
        kind = getattr(bq, kind_name)
        si, so = bq.OP_SUBSETS[kind]
        fi = bq.Field(ctx, dims, si, prec, nrhs)
        fo = bq.Field(ctx, dims, so, prec, nrhs)
        fi.put(psi)
        op.apply(kind, fi, fo)
        got = fo.get()
        mask = {bq.BQ_EVEN: ref.parity == 0, bq.BQ_ODD: ref.parity == 1, bq.BQ_FULL: np.ones(ref.V, bool)}[so]
        for c in range(nrhs):
            want = oracle_apply(ref, bq, kind, psi[c])
            err = maxrel(got[c][mask], want[mask])
            print(f"{case} {kind_name} prec={prec} col={c} maxrel={err:.3e}", flush=True)
            assert err < TOL[prec], (case, kind_name, prec, c, err)
            assert np.all(got[c][~mask] == 0)
            if case == "kappa0" and kind_name in IDENTITY_KINDS and prec < 2:
                # kappa = 0: T = 1 exactly and the hopping term is scaled by zero; in FP32 the input
                # is first rounded to FP32, and the identity returns exactly those values
                sub = psi[c][mask] if prec == 0 else psi[c][mask].astype(np.complex64).astype(np.complex128)
                assert np.array_equal(got[c][mask], sub), (kind_name, prec)


def _dense_solve_check(bq, ctx, dims, kappa, csw, mu, tbc, seed):
    U = inputs.gauge_field(dims, 0.3, seed=seed)
    G = bq.Gauge(ctx, dims, U, t_bc=tbc)
    op = bq.Op(G, kappa, csw, mu)
    ref = orc.Operator(dims, U, kappa, csw, mu=mu, t_bc=tbc)
    V = ref.V
    Md = orc.dense_matrix(ref.M, V)
    b = inputs.gaussian_spinor(dims, 2, seed=seed + 1)
    for system in (bq.BQ_SYS_M, bq.BQ_SYS_FULL_NORMAL):
        fb = bq.Field(ctx, dims, bq.BQ_FULL, bq.BQ_F64, 2)
        fx = bq.Field(ctx, dims, bq.BQ_FULL, bq.BQ_F64, 2)
        fb.put(b)
        rc, info = op.solve(fb, fx, 1e-13, system=system, inner_prec=bq.BQ_F64)
        x = fx.get()
        A = Md if system == bq.BQ_SYS_M else Md.conj().T @ Md
        for c in range(2):
            want = np.linalg.solve(A, b[c].reshape(-1)).reshape(V, 4, 3)
            err = np.linalg.norm(x[c] - want) / np.linalg.norm(want)
            print(f"dense {dims} system={system} col={c}: rel err {err:.2e}, iters {info[c]['iters']}", flush=True)
            assert info[c]["converged"]
            assert err < 1e-10, (system, c, err)


@pytest.mark.parametrize("tbc,mu", [(-1, 0.1), (+1, -0.2)])
def test_dense_2222_solve(bq, ctx, tbc, mu):
    """2^4 (192 x 192 complex): the GPU FP64 CG solution equals numpy's dense solve of the oracle's M."""
    _dense_solve_check(bq, ctx, (2, 2, 2, 2), 0.12, 1.0, mu, tbc, seed=2222)


def test_non_su3_links(bq, ctx):
    """Links scaled off SU(3): the two-row link form must not be used.  FP64 and FP32 stencils (asked for
    12-real links) still match the oracle with the links as given; FP16 storage and the server, which
    need the two-row form, report BQ_ERR_UNSUPPORTED."""
    dims = (6, 4, 4, 6)
    U = inputs.gauge_field(dims, 0.3, seed=31) * 1.02
    U[1, 5] += 0.01  # one link off U(3) as well
    G = bq.Gauge(ctx, dims, U, t_bc=-1)
    assert G.su3_deviation() > 0.04
    Gok = bq.Gauge(ctx, dims, inputs.gauge_field(dims, 0.3, seed=31), t_bc=-1)
    assert Gok.su3_deviation() < 1e-13
    op = bq.Op(G, 0.124, 1.3, 0.1)
    ref = orc.Operator(dims, U, 0.124, 1.3, mu=0.1)
    psi = inputs.gaussian_spinor(dims, 3, seed=5)
    for prec in (0, 1):
        ctx.tune_set(prec, 3, 12, 1, 64)
        for kind in (bq.BQ_OP_K1, bq.BQ_OP_M, bq.BQ_OP_MHATDAG_MHAT):
            si, so = bq.OP_SUBSETS[kind]
            fi = bq.Field(ctx, dims, si, prec, 3)
            fo = bq.Field(ctx, dims, so, prec, 3)
            fi.put(psi)
            op.apply(kind, fi, fo)
            got = fo.get()
            mask = {bq.BQ_EVEN: ref.parity == 0, bq.BQ_ODD: ref.parity == 1, bq.BQ_FULL: np.ones(ref.V, bool)}[so]
            for c in range(3):
                want = oracle_apply(ref, bq, kind, psi[c])
                assert maxrel(got[c][mask], want[mask]) < TOL[prec], (prec, kind, c)
    fi = bq.Field(ctx, dims, bq.BQ_ODD, bq.BQ_F16, 1)
    fo = bq.Field(ctx, dims, bq.BQ_EVEN, bq.BQ_F16, 1)
    fi.put(psi[:1])
    with pytest.raises(bq.BqError) as e:
        op.apply(bq.BQ_OP_K1, fi, fo)
    assert e.value.code == bq.BQ_ERR_UNSUPPORTED
    srv = bq.Server(ctx, 4, 8)
    with pytest.raises(bq.BqError) as e:
        srv.submit(G, psi[:1], 0.12, 1.5)
    assert e.value.code == bq.BQ_ERR_UNSUPPORTED
    srv.close()
    op.close()
    G.close()


def test_caller_allocator(bq):
    """Every device allocation of a context goes through the caller's allocator (here torch's caching
    allocator, counted); results are bitwise those of a context on hipMalloc, and every block is given
    back when the handles are freed."""
    import torch
    live = {}
    count = {"alloc": 0, "free": 0}

    def alloc(n):
        p = torch.cuda.caching_allocator_alloc(n, 0)
        live[p] = n
        count["alloc"] += 1
        return p

    def dealloc(p):
        assert p in live
        del live[p]
        count["free"] += 1
        torch.cuda.caching_allocator_delete(p)

    dims = (4, 4, 4, 8)
    U = inputs.gauge_field(dims, 0.2, seed=77)
    b = inputs.gaussian_spinor(dims, 2, seed=78)
    results = []
    for use in (False, True):
        ctx = bq.Context(0, alloc=alloc, dealloc=dealloc) if use else bq.Context(0)
        G = bq.Gauge(ctx, dims, U, -1)
        op = bq.Op(G, 0.124, 1.5, 0.1)
        fb = bq.Field(ctx, dims, bq.BQ_FULL, bq.BQ_F64, 2)
        fx = bq.Field(ctx, dims, bq.BQ_FULL, bq.BQ_F64, 2)
        fb.put(b)
        op.solve(fb, fx, 1e-10, system=bq.BQ_SYS_M, inner_prec=bq.BQ_F32)
        results.append(fx.get())
        if use:
            assert count["alloc"] > 0 and len(live) > 0
            assert sum(live.values()) == ctx.hbm_used()
        for h in (fx, fb, op, G):
            h.close()
        if use:
            assert not live and count["alloc"] == count["free"], count
        ctx.close()
    assert np.array_equal(results[0], results[1])
