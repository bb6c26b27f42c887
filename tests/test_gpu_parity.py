"""HIP path vs the CPU oracle, element by element, through the C ABI.

Tolerances (relative to the largest reference element):
  FP64 1e-12 (field agreement bar), FP32 1e-5, FP16 4e-3.
The FP16 bound follows from binary16 rounding (unit roundoff 2^-11 = 4.9e-4)
of links, clover entries and per-site-scaled spinors, accumulated over the
8 hops and the clover matvec with FP32 arithmetic.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1711_03836_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5, 2: 4e-3}
# 6x4x4x6: V/2 = 288 sites = 4.5 wavefronts (several tiles and a ragged tail); mu != 0, antiperiodic t
DIMS = (6, 4, 4, 6)
KAPPA, CSW, MU = 0.124, 1.5, 0.1


@pytest.fixture(scope="module")
def bq():
    from paper_1711_03836_amd import bqhip
    return bqhip


@pytest.fixture(scope="module")
def setup(bq):
    ctx = bq.Context(0)
    U = inputs.gauge_field(DIMS, 0.3, seed=101)
    G = bq.Gauge(ctx, DIMS, U, t_bc=-1)
    op = bq.Op(G, KAPPA, CSW, MU)
    ref = orc.Operator(DIMS, U, KAPPA, CSW, mu=MU, t_bc=-1)
    return ctx, G, op, ref, U


def maxrel(got, want):
    return np.abs(got - want).max() / np.abs(want).max()


def oracle_apply(ref, kind, bq, psi):
    """Reference for one column (V, 4, 3)."""
    K = bq
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


KINDS = ["BQ_OP_M", "BQ_OP_MDAG", "BQ_OP_MDAGM", "BQ_OP_MHAT", "BQ_OP_MHATDAG", "BQ_OP_MHATDAG_MHAT", "BQ_OP_DEO",
         "BQ_OP_DOE", "BQ_OP_DEO_DAG", "BQ_OP_DOE_DAG", "BQ_OP_K1", "BQ_OP_K1_DAG", "BQ_OP_CLOVER",
         "BQ_OP_CLOVER_INV"]


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("kind_name", KINDS)
def test_operator_parity(bq, setup, kind_name, prec):
    ctx, G, op, ref, U = setup
    kind = getattr(bq, kind_name)
    si, so = bq.OP_SUBSETS[kind]
    nrhs = 3
    psi = inputs.gaussian_spinor(DIMS, nrhs, seed=7 + prec)
    fi = bq.Field(ctx, DIMS, si, prec, nrhs)
    fo = bq.Field(ctx, DIMS, so, prec, nrhs)
    fi.put(psi)
    op.apply(kind, fi, fo)
    got = fo.get()
    mask = {bq.BQ_EVEN: ref.parity == 0, bq.BQ_ODD: ref.parity == 1, bq.BQ_FULL: np.ones(ref.V, bool)}[so]
    for c in range(nrhs):
        want = oracle_apply(ref, kind, bq, psi[c])
        err = maxrel(got[c][mask], want[mask])
        print(f"{kind_name} prec={prec} col={c} maxrel={err:.3e}", flush=True)
        assert err < TOL[prec], (kind_name, prec, c, err)
        # sites outside the output subset are not written
        assert np.all(got[c][~mask] == 0)


@pytest.mark.parametrize("prec,recon,R,bs", [(0, 12, 1, 64), (0, 18, 2, 128), (0, 12, 2, 512), (1, 12, 3, 256),
                                             (1, 18, 4, 64), (1, 12, 1, 512), (2, 12, 2, 128), (2, 12, 4, 256)])
def test_kernel_configurations(bq, setup, prec, recon, R, bs):
    """Every link form, column tile and workgroup shape gives the oracle's result (12 columns, K1 and Mhat)."""
    ctx, G, op, ref, U = setup
    nrhs = 12
    ctx.tune_set(prec, nrhs, recon, R, bs)
    psi = inputs.gaussian_spinor(DIMS, nrhs, seed=55)
    for kind in (bq.BQ_OP_K1, bq.BQ_OP_MHATDAG_MHAT):
        si, so = bq.OP_SUBSETS[kind]
        fi = bq.Field(ctx, DIMS, si, prec, nrhs)
        fo = bq.Field(ctx, DIMS, so, prec, nrhs)
        fi.put(psi)
        op.apply(kind, fi, fo)
        got = fo.get()
        mask = ref.parity == (0 if so == bq.BQ_EVEN else 1)
        for c in (0, 5, 11):
            want = oracle_apply(ref, kind, bq, psi[c])
            assert maxrel(got[c][mask], want[mask]) < TOL[prec]


def test_plaquette(bq, setup):
    ctx, G, op, ref, U = setup
    assert abs(G.plaquette() - orc.plaquette(DIMS, U)) < 1e-14


def test_field_roundtrip_and_untouched_sites(bq, setup):
    ctx = setup[0]
    psi = inputs.gaussian_spinor(DIMS, 2, seed=3)
    f = bq.Field(ctx, DIMS, bq.BQ_ODD, bq.BQ_F64, 2)
    f.put(psi)
    out = np.full_like(psi, 7.0)
    f.get(out)
    par = orc.site_parity(DIMS)
    assert np.array_equal(out[:, par == 1], psi[:, par == 1])
    assert np.all(out[:, par == 0] == 7.0)


def test_clover_not_hpd(bq, setup):
    ctx, G = setup[0], setup[1]
    with pytest.raises(bq.BqError) as e:
        bq.Op(G, 5.0, 10.0, 0.0)
    assert e.value.code == bq.BQ_ERR_CLOVER_NOT_HPD


def test_gauge_busy_and_invalid(bq, setup):
    ctx, G = setup[0], setup[1]
    with pytest.raises(bq.BqError) as e:
        G.close()
    assert e.value.code == bq.BQ_ERR_BUSY
    with pytest.raises(bq.BqError) as e:
        bq.Field(ctx, (4, 4, 3, 4), bq.BQ_FULL, 0, 1)
    assert e.value.code == bq.BQ_ERR_INVALID


# ---------------------------------------------------------------------------
# solves
# ---------------------------------------------------------------------------

def _solve(bq, op, dims, b, system, prec, tol, nrhs, use_graph=False, chunk=8):
    sub = bq.BQ_ODD if system == bq.BQ_SYS_NORMAL else bq.BQ_FULL
    fb = bq.Field(op.ctx, dims, sub, 0, nrhs)
    fx = bq.Field(op.ctx, dims, sub, 0, nrhs)
    fb.put(b)
    rc, info = op.solve(fb, fx, tol, system=system, inner_prec=prec, use_graph=use_graph, chunk=chunk)
    return fx.get(), info


def test_config0_full_normal_4444(bq):
    """4^4, unpreconditioned CG on M^dag M, kappa=0.12, c_SW=1.0, U=exp(0.3 i H), tol 1e-12."""
    dims = (4, 4, 4, 4)
    U = inputs.gauge_field(dims, 0.3, seed=2024)
    ctx = bq.Context(0)
    G = bq.Gauge(ctx, dims, U, -1)
    op = bq.Op(G, 0.12, 1.0, 0.0)
    ref = orc.Operator(dims, U, 0.12, 1.0)
    b = inputs.gaussian_spinor(dims, 1, seed=1)
    x, info = _solve(bq, op, dims, b, bq.BQ_SYS_FULL_NORMAL, 0, 1e-12, 1)
    r = b[0] - ref.M(ref.M(x[0]), dagger=True)
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(b[0]) * 1.01
    assert info[0]["converged"] and info[0]["true_rel_resid"] <= 1e-12
    xo, it = ref.cg(b[0], 0, 1e-12, 10000)
    assert abs(info[0]["iters"] - it) <= 2 + it // 50
    assert np.linalg.norm(x[0] - xo) / np.linalg.norm(xo) < 1e-9


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_eo_solve_sys_m(bq, setup, prec):
    """M x = b through the Schur system; oracle recomputes |b - M x|."""
    ctx, G, op, ref, U = setup
    b = inputs.gaussian_spinor(DIMS, 2, seed=31)
    x, info = _solve(bq, op, DIMS, b, bq.BQ_SYS_M, prec, 1e-10, 2)
    for c in range(2):
        assert info[c]["converged"], info[c]
        full = np.linalg.norm(b[c] - ref.M(x[c])) / np.linalg.norm(b[c])
        assert abs(full - info[c]["full_rel_resid"]) <= 1e-3 * full + 1e-14
        bh = ref.prepare(b[c])
        bp = ref.Mhat(bh, dagger=True)
        xo = ref.odd(x[c])
        tr = np.linalg.norm(bp - ref.Mhat(ref.Mhat(xo), dagger=True)) / np.linalg.norm(bp)
        assert tr <= 1e-10 * 1.05, tr
        if prec > 0:
            assert info[c]["reliable_updates"] >= 1


def test_normal_solve_and_graph(bq, setup):
    ctx, G, op, ref, U = setup
    b = inputs.gaussian_spinor(DIMS, 3, seed=41)
    par = orc.site_parity(DIMS)
    b[:, par == 0] = 0
    x1, i1 = _solve(bq, op, DIMS, b, bq.BQ_SYS_NORMAL, 1, 1e-10, 3, use_graph=False)
    x2, i2 = _solve(bq, op, DIMS, b, bq.BQ_SYS_NORMAL, 1, 1e-10, 3, use_graph=True)
    assert np.array_equal(x1, x2)  # graph replay = direct launches, bit for bit
    assert [a["iters"] for a in i1] == [a["iters"] for a in i2]
    for c in range(3):
        r = b[c] - ref.Mhat(ref.Mhat(x1[c]), dagger=True)
        assert np.linalg.norm(r[par == 1]) <= 1.05e-10 * np.linalg.norm(b[c])


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_batch_invariance(bq, setup, prec):
    """A column's solution is the same alone and inside a batch (bit for bit)."""
    ctx, G, op, ref, U = setup
    b = inputs.gaussian_spinor(DIMS, 4, seed=77)
    xa, ia = _solve(bq, op, DIMS, b[1:2], bq.BQ_SYS_M, prec, 1e-10, 1)
    xb, ib = _solve(bq, op, DIMS, b, bq.BQ_SYS_M, prec, 1e-10, 4)
    assert np.array_equal(xa[0], xb[1])
    assert ia[0]["iters"] == ib[1]["iters"]


def test_nonconverged_and_nonfinite(bq, setup):
    ctx, G, op, ref, U = setup
    b = inputs.gaussian_spinor(DIMS, 1, seed=5)
    fb = bq.Field(ctx, DIMS, bq.BQ_FULL, 0, 1)
    fx = bq.Field(ctx, DIMS, bq.BQ_FULL, 0, 1)
    fb.put(b)
    rc, info = op.solve(fb, fx, 1e-10, system=bq.BQ_SYS_M, maxiter=8, chunk=4, raise_on_error=False)
    assert rc == bq.BQ_ERR_NOT_CONVERGED and not info[0]["converged"] and info[0]["iters"] == 8
    b[0, 3, 1, 1] = np.nan
    fb.put(b)
    rc, info = op.solve(fb, fx, 1e-10, system=bq.BQ_SYS_M, raise_on_error=False)
    assert rc == bq.BQ_ERR_NONFINITE


def test_zero_source(bq, setup):
    ctx, G, op, ref, U = setup
    b = np.zeros((1, ref.V, 4, 3), complex)
    x, info = _solve(bq, op, DIMS, b, bq.BQ_SYS_M, 1, 1e-10, 1)
    assert np.all(x == 0) and info[0]["converged"]


def test_point_sources_mu(bq):
    """12 spin-colour point sources with mu = 0.1 in one batch (small lattice of the 32^3x64 workload's kind)."""
    dims = (4, 4, 4, 8)
    U = inputs.gauge_field(dims, 0.2, seed=9)
    ctx = bq.Context(0)
    G = bq.Gauge(ctx, dims, U, -1)
    op = bq.Op(G, 0.124, 1.5, 0.1)
    ref = orc.Operator(dims, U, 0.124, 1.5, mu=0.1)
    b = inputs.point_sources(dims)
    x, info = _solve(bq, op, dims, b, bq.BQ_SYS_M, 2, 1e-10, 12)
    for c in range(12):
        assert info[c]["converged"]
        assert np.linalg.norm(b[c] - ref.M(x[c])) / np.linalg.norm(b[c]) < 1e-7


def test_trace_per_noise(bq, setup):
    ctx, G, op, ref, U = setup
    t1, t2, info = op.trace(seed=2718, nnoise=5, block=2, tol=1e-10, inner_prec=bq.BQ_F32)
    for n in range(5):
        eta = orc.z2_noise(DIMS, 2718, n)
        x1, _ = ref.solve_M(eta, 1e-12)
        x2, _ = ref.solve_M(x1, 1e-12)
        w1 = np.vdot(eta.ravel(), x1.ravel())
        w2 = np.vdot(eta.ravel(), x2.ravel())
        assert abs(t1[n] - w1) < 1e-6 * abs(w1)
        assert abs(t2[n] - w2) < 1e-6 * abs(w2)


def test_hbm_budget(bq):
    ctx = bq.Context(0, hbm_budget=1 << 20)
    with pytest.raises(bq.BqError) as e:
        bq.Field(ctx, (8, 8, 8, 8), bq.BQ_FULL, 0, 4)
    assert e.value.code == bq.BQ_ERR_OOM


@pytest.mark.parametrize("dims", [(8, 16, 8, 8), (8, 32, 4, 6)])
@pytest.mark.parametrize("prec,recon,R,sb", [(0, 18, 2, 64), (1, 12, 3, 128), (2, 12, 4, 64), (1, 12, 1, 256)])
def test_blocked_traversal_lattices(bq, dims, prec, recon, R, sb):
    """Lattices whose (x,y) planes hold whole 64-site tiles are visited in (z,t) blocks; results unchanged."""
    U = inputs.gauge_field(dims, 0.3, seed=17)
    ctx = bq.Context(0)
    G = bq.Gauge(ctx, dims, U, -1)
    op = bq.Op(G, 0.124, 1.5, 0.1)
    ref = orc.Operator(dims, U, 0.124, 1.5, mu=0.1)
    nrhs = 12 if R > 1 else 1
    ctx.tune_set(prec, nrhs, recon, R, sb)
    psi = inputs.gaussian_spinor(dims, nrhs, seed=23)
    for kind in (bq.BQ_OP_K1, bq.BQ_OP_MHATDAG_MHAT, bq.BQ_OP_M):
        si, so = bq.OP_SUBSETS[kind]
        fi = bq.Field(ctx, dims, si, prec, nrhs)
        fo = bq.Field(ctx, dims, so, prec, nrhs)
        fi.put(psi)
        op.apply(kind, fi, fo)
        got = fo.get()
        mask = {bq.BQ_EVEN: ref.parity == 0, bq.BQ_ODD: ref.parity == 1, bq.BQ_FULL: np.ones(ref.V, bool)}[so]
        for c in sorted({0, nrhs // 2, nrhs - 1}):
            want = oracle_apply(ref, kind, bq, psi[c])
            assert maxrel(got[c][mask], want[mask]) < TOL[prec], (kind, c)
    b = inputs.gaussian_spinor(dims, 2, seed=29)
    x, info = _solve(bq, op, dims, b, bq.BQ_SYS_M, prec, 1e-10, 2)
    for c in range(2):
        assert info[c]["converged"]
        assert np.linalg.norm(b[c] - ref.M(x[c])) / np.linalg.norm(b[c]) < 1e-7


@pytest.mark.parametrize("prec,nrhs,recon,R,sb", [(1, 12, 12, 3, 64), (0, 1, 18, 1, 64), (2, 12, 12, 4, 128)])
def test_larger_lattice_k1(bq, prec, nrhs, recon, R, sb):
    """16^3x32 (blocked traversal, 1024 tiles per parity): K1 against the oracle on the whole lattice."""
    dims = (16, 16, 16, 32)
    U = inputs.gauge_field(dims, 0.2, seed=41)
    ctx = bq.Context(0)
    G = bq.Gauge(ctx, dims, U, -1)
    op = bq.Op(G, 0.125, 1.7, 0.0)
    ref = orc.Operator(dims, U, 0.125, 1.7)
    ctx.tune_set(prec, nrhs, recon, R, sb)
    psi = inputs.gaussian_spinor(dims, nrhs, seed=43)
    fi = bq.Field(ctx, dims, bq.BQ_ODD, prec, nrhs)
    fo = bq.Field(ctx, dims, bq.BQ_EVEN, prec, nrhs)
    fi.put(psi)
    op.apply(bq.BQ_OP_K1, fi, fo)
    got = fo.get()
    even = ref.parity == 0
    for c in sorted({0, nrhs - 1}):
        want = oracle_apply(ref, bq.BQ_OP_K1, bq, psi[c])
        assert maxrel(got[c][even], want[even]) < TOL[prec]


MARCH_KINDS = ("K1", "K1_DAG", "MHATDAG_MHAT", "M", "MDAG")


@pytest.mark.parametrize("dims,march", [((8, 16, 8, 8), 4), ((8, 16, 8, 8), 8), ((8, 32, 4, 6), 3),
                                        ((8, 32, 4, 6), 2)])
@pytest.mark.parametrize("prec,recon,R,bs", [(0, 18, 1, 256), (0, 12, 2, 128), (1, 12, 3, 256), (1, 18, 1, 512),
                                             (2, 12, 2, 128), (2, 12, 4, 64)])
def test_march_matches_plain_and_oracle(bq, dims, march, prec, recon, R, bs):
    """The t-marching stencil performs each site's arithmetic in the plain stencil's order, so every
    operator kind is bitwise the plain result; both match the oracle.  A solve with it converges to
    bitwise the plain solve's solution."""
    U = inputs.gauge_field(dims, 0.3, seed=19)
    ctx = bq.Context(0)
    G = bq.Gauge(ctx, dims, U, -1)
    op = bq.Op(G, 0.124, 1.5, 0.1)
    ref = orc.Operator(dims, U, 0.124, 1.5, mu=0.1)
    nrhs = 12 if R > 1 else 3
    psi = inputs.gaussian_spinor(dims, nrhs, seed=31)
    for name in MARCH_KINDS:
        kind = getattr(bq, "BQ_OP_" + name)
        si, so = bq.OP_SUBSETS[kind]
        out = {}
        for m in (0, march):
            ctx.tune_set(prec, nrhs, recon, R, bs, m)
            assert ctx.tune_get(prec, nrhs) == (recon, R, bs, m, 0, 0)
            fi = bq.Field(ctx, dims, si, prec, nrhs)
            fo = bq.Field(ctx, dims, so, prec, nrhs)
            fi.put(psi)
            op.apply(kind, fi, fo)
            out[m] = fo.get()
        assert np.array_equal(out[0], out[march]), name
        mask = {bq.BQ_EVEN: ref.parity == 0, bq.BQ_ODD: ref.parity == 1, bq.BQ_FULL: np.ones(ref.V, bool)}[so]
        for c in sorted({0, nrhs - 1}):
            want = oracle_apply(ref, kind, bq, psi[c])
            assert maxrel(out[march][c][mask], want[mask]) < TOL[prec], (name, c)
    b = inputs.gaussian_spinor(dims, 2, seed=37)
    xs = {}
    for m in (0, march):
        ctx.tune_set(prec, 2, recon, min(R, 2), bs, m)
        x, info = _solve(bq, op, dims, b, bq.BQ_SYS_M, prec, 1e-10, 2)
        assert all(c["converged"] for c in info)
        xs[m] = x
    assert np.array_equal(xs[0], xs[march])
    for c in range(2):
        assert np.linalg.norm(b[c] - ref.M(xs[march][c])) / np.linalg.norm(b[c]) < 1e-7


@pytest.mark.parametrize("prec,recon,R,bs,march", [(1, 12, 3, 256, 16), (1, 12, 1, 512, 8), (0, 18, 1, 256, 32),
                                                   (2, 12, 2, 128, 4)])
def test_march_larger_lattice_bitwise(bq, prec, recon, R, bs, march):
    """16^3x32 (16 tiles per (x,y) plane): t-marching K1, K2-type and residual-update kernels (through
    Mhat^dag Mhat and a solve) are bitwise the plain stencil's."""
    dims = (16, 16, 16, 32)
    U = inputs.gauge_field(dims, 0.2, seed=43)
    ctx = bq.Context(0)
    G = bq.Gauge(ctx, dims, U, -1)
    op = bq.Op(G, 0.125, 1.7, 0.05)
    nrhs = 12
    psi = inputs.gaussian_spinor(dims, nrhs, seed=47)
    for name in ("K1", "MHATDAG_MHAT"):
        kind = getattr(bq, "BQ_OP_" + name)
        si, so = bq.OP_SUBSETS[kind]
        out = {}
        for m in (0, march):
            ctx.tune_set(prec, nrhs, recon, R, bs, m)
            fi = bq.Field(ctx, dims, si, prec, nrhs)
            fo = bq.Field(ctx, dims, so, prec, nrhs)
            fi.put(psi)
            op.apply(kind, fi, fo)
            out[m] = fo.get()
        assert np.array_equal(out[0], out[march]), name
    xs = {}
    for m in (0, march):
        ctx.tune_set(prec, nrhs, recon, R, bs, m)
        x, info = _solve(bq, op, dims, psi, bq.BQ_SYS_M, prec, 1e-9, nrhs)
        assert all(c["converged"] for c in info)
        xs[m] = x
    assert np.array_equal(xs[0], xs[march])


def test_tuning_json_roundtrip(bq, setup, tmp_path):
    """Autotuned and hand-set stencil configurations survive save_tuning / load_tuning into a
    fresh context, and the operator's results do not depend on them."""
    ctx, G, op, ref, U = setup
    op.autotune(bq.BQ_F32, 4)
    ctx.tune_set(bq.BQ_F64, 1, 18, 1, 256, 0)
    path = tmp_path / "tune.json"
    ctx.save_tuning(path, [(bq.BQ_F32, 4), (bq.BQ_F64, 1)], lattice=DIMS)
    ctx2 = bq.Context(0)
    assert ctx2.load_tuning(path) == [(bq.BQ_F32, 4), (bq.BQ_F64, 1)]
    assert ctx2.tune_get(bq.BQ_F32, 4) == ctx.tune_get(bq.BQ_F32, 4)
    assert ctx2.tune_get(bq.BQ_F64, 1) == (18, 1, 256, 0, 0, 0)
    ctx2.close()


@pytest.mark.parametrize("dims", [(6, 4, 4, 6), (8, 16, 8, 8)])
@pytest.mark.parametrize("prec,recon,R,nrhs,lbs,mode", [
    (0, 18, 1, 12, 768, 1), (0, 12, 2, 5, 256, 1), (1, 12, 1, 12, 768, 1), (1, 18, 2, 12, 384, 1),
    (1, 12, 1, 17, 1024, 1), (1, 12, 1, 12, 256, 1), (2, 12, 1, 12, 768, 1), (2, 12, 2, 3, 64, 1),
    (0, 18, 1, 12, 768, 2), (1, 12, 1, 12, 768, 2), (1, 18, 1, 17, 1024, 2), (1, 12, 1, 5, 192, 2),
    (2, 12, 1, 12, 768, 2), (2, 12, 1, 3, 64, 2)])
def test_tile_shared_matches_plain_and_oracle(bq, dims, prec, recon, R, nrhs, lbs, mode):
    """The tile-shared stencil (links and clover staged in LDS once per tile, one column group per
    wave, at most lbs/64 waves per workgroup: 17 columns with 16 waves take two workgroups of 9 and
    8 waves per tile, 12 columns with 4 waves three workgroups) does each site's arithmetic in the
    plain stencil's order: every operator kind and a solve are bitwise the plain results, and both
    match the oracle.  Mode 2 takes the x and y neighbours from other lanes of the wave where they
    lie in the tile (all of them on 8x16x8x8, most on 6x4x4x6, whose last tile is ragged)."""
    U = inputs.gauge_field(dims, 0.3, seed=57)
    ctx = bq.Context(0)
    G = bq.Gauge(ctx, dims, U, -1)
    op = bq.Op(G, 0.124, 1.5, 0.1)
    ref = orc.Operator(dims, U, 0.124, 1.5, mu=0.1)
    psi = inputs.gaussian_spinor(dims, nrhs, seed=58)
    for name in MARCH_KINDS + ("MHAT", "DEO", "CLOVER_INV"):
        kind = getattr(bq, "BQ_OP_" + name)
        si, so = bq.OP_SUBSETS[kind]
        out = {}
        for lds in (0, 1):
            ctx.tune_set(prec, nrhs, recon, R, lbs if lds else 64, 0, mode if lds else 0)
            fi = bq.Field(ctx, dims, si, prec, nrhs)
            fo = bq.Field(ctx, dims, so, prec, nrhs)
            fi.put(psi)
            op.apply(kind, fi, fo)
            out[lds] = fo.get()
        assert np.array_equal(out[0], out[1]), name
        mask = {bq.BQ_EVEN: ref.parity == 0, bq.BQ_ODD: ref.parity == 1, bq.BQ_FULL: np.ones(ref.V, bool)}[so]
        for c in sorted({0, nrhs - 1}):
            want = oracle_apply(ref, kind, bq, psi[c])
            assert maxrel(out[1][c][mask], want[mask]) < TOL[prec], (name, c)
    b = inputs.gaussian_spinor(dims, nrhs, seed=59)
    xs = {}
    for lds in (0, 1):
        for p in {prec, 0}:
            ctx.tune_set(p, nrhs, recon if p == prec else 18, R if lds else min(R, 2), lbs if lds else 64, 0,
                         mode if lds else 0)
        x, info = _solve(bq, op, dims, b, bq.BQ_SYS_M, prec, 1e-10, nrhs)
        assert all(c["converged"] for c in info)
        xs[lds] = x
    assert np.array_equal(xs[0], xs[1])


@pytest.mark.parametrize("dims", [(8, 16, 8, 8), (8, 16, 6, 4)])
@pytest.mark.parametrize("prec,recon,R,bs,lds", [(0, 18, 2, 128, 0), (1, 12, 3, 256, 0), (1, 12, 1, 768, 1),
                                                  (1, 12, 1, 256, 1), (2, 12, 1, 384, 1), (0, 12, 1, 384, 1)])
def test_traversal_order_bitwise(bq, dims, prec, recon, R, bs, lds):
    """Traversal order 1 (one z slab per XCD, walked t plane by t plane; on 8x16x6x4 slabs of 3 z
    planes) and order 2 (the same with each XCD walking its tiles once per column-group chunk) visit
    the same work items as order 0 and do each site's arithmetic in the same order: every operator
    kind is bitwise the order-0 result and matches the oracle."""
    nrhs = 12
    U = inputs.gauge_field(dims, 0.3, seed=61)
    ctx = bq.Context(0)
    G = bq.Gauge(ctx, dims, U, -1)
    op = bq.Op(G, 0.124, 1.5, 0.1)
    ref = orc.Operator(dims, U, 0.124, 1.5, mu=0.1)
    psi = inputs.gaussian_spinor(dims, nrhs, seed=62)
    for name in MARCH_KINDS + ("MHAT", "DEO"):
        kind = getattr(bq, "BQ_OP_" + name)
        si, so = bq.OP_SUBSETS[kind]
        out = {}
        for order in (0, 1, 2):
            ctx.tune_set(prec, nrhs, recon, R, bs, 0, lds, order)
            assert ctx.tune_get(prec, nrhs)[5] == order
            fi = bq.Field(ctx, dims, si, prec, nrhs)
            fo = bq.Field(ctx, dims, so, prec, nrhs)
            fi.put(psi)
            op.apply(kind, fi, fo)
            out[order] = fo.get()
        assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2]), name
        mask = {bq.BQ_EVEN: ref.parity == 0, bq.BQ_ODD: ref.parity == 1, bq.BQ_FULL: np.ones(ref.V, bool)}[so]
        for c in (0, nrhs - 1):
            want = oracle_apply(ref, kind, bq, psi[c])
            assert maxrel(out[2][c][mask], want[mask]) < TOL[prec], (name, c)


def test_time_copy(bq, setup):
    """The plain device copy that serves as the bandwidth reference runs, moves data at a rate
    between 1 and 8 TB/s (read + write) on one MI355X, and refuses sizes that are not whole 16-byte
    words."""
    ctx = setup[0]
    nbytes = 256 << 20
    ms = ctx.time_copy(nbytes, reps=5)
    gbs = 2 * nbytes / ms / 1e6
    assert 1000 < gbs < 8000, gbs
    with pytest.raises(bq.BqError):
        ctx.time_copy(15)
