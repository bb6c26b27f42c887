"""Continuous-batching server: results against the oracle, and each request's result is the
same alone and in the mix (bit for bit: a column's arithmetic does not depend on the other
columns and it enters the batch at a chunk boundary)."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1711_03836_amd import inputs

pytestmark = pytest.mark.gpu

DIMS_A = (4, 4, 4, 8)
DIMS_B = (8, 4, 4, 4)


@pytest.fixture(scope="module")
def world():
    from paper_1711_03836_amd import bqhip as bq
    ctx = bq.Context(0)
    UA = inputs.gauge_field(DIMS_A, 0.2, seed=61)
    UB = inputs.gauge_field(DIMS_B, 0.2, seed=62)
    return bq, ctx, {DIMS_A: (bq.Gauge(ctx, DIMS_A, UA), UA), DIMS_B: (bq.Gauge(ctx, DIMS_B, UB), UB)}


def serve(bq, ctx, reqs, slots=8, chunk=8, stagger=False):
    """reqs: list of (dims, gauge, b, kappa, prec). Returns {index: (rc, info, x)}."""
    srv = bq.Server(ctx, slots, chunk)
    tickets, out = {}, {}
    order = list(range(len(reqs)))
    pending = list(order)
    while len(out) < len(reqs):
        # staggered arrival: one new request per step
        for _ in range(1 if stagger else len(pending)):
            if pending:
                i = pending.pop(0)
                d, G, b, k, prec = reqs[i]
                tickets[srv.submit(G, b, k, 1.5, 0.0, 1e-10, prec)] = i
        for t in srv.step():
            out[tickets[t]] = srv.result(t)
    srv.close()
    return out


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_server_alone_vs_mix(world, prec):
    bq, ctx, G = world
    rng = np.random.default_rng(5)
    reqs = []
    for i in range(7):
        d = DIMS_A if i % 3 else DIMS_B
        reqs.append((d, G[d][0], inputs.gaussian_spinor(d, 1 + i % 3, seed=200 + i), float(rng.uniform(0.118, 0.124)),
                     prec))
    mix = serve(bq, ctx, reqs, stagger=True)
    for i in (0, 3, 5):
        alone = serve(bq, ctx, [reqs[i]])[0]
        rc_m, info_m, x_m = mix[i]
        rc_a, info_a, x_a = alone
        assert rc_m == rc_a == bq.BQ_OK
        assert np.array_equal(x_m, x_a), i
        assert [c["iters"] for c in info_m] == [c["iters"] for c in info_a]
    # every result solves M x = b for its own kappa (checked by the oracle)
    for i, (d, _, b, k, _) in enumerate(reqs):
        rc, info, x = mix[i]
        ref = orc.Operator(d, G[d][1], k, 1.5)
        for c in range(b.shape[0]):
            assert info[c]["converged"] and info[c]["true_rel_resid"] <= 1e-10
            assert np.linalg.norm(b[c] - ref.M(x[c])) / np.linalg.norm(b[c]) < 1e-7


def test_server_admission_by_budget(world):
    """A request that does not fit the slots waits; all complete in order of capacity."""
    bq, ctx, G = world
    reqs = [(DIMS_A, G[DIMS_A][0], inputs.gaussian_spinor(DIMS_A, 3, seed=300 + i), 0.12, 1) for i in range(4)]
    out = serve(bq, ctx, reqs, slots=4)  # only one 3-column request fits at a time
    assert len(out) == 4 and all(v[0] == bq.BQ_OK for v in out.values())


def test_server_device_buffers(world):
    """Sources and solutions in device memory (torch tensors) give bitwise the host-memory results."""
    import torch
    bq, ctx, G = world
    reqs = [(DIMS_A, G[DIMS_A][0], inputs.gaussian_spinor(DIMS_A, 2, seed=400 + i), 0.121 + 0.001 * i, 1)
            for i in range(3)]
    host = serve(bq, ctx, reqs)
    dev_reqs = [(d, g, torch.from_numpy(b).to("cuda"), k, p) for (d, g, b, k, p) in reqs]
    dev = serve(bq, ctx, dev_reqs)
    for i in range(3):
        rc_h, info_h, x_h = host[i]
        rc_d, info_d, x_d = dev[i]
        assert rc_h == rc_d == bq.BQ_OK
        assert isinstance(x_d, torch.Tensor) and x_d.is_cuda
        assert np.array_equal(x_h, x_d.cpu().numpy())


def test_server_full_residual_reported(world):
    """full_rel_resid of a served request is |b - M x| / |b| on the full lattice: the oracle recomputes it
    from the returned solution."""
    bq, ctx, G = world
    b = inputs.gaussian_spinor(DIMS_A, 2, seed=510)
    out = serve(bq, ctx, [(DIMS_A, G[DIMS_A][0], b, 0.1215, 1)])
    rc, info, x = out[0]
    assert rc == bq.BQ_OK
    ref = orc.Operator(DIMS_A, G[DIMS_A][1], 0.1215, 1.5)
    for c in range(2):
        rel = np.linalg.norm(b[c] - ref.M(x[c])) / np.linalg.norm(b[c])
        print(f"[serve] column {c}: oracle |b - Mx|/|b| {rel:.3e}, reported {info[c]['full_rel_resid']:.3e}",
              flush=True)
        assert abs(rel - info[c]["full_rel_resid"]) <= 0.01 * rel + 1e-15


def test_server_bad_request_isolated(world):
    """A request whose clover is not positive definite finishes with BQ_ERR_CLOVER_NOT_HPD at admission;
    the requests around it complete and match their results alone."""
    bq, ctx, G = world
    g = G[DIMS_A][0]
    good = [inputs.gaussian_spinor(DIMS_A, 1, seed=520 + i) for i in range(3)]
    srv = bq.Server(ctx, 8, 8)
    t0 = srv.submit(g, good[0], 0.12, 1.5)
    tbad = srv.submit(g, inputs.gaussian_spinor(DIMS_A, 1, seed=529), 4.0, 20.0)
    t1 = srv.submit(g, good[1], 0.121, 1.5)
    t2 = srv.submit(g, good[2], 0.122, 1.5)
    res = {}
    for _ in range(1000):
        for t in srv.step():
            res[t] = srv.result(t)
        if len(res) == 4:
            break
    srv.close()
    assert res[tbad][0] == bq.BQ_ERR_CLOVER_NOT_HPD
    for t, b, k in ((t0, good[0], 0.12), (t1, good[1], 0.121), (t2, good[2], 0.122)):
        rc, info, x = res[t]
        assert rc == bq.BQ_OK and info[0]["converged"]
        alone = serve(bq, ctx, [(DIMS_A, g, b, k, 1)])[0]
        assert np.array_equal(alone[2], x)


def _run_to_done(srv, tickets, limit=2000):
    res = {}
    for _ in range(limit):
        for t in srv.step():
            res[t] = srv.result(t)
        if len(res) == len(tickets):
            return res
    raise AssertionError("server did not finish")


def test_server_admission_by_hbm_budget():
    """With a context budget that holds the session and one request's operator but not two, the second
    request waits until the first retires, then completes (in the first one's recycled operator) bitwise
    equal to its result alone."""
    from paper_1711_03836_amd import bqhip as bq
    U = inputs.gauge_field(DIMS_A, 0.2, seed=61)
    ba = inputs.gaussian_spinor(DIMS_A, 1, seed=540)
    bb = inputs.gaussian_spinor(DIMS_A, 1, seed=541)
    # measure: everything held while one request runs, then while two run side by side
    big = bq.Context(0)
    g = bq.Gauge(big, DIMS_A, U)
    srv = bq.Server(big, 4, 4)
    ta = srv.submit(g, ba, 0.12, 1.5)
    srv.step()
    assert srv.pending() == (0, 1)
    used_one = big.hbm_used()
    alone_a = _run_to_done(srv, [ta])[ta]
    srv.close()
    srv = bq.Server(big, 4, 4)
    tb = srv.submit(g, bb, 0.121, 1.5)
    alone_b = _run_to_done(srv, [tb])[tb]
    srv.close()
    srv = bq.Server(big, 4, 4)
    ta = srv.submit(g, ba, 0.12, 1.5)
    tb = srv.submit(g, bb, 0.121, 1.5)
    srv.step()
    assert srv.pending() == (0, 2)
    op_bytes = big.hbm_used() - used_one
    assert op_bytes > 0
    _run_to_done(srv, [ta, tb])
    srv.close()
    srv = None
    # the same work under a budget with room for 1.5 operators
    ctx = bq.Context(0, hbm_budget=used_one + op_bytes // 2)
    g2 = bq.Gauge(ctx, DIMS_A, U)
    srv = bq.Server(ctx, 4, 4)
    ta = srv.submit(g2, ba, 0.12, 1.5)
    tb = srv.submit(g2, bb, 0.121, 1.5)
    srv.step()
    assert srv.pending() == (1, 1)  # b waits for memory, not for slots (4 slots, 2 columns)
    res = _run_to_done(srv, [ta, tb])
    assert res[ta][0] == res[tb][0] == bq.BQ_OK
    assert np.array_equal(res[ta][2], alone_a[2])
    assert np.array_equal(res[tb][2], alone_b[2])
    srv.close()


def test_server_spare_operators_freed_for_budget():
    """A retired request's operator is kept for the next request of its session; when another session
    needs that memory under the budget, the kept operator is freed and the request is admitted."""
    from paper_1711_03836_amd import bqhip as bq
    U = inputs.gauge_field(DIMS_A, 0.2, seed=61)
    b32 = inputs.gaussian_spinor(DIMS_A, 1, seed=545)
    b64 = inputs.gaussian_spinor(DIMS_A, 1, seed=546)
    big = bq.Context(0)
    g = bq.Gauge(big, DIMS_A, U)
    srv = bq.Server(big, 4, 4)
    t32 = srv.submit(g, b32, 0.12, 1.5, inner_prec=1)
    alone32 = _run_to_done(srv, [t32])[t32]
    used_kept = big.hbm_used()  # gauge field, FP32-inner session and its kept operator
    t64 = srv.submit(g, b64, 0.121, 1.5, inner_prec=0)
    srv.step()
    assert srv.pending() == (0, 1)
    used_both = big.hbm_used()  # plus the FP64 session and its operator
    alone64 = _run_to_done(srv, [t64])[t64]
    srv.close()
    assert used_both > used_kept
    # a budget one byte short of holding both sessions with the FP32 operator still kept
    ctx = bq.Context(0, hbm_budget=used_both - 1)
    g2 = bq.Gauge(ctx, DIMS_A, U)
    srv = bq.Server(ctx, 4, 4)
    t32 = srv.submit(g2, b32, 0.12, 1.5, inner_prec=1)
    r32 = _run_to_done(srv, [t32])[t32]
    assert ctx.hbm_used() == used_kept
    t64 = srv.submit(g2, b64, 0.121, 1.5, inner_prec=0)
    r64 = _run_to_done(srv, [t64])[t64]
    assert r32[0] == r64[0] == bq.BQ_OK
    assert np.array_equal(r32[2], alone32[2]) and np.array_equal(r64[2], alone64[2])
    assert ctx.hbm_used() < used_both
    srv.close()


def test_server_release_and_gauge_replacement():
    """Sessions hold their gauge field: freeing it is BQ_ERR_BUSY until bq_server_release; a new field
    of other extents then serves correctly on the same server."""
    from paper_1711_03836_amd import bqhip as bq
    ctx = bq.Context(0)
    U = inputs.gauge_field(DIMS_A, 0.2, seed=61)
    g = bq.Gauge(ctx, DIMS_A, U)
    srv = bq.Server(ctx, 4, 8)
    t = srv.submit(g, inputs.gaussian_spinor(DIMS_A, 1, seed=550), 0.12, 1.5)
    with pytest.raises(bq.BqError) as e:
        srv.release(g)  # the request is still queued
    assert e.value.code == bq.BQ_ERR_BUSY
    _run_to_done(srv, [t])
    with pytest.raises(bq.BqError) as e:
        g.close()
    assert e.value.code == bq.BQ_ERR_BUSY
    held = ctx.hbm_used()
    srv.release(g)
    assert ctx.hbm_used() < held
    g.close()
    U2 = inputs.gauge_field(DIMS_B, 0.2, seed=62)
    g2 = bq.Gauge(ctx, DIMS_B, U2)
    b = inputs.gaussian_spinor(DIMS_B, 2, seed=551)
    t = srv.submit(g2, b, 0.121, 1.5)
    rc, info, x = _run_to_done(srv, [t])[t]
    assert rc == bq.BQ_OK
    ref = orc.Operator(DIMS_B, U2, 0.121, 1.5)
    for c in range(2):
        assert np.linalg.norm(b[c] - ref.M(x[c])) / np.linalg.norm(b[c]) < 1e-7
    srv.close()


def test_server_backfill_order(world):
    """A wide request that does not fit waits; with backfill a later narrow request passes it, with
    backfill 0 (strict arrival order) it does not."""
    bq, ctx, G = world
    g = G[DIMS_A][0]
    first = {}
    for backfill in (0, 8):
        srv = bq.Server(ctx, 4, 4)
        srv.set_backfill(backfill)
        done = {}

        def step():
            for t in srv.step():
                done[t] = srv.result(t)
        t_hold = srv.submit(g, inputs.gaussian_spinor(DIMS_A, 2, seed=560), 0.12, 1.5)
        step()  # the 2-column request now holds 2 of the 4 slots
        t_wide = srv.submit(g, inputs.gaussian_spinor(DIMS_A, 3, seed=561), 0.12, 1.5)
        t_narrow = srv.submit(g, inputs.gaussian_spinor(DIMS_A, 1, seed=562), 0.12, 1.5)
        step()
        first[backfill] = srv.pending()
        for _ in range(2000):
            if len(done) == 3:
                break
            step()
        assert sorted(done) == sorted([t_hold, t_wide, t_narrow])
        assert all(v[0] == bq.BQ_OK for v in done.values())
        srv.close()
    assert first[0] == (2, 1)  # strict order: the narrow request waits behind the wide one
    assert first[8] == (1, 2)  # backfill: the narrow request runs beside the holder


def test_server_idle_step_and_sessions_apart(world):
    """A step with nothing queued or in flight returns at once; requests on two lattices, whose sessions
    advance chunk by chunk independently, each give their result alone bit for bit."""
    bq, ctx, G = world
    srv = bq.Server(ctx, 4, 4)
    assert srv.step() == [] and srv.pending() == (0, 0)
    srv.close()
    reqs = [(DIMS_B, G[DIMS_B][0], inputs.gaussian_spinor(DIMS_B, 3, seed=570), 0.123, 1),
            (DIMS_A, G[DIMS_A][0], inputs.gaussian_spinor(DIMS_A, 1, seed=571), 0.119, 1),
            (DIMS_A, G[DIMS_A][0], inputs.gaussian_spinor(DIMS_A, 2, seed=572), 0.121, 1)]
    mix = serve(bq, ctx, reqs, slots=4, chunk=2)
    for i, r in enumerate(reqs):
        alone = serve(bq, ctx, [r], slots=4, chunk=2)[0]
        assert mix[i][0] == alone[0] == bq.BQ_OK
        assert np.array_equal(mix[i][2], alone[2]), i


def test_server_sessions_per_key(world):
    """With two sessions per gauge field, a request that does not fit the first session's free slots
    opens a second one and starts at once; every result is bitwise its result alone."""
    bq, ctx, G = world
    g = G[DIMS_A][0]
    bs = [inputs.gaussian_spinor(DIMS_A, 3, seed=580 + i) for i in range(3)]
    alone = [serve(bq, ctx, [(DIMS_A, g, b, 0.12 + 0.001 * i, 1)], slots=4, chunk=4)[0] for i, b in enumerate(bs)]
    for per_key, running in ((1, 1), (2, 2)):
        srv = bq.Server(ctx, 4, 4)
        srv.set_sessions(per_key)
        tickets = [srv.submit(g, b, 0.12 + 0.001 * i, 1.5) for i, b in enumerate(bs)]
        srv.step()
        assert srv.pending() == (len(bs) - running, running), per_key
        res = _run_to_done(srv, tickets)
        srv.close()
        for i, t in enumerate(tickets):
            assert res[t][0] == bq.BQ_OK
            assert np.array_equal(res[t][2], alone[i][2]), (per_key, i)
    with pytest.raises(bq.BqError):
        bq.Server(ctx, 4, 4).set_sessions(0)
