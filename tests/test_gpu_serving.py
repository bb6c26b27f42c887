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
