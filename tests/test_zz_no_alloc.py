"""bq_apply_noalloc (the allocation-free form of bq_apply) through the C ABI.

Its work fields live in a static per-device array instead of fresh device memory, so for every
operator kind that needs them (M^dag M, Mhat, Mhat^dag, Mhat^dag Mhat) and one that does not (K1),
in FP64, FP32 and FP16:
  - two calls in a row, the second on a smaller lattice with fewer columns (the array still holds
    the first call's larger intermediate), each give bitwise the output of bq_apply on the same
    input, and both are within the precision's bar of the oracle;
  - the context's allocator is not called and its device memory does not grow;
  - work fields beyond the array's size are refused with BQ_ERR_INVALID, and the same kind with
    fewer columns then runs.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1711_03836_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5, 2: 4e-3}
KINDS = ("BQ_OP_MDAGM", "BQ_OP_MHAT", "BQ_OP_MHATDAG", "BQ_OP_MHATDAG_MHAT", "BQ_OP_K1")


def oracle_apply(ref, bq, kind, psi):
    if kind == bq.BQ_OP_MDAGM:
        return ref.M(ref.M(psi), dagger=True)
    if kind == bq.BQ_OP_MHAT:
        return ref.Mhat(ref.odd(psi))
    if kind == bq.BQ_OP_MHATDAG:
        return ref.Mhat(ref.odd(psi), dagger=True)
    if kind == bq.BQ_OP_MHATDAG_MHAT:
        return ref.Mhat(ref.Mhat(ref.odd(psi)), dagger=True)
    if kind == bq.BQ_OP_K1:
        h = ref.even(ref.hop(ref.odd(psi)))
        return orc.clover_apply(ref.dims, ref.Tinv, h, parity_mask=1)
    raise ValueError(kind)


@pytest.fixture(scope="module")
def bq():
    from paper_1711_03836_amd import bqhip
    return bqhip


@pytest.fixture(scope="module")
def counted(bq):
    """A context whose device memory comes from torch's caching allocator, with every call counted."""
    import torch
    count = {"alloc": 0, "free": 0}

    def alloc(n):
        count["alloc"] += 1
        return torch.cuda.caching_allocator_alloc(n, 0)

    def dealloc(p):
        count["free"] += 1
        torch.cuda.caching_allocator_delete(p)
    ctx = bq.Context(0, alloc=alloc, dealloc=dealloc)
    yield ctx, count
    ctx.close()


def _world(bq, ctx, dims, seed):
    U = inputs.gauge_field(dims, 0.3, seed=seed)
    G = bq.Gauge(ctx, dims, U, t_bc=-1)
    op = bq.Op(G, 0.124, 1.4, 0.1)
    ref = orc.Operator(dims, U, 0.124, 1.4, mu=0.1, t_bc=-1)
    return G, op, ref


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_noalloc_matches_apply_two_calls(bq, counted, prec):
    ctx, count = counted
    big, small = (8, 8, 8, 16), (4, 4, 4, 8)
    worlds = {big: _world(bq, ctx, big, 400 + prec), small: _world(bq, ctx, small, 410 + prec)}
    for kind_name in KINDS:
        kind = getattr(bq, kind_name)
        si, so = bq.OP_SUBSETS[kind]
        runs = []
        for dims, nrhs in ((big, 3), (small, 1)):
            G, op, ref = worlds[dims]
            psi = inputs.gaussian_spinor(dims, nrhs, seed=50 + nrhs + prec)
            fi = bq.Field(ctx, dims, si, prec, nrhs)
            fo = bq.Field(ctx, dims, so, prec, nrhs)
            fi.put(psi)
            runs.append((dims, nrhs, psi, fi, fo))
        # the two allocation-free calls back to back, then the allocating entry point
        n0, used0 = dict(count), ctx.hbm_used()
        got = []
        for dims, nrhs, psi, fi, fo in runs:
            print(f"noalloc {kind_name} prec={prec} dims={dims} nrhs={nrhs}", flush=True)
            worlds[dims][1].apply_noalloc(kind, fi, fo)
        assert count == n0, (kind_name, count, n0)
        assert ctx.hbm_used() == used0
        for dims, nrhs, psi, fi, fo in runs:
            got.append(fo.get())  # (a host copy stages through device memory)
        for (dims, nrhs, psi, fi, fo), g in zip(runs, got):
            G, op, ref = worlds[dims]
            op.apply(kind, fi, fo)
            want = fo.get()
            assert np.array_equal(g, want), (kind_name, prec, dims)
            mask = {bq.BQ_EVEN: ref.parity == 0, bq.BQ_ODD: ref.parity == 1, bq.BQ_FULL: np.ones(ref.V, bool)}[so]
            for c in range(nrhs):
                o = oracle_apply(ref, bq, kind, psi[c])
                err = np.abs(g[c][mask] - o[mask]).max() / np.abs(o[mask]).max()
                assert err < TOL[prec], (kind_name, prec, dims, c, err)
            fi.close()
            fo.close()
    for G, op, ref in worlds.values():
        op.close()
        G.close()


def test_noalloc_size_limit(bq, counted):
    ctx, count = counted
    dims = (12, 12, 12, 24)  # one FP64 full-lattice spinor column: 41472 x 24 x 8 bytes = 7.96 MB
    G, op, ref = _world(bq, ctx, dims, 420)
    assert bq.BQ_NOALLOC_SCRATCH_BYTES == 64 << 20
    big_in = bq.Field(ctx, dims, bq.BQ_FULL, bq.BQ_F64, 12)  # M^dag M work field: 95.6 MB
    big_out = bq.Field(ctx, dims, bq.BQ_FULL, bq.BQ_F64, 12)
    with pytest.raises(bq.BqError) as e:
        op.apply_noalloc(bq.BQ_OP_MDAGM, big_in, big_out)
    assert e.value.code == bq.BQ_ERR_INVALID
    # the same kind with 4 columns (31.9 MB) runs and matches bq_apply
    psi = inputs.gaussian_spinor(dims, 4, seed=421)
    fi = bq.Field(ctx, dims, bq.BQ_FULL, bq.BQ_F64, 4)
    fo = bq.Field(ctx, dims, bq.BQ_FULL, bq.BQ_F64, 4)
    fi.put(psi)
    n0 = dict(count)
    op.apply_noalloc(bq.BQ_OP_MDAGM, fi, fo)
    assert count == n0
    got = fo.get()
    op.apply(bq.BQ_OP_MDAGM, fi, fo)
    assert np.array_equal(got, fo.get())
    for h in (fo, fi, big_out, big_in, op, G):
        h.close()
