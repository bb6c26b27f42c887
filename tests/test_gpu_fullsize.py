"""The 32^3x64 multi-column workload at full size, in the launch configuration the autotuner picks
(the configuration bench.py times), against the oracle on the whole lattice.

  - K1 = T_ee^-1 D_eo, Mhat, Mhat^dag and Mhat^dag Mhat on 12 FP32 Gaussian columns: every site of
    every column, 1e-5 relative to the largest reference element (the FP32 field-agreement bar);
  - the 12 point-source solve (FP32 inner, FP64 reliable updates, tol 1e-10): for every column the
    oracle recomputes |b - M x| / |b| on the whole lattice from the GPU solution, and it must agree
    with the full-system residual the library reports to 1%;
  - FP32 Mhat on 48^3x96 with 16 columns in the t-marching configuration the trace workload uses,
    at sampled odd sites;
  - FP64 Mhat on 48^3x160, where a parity's FP64 clover array is larger than 4 GiB.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_1711_03836_amd import inputs

pytestmark = pytest.mark.gpu

DIMS = (32, 32, 32, 64)
KAPPA, CSW, MU, EPS = 0.124, 1.5, 0.1, 0.2


@pytest.fixture(scope="module")
def world():
    from paper_1711_03836_amd import bqhip as bq
    U = inputs.gauge_field(DIMS, EPS, seed=20171110)
    ctx = bq.Context(0)
    G = bq.Gauge(ctx, DIMS, U, -1)
    op = bq.Op(G, KAPPA, CSW, MU)
    op.autotune(bq.BQ_F32, 12)
    print(f"[fullsize] tune f32 x12 = {ctx.tune_get(bq.BQ_F32, 12)}", flush=True)
    ref = orc.Operator(DIMS, U, KAPPA, CSW, mu=MU, t_bc=-1)
    return bq, U, ctx, G, op, ref


@pytest.mark.timeout(900)
def test_whole_lattice_12_columns(world):
    bq, U, ctx, G, op, ref = world
    psi = inputs.gaussian_spinor(DIMS, 12, seed=5)
    for name in ("K1", "MHAT", "MHATDAG", "MHATDAG_MHAT"):
        kind = getattr(bq, "BQ_OP_" + name)
        si, so = bq.OP_SUBSETS[kind]
        fi = bq.Field(ctx, DIMS, si, bq.BQ_F32, 12)
        fo = bq.Field(ctx, DIMS, so, bq.BQ_F32, 12)
        fi.put(psi)
        op.apply(kind, fi, fo)
        got = fo.get()
        fi.close()
        fo.close()
        mask = ref.parity == (0 if so == bq.BQ_EVEN else 1)
        worst = 0.0
        for c in range(12):
            p = psi[c]
            if name == "K1":
                want = orc.clover_apply(DIMS, ref.Tinv, ref.even(ref.hop(ref.odd(p))), parity_mask=1)
            elif name == "MHAT":
                want = ref.Mhat(ref.odd(p))
            elif name == "MHATDAG":
                want = ref.Mhat(ref.odd(p), dagger=True)
            else:
                want = ref.Mhat(ref.Mhat(ref.odd(p)), dagger=True)
            err = np.abs(got[c][mask] - want[mask]).max() / np.abs(want[mask]).max()
            worst = max(worst, err)
            assert err < 1e-5, (name, c, err)
            assert np.all(got[c][~mask] == 0)
        print(f"[fullsize] {name} x12 FP32, whole lattice: worst max rel err {worst:.2e}", flush=True)
        del got


@pytest.mark.timeout(900)
def test_point_source_solve_oracle_residual(world):
    bq, U, ctx, G, op, ref = world
    b = inputs.point_sources(DIMS)
    fb = bq.Field(ctx, DIMS, bq.BQ_FULL, bq.BQ_F64, 12)
    fx = bq.Field(ctx, DIMS, bq.BQ_FULL, bq.BQ_F64, 12)
    fb.put(b)
    rc, info = op.solve(fb, fx, 1e-10, system=bq.BQ_SYS_M, inner_prec=bq.BQ_F32)
    assert rc == bq.BQ_OK, info
    x = fx.get()
    for c in range(12):
        assert info[c]["converged"] and info[c]["true_rel_resid"] <= 1e-10
        rel = np.linalg.norm(b[c] - ref.M(x[c])) / np.linalg.norm(b[c])
        print(f"[fullsize] point source {c}: oracle |b - Mx|/|b| {rel:.3e}, reported "
              f"{info[c]['full_rel_resid']:.3e}, {info[c]['iters']} iterations", flush=True)
        assert abs(rel - info[c]["full_rel_resid"]) <= 0.01 * rel + 1e-15, (c, rel, info[c])
        assert rel < 1e-8


@pytest.mark.timeout(900)
def test_trace_configuration_48x96_sampled():
    """48^3x96 with 16 columns in the launch configurations the trace workload takes (FP32, two-row
    links: 2 columns per thread, 256 sites per workgroup, t-marching in segments of 4; and the
    tile-shared stencil with 16 column waves per tile in the z-slab traversal): FP32 Mhat at sampled
    odd sites, most on time and space boundaries.  The links are a 48^3x32 field U = exp(0.15 i H)
    repeated three times along t; the 16 columns cycle through three Gaussian fields, so a column
    read from a neighbouring column's storage would show."""
    import torch
    from paper_1711_03836_amd import bqhip as bq
    dims = (48, 48, 48, 96)
    base = inputs.gauge_field((48, 48, 48, 32), 0.15, seed=4896)
    U = np.concatenate([base] * 3, axis=1)
    del base
    ctx = bq.Context(0)
    G = bq.Gauge(ctx, dims, U, -1)
    op = bq.Op(G, 0.1235, 1.9, 0.0)
    psi3 = inputs.gaussian_spinor(dims, 3, seed=96)
    cols = [c % 3 for c in range(16)]
    dev = torch.from_numpy(psi3).to("cuda")[cols].contiguous()
    fi = bq.Field(ctx, dims, bq.BQ_ODD, bq.BQ_F32, 16)
    fo = bq.Field(ctx, dims, bq.BQ_ODD, bq.BQ_F32, 16)
    fi.put(dev)
    outs = []
    for tune in ((12, 2, 256, 4, 0, 0), (12, 1, 1024, 0, 1, 1)):
        ctx.tune_set(bq.BQ_F32, 16, *tune)
        op.apply(bq.BQ_OP_MHAT, fi, fo)
        out = torch.zeros_like(dev)
        fo.get(out)
        outs.append(out)
    assert torch.equal(outs[0], outs[1])
    out = outs[0]
    del outs
    rng = np.random.default_rng(4896)
    L = dims
    pts = [(1, 0, 0, 0), (0, 0, 0, 95), (47, 47, 47, 94), (0, 47, 0, 31), (1, 0, 47, 32), (0, 1, 0, 64)]
    while len(pts) < 120:
        pts.append(tuple(int(rng.integers(l)) for l in L))
    sites = np.array(sorted({x[0] + L[0] * (x[1] + L[1] * (x[2] + L[2] * x[3])) for x in pts if sum(x) % 2 == 1}),
                     dtype=np.int64)
    got = out[:, torch.from_numpy(sites).to("cuda")].cpu().numpy()
    del out, dev
    want = [orc.Mhat_sites(dims, U, 0.1235, 1.9, psi3[k], sites, t_bc=-1, mu=0.0) for k in range(3)]
    for c in range(16):
        err = np.abs(got[c] - want[cols[c]]).max() / np.abs(want[cols[c]]).max()
        assert err < 1e-5, (c, err)
    print(f"[fullsize] 48^3x96 Mhat x16 (march 4 and tile-shared, bitwise equal) at {len(sites)} odd sites: ok",
          flush=True)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("inner", [0, 1, 2])
def test_single_source_16x32_oracle_residual(inner):
    """16^3x32, U = exp(0.2 i H), kappa 0.125, c_SW 1.7, one Gaussian source, tol 1e-10 through the
    Schur system with FP64, FP32-inner and FP16-inner CG: the oracle recomputes b - M x on the whole
    lattice from the GPU solution and agrees with the full-system residual the library reports."""
    from paper_1711_03836_amd import bqhip as bq
    dims = (16, 16, 16, 32)
    U = inputs.gauge_field(dims, 0.2, seed=1711)
    b = inputs.gaussian_spinor(dims, 1, seed=3836)
    ctx = bq.Context(0)
    G = bq.Gauge(ctx, dims, U, -1)
    op = bq.Op(G, 0.125, 1.7, 0.0)
    fb = bq.Field(ctx, dims, bq.BQ_FULL, bq.BQ_F64, 1)
    fx = bq.Field(ctx, dims, bq.BQ_FULL, bq.BQ_F64, 1)
    fb.put(b)
    rc, info = op.solve(fb, fx, 1e-10, system=bq.BQ_SYS_M, inner_prec=inner, chunk=16)
    assert rc == bq.BQ_OK and info[0]["converged"] and info[0]["true_rel_resid"] <= 1e-10
    x = fx.get()[0]
    ref = orc.Operator(dims, U, 0.125, 1.7)
    rel = np.linalg.norm(b[0] - ref.M(x)) / np.linalg.norm(b[0])
    print(f"[single16] inner {inner}: {info[0]['iters']} iterations, oracle residual {rel:.3e}, "
          f"reported {info[0]['full_rel_resid']:.3e}", flush=True)
    assert abs(rel - info[0]["full_rel_resid"]) <= 0.01 * rel + 1e-15
    assert rel < 1e-8


@pytest.mark.timeout(900)
def test_large_lattice_fp64_mhat_sampled():
    """48^3x160 (V/2 = 8.8M sites per parity), where one FP64 clover array of a parity takes
    4.9 GB, more than a 32-bit byte offset reaches: FP64 Mhat on one Gaussian column against the
    oracle at sampled odd sites, most of them in the last 25 time slices, whose clover entries lie
    beyond the first 4 GiB of the array (1e-12 relative to the largest sampled element).  The
    links are a 48^3x32 field U = exp(0.2 i H) repeated five times along t."""
    from paper_1711_03836_amd import bqhip as bq
    dims = (48, 48, 48, 160)
    base = inputs.gauge_field((48, 48, 48, 32), 0.2, seed=48160)
    U = np.concatenate([base] * 5, axis=1)
    del base
    psi = inputs.gaussian_spinor(dims, 1, seed=7)
    ctx = bq.Context(0)
    G = bq.Gauge(ctx, dims, U, -1)
    op = bq.Op(G, 0.124, 1.5, 0.1)
    fi = bq.Field(ctx, dims, bq.BQ_ODD, bq.BQ_F64, 1)
    fo = bq.Field(ctx, dims, bq.BQ_ODD, bq.BQ_F64, 1)
    fi.put(psi)
    op.apply(bq.BQ_OP_MHAT, fi, fo)
    got = fo.get()[0]
    rng = np.random.default_rng(160)
    L = dims
    pts = [(0, 0, 0, 159), (47, 47, 47, 158), (1, 0, 0, 135), (0, 47, 0, 136), (13, 5, 40, 0)]
    while len(pts) < 160:
        t = int(rng.integers(135, 160)) if len(pts) % 4 else int(rng.integers(160))
        pts.append((int(rng.integers(48)), int(rng.integers(48)), int(rng.integers(48)), t))
    sites = np.array(sorted({x[0] + L[0] * (x[1] + L[1] * (x[2] + L[2] * x[3]))
                             for x in pts if sum(x) % 2 == 1}), dtype=np.int64)
    assert len(sites) >= 40
    want = orc.Mhat_sites(dims, U, 0.124, 1.5, psi[0], sites, t_bc=-1, mu=0.1)
    err = np.abs(got[sites] - want).max() / np.abs(want).max()
    print(f"[large] 48^3x160 FP64 Mhat at {len(sites)} odd sites: max rel err {err:.2e}", flush=True)
    assert err < 1e-12, err
