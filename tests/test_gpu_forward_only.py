"""NUASM_FORWARD_ONLY: a type-2 plan whose points are binned for
interpolation alone -- one record per point, in the bin that holds its first
tap, instead of one in every bin its taps touch.  Interpolation reads only
those records, so its outputs must equal a fully binned plan's bit for bit
(each output is one point's own sum over the same staged tile, whatever the
order of the records); the adjoint, which spreads and needs every bin's
records, is refused; the flag is refused on other plan types.  Default and
deterministic binning, 32- and 64-cell bins, rejected points under a
deferred range check, and a batch.
"""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import check_close, dev, geometry, host, make_plan
from test_gpu_determinism import decode, expected_records

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1308_6644_amd as P
    P.load()
    return P


@pytest.mark.parametrize("deterministic", [False, True])
def test_records_are_the_first_tap_bins(P, deterministic):
    N, M = 32, 3000
    print(f"forward-only records: det={deterministic}", flush=True)
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.01, tf="asm", band="full")
    rng = np.random.default_rng(51)
    x, y = synth.clustered_box(rng, M, N * geo.g, frac=0.8, sigma_frac=0.05)
    plan = make_plan(P, geo, 2, deterministic=deterministic, forward_only=True)
    plan.set_points(dev(torch, x), dev(torch, y))
    recs, counts = plan.debug_records()
    idx, bins, lx, ly, prim, dx, dy, c = decode(recs, counts)
    assert c.sum() == idx.size == M
    exp = [e for e in expected_records(x, y, plan.info, geo.g) if e[4]]
    got = sorted(zip(idx.tolist(), bins.tolist(), lx.tolist(), ly.tolist(), prim.tolist()))
    want = sorted((e[0], e[1], e[2], e[3], 1) for e in exp)
    assert got == want
    if deterministic:
        for b in np.unique(bins):
            assert np.all(np.diff(idx[bins == b]) > 0), f"bin {b} not in point order"


@pytest.mark.parametrize("tile", [32, 64])
@pytest.mark.parametrize("deterministic", [False, True])
def test_outputs_equal_full_binning_and_oracle(P, tile, deterministic):
    N, M = 128, 40000
    print(f"forward-only outputs: tile={tile} det={deterministic} N={N} M={M}", flush=True)
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.05, tf="asm", band="limited", ox=2e-4)
    rng = np.random.default_rng(53)
    x, y = synth.clustered_box(rng, M, N * geo.g)
    u1 = synth.unit_phase(rng, (N, N))
    xd, yd, ud = dev(torch, x), dev(torch, y), dev(torch, u1)
    outs = []
    for fwd in (False, True):
        plan = make_plan(P, geo, 2, deterministic=deterministic, forward_only=fwd)
        plan.set_tuning(bin_tile=tile)
        plan.set_points(xd, yd)
        outs.append(host(plan.execute(ud)))
    assert np.array_equal(outs[0].view(np.uint32), outs[1].view(np.uint32))
    sel = rng.choice(M, size=256, replace=False)
    ref = O.nuasm2(geo, u1, x[sel], y[sel], O.transfer(geo))
    check_close(outs[1][sel], ref, 1e-5)


def test_adjoint_and_other_types_refused(P):
    N, M = 32, 500
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.01, tf="asm", band="full")
    rng = np.random.default_rng(55)
    x, y = synth.clustered_box(rng, M, N * geo.g)
    plan = make_plan(P, geo, 2, forward_only=True)
    plan.set_points(dev(torch, x), dev(torch, y))
    with pytest.raises(P.NuasmError) as e:
        plan.adjoint(dev(torch, synth.unit_phase(rng, M)))
    assert e.value.status == 4  # NUASM_ERR_UNSUPPORTED
    for t in (1, 3):
        with pytest.raises(P.NuasmError) as e:
            make_plan(P, geo, t, forward_only=True)
        assert e.value.status == 1  # NUASM_ERR_INVALID_ARG


@pytest.mark.parametrize("deterministic", [False, True])
def test_rejected_points_with_forward_only(P, deterministic):
    N, M = 64, 3000
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.01, tf="asm", band="limited", ox=1e-4)
    rng = synth.rng_for(57, 0)
    x, y = synth.clustered_box(rng, M, N * geo.g)
    bad = rng.choice(M, size=150, replace=False)
    x = x.copy()
    x[bad[::2]] = 0.7 * N * geo.g
    y = y.copy()
    y[bad[1::2]] = np.nan
    acc = np.ones(M, bool)
    acc[bad] = False
    u1 = synth.unit_phase(rng, (N, N))
    plan = make_plan(P, geo, 2, defer_range_check=True, deterministic=deterministic, forward_only=True)
    plan.set_points(dev(torch, x), dev(torch, y))
    out = host(plan.execute(dev(torch, u1)))
    with pytest.raises(P.NuasmError):
        plan.check_points()
    assert np.all(np.isnan(out[~acc]))
    ref = O.nuasm2(geo, u1, x[acc], y[acc], O.transfer(geo))
    check_close(out[acc], ref, 1e-5)


@pytest.mark.parametrize("grouped", [True, False])
def test_batch_with_forward_only_planes(P, grouped):
    rng = np.random.default_rng(59)
    specs, xs, ys, ins, refs = [], [], [], [], []
    for k, (N, tf, z) in enumerate([(64, "asm", 0.01), (128, "fresnel", 0.05), (64, "asm", 0.2)]):
        geo = geometry(N=N, g=4e-6, lam=633e-9, z=z, tf=tf, band="limited" if tf == "asm" else "full")
        M = 5000 + 3000 * k
        x, y = synth.clustered_box(rng, M, N * geo.g)
        u = synth.unit_phase(rng, (N, N))
        for fwd in (True, False):
            specs.append(dict(N=N, type=2, lam=geo.lam, z=z, g=geo.g, tf=tf, band=geo.band, tol=1e-6,
                              forward_only=fwd))
            xs.append(dev(torch, x))
            ys.append(dev(torch, y))
            ins.append(dev(torch, u))
        plan = make_plan(P, geo, 2)
        plan.set_points(xs[-1], ys[-1])
        refs.append(host(plan.execute(ins[-1])))
    print(f"forward-only batch: grouped={grouped} {len(specs)} planes", flush=True)
    b = P.Batch(specs)
    b.set_grouped(grouped)
    outs = [torch.full((x.numel(),), float("nan"), dtype=torch.complex64, device="cuda") for x in xs]
    for _ in range(2):
        b.run(xs, ys, ins, outs)
    for p in range(len(specs)):
        got = host(outs[p])
        assert np.array_equal(got.view(np.uint32), refs[p // 2].view(np.uint32)), f"plane {p}"
