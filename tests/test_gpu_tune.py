"""Launch-shape tuning: every tunable setting (small spreading chunks,
interpolation chunk sizes, binning ranges, graph branches) must give the
oracle's result to the operator bar, and the autotuner must produce a
setting, cache it and apply it to a batch whose results stay those of plain
plans."""
import sys

import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import check_close, dev, geometry, host, make_plan, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1308_6644_amd as P
    P.load()
    return P


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


TUNINGS = [
    dict(spread_chunk=896),
    dict(interp_chunk=256),
    dict(interp_chunk=8192, bin_range_points=1024),
    dict(spread_chunk=896, interp_chunk=1024, bin_range_points=65535),
    dict(bin_tile=64),
    dict(bin_tile=64, spread_chunk=896, interp_chunk=1024, bin_range_points=1024),
    dict(spread_method=1),
]


@pytest.mark.parametrize("tol", [1e-6, 1e-12])
@pytest.mark.parametrize("tuning", TUNINGS, ids=lambda t: "-".join(f"{k}{v}" for k, v in t.items()))
def test_tuned_shapes_match_oracle(P, tuning, tol):
    """Dense clustered points so that bins split into several chunks at every
    chunk size (w = 7 and w = 13: both spreading sub-batch sizes)."""
    N, M = 64, 12000
    _say("tuned", tuning, tol)
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.01, tf="asm", band="limited", ox=1e-4)
    rng = np.random.default_rng(17)
    x, y = synth.clustered_box(rng, M, N * geo.g, frac=0.9, sigma_frac=0.03)
    c = synth.unit_phase(rng, M)
    u1 = synth.unit_phase(rng, (N, N))
    bound = 1e-5 if tol == 1e-6 else 2e-6
    for t, inp, ref in ((1, c, O.nuasm1(geo, x, y, c)), (2, u1, O.nuasm2(geo, u1, x, y))):
        plan = make_plan(P, geo, t, tol=tol)
        plan.set_tuning(**tuning)
        plan.set_points(dev(torch, x), dev(torch, y))
        info = plan.info
        if tuning.get("interp_chunk"):
            assert info["interp_chunk"] == tuning["interp_chunk"]
        assert info["tile"] == (tuning.get("bin_tile") or 32)
        if tuning.get("spread_chunk"):
            assert info["spread_chunk"] == (896 if tol == 1e-6 else 1024)
        check_close(host(plan.execute(dev(torch, inp))), ref, bound)


def test_set_tuning_requires_rebinding(P):
    _say("tuning rebinding")
    geo = geometry(N=32, g=4e-6, lam=633e-9, z=0.01)
    rng = np.random.default_rng(3)
    x, y = synth.uniform_box(rng, 500, 32 * geo.g)
    c = dev(torch, synth.unit_phase(rng, 500))
    plan = make_plan(P, geo, 1)
    plan.set_points(dev(torch, x), dev(torch, y))
    plan.execute(c)
    plan.set_tuning(interp_chunk=1024)
    with pytest.raises(P.NuasmError) as ei:
        plan.execute(c)
    assert ei.value.name == "NUASM_ERR_NOT_READY"
    plan.set_points(dev(torch, x), dev(torch, y))
    plan.execute(c)
    with pytest.raises(P.NuasmError):
        plan.set_tuning(interp_chunk=100)
    # a grid stays bound across tuning changes
    plan.set_grid_points(10, 10, geo.g)
    plan.set_tuning()
    plan.execute(dev(torch, synth.unit_phase(rng, 100)))



def test_tuning_while_grid_bound_resizes_tables(P):
    """A point set bound as a grid across a tuning change keeps buffers sized
    for the old chunk sizes; binning points into it again afterwards, with
    fewer points than it held before and much smaller chunks, must resize its
    chunk tables and histogram rows and give the oracle's result."""
    N = 64
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.01, tf="asm", band="limited", ox=1e-4)
    rng = np.random.default_rng(29)
    x0, y0 = synth.uniform_box(rng, 20000, N * geo.g)
    x, y = synth.clustered_box(rng, 12000, N * geo.g, frac=0.9, sigma_frac=0.03)
    c = synth.unit_phase(rng, 12000)
    u1 = synth.unit_phase(rng, (N, N))
    for t, inp, ref in ((1, c, O.nuasm1(geo, x, y, c)), (2, u1, O.nuasm2(geo, u1, x, y))):
        _say("tuning while grid-bound, type", t)
        plan = make_plan(P, geo, t)
        plan.set_points(dev(torch, x0), dev(torch, y0))
        plan.set_grid_points(16, 16, geo.g)
        plan.set_tuning(spread_chunk=896, interp_chunk=256, bin_range_points=1024)
        plan.set_points(dev(torch, x), dev(torch, y))
        assert plan.info["interp_chunk"] == 256
        check_close(host(plan.execute(dev(torch, inp))), ref, 1e-5)

def test_autotuner_batch(P, tmp_path):
    """Tune a small mixed batch into a fresh cache, check the cache and the
    results against plain plans, then apply the cache to a new batch."""
    from paper_1308_6644_amd import tune
    _say("autotuner")
    rng = np.random.default_rng(21)
    specs, xs, ys, ins, outs = [], [], [], [], []
    for p in range(6):
        n = [64, 128][p % 2]
        m = [3000, 20000, 70000][p % 3]
        t = 1 + (p % 2)
        tf = "asm" if p < 3 else "fresnel"
        specs.append(dict(N=n, type=t, lam=633e-9, z=0.01 * (p + 1), g=4e-6, tf=tf,
                          band="limited" if tf == "asm" else "full", tol=1e-6))
        x, y = synth.clustered_box(rng, m, n * 4e-6)
        xs.append(dev(torch, x))
        ys.append(dev(torch, y))
        ins.append(dev(torch, synth.unit_phase(rng, m if t == 1 else (n, n))))
        outs.append(torch.empty((2 * n, 2 * n) if t == 1 else (m,), dtype=torch.complex64, device="cuda"))
    cache = tune.TuneCache(str(tmp_path / "tune.json"))
    b = P.Batch(specs)
    summary = tune.tune_batch(b, specs, xs, ys, ins, outs, cache, reps=2)
    _say("  ", summary)
    assert summary["planes_tuned"] >= 1 and 1 <= summary["branches"] <= 4
    assert (tmp_path / "tune.json").exists()
    b.run(xs, ys, ins, outs)
    assert b.check_points() == -1
    for p, s in enumerate(specs):
        plain = P.Plan(**s)
        plain.set_points(xs[p], ys[p])
        ref = host(plain.execute(ins[p]))
        check_close(host(outs[p]), ref, 2e-6)
    # a second batch of the same shapes takes everything from the cache
    b2 = P.Batch(specs)
    assert tune.apply_cached(b2, specs, [x.numel() for x in xs], tune.TuneCache(str(tmp_path / "tune.json"))) == 6
    outs2 = [torch.empty_like(o) for o in outs]
    b2.set_grouped(True)
    b2.run(xs, ys, ins, outs2)
    for p in range(6):
        check_close(host(outs2[p]), host(outs[p]), 2e-6)
    b2.set_grouped(False)
    for k in (1, 2, 3, 4):
        b2.set_branches(k)
        b2.run(xs, ys, ins, outs2)
        for p in range(6):
            check_close(host(outs2[p]), host(outs[p]), 2e-6)
    with pytest.raises(P.NuasmError):
        b2.set_branches(5)
