"""Batched execution: planes of different size, type, transfer function,
distance and point count recorded into one HIP graph must give, plane by
plane, what the plain single-plane path gives; graph replays (with the
program's own eager work between them) must keep giving it."""
import numpy as np
import pytest

import synth
from gpu_util import check_close, dev, host, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _planes(seed, P):
    rng = np.random.default_rng(seed)
    specs, data = [], []
    for p in range(P):
        N = int(rng.choice([32, 64, 128, 256]))
        t = int(rng.integers(1, 3))
        tf = "asm" if rng.uniform() < 0.5 else "fresnel"
        z = float(rng.uniform(0.005, 0.5)) * (1e-1 if N <= 64 else 1.0)
        g = 4e-6
        M = int(np.exp(rng.uniform(np.log(100), np.log(40000))))
        x, y = synth.clustered_box(rng, M, N * g)
        inp = synth.unit_phase(rng, M if t == 1 else (N, N))
        specs.append(dict(N=N, type=t, lam=633e-9, z=z, g=g, tf=tf,
                          band="limited" if tf == "asm" else "full", tol=1e-6))
        data.append((x, y, inp))
    return specs, data


def test_batch_matches_plain_plans_and_replays(capfd):
    import paper_1308_6644_amd as P
    P.load()
    specs, data = _planes(11, 12)
    print(f"batch of {len(specs)} planes", flush=True)
    xs = [dev(torch, d[0]) for d in data]
    ys = [dev(torch, d[1]) for d in data]
    ins = [dev(torch, d[2]) for d in data]
    outs = []
    refs = []
    for s, x, y, i in zip(specs, xs, ys, ins):
        plan = P.Plan(**{k: v for k, v in s.items()})
        plan.set_points(x, y)
        refs.append(host(plan.execute(i)))
        N = s["N"]
        outs.append(torch.empty((2 * N, 2 * N) if s["type"] == 1 else (x.numel(),),
                                dtype=torch.complex64, device="cuda"))
    b = P.Batch(specs)
    for rep in range(3):
        for o in outs:
            o.zero_()               # eager work between graph replays
        torch.cuda.synchronize()
        b.run(xs, ys, ins, outs)
        assert b.check_points() == -1
        for p, (o, r) in enumerate(zip(outs, refs)):
            err = check_close(host(o), r, 1e-6, what=str((rep, p, specs[p])))
    t = b.plane_times()
    assert len(t) == len(specs) and all(v > 0 for v in t)


def test_grouped_and_per_plane_forms_match_plain_plans():
    """The batch's two graph forms -- grouped stage launches over descriptor
    tables (default) and every plane's own launches on parallel branches --
    against plain plans, for the one-shot run and for points bound once with
    two operator runs (set_points_many / execute_many)."""
    import paper_1308_6644_amd as P
    P.load()
    specs, data = _planes(23, 10)
    print(f"grouped vs per-plane: {len(specs)} planes", flush=True)
    xs = [dev(torch, d[0]) for d in data]
    ys = [dev(torch, d[1]) for d in data]
    ins = [dev(torch, d[2]) for d in data]
    refs = []
    for s, x, y, i in zip(specs, xs, ys, ins):
        plan = P.Plan(**s)
        plan.set_points(x, y)
        refs.append(host(plan.execute(i)))

    def outs():
        return [torch.full((2 * s["N"], 2 * s["N"]) if s["type"] == 1 else (x.numel(),), float("nan"),
                           dtype=torch.complex64, device="cuda") for s, x in zip(specs, xs)]
    for grouped in (True, False):
        b = P.Batch(specs)
        b.set_grouped(grouped)
        o = outs()
        for rep in range(2):
            b.run(xs, ys, ins, o)
            assert b.check_points() == -1
            for p, r in enumerate(refs):
                check_close(host(o[p]), r, 1e-6, what=f"run grouped={grouped} rep={rep} plane {p}")
        o2 = outs()
        b.set_points(xs, ys)
        for rep in range(2):
            b.execute(ins, o2)
            for p, r in enumerate(refs):
                check_close(host(o2[p]), r, 1e-6, what=f"many grouped={grouped} rep={rep} plane {p}")
        t = b.plane_times()
        assert len(t) == len(specs) and all(v > 0 for v in t)
        # without completion stamps: the same results; plane times refused
        b.set_plane_times(False)
        o3 = outs()
        b.run(xs, ys, ins, o3)
        for p, r in enumerate(refs):
            check_close(host(o3[p]), r, 1e-6, what=f"no stamps grouped={grouped} plane {p}")
        with pytest.raises(P.NuasmError):
            b.plane_times()
        b.set_plane_times(True)
        with pytest.raises(P.NuasmError):
            b.plane_times()  # the graphs were dropped: nothing has run since
        b.run(xs, ys, ins, o3)
        t2 = b.plane_times()
        assert all(v > 0 for v in t2)
        b.close()
