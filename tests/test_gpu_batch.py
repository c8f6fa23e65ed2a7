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


def test_grouped_graph_takes_new_buffers_without_recording():
    """A grouped graph run with other buffers but the same point counts keeps
    its recording and only rewrites its argument tables (one-shot run and
    execute_many); the results are those of plain plans on the new data.
    A changed count, and any change in the per-plane form, record again."""
    import paper_1308_6644_amd as P
    P.load()
    specs, data_a = _planes(29, 6)
    rng = np.random.default_rng(30)
    data_b = []
    for s, (x, y, inp) in zip(specs, data_a):
        M = x.size
        xb, yb = synth.clustered_box(rng, M, s["N"] * s["g"])
        data_b.append((xb, yb, synth.unit_phase(rng, M if s["type"] == 1 else (s["N"], s["N"]))))
    print(f"new buffers: {len(specs)} planes", flush=True)

    def upload(data):
        return ([dev(torch, d[0]) for d in data], [dev(torch, d[1]) for d in data],
                [dev(torch, d[2]) for d in data])

    def plain(data):
        refs = []
        for s, (x, y, inp) in zip(specs, data):
            plan = P.Plan(**s)
            plan.set_points(dev(torch, x), dev(torch, y))
            refs.append(host(plan.execute(dev(torch, inp))))
        return refs

    def outs():
        return [torch.full((2 * s["N"], 2 * s["N"]) if s["type"] == 1 else (d[0].size,), float("nan"),
                           dtype=torch.complex64, device="cuda") for s, d in zip(specs, data_a)]

    A, B = upload(data_a), upload(data_b)
    ref_a, ref_b = plain(data_a), plain(data_b)
    b = P.Batch(specs)
    oa, ob = outs(), outs()
    b.run(*A, oa)
    assert b.debug_graphs() == (1, 0)
    b.run(*B, ob)
    assert b.debug_graphs() == (1, 1)
    oa2 = outs()
    b.run(*A, oa2)
    assert b.debug_graphs() == (1, 2)
    for p in range(len(specs)):
        check_close(host(oa[p]), ref_a[p], 1e-6, what=f"A plane {p}")
        check_close(host(ob[p]), ref_b[p], 1e-6, what=f"B plane {p}")
        check_close(host(oa2[p]), ref_a[p], 1e-6, what=f"A again plane {p}")
    # points bound once, operators on other buffers: the execute graph too
    b.set_points(A[0], A[1])
    r0, f0 = b.debug_graphs()
    e1, e2 = outs(), outs()
    b.execute(A[2], e1)
    b.execute(A[2], e2)
    assert b.debug_graphs() == (r0 + 1, f0 + 1)
    for p in range(len(specs)):
        check_close(host(e1[p]), ref_a[p], 1e-6, what=f"execute plane {p}")
        check_close(host(e2[p]), ref_a[p], 1e-6, what=f"execute, new outputs, plane {p}")
    # a changed point count records again
    xs, ys, ins = A
    xs2, ys2 = list(xs), list(ys)
    p1 = next(p for p, s in enumerate(specs) if s["type"] == 1)
    xs2[p1], ys2[p1] = xs[p1][:100].clone(), ys[p1][:100].clone()
    ins2 = list(ins)
    ins2[p1] = ins[p1][:100].clone()
    r0, f0 = b.debug_graphs()
    b.run(xs2, ys2, ins2, outs())
    assert b.debug_graphs() == (r0 + 1, f0)
    # the per-plane form records on every change
    b.set_grouped(False)
    r0, f0 = b.debug_graphs()
    b.run(*A, outs())
    b.run(*B, ob)
    assert b.debug_graphs() == (r0 + 2, f0)
    for p in range(len(specs)):
        check_close(host(ob[p]), ref_b[p], 1e-6, what=f"per-plane B plane {p}")
    b.close()
