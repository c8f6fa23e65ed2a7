"""The rest of the C-ABI boundary on the GPU: caller-owned workspaces
(nuasm_plan_workspace_bytes / nuasm_plan_set_workspace), batches in two steps
(nuasm_set_points_many / nuasm_execute_many: points bound once, operators run
many times), both spreading methods (register gather and matrix cores)
against the oracle, and bins split over several spreading workgroups."""
import sys

import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import check_close, dev, geometry, host, make_plan

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


def _ws(nbytes):
    # torch's caching allocator returns blocks aligned to at least 512 bytes
    t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
    assert t.data_ptr() % 256 == 0
    return t


# ------------------------------------------------------------ workspace
@pytest.mark.parametrize("t", [1, 2])
def test_workspace_plan_matches_plan_owned_memory_bitwise(P, t):
    """Deterministic mode makes every sum run in one order, so a plan whose
    buffers live in a caller's workspace must reproduce the plan-owned
    result bit for bit; then back to plan-owned memory (workspace = None)."""
    _say("workspace bitwise", t)
    N, M = 128, 30000
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.05, tf="asm", band="limited", ox=2e-4)
    rng = np.random.default_rng(71 + t)
    x, y = synth.clustered_box(rng, M, N * geo.g)
    inp = synth.unit_phase(rng, M if t == 1 else (N, N))
    xd, yd, ind = dev(torch, x), dev(torch, y), dev(torch, inp)
    own = make_plan(P, geo, t, deterministic=True)
    own.set_points(xd, yd)
    ref = host(own.execute(ind))
    p = make_plan(P, geo, t, deterministic=True)
    p.set_points(xd, yd)  # bound in plan-owned memory first
    nb = p.workspace_bytes(M)
    owned_before = p.info["device_bytes"]
    p.set_workspace(_ws(nb))
    assert p.info["device_bytes"] < owned_before  # the grids now live in the workspace
    with pytest.raises(P.NuasmError) as ei:
        p.execute(ind)
    assert ei.value.name == "NUASM_ERR_NOT_READY"  # points must be bound again
    p.set_points(xd, yd)
    got = host(p.execute(ind))
    assert np.array_equal(got, ref)
    check_close(got, O.nuasm1(geo, x, y, inp) if t == 1 else O.nuasm2(geo, inp, x, y), 1e-5)
    # back to plan-owned memory
    p.set_workspace(None)
    p.set_points(xd, yd)
    assert np.array_equal(host(p.execute(ind)), ref)


def test_workspace_capacity_and_errors(P):
    _say("workspace capacity")
    N = 64
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.02, tf="fresnel")
    p = make_plan(P, geo, 2)
    nb = p.workspace_bytes(5000)
    assert nb > p.workspace_bytes(0) > 0
    ws = _ws(nb + 512)
    # misaligned and too small workspaces are refused and change nothing
    lib = P.load()
    import ctypes
    st = lib.nuasm_plan_set_workspace(p._h, ctypes.c_void_p(ws.data_ptr() + 8), nb)
    assert lib.nuasm_status_string(st).decode() == "NUASM_ERR_INVALID_ARG"
    with pytest.raises(P.NuasmError) as ei:
        p.set_workspace(_ws(p.workspace_bytes(0) // 2))
    assert ei.value.name == "NUASM_ERR_INVALID_ARG"
    p.set_workspace(ws[:nb])
    rng = np.random.default_rng(5)
    u1 = dev(torch, synth.unit_phase(rng, (N, N)))
    for M in (5000, 1200, 0):
        x, y = synth.uniform_box(rng, M, N * geo.g)
        p.set_points(dev(torch, x), dev(torch, y))
        got = host(p.execute(u1))
        if M:
            check_close(got, O.nuasm2(geo, host(u1), x, y), 1e-5)
    # more points than the workspace holds
    x, y = synth.uniform_box(rng, 400000, N * geo.g)
    with pytest.raises(P.NuasmError) as ei:
        p.set_points(dev(torch, x), dev(torch, y))
    assert ei.value.name == "NUASM_ERR_INVALID_ARG"
    # a tuning whose buffers fit re-carves the workspace
    p.set_tuning(interp_chunk=1024)
    x, y = synth.uniform_box(rng, 3000, N * geo.g)
    p.set_points(dev(torch, x), dev(torch, y))
    check_close(host(p.execute(u1)), O.nuasm2(geo, host(u1), x, y), 1e-5)
    # a workspace at the minimum (1024 points) cannot take a tuning with more
    # partial tiles per point: refused, and the old tuning stays
    q = make_plan(P, geo, 1)
    q.set_workspace(_ws(q.workspace_bytes(0)))
    with pytest.raises(P.NuasmError) as ei:
        q.set_tuning(spread_chunk=896)
    assert ei.value.name == "NUASM_ERR_INVALID_ARG"
    assert q.info["spread_chunk"] == 1792
    x, y = synth.uniform_box(rng, 1024, N * geo.g)
    c = synth.unit_phase(rng, 1024)
    q.set_points(dev(torch, x), dev(torch, y))
    check_close(host(q.execute(dev(torch, c))), O.nuasm1(geo, x, y, c), 1e-5)


def test_workspace_type3(P):
    _say("workspace type 3")
    N = 64
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.01, tf="asm", band="limited")
    rng = np.random.default_rng(8)
    xs, ys = synth.clustered_box(rng, 4000, N * geo.g)
    xd, yd = synth.uniform_box(rng, 3000, N * geo.g)
    c = synth.unit_phase(rng, 4000)
    p = make_plan(P, geo, 3)
    p.set_workspace(_ws(p.workspace_bytes(4000)))
    p.set_points(dev(torch, xs), dev(torch, ys))
    p.set_dest_points(dev(torch, xd), dev(torch, yd))
    check_close(host(p.execute(dev(torch, c))), O.nuasm3(geo, xs, ys, c, xd, yd), 1e-5)


# ------------------------------------------------- batches in two steps
def test_set_points_many_then_execute_many(P):
    """Points bound once for every plane, the operators run with two different
    inputs (two recordings of the operator graph plus a replay), then the
    points of one plane change count (the operator graph is recorded again);
    every output equals a plain plan's."""
    _say("many")
    rng = np.random.default_rng(303)
    specs, pts, ins2 = [], [], []
    for p in range(6):
        N = [64, 128, 256][p % 3]
        t = 1 + p % 2
        tf = "asm" if p < 3 else "fresnel"
        M = int(rng.integers(2000, 30000))
        x, y = synth.clustered_box(rng, M, N * 4e-6)
        specs.append(dict(N=N, type=t, lam=633e-9, z=float(rng.uniform(0.01, 0.2)), g=4e-6, tf=tf,
                          band="limited" if tf == "asm" else "full", tol=1e-6))
        pts.append((dev(torch, x), dev(torch, y)))
        ins2.append([dev(torch, synth.unit_phase(rng, M if t == 1 else (N, N))) for _ in range(2)])
    b = P.Batch(specs)
    outs = [torch.empty((2 * s["N"], 2 * s["N"]) if s["type"] == 1 else (pts[i][0].numel(),),
                        dtype=torch.complex64, device="cuda") for i, s in enumerate(specs)]
    with pytest.raises(P.NuasmError) as ei:
        b.execute([i[0] for i in ins2], outs)
    assert ei.value.name == "NUASM_ERR_NOT_READY"
    b.set_points([q[0] for q in pts], [q[1] for q in pts])
    plans = []
    for s, (x, y) in zip(specs, pts):
        pl = P.Plan(**s)
        pl.set_points(x, y)
        plans.append(pl)
    for rep in (0, 1, 0):
        ins = [i[rep] for i in ins2]
        b.execute(ins, outs)
        assert b.check_points() == -1
        for p, pl in enumerate(plans):
            check_close(host(outs[p]), host(pl.execute(ins[p])), 1e-6, what=f"rep {rep} plane {p}")
    # rebind plane 0 with fewer points
    x, y = pts[0][0][:1000].clone(), pts[0][1][:1000].clone()
    pts[0] = (x, y)
    b.set_points([q[0] for q in pts], [q[1] for q in pts])
    plans[0].set_points(x, y)
    ins = [i[1] for i in ins2]
    ins[0] = ins[0][:1000].clone() if specs[0]["type"] == 1 else ins[0]
    if specs[0]["type"] == 2:
        outs[0] = torch.empty((1000,), dtype=torch.complex64, device="cuda")
    b.execute(ins, outs)
    for p, pl in enumerate(plans):
        check_close(host(outs[p]), host(pl.execute(ins[p])), 1e-6, what=f"rebound plane {p}")
    t = b.plane_times()
    assert len(t) == len(specs) and all(v > 0 for v in t)


# ---------------------------------------------------- spreading methods
@pytest.mark.parametrize("method", [1, 2], ids=["gather", "matrix"])
@pytest.mark.parametrize("tol", [1e-2, 1e-3, 1e-6, 1e-12])
def test_spreading_methods_match_oracle(P, method, tol):
    """Register gather and matrix-core spreading (w = 3, 4, 7, 13) against
    the oracle, through NU-ASM_1 and the NU-ASM_2 adjoint (which spreads)."""
    _say("spread method", method, tol)
    N, M = 128, 20000
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.08, tf="asm", band="limited", ox=5e-4)
    rng = np.random.default_rng(int(1000 * method + 17 * np.log10(1 / tol)))
    x, y = synth.three_clusters(rng, M, N * geo.g)
    c = synth.unit_phase(rng, M)
    bound = {1e-2: 2e-2, 1e-3: 2e-3, 1e-6: 1e-5, 1e-12: 2e-6}[tol]
    p = make_plan(P, geo, 1, tol=tol)
    p.set_tuning(spread_method=method)
    p.set_points(dev(torch, x), dev(torch, y))
    check_close(host(p.execute(dev(torch, c))), O.nuasm1(geo, x, y, c), bound)
    p2 = make_plan(P, geo, 2, tol=tol)
    p2.set_tuning(spread_method=method)
    p2.set_points(dev(torch, x), dev(torch, y))
    check_close(host(p2.adjoint(dev(torch, c))), O.nuasm2_adjoint(geo, c, x, y), bound)


@pytest.mark.parametrize("method", [1, 2], ids=["gather", "matrix"])
def test_spreading_methods_deterministic_bitwise(P, method):
    """Deterministic mode: repeated runs and a second plan agree bit for bit
    with either spreading method."""
    _say("deterministic method", method)
    N, M = 128, 40000
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.05, tf="fresnel", ox=1e-4)
    rng = np.random.default_rng(44)
    x, y = synth.clustered_box(rng, M, N * geo.g)
    c = dev(torch, synth.unit_phase(rng, M))
    outs = []
    for _ in range(2):
        p = make_plan(P, geo, 1, deterministic=True)
        p.set_tuning(spread_method=method)
        p.set_points(dev(torch, x), dev(torch, y))
        outs.append(host(p.execute(c)))
        outs.append(host(p.execute(c)))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    check_close(outs[0], O.nuasm1(geo, x, y, host(c)), 1e-5)


# ------------------------------------------------------- split bins
@pytest.mark.parametrize("method", [1, 2], ids=["gather", "matrix"])
@pytest.mark.parametrize("small", [False, True])
def test_spreading_split_bins(P, small, method):
    """20000 points in a few pixels: bins split over several chunks write
    partial tiles at their compact slots, summed by the reduction (slots
    counted exactly when set_points synchronises, bounded when deferred)."""
    _say("split bins", small, method)
    N, g = 64, 4e-6
    geo = geometry(N=N, g=g, lam=633e-9, z=0.01, tf="asm", band="limited", ox=1e-4)
    rng = np.random.default_rng(19)
    M = 20000
    x = rng.uniform(-3 * g, 3 * g, M)
    y = rng.uniform(-1 * g, 4 * g, M)
    x[:800] = rng.uniform(-N * g / 2, N * g / 2, 800)
    c = synth.unit_phase(rng, M)
    for defer in (False, True):
        p = make_plan(P, geo, 1, defer_range_check=defer)
        p.set_tuning(spread_chunk=896 if small else 0, spread_method=method)
        p.set_points(dev(torch, x), dev(torch, y))
        check_close(host(p.execute(dev(torch, c))), O.nuasm1(geo, x, y, c), 1e-5, what=f"defer={defer}")
        # the type-2 adjoint spreads too
        p2 = make_plan(P, geo, 2, defer_range_check=defer)
        p2.set_tuning(spread_chunk=896 if small else 0, spread_method=method)
        p2.set_points(dev(torch, x), dev(torch, y))
        check_close(host(p2.adjoint(dev(torch, c))), O.nuasm2_adjoint(geo, c, x, y), 1e-5, what=f"adj defer={defer}")
