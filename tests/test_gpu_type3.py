"""GPU parity of NU-ASM_3 / NU-FRE_3 (non-uniform source and destination
points, the combination of the first two operator types) and of its adjoint,
through the C ABI, against the FP64 oracle.

Bars as for the other operators: rel-L2 <= 1e-5 at kernel tolerance 1e-6
(the error of a spreading and an interpolation add), 2e-3 at 1e-3, 2e-2 at
1e-2, 2e-6 (float32 floor) at 1e-9 and 1e-12.  At the benchmark's size
(N' = 2048, 2^20 points on each side) the oracle evaluates 512 sampled
destinations of a source vector that is non-zero on 64 seeded points while
the library still binds, spreads and transforms all 2^20; the dot test of
the adjoint runs on dense inputs at that size.
"""
import sys

import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import check_close, dev, geometry, host, make_plan, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BOUND = {1e-2: 2e-2, 1e-3: 2e-3, 1e-6: 1e-5, 1e-9: 2e-6, 1e-12: 2e-6}


@pytest.fixture(scope="module")
def P():
    import paper_1308_6644_amd as P
    P.load()
    return P


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pts(kind, seed, M, N, g):
    rng = np.random.default_rng(seed)
    x, y = synth.make_points(kind, rng, M, N, g)
    return x, y, rng


CASES = [
    # (N, M source, source points, M destination, destination points, geometry, tol)
    (16, 1, "uniform", 1, "uniform", dict(g=4e-6, lam=633e-9, z=0.001, tf="asm", band="full"), 1e-6),
    (32, 300, "clustered", 257, "uniform", dict(g=4e-6, lam=633e-9, z=0.004, tf="fresnel", ox=2e-5), 1e-6),
    (64, 4000, "uniform", 3500, "clustered", dict(g=8e-6, lam=532e-9, z=0.05, tf="asm", band="full"), 1e-6),
    (64, 3001, "clustered", 2999, "three_clusters",
     dict(g=4e-6, lam=633e-9, z=0.01, tf="asm", band="limited", ox=1e-4), 1e-6),
    (128, 20011, "clustered", 15000, "uniform",
     dict(g=4e-6, lam=633e-9, z=0.1, tf="asm", band="limited", ox=1e-3), 1e-6),
    (128, 7000, "uniform", 9000, "clustered",
     dict(g=4e-6, lam=532e-9, z=-0.03, tf="asm", band="limited", oy=3e-4), 1e-6),
    (256, 30000, "clustered", 20000, "clustered",
     dict(g=4e-6, lam=633e-9, z=0.02, tf="asm", band="explicit", band_c=(12.0, -7.5), band_w=(300.0, 211.0)),
     1e-6),
    (64, 2000, "uniform", 2100, "uniform", dict(g=4e-6, lam=633e-9, z=0.01, tf="asm", band="full"), 1e-3),
    (64, 3000, "clustered", 2500, "uniform", dict(g=4e-6, lam=633e-9, z=0.01, tf="asm", band="full"), 1e-2),
    (64, 3000, "clustered", 2500, "clustered",
     dict(g=4e-6, lam=633e-9, z=0.01, tf="fresnel", ox=1e-5), 1e-12),
    (64, 2000, "three_clusters", 2000, "uniform",
     dict(g=4e-6, lam=633e-9, z=0.01, tf="asm", band="full"), 1e-9),
]


def _id(c):
    N, M1, k1, M2, k2, kw, tol = c
    return f"N{N}-{k1}{M1}-{k2}{M2}-{kw['tf']}-{kw.get('band', '-')}-z{kw['z']}-tol{tol:g}"


@pytest.mark.parametrize("case", CASES, ids=_id)
def test_nuasm3_matches_oracle(P, case):
    N, M1, k1, M2, k2, kw, tol = case
    _say("nuasm3", _id(case))
    geo = geometry(N=N, **kw)
    x1, y1, rng = _pts(k1, 300 + N + M1, M1, N, geo.g)
    x2, y2, _ = _pts(k2, 400 + N + M2, M2, N, geo.g)
    c = synth.unit_phase(rng, M1)
    plan = make_plan(P, geo, 3, tol=tol)
    plan.set_points(dev(torch, x1), dev(torch, y1))
    plan.set_dest_points(dev(torch, x2), dev(torch, y2))
    got = host(plan.execute(dev(torch, c)))
    assert got.shape == (M2,)
    ref = O.nuasm3(geo, x1, y1, c, x2, y2)
    check_close(got, ref, BOUND[tol])


@pytest.mark.parametrize("tf,band,z", [("asm", "limited", 0.02), ("fresnel", "full", 0.03)])
def test_nuasm3_adjoint_matches_oracle_and_dot_test(P, tf, band, z):
    N, M1, M2 = 64, 2500, 1900
    _say("nuasm3 adjoint", tf, band, z)
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=z, tf=tf, band=band, ox=1e-4)
    x1, y1, rng = _pts("clustered", 81, M1, N, geo.g)
    x2, y2, _ = _pts("uniform", 82, M2, N, geo.g)
    plan = make_plan(P, geo, 3)
    plan.set_points(dev(torch, x1), dev(torch, y1))
    plan.set_dest_points(dev(torch, x2), dev(torch, y2))
    c = synth.unit_phase(rng, M1)
    w = synth.unit_phase(rng, M2)
    a = host(plan.adjoint(dev(torch, w)))
    assert a.shape == (M1,)
    check_close(a, O.nuasm3_adjoint(geo, w, x1, y1, x2, y2), 1e-5)
    f = host(plan.execute(dev(torch, c)))
    lhs, rhs = np.vdot(w, f), np.vdot(a, c.astype(np.complex128))
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(w) * np.linalg.norm(f)


def test_nuasm3_rebinding_one_side_and_shared_points(P):
    """Each point set has its own buffers: rebinding the destination leaves the
    source binning intact, and one set may serve as both."""
    N = 64
    _say("nuasm3 rebinding")
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.02, tf="asm", band="limited", ox=-1e-4)
    x1, y1, rng = _pts("clustered", 91, 4000, N, geo.g)
    xa, ya, _ = _pts("uniform", 92, 3000, N, geo.g)
    xb, yb, _ = _pts("three_clusters", 93, 5000, N, geo.g)
    c = synth.unit_phase(rng, 4000)
    plan = make_plan(P, geo, 3)
    plan.set_points(dev(torch, x1), dev(torch, y1))
    plan.set_dest_points(dev(torch, xa), dev(torch, ya))
    ca = dev(torch, c)
    check_close(host(plan.execute(ca)), O.nuasm3(geo, x1, y1, c, xa, ya), 1e-5)
    plan.set_dest_points(dev(torch, xb), dev(torch, yb))   # larger: buffers grow
    check_close(host(plan.execute(ca)), O.nuasm3(geo, x1, y1, c, xb, yb), 1e-5)
    plan.set_dest_points(dev(torch, x1), dev(torch, y1))   # the source set as destination
    check_close(host(plan.execute(ca)), O.nuasm3(geo, x1, y1, c, x1, y1), 1e-5)


def test_nuasm3_empty_sets_errors_and_autograd(P):
    N = 32
    _say("nuasm3 edge cases")
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.01, tf="fresnel", ox=2e-5)
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    x1, y1, rng = _pts("uniform", 95, 600, N, geo.g)
    x2, y2, _ = _pts("clustered", 96, 500, N, geo.g)
    plan = make_plan(P, geo, 3)
    with pytest.raises(P.NuasmError) as ei:
        plan.execute(torch.zeros(0, dtype=torch.complex64, device="cuda"))
    assert ei.value.name == "NUASM_ERR_NOT_READY"
    plan.set_points(dev(torch, x1), dev(torch, y1))
    with pytest.raises(P.NuasmError) as ei:   # destination not bound yet
        plan.execute(torch.zeros(600, dtype=torch.complex64, device="cuda"))
    assert ei.value.name == "NUASM_ERR_NOT_READY"
    # no destinations: empty output; no sources: zeros
    plan.set_dest_points(e, e)
    assert plan.execute(dev(torch, synth.unit_phase(rng, 600))).shape == (0,)
    plan.set_dest_points(dev(torch, x2), dev(torch, y2))
    plan.set_points(e, e)
    out = plan.execute(torch.empty(0, dtype=torch.complex64, device="cuda"))
    assert out.shape == (500,) and float(out.abs().max()) == 0.0
    # out-of-range destination is reported and leaves the plan not ready
    h = N * geo.g / 2
    bad = torch.tensor([0.0, 1.5 * h], dtype=torch.float64, device="cuda")
    with pytest.raises(P.NuasmError) as ei:
        plan.set_dest_points(bad, torch.zeros(2, dtype=torch.float64, device="cuda"))
    assert ei.value.name == "NUASM_ERR_OUT_OF_RANGE"
    with pytest.raises(P.NuasmError) as ei:
        plan.execute(torch.empty(0, dtype=torch.complex64, device="cuda"))
    assert ei.value.name == "NUASM_ERR_NOT_READY"
    # destination points belong to type-3 plans only
    p1 = make_plan(P, geo, 1)
    with pytest.raises(P.NuasmError) as ei:
        p1.set_dest_points(dev(torch, x2), dev(torch, y2))
    assert ei.value.name == "NUASM_ERR_INVALID_ARG"
    # autograd: torch's gradient of a real loss is 2 A^H (A c - v)
    plan.set_points(dev(torch, x1), dev(torch, y1))
    plan.set_dest_points(dev(torch, x2), dev(torch, y2))
    c = synth.unit_phase(rng, 600)
    v = synth.unit_phase(rng, 500)
    ct = dev(torch, c).requires_grad_(True)
    loss = torch.sum(torch.abs(P.nuasm3(ct, plan) - dev(torch, v)) ** 2)
    loss.backward()
    ref = 2.0 * O.nuasm3_adjoint(geo, O.nuasm3(geo, x1, y1, c, x2, y2) - v, x1, y1, x2, y2)
    check_close(host(ct.grad), ref, 1e-5)


def test_nuasm3_stage_timing(P):
    N, M1, M2 = 64, 5000, 4000
    _say("nuasm3 stage timing")
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.01, tf="asm", band="limited", ox=1e-4)
    x1, y1, rng = _pts("clustered", 97, M1, N, geo.g)
    x2, y2, _ = _pts("uniform", 98, M2, N, geo.g)
    plan = make_plan(P, geo, 3)
    plan.set_timing(True)
    plan.set_points(dev(torch, x1), dev(torch, y1))
    plan.set_dest_points(dev(torch, x2), dev(torch, y2))
    c = dev(torch, synth.unit_phase(rng, M1))
    plan.execute(c)
    got = plan.read_timing()
    expect = dict(bin_hist=2, bin_colscan=2, bin_scatter=2, spread=1, spread_reduce=1, t1_rows=1, t3_cols=1,
                  t2_rows_inv=1, interp=1, t1_cols=0, t1_rows_inv=0, t2_rows=0, t2_cols=0, bin_scan=2)
    for st, n in expect.items():
        assert got[st][1] == n, (st, got[st])


# --------------------------------------------------- benchmark-sized case
NF, GF, LAMF, OXF, MF = 1024, 4e-6, 633e-9, 1e-3, 1 << 20


@pytest.mark.parametrize("z,tf", [(0.1, "asm"), (0.5, "fresnel")])
def test_fullsize_nuasm3_sampled_destinations(P, z, tf):
    """N' = 2048, 2^20 clustered sources and 2^20 clustered destinations,
    o = (1 mm, 0), tolerance 1e-6, deferred range check: the whole path runs
    on every point; the source vector is non-zero on 64 seeded points so that
    the oracle's type-1 sum over them and its type-2 sums at 512 sampled
    destinations finish in seconds."""
    _say("nuasm3 full size", z, tf)
    W = NF * GF
    r1 = synth.rng_for(2, 0)
    x1, y1 = synth.clustered_box(r1, MF, W)
    r2 = synth.rng_for(2, 1)
    x2, y2 = synth.clustered_box(r2, MF, W)
    rs = np.random.default_rng(3030)
    src = rs.choice(MF, size=64, replace=False)
    sel = rs.choice(MF, size=512, replace=False)
    c = np.zeros(MF, dtype=np.complex64)
    c[src] = synth.unit_phase(rs, 64)
    band = "limited" if tf == "asm" else "full"
    geo = O.Geometry(N=NF, g=GF, lam=LAMF, z=z, ox=OXF, tf=tf, band=band)
    plan = P.Plan(NF, 3, LAMF, z, GF, tf=tf, band=band, ox=OXF, tol=1e-6, defer_range_check=True)
    plan.set_points(dev(torch, x1), dev(torch, y1))
    plan.set_dest_points(dev(torch, x2), dev(torch, y2))
    plan.check_points()
    got = host(plan.execute(dev(torch, c)))[sel]
    ref = O.nuasm3(geo, x1[src], y1[src], c[src], x2[sel], y2[sel])
    err = check_close(got, ref, 1e-5)
    _say(f"  sampled rel-L2 {err:.3e}")
    # dense inputs at the same size: the adjoint is the transpose-conjugate
    rd = np.random.default_rng(3031)
    cd = dev(torch, synth.unit_phase(rd, MF))
    wd = dev(torch, synth.unit_phase(rd, MF))
    f = plan.execute(cd).to(torch.complex128)
    a = plan.adjoint(wd).to(torch.complex128)
    lhs = complex(torch.vdot(wd.to(torch.complex128), f))
    rhs = complex(torch.vdot(a, cd.to(torch.complex128)))
    scale = float(torch.linalg.vector_norm(wd.to(torch.complex128)) * torch.linalg.vector_norm(f))
    _say(f"  dot test |lhs - rhs| / (|w||Ac|) = {abs(lhs - rhs) / scale:.3e}")
    assert abs(lhs - rhs) <= 1e-5 * scale
