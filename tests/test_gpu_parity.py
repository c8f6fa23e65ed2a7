"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Bars: rel-L2 <= 1e-5 at kernel tolerance 1e-6 (the stated accuracy target of
the path); for other tolerances the bound follows the kernel's accuracy
(w = 4: 2e-3, w = 10: float32 floor 2e-6).  Inputs are seeded; every case
prints its name, seed and shape before touching the GPU.
"""
import sys

import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import check_close, dev, geometry, host, make_plan, rel_l2, type1_spectral_samples

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


BOUND = {1e-2: 2e-2, 1e-3: 2e-3, 1e-6: 1e-5, 1e-9: 2e-6, 1e-12: 2e-6}


# ---------------------------------------------------------------- FFT
@pytest.mark.parametrize("logn", list(range(5, 15)))
@pytest.mark.parametrize("sign", [-1, 1])
def test_stockham_fft_matches_numpy(P, logn, sign):
    n = 1 << logn
    _say(f"fft n={n} sign={sign}")
    rng = np.random.default_rng(logn)
    x = (rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))).astype(np.complex64)
    got = host(P.debug_fft(dev(torch, x), sign))
    xd = x.astype(np.complex128)
    ref = np.fft.fft(xd, axis=-1) if sign < 0 else np.fft.ifft(xd, axis=-1) * n
    # float32 Stockham: error grows like eps32 * sqrt(log2 n)
    check_close(got, ref, 2e-6)


# ---------------------------------------------------- transfer function
TRANSFER_CASES = [
    dict(N=64, g=8e-6, lam=532e-9, z=0.05, tf="asm", band="full"),
    dict(N=256, g=4e-6, lam=633e-9, z=0.01, tf="asm", band="limited", ox=1e-3),
    dict(N=256, g=4e-6, lam=633e-9, z=0.1, tf="asm", band="limited", ox=1e-3),
    dict(N=256, g=4e-6, lam=633e-9, z=0.5, tf="asm", band="limited", ox=1e-3, oy=-2e-4),
    dict(N=1024, g=4e-6, lam=532e-9, z=1.0, tf="asm", band="limited"),
    dict(N=128, g=4e-6, lam=633e-9, z=-0.02, tf="asm", band="limited", ox=2e-4),
    dict(N=128, g=4e-6, lam=633e-9, z=0.02, tf="asm", band="explicit", band_c=(10.5, -3.0), band_w=(40.0, 61.0)),
    dict(N=128, g=4e-6, lam=633e-9, z=0.05, tf="fresnel", ox=1e-4, oy=-3e-5),
    dict(N=256, g=4e-6, lam=633e-9, z=0.5, tf="fresnel", ox=1e-3),
]


@pytest.mark.parametrize("case", TRANSFER_CASES, ids=lambda c: f"{c['tf']}-{c.get('band','-')}-N{c['N']}-z{c['z']}")
def test_transfer_function_matches_oracle(P, case):
    _say("transfer", case)
    geo = geometry(**case)
    plan = make_plan(P, geo, 1)
    got = host(plan.transfer())
    ref = O.transfer(geo)
    scale = np.max(np.abs(ref))
    # float32 sincospi of a phase reduced in float64 (ASM) or float32 products
    # of float64 axis tables (Fresnel): a few float32 ulps of |H|
    assert np.max(np.abs(got - ref)) <= 2e-6 * scale
    assert np.array_equal(np.abs(ref) == 0, np.abs(got) == 0)


# ------------------------------------------------------------- operators
def _points(kind, seed, M, N, g):
    rng = np.random.default_rng(seed)
    x, y = synth.make_points(kind, rng, M, N, g)
    return x, y, rng


OP_CASES = [
    # (N, M, points, geometry kwargs, tol)
    (64, 4096, "uniform", dict(g=8e-6, lam=532e-9, z=0.05, tf="asm", band="full"), 1e-6),
    (16, 1, "uniform", dict(g=4e-6, lam=633e-9, z=0.001, tf="asm", band="full"), 1e-6),
    (16, 37, "clustered", dict(g=4e-6, lam=633e-9, z=0.002, tf="fresnel", ox=2e-5), 1e-6),
    (64, 3001, "clustered", dict(g=4e-6, lam=633e-9, z=0.01, tf="asm", band="limited", ox=1e-4), 1e-6),
    (128, 20011, "clustered", dict(g=4e-6, lam=633e-9, z=0.1, tf="asm", band="limited", ox=1e-3), 1e-6),
    (128, 5000, "three_clusters", dict(g=4e-6, lam=633e-9, z=0.05, tf="fresnel", ox=1e-4, oy=-1e-4), 1e-6),
    (128, 7000, "uniform", dict(g=4e-6, lam=532e-9, z=-0.03, tf="asm", band="limited", oy=3e-4), 1e-6),
    (64, 2000, "uniform", dict(g=4e-6, lam=633e-9, z=0.01, tf="asm", band="full"), 1e-3),
    (64, 2000, "clustered", dict(g=4e-6, lam=633e-9, z=0.01, tf="asm", band="full"), 1e-9),
    (256, 30000, "clustered", dict(g=4e-6, lam=633e-9, z=0.02, tf="asm", band="explicit",
                                   band_c=(12.0, -7.5), band_w=(300.0, 211.0)), 1e-6),
    # the narrowest and the widest kernels the tolerance range allows (w = 3 and w = 13)
    (64, 3000, "clustered", dict(g=4e-6, lam=633e-9, z=0.01, tf="asm", band="full"), 1e-2),
    (64, 3000, "clustered", dict(g=4e-6, lam=633e-9, z=0.01, tf="fresnel", ox=1e-5), 1e-12),
    # back-propagation with the Fresnel transfer function and a 2-D offset
    (128, 6000, "three_clusters", dict(g=4e-6, lam=532e-9, z=-0.04, tf="fresnel", ox=-2e-4, oy=1.5e-4), 1e-6),
    # a narrow explicit band off the centre (the band-adaptive grid shrinks N'')
    (128, 8000, "uniform", dict(g=4e-6, lam=633e-9, z=0.03, tf="asm", band="explicit",
                                band_c=(-20.0, 9.0), band_w=(40.0, 26.0)), 1e-6),
]


def _id(c):
    N, M, kind, kw, tol = c
    return f"N{N}-M{M}-{kind}-{kw['tf']}-{kw.get('band','-')}-z{kw['z']}-tol{tol:g}"


@pytest.mark.parametrize("case", OP_CASES, ids=_id)
def test_nuasm1_matches_oracle(P, case):
    N, M, kind, kw, tol = case
    _say("nuasm1", _id(case))
    geo = geometry(N=N, **kw)
    x, y, rng = _points(kind, 100 + N + M, M, N, geo.g)
    c = synth.unit_phase(rng, M)
    plan = make_plan(P, geo, 1, tol=tol)
    plan.set_points(dev(torch, x), dev(torch, y))
    got = host(plan.execute(dev(torch, c)))
    ref = O.nuasm1(geo, x, y, c)
    check_close(got, ref, BOUND[tol])


@pytest.mark.parametrize("case", OP_CASES, ids=_id)
def test_nuasm2_matches_oracle(P, case):
    N, M, kind, kw, tol = case
    _say("nuasm2", _id(case))
    geo = geometry(N=N, **kw)
    x, y, rng = _points(kind, 200 + N + M, M, N, geo.g)
    u1 = synth.unit_phase(rng, (N, N))
    plan = make_plan(P, geo, 2, tol=tol)
    plan.set_points(dev(torch, x), dev(torch, y))
    got = host(plan.execute(dev(torch, u1)))
    ref = O.nuasm2(geo, u1, x, y)
    check_close(got, ref, BOUND[tol])


def test_tiny_nuasm1_N64_M4096(P):
    """N = 64 (N' = 128), M = 4096 uniform, pitch 8 um, 532 nm, z = 0.05 m,
    full band, tolerance 1e-6: the whole 128 x 128 output vs the oracle."""
    cfg = synth.WORKLOADS["nuasm1_tiny_N64_M4096"]
    _say("tiny", cfg)
    geo = geometry(N=cfg["N"], g=cfg["g"], lam=cfg["lam"], z=cfg["z"], tf="asm", band="full")
    rng = synth.rng_for(cfg["seed"])
    x, y = synth.uniform_box(rng, cfg["M"], cfg["N"] * cfg["g"])
    c = synth.unit_phase(rng, cfg["M"])
    plan = make_plan(P, geo, 1, tol=cfg["tol"])
    plan.set_points(dev(torch, x), dev(torch, y))
    got = host(plan.execute(dev(torch, c)))
    assert got.shape == (128, 128)
    check_close(got, O.nuasm1(geo, x, y, c), 1e-5)


# --------------------------------------------------------------- adjoints
@pytest.mark.parametrize("tf,band,z", [("asm", "limited", 0.02), ("fresnel", "full", 0.03)])
def test_adjoints_match_oracle_and_dot_test(P, tf, band, z):
    N, M = 64, 2500
    _say("adjoint", tf, band, z)
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=z, tf=tf, band=band, ox=1e-4)
    x, y, rng = _points("clustered", 77, M, N, geo.g)
    p1 = make_plan(P, geo, 1)
    p2 = make_plan(P, geo, 2)
    xd, yd = dev(torch, x), dev(torch, y)
    p1.set_points(xd, yd)
    p2.set_points(xd, yd)
    v = synth.unit_phase(rng, (2 * N, 2 * N))
    w = synth.unit_phase(rng, M)
    c = synth.unit_phase(rng, M)
    u1 = synth.unit_phase(rng, (N, N))
    a1 = host(p1.adjoint(dev(torch, v)))
    a2 = host(p2.adjoint(dev(torch, w)))
    check_close(a1, O.nuasm1_adjoint(geo, v, x, y), 1e-5)
    check_close(a2, O.nuasm2_adjoint(geo, w, x, y), 1e-5)
    f1 = host(p1.execute(dev(torch, c)))
    f2 = host(p2.execute(dev(torch, u1)))
    lhs, rhs = np.vdot(v, f1), np.vdot(a1, c.astype(np.complex128))
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(v) * np.linalg.norm(f1)
    lhs, rhs = np.vdot(w, f2), np.vdot(a2, u1.astype(np.complex128))
    assert abs(lhs - rhs) <= 1e-5 * np.linalg.norm(w) * np.linalg.norm(f2)


# ------------------------------------------------------------- edge cases
@pytest.mark.parametrize("det", [False, True], ids=["default", "deterministic"])
def test_empty_point_set(P, det):
    _say("empty", det)
    geo = geometry(N=32, g=4e-6, lam=633e-9, z=0.01, tf="asm", band="limited")
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    p1 = make_plan(P, geo, 1, deterministic=det)
    p1.set_points(e, e)
    out = p1.execute(torch.empty(0, dtype=torch.complex64, device="cuda"))
    assert out.shape == (64, 64) and float(out.abs().max()) == 0.0
    p2 = make_plan(P, geo, 2, deterministic=det)
    p2.set_points(e, e)
    out2 = p2.execute(torch.ones((32, 32), dtype=torch.complex64, device="cuda"))
    assert out2.shape == (0,)


@pytest.mark.parametrize("det", [False, True], ids=["default", "deterministic"])
def test_points_on_window_edges(P, det):
    _say("edges", det)
    N, g = 32, 4e-6
    geo = geometry(N=N, g=g, lam=633e-9, z=0.01, tf="asm", band="full")
    h = N * g / 2
    x = np.array([-h, h, -h, h, 0.0, h, -h, 0.3 * h])
    y = np.array([-h, -h, h, h, h, 0.0, 0.1 * h, -h])
    rng = np.random.default_rng(5)
    c = synth.unit_phase(rng, x.size)
    for tol in (1e-6, 1e-9):
        p1 = make_plan(P, geo, 1, tol=tol, deterministic=det)
        p1.set_points(dev(torch, x), dev(torch, y))
        check_close(host(p1.execute(dev(torch, c))), O.nuasm1(geo, x, y, c), 1e-5)
        u1 = synth.unit_phase(rng, (N, N))
        p2 = make_plan(P, geo, 2, tol=tol, deterministic=det)
        p2.set_points(dev(torch, x), dev(torch, y))
        check_close(host(p2.execute(dev(torch, u1))), O.nuasm2(geo, u1, x, y), 1e-5)


@pytest.mark.parametrize("det", [False, True], ids=["default", "deterministic"])
def test_out_of_range_and_not_ready(P, det):
    _say("errors", det)
    geo = geometry(N=32, g=4e-6, lam=633e-9, z=0.01)
    p = make_plan(P, geo, 1, deterministic=det)
    with pytest.raises(P.NuasmError) as ei:
        p.execute(torch.zeros(0, dtype=torch.complex64, device="cuda"))
    assert ei.value.name == "NUASM_ERR_NOT_READY"
    h = 32 * 4e-6 / 2
    x = torch.tensor([0.0, 1.01 * h, 0.0], dtype=torch.float64, device="cuda")
    y = torch.tensor([0.0, 0.0, float("nan")], dtype=torch.float64, device="cuda")
    with pytest.raises(P.NuasmError) as ei:
        p.set_points(x, y)
    assert ei.value.name == "NUASM_ERR_OUT_OF_RANGE"
    with pytest.raises(P.NuasmError) as ei:
        p.execute(torch.zeros(0, dtype=torch.complex64, device="cuda"))
    assert ei.value.name == "NUASM_ERR_NOT_READY"
    pd = make_plan(P, geo, 1, defer_range_check=True, deterministic=det)
    pd.set_points(x, y)
    with pytest.raises(P.NuasmError):
        pd.check_points()


def test_dense_bin_multi_chunk(P):
    """5000 points inside a few pixels: the bins there hold more records than
    one workgroup takes, exercising the chunk split and its reduction."""
    _say("dense")
    N, g = 64, 4e-6
    geo = geometry(N=N, g=g, lam=633e-9, z=0.01, tf="asm", band="limited", ox=1e-4)
    rng = np.random.default_rng(9)
    M = 6000
    x = rng.uniform(-2 * g, 2 * g, M)
    y = rng.uniform(3 * g, 6 * g, M)
    x[:500] = rng.uniform(-N * g / 2, N * g / 2, 500)
    c = synth.unit_phase(rng, M)
    p1 = make_plan(P, geo, 1)
    p1.set_points(dev(torch, x), dev(torch, y))
    check_close(host(p1.execute(dev(torch, c))), O.nuasm1(geo, x, y, c), 1e-5)
    u1 = synth.unit_phase(rng, (N, N))
    p2 = make_plan(P, geo, 2)
    p2.set_points(dev(torch, x), dev(torch, y))
    check_close(host(p2.execute(dev(torch, u1))), O.nuasm2(geo, u1, x, y), 1e-5)
    w = synth.unit_phase(rng, M)
    check_close(host(p2.adjoint(dev(torch, w))), O.nuasm2_adjoint(geo, w, x, y), 1e-5)


def test_crop_output(P):
    _say("crop")
    N = 32
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.004, tf="fresnel")
    x, y, rng = _points("uniform", 3, 500, N, geo.g)
    c = synth.unit_phase(rng, 500)
    p = make_plan(P, geo, 1, crop=True)
    p.set_points(dev(torch, x), dev(torch, y))
    got = host(p.execute(dev(torch, c)))
    ref = O.nuasm1(geo, x, y, c)[N // 2:3 * N // 2, N // 2:3 * N // 2]
    assert got.shape == (N, N)
    check_close(got, ref, 1e-5)


def test_repeated_execute_is_stable(P):
    """The counting sorts rank records with LDS atomics, so the order in
    which a cell's contributions are summed may change between runs;
    repeated runs must agree to float32 rounding."""
    _say("repeat")
    geo = geometry(N=128, g=4e-6, lam=633e-9, z=0.05, tf="asm", band="limited")
    x, y, rng = _points("clustered", 4, 50000, 128, geo.g)
    c = dev(torch, synth.unit_phase(rng, 50000))
    p = make_plan(P, geo, 1)
    p.set_points(dev(torch, x), dev(torch, y))
    a = host(p.execute(c))
    for _ in range(5):
        check_close(host(p.execute(c)), a, 1e-6)



def test_stream_change_orders_after_previous_work(P):
    """Points bound on one stream, the operator run on another with no host
    synchronisation in between: the plan orders the new stream after the
    old one, so the result is the oracle's."""
    _say("stream handoff")
    geo = geometry(N=128, g=4e-6, lam=633e-9, z=0.05, tf="asm", band="limited")
    x, y, rng = _points("clustered", 6, 200000, 128, geo.g)
    xs, ys = dev(torch, x), dev(torch, y)
    sub = 4000
    c = synth.unit_phase(rng, 200000)
    c[sub:] = 0
    ref = O.nuasm1(geo, x[:sub], y[:sub], c[:sub])
    cd = dev(torch, c)
    p = make_plan(P, geo, 1, defer_range_check=True)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        p.set_points(xs, ys)
    with torch.cuda.stream(s2):
        out = p.execute(cd)
        got = out.cpu()
    torch.cuda.synchronize()
    check_close(got.numpy(), ref, 1e-5)

def test_stage_timing_counts_every_kernel(P):
    """Stage timing records one (start, end) pair per launch on the plan's
    stream, accumulates until read, and records nothing once switched off."""
    _say("stage timing")
    N, M = 64, 5000
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.01, tf="asm", band="limited", ox=1e-4)
    x, y, rng = _points("clustered", 7, M, N, geo.g)
    for t, inp in ((1, synth.unit_phase(rng, M)), (2, synth.unit_phase(rng, (N, N)))):
        plan = make_plan(P, geo, t)
        plan.set_timing(True)
        plan.set_points(dev(torch, x), dev(torch, y))
        plan.execute(dev(torch, inp))
        plan.execute(dev(torch, inp))
        got = plan.read_timing()
        expect = {"bin_hist": 1, "bin_colscan": 1, "bin_scan": 1, "bin_scatter": 1}
        if t == 1:
            expect.update(spread=2, t1_rows=2, t1_cols=2, t1_rows_inv=2)
        else:
            expect.update(t2_rows=2, t2_cols=2, t2_rows_inv=2, interp=2)
        for st, n in expect.items():
            ms, launches = got[st]
            assert launches == n, (st, got[st])
            assert ms > 0.0
        again = plan.read_timing()
        assert all(n == 0 for _, n in again.values())  # reading clears
        plan.set_timing(False)
        plan.execute(dev(torch, inp))
        assert all(n == 0 for _, n in plan.read_timing().values())
