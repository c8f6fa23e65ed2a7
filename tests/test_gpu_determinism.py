"""Binning as a permutation, and the deterministic mode (NUASM_DETERMINISTIC).

* The bin records are exactly the (point, bin) pairs of every point's w x w
  footprint, with first-tap offsets and kernel offsets as the binning rule
  defines them, whatever the mode (checked against a numpy restatement of that
  rule from the coordinates).
* In deterministic mode every bin's records are in point order and spreading
  ranks its sub-batches stably, so repeated bindings and executions, other
  plans and batches give bitwise-identical results, still the oracle's to the
  operator bar, however dense the bins.
"""
import sys

import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import check_close, dev, geometry, host, make_plan, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TILE = 32


@pytest.fixture(scope="module")
def P():
    import paper_1308_6644_amd as P
    P.load()
    return P


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def expected_records(x, y, info, g):
    """(idx, bin, lx, ly, primary, dx, dy) of every (point, bin) pair, from the
    binning rule: fine coordinate tau = 2 x Npf / (Np g) + Npf/2 + 8 (window
    edges clamped to +-Npf/4 raster pixels), first tap ceil(tau - w/2), bins of
    32 fine cells that the taps first .. first + w - 1 reach."""
    Npf, Np, w, L = info["Npf"], info["Np"], info["w"], info["L"]
    TX = (L + TILE - 1) // TILE
    inv_g = Npf / (Np * g)
    half = 0.25 * Npf
    tau0 = Npf / 2 + 8
    out = []
    for j in range(x.size):
        xp = min(max(x[j] * inv_g, -half), half)
        yp = min(max(y[j] * inv_g, -half), half)
        tx, ty = 2.0 * xp + tau0, 2.0 * yp + tau0
        fx, fy = np.ceil(tx - 0.5 * w), np.ceil(ty - 0.5 * w)
        i0x, i0y = int(fx), int(fy)
        bx0, by0 = i0x // TILE, i0y // TILE
        for by in range(by0, (i0y + w - 1) // TILE + 1):
            for bx in range(bx0, (i0x + w - 1) // TILE + 1):
                out.append((j, by * TX + bx, i0x - bx * TILE, i0y - by * TILE, bx == bx0 and by == by0,
                            fx - tx, fy - ty))
    return out


def decode(recs, counts):
    r = recs.cpu().numpy()
    packed = r[:, 0]
    lx = ((packed & 0xFF) ^ 0x80) - 0x80
    ly = (((packed >> 8) & 0xFF) ^ 0x80) - 0x80
    prim = (packed >> 16) & 1
    dx = r[:, 1].view(np.float32)
    dy = r[:, 2].view(np.float32)
    idx = r[:, 3]
    c = counts.cpu().numpy()
    bins = np.repeat(np.arange(c.size), c)
    return idx, bins, lx, ly, prim, dx, dy, c


@pytest.mark.parametrize("deterministic", [False, True])
def test_records_are_the_footprint_pairs(P, deterministic):
    N, M = 32, 3000
    _say("records", deterministic)
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.01, tf="asm", band="full")
    rng = np.random.default_rng(41)
    x, y = synth.clustered_box(rng, M, N * geo.g, frac=0.8, sigma_frac=0.05)
    plan = make_plan(P, geo, 1, deterministic=deterministic)
    plan.set_points(dev(torch, x), dev(torch, y))
    recs, counts = plan.debug_records()
    idx, bins, lx, ly, prim, dx, dy, c = decode(recs, counts)
    assert c.sum() == idx.size
    exp = expected_records(x, y, plan.info, geo.g)
    assert idx.size == len(exp)
    got = sorted(zip(idx.tolist(), bins.tolist(), lx.tolist(), ly.tolist(), prim.tolist()))
    want = sorted((e[0], e[1], e[2], e[3], int(e[4])) for e in exp)
    assert got == want
    # kernel offsets: float32 of the float64 offset of the first tap
    ed = {(e[0], e[1]): (e[5], e[6]) for e in exp}
    d = np.array([ed[(int(i), int(b))] for i, b in zip(idx, bins)])
    assert np.max(np.abs(dx - d[:, 0])) <= 1e-6 and np.max(np.abs(dy - d[:, 1])) <= 1e-6
    if deterministic:
        for b in np.unique(bins):
            assert np.all(np.diff(idx[bins == b]) > 0), f"bin {b} not in point order"


def _run(P, geo, t, x, y, inp, **kw):
    plan = make_plan(P, geo, t, **kw)
    plan.set_points(dev(torch, x), dev(torch, y))
    return plan, plan.execute(dev(torch, inp))


@pytest.mark.parametrize("t", [1, 2])
def test_deterministic_runs_are_bitwise_equal(P, t):
    N, M = 128, 60000
    _say("bitwise", t)
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.05, tf="asm", band="limited", ox=2e-4)
    rng = np.random.default_rng(43)
    x, y = synth.clustered_box(rng, M, N * geo.g)
    inp = synth.unit_phase(rng, M if t == 1 else (N, N))
    plan, a = _run(P, geo, t, x, y, inp, deterministic=True)
    xs, ys, di = dev(torch, x), dev(torch, y), dev(torch, inp)
    for _ in range(3):
        plan.set_points(xs, ys)
        assert torch.equal(plan.execute(di), a)
    _, b = _run(P, geo, t, x, y, inp, deterministic=True)
    assert torch.equal(a, b)
    _, c = _run(P, geo, t, x, y, inp)
    check_close(host(a), host(c), 1e-6)


@pytest.mark.parametrize("t", [1, 2])
def test_deterministic_matches_oracle(P, t):
    N, M = 64, 6000
    _say("deterministic oracle", t)
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.01, tf="fresnel", ox=5e-5)
    rng = np.random.default_rng(47)
    x, y = synth.clustered_box(rng, M, N * geo.g, frac=0.9, sigma_frac=0.03)
    if t == 1:
        c = synth.unit_phase(rng, M)
        ref, inp = O.nuasm1(geo, x, y, c), c
    else:
        u1 = synth.unit_phase(rng, (N, N))
        ref, inp = O.nuasm2(geo, u1, x, y), u1
    _, got = _run(P, geo, t, x, y, inp, deterministic=True)
    check_close(host(got), ref, 1e-5)


@pytest.mark.parametrize("t", [1, 2])
def test_dense_bin_deterministic(P, t):
    """20000 points within half a pixel of the window centre: one bin holds
    them all, split over several spreading chunks and binning ranges."""
    N, M = 32, 20000
    _say("big bin", t)
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.002, tf="asm", band="full")
    rng = np.random.default_rng(53)
    x = rng.uniform(-0.5, 0.5, M) * geo.g
    y = rng.uniform(-0.5, 0.5, M) * geo.g
    inp = synth.unit_phase(rng, M if t == 1 else (N, N))
    plan, a = _run(P, geo, t, x, y, inp, deterministic=True)
    recs, counts = plan.debug_records()
    assert int(counts.max()) == M
    idx, bins, lx, ly, prim, dx, dy, c = decode(recs, counts)
    for b in np.unique(bins):
        assert np.all(np.diff(idx[bins == b]) > 0)
    plan.set_points(dev(torch, x), dev(torch, y))
    assert torch.equal(plan.execute(dev(torch, inp)), a)
    ref = O.nuasm1(geo, x, y, inp) if t == 1 else O.nuasm2(geo, inp, x, y)
    check_close(host(a), ref, 1e-5)


def test_deterministic_ranges_and_a_very_dense_bin(P):
    """Deterministic binning takes ranges of at most 1024 points (tuned or
    not); 2^21 + 5 points on the window centre (one bin of that many records)
    give bitwise-equal results on rebinding."""
    N, M = 16, (1 << 21) + 5
    _say("dense bin, 2^21 + 5 records")
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.002)
    zc = torch.zeros(M, dtype=torch.float64, device="cuda")
    c = torch.ones(M, dtype=torch.complex64, device="cuda")
    plan = make_plan(P, geo, 1, deterministic=True)
    plan.set_points(zc, zc)
    assert plan.info["bin_range_points"] == 1024
    a = plan.execute(c).clone()
    assert torch.isfinite(torch.view_as_real(a)).all()
    plan.set_tuning(bin_range_points=65535)
    plan.set_points(zc, zc)
    assert plan.info["bin_range_points"] == 1024
    assert torch.equal(plan.execute(c), a)
    ref = make_plan(P, geo, 1)
    ref.set_points(zc, zc)
    check_close(host(ref.execute(c)), host(a), 1e-5)


def test_deterministic_type3_and_adjoints(P):
    """Type 3 (two binned point sets) and the adjoints of types 1 and 2 (the
    other pipeline on the same bins) are bitwise reproducible too."""
    N = 64
    _say("deterministic type 3 and adjoints")
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.02, tf="asm", band="limited", ox=1e-4)
    rng = np.random.default_rng(73)
    xs, ys = synth.clustered_box(rng, 5000, N * geo.g)
    xd, yd = synth.clustered_box(rng, 4000, N * geo.g)
    c, wv = synth.unit_phase(rng, 5000), synth.unit_phase(rng, 4000)
    v = synth.unit_phase(rng, (2 * N, 2 * N))

    def run():
        p3 = make_plan(P, geo, 3, deterministic=True)
        p3.set_points(dev(torch, xs), dev(torch, ys)).set_dest_points(dev(torch, xd), dev(torch, yd))
        p1 = make_plan(P, geo, 1, deterministic=True)
        p1.set_points(dev(torch, xs), dev(torch, ys))
        p2 = make_plan(P, geo, 2, deterministic=True)
        p2.set_points(dev(torch, xd), dev(torch, yd))
        return (p3.execute(dev(torch, c)), p3.adjoint(dev(torch, wv)), p1.adjoint(dev(torch, v)),
                p2.adjoint(dev(torch, wv)))
    first, second = run(), run()
    for a, b in zip(first, second):
        assert torch.equal(a, b)
    check_close(host(first[0]), O.nuasm3(geo, xs, ys, c, xd, yd), 1e-5)


def test_deterministic_at_the_largest_grid(P):
    """N' = 8192 on the full fine grid (257 x 257 bins, the largest bin keys
    and histogram rows of the stable scatter), 2^24 jittered points: the
    deterministic result equals itself bitwise on rebinding and the default
    mode's to float32 rounding."""
    N, M = 4096, 1 << 24
    _say("deterministic, N'=8192, M=2^24, full fine grid")
    geo = geometry(N=N, g=4e-6, lam=532e-9, z=1.0, tf="asm", band="limited")
    rng = synth.rng_for(3, 0)
    x, y = synth.jittered_roi(rng, N, geo.g, M=M)
    xs, ys = dev(torch, x), dev(torch, y)
    u1 = dev(torch, synth.unit_phase(rng, (N, N)))
    pd = make_plan(P, geo, 2, deterministic=True, full_fine_grid=True, defer_range_check=True)
    assert pd.info["tiles"] == 257 * 257
    pd.set_points(xs, ys)
    a = pd.execute(u1).clone()
    pd.set_points(xs, ys)
    assert torch.equal(pd.execute(u1), a)
    pd.check_points()
    del pd
    p0 = make_plan(P, geo, 2, full_fine_grid=True, defer_range_check=True)
    p0.set_points(xs, ys)
    check_close(host(p0.execute(u1)), host(a), 1e-6)


def test_batch_matches_plain_plans_bitwise(P):
    rng = np.random.default_rng(59)
    specs, xs, ys, ins, outs = [], [], [], [], []
    for p in range(5):
        n = [64, 128][p % 2]
        m = [3000, 20000, 45000][p % 3]
        t = 1 + (p % 2)
        tf = "asm" if p < 3 else "fresnel"
        specs.append(dict(N=n, type=t, lam=633e-9, z=0.01 * (p + 1), g=4e-6, tf=tf,
                          band="limited" if tf == "asm" else "full", tol=1e-6, deterministic=True))
        x, y = synth.clustered_box(rng, m, n * 4e-6)
        xs.append(dev(torch, x))
        ys.append(dev(torch, y))
        ins.append(dev(torch, synth.unit_phase(rng, m if t == 1 else (n, n))))
        outs.append(torch.empty((2 * n, 2 * n) if t == 1 else (m,), dtype=torch.complex64, device="cuda"))
    _say("batch bitwise")
    b = P.Batch(specs)
    for rep in range(2):
        b.run(xs, ys, ins, outs)
        assert b.check_points() == -1
        for p, s in enumerate(specs):
            plain = P.Plan(**s)
            plain.set_points(xs[p], ys[p])
            assert torch.equal(plain.execute(ins[p]), outs[p]), f"plane {p}, run {rep}"
