"""Points outside the window under a deferred range check
(NUASM_DEFER_RANGE_CHECK): such a point gets no record, nuasm_check_points
reports NUASM_ERR_OUT_OF_RANGE, and every output slot that belongs to it --
a type-2 destination, a type-1 adjoint value, a type-3 destination -- is
NaN, while every other output is the oracle's over the points inside the
window (outputs of a type-2 operator are independent sums, and a type-1
result only receives the accepted points).  Default and deterministic
binning (two different scatters), points beyond the window and NaN
coordinates, and a support of more than 16383 bins (where the scatter ranks
records with 16-bit LDS counters instead of staged 32-bit cursors), which is
compared with a plain plan over the accepted points.
"""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import check_close, dev, host, make_plan

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1308_6644_amd as P
    P.load()
    return P


def _points_with_rejects(seed, M, N, g, frac=0.05):
    rng = synth.rng_for(seed, 0)
    x, y = synth.clustered_box(rng, M, N * g)
    bad = rng.choice(M, size=max(1, int(frac * M)), replace=False)
    half = 0.5 * N * g
    x = x.copy()
    y = y.copy()
    # beyond the window on either side, or NaN
    kind = np.arange(bad.size) % 3
    x[bad[kind == 0]] = 1.2 * half
    y[bad[kind == 1]] = -1.5 * half
    x[bad[kind == 2]] = np.nan
    acc = np.ones(M, bool)
    acc[bad] = False
    return x, y, acc, rng


@pytest.mark.parametrize("det", [False, True])
def test_rejected_points_give_nan_outputs(P, det):
    N, M = 64, 3000
    geo = O.Geometry(N=N, g=4e-6, lam=633e-9, z=0.01, ox=1e-4, oy=0.0, tf="asm", band="limited")
    x, y, acc, rng = _points_with_rejects(11, M, N, geo.g)
    print(f"rejected: det={det} N={N} M={M} rejected={int((~acc).sum())}", flush=True)
    xd, yd = dev(torch, x), dev(torch, y)
    u1 = synth.unit_phase(rng, (N, N))
    c = synth.unit_phase(rng, M)
    v = synth.unit_phase(rng, (2 * N, 2 * N))
    # type 2: NaN at the rejected destinations, the oracle elsewhere
    p2 = make_plan(P, geo, 2, defer_range_check=True, deterministic=det)
    p2.set_points(xd, yd)
    out = host(p2.execute(dev(torch, u1)))
    assert np.isnan(out[~acc]).all() and np.isfinite(out[acc]).all()
    check_close(out[acc], O.nuasm2(geo, u1, x[acc], y[acc]), 1e-5, what="type 2")
    with pytest.raises(P.NuasmError) as ei:
        p2.check_points()
    assert ei.value.name == "NUASM_ERR_OUT_OF_RANGE"
    # type 1: the accepted points only; its adjoint: NaN at the rejected points
    p1 = make_plan(P, geo, 1, defer_range_check=True, deterministic=det)
    p1.set_points(xd, yd)
    got = host(p1.execute(dev(torch, c)))
    check_close(got, O.nuasm1(geo, x[acc], y[acc], c[acc]), 1e-5, what="type 1")
    w = host(p1.adjoint(dev(torch, v)))
    assert np.isnan(w[~acc]).all() and np.isfinite(w[acc]).all()
    check_close(w[acc], O.nuasm1_adjoint(geo, v, x[acc], y[acc]), 1e-5, what="type-1 adjoint")


def test_rejected_type3_destinations(P):
    N, M = 64, 2000
    geo = O.Geometry(N=N, g=4e-6, lam=633e-9, z=0.02, ox=0.0, oy=0.0, tf="fresnel", band="full")
    xs, ys, _, rng = _points_with_rejects(12, M, N, geo.g, frac=0.0)
    xs = np.where(np.isnan(xs), 0.0, np.clip(xs, -0.45 * N * geo.g, 0.45 * N * geo.g))
    ys = np.clip(ys, -0.45 * N * geo.g, 0.45 * N * geo.g)
    xt, yt, acc, _ = _points_with_rejects(13, M, N, geo.g)
    c = synth.unit_phase(rng, M)
    p3 = make_plan(P, geo, 3, defer_range_check=True)
    p3.set_points(dev(torch, xs), dev(torch, ys))
    p3.set_dest_points(dev(torch, xt), dev(torch, yt))
    out = host(p3.execute(dev(torch, c)))
    assert np.isnan(out[~acc]).all() and np.isfinite(out[acc]).all()
    check_close(out[acc], O.nuasm3(geo, xs, ys, c, xt[acc], yt[acc]), 1e-5, what="type 3")


def test_rejected_points_many_bins(P):
    """N' = 4096 (T = 129^2 > 16383 bins): the 16-bit-rank scatter; the
    accepted outputs equal a plain plan's over the accepted points."""
    N, M = 2048, 20000
    geo = O.Geometry(N=N, g=4e-6, lam=633e-9, z=0.05, ox=0.0, oy=0.0, tf="asm", band="full")
    x, y, acc, rng = _points_with_rejects(14, M, N, geo.g)
    print(f"rejected: many bins N={N} M={M} rejected={int((~acc).sum())}", flush=True)
    assert make_plan(P, geo, 2).info["tiles"] > 16383
    u1 = dev(torch, synth.unit_phase(rng, (N, N)))
    p = make_plan(P, geo, 2, defer_range_check=True)
    p.set_points(dev(torch, x), dev(torch, y))
    out = host(p.execute(u1))
    q = make_plan(P, geo, 2)
    q.set_points(dev(torch, x[acc]), dev(torch, y[acc]))
    ref = host(q.execute(u1))
    assert np.isnan(out[~acc]).all()
    check_close(out[acc], ref, 1e-6, what="many bins")
