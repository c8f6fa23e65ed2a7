"""Band-adaptive fine grid: when the Rect of Eq. 4 keeps only a narrow band,
the plan runs the non-uniform sums and the fine-grid FFTs on a spectral grid
N'' < N' (fine grid 2 N'').  Results must match the oracle to the operator
bar and the full 2 N' fine grid (NUASM_FULL_FINE_GRID) to float32 rounding,
for every operator type, adjoint and point representation."""
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


# (N, geometry, expected N'') -- bands of Eq. 4 that shrink with z and move with o
CASES = [
    (256, dict(g=4e-6, lam=633e-9, z=0.1, tf="asm", band="limited", ox=1e-3), 256),
    (256, dict(g=4e-6, lam=633e-9, z=0.5, tf="asm", band="limited"), 64),
    (128, dict(g=8e-6, lam=532e-9, z=-0.3, tf="asm", band="limited", oy=-5e-4), 64),
    (256, dict(g=4e-6, lam=633e-9, z=0.05, tf="asm", band="explicit", band_c=(20.0, -10.0),
               band_w=(60.0, 41.0)), 128),
]


def _id(c):
    N, kw, npf = c
    return f"N{N}-{kw['band']}-z{kw['z']}-Npf{npf}"


@pytest.mark.parametrize("case", CASES, ids=_id)
def test_band_grid_types_1_2_3_and_adjoints(P, case):
    N, kw, npf = case
    _say("band grid", _id(case))
    geo = geometry(N=N, **kw)
    rng = np.random.default_rng(N + npf)
    M1, M2 = 5000, 4000
    x1, y1 = synth.clustered_box(rng, M1, N * geo.g)
    x2, y2 = synth.uniform_box(rng, M2, N * geo.g)
    c = synth.unit_phase(rng, M1)
    u1 = synth.unit_phase(rng, (N, N))
    w2 = synth.unit_phase(rng, M2)
    v = synth.unit_phase(rng, (2 * N, 2 * N))
    outs = {}
    for full in (False, True):
        p1 = make_plan(P, geo, 1, full_fine_grid=full)
        p2 = make_plan(P, geo, 2, full_fine_grid=full)
        p3 = make_plan(P, geo, 3, full_fine_grid=full)
        assert p1.info["Npf"] == (2 * N if full else npf)
        p1.set_points(dev(torch, x1), dev(torch, y1))
        p2.set_points(dev(torch, x2), dev(torch, y2))
        p3.set_points(dev(torch, x1), dev(torch, y1))
        p3.set_dest_points(dev(torch, x2), dev(torch, y2))
        outs[full] = [host(p1.execute(dev(torch, c))), host(p2.execute(dev(torch, u1))),
                      host(p3.execute(dev(torch, c))), host(p1.adjoint(dev(torch, v))),
                      host(p2.adjoint(dev(torch, w2))), host(p3.adjoint(dev(torch, w2)))]
    refs = [O.nuasm1(geo, x1, y1, c), O.nuasm2(geo, u1, x2, y2), O.nuasm3(geo, x1, y1, c, x2, y2),
            O.nuasm1_adjoint(geo, v, x1, y1), O.nuasm2_adjoint(geo, w2, x2, y2),
            O.nuasm3_adjoint(geo, w2, x1, y1, x2, y2)]
    for k, ref in enumerate(refs):
        check_close(outs[False][k], ref, 1e-5, what=str(k))
        check_close(outs[False][k], outs[True][k], 3e-6, what=str(k))


def test_band_grid_with_grid_points(P):
    """A scaled destination grid on the reduced fine grid (separable passes
    with the coarser cells)."""
    N = 256
    _say("band grid + scaled grid")
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.5, tf="asm", band="limited")
    rng = np.random.default_rng(5)
    u1 = synth.unit_phase(rng, (N, N))
    plan = make_plan(P, geo, 2)
    assert plan.info["Npf"] == 64
    plan.set_grid_points(150, 130, 1.3 * geo.g, 2 * geo.g, -3 * geo.g)
    x, y = O.grid_points(150, 130, 1.3 * geo.g, 2 * geo.g, -3 * geo.g)
    check_close(host(plan.execute(dev(torch, u1))), O.nuasm2(geo, u1, x, y), 1e-5)
    c = synth.unit_phase(rng, 150 * 130)
    p1 = make_plan(P, geo, 1)
    p1.set_grid_points(150, 130, 1.3 * geo.g, 2 * geo.g, -3 * geo.g)
    check_close(host(p1.execute(dev(torch, c))), O.nuasm1(geo, x, y, c), 1e-5)


def test_band_grid_choice(P):
    """Full band and Fresnel keep N'' = N'; the reduction stops at N'/8 and 32."""
    _say("band grid choice")
    g = 4e-6
    assert make_plan(P, geometry(N=256, g=g, lam=633e-9, z=0.5, tf="asm", band="full"), 1).info["Npf"] == 512
    assert make_plan(P, geometry(N=256, g=g, lam=633e-9, z=0.5, tf="fresnel"), 2).info["Npf"] == 512
    assert make_plan(P, geometry(N=1024, g=g, lam=633e-9, z=5.0, tf="asm", band="limited"), 2).info["Npf"] == 256
    assert make_plan(P, geometry(N=16, g=g, lam=633e-9, z=5.0, tf="asm", band="limited"), 2).info["Npf"] == 32
