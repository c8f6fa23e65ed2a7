"""Kernel unit tests: spreading and interpolation alone (nuasm_debug_spread /
nuasm_debug_interp) against the kernel sums written out from their
definition in numpy, float64:

    grid[i0y + my][i0x + mx] += c_j psi(dx_j + mx) psi(dy_j + my)      (spreading)
    u_j = sum_{my, mx} grid[i0y + my][i0x + mx] psi(dx_j + mx) psi(dy_j + my)

with psi(d) = exp(beta (sqrt(1 - (2 d / w)^2) - 1)) for |d| <= w/2 (the ES
kernel, beta = 2.30 w), first tap i0 = ceil(tau - w/2) and dx = i0 - tau at
the fine coordinate tau = 2 x N'' / (N' g) + N''/2 + 8 of a point.  Binned
point sets (several chunk sizes, dense bins split into partial tiles) and
uniform grids of another pitch (the separable kernels) are both covered.
"""
import sys

import numpy as np
import pytest

import synth
from gpu_util import dev, geometry, make_plan

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


def psi(d, w, beta):
    t = d * 2.0 / w
    r = 1.0 - t * t
    return np.where(r > 0.0, np.exp(beta * (np.sqrt(np.maximum(r, 0.0)) - 1.0)), 0.0)


def taps(x, y, info, g):
    Npf, Np, w = info["Npf"], info["Np"], info["w"]
    inv_g = Npf / (Np * g)
    half = 0.25 * Npf
    tau0 = Npf / 2 + 8
    tx = 2.0 * np.clip(x * inv_g, -half, half) + tau0
    ty = 2.0 * np.clip(y * inv_g, -half, half) + tau0
    fx, fy = np.ceil(tx - 0.5 * w), np.ceil(ty - 0.5 * w)
    return fx.astype(np.int64), fy.astype(np.int64), fx - tx, fy - ty


def weights(x, y, info, g):
    w, beta = info["w"], float(info["beta"])
    i0x, i0y, dx, dy = taps(x, y, info, g)
    m = np.arange(w)
    return i0x, i0y, psi(dx[:, None] + m, w, beta), psi(dy[:, None] + m, w, beta)


def spread_ref(x, y, c, info, g):
    L, w = info["L"], info["w"]
    i0x, i0y, wx, wy = weights(x, y, info, g)
    grid = np.zeros((L, L), dtype=np.complex128)
    for my in range(w):
        for mx in range(w):
            np.add.at(grid, (i0y + my, i0x + mx), c * wy[:, my] * wx[:, mx])
    return grid


def interp_ref(x, y, grid, info, g):
    w = info["w"]
    i0x, i0y, wx, wy = weights(x, y, info, g)
    out = np.zeros(x.size, dtype=np.complex128)
    for my in range(w):
        for mx in range(w):
            out += grid[i0y + my, i0x + mx] * wy[:, my] * wx[:, mx]
    return out


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_spread_of_single_points(P):
    """One point at a time: the w x w footprint holds psi(dx + mx) psi(dy + my)
    times the value, and every other support cell is exactly zero."""
    geo = geometry(N=64, g=4e-6, lam=633e-9, z=0.01)
    rng = np.random.default_rng(61)
    plan = make_plan(P, geo, 1)
    info = None
    for k in range(6):
        x = rng.uniform(-0.5, 0.5, 1) * 64 * geo.g
        y = rng.uniform(-0.5, 0.5, 1) * 64 * geo.g
        if k == 5:  # a window corner
            x[:] = -32 * geo.g
            y[:] = 32 * geo.g
        c = np.array([np.exp(1j * rng.uniform(0, 2 * np.pi))])
        plan.set_points(dev(torch, x), dev(torch, y))
        info = plan.info
        got = plan.debug_spread(dev(torch, c.astype(np.complex64))).cpu().numpy().astype(np.complex128)
        ref = spread_ref(x, y, c, info, geo.g)
        _say("single point", k, np.max(np.abs(got - ref)))
        assert np.max(np.abs(got - ref)) <= 2e-6
        assert np.all(got[ref == 0] == 0)


CASES = [
    # (tol, M, points, geometry kwargs, tuning)
    (1e-2, 20000, "clustered", dict(z=0.01, tf="asm", band="full"), {}),
    (1e-6, 20000, "clustered", dict(z=0.01, tf="asm", band="full"), {}),
    (1e-6, 20000, "clustered", dict(z=0.01, tf="asm", band="full"), dict(spread_chunk=896, interp_chunk=256)),
    (1e-12, 20000, "clustered", dict(z=0.01, tf="fresnel"), {}),
    (1e-6, 30000, "uniform", dict(z=0.5, tf="asm", band="limited"), {}),  # band-adaptive grid N'' < N'
]


def _id(c):
    tol, M, kind, kw, tun = c
    return f"tol{tol:g}-M{M}-{kind}-{kw['tf']}-{kw.get('band', '-')}-z{kw['z']}" + ("-tuned" if tun else "")


def _bound_plan(P, case, t):
    tol, M, kind, kw, tun = case
    N = 128
    geo = geometry(N=N, g=4e-6, lam=633e-9, **kw)
    rng = np.random.default_rng(67)
    x, y = synth.make_points(kind, rng, M, N, geo.g)
    plan = make_plan(P, geo, t, tol=tol)
    if tun:
        plan.set_tuning(**tun)
    plan.set_points(dev(torch, x), dev(torch, y))
    return plan, geo, x, y, rng


@pytest.mark.parametrize("case", CASES, ids=_id)
def test_spread_matches_the_kernel_sum(P, case):
    plan, geo, x, y, rng = _bound_plan(P, case, 1)
    _say("spread", _id(case), plan.info["Npf"], plan.info["w"])
    c = synth.unit_phase(rng, x.size)
    got = plan.debug_spread(dev(torch, c)).cpu().numpy().astype(np.complex128)
    ref = spread_ref(x, y, c.astype(np.complex128), plan.info, geo.g)
    assert rel(got, ref) <= 2e-6


@pytest.mark.parametrize("case", CASES, ids=_id)
def test_interp_matches_the_kernel_sum(P, case):
    plan, geo, x, y, rng = _bound_plan(P, case, 2)
    _say("interp", _id(case), plan.info["Npf"], plan.info["w"])
    L = plan.info["L"]
    grid = (rng.standard_normal((L, L)) + 1j * rng.standard_normal((L, L))).astype(np.complex64)
    got = plan.debug_interp(dev(torch, grid)).cpu().numpy().astype(np.complex128)
    ref = interp_ref(x, y, grid.astype(np.complex128), plan.info, geo.g)
    assert rel(got, ref) <= 2e-6


@pytest.mark.parametrize("tol", [1e-3, 1e-9])
def test_grid_point_sets_match_the_kernel_sums(P, tol):
    """An 80 x 60 grid of pitch g / sqrt(2), off-centre: the separable
    spreading and interpolation give the same sums as the generic definition.
    (The pitch and centre are incommensurate with the fine cells: psi jumps
    from exp(-beta) to 0 at the support edge, and a grid that puts taps
    exactly on that edge would make the comparison depend on the last bit of
    the tap offset.)"""
    N, nx, ny, pitch_f = 64, 80, 60, 2.0 ** -0.5
    geo = geometry(N=N, g=4e-6, lam=633e-9, z=0.01)
    pitch, cx, cy = pitch_f * geo.g, 3.3137 * geo.g, -5.0891 * geo.g
    a, b = np.arange(nx) - nx // 2, np.arange(ny) - ny // 2
    X, Y = np.meshgrid(cx + a * pitch, cy + b * pitch)  # [ny][nx], row-major = the grid order
    x, y = X.ravel(), Y.ravel()
    rng = np.random.default_rng(71)
    for t in (1, 2):
        _say("grid points", tol, t)
        plan = make_plan(P, geo, t, tol=tol)
        plan.set_grid_points(nx, ny, pitch, cx, cy)
        info = plan.info
        if t == 1:
            c = synth.unit_phase(rng, x.size)
            got = plan.debug_spread(dev(torch, c)).cpu().numpy().astype(np.complex128)
            assert rel(got, spread_ref(x, y, c.astype(np.complex128), info, geo.g)) <= 2e-6
        else:
            L = info["L"]
            grid = (rng.standard_normal((L, L)) + 1j * rng.standard_normal((L, L))).astype(np.complex64)
            got = plan.debug_interp(dev(torch, grid)).cpu().numpy().astype(np.complex128)
            assert rel(got, interp_ref(x, y, grid.astype(np.complex128), info, geo.g)) <= 2e-6
