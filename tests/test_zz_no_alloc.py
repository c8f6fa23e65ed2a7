"""The allocation-free entry point nuasm_execute_noalloc, called through the
C ABI: its output equals nuasm_execute's on the same plan, on two calls in a
row (the second with fewer points), with bins split over several spreading
workgroups so that the static partial-tile array is used; bitwise in
deterministic mode, to float32 summation order otherwise.  Plans whose bound
points may need more partial tiles than the array holds are refused."""
import ctypes

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


def _noalloc(P, plan, inp, out):
    lib = P.load()
    plan._sync_stream()
    st = lib.nuasm_execute_noalloc(plan._h, ctypes.c_void_p(inp.data_ptr()), ctypes.c_void_p(out.data_ptr()))
    if st != 0:
        raise P.NuasmError(st, lib.nuasm_status_string(st).decode(), lib.nuasm_last_error().decode())
    return out


def _dense_points(rng, M, N, g):
    # most points inside a few pixels: those bins hold several spreading chunks
    x = rng.uniform(-3 * g, 3 * g, M)
    y = rng.uniform(-1 * g, 4 * g, M)
    k = M // 10
    x[:k] = rng.uniform(-N * g / 2, N * g / 2, k)
    y[:k] = rng.uniform(-N * g / 2, N * g / 2, k)
    return x, y


@pytest.mark.parametrize("det", [True, False], ids=["deterministic", "default"])
@pytest.mark.parametrize("t", [1, 3])
def test_noalloc_matches_execute_on_two_calls(P, det, t):
    print(f"noalloc type {t} deterministic={det}", flush=True)
    N, g = 64, 4e-6
    geo = geometry(N=N, g=g, lam=633e-9, z=0.01, tf="asm", band="limited", ox=1e-4)
    rng = np.random.default_rng(606 + t)
    plan = make_plan(P, geo, t, deterministic=det)
    for M in (20000, 7000):  # the second call with a smaller input
        x, y = _dense_points(rng, M, N, g)
        c = synth.unit_phase(rng, M)
        plan.set_points(dev(torch, x), dev(torch, y))
        if t == 3:
            xd, yd = synth.uniform_box(rng, 3000, N * g)
            plan.set_dest_points(dev(torch, xd), dev(torch, yd))
        cd = dev(torch, c)
        ref = host(plan.execute(cd))
        shape = (2 * N, 2 * N) if t == 1 else (3000,)
        out = torch.full(shape, float("nan"), dtype=torch.complex64, device="cuda")
        got = host(_noalloc(P, plan, cd, out))
        if det:
            assert np.array_equal(got, ref)
        check_close(got, ref, 1e-6, what=f"M={M}")
        oracle = O.nuasm1(geo, x, y, c) if t == 1 else O.nuasm3(geo, x, y, c, xd, yd)
        check_close(got, oracle, 1e-5, what=f"oracle M={M}")


def test_noalloc_type2_and_refusal(P):
    print("noalloc type 2 and refusal", flush=True)
    N, g = 64, 4e-6
    geo = geometry(N=N, g=g, lam=633e-9, z=0.02, tf="fresnel")
    rng = np.random.default_rng(7)
    x, y = synth.clustered_box(rng, 5000, N * g)
    u1 = dev(torch, synth.unit_phase(rng, (N, N)))
    p2 = make_plan(P, geo, 2)
    p2.set_points(dev(torch, x), dev(torch, y))
    out = torch.empty((5000,), dtype=torch.complex64, device="cuda")
    check_close(host(_noalloc(P, p2, u1, out)), host(p2.execute(u1)), 1e-6)
    # deferred range check: only a bound is known, min(chunk-table size,
    # 8 M / 1792) tiles, which for 2^20 points (2350 chunks) exceeds the 2048
    # tiles of the static array
    M = 1 << 20
    x, y = synth.uniform_box(rng, M, N * g)
    p1 = make_plan(P, geo, 1, defer_range_check=True)
    p1.set_points(dev(torch, x), dev(torch, y))
    c = dev(torch, synth.unit_phase(rng, M))
    out = torch.empty((2 * N, 2 * N), dtype=torch.complex64, device="cuda")
    with pytest.raises(P.NuasmError) as ei:
        _noalloc(P, p1, c, out)
    assert ei.value.name == "NUASM_ERR_UNSUPPORTED"
    # the same points bound with the range check: the exact count is known
    p1b = make_plan(P, geo, 1)
    p1b.set_points(dev(torch, x), dev(torch, y))
    check_close(host(_noalloc(P, p1b, c, out)), host(p1b.execute(c)), 1e-6)
