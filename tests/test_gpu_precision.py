"""Precision sweep at scale: NU-ASM_2 with N = 4096 (N' = 8192), M = 2^24
destination points (jittered pixel grid, 4x denser in a 512 x 512 region of
interest), 532 nm, z = 1.0 m (about 1.9e6 phase cycles), band-limited ASM,
kernel tolerances 1e-3 / 1e-6 / 1e-9, and the transfer-function phase in FP64
(the path's default) or naively in FP32.  Errors are measured against the FP64
oracle on 256 sampled destination points (half inside the region of
interest); every output is an independent sum, so this is exact per point."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import check_close, dev, geometry, host, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N, G, LAM, Z, M = 4096, 4e-6, 532e-9, 1.0, 1 << 24


@pytest.fixture(scope="module")
def data():
    import paper_1308_6644_amd as P
    P.load()
    print(f"precision sweep: generating N={N} M={M}", flush=True)
    rng = synth.rng_for(3, 0)
    x, y = synth.jittered_roi(rng, N, G, M=M)
    u1 = synth.unit_phase(rng, (N, N))
    roi = (np.abs(x) < 256 * G) & (np.abs(y) < 256 * G)
    rs = np.random.default_rng(77)
    sel = np.concatenate([rs.choice(np.flatnonzero(roi), 128, replace=False),
                          rs.choice(np.flatnonzero(~roi), 128, replace=False)])
    geo = geometry(N=N, g=G, lam=LAM, z=Z, tf="asm", band="limited")
    print("  oracle: uniform spectrum, transfer function, 256 sampled points", flush=True)
    U = O.uniform_spectrum(u1, 2 * N, "fft")
    ref = O.nuasm2_from_spectrum(geo, U, x[sel], y[sel])
    del U
    return dict(P=P, xd=dev(torch, x), yd=dev(torch, y), ud=dev(torch, u1), sel=sel, ref=ref)


RESULTS = {}


@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-9])
@pytest.mark.parametrize("phase_fp64", [True, False])
def test_precision_sweep(data, tol, phase_fp64):
    P = data["P"]
    print(f"precision tol={tol} phase_fp64={phase_fp64}", flush=True)
    plan = P.Plan(N, 2, LAM, Z, G, tf="asm", band="limited", tol=tol, phase_fp64=phase_fp64,
                  defer_range_check=True)
    plan.set_points(data["xd"], data["yd"])
    out = plan.execute(data["ud"])
    plan.check_points()
    got = host(out[torch.from_numpy(data["sel"]).cuda()])
    err = rel_l2(got, data["ref"])
    RESULTS[(tol, phase_fp64)] = err
    print(f"  rel-L2 on 256 sampled points = {err:.3e}", flush=True)
    del plan, out
    torch.cuda.empty_cache()
    if phase_fp64:
        # kernel error at 1e-3 / 1e-6; float32 floor of an 8192^2 pipeline at 1e-9
        check_close(got, data["ref"], {1e-3: 3e-3, 1e-6: 1e-5, 1e-9: 1e-5}[tol])
    else:
        # z / lambda ~ 1.9e6 cycles: a float32 phase is wrong by O(1) radian
        assert err >= 0.1
