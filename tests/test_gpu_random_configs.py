"""Seeded sweep over parameter combinations: each case draws the operator
type (1, 2 or 3), transfer function and band, the sign of z, 2-D offsets,
pitch, wavelength, kernel tolerance, point distribution, point count and the
deterministic flag from one generator, and compares the GPU operator with the
FP64 oracle at the tolerance's bound.  The list of cases is fixed by the seed,
so a failure names a reproducible case."""
import sys

import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import check_close, dev, geometry, host, make_plan, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BOUND = {1e-3: 2e-3, 1e-6: 1e-5, 1e-9: 2e-6}


def _cases(n=16, seed=20240611):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        N = int(rng.choice([16, 32, 64]))
        g = float(rng.choice([2e-6, 4e-6, 8e-6]))
        lam = float(rng.choice([488e-9, 532e-9, 633e-9]))
        tf = str(rng.choice(["asm", "fresnel"]))
        band = str(rng.choice(["full", "limited"])) if tf == "asm" else "full"
        z = float(rng.uniform(0.002, 0.08)) * (1 if rng.random() < 0.7 else -1)
        ox, oy = (float(v) for v in rng.uniform(-0.3, 0.3, 2) * N * g)
        out.append(dict(i=i, N=N, g=g, lam=lam, tf=tf, band=band, z=z, ox=ox, oy=oy,
                        type=int(rng.choice([1, 2, 3])), tol=float(rng.choice([1e-3, 1e-6, 1e-9])),
                        kind=str(rng.choice(["uniform", "clustered", "three_clusters"])),
                        M=int(rng.integers(1, 6000)), M2=int(rng.integers(1, 4000)),
                        det=bool(rng.random() < 0.3)))
    return out


@pytest.fixture(scope="module")
def P():
    import paper_1308_6644_amd as P
    P.load()
    return P


@pytest.mark.parametrize("c", _cases(), ids=lambda c: f"case{c['i']}-t{c['type']}-{c['tf']}-{c['band']}-N{c['N']}")
def test_random_configuration_matches_oracle(P, c):
    print(f"random case {c}", flush=True)
    sys.stdout.flush()
    geo = geometry(N=c["N"], g=c["g"], lam=c["lam"], z=c["z"], tf=c["tf"], band=c["band"], ox=c["ox"], oy=c["oy"])
    rng = np.random.default_rng(1000 + c["i"])
    x, y = synth.make_points(c["kind"], rng, c["M"], c["N"], c["g"])
    plan = make_plan(P, geo, c["type"], tol=c["tol"], deterministic=c["det"])
    plan.set_points(dev(torch, x), dev(torch, y))
    if c["type"] == 1:
        v = synth.unit_phase(rng, c["M"])
        got, ref = plan.execute(dev(torch, v)), O.nuasm1(geo, x, y, v)
    elif c["type"] == 2:
        u1 = synth.unit_phase(rng, (c["N"], c["N"]))
        got, ref = plan.execute(dev(torch, u1)), O.nuasm2(geo, u1, x, y)
    else:
        x2, y2 = synth.make_points(c["kind"], rng, c["M2"], c["N"], c["g"])
        plan.set_dest_points(dev(torch, x2), dev(torch, y2))
        v = synth.unit_phase(rng, c["M"])
        got, ref = plan.execute(dev(torch, v)), O.nuasm3(geo, x, y, v, x2, y2)
    err = check_close(host(got), ref, BOUND[c["tol"]])
    print(f"  rel-L2 {err:.3e}", flush=True)
