"""Shared helpers of the GPU tests: build oracle geometries and library plans
from one plain description, move seeded inputs to the device, and compare."""
from __future__ import annotations

import numpy as np

import oracle as O


def geometry(N, g, lam, z, tf="asm", band="full", ox=0.0, oy=0.0, band_c=(0.0, 0.0),
             band_w=(0.0, 0.0)):
    return O.Geometry(N=N, g=g, lam=lam, z=z, ox=ox, oy=oy, tf=tf, band=band,
                      band_c=tuple(band_c), band_w=tuple(band_w))


def make_plan(P, geo: O.Geometry, type_, tol=1e-6, **kw):
    return P.Plan(geo.N, type_, geo.lam, geo.z, geo.g, tf=geo.tf, ox=geo.ox, oy=geo.oy,
                  band=geo.band, band_c=geo.band_c, band_w=geo.band_w, tol=tol, **kw)


def dev(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t) -> np.ndarray:
    return t.detach().cpu().numpy().astype(np.complex128)


def rel_l2(a, b) -> float:
    return O.rel_l2(a, b)


def type1_spectral_samples(u2: np.ndarray, kx: np.ndarray, ky: np.ndarray) -> np.ndarray:
    """DFT of a centred N' x N' plane at frequency indices (kx, ky):
    sum_n u2[n] exp(-2 pi i k.n / N').  For NU-ASM_1 this equals H(k) F(k)."""
    Np = u2.shape[0]
    n = np.arange(-Np // 2, Np // 2, dtype=np.float64)
    ex = O.cis_cycles(-np.outer(n, kx) / Np)      # [nx, s]
    ey = O.cis_cycles(-np.outer(n, ky) / Np)      # [ny, s]
    a = u2 @ ex                                   # [ny, s]
    return np.sum(ey * a, axis=0)


def check_close(got, ref, bound: float, what: str = "", k: float = 10.0) -> float:
    """Element-wise and whole-array agreement: rel-L2 <= bound, and every
    element within k * bound * rms(ref) of the reference (a localised defect
    on a few bins or window-edge points fails the second even when the norm
    hides it).  Returns the rel-L2."""
    got = np.asarray(got).astype(np.complex128)
    ref = np.asarray(ref).astype(np.complex128)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    d = np.abs(got - ref).ravel()
    rms = float(np.sqrt(np.mean(np.abs(ref.ravel()) ** 2))) if ref.size else 0.0
    rel = O.rel_l2(got, ref) if ref.size and rms > 0 else float(d.max(initial=0.0))
    assert rel <= bound, f"{what} rel-L2 {rel:.3e} > {bound:.1e}"
    worst = float(d.max(initial=0.0))
    assert worst <= k * bound * rms, (f"{what} max |err| {worst:.3e} > {k:g} * {bound:.1e} * rms(ref) "
                                      f"= {k * bound * rms:.3e} (at element {int(np.argmax(d))})")
    return rel
