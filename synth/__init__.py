"""Seeded synthetic inputs for the non-uniform diffraction workloads.

This module is shared by the tests, the benchmark and the smoke check.  It
draws random numbers and arranges them into the shapes the workloads need
(point sets, unit-amplitude random-phase fields, target intensities); it holds
none of the diffraction arithmetic, so neither the CPU oracle nor the GPU
library depends on it.

Conventions
-----------
* Generator: ``numpy.random.default_rng(1000 * cfg + rep)`` (PCG64).
* Coordinates are FP64 metres in the plane's local frame, centred on the
  plane window of side ``W = N * g``; every point lies in ``[-W/2, W/2)^2``.
* Complex values are ``exp(i*theta)``, ``theta ~ U[0, 2*pi)``, rounded to
  complex64.  That complex64 array is the input both sides receive.
* Point order is shuffled, so sorting is part of the measured path.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "rng_for", "unit_phase", "uniform_box", "clustered_box", "three_clusters",
    "jittered_roi", "gaussian_blobs", "quadrant_grid", "experiment_field", "WORKLOADS", "HEADLINE",
    "batched_planes",
]


def rng_for(stream: int, rep: int = 0) -> np.random.Generator:
    """Seeded generator of input stream `stream` (a workload's `seed`),
    repetition `rep`: PCG64 seeded with 1000 stream + rep."""
    return np.random.default_rng(1000 * int(stream) + int(rep))


def unit_phase(rng: np.random.Generator, shape) -> np.ndarray:
    """Unit-amplitude values with uniform random phase, complex64."""
    th = rng.uniform(0.0, 2.0 * np.pi, size=shape)
    return np.exp(1j * th).astype(np.complex64)


def _clip_box(v: np.ndarray, W: float) -> np.ndarray:
    # uniform draws are already in [-W/2, W/2); guard the open upper edge
    # against rounding of the scaled draw
    hi = np.nextafter(W / 2.0, -np.inf)
    return np.minimum(v, hi)


def uniform_box(rng: np.random.Generator, M: int, W: float):
    """M points uniform in [-W/2, W/2)^2 (FP64 metres)."""
    x = _clip_box(rng.uniform(-W / 2.0, W / 2.0, size=M), W)
    y = _clip_box(rng.uniform(-W / 2.0, W / 2.0, size=M), W)
    return x, y


def _gauss_in_box(rng, n, center, sigma, W):
    """n draws per axis from N(center, sigma^2), redrawn until inside the box."""
    out = np.empty(n, dtype=np.float64)
    filled = 0
    while filled < n:
        need = n - filled
        v = rng.normal(center, sigma, size=max(need + need // 4 + 16, 64))
        v = v[(v >= -W / 2.0) & (v < W / 2.0)]
        take = min(need, v.size)
        out[filled:filled + take] = v[:take]
        filled += take
    return out


def clustered_box(rng: np.random.Generator, M: int, W: float,
                  frac: float = 0.7, sigma_frac: float = 0.1):
    """Clustered point set: round(frac*M) points from an isotropic Gaussian of
    standard deviation ``sigma_frac*W`` at the window centre (rejected and
    redrawn outside the window), the rest uniform in the window; shuffled."""
    mg = int(round(frac * M))
    xg = _gauss_in_box(rng, mg, 0.0, sigma_frac * W, W)
    yg = _gauss_in_box(rng, mg, 0.0, sigma_frac * W, W)
    xu, yu = uniform_box(rng, M - mg, W)
    x = np.concatenate([xg, xu])
    y = np.concatenate([yg, yu])
    p = rng.permutation(M)
    return x[p].copy(), y[p].copy()


def three_clusters(rng: np.random.Generator, M: int, W: float,
                   sigma_frac: float = 0.05, spread: float = 0.3):
    """Three Gaussian clusters (centres ~ U[-spread*W, spread*W]^2, standard
    deviation sigma_frac*W, equal split, rejection to the window); shuffled."""
    cx = rng.uniform(-spread * W, spread * W, size=3)
    cy = rng.uniform(-spread * W, spread * W, size=3)
    sizes = [M // 3, M // 3, M - 2 * (M // 3)]
    xs, ys = [], []
    for i, n in enumerate(sizes):
        xs.append(_gauss_in_box(rng, n, cx[i], sigma_frac * W, W))
        ys.append(_gauss_in_box(rng, n, cy[i], sigma_frac * W, W))
    x = np.concatenate(xs)
    y = np.concatenate(ys)
    p = rng.permutation(M)
    return x[p].copy(), y[p].copy()


def jittered_roi(rng: np.random.Generator, N: int, g: float, roi: int = 512,
                 M: int = 1 << 24):
    """Jittered pixel grid with a 4x denser region of interest.

    Outside a centred roi x roi pixel region there is one point uniform in each
    pixel; inside it, one point uniform in each half-pixel cell.  A seeded
    uniform deletion of background points brings the count to exactly M.
    Returns FP64 metres, shuffled.
    """
    half = N // 2
    r0, r1 = -roi // 2, roi // 2
    # background: every pixel outside the ROI
    iy, ix = np.meshgrid(np.arange(-half, half), np.arange(-half, half), indexing="ij")
    outside = ~((ix >= r0) & (ix < r1) & (iy >= r0) & (iy < r1))
    bx = ix[outside].astype(np.float64)
    by = iy[outside].astype(np.float64)
    del ix, iy, outside
    n_roi = (2 * roi) ** 2
    n_bg_keep = M - n_roi
    if n_bg_keep < 0 or n_bg_keep > bx.size:
        raise ValueError("jittered_roi: M incompatible with N and roi")
    keep = rng.choice(bx.size, size=n_bg_keep, replace=False)
    keep.sort()
    bx = bx[keep] + rng.uniform(0.0, 1.0, size=n_bg_keep)
    by = by[keep] + rng.uniform(0.0, 1.0, size=n_bg_keep)
    # ROI: half-pixel cells
    h = np.arange(2 * r0, 2 * r1, dtype=np.float64) * 0.5
    qy, qx = np.meshgrid(h, h, indexing="ij")
    qx = qx.ravel() + rng.uniform(0.0, 0.5, size=n_roi)
    qy = qy.ravel() + rng.uniform(0.0, 0.5, size=n_roi)
    x = np.concatenate([bx, qx]) * g
    y = np.concatenate([by, qy]) * g
    W = N * g
    x = _clip_box(x, W)
    y = _clip_box(y, W)
    p = rng.permutation(M)
    return x[p].copy(), y[p].copy()


def gaussian_blobs(rng: np.random.Generator, x: np.ndarray, y: np.ndarray,
                   W: float, nb: int = 32) -> np.ndarray:
    """Target intensity at the points: a sum of nb random Gaussian blobs
    (centres ~ U[-0.4W, 0.4W]^2, widths ~ U[0.02W, 0.08W], amplitudes
    ~ U[0.5, 1]).  Unscaled; FP64."""
    mu_x = rng.uniform(-0.4 * W, 0.4 * W, size=nb)
    mu_y = rng.uniform(-0.4 * W, 0.4 * W, size=nb)
    s = rng.uniform(0.02 * W, 0.08 * W, size=nb)
    a = rng.uniform(0.5, 1.0, size=nb)
    t = np.zeros(x.shape, dtype=np.float64)
    for b in range(nb):
        t += a[b] * np.exp(-((x - mu_x[b]) ** 2 + (y - mu_y[b]) ** 2) / (2.0 * s[b] ** 2))
    return t


def experiment_field(rng: np.random.Generator, x: np.ndarray, y: np.ndarray, W: float) -> np.ndarray:
    """Complex source values standing in for the paper's two photographs
    (one as amplitude, one as phase): amplitude from a blob field scaled to
    [0, 1], phase from a second blob field scaled to [-pi/2, pi/2] (the
    paper's mapping of pixel values 0..255).  complex128 at the points."""
    a = gaussian_blobs(rng, x, y, W)
    p = gaussian_blobs(rng, x, y, W)
    a = (a - a.min()) / max(a.max() - a.min(), 1e-300)
    p = (p - p.min()) / max(p.max() - p.min(), 1e-300)
    return a * np.exp(1j * np.pi * (p - 0.5))


def quadrant_grid(N: int, pitch: float, factors=(0.9, 0.8, 0.7, 1.0)):
    """Quadrant-wise uniform sampling of an N x N plane: quadrant q (first to
    fourth, counter-clockwise from +x,+y) is an (N/2) x (N/2) grid whose pitch
    is factors[q-1] * pitch, anchored at the plane centre.  Returns FP64
    metres (not shuffled; the caller may shuffle)."""
    h = N // 2
    i = np.arange(h, dtype=np.float64)
    xs, ys = [], []
    signs = [(1, 1), (-1, 1), (-1, -1), (1, -1)]
    for (sx, sy), f in zip(signs, factors):
        p = f * pitch
        a = (i + 0.5) * p
        gy, gx = np.meshgrid(a, a, indexing="ij")
        xs.append((sx * gx).ravel())
        ys.append((sy * gy).ravel())
    return np.concatenate(xs), np.concatenate(ys)


# Workload table, keyed by what each workload is.  Each entry is plain data;
# the tests, the benchmark and the smoke check read it.  Pitch, wavelength,
# band and offset follow the stated workloads; where a workload leaves them
# open the values here fill them in.  `seed` is the stream number its inputs
# are drawn from (rng_for).
WORKLOADS = {
    "nuasm1_tiny_N64_M4096": dict(seed=1, N=64, g=8e-6, lam=532e-9, z=0.05,
                                  ox=0.0, oy=0.0, tf="asm", band="full", tol=1e-6, M=4096,
                                  points="uniform", types=(1,)),
    "nuasm12_N1024_M1M_clustered": dict(seed=2, N=1024, g=4e-6, lam=633e-9,
                                        zs=(0.01, 0.1, 0.5), ox=1e-3, oy=0.0, tfs=("asm", "fresnel"),
                                        band="limited", tol=1e-6, M=1 << 20, points="clustered",
                                        types=(1, 2)),
    "nuasm2_N4096_M16M_roi": dict(seed=3, N=4096, g=4e-6, lam=532e-9, z=1.0,
                                  ox=0.0, oy=0.0, tf="asm", band="limited", tols=(1e-3, 1e-6, 1e-9),
                                  M=1 << 24, points="jittered_roi", types=(2,)),
    "batched_64_planes": dict(seed=4, P=64, Ns=(256, 512, 1024, 2048), g=4e-6,
                              lam=633e-9, zrange=(0.005, 0.5), Mrange=(1e4, 2e6), ox=0.0, oy=0.0,
                              band="limited", tol=1e-6, points="clustered"),
    "cgh_N2048_M4M": dict(seed=5, N=2048, g=4e-6, lam=532e-9, z=0.2, ox=0.0,
                          oy=0.0, tf="asm", band="limited", tol=1e-6, M=1 << 22,
                          points="three_clusters", types=(2,)),
}

HEADLINE = WORKLOADS["nuasm12_N1024_M1M_clustered"]


def plane_width(N: int, g: float) -> float:
    return N * g


def make_points(kind: str, rng: np.random.Generator, M: int, N: int, g: float):
    W = plane_width(N, g)
    if kind == "uniform":
        return uniform_box(rng, M, W)
    if kind == "clustered":
        return clustered_box(rng, M, W)
    if kind == "three_clusters":
        return three_clusters(rng, M, W)
    if kind == "jittered_roi":
        return jittered_roi(rng, N, g, M=M)
    raise ValueError(kind)


def log_uniform_int(rng: np.random.Generator, lo: float, hi: float) -> int:
    return int(math.floor(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def batched_planes(P: int = 64, g: float = 4e-6, lam: float = 633e-9, tol: float = 1e-6):
    """The 64-plane batched workload (input stream 4), drawn plane by plane in
    one fixed order: N ~ U{256, 512, 1024, 2048}, M = floor(exp(U[ln 1e4,
    ln 2e6])), z ~ U[0.005, 0.5] m, type ~ U{1, 2}, transfer function
    ~ U{band-limited ASM, Fresnel}, clustered points in the N g window, then
    the plane's input (c[M] for type 1, u1[N][N] for type 2).  Returns a list
    of dicts: ``spec`` (keyword arguments of a plan: N, type, lam, z, g, tf,
    band, tol) and the host arrays ``x``, ``y``, ``inp``."""
    rng = rng_for(4)
    planes = []
    for _ in range(P):
        n = int(rng.choice([256, 512, 1024, 2048]))
        m = log_uniform_int(rng, 1e4, 2e6)
        z = float(rng.uniform(0.005, 0.5))
        t = int(rng.integers(1, 3))
        tf = "asm" if rng.uniform() < 0.5 else "fresnel"
        x, y = clustered_box(rng, m, n * g)
        inp = unit_phase(rng, m if t == 1 else (n, n))
        planes.append(dict(spec=dict(N=n, type=t, lam=lam, z=z, g=g, tf=tf,
                                     band="limited" if tf == "asm" else "full", tol=tol),
                           x=x, y=y, inp=np.ascontiguousarray(inp)))
    return planes
