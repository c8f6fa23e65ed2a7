"""FP64 CPU oracle for non-uniform sampled angular-spectrum (ASM) and Fresnel
diffraction (Shimobaba et al., "Non-uniform sampled scalar diffraction
calculation using non-uniform fast Fourier transform", arXiv 1308.6644).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this module.  The GPU library never calls it,
and it imports nothing from the library: it is the plain definition of what the
library computes, written as slow direct sums in float64.

What is computed (every function cites the passage it follows):

* Transfer functions: the shifted band-limited ASM transfer function (Eq. 4)
  and the Fresnel transfer function as the DFT of the sampled impulse response
  (Eq. 5).
* NU-ASM_1 / NU-FRE_1 (Eq. 6 with the type-1 sum of Eq. 7): non-uniform source
  samples to a uniform N' x N' destination plane.
* NU-ASM_2 / NU-FRE_2 (Eq. 9 with the type-2 sum of Eq. 8): uniform N x N source
  to non-uniform destination samples.
* NU-ASM_3 / NU-FRE_3 (the third operator type, stated after Eq. 9 as the
  combination of the first two): non-uniform source samples to non-uniform
  destination samples, the type-1 sum of Eq. 7 times H fed to the type-2 sum
  of Eq. 8.
* Their adjoints, the hologram loss gradient, and Rayleigh-Sommerfeld direct
  integration (Eq. 10) used as an independent physical cross-check.

Readings of the paper (where it is silent or its printed form is garbled):

* Kernel of the non-uniform sums.  With frequency pitch df = 1/(N' g) the
  kernel is exp(-+ 2 pi i df k.x); in pixel units x/g this is
  exp(-+ 2 pi i k (x/g) / N').  The N x N window occupies half of the N' period,
  which is what the coordinate normalisation of Fig. 1 expresses.
* Index sets.  Frequencies and destination samples are centred:
  k, n in K = {-N'/2, ..., N'/2 - 1}; array element [a_y][a_x] holds index
  (a_y - N'/2, a_x - N'/2).  Uniform sources are N x N with element [b][a] at
  pixel (a - N/2, b - N/2).
* Offset o is in metres and enters Eq. 4 as o . f with f = k df; the output
  sample [n] sits at global position n g + o.
* Evanescent frequencies (|f| > 1/lambda) have H = 0.
* Band of Eq. 4 (deferred by the paper to its reference on shifted ASM):
  per axis the local spatial frequency of the transfer function's phase must
  not exceed the window half-width S = N g, i.e. |o - z f / s(f)| <= S with
  s(f) = sqrt(1/lambda^2 - f^2).  Boundaries are inclusive.
* Fresnel impulse response: h(x) = exp(i k z)/(i lambda z) exp(i pi |x|^2/(lambda z))
  with k = 2 pi / lambda, sampled at m g + o over the centred N' x N' grid and
  weighted by the area element g^2, so that |H| is about 1 in the chirp band.
* Both types carry the factor N'^-2 of the inverse FFT, so points that lie on
  the pixel grid reproduce the uniform FFT-ASM of Eq. 3 exactly.
* Non-uniform source samples carry no quadrature weights: raw sums.
* NU-ASM_3: the paper gives no intermediate grid; N' and g are those of the
  destination window, and both point sets lie in the same N g window.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

__all__ = [
    "Geometry", "freq_index", "cis_cycles", "band_index_bounds", "band_mask",
    "transfer_asm", "transfer_fresnel", "transfer", "nuasm1", "nuasm2",
    "nuasm1_adjoint", "nuasm2_adjoint", "type1_spectrum", "spectrum_at",
    "cgh_loss", "cgh_grad", "rayleigh_sommerfeld", "rel_l2", "snr_db", "uniform_spectrum",
    "nuasm2_from_spectrum", "nuasm3", "nuasm3_adjoint", "rayleigh_sommerfeld_points", "grid_points",
    "scaled_asm",
]


@dataclass
class Geometry:
    """Problem statement of one plane pair (paper symbols in brackets).

    N       pixels per side of the uniform plane; N' = 2N  [N, N']
    g       pitch of the uniform plane, metres: Delta_2 for type 1, Delta_1
            for type 2  [Delta_1, Delta_2]
    lam     wavelength, metres  [lambda]
    z       propagation distance, metres (negative = back-propagation)  [z]
    ox, oy  off-axis offset, metres  [o]
    tf      "asm" (Eq. 4) or "fresnel" (Eq. 5)
    band    "full", "limited" or "explicit" (ASM only)
    band_c, band_w   explicit band centre and width in frequency-index units
    """
    N: int
    g: float
    lam: float
    z: float
    ox: float = 0.0
    oy: float = 0.0
    tf: str = "asm"
    band: str = "full"
    band_c: tuple = (0.0, 0.0)
    band_w: tuple = (0.0, 0.0)

    @property
    def Np(self) -> int:
        return 2 * self.N

    @property
    def df(self) -> float:
        return 1.0 / (self.Np * self.g)


def freq_index(Np: int) -> np.ndarray:
    """Centred index set K = {-N'/2, ..., N'/2 - 1} (float64)."""
    return np.arange(-Np // 2, Np // 2, dtype=np.float64)


def cis_cycles(c: np.ndarray) -> np.ndarray:
    """exp(2 pi i c) with the argument reduced to [-1/2, 1/2] cycles first."""
    c = np.asarray(c, dtype=np.float64)
    return np.exp(2j * np.pi * (c - np.round(c)))


# ---------------------------------------------------------------- Eq. 4 band
def _band_interval(lam: float, z: float, o: float, S: float):
    """Frequency interval [lo, hi] (m^-1) on one axis where the transfer
    function's phase is sampled without aliasing: |o - z f/s(f)| <= S.

    Solving u = z f / s(f) for f gives f = sign(z) u / (lam sqrt(z^2 + u^2)),
    monotone in u, so the interval follows from u = o - S and u = o + S.
    """
    if z == 0.0:
        return (-math.inf, math.inf) if abs(o) <= S else (1.0, -1.0)

    def gam(t):
        return t / (lam * math.sqrt(z * z + t * t))

    if z > 0.0:
        return gam(o - S), gam(o + S)
    return -gam(o + S), -gam(o - S)


def band_index_bounds(geo: Geometry):
    """Inclusive integer index bounds ((kx_lo, kx_hi), (ky_lo, ky_hi)) of the
    Rect of Eq. 4, clipped to K.  'full' keeps all of K."""
    Np = geo.Np
    kmin, kmax = -Np // 2, Np // 2 - 1
    if geo.tf != "asm" or geo.band == "full":
        return (kmin, kmax), (kmin, kmax)
    if geo.band == "explicit":
        out = []
        for c, w in zip(geo.band_c, geo.band_w):
            lo = math.ceil(c - w / 2.0)
            hi = math.floor(c + w / 2.0)
            out.append((max(lo, kmin), min(hi, kmax)))
        return tuple(out)
    if geo.band != "limited":
        raise ValueError(geo.band)
    S = geo.N * geo.g
    out = []
    for o in (geo.ox, geo.oy):
        lo, hi = _band_interval(geo.lam, geo.z, o, S)
        klo = -math.inf if math.isinf(lo) else lo / geo.df
        khi = math.inf if math.isinf(hi) else hi / geo.df
        ilo = kmin if math.isinf(klo) else max(math.ceil(klo), kmin)
        ihi = kmax if math.isinf(khi) else min(math.floor(khi), kmax)
        out.append((ilo, ihi))
    return tuple(out)


def band_mask(geo: Geometry) -> np.ndarray:
    """Rect of Eq. 4 on the centred N' x N' frequency grid, [ky][kx]."""
    K = freq_index(geo.Np)
    (xlo, xhi), (ylo, yhi) = band_index_bounds(geo)
    mx = (K >= xlo) & (K <= xhi)
    my = (K >= ylo) & (K <= yhi)
    return my[:, None] & mx[None, :]


# ----------------------------------------------------------- transfer funcs
def transfer_asm(geo: Geometry) -> np.ndarray:
    """Shifted band-limited ASM transfer function, Eq. 4:
    H(k) = Rect(k) exp(2 pi i (df k.o + z sqrt(1/lambda^2 - |k df|^2))),
    zero where the root is imaginary.  [ky][kx], complex128."""
    K = freq_index(geo.Np)
    fx = K[None, :] * geo.df
    fy = K[:, None] * geo.df
    rad = 1.0 / geo.lam ** 2 - (fx * fx + fy * fy)
    prop = rad >= 0.0
    s = np.sqrt(np.where(prop, rad, 0.0))
    cyc = fx * geo.ox + fy * geo.oy + geo.z * s
    H = cis_cycles(cyc)
    H = np.where(prop, H, 0.0)
    return H * band_mask(geo)


def fresnel_axis(geo: Geometry, o: float) -> np.ndarray:
    """One axis of the Fresnel transfer function of Eq. 5 without its
    constant factor: H_1(k) = sum_{m in K} exp(i pi (m g + o)^2/(lambda z))
    exp(-2 pi i k m / N'), as a dense DFT in float64."""
    K = freq_index(geo.Np)
    chirp = ((K * geo.g + o) ** 2) / (2.0 * geo.lam * geo.z)    # cycles
    cyc = chirp[None, :] - np.outer(K, K) / geo.Np              # [k, m]
    return cis_cycles(cyc).sum(axis=1)


def transfer_fresnel(geo: Geometry) -> np.ndarray:
    """Fresnel transfer function, Eq. 5: the DFT over the centred N' x N' grid
    of g^2 exp(i k z)/(i lambda z) exp(i pi |m g + o|^2/(lambda z)).  The
    exponent separates over x and y, so H = A H_y(k_y) H_x(k_x).  [ky][kx]."""
    if geo.z == 0.0:
        raise ValueError("Fresnel transfer function needs z != 0")
    A = geo.g ** 2 * cis_cycles(geo.z / geo.lam) / (1j * geo.lam * geo.z)
    hx = fresnel_axis(geo, geo.ox)
    hy = fresnel_axis(geo, geo.oy)
    return A * hy[:, None] * hx[None, :]


def transfer(geo: Geometry) -> np.ndarray:
    if geo.tf == "asm":
        return transfer_asm(geo)
    if geo.tf == "fresnel":
        return transfer_fresnel(geo)
    raise ValueError(geo.tf)


# ----------------------------------------------------- non-uniform sums
def _pix(v, g):
    return np.asarray(v, dtype=np.float64) / g


def type1_spectrum(geo: Geometry, x, y, c, chunk: int = 8192) -> np.ndarray:
    """Type-1 sum of Eq. 7: F(k) = sum_j c_j exp(-2 pi i df k.p_j), k in K^2,
    for source points p_j = (x_j, y_j) in metres.  [ky][kx], complex128."""
    K = freq_index(geo.Np)
    xp, yp = _pix(x, geo.g), _pix(y, geo.g)
    c = np.asarray(c).astype(np.complex128)
    F = np.zeros((geo.Np, geo.Np), dtype=np.complex128)
    for s in range(0, xp.size, chunk):
        ex = cis_cycles(-np.outer(xp[s:s + chunk], K) / geo.Np)    # [j, kx]
        ey = cis_cycles(-np.outer(yp[s:s + chunk], K) / geo.Np)    # [j, ky]
        F += ey.T @ (c[s:s + chunk, None] * ex)
    return F


def spectrum_at(geo: Geometry, x, y, c, kx, ky) -> np.ndarray:
    """F(k) of Eq. 7 at a list of frequency indices (one by one)."""
    xp, yp = _pix(x, geo.g), _pix(y, geo.g)
    c = np.asarray(c).astype(np.complex128)
    out = np.empty(len(kx), dtype=np.complex128)
    for i, (a, b) in enumerate(zip(kx, ky)):
        out[i] = np.sum(c * cis_cycles(-(a * xp + b * yp) / geo.Np))
    return out


def _type2_eval(geo: Geometry, G: np.ndarray, x, y, chunk: int = 4096) -> np.ndarray:
    """Type-2 sum of Eq. 8: u_j = sum_{k in K^2} G(k) exp(2 pi i df k.q_j)."""
    K = freq_index(geo.Np)
    xp, yp = _pix(x, geo.g), _pix(y, geo.g)
    out = np.empty(xp.size, dtype=np.complex128)
    for s in range(0, xp.size, chunk):
        ax = cis_cycles(np.outer(xp[s:s + chunk], K) / geo.Np)     # [j, kx]
        ay = cis_cycles(np.outer(yp[s:s + chunk], K) / geo.Np)     # [j, ky]
        t = G @ ax.T                                                # [ky, j]
        out[s:s + chunk] = np.einsum("jk,kj->j", ay, t)
    return out


def _centred_idft(Np: int) -> np.ndarray:
    """E[n, k] = exp(+2 pi i n k / N'), n, k in K."""
    K = freq_index(Np)
    return cis_cycles(np.outer(K, K) / Np)


def _source_dft(N: int, Np: int) -> np.ndarray:
    """D[k, m] = exp(-2 pi i k m / N'), k in K, m in {-N/2, ..., N/2 - 1}."""
    K = freq_index(Np)
    m = np.arange(-N // 2, N // 2, dtype=np.float64)
    return cis_cycles(-np.outer(K, m) / Np)


def uniform_spectrum(u1: np.ndarray, Np: int, method: str = "dense") -> np.ndarray:
    """U(k) = sum_m u1[m] exp(-2 pi i k.m / N') of Eq. 9 for a centred N x N
    source, k in K^2, [ky][kx].  'dense' uses DFT matrices; 'fft' uses numpy's
    float64 FFT (a library primitive, for sizes where the dense form is slow)."""
    u1 = np.asarray(u1).astype(np.complex128)
    n = u1.shape[0]
    if method == "dense":
        D = _source_dft(n, Np)
        return D @ u1 @ D.T
    pad = np.zeros((Np, Np), dtype=np.complex128)
    pad[Np // 2 - n // 2:Np // 2 + n // 2, Np // 2 - n // 2:Np // 2 + n // 2] = u1
    return np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(pad)))


def nuasm2_from_spectrum(geo: Geometry, U: np.ndarray, x, y, H: np.ndarray | None = None) -> np.ndarray:
    """NU-ASM_2 (Eq. 9) at the given destination points from a precomputed
    uniform spectrum U (see uniform_spectrum): each output is its own sum."""
    if H is None:
        H = transfer(geo)
    return _type2_eval(geo, H * U / float(geo.Np) ** 2, x, y)


def nuasm1(geo: Geometry, x, y, c, H: np.ndarray | None = None) -> np.ndarray:
    """NU-ASM_1 / NU-FRE_1, Eq. 6: u2 = N'^-2 IDFT[ NUFFT_1[c](k) H(k) ] on the
    centred N' x N' destination grid.  [ny][nx], complex128."""
    if H is None:
        H = transfer(geo)
    F = type1_spectrum(geo, x, y, c)
    E = _centred_idft(geo.Np)
    return (E @ (H * F) @ E.T) / float(geo.Np) ** 2


def nuasm2(geo: Geometry, u1: np.ndarray, x, y, H: np.ndarray | None = None) -> np.ndarray:
    """NU-ASM_2 / NU-FRE_2, Eq. 9: u2_j = N'^-2 NUFFT_2[ DFT[u1] H ](q_j) for an
    N x N uniform source u1 [my][mx] zero-padded to N' x N'.  complex128[M]."""
    if H is None:
        H = transfer(geo)
    u1 = np.asarray(u1).astype(np.complex128)
    n = u1.shape[0]
    D = _source_dft(n, geo.Np)
    U = D @ u1 @ D.T
    return _type2_eval(geo, H * U / float(geo.Np) ** 2, x, y)


def nuasm1_adjoint(geo: Geometry, v: np.ndarray, x, y, H: np.ndarray | None = None) -> np.ndarray:
    """Adjoint of NU-ASM_1 (derived from Eq. 6): w_j = N'^-2 sum_k conj(H)(k)
    V(k) exp(+2 pi i df k.p_j), V the forward DFT of the N' x N' input v."""
    if H is None:
        H = transfer(geo)
    v = np.asarray(v).astype(np.complex128)
    E = _centred_idft(geo.Np)
    V = E.conj() @ v @ E.conj().T
    return _type2_eval(geo, np.conj(H) * V / float(geo.Np) ** 2, x, y)


def nuasm2_adjoint(geo: Geometry, w: np.ndarray, x, y, H: np.ndarray | None = None) -> np.ndarray:
    """Adjoint of NU-ASM_2 (derived from Eq. 9): the N x N plane
    N'^-2 sum_k conj(H)(k) W(k) exp(2 pi i k.m / N') with
    W(k) = sum_j w_j exp(-2 pi i df k.q_j)."""
    if H is None:
        H = transfer(geo)
    W = type1_spectrum(geo, x, y, w)
    D = _source_dft(geo.N, geo.Np)
    Em = D.conj().T                                   # [m, k] = exp(+2 pi i m k/N')
    return (Em @ (np.conj(H) * W) @ Em.T) / float(geo.Np) ** 2


def nuasm3(geo: Geometry, x1, y1, c, x2, y2, H: np.ndarray | None = None) -> np.ndarray:
    """NU-ASM_3 / NU-FRE_3 (the combination of Eqs. 6 and 9 stated after
    Eq. 9): u2_j = N'^-2 sum_{k in K^2} H(k) F(k) exp(+2 pi i df k.q_j) with
    F the type-1 sum of Eq. 7 over the source points p_i = (x1, y1) and
    q_j = (x2, y2) the destination points.  complex128[M2]."""
    if H is None:
        H = transfer(geo)
    F = type1_spectrum(geo, x1, y1, c)
    return _type2_eval(geo, H * F / float(geo.Np) ** 2, x2, y2)


def nuasm3_adjoint(geo: Geometry, w: np.ndarray, x1, y1, x2, y2, H: np.ndarray | None = None) -> np.ndarray:
    """Adjoint of NU-ASM_3: the same operator from the destination points to
    the source points with conj(H).  complex128[M1]."""
    if H is None:
        H = transfer(geo)
    W = type1_spectrum(geo, x2, y2, w)
    return _type2_eval(geo, np.conj(H) * W / float(geo.Np) ** 2, x1, y1)


def grid_points(nx: int, ny: int, pitch: float, cx: float = 0.0, cy: float = 0.0):
    """A uniform nx x ny grid of the given pitch centred at (cx, cy), as
    point coordinates in row-major order: point [b][a] at
    (cx + (a - nx/2) pitch, cy + (b - ny/2) pitch) (integer division)."""
    a = np.arange(nx, dtype=np.float64) - (nx // 2)
    b = np.arange(ny, dtype=np.float64) - (ny // 2)
    X, Y = np.meshgrid(cx + a * pitch, cy + b * pitch, indexing="xy")
    return X.ravel(), Y.ravel()


def scaled_asm(geo: Geometry, u1: np.ndarray, n2: int, d2: float, cx: float = 0.0, cy: float = 0.0,
               H: np.ndarray | None = None) -> np.ndarray:
    """Scaled ASM / Fresnel (destination pitch d2 != source pitch g: the
    scaled diffraction of the introduction, which NU-ASM generalises):
    NU-ASM_2 of the N x N source at the n2 x n2 destination grid of
    pitch d2 centred at (cx, cy).  [n2][n2], complex128."""
    x, y = grid_points(n2, n2, d2, cx, cy)
    return nuasm2(geo, u1, x, y, H).reshape(n2, n2)


# ------------------------------------------------------------ hologram loss
def cgh_loss(geo: Geometry, phi: np.ndarray, x, y, T: np.ndarray, H=None) -> float:
    """L(phi) = sum_j (|u_j|^2 - T_j)^2 with u = NU-ASM_2(exp(i phi))."""
    u = nuasm2(geo, np.exp(1j * np.asarray(phi, dtype=np.float64)), x, y, H)
    r = np.abs(u) ** 2 - T
    return float(np.sum(r * r))


def cgh_grad(geo: Geometry, phi: np.ndarray, x, y, T: np.ndarray, H=None) -> np.ndarray:
    """dL/dphi = 4 Im(G exp(-i phi)), G = NU-ASM_2^H((|u|^2 - T) u)."""
    if H is None:
        H = transfer(geo)
    e = np.exp(1j * np.asarray(phi, dtype=np.float64))
    u = nuasm2(geo, e, x, y, H)
    r = np.abs(u) ** 2 - T
    G = nuasm2_adjoint(geo, r * u, x, y, H)
    return 4.0 * np.imag(G * np.conj(e))


# ----------------------------------------------------- Eq. 10, direct sum
def rayleigh_sommerfeld(u1: np.ndarray, g: float, lam: float, z: float, x2, y2,
                        ox: float = 0.0, oy: float = 0.0) -> np.ndarray:
    """Rayleigh-Sommerfeld diffraction by direct integration, Eq. 10:
    u2(x2) = 1/(2 pi) sum_m u1(x1_m) (z/r)(1 - i k r) exp(i k r)/r^2 g^2 with
    r = sqrt(|x1 - x2|^2 + z^2), for a uniform N x N source of pitch g
    (area element g^2) and destination points at (x2 + ox, y2 + oy)."""
    u1 = np.asarray(u1).astype(np.complex128)
    n = u1.shape[0]
    m = np.arange(-n // 2, n // 2, dtype=np.float64) * g
    X1, Y1 = np.meshgrid(m, m, indexing="xy")
    X1 = X1.ravel()
    Y1 = Y1.ravel()
    a = u1.ravel()
    k = 2.0 * np.pi / lam
    x2 = np.asarray(x2, dtype=np.float64) + ox
    y2 = np.asarray(y2, dtype=np.float64) + oy
    out = np.empty(x2.size, dtype=np.complex128)
    for j in range(x2.size):
        r = np.sqrt((X1 - x2[j]) ** 2 + (Y1 - y2[j]) ** 2 + z * z)
        ph = cis_cycles(r / lam)
        out[j] = np.sum(a * (z / r) * (1.0 - 1j * k * r) * ph / (r * r)) * g * g / (2.0 * np.pi)
    return out


def rayleigh_sommerfeld_points(x1, y1, c, x2, y2, lam: float, z: float,
                               ox: float = 0.0, oy: float = 0.0) -> np.ndarray:
    """Rayleigh-Sommerfeld diffraction by direct summation over source samples
    at arbitrary points (Eq. 10 with the integral replaced by a sum):
    u2_j = 1/(2 pi) sum_i c_i (z/r)(1 - i k r) exp(i k r)/r^2,
    r = sqrt(|q_j + o - p_i|^2 + z^2), k = 2 pi / lambda.  The weights c_i
    carry each sample's area element (g^2 for a uniform grid of pitch g), so a
    uniform grid reproduces rayleigh_sommerfeld.  The phase k r is formed in
    cycles as z/lambda + (r - |z|)/lambda with r - |z| = rho^2/(r + |z|),
    which keeps the large z/lambda out of the rounding of the small part."""
    x1 = np.asarray(x1, dtype=np.float64)
    y1 = np.asarray(y1, dtype=np.float64)
    c = np.asarray(c).astype(np.complex128)
    x2 = np.asarray(x2, dtype=np.float64) + ox
    y2 = np.asarray(y2, dtype=np.float64) + oy
    k = 2.0 * np.pi / lam
    az = abs(z)
    out = np.empty(x2.size, dtype=np.complex128)
    for j in range(x2.size):
        rho2 = (x2[j] - x1) ** 2 + (y2[j] - y1) ** 2
        r = np.sqrt(rho2 + z * z)
        ph = cis_cycles(az / lam + rho2 / (r + az) / lam)
        out[j] = np.sum(c * (z / r) * (1.0 - 1j * k * r) * ph / (r * r)) / (2.0 * np.pi)
    return out


# ------------------------------------------------------------------ metrics
def rel_l2(y, yref) -> float:
    y = np.asarray(y).astype(np.complex128)
    yref = np.asarray(yref).astype(np.complex128)
    return float(np.linalg.norm((y - yref).ravel()) / np.linalg.norm(yref.ravel()))


def snr_db(test, ref) -> float:
    """SNR = 10 log10(sum |ref|^2 / sum |ref - test|^2) (the paper's SNR of
    Figs. 4-5 is not defined in the text; this is the usual reading)."""
    ref = np.asarray(ref).astype(np.complex128)
    test = np.asarray(test).astype(np.complex128)
    return 10.0 * math.log10(np.sum(np.abs(ref) ** 2) / np.sum(np.abs(ref - test) ** 2))
