"""Pins of the FP64 oracle against facts other than itself.

Each test checks the oracle against something it does not compute the same
way: a library FFT (the on-grid special case of Eq. 3), closed forms
(geometric-series energy, the z = 0 Dirichlet kernel, the paraxial limit of
Eq. 2), invariants (integer shifts, the band condition of Eq. 4, adjoint dot
products), brute force (direct spatial convolution with the Fresnel impulse
response of Eq. 5), 50-digit arithmetic, and an independent physical model
(Rayleigh-Sommerfeld direct integration, Eq. 10).
"""
import math

import numpy as np
import pytest

import oracle as O
import synth


def _geo(**kw):
    base = dict(N=16, g=4e-6, lam=633e-9, z=0.01, ox=0.0, oy=0.0, tf="asm", band="full")
    base.update(kw)
    return O.Geometry(**base)


def _dirichlet(d, Np):
    """sum_{k=-Np/2}^{Np/2-1} exp(-2 pi i k d / Np), closed form of the
    geometric series (d in pixels, any real)."""
    d = np.asarray(d, dtype=np.float64)
    out = np.empty(d.shape, dtype=np.complex128)
    near = np.abs(np.sin(np.pi * d / Np)) < 1e-300
    dn = d[~near]
    out[~near] = np.exp(1j * np.pi * dn / Np) * np.sin(np.pi * dn) / np.sin(np.pi * dn / Np)
    out[near] = Np * np.cos(np.pi * d[near])  # d = multiple of Np
    return out


# ----------------------------------------------------------- transfer funcs
@pytest.mark.parametrize("z", [0.01, 0.5, 1.0])
def test_asm_transfer_matches_50_digit_arithmetic(z):
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    geo = _geo(N=1024, g=4e-6, lam=532e-9, z=z, ox=1e-3, oy=-2e-4)
    H = O.transfer_asm(geo)
    rng = np.random.default_rng(7)
    idx = rng.integers(0, geo.Np, size=(300, 2))
    K = O.freq_index(geo.Np)
    err = 0.0
    for a, b in idx:
        kx, ky = K[b], K[a]
        fx = mp.mpf(int(kx)) / (geo.Np * mp.mpf(geo.g))
        fy = mp.mpf(int(ky)) / (geo.Np * mp.mpf(geo.g))
        ph = 2 * mp.pi * (fx * mp.mpf(geo.ox) + fy * mp.mpf(geo.oy)
                          + mp.mpf(z) * mp.sqrt(1 / mp.mpf(geo.lam) ** 2 - fx * fx - fy * fy))
        ref = complex(mp.cos(ph), mp.sin(ph))
        err = max(err, abs(H[a, b] - ref))
    # float64 forms z*sqrt(.) ~ z/lambda cycles before reducing them mod 1: a
    # few roundings of relative size 2^-53 on that many cycles bound the error
    bound = 2 * np.pi * 16 * 2.0 ** -53 * (abs(z) / geo.lam + 1.0)
    assert err < bound


def test_asm_transfer_paraxial_limit():
    """Near k = 0, sqrt(1/l^2 - f^2) = 1/l - l f^2/2 - l^3 f^4/8 - ...; the
    oracle must agree with the paraxial phase up to the quartic remainder."""
    geo = _geo(N=1024, g=4e-6, lam=633e-9, z=0.3, ox=2e-4, oy=1e-4)
    H = O.transfer_asm(geo)
    K = O.freq_index(geo.Np)
    c = geo.Np // 2
    for kx in range(-20, 21, 5):
        for ky in range(-20, 21, 4):
            fx, fy = kx * geo.df, ky * geo.df
            f2 = fx * fx + fy * fy
            par = 2 * np.pi * (fx * geo.ox + fy * geo.oy + geo.z / geo.lam
                               - geo.lam * geo.z * f2 / 2.0)
            bound = 2 * np.pi * 1.01 * geo.z * geo.lam ** 3 * f2 * f2 / 8.0 + 1e-9
            assert K[ky + c] == ky and K[kx + c] == kx
            assert abs(H[ky + c, kx + c] - np.exp(1j * par)) <= bound


@pytest.mark.parametrize("z,ox,oy", [(0.1, 1e-3, 0.0), (0.5, 1e-3, 0.0), (-0.2, 3e-4, -5e-4),
                                     (0.01, 1e-3, 0.0), (1.0, 0.0, 0.0)])
def test_band_edges_satisfy_local_frequency_condition(z, ox, oy):
    """Band of Eq. 4 (reading: |o - z f/s(f)| <= S per axis, S = N g).  The
    inequality is evaluated directly at the integer bounds and one past them."""
    geo = _geo(N=1024, g=4e-6, lam=633e-9, z=z, ox=ox, oy=oy, band="limited")
    S = geo.N * geo.g
    kmin, kmax = -geo.Np // 2, geo.Np // 2 - 1

    def ok(k, o):
        f = k * geo.df
        s = math.sqrt(1.0 / geo.lam ** 2 - f * f)
        return abs(o - geo.z * f / s) <= S * (1 + 1e-12)

    for (lo, hi), o in zip(O.band_index_bounds(geo), (ox, oy)):
        assert lo <= hi
        assert ok(lo, o) and ok(hi, o)
        if lo > kmin:
            assert not ok(lo - 1, o)
        if hi < kmax:
            assert not ok(hi + 1, o)
        mid = (lo + hi) // 2
        assert ok(mid, o)


# explicit Rect of Eq. 4: (centre, width) pairs in index units, chosen so that
# every comparison below is exact in binary floating point
EXPLICIT_CASES = [
    ((10.5, -3.0), (40.0, 61.0)),     # half-integer centre, odd width: both edges on K
    ((10.5, 2.25), (3.0, 0.5)),       # edges exactly at +-1.5 and +-0.25 from the centre
    ((7.0, -4.0), (0.0, 0.0)),        # w = 0 at an integer centre: one index per axis
    ((7.5, -4.25), (0.0, 0.0)),       # w = 0 off the integers: empty
    ((30.0, -29.5), (20.0, 9.0)),     # crosses the top (x) and the bottom (y) of K: clipped
    ((-3.75, 0.0), (200.0, 1.0)),     # wider than K on x
]


@pytest.mark.parametrize("c,w", EXPLICIT_CASES)
def test_explicit_band_is_the_closed_interval_around_the_centre(c, w):
    """Explicit band of Eq. 4: per axis k is kept iff |k - c| <= w/2 (edges
    inclusive), clipped to K.  Checked index by index against that
    inequality, not through the ceil/floor bounds the oracle computes."""
    geo = _geo(N=32, band="explicit", band_c=c, band_w=w)
    K = O.freq_index(geo.Np)
    mask = O.band_mask(geo)
    for axis in (0, 1):
        keep = np.array([abs(k - c[axis]) <= 0.5 * w[axis] for k in K])
        got = mask.any(axis=0) if axis == 0 else mask.any(axis=1)
        assert np.array_equal(got, keep), (axis, c, w)
    # the mask is the outer product of the two axes
    keep_x = np.array([abs(k - c[0]) <= 0.5 * w[0] for k in K])
    keep_y = np.array([abs(k - c[1]) <= 0.5 * w[1] for k in K])
    assert np.array_equal(mask, keep_y[:, None] & keep_x[None, :])
    if w == (0.0, 0.0) and float(c[0]).is_integer() and float(c[1]).is_integer():
        assert mask.sum() == 1


def _local_frequency_edge(geo, o, target):
    """Frequency f (m^-1) where the local spatial frequency of H's phase,
    o - z f / s(f), equals `target`, by bisection on the monotone map
    f -> z f / s(f) (an independent route to the closed-form edges)."""
    lo, hi = -0.999999 / geo.lam, 0.999999 / geo.lam

    def u(f):
        return geo.z * f / math.sqrt(1.0 / geo.lam ** 2 - f * f)

    want = o - target
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if (u(mid) < want) == (geo.z > 0):
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


@pytest.mark.parametrize("z,ox,oy", [(0.1, 1e-3, 0.0), (0.5, -1e-3, 2e-4), (-0.2, 3e-4, -5e-4),
                                     (0.3, -7.3e-4, 6.1e-4)])
def test_explicit_band_from_limited_edges_reproduces_limited_mask(z, ox, oy):
    """The limited band of Eq. 4 written as an explicit (c, w) pair: the band
    edges f_lo, f_hi (where the local frequency reaches +-S) give
    c = (f_lo + f_hi) / (2 df) and w = (f_hi - f_lo) / df.  An explicit plan
    with that centre and width must keep exactly the limited plan's
    frequencies on both axes, for offsets of both signs and both signs of z."""
    base = dict(N=1024, g=4e-6, lam=633e-9, z=z, ox=ox, oy=oy)
    lim = _geo(band="limited", **base)
    S = lim.N * lim.g
    cs, ws = [], []
    for o in (ox, oy):
        f1 = _local_frequency_edge(lim, o, S)
        f2 = _local_frequency_edge(lim, o, -S)
        flo, fhi = min(f1, f2), max(f1, f2)
        # the edges must not sit on an integer index (a rounding there could
        # legitimately flip a boundary frequency)
        for f in (flo, fhi):
            assert abs(f / lim.df - round(f / lim.df)) > 1e-6
        cs.append((flo + fhi) / (2.0 * lim.df))
        ws.append((fhi - flo) / lim.df)
    exp = _geo(band="explicit", band_c=tuple(cs), band_w=tuple(ws), **base)
    assert np.array_equal(O.band_mask(exp), O.band_mask(lim))
    assert O.band_index_bounds(exp) == O.band_index_bounds(lim)


def test_fresnel_separable_equals_direct_2d_dft():
    geo = _geo(N=8, g=5e-6, lam=500e-9, z=0.002, ox=7e-6, oy=-3e-6, tf="fresnel")
    H = O.transfer_fresnel(geo)
    K = O.freq_index(geo.Np)
    k = 2 * np.pi / geo.lam
    MX, MY = np.meshgrid(K, K, indexing="xy")
    h = (geo.g ** 2 * np.exp(1j * k * geo.z) / (1j * geo.lam * geo.z)
         * np.exp(1j * np.pi * ((MX * geo.g + geo.ox) ** 2 + (MY * geo.g + geo.oy) ** 2)
                  / (geo.lam * geo.z)))
    ref = np.zeros_like(H)
    for a, ky in enumerate(K):
        for b, kx in enumerate(K):
            ref[a, b] = np.sum(h * np.exp(-2j * np.pi * (kx * MX + ky * MY) / geo.Np))
    assert np.max(np.abs(H - ref)) <= 1e-11 * np.max(np.abs(ref))


def _fresnel_h(geo, dx, dy):
    """Fresnel impulse response exp(ikz)/(i l z) exp(i pi |x|^2/(l z)) at (dx, dy)."""
    k = 2 * np.pi / geo.lam
    return (np.exp(1j * k * geo.z) / (1j * geo.lam * geo.z)
            * np.exp(1j * np.pi * (dx * dx + dy * dy) / (geo.lam * geo.z)))


def test_nufre2_on_grid_equals_direct_fresnel_convolution():
    """NU-FRE_2 at destinations on the pixel grid is the linear convolution
    sum_m u1[m] g^2 h((n - m) g + o) (zero padding to N' = 2N removes the wrap)."""
    geo = _geo(N=8, g=5e-6, lam=500e-9, z=0.003, ox=6e-6, oy=-4e-6, tf="fresnel")
    rng = np.random.default_rng(11)
    u1 = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    n = np.arange(-4, 4)
    NX, NY = np.meshgrid(n, n, indexing="xy")
    sel = rng.permutation(64)[:40]
    qx, qy = NX.ravel()[sel], NY.ravel()[sel]
    got = O.nuasm2(geo, u1, qx * geo.g, qy * geo.g)
    ref = np.zeros(sel.size, dtype=np.complex128)
    for j in range(sel.size):
        for my in range(8):
            for mx in range(8):
                dx = (qx[j] - (mx - 4)) * geo.g + geo.ox
                dy = (qy[j] - (my - 4)) * geo.g + geo.oy
                ref[j] += u1[my, mx] * geo.g ** 2 * _fresnel_h(geo, dx, dy)
    # the brute force evaluates exp(i k z) unreduced (k z ~ 4e4 rad), so its own
    # rounding is ~ 4e4 * 2^-53 per term
    assert O.rel_l2(got, ref) < 1e-10


def test_nufre1_on_grid_equals_direct_fresnel_convolution():
    geo = _geo(N=8, g=5e-6, lam=500e-9, z=0.004, ox=-5e-6, oy=2e-6, tf="fresnel")
    rng = np.random.default_rng(12)
    M = 25
    mx = rng.integers(-4, 4, size=M)
    my = rng.integers(-4, 4, size=M)
    c = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    u2 = O.nuasm1(geo, mx * geo.g, my * geo.g, c)
    # central N x N of the N' x N' output has no circular wrap
    ref = np.zeros((8, 8), dtype=np.complex128)
    for b in range(8):
        for a in range(8):
            nx, ny = a - 4, b - 4
            dx = (nx - mx) * geo.g + geo.ox
            dy = (ny - my) * geo.g + geo.oy
            ref[b, a] = np.sum(c * geo.g ** 2 * _fresnel_h(geo, dx, dy))
    got = u2[4:12, 4:12]
    assert O.rel_l2(got, ref) < 1e-10


# ------------------------------------------- on-grid reduction to Eq. 3
def _fft_asm_full(H, img):
    """Eq. 3 with numpy's FFT on a centred N' x N' array."""
    X = np.fft.fft2(np.fft.ifftshift(img))
    return np.fft.fftshift(np.fft.ifft2(X * np.fft.ifftshift(H)))


@pytest.mark.parametrize("tf,band,z", [("asm", "full", 0.01), ("asm", "limited", 0.02),
                                       ("fresnel", "full", 0.005)])
def test_nuasm2_on_grid_equals_fft_asm(tf, band, z):
    geo = _geo(N=16, g=4e-6, lam=633e-9, z=z, ox=3e-5, oy=-1e-5, tf=tf, band=band)
    rng = np.random.default_rng(21)
    u1 = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    H = O.transfer(geo)
    img = np.zeros((geo.Np, geo.Np), dtype=np.complex128)
    img[8:24, 8:24] = u1
    ref = _fft_asm_full(H, img)
    # destinations: a shuffled subset of the N' x N' grid (x != y pattern)
    nx = rng.integers(-16, 16, size=60)
    ny = rng.integers(-16, 16, size=60)
    got = O.nuasm2(geo, u1, nx * geo.g, ny * geo.g, H)
    assert O.rel_l2(got, ref[ny + 16, nx + 16]) < 1e-13


@pytest.mark.parametrize("tf,band,z", [("asm", "full", 0.01), ("asm", "limited", 0.05),
                                       ("fresnel", "full", 0.01)])
def test_nuasm1_on_grid_equals_fft_asm(tf, band, z):
    geo = _geo(N=16, g=4e-6, lam=633e-9, z=z, ox=-2e-5, oy=1e-5, tf=tf, band=band)
    rng = np.random.default_rng(22)
    M = 50
    mx = rng.integers(-8, 8, size=M)
    my = rng.integers(-8, 8, size=M)
    c = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    H = O.transfer(geo)
    img = np.zeros((geo.Np, geo.Np), dtype=np.complex128)
    np.add.at(img, (my + 16, mx + 16), c)           # duplicate points add
    ref = _fft_asm_full(H, img)
    got = O.nuasm1(geo, mx * geo.g, my * geo.g, c, H)
    assert O.rel_l2(got, ref) < 1e-13


# ------------------------------------------------------------ closed forms
@pytest.mark.parametrize("z,ox", [(0.01, 0.0), (0.3, 2e-4), (-0.05, -1e-4)])
def test_nuasm1_energy_closed_form(z, ox):
    """Full band, |H| = 1: sum_n |u2|^2 = N'^-2 sum_{j,l} c_j conj(c_l)
    D(x_j - x_l) D(y_j - y_l), D the Dirichlet kernel over K."""
    geo = _geo(N=16, g=4e-6, z=z, ox=ox, oy=1e-5)
    rng = np.random.default_rng(31)
    M = 40
    x, y = synth.uniform_box(rng, M, geo.N * geo.g)
    c = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    u2 = O.nuasm1(geo, x, y, c)
    xp, yp = x / geo.g, y / geo.g
    Dx = _dirichlet(xp[:, None] - xp[None, :], geo.Np)
    Dy = _dirichlet(yp[:, None] - yp[None, :], geo.Np)
    ref = np.real(np.sum(c[:, None] * np.conj(c)[None, :] * Dx * Dy)) / geo.Np ** 2
    assert abs(np.sum(np.abs(u2) ** 2) - ref) <= 1e-12 * ref


def test_nuasm1_z0_is_dirichlet_interpolation_at_offset_window():
    """z = 0, full band: H = exp(2 pi i df k.o) and the output sample n sits at
    n g + o, so u2[n] = N'^-2 sum_j c_j conj(D)(n + o/g - p_j) per axis."""
    geo = _geo(N=8, g=4e-6, z=0.0, ox=1.3e-6, oy=-2.9e-6)
    rng = np.random.default_rng(41)
    M = 12
    x, y = synth.uniform_box(rng, M, geo.N * geo.g)
    c = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    u2 = O.nuasm1(geo, x, y, c)
    K = O.freq_index(geo.Np)
    ref = np.zeros_like(u2)
    for b, ny in enumerate(K):
        for a, nx in enumerate(K):
            dx = nx + geo.ox / geo.g - x / geo.g
            dy = ny + geo.oy / geo.g - y / geo.g
            ref[b, a] = np.sum(c * np.conj(_dirichlet(dx, geo.Np)) * np.conj(_dirichlet(dy, geo.Np)))
    ref /= geo.Np ** 2
    assert O.rel_l2(u2, ref) < 1e-12


def test_nuasm1_integer_shift_rolls_output():
    geo = _geo(N=16, g=4e-6, z=0.02, ox=1e-5, band="limited")
    rng = np.random.default_rng(51)
    M = 30
    x, y = synth.uniform_box(rng, M, 0.5 * geo.N * geo.g)
    c = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    H = O.transfer(geo)
    u = O.nuasm1(geo, x, y, c, H)
    dx, dy = 3, -2
    v = O.nuasm1(geo, x + dx * geo.g, y + dy * geo.g, c, H)
    assert O.rel_l2(v, np.roll(u, (dy, dx), axis=(0, 1))) < 1e-12


# --------------------------------------- Rayleigh-Sommerfeld (Eq. 10) pin
def _gauss_src(X, Y, w0=8e-6):
    return np.exp(-(X ** 2 + Y ** 2) / (2 * w0 ** 2)) * np.exp(2j * np.pi * (2.5e4 * X + 1.0e4 * Y))


@pytest.mark.parametrize("z", [50e-6, 100e-6])
def test_nuasm2_matches_rayleigh_sommerfeld(z):
    """A resolved Gaussian beam well inside the window: the oracle's NU-ASM_2
    equals direct RS integration of the same analytic source (sampled 8x finer)
    at off-grid destinations, and the sign of z matters."""
    N, g, lam = 32, 2e-6, 633e-9
    m = np.arange(-N // 2, N // 2) * g
    u1 = _gauss_src(*np.meshgrid(m, m, indexing="xy"))
    rng = np.random.default_rng(3)
    xq = rng.uniform(-N * g / 4, N * g / 4, 48)
    yq = rng.uniform(-N * g / 4, N * g / 4, 48)
    gf, n = g / 8, 320
    mf = np.arange(-n // 2, n // 2) * gf
    src = _gauss_src(*np.meshgrid(mf, mf, indexing="xy"))
    ox, oy = 3e-6, -2e-6
    ref = O.rayleigh_sommerfeld(src, gf, lam, z, xq, yq, ox, oy)
    got = O.nuasm2(O.Geometry(N=N, g=g, lam=lam, z=z, ox=ox, oy=oy), u1, xq, yq)
    assert O.rel_l2(got, ref) < 1e-4
    wrong = O.nuasm2(O.Geometry(N=N, g=g, lam=lam, z=-z, ox=ox, oy=oy), u1, xq, yq)
    assert O.rel_l2(wrong, ref) > 0.1


def test_rs_points_on_a_grid_equals_uniform_rs():
    """The point-set form of Eq. 10 with the samples of a uniform grid and
    weights u1 g^2 is the uniform-grid integral (whose phase is evaluated
    directly as k r, not split into z/lambda + (r - |z|)/lambda)."""
    N, g, lam, z = 16, 5e-6, 500e-9, 0.004
    rng = np.random.default_rng(13)
    u1 = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    m = np.arange(-N // 2, N // 2) * g
    X, Y = np.meshgrid(m, m, indexing="xy")
    x2 = rng.uniform(-N * g / 2, N * g / 2, 30)
    y2 = rng.uniform(-N * g / 2, N * g / 2, 30)
    ox, oy = 7e-6, -3e-6
    ref = O.rayleigh_sommerfeld(u1, g, lam, z, x2, y2, ox, oy)
    got = O.rayleigh_sommerfeld_points(X.ravel(), Y.ravel(), u1.ravel() * g * g, x2, y2, lam, z, ox, oy)
    # the uniform form rounds k r ~ 5e4 rad unreduced: ~1e-11 relative
    assert O.rel_l2(got, ref) < 1e-10


def test_rs_points_reciprocity():
    """The kernel depends on |q + o - p| only, so exchanging the source and
    destination sets (and negating the offset) transposes the operator:
    w . RS(p -> q) c = c . RS(q -> p) w, without conjugation."""
    rng = np.random.default_rng(14)
    lam, z, W = 633e-9, 0.002, 1e-4
    x1, y1 = synth.clustered_box(rng, 23, W)
    x2, y2 = synth.uniform_box(rng, 19, W)
    c = rng.standard_normal(23) + 1j * rng.standard_normal(23)
    w = rng.standard_normal(19) + 1j * rng.standard_normal(19)
    ox, oy = 4e-6, 9e-6
    a = np.dot(w, O.rayleigh_sommerfeld_points(x1, y1, c, x2, y2, lam, z, ox, oy))
    b = np.dot(c, O.rayleigh_sommerfeld_points(x2, y2, w, x1, y1, lam, z, -ox, -oy))
    assert abs(a - b) <= 1e-12 * abs(a)
    # a sign slip in the offset breaks it
    b2 = np.dot(c, O.rayleigh_sommerfeld_points(x2, y2, w, x1, y1, lam, z, ox, oy))
    assert abs(a - b2) > 1e-3 * abs(a)


# -------------------------------------------------------------- adjoints
@pytest.mark.parametrize("tf,band", [("asm", "limited"), ("asm", "full"), ("fresnel", "full")])
def test_adjoint_dot_products(tf, band):
    geo = _geo(N=8, z=0.002, ox=1e-5, oy=-4e-6, tf=tf, band=band)
    rng = np.random.default_rng(61)
    M = 37
    x, y = synth.clustered_box(rng, M, geo.N * geo.g)
    c = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    v = rng.standard_normal((geo.Np, geo.Np)) + 1j * rng.standard_normal((geo.Np, geo.Np))
    lhs = np.vdot(v, O.nuasm1(geo, x, y, c))
    rhs = np.vdot(O.nuasm1_adjoint(geo, v, x, y), c)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    u1 = rng.standard_normal((geo.N, geo.N)) + 1j * rng.standard_normal((geo.N, geo.N))
    w = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    lhs = np.vdot(w, O.nuasm2(geo, u1, x, y))
    rhs = np.vdot(O.nuasm2_adjoint(geo, w, x, y), u1)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_cgh_gradient_matches_central_differences():
    geo = _geo(N=8, g=4e-6, lam=532e-9, z=0.001, band="limited")
    rng = np.random.default_rng(71)
    M = 30
    x, y = synth.three_clusters(rng, M, geo.N * geo.g)
    phi = rng.uniform(0, 2 * np.pi, size=(8, 8))
    H = O.transfer(geo)
    u0 = O.nuasm2(geo, np.exp(1j * phi), x, y, H)
    T = 0.5 * np.abs(u0) ** 2 + 0.1 * rng.uniform(size=M) * np.mean(np.abs(u0) ** 2)
    g = O.cgh_grad(geo, phi, x, y, T, H)
    eps = 1e-6
    for (a, b) in [(0, 0), (3, 5), (7, 7), (4, 1), (6, 2)]:
        p = phi.copy()
        p[a, b] += eps
        lp = O.cgh_loss(geo, p, x, y, T, H)
        p[a, b] -= 2 * eps
        lm = O.cgh_loss(geo, p, x, y, T, H)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[a, b]) <= 1e-6 * np.max(np.abs(g))


def test_spectrum_at_matches_fft_of_z0_output():
    """F(k) at single frequencies (used for full-size sampled checks) equals the
    numpy FFT of the z = 0, o = 0, full-band NU-ASM_1 output (H = 1)."""
    geo = _geo(N=8, z=0.0)
    rng = np.random.default_rng(81)
    M = 20
    x, y = synth.uniform_box(rng, M, geo.N * geo.g)
    c = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    u2 = O.nuasm1(geo, x, y, c)
    F = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(u2)))
    kx = rng.integers(-8, 8, size=10)
    ky = rng.integers(-8, 8, size=10)
    got = O.spectrum_at(geo, x, y, c, kx, ky)
    assert O.rel_l2(got, F[ky + 8, kx + 8]) < 1e-12


def test_uniform_spectrum_fft_path_equals_dense_dft():
    rng = np.random.default_rng(91)
    u1 = rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16))
    a = O.uniform_spectrum(u1, 32, "dense")
    b = O.uniform_spectrum(u1, 32, "fft")
    assert O.rel_l2(b, a) < 1e-13
    geo = _geo(N=16, z=0.02, band="limited", ox=1e-5)
    x, y = synth.uniform_box(rng, 20, geo.N * geo.g)
    assert O.rel_l2(O.nuasm2_from_spectrum(geo, b, x, y), O.nuasm2(geo, u1, x, y)) < 1e-12


# ------------------------------------------------- the paper's experiment set-up
def test_paper_experiment_nuasm2_reaches_reported_snr():
    """NU-ASM_2 on the paper's experiment geometry (tests/golden/
    paper_experiment.json: 500 nm, 5 um uniform pitch, quadrant-wise
    0.9/0.8/0.7/1.0 destination sampling, z = 8 mm) against Rayleigh-Sommerfeld
    direct integration (Eq. 10) reaches at least the SNR the paper reports.
    The photographs the paper uses are absent; the source is a smooth
    amplitude with phase in [-pi/2, pi/2] (the paper's phase range), on a
    64 x 64 plane instead of 256 x 256 to keep the O(N^4) integral short."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_experiment.json")) as f:
        ex = json.load(f)
    N, lam, d, z = 64, ex["lambda_m"], ex["pitch_m"], ex["z_m"]
    n = np.arange(N) - N / 2
    X, Y = np.meshgrid(n, n)
    amp = np.exp(-(X ** 2 + Y ** 2) / (2 * (N / 5) ** 2))
    ph = (np.pi / 2) * np.sin(2 * np.pi * X / N) * np.cos(2 * np.pi * Y / N)
    u1 = amp * np.exp(1j * ph)
    x, y = synth.quadrant_grid(N, d, tuple(ex["quadrant_factors"]))
    geo = O.Geometry(N=N, g=d, lam=lam, z=z, tf="asm", band="limited")
    u2 = O.nuasm2(geo, u1, x, y, O.transfer(geo))
    ref = O.rayleigh_sommerfeld(u1, d, lam, z, x, y)
    assert O.snr_db(u2, ref) >= ex["snr_db_reported"]
    # the same comparison with z -> -z (wrong propagation direction) fails
    geo_m = O.Geometry(N=N, g=d, lam=lam, z=-z, tf="asm", band="limited")
    assert O.snr_db(O.nuasm2(geo_m, u1, x, y, O.transfer(geo_m)), ref) < 10.0


# ------------------------------------------------- NU-ASM_3 / NU-FRE_3 pins
@pytest.mark.parametrize("tf,band,z", [("asm", "full", 0.01), ("asm", "limited", 0.04),
                                       ("fresnel", "full", 0.006)])
def test_nuasm3_on_grid_equals_fft_asm(tf, band, z):
    """Sources on the N x N pixel grid and destinations on the N' x N' grid:
    the composition is Eq. 3 with numpy's FFT, sampled at the destinations."""
    geo = _geo(N=16, g=4e-6, lam=633e-9, z=z, ox=1.5e-5, oy=-2.5e-5, tf=tf, band=band)
    rng = np.random.default_rng(71)
    M1, M2 = 45, 55
    mx = rng.integers(-8, 8, size=M1)
    my = rng.integers(-8, 8, size=M1)
    c = rng.standard_normal(M1) + 1j * rng.standard_normal(M1)
    H = O.transfer(geo)
    img = np.zeros((geo.Np, geo.Np), dtype=np.complex128)
    np.add.at(img, (my + 16, mx + 16), c)
    ref = _fft_asm_full(H, img)
    nx = rng.integers(-16, 16, size=M2)
    ny = rng.integers(-16, 16, size=M2)
    got = O.nuasm3(geo, mx * geo.g, my * geo.g, c, nx * geo.g, ny * geo.g, H)
    assert O.rel_l2(got, ref[ny + 16, nx + 16]) < 1e-13


def test_nuasm3_z0_is_dirichlet_kernel_between_point_sets():
    """z = 0, full band: H = exp(2 pi i df k.o), so per axis
    u2_j = N'^-2 sum_i c_i conj(D)(q_j + o/g - p_i) with D the closed-form
    Dirichlet kernel over K; both point sets off the grid."""
    geo = _geo(N=8, g=4e-6, z=0.0, ox=2.3e-6, oy=-1.1e-6)
    rng = np.random.default_rng(72)
    x1, y1 = synth.uniform_box(rng, 14, geo.N * geo.g)
    x2, y2 = synth.clustered_box(rng, 17, geo.N * geo.g)
    c = rng.standard_normal(14) + 1j * rng.standard_normal(14)
    got = O.nuasm3(geo, x1, y1, c, x2, y2)
    ref = np.empty(17, dtype=np.complex128)
    for j in range(17):
        dx = (x2[j] + geo.ox - x1) / geo.g
        dy = (y2[j] + geo.oy - y1) / geo.g
        ref[j] = np.sum(c * np.conj(_dirichlet(dx, geo.Np)) * np.conj(_dirichlet(dy, geo.Np)))
    ref /= geo.Np ** 2
    assert O.rel_l2(got, ref) < 1e-12


def test_nuasm3_common_shift_leaves_output_unchanged():
    """Only q_j - p_i enters: moving both point sets by the same non-integer
    amount changes nothing (a sign slip in either sum breaks this)."""
    geo = _geo(N=16, g=4e-6, z=0.03, ox=1e-5, band="limited")
    rng = np.random.default_rng(73)
    half = 0.35 * geo.N * geo.g
    x1, y1 = synth.uniform_box(rng, 30, half)
    x2, y2 = synth.uniform_box(rng, 25, half)
    c = rng.standard_normal(30) + 1j * rng.standard_normal(30)
    H = O.transfer(geo)
    u = O.nuasm3(geo, x1, y1, c, x2, y2, H)
    dx, dy = 2.37 * geo.g, -1.61 * geo.g
    v = O.nuasm3(geo, x1 + dx, y1 + dy, c, x2 + dx, y2 + dy, H)
    assert O.rel_l2(v, u) < 1e-12


def test_nuasm3_reduces_to_types_1_and_2():
    """Destinations on the N' grid give NU-ASM_1's samples; sources on the
    N x N grid give NU-ASM_2 of the corresponding image."""
    geo = _geo(N=8, g=5e-6, lam=500e-9, z=0.004, ox=-3e-6, oy=7e-6, tf="fresnel")
    rng = np.random.default_rng(74)
    x1, y1 = synth.clustered_box(rng, 21, geo.N * geo.g)
    c = rng.standard_normal(21) + 1j * rng.standard_normal(21)
    H = O.transfer(geo)
    nx = rng.integers(-8, 8, size=30)
    ny = rng.integers(-8, 8, size=30)
    u1 = O.nuasm1(geo, x1, y1, c, H)
    got = O.nuasm3(geo, x1, y1, c, nx * geo.g, ny * geo.g, H)
    assert O.rel_l2(got, u1[ny + 8, nx + 8]) < 1e-13
    img = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    px, py = np.meshgrid(np.arange(-4, 4), np.arange(-4, 4), indexing="xy")
    x2, y2 = synth.uniform_box(rng, 19, geo.N * geo.g)
    got = O.nuasm3(geo, px.ravel() * geo.g, py.ravel() * geo.g, img.ravel(), x2, y2, H)
    assert O.rel_l2(got, O.nuasm2(geo, img, x2, y2, H)) < 1e-13


@pytest.mark.parametrize("tf,band", [("asm", "limited"), ("fresnel", "full")])
def test_nuasm3_adjoint_dot_product(tf, band):
    geo = _geo(N=8, z=0.002, ox=1e-5, oy=-4e-6, tf=tf, band=band)
    rng = np.random.default_rng(75)
    x1, y1 = synth.clustered_box(rng, 29, geo.N * geo.g)
    x2, y2 = synth.uniform_box(rng, 33, geo.N * geo.g)
    c = rng.standard_normal(29) + 1j * rng.standard_normal(29)
    w = rng.standard_normal(33) + 1j * rng.standard_normal(33)
    lhs = np.vdot(w, O.nuasm3(geo, x1, y1, c, x2, y2))
    rhs = np.vdot(O.nuasm3_adjoint(geo, w, x1, y1, x2, y2), c)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


# ------------------------------------------------------------- scaled ASM
def _chirp_z_axis(G, alpha, beta, n2, axis):
    """sum_k G[.., k, ..] exp(2 pi i k ((m - n2/2) alpha + beta) / N') along
    `axis` for m = 0..n2-1, by Bluestein's chirp-z identity
    k m = (k^2 + m^2 - (k - m)^2) / 2: a chirp-weighted linear correlation
    evaluated with FFT convolution (an O(N log N) method the oracle's direct
    sums do not use)."""
    from scipy.signal import fftconvolve
    G = np.moveaxis(np.asarray(G, dtype=np.complex128), axis, -1)
    Np = G.shape[-1]
    K = np.arange(-Np // 2, Np // 2, dtype=np.float64)
    Mp = np.arange(n2, dtype=np.float64) - n2 // 2
    w = lambda t: np.exp(1j * np.pi * alpha * t * t / Np)
    a = G * np.exp(2j * np.pi * K * beta / Np) * w(K)
    tmin = K[0] - Mp[-1]
    t = np.arange(tmin, K[-1] - Mp[0] + 1)
    b = np.conj(w(t))
    # c(m) = sum_j a[j] b[j + s(m)], s(m) = K0 - tmin - m, as a convolution with reversed a
    conv = fftconvolve(a[..., ::-1], np.broadcast_to(b, a.shape[:-1] + b.shape), axes=-1)
    s = (K[0] - tmin - Mp).astype(int)
    out = conv[..., Np - 1 + s] * w(Mp)
    return np.moveaxis(out, -1, axis)


@pytest.mark.parametrize("tf,band", [("asm", "limited"), ("fresnel", "full")])
def test_scaled_asm_equals_chirp_z_evaluation(tf, band):
    """Scaled diffraction (d2 != g) through NU-ASM_2 at a uniform destination
    grid equals the same spectral sum evaluated per axis by the chirp-z
    transform (Bluestein), the method the scaled-ASM literature uses."""
    geo = _geo(N=32, g=4e-6, lam=633e-9, z=0.006, ox=2e-5, oy=-1e-5, tf=tf, band=band)
    rng = np.random.default_rng(101)
    u1 = rng.standard_normal((32, 32)) + 1j * rng.standard_normal((32, 32))
    n2, d2 = 40, 0.6 * geo.g
    cx, cy = 3.1 * geo.g, -2.2 * geo.g
    got = O.scaled_asm(geo, u1, n2, d2, cx, cy)
    G = O.transfer(geo) * O.uniform_spectrum(u1, geo.Np, "fft") / geo.Np ** 2    # [ky][kx]
    alpha = d2 / geo.g
    A = _chirp_z_axis(G, alpha, cx / geo.g, n2, axis=1)                           # [ky][mx]
    ref = _chirp_z_axis(A, alpha, cy / geo.g, n2, axis=0)                          # [my][mx]
    assert O.rel_l2(got, ref) < 1e-11
