// Grid passes of the two pipelines on gfx950: pruned row FFTs, the fused
// column pass (FFT -> deconvolution x transfer function x Rect -> inverse FFT),
// and the final row passes.  Every 1-D transform lives in LDS (Stockham,
// radix 8 with a 4/2 tail); HBM is touched once per pass.
//
// Index conventions (centred, as in Eqs. 3, 6 and 9): a plane element [b][a]
// of an N' x N' array holds n = (a - N'/2, b - N'/2); frequency k = a - N'/2.
// The non-uniform sums run on the spectral grid K'' of N'' modes (N'' = N',
// or smaller when the band of Eq. 4 is narrow) and a fine grid of nf = 2 N''
// cells per axis; the non-uniform window occupies fine cells
// [N''/2, 3N''/2), and only the support rows/columns [s0, s0 + L),
// L = N'' + 16, are ever stored.  Row passes over the fine grid are
// instantiated at N''; the column passes go between N'' and N'.
#include "group.h"
#include "launch.h"

namespace nuasm {

// Row passes: C rows per workgroup, C * n = 4096 complex values in LDS.
template <int LOGN>
struct RowCfg {
  static constexpr int N = 1 << LOGN;
  static constexpr int C = N >= 4096 ? 1 : 4096 / N;
  static constexpr int NB = C * N / 8;   // radix-8 butterflies per pass
  static constexpr int NT = NB < 64 ? 64 : (NB > 1024 ? 1024 : NB);
  static constexpr int DATA = lds_elems(C * N);  // complex elements of data
  static constexpr int LDS = (DATA + Tw2<LOGN>::SIZE) * 8;
};

// Column passes: C adjacent columns per workgroup, C * nf = kColElems complex
// values in LDS (one column when nf exceeds it), two workgroups per CU.
constexpr int kColElems = 8192;  // complex values of fine length held per column workgroup

template <int LOGNF>
struct ColCfg {
  static constexpr int NF = 1 << LOGNF;
  static constexpr int C0 = kColElems / NF;
  static constexpr int C = C0 < 1 ? 1 : (C0 > 16 ? 16 : C0);
  static constexpr int NB = C * NF / 8;
  static constexpr int NT = NB < 64 ? 64 : (NB > 1024 ? 1024 : NB);
  static constexpr int DATA = lds_elems(C * NF);
  // twiddle tables for the fine length and for N' = NF / 2
  static constexpr int LDS = (DATA + Tw2<LOGNF>::SIZE + Tw2<LOGNF - 1>::SIZE) * 8;
};

__device__ __forceinline__ bool in_band(int k, int lo, int hi) { return k >= lo && k <= hi; }

// float64 square root from the hardware seed (v_rsq_f64) refined by Newton
// steps: each step squares the relative error, so two steps from the ~2^-23
// seed are far below 2^-53; a final residual correction gives sqrt to about
// one ulp.
__device__ __forceinline__ double sqrt_nr(double r) {
  double y = __builtin_amdgcn_rsq(r);
  y = y * (1.5 - 0.5 * r * y * y);
  y = y * (1.5 - 0.5 * r * y * y);
  const double s = r * y;
  return s + 0.5 * y * (r - s * s);
}

// Transfer function of Eq. 4 (ASM) or Eq. 5 (Fresnel) at integer frequency
// (kx, ky), without the Rect.  The ASM phase is formed in cycles:
// z sqrt(1/l^2 - df^2 k^2) = z/l - (z/l)(1 - sqrt(1 - t)), t = (l df)^2 k^2.
// sqrt(1 - t) is accurate to about one ulp of 1, so the subtracted term is
// off by about (z/l) 2^-53 cycles however large z/l is (1e-10 cycles at
// z/l = 2e6); z/l itself enters only as its fraction c0.  The phase is then
// reduced to [-1/2, 1/2] before the float32 sine and cosine.  Evanescent
// frequencies (t > 1) give 0.
__device__ __forceinline__ float2 transfer_at(const Spectral& sp, int Np, int kx, int ky) {
  float2 h;
  if (sp.tf == 1) {
    h = cmul(sp.fre_x[kx + Np / 2], sp.fre_y[ky + Np / 2]);
  } else if (sp.phase_fp64) {
    const double k2 = (double)kx * kx + (double)ky * ky;
    const double u = 1.0 - sp.ql2 * k2;
    if (u < 0.0) return czero();
    const double s = u > 0.0 ? sqrt_nr(u) : 0.0;
    double cyc = sp.c0 + sp.ax * kx + sp.ay * ky - sp.zl * (1.0 - s);
    cyc -= rint(cyc);
    h = cis_rev((float)cyc);
  } else {
    const float k2 = (float)kx * (float)kx + (float)ky * (float)ky;
    const float r = sp.inv_lam2f - sp.qf * k2;
    if (r < 0.0f) return czero();
    float cyc = sp.axf * (float)kx + sp.ayf * (float)ky + sp.zf * sqrtf(r);
    cyc -= rintf(cyc);
    h = cis_rev(cyc);
  }
  if (sp.conj) h.y = -h.y;
  return h;
}

// ----------------------------------------------------------------- type 1
// Fine support rows -> nf-point FFT along x -> keep k_x in K, times 1/psihat.
// T[i][a] = sum_l G[i][l] exp(-2 pi i k_x (s0 + l) / nf) / psihat(k_x).
template <int LOGNP>
__device__ __forceinline__ void t1_rows_body(const RowArgs& a, int bid, int) {
  const float2* __restrict__ fine = a.in;
  float2* __restrict__ T = a.out;
  const GridGeom& g = a.g;
  const float* __restrict__ dinv = a.dinv;
  constexpr int LOGN = LOGNP + 1, NF = 1 << LOGN, NP = 1 << LOGNP;
  using Cfg = RowCfg<LOGN>;
  constexpr int C = Cfg::C, NT = Cfg::NT;
  extern __shared__ float2 s[];
  float2* tw = s + Cfg::DATA;
  load_tw2<LOGN, NT>(tw, tw_for(a.tw, LOGN));
  const int r0 = bid * C;
  const int L = g.L, s0 = g.s0;
  // the first pass reads the support rows (zero outside), the last one
  // writes the kept k_x; loads are clamped and selected, never branched over
  const auto ld = [&](int t, int c) -> float2 {
    const int row = r0 + c, i = t - s0;
    const float2 v = fine[(size_t)min(row, L - 1) * L + min(max(i, 0), L - 1)];
    return (row < L && i >= 0 && i < L) ? v : czero();
  };
  const auto st = [&](int t, int c, float2 v) {
    const int row = r0 + c, kx = t < NF / 2 ? t : t - NF;
    if (row < L && kx >= -NP / 2 && kx < NP / 2 && in_band(kx, g.kxlo, g.kxhi))
      T[(size_t)row * NP + kx + NP / 2] = cscale(v, dinv[kx + NP / 2]);
  };
  fft_io<LOGN, C, NT, -1, true, true>(s, tw, (int)threadIdx.x, ld, st, NoIO{});
}

// Column passes that change length: a forward FFT of one length and an
// inverse FFT of another over the same columns; C adjacent columns sized by
// the longer of the two.
template <int LOGA, int LOGB>
struct Col2Cfg {
  static constexpr int LMAX = LOGA > LOGB ? LOGA : LOGB;
  static constexpr int NMAX = 1 << LMAX;
  static constexpr int C0 = kColElems / NMAX;
  static constexpr int C = C0 < 1 ? 1 : (C0 > 16 ? 16 : C0);
  static constexpr int NB = C * NMAX / 8;
  static constexpr int NT = NB < 64 ? 64 : (NB > 1024 ? 1024 : NB);
  static constexpr int DATA = lds_elems(C * NMAX);
  static constexpr int LDS = (DATA + Tw2<LOGA>::SIZE + Tw2<LOGB>::SIZE) * 8;
};

// Columns of T -> nf-point FFT along y -> keep k_y in the spectral grid K''
// (N'' = NPF modes, a superset of the band of Eq. 4; N'' = N' unless the band
// is narrow) -> times H(k) Rect(k) / psihat(k_y) / N'^2 -> embedded in K ->
// N'-point inverse FFT along y.  T holds the columns k_x + N''/2; V is
// written with N' columns, k_x + N'/2.  The (-1)^k factors of the centred
// fine grid and of the centred inverse DFT cancel (N'/2 is even); the
// remaining output sign (-1)^n_y is applied here.
template <int LOGNPF, int LOGNP>
__device__ __forceinline__ void t1_cols_body(const ColArgs& a, int bid, int nbid) {
  const float2* __restrict__ T = a.in;
  float2* __restrict__ V = a.out;
  const GridGeom& g = a.g;
  const Spectral& sp = a.sp;
  const float2* __restrict__ twall = a.tw;
  constexpr int LOGN = LOGNPF + 1, NF = 1 << LOGN, NPF = 1 << LOGNPF, NP = 1 << LOGNP;
  using Cfg = Col2Cfg<LOGN, LOGNP>;
  constexpr int C = Cfg::C, NT = Cfg::NT;
  extern __shared__ float2 s[];
  const int strip = xcd_remap(bid, nbid);
  const int a0 = strip * C;
  const int kx0 = a0 - NPF / 2;
  if (kx0 + C - 1 < g.kxlo || kx0 > g.kxhi) return;  // whole strip outside the band
  float2* twf = s + Cfg::DATA;
  float2* twp = twf + Tw2<LOGN>::SIZE;
  load_tw2<LOGN, NT>(twf, tw_for(twall, LOGN));
  load_tw2<LOGNP, NT>(twp, tw_for(twall, LOGNP));
  const int L = g.L, s0 = g.s0;
  // forward transform: the first pass reads the support rows of T, the last
  // one applies H Rect / psihat / N'^2 to the modes of K'' and writes them,
  // embedded in K, as the inverse transform's input (the rest of K zeroed)
  const auto ld = [&](int t, int c) -> float2 {
    const int i = t - s0;
    const float2 v = T[(size_t)min(max(i, 0), L - 1) * NPF + a0 + c];
    return (i >= 0 && i < L && in_band(kx0 + c, g.kxlo, g.kxhi)) ? v : czero();
  };
  const auto mid = [&](int t, int c, float2 v) {
    const int ky = t < NF / 2 ? t : t - NF, kx = kx0 + c;
    if (ky < -NPF / 2 || ky >= NPF / 2) return;  // outside K''
    float2 x = czero();
    if (in_band(kx, g.kxlo, g.kxhi) && in_band(ky, g.kylo, g.kyhi)) {
      x = cmul(v, transfer_at(sp, NP, kx, ky));
      x = cscale(x, sp.dinv[ky + NPF / 2] * sp.scale);
    }
    s[pidx((ky + NP / 2) * C + c)] = x;
  };
  const auto gap = [&]() {
    if constexpr (NPF < NP) {
      // K outside K'': [0, (N' - N'')/2) and [(N' + N'')/2, N')
      constexpr int H = (NP - NPF) / 2;
      for (int e = threadIdx.x; e < 2 * H * C; e += NT) {
        const int u = e / C, c = e % C;
        const int ay = u < H ? u : u + NPF;
        s[pidx(ay * C + c)] = czero();
      }
    }
  };
  fft_io<LOGN, C, NT, -1, true, true>(s, twf, (int)threadIdx.x, ld, mid, gap);
  // inverse transform along y; the last pass writes V with the (-1)^n_y sign
  const auto st = [&](int by, int c, float2 x) {
    const int kx = kx0 + c;
    if (in_band(kx, g.kxlo, g.kxhi)) {
      if (by & 1) x = make_float2(-x.x, -x.y);
      V[(size_t)by * NP + kx + NP / 2] = x;
    }
  };
  fft_io<LOGNP, C, NT, +1, false, true>(s, twp, opaque_tid(), NoIO{}, st, NoIO{});
}

// Rows of V -> N'-point inverse FFT along x -> times (-1)^n_x -> plane
// (N' x N', or the central N x N when cropping).
template <int LOGNP>
__device__ __forceinline__ void t1_rows_inv_body(const RowArgs& a, int bid, int) {
  const float2* __restrict__ V = a.in;
  float2* __restrict__ out = a.out;
  const GridGeom& g = a.g;
  constexpr int NP = 1 << LOGNP;
  using Cfg = RowCfg<LOGNP>;
  constexpr int C = Cfg::C, NT = Cfg::NT;
  extern __shared__ float2 s[];
  float2* tw = s + Cfg::DATA;
  load_tw2<LOGNP, NT>(tw, tw_for(a.tw, LOGNP));
  const int nrows = g.crop ? g.N : NP;
  const int rowoff = g.crop ? g.N / 2 : 0;
  const int r0 = bid * C;
  const auto ld = [&](int a, int c) -> float2 {
    const int r = r0 + c, kx = a - NP / 2;
    const float2 v = V[(size_t)(min(r, nrows - 1) + rowoff) * NP + a];
    return (r < nrows && in_band(kx, g.kxlo, g.kxhi)) ? v : czero();
  };
  const auto st = [&](int bx, int c, float2 x) {
    const int r = r0 + c;
    if (r >= nrows) return;
    if (bx & 1) x = make_float2(-x.x, -x.y);
    if (g.crop) {
      const int ox = bx - g.N / 2;
      if (ox >= 0 && ox < g.N) out[(size_t)r * g.N + ox] = x;
    } else {
      out[(size_t)r * NP + bx] = x;
    }
  };
  fft_io<LOGNP, C, NT, +1, true, true>(s, tw, (int)threadIdx.x, ld, st, NoIO{});
}

// ----------------------------------------------------------------- type 2
// Rows of the Nin x Nin plane, zero-padded circularly to N' -> FFT along x ->
// times (-1)^k_x / psihat(k_x), centred output T[row][k_x + N'/2].
template <int LOGNP>
__device__ __forceinline__ void t2_rows_body(const RowArgs& a, int bid, int) {
  const float2* __restrict__ u1 = a.in;
  float2* __restrict__ T = a.out;
  const GridGeom& g = a.g;
  const float* __restrict__ dinv = a.dinv;
  constexpr int NP = 1 << LOGNP;
  using Cfg = RowCfg<LOGNP>;
  constexpr int C = Cfg::C, NT = Cfg::NT;
  extern __shared__ float2 s[];
  float2* tw = s + Cfg::DATA;
  load_tw2<LOGNP, NT>(tw, tw_for(a.tw, LOGNP));
  const int Nin = g.Nin;
  const int r0 = bid * C;
  const auto ld = [&](int t, int c) -> float2 {
    const int r = r0 + c, mx = t < NP / 2 ? t : t - NP;
    const int mc = min(max(mx, -Nin / 2), Nin / 2 - 1);
    const float2 v = u1[(size_t)min(r, Nin - 1) * Nin + mc + Nin / 2];
    return (r < Nin && mx >= -Nin / 2 && mx < Nin / 2) ? v : czero();
  };
  const auto st = [&](int t, int c, float2 v) {
    const int r = r0 + c, kx = t < NP / 2 ? t : t - NP;
    if (r < Nin && in_band(kx, g.kxlo, g.kxhi)) {
      float2 x = cscale(v, dinv[kx + NP / 2]);
      if (kx & 1) x = make_float2(-x.x, -x.y);
      T[(size_t)r * NP + kx + NP / 2] = x;
    }
  };
  fft_io<LOGNP, C, NT, -1, true, true>(s, tw, (int)threadIdx.x, ld, st, NoIO{});
}

// Columns of T (Nin rows, N' columns k_x + N'/2) -> N'-point FFT along y ->
// the modes k_y of the spectral grid K'' (N'' = NPF, a superset of the band
// of Eq. 4) times H(k) Rect(k) (-1)^k_y / psihat(k_y) / N'^2, embedded in the
// nf-point spectrum (nf = 2 N'', the gap zero) -> inverse nf-point FFT along
// y -> the support rows [s0, s0 + L), written with N'' columns k_x + N''/2.
template <int LOGNPF, int LOGNP>
__device__ __forceinline__ void t2_cols_body(const ColArgs& a, int bid, int nbid) {
  const float2* __restrict__ T = a.in;
  float2* __restrict__ V = a.out;
  const GridGeom& g = a.g;
  const Spectral& sp = a.sp;
  const float2* __restrict__ twall = a.tw;
  constexpr int LOGN = LOGNPF + 1, NF = 1 << LOGN, NPF = 1 << LOGNPF, NP = 1 << LOGNP;
  using Cfg = Col2Cfg<LOGNP, LOGN>;
  constexpr int C = Cfg::C, NT = Cfg::NT;
  extern __shared__ float2 s[];
  const int strip = xcd_remap(bid, nbid);
  const int a0 = strip * C;
  const int kx0 = a0 - NP / 2;
  if (kx0 + C - 1 < g.kxlo || kx0 > g.kxhi) return;
  float2* twp = s + Cfg::DATA;
  float2* twf = twp + Tw2<LOGNP>::SIZE;
  load_tw2<LOGNP, NT>(twp, tw_for(twall, LOGNP));
  load_tw2<LOGN, NT>(twf, tw_for(twall, LOGN));
  const int Nin = g.Nin;
  // forward transform along y: the first pass reads the Nin rows of T
  // (circularly zero-padded), the last one applies H Rect (-1)^k_y / psihat /
  // N'^2 to the modes of K'' and writes them into the nf-point spectrum of the
  // inverse transform, whose gap it zeroes
  const auto ld = [&](int t, int c) -> float2 {
    const int my = t < NP / 2 ? t : t - NP;
    const int mc = min(max(my, -Nin / 2), Nin / 2 - 1);
    const float2 v = T[(size_t)(mc + Nin / 2) * NP + a0 + c];
    return (my >= -Nin / 2 && my < Nin / 2 && in_band(kx0 + c, g.kxlo, g.kxhi)) ? v : czero();
  };
  const auto mid = [&](int t, int c, float2 v) {
    const int ky = t < NP / 2 ? t : t - NP, kx = kx0 + c;
    if (ky < -NPF / 2 || ky >= NPF / 2) return;  // outside K''
    float2 x = czero();
    if (in_band(kx, g.kxlo, g.kxhi) && in_band(ky, g.kylo, g.kyhi)) {
      x = cmul(v, transfer_at(sp, NP, kx, ky));
      x = cscale(x, sp.dinv[ky + NPF / 2] * sp.scale * ((ky & 1) ? -1.0f : 1.0f));
    }
    s[pidx(((ky + NF) & (NF - 1)) * C + c)] = x;
  };
  const auto gap = [&]() {
    // the gap between the two halves of K'' inside the nf-point spectrum
    for (int e = threadIdx.x; e < C * (NF - NPF); e += NT) {
      const int t = NPF / 2 + e / C, c = e % C;
      s[pidx(t * C + c)] = czero();
    }
  };
  fft_io<LOGNP, C, NT, -1, true, true>(s, twp, (int)threadIdx.x, ld, mid, gap);
  // inverse nf-point transform; the last pass keeps the support rows
  const int L = g.L, s0 = g.s0;
  const auto st = [&](int t, int c, float2 v) {
    const int i = t - s0, kx = kx0 + c;
    if (i >= 0 && i < L && in_band(kx, g.kxlo, g.kxhi)) V[(size_t)i * NPF + kx + NPF / 2] = v;
  };
  fft_io<LOGN, C, NT, +1, false, true>(s, twf, opaque_tid(), NoIO{}, st, NoIO{});
}

// Support rows of V -> embed k_x into nf -> inverse nf-point FFT along x ->
// keep support columns: the fine grid the interpolation reads.
template <int LOGNP>
__device__ __forceinline__ void t2_rows_inv_body(const RowArgs& a, int bid, int) {
  const float2* __restrict__ V = a.in;
  float2* __restrict__ fine = a.out;
  const GridGeom& g = a.g;
  constexpr int LOGN = LOGNP + 1, NF = 1 << LOGN, NP = 1 << LOGNP;
  using Cfg = RowCfg<LOGN>;
  constexpr int C = Cfg::C, NT = Cfg::NT;
  extern __shared__ float2 s[];
  float2* tw = s + Cfg::DATA;
  load_tw2<LOGN, NT>(tw, tw_for(a.tw, LOGN));
  const int L = g.L, s0 = g.s0;
  const int r0 = bid * C;
  // the first pass reads the row's k_x into the nf-point spectrum (the gap
  // zero), the last one keeps the support columns
  const auto ld = [&](int t, int c) -> float2 {
    const int r = r0 + c;
    const bool lo = t < NP / 2, hi = t >= NF - NP / 2;
    const int kx = lo ? t : hi ? t - NF : 0;
    const float2 v = V[(size_t)min(r, L - 1) * NP + kx + NP / 2];
    return (r < L && (lo || hi) && in_band(kx, g.kxlo, g.kxhi)) ? v : czero();
  };
  const auto st = [&](int t, int c, float2 v) {
    const int r = r0 + c, i = t - s0;
    if (r < L && i >= 0 && i < L) fine[(size_t)r * L + i] = v;
  };
  fft_io<LOGN, C, NT, +1, true, true>(s, tw, (int)threadIdx.x, ld, st, NoIO{});
}

// ----------------------------------------------------------------- type 3
// Column pass of NU-ASM_3 / NU-FRE_3 (non-uniform source and destination),
// between the type-1 row pass over the source's fine support and the type-2
// inverse row pass over the destination's: columns of T -> nf-point FFT along
// y -> keep k_y in K (the gap outside K zeroed) -> times H(k) Rect(k) N'^-2
// and the three deconvolutions not applied elsewhere, 1/psihat(k_y) of the
// spreading, 1/psihat(k_y) and 1/psihat(k_x) of the interpolation -> inverse
// nf-point FFT along y -> the support rows [s0, s0 + L).  Both grids are fine
// grids, so the (-1)^k factors of the window offset cancel between the
// forward and the inverse transform on each axis.  Every element is scaled
// in place by its own thread: one LDS buffer, no register staging.
template <int LOGNF>
struct T3Cfg {
  using Col = ColCfg<LOGNF>;
  static constexpr int C = Col::C, NT = Col::NT, DATA = Col::DATA;
  static constexpr int LDS = (DATA + Tw2<LOGNF>::SIZE) * 8;
  // waves per SIMD when two workgroups share a CU (LDS permitting): the
  // register budget is held to what that occupancy allows
  static constexpr int WAVES = LDS <= 80 * 1024 ? 2 * NT / 256 : NT / 256;
};

template <int LOGNP>
__global__ void __launch_bounds__(T3Cfg<LOGNP + 1>::NT)
__attribute__((amdgpu_waves_per_eu(T3Cfg<LOGNP + 1>::WAVES)))
k_t3_cols(const float2* __restrict__ T, float2* __restrict__ V, GridGeom g, Spectral sp,
          const float2* __restrict__ twall) {
  constexpr int LOGN = LOGNP + 1, NF = 1 << LOGN, NP = 1 << LOGNP;
  using Cfg = T3Cfg<LOGN>;
  constexpr int C = Cfg::C, NT = Cfg::NT;
  extern __shared__ float2 s[];
  const int strip = xcd_remap(blockIdx.x, gridDim.x);
  const int a0 = strip * C;
  const int kx0 = a0 - NP / 2;
  if (kx0 + C - 1 < g.kxlo || kx0 > g.kxhi) return;  // whole strip outside the band
  float2* twf = s + Cfg::DATA;
  load_tw2<LOGN, NT>(twf, tw_for(twall, LOGN));
  const int L = g.L, s0 = g.s0;
  // forward transform: the first pass reads the support rows of T, the last
  // one scales every mode in place (zero outside K and the band)
  const auto ld = [&](int t, int c) -> float2 {
    const int i = t - s0;
    const float2 v = T[(size_t)min(max(i, 0), L - 1) * NP + a0 + c];
    return (i >= 0 && i < L && in_band(kx0 + c, g.kxlo, g.kxhi)) ? v : czero();
  };
  const auto mid = [&](int t, int c, float2 v) {
    const int ky = t < NF / 2 ? t : t - NF;
    const int kx = kx0 + c;
    float2 x = czero();
    if (ky >= -NP / 2 && ky < NP / 2 && in_band(kx, g.kxlo, g.kxhi) && in_band(ky, g.kylo, g.kyhi)) {
      const float2 h = transfer_at(sp, g.Np, kx, ky);
      const float dy = sp.dinv[ky + NP / 2];
      x = cmul(v, h);
      x = cscale(x, dy * dy * sp.dinv[kx + NP / 2] * sp.scale);
    }
    s[pidx(t * C + c)] = x;
  };
  fft_io<LOGN, C, NT, -1, true, true>(s, twf, (int)threadIdx.x, ld, mid, NoIO{});
  // inverse transform; the last pass keeps the support rows
  const auto st = [&](int t, int c, float2 v) {
    const int i = t - s0;
    if (i >= 0 && i < L && in_band(kx0 + c, g.kxlo, g.kxhi)) V[(size_t)i * NP + a0 + c] = v;
  };
  fft_io<LOGN, C, NT, +1, false, true>(s, twf, opaque_tid(), NoIO{}, st, NoIO{});
}

// ----------------------------------------------------------- test kernels
template <int LOGN, int DIR>
__global__ void __launch_bounds__(RowCfg<LOGN>::NT)
k_fft_rows(const float2* __restrict__ in, float2* __restrict__ out, int64_t batch,
           const float2* __restrict__ twall) {
  constexpr int N = 1 << LOGN;
  using Cfg = RowCfg<LOGN>;
  constexpr int C = Cfg::C, NT = Cfg::NT;
  extern __shared__ float2 s[];
  float2* tw = s + Cfg::DATA;
  load_tw2<LOGN, NT>(tw, tw_for(twall, LOGN));
  const int64_t r0 = (int64_t)blockIdx.x * C;
  const auto ld = [&](int t, int c) -> float2 {
    const int64_t r = r0 + c;
    const float2 v = in[(r < batch ? r : batch - 1) * N + t];
    return r < batch ? v : czero();
  };
  const auto st = [&](int t, int c, float2 v) {
    const int64_t r = r0 + c;
    if (r < batch) out[r * N + t] = v;
  };
  fft_io<LOGN, C, NT, DIR, true, true>(s, tw, (int)threadIdx.x, ld, st, NoIO{});
}

__global__ void k_transfer_table(GridGeom g, Spectral sp, float2* __restrict__ out) {
  const int Np = g.Np;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)Np * Np) return;
  const int ay = (int)(e / Np), ax = (int)(e % Np);
  const int kx = ax - Np / 2, ky = ay - Np / 2;
  float2 h = czero();
  if (in_band(kx, g.kxlo, g.kxhi) && in_band(ky, g.kylo, g.kyhi)) h = transfer_at(sp, Np, kx, ky);
  out[e] = h;
}

// One axis of the Fresnel transfer function (Eq. 5) in float64:
// out[k + N'/2] = amp * sum_{m in K} exp(i pi (m g + o)^2 / (lambda z)) exp(-2 pi i k m / N').
// Both phases are reduced to whole cycles exactly (k m mod N' in integers)
// before the float64 sincospi.  One workgroup per output frequency; its 256
// threads split the N' terms and meet in an LDS tree.
constexpr int kFresnelThreads = 256;

__global__ void __launch_bounds__(kFresnelThreads)
k_fresnel_axis(int Np, double g, double two_lam_z, double o, double2 amp, float2* __restrict__ out) {
  __shared__ double2 part[kFresnelThreads];
  const int a = blockIdx.x;
  const int64_t k = a - Np / 2;
  double re = 0.0, im = 0.0;
  for (int m = -Np / 2 + (int)threadIdx.x; m < Np / 2; m += kFresnelThreads) {
    const double xm = m * g + o;
    double c = xm * xm / two_lam_z;
    c -= rint(c);
    const int64_t km = (k * m) % Np;
    double cyc = c - (double)km / (double)Np;
    double sn, cs;
    sincospi(2.0 * cyc, &sn, &cs);
    re += cs;
    im += sn;
  }
  part[threadIdx.x] = make_double2(re, im);
  __syncthreads();
  for (int h = kFresnelThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      part[threadIdx.x].x += part[threadIdx.x + h].x;
      part[threadIdx.x].y += part[threadIdx.x + h].y;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    re = part[0].x;
    im = part[0].y;
    out[a] = make_float2((float)(re * amp.x - im * amp.y), (float)(re * amp.y + im * amp.x));
  }
}

// --------------------------------------------------------------- launchers
template <typename K>
static hipError_t set_lds(K kernel, int bytes) {
  if (bytes > 64 * 1024)
    return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  return hipSuccess;
}

#define NUASM_DISPATCH_NP(logNp, CALL)                  \
  switch (logNp) {                                      \
    case 5: CALL(5); break;                             \
    case 6: CALL(6); break;                             \
    case 7: CALL(7); break;                             \
    case 8: CALL(8); break;                             \
    case 9: CALL(9); break;                             \
    case 10: CALL(10); break;                           \
    case 11: CALL(11); break;                           \
    case 12: CALL(12); break;                           \
    case 13: CALL(13); break;                           \
    default: return hipErrorInvalidValue;               \
  }

hipError_t launch_t1_rows(int logNp, const float2* fine, float2* T, GridGeom g, const float* dinv,
                          const float2* tw, hipStream_t st) {
  const RowArgs a{fine, T, g, dinv, tw};
#define CALL(LP)                                                                              \
  {                                                                                           \
    using Cfg = RowCfg<LP + 1>;                                                               \
    return launch_or_record<RowArgs, t1_rows_body<LP>, Cfg::NT>(a, (g.L + Cfg::C - 1) / Cfg::C, \
                                                                Cfg::LDS, st);                \
  }
  NUASM_DISPATCH_NP(logNp, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

// Column passes: the spectral grid N'' = 2^logNpf may be N', N'/2, N'/4 or
// N'/8 (at least 32).
template <int LPF, int LP>
static hipError_t t1_cols_at(const float2* T, float2* V, const GridGeom& g, const Spectral& sp, const float2* tw,
                             hipStream_t st) {
  using Cfg = Col2Cfg<LPF + 1, LP>;
  return launch_or_record<ColArgs, t1_cols_body<LPF, LP>, Cfg::NT>(ColArgs{T, V, g, sp, tw}, (1 << LPF) / Cfg::C,
                                                                   Cfg::LDS, st);
}

template <int LPF, int LP>
static hipError_t t2_cols_at(const float2* T, float2* V, const GridGeom& g, const Spectral& sp, const float2* tw,
                             hipStream_t st) {
  using Cfg = Col2Cfg<LP, LPF + 1>;
  return launch_or_record<ColArgs, t2_cols_body<LPF, LP>, Cfg::NT>(ColArgs{T, V, g, sp, tw}, (1 << LP) / Cfg::C,
                                                                   Cfg::LDS, st);
}

template <int LP, bool T1>
static hipError_t cols_by_reduction(int d, const float2* T, float2* V, const GridGeom& g, const Spectral& sp,
                                    const float2* tw, hipStream_t st) {
#define NUASM_COLS_AT(D)                                                    \
  if constexpr (LP - D >= 5) {                                              \
    if (d == D)                                                             \
      return T1 ? t1_cols_at<LP - D, LP>(T, V, g, sp, tw, st)               \
                : t2_cols_at<LP - D, LP>(T, V, g, sp, tw, st);              \
  }
  NUASM_COLS_AT(0)
  NUASM_COLS_AT(1)
  NUASM_COLS_AT(2)
  NUASM_COLS_AT(3)
#undef NUASM_COLS_AT
  return hipErrorInvalidValue;
}

hipError_t launch_t1_cols(int logNpf, int logNp, const float2* T, float2* V, GridGeom g, Spectral sp,
                          const float2* tw, hipStream_t st) {
  const int d = logNp - logNpf;
#define CALL(LP) return cols_by_reduction<LP, true>(d, T, V, g, sp, tw, st)
  NUASM_DISPATCH_NP(logNp, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

hipError_t launch_t1_rows_inv(int logNp, const float2* V, float2* out, GridGeom g, const float2* tw,
                              hipStream_t st) {
  const RowArgs a{V, out, g, nullptr, tw};
#define CALL(LP)                                                                                      \
  {                                                                                                   \
    using Cfg = RowCfg<LP>;                                                                           \
    const int nrows = g.crop ? g.N : (1 << LP);                                                       \
    return launch_or_record<RowArgs, t1_rows_inv_body<LP>, Cfg::NT>(a, (nrows + Cfg::C - 1) / Cfg::C, \
                                                                    Cfg::LDS, st);                    \
  }
  NUASM_DISPATCH_NP(logNp, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

hipError_t launch_t2_rows(int logNp, const float2* u1, float2* T, GridGeom g, const float* dinv,
                          const float2* tw, hipStream_t st) {
  const RowArgs a{u1, T, g, dinv, tw};
#define CALL(LP)                                                                                \
  {                                                                                             \
    using Cfg = RowCfg<LP>;                                                                     \
    return launch_or_record<RowArgs, t2_rows_body<LP>, Cfg::NT>(a, (g.Nin + Cfg::C - 1) / Cfg::C, \
                                                                Cfg::LDS, st);                  \
  }
  NUASM_DISPATCH_NP(logNp, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

hipError_t launch_t2_cols(int logNpf, int logNp, const float2* T, float2* V, GridGeom g, Spectral sp,
                          const float2* tw, hipStream_t st) {
  const int d = logNp - logNpf;
#define CALL(LP) return cols_by_reduction<LP, false>(d, T, V, g, sp, tw, st)
  NUASM_DISPATCH_NP(logNp, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

hipError_t launch_t2_rows_inv(int logNp, const float2* V, float2* fine, GridGeom g, const float2* tw,
                              hipStream_t st) {
  const RowArgs a{V, fine, g, nullptr, tw};
#define CALL(LP)                                                                                   \
  {                                                                                                \
    using Cfg = RowCfg<LP + 1>;                                                                    \
    return launch_or_record<RowArgs, t2_rows_inv_body<LP>, Cfg::NT>(a, (g.L + Cfg::C - 1) / Cfg::C, \
                                                                    Cfg::LDS, st);                 \
  }
  NUASM_DISPATCH_NP(logNp, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

hipError_t launch_t3_cols(int logNp, const float2* T, float2* V, GridGeom g, Spectral sp,
                          const float2* tw, hipStream_t st) {
#define CALL(LP)                                                                         \
  {                                                                                      \
    using Cfg = T3Cfg<LP + 1>;                                                           \
    hipError_t e = set_lds(k_t3_cols<LP>, Cfg::LDS);                                     \
    if (e != hipSuccess) return e;                                                       \
    const int grid = (1 << LP) / Cfg::C;                                                 \
    hipLaunchKernelGGL(k_t3_cols<LP>, dim3(grid), dim3(Cfg::NT), Cfg::LDS, st, T, V, g, sp, tw); \
  }
  NUASM_DISPATCH_NP(logNp, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_fft_rows(int logn, int64_t batch, int sign, const float2* in, float2* out,
                           const float2* tw, hipStream_t st) {
#define CALL2(LN, D)                                                                     \
  {                                                                                      \
    using Cfg = RowCfg<LN>;                                                              \
    hipError_t e = set_lds(k_fft_rows<LN, D>, Cfg::LDS);                                 \
    if (e != hipSuccess) return e;                                                       \
    const int64_t grid = (batch + Cfg::C - 1) / Cfg::C;                                  \
    hipLaunchKernelGGL((k_fft_rows<LN, D>), dim3((unsigned)grid), dim3(Cfg::NT), Cfg::LDS, st, in, out, batch, tw); \
  }
#define CALL(LN) \
  if (sign < 0) CALL2(LN, -1) else CALL2(LN, 1)
  switch (logn) {
    case 5: CALL(5); break;
    case 6: CALL(6); break;
    case 7: CALL(7); break;
    case 8: CALL(8); break;
    case 9: CALL(9); break;
    case 10: CALL(10); break;
    case 11: CALL(11); break;
    case 12: CALL(12); break;
    case 13: CALL(13); break;
    case 14: CALL(14); break;
    default: return hipErrorInvalidValue;
  }
#undef CALL
#undef CALL2
  return hipGetLastError();
}

hipError_t launch_transfer_table(const GridGeom& g, const Spectral& sp, float2* out, hipStream_t st) {
  const int64_t n = (int64_t)g.Np * g.Np;
  hipLaunchKernelGGL(k_transfer_table, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, sp, out);
  return hipGetLastError();
}

hipError_t launch_fresnel_axis(int Np, double g, double two_lam_z, double o, double2 amp,
                               float2* out, hipStream_t st) {
  hipLaunchKernelGGL(k_fresnel_axis, dim3(Np), dim3(kFresnelThreads), 0, st, Np, g, two_lam_z, o, amp, out);
  return hipGetLastError();
}

}  // namespace nuasm
