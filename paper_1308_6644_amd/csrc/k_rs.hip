// Rayleigh-Sommerfeld diffraction by direct summation over point pairs
// (Eq. 10 with the integral over the source replaced by a weighted sum), the
// accuracy reference the paper measures NU-ASM and NU-FRE against.  O(M1 M2)
// and bound by the vector ALUs: every pair costs a square root, a
// reciprocal, a sine and a cosine.
//
// Work split on gfx950: one workgroup holds 64 destinations (one per lane)
// and eight waves; each wave sums an eighth of the sources, read with scalar
// loads (every lane of a wave needs the same source at the same time, so the
// source stream costs no LDS and no vector memory traffic), and the eight
// partial sums meet in LDS at the end.
#include "launch.h"

namespace nuasm {

constexpr int kRsWaves = 8;   // waves per workgroup, each over an eighth of the sources
constexpr int kRsBlock = 64;  // sources per float32 partial sum (then added in float64)
constexpr int kRsUnroll = 8;  // sources whose scalar loads are issued together

// One pair's term of the sum, without the source weight:
// (z/r)(1 - i k r) exp(i k r)/r^2 with r = sqrt(rho^2 + z^2).
// The phase k r / (2 pi) = |z|/l + (r - |z|)/l is formed in float64 as
// c0 + rho^2 / (l |z| (1 + s)), s = r/|z| = sqrt(1 + rho^2/z^2), where c0 is
// |z|/l reduced mod 1 on the host: no cancellation in r - |z| and no large
// argument.  s and 1/(1 + s) come from the float32 hardware estimates refined
// by one float64 Newton step each (relative error ~1e-14, i.e. ~1e-11 cycles
// at 1000 cycles of phase).  The amplitude needs float32 only:
// z/r^3 = (z/|z|^3) y^3 and k z/r^2 = (k z/z^2) y^2 with y = |z|/r.
__device__ __forceinline__ float2 rs_term(double rho2, const RsConst& k) {
  const double u = fma(rho2, k.inv_z2, 1.0);
  double y = (double)__builtin_amdgcn_rsqf((float)u);
  y = y * fma(-0.5 * u, y * y, 1.5);          // 1/sqrt(u) = |z|/r
  const double d = fma(u, y, 1.0);            // 1 + r/|z|
  double q = (double)__builtin_amdgcn_rcpf((float)d);
  q = q * fma(-d, q, 2.0);                    // 1/(1 + r/|z|)
  double cyc = fma(rho2 * k.inv_lz, q, k.c0);
  cyc -= rint(cyc);
  const float2 e = cis_rev((float)cyc);
  const float yf = (float)y;
  const float y2 = yf * yf;
  const float ar = k.a3 * y2 * yf;            // z / r^3
  const float ai = -k.ak * y2;                // -k z / r^2
  return make_float2(ar * e.x - ai * e.y, ar * e.y + ai * e.x);
}

__global__ void __launch_bounds__(64 * kRsWaves)
k_rs_direct(const double* __restrict__ x1, const double* __restrict__ y1, const float2* __restrict__ c,
            int64_t M1, const double* __restrict__ x2, const double* __restrict__ y2, int64_t M2, RsConst k,
            float2* __restrict__ out) {
  __shared__ double2 part[kRsWaves][64];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t j = (int64_t)blockIdx.x * 64 + lane;
  const bool live = j < M2;
  const double X = (live ? x2[j] : 0.0) + k.ox;
  const double Y = (live ? y2[j] : 0.0) + k.oy;
  const int64_t per = (M1 + kRsWaves - 1) / kRsWaves;
  const int64_t i0 = min(M1, (int64_t)wave * per);
  const int64_t i1 = min(M1, i0 + per);
  double accr = 0.0, acci = 0.0;
  float sr = 0.f, si = 0.f;
  auto pair = [&](double sx, double sy, float2 w) {
    const double dx = X - sx, dy = Y - sy;
    const float2 t = rs_term(fma(dx, dx, dy * dy), k);
    sr = fmaf(w.x, t.x, fmaf(-w.y, t.y, sr));
    si = fmaf(w.x, t.y, fmaf(w.y, t.x, si));
  };
  int64_t i = i0;
  // full groups of kRsUnroll sources: their scalar loads are issued together
  // ahead of the arithmetic; the float32 partial sums go into float64 every
  // kRsBlock sources
  int n = 0;
  for (; i + kRsUnroll <= i1; i += kRsUnroll) {
    double sx[kRsUnroll], sy[kRsUnroll];
    float2 sw[kRsUnroll];
#pragma unroll
    for (int u = 0; u < kRsUnroll; ++u) {
      sx[u] = x1[i + u];
      sy[u] = y1[i + u];
      sw[u] = c[i + u];
    }
#pragma unroll
    for (int u = 0; u < kRsUnroll; ++u) pair(sx[u], sy[u], sw[u]);
    if (++n == kRsBlock / kRsUnroll) {
      accr += (double)sr;
      acci += (double)si;
      sr = si = 0.f;
      n = 0;
    }
  }
  for (; i < i1; ++i) pair(x1[i], y1[i], c[i]);
  accr += (double)sr;
  acci += (double)si;
  part[wave][lane] = make_double2(accr, acci);
  __syncthreads();
  if (wave == 0 && live) {
    double r = 0.0, i = 0.0;
#pragma unroll
    for (int w = 0; w < kRsWaves; ++w) {
      r += part[w][lane].x;
      i += part[w][lane].y;
    }
    out[j] = make_float2((float)(r * k.inv_2pi), (float)(i * k.inv_2pi));
  }
}

hipError_t launch_rs_direct(const double* x1, const double* y1, const float2* c, int64_t M1, const double* x2,
                            const double* y2, int64_t M2, const RsConst& k, float2* out, hipStream_t st) {
  if (M2 <= 0) return hipSuccess;
  const int64_t grid = (M2 + 63) / 64;
  hipLaunchKernelGGL(k_rs_direct, dim3((unsigned)grid), dim3(64 * kRsWaves), 0, st, x1, y1, c, M1, x2, y2, M2, k,
                     out);
  return hipGetLastError();
}

}  // namespace nuasm
