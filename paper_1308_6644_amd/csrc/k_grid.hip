// Spreading and interpolation for a non-uniform plane that is a uniform grid
// of its own pitch (scaled diffraction, the case NU-ASM generalises).  The
// weights psi(tx - tau_x(a)) psi(ty - tau_y(b)) of such a plane factor over
// the axes, so both operations split into two 1-D gather passes and need no
// binning at all:
//   interpolation  R[ty][a] = sum_j psi_x(a, j) G[ty][i0x(a) + j]        (x pass)
//                  u[b][a]  = sum_j psi_y(b, j) R[i0y(b) + j][a]         (y pass)
//   spreading      S[b][tx] = sum_{a: tx in taps(a)} psi(tx - tau_x(a)) c[b][a]
//                  G[ty][tx] = sum_{b: ty in taps(b)} psi(ty - tau_y(b)) S[b][tx]
// Lanes run along x in every pass, so every global access is a contiguous
// row segment.
#include "launch.h"

namespace nuasm {

constexpr int kGridRows = 8;  // rows per wave in the passes along x

// First tap and offset (i0 - tau) of grid index k on one axis (centre c, n
// points): the rule of the binned points, clamped to the closed window.
__device__ __forceinline__ void grid_tap(const GridPts& p, int k, int n, double c, int w, int* i0, float* d) {
  double xp = (c + (double)(k - n / 2) * p.pitch) * p.inv_g;
  xp = fmin(fmax(xp, -p.half_n), p.half_n);
  const double t = 2.0 * xp + p.tau0;
  const double f = ceil(t - 0.5 * w);
  *i0 = (int)f;
  *d = (float)(f - t);
}

// x pass of the interpolation: lane = grid column a, each wave kGridRows
// support rows starting at ty0 + blockIdx.y * 4 kGridRows.
template <int W>
__global__ void __launch_bounds__(256) k_grid_interp_x(const float2* __restrict__ G, float2* __restrict__ R,
                                                       GridPts p) {
  const int a = blockIdx.x * 64 + (threadIdx.x & 63);
  const int wave = threadIdx.x >> 6;
  if (a >= p.nx) return;
  int i0;
  float d;
  grid_tap(p, a, p.nx, p.cx, W, &i0, &d);
  float wt[W];
#pragma unroll
  for (int j = 0; j < W; ++j) wt[j] = es_kernel_fast(d + (float)j, p.two_over_w, p.beta_log2e);
  const int r0 = (blockIdx.y * 4 + wave) * kGridRows;
  const int r1 = min(p.nrows, r0 + kGridRows);
  for (int r = r0; r < r1; ++r) {
    const int ty = p.ty0 + r;
    float2 acc = czero();
    if (ty >= 0 && ty < p.L) {
      const float2* row = G + (size_t)ty * p.L + i0;
#pragma unroll
      for (int j = 0; j < W; ++j) {
        const float2 g = row[j];
        acc.x = fmaf(wt[j], g.x, acc.x);
        acc.y = fmaf(wt[j], g.y, acc.y);
      }
    }
    R[(size_t)r * p.nx + a] = acc;
  }
}

// y pass of the interpolation: lane = grid column a, one output row b per
// wave (its taps and weights are the same for every lane).
template <int W>
__global__ void __launch_bounds__(256) k_grid_interp_y(const float2* __restrict__ R, float2* __restrict__ out,
                                                       GridPts p) {
  const int a = blockIdx.x * 64 + (threadIdx.x & 63);
  const int b = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (a >= p.nx || b >= p.ny) return;
  int i0;
  float d;
  grid_tap(p, b, p.ny, p.cy, W, &i0, &d);
  float2 acc = czero();
#pragma unroll
  for (int j = 0; j < W; ++j) {
    const int r = i0 + j - p.ty0;
    if (r >= 0 && r < p.nrows) {
      const float wt = es_kernel_fast(d + (float)j, p.two_over_w, p.beta_log2e);
      const float2 v = R[(size_t)r * p.nx + a];
      acc.x = fmaf(wt, v.x, acc.x);
      acc.y = fmaf(wt, v.y, acc.y);
    }
  }
  out[(size_t)b * p.nx + a] = acc;
}

// Grid indices whose taps may contain support cell t on one axis: tau(k) is
// increasing in k with step s = 2 pitch / g cells, and the taps of k cover
// [ceil(tau - w/2), ceil(tau - w/2) + w), so a range widened by one index on
// each side holds them all; membership is then tested exactly.
__device__ __forceinline__ void grid_candidates(const GridPts& p, int t, int n, double c, int w, int* k0, int* k1) {
  const double s = 2.0 * p.pitch * p.inv_g;
  const double tau_first = 2.0 * ((c + (double)(0 - n / 2) * p.pitch) * p.inv_g) + p.tau0;
  const double lo = (t - 0.5 * w - tau_first) / s;
  const double hi = (t + 0.5 * w - tau_first) / s;
  *k0 = max(0, (int)floor(lo) - 1);
  *k1 = min(n - 1, (int)ceil(hi) + 1);
}

// x pass of the spreading: lane = support column tx, each wave kGridRows
// grid rows; the candidate columns and their weights are shared by the rows.
template <int W>
__global__ void __launch_bounds__(256) k_grid_spread_x(const float2* __restrict__ c, float2* __restrict__ S,
                                                       GridPts p) {
  const int tx = blockIdx.x * 64 + (threadIdx.x & 63);
  const int b0 = (blockIdx.y * 4 + (threadIdx.x >> 6)) * kGridRows;
  if (tx >= p.L || b0 >= p.ny) return;
  const int nb = min(kGridRows, p.ny - b0);
  float2 acc[kGridRows];
#pragma unroll
  for (int r = 0; r < kGridRows; ++r) acc[r] = czero();
  int k0, k1;
  grid_candidates(p, tx, p.nx, p.cx, W, &k0, &k1);
  for (int a = k0; a <= k1; ++a) {
    int i0;
    float d;
    grid_tap(p, a, p.nx, p.cx, W, &i0, &d);
    const int j = tx - i0;
    if (j < 0 || j >= W) continue;
    const float wt = es_kernel_fast(d + (float)j, p.two_over_w, p.beta_log2e);
#pragma unroll
    for (int r = 0; r < kGridRows; ++r) {
      if (r < nb) {
        const float2 v = c[(size_t)(b0 + r) * p.nx + a];
        acc[r].x = fmaf(wt, v.x, acc[r].x);
        acc[r].y = fmaf(wt, v.y, acc[r].y);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kGridRows; ++r)
    if (r < nb) S[(size_t)(b0 + r) * p.L + tx] = acc[r];
}

// y pass of the spreading: lane = support column tx, one support row ty per
// wave; every support cell is written (zero where no grid row reaches).
template <int W>
__global__ void __launch_bounds__(256) k_grid_spread_y(const float2* __restrict__ S, float2* __restrict__ G,
                                                       GridPts p) {
  const int tx = blockIdx.x * 64 + (threadIdx.x & 63);
  const int ty = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (tx >= p.L || ty >= p.L) return;
  float2 acc = czero();
  int k0, k1;
  grid_candidates(p, ty, p.ny, p.cy, W, &k0, &k1);
  for (int b = k0; b <= k1; ++b) {
    int i0;
    float d;
    grid_tap(p, b, p.ny, p.cy, W, &i0, &d);
    const int j = ty - i0;
    if (j < 0 || j >= W) continue;
    const float wt = es_kernel_fast(d + (float)j, p.two_over_w, p.beta_log2e);
    const float2 v = S[(size_t)b * p.L + tx];
    acc.x = fmaf(wt, v.x, acc.x);
    acc.y = fmaf(wt, v.y, acc.y);
  }
  G[(size_t)ty * p.L + tx] = acc;
}

#define NUASM_GRID_DISPATCH_W(w, CALL) \
  switch (w) {                         \
    case 2: CALL(2); break;            \
    case 3: CALL(3); break;            \
    case 4: CALL(4); break;            \
    case 5: CALL(5); break;            \
    case 6: CALL(6); break;            \
    case 7: CALL(7); break;            \
    case 8: CALL(8); break;            \
    case 9: CALL(9); break;            \
    case 10: CALL(10); break;          \
    case 11: CALL(11); break;          \
    case 12: CALL(12); break;          \
    case 13: CALL(13); break;          \
    case 14: CALL(14); break;          \
    case 15: CALL(15); break;          \
    case 16: CALL(16); break;          \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_grid_interp(int w, const float2* fine, float2* R, float2* out, const GridPts& p, hipStream_t st) {
  if (p.nx <= 0 || p.ny <= 0) return hipSuccess;
  const dim3 gx((p.nx + 63) / 64, (p.nrows + 4 * kGridRows - 1) / (4 * kGridRows));
  const dim3 gy((p.nx + 63) / 64, (p.ny + 3) / 4);
#define CALL(W)                                                                   \
  {                                                                               \
    hipLaunchKernelGGL(k_grid_interp_x<W>, gx, dim3(256), 0, st, fine, R, p);     \
    hipError_t e = hipGetLastError();                                             \
    if (e != hipSuccess) return e;                                                \
    hipLaunchKernelGGL(k_grid_interp_y<W>, gy, dim3(256), 0, st, R, out, p);      \
  }
  NUASM_GRID_DISPATCH_W(w, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_grid_spread(int w, const float2* vals, float2* S, float2* fine, const GridPts& p, hipStream_t st) {
  const dim3 gx((p.L + 63) / 64, (p.ny + 4 * kGridRows - 1) / (4 * kGridRows));
  const dim3 gy((p.L + 63) / 64, (p.L + 3) / 4);
#define CALL(W)                                                                    \
  {                                                                                \
    if (p.ny > 0 && p.nx > 0) {                                                    \
      hipLaunchKernelGGL(k_grid_spread_x<W>, gx, dim3(256), 0, st, vals, S, p);    \
      hipError_t e = hipGetLastError();                                            \
      if (e != hipSuccess) return e;                                               \
    }                                                                              \
    GridPts q = p;                                                                 \
    if (p.ny <= 0 || p.nx <= 0) q.ny = 0;                                          \
    hipLaunchKernelGGL(k_grid_spread_y<W>, gy, dim3(256), 0, st, S, fine, q);      \
  }
  NUASM_GRID_DISPATCH_W(w, CALL)
#undef CALL
  return hipGetLastError();
}

}  // namespace nuasm
