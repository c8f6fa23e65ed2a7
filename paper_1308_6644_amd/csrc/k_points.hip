// Non-uniform side of the pipelines on gfx950: coordinate normalisation and
// binning (the conversion of Fig. 1 into fine-grid cells), LDS-tiled
// spreading (gridding of the type-1 sum, Eq. 7) and LDS-tiled interpolation
// (the type-2 sum, Eq. 8).
//
// Fine-grid coordinates: a point at x metres sits at tau = 2 x / g + N + 8 in
// support cells (pixel 0 at support cell N + 8; two fine cells per pixel).
// Its w taps are the cells i0 .. i0 + w - 1, i0 = ceil(tau - w/2).  The
// support is cut into 32 x 32 bins; a point is recorded in every bin its taps
// touch (at most 4), flagged "primary" in the bin holding its first tap.
#include "launch.h"

namespace nuasm {

__global__ void k_fill_i32(int* __restrict__ p, int v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

constexpr double kEdgeSlack = 1e-9;  // pixels

struct PointCells {
  int i0x, i0y;
  float dx, dy;
  bool ok;
};

__device__ __forceinline__ PointCells point_cells(double x, double y, const BinGeom& g) {
  PointCells pc;
  double xp = x * g.inv_g, yp = y * g.inv_g;
  // closed window [-N/2, N/2] in pixels, widened by kEdgeSlack for the
  // rounding of x / g; NaN fails every comparison
  const double lim = g.half_n + kEdgeSlack;
  pc.ok = xp >= -lim && xp <= lim && yp >= -lim && yp <= lim;
  // clamp so that the taps stay inside the support at the closed edges
  xp = fmin(fmax(xp, -g.half_n), g.half_n);
  yp = fmin(fmax(yp, -g.half_n), g.half_n);
  const double tx = 2.0 * xp + g.tau0, ty = 2.0 * yp + g.tau0;
  const double hw = 0.5 * g.w;
  const double fx = ceil(tx - hw), fy = ceil(ty - hw);
  pc.i0x = pc.ok ? (int)fx : 0;
  pc.i0y = pc.ok ? (int)fy : 0;
  pc.dx = (float)(fx - tx);
  pc.dy = (float)(fy - ty);
  return pc;
}

__global__ void k_bin_count(const double* __restrict__ x, const double* __restrict__ y, int64_t M,
                            BinGeom g, int* __restrict__ counts, int* __restrict__ bad) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < M; j += (int64_t)gridDim.x * blockDim.x) {
    const PointCells pc = point_cells(x[j], y[j], g);
    if (!pc.ok) {
      atomicAdd(bad, 1);
      continue;
    }
    const int bx0 = pc.i0x / kTile, bx1 = (pc.i0x + g.w - 1) / kTile;
    const int by0 = pc.i0y / kTile, by1 = (pc.i0y + g.w - 1) / kTile;
    for (int by = by0; by <= by1; ++by)
      for (int bx = bx0; bx <= bx1; ++bx) atomicAdd(&counts[by * g.TX + bx], 1);
  }
}

__global__ void k_bin_scatter(const double* __restrict__ x, const double* __restrict__ y, int64_t M,
                              BinGeom g, int* __restrict__ cursor, BinRec* __restrict__ recs) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < M; j += (int64_t)gridDim.x * blockDim.x) {
    const PointCells pc = point_cells(x[j], y[j], g);
    if (!pc.ok) continue;
    const int bx0 = pc.i0x / kTile, bx1 = (pc.i0x + g.w - 1) / kTile;
    const int by0 = pc.i0y / kTile, by1 = (pc.i0y + g.w - 1) / kTile;
    for (int by = by0; by <= by1; ++by)
      for (int bx = bx0; bx <= bx1; ++bx) {
        const int slot = atomicAdd(&cursor[by * g.TX + bx], 1);
        const int lx = pc.i0x - bx * kTile, ly = pc.i0y - by * kTile;
        BinRec r;
        r.packed = (lx & 0xff) | ((ly & 0xff) << 8) | ((bx == bx0 && by == by0) ? (1 << 16) : 0);
        r.dx = pc.dx;
        r.dy = pc.dy;
        r.idx = (int32_t)j;
        recs[slot] = r;
      }
  }
}

// Single-workgroup scan over the bins: record offsets (written to `cursor`,
// which the scatter then advances), and the chunk tables.  Spreading needs a
// chunk for every bin (empty bins write zeros); interpolation only for
// non-empty bins.  A bin with more than kChunk records is split into several
// chunks; for spreading those bins are listed in `multi` for the reduction.
constexpr int kScanThreads = 1024;

__global__ void __launch_bounds__(kScanThreads)
k_bin_scan(const int* __restrict__ counts, int T, int* __restrict__ cursor, int4* __restrict__ sp_chunks,
           int* __restrict__ sp_first, int* __restrict__ sp_n, int* __restrict__ multi,
           int4* __restrict__ ip_chunks, int* __restrict__ nch) {
  __shared__ int sh[4][kScanThreads];
  const int tid = threadIdx.x;
  const int per = (T + kScanThreads - 1) / kScanThreads;
  const int b0 = min(T, tid * per), b1 = min(T, b0 + per);
  int acc[4] = {0, 0, 0, 0};  // records, spread chunks, interp chunks, multi bins
  for (int b = b0; b < b1; ++b) {
    const int c = counts[b];
    const int nsp = c > kChunk ? (c + kChunk - 1) / kChunk : 1;
    acc[0] += c;
    acc[1] += nsp;
    acc[2] += (c + kChunk - 1) / kChunk;
    acc[3] += nsp > 1 ? 1 : 0;
  }
  for (int q = 0; q < 4; ++q) sh[q][tid] = acc[q];
  __syncthreads();
  // inclusive Hillis-Steele scan of the four per-thread sums
  for (int off = 1; off < kScanThreads; off <<= 1) {
    int v[4];
    for (int q = 0; q < 4; ++q) v[q] = tid >= off ? sh[q][tid - off] : 0;
    __syncthreads();
    for (int q = 0; q < 4; ++q) sh[q][tid] += v[q];
    __syncthreads();
  }
  int run[4];
  for (int q = 0; q < 4; ++q) run[q] = sh[q][tid] - acc[q];
  for (int b = b0; b < b1; ++b) {
    const int c = counts[b];
    const int nsp = c > kChunk ? (c + kChunk - 1) / kChunk : 1;
    const int nip = (c + kChunk - 1) / kChunk;
    cursor[b] = run[0];
    sp_first[b] = run[1];
    sp_n[b] = nsp;
    for (int q = 0; q < nsp; ++q)
      sp_chunks[run[1] + q] = make_int4(b, run[0] + q * kChunk, min(kChunk, c - q * kChunk), nsp);
    for (int q = 0; q < nip; ++q)
      ip_chunks[run[2] + q] = make_int4(b, run[0] + q * kChunk, min(kChunk, c - q * kChunk), nip);
    if (nsp > 1) multi[run[3]] = b;
    run[0] += c;
    run[1] += nsp;
    run[2] += nip;
    run[3] += nsp > 1 ? 1 : 0;
  }
  if (tid == kScanThreads - 1) {
    nch[0] = sh[1][tid];
    nch[1] = sh[2][tid];
    nch[2] = sh[0][tid];
    nch[3] = sh[3][tid];
  }
}

// ------------------------------------------------------------- spreading
// One workgroup per chunk of a bin: accumulate c_j psi(.) psi(.) into a 32 x 32
// LDS tile with LDS float atomics (only the taps that fall inside this bin;
// the point's other bins hold their own copy of the record), then write the
// tile.  A bin split into several chunks writes per-chunk partial tiles that
// k_spread_reduce sums.
constexpr int kSpreadThreads = 256;
constexpr int kTS = kTile + 1;  // padded LDS row

template <int W>
__global__ void __launch_bounds__(kSpreadThreads) k_spread(SpreadArgs a) {
  __shared__ float sre[kTile * kTS];
  __shared__ float sim[kTile * kTS];
  const int cid = blockIdx.x;
  if (cid >= a.nchunks[0]) return;
  const int4 ch = a.chunks[cid];
  const int bin = ch.x, start = ch.y, n = ch.z, nb = ch.w;
  for (int e = threadIdx.x; e < kTile * kTS; e += kSpreadThreads) {
    sre[e] = 0.f;
    sim[e] = 0.f;
  }
  __syncthreads();
  for (int r = threadIdx.x; r < n; r += kSpreadThreads) {
    const BinRec rec = a.recs[start + r];
    const float2 c = a.vals[rec.idx];
    const int lx = rec_lx(rec.packed), ly = rec_ly(rec.packed);
    float wx[W], wy[W];
#pragma unroll
    for (int m = 0; m < W; ++m) {
      wx[m] = es_kernel(rec.dx + (float)m, a.two_over_w, a.beta);
      wy[m] = es_kernel(rec.dy + (float)m, a.two_over_w, a.beta);
    }
#pragma unroll
    for (int my = 0; my < W; ++my) {
      const int yy = ly + my;
      if ((unsigned)yy >= (unsigned)kTile) continue;
      const float cyr = c.x * wy[my], cyi = c.y * wy[my];
#pragma unroll
      for (int mx = 0; mx < W; ++mx) {
        const int xx = lx + mx;
        if ((unsigned)xx >= (unsigned)kTile) continue;
        atomicAdd(&sre[yy * kTS + xx], cyr * wx[mx]);
        atomicAdd(&sim[yy * kTS + xx], cyi * wx[mx]);
      }
    }
  }
  __syncthreads();
  if (nb == 1) {
    const int bx = bin % a.TX, by = bin / a.TX;
    for (int e = threadIdx.x; e < kTile * kTile; e += kSpreadThreads) {
      const int yy = e / kTile, xx = e % kTile;
      const int gy = by * kTile + yy, gx = bx * kTile + xx;
      if (gy < a.L && gx < a.L) a.grid[(size_t)gy * a.L + gx] = make_float2(sre[yy * kTS + xx], sim[yy * kTS + xx]);
    }
  } else {
    float2* part = a.scratch + (size_t)cid * (kTile * kTile);
    for (int e = threadIdx.x; e < kTile * kTile; e += kSpreadThreads) {
      const int yy = e / kTile, xx = e % kTile;
      part[e] = make_float2(sre[yy * kTS + xx], sim[yy * kTS + xx]);
    }
  }
}

// Sum the partial tiles of every multi-chunk bin, in chunk order.
__global__ void __launch_bounds__(256) k_spread_reduce(SpreadReduceArgs a) {
  if ((int)blockIdx.x >= a.nmulti[0]) return;
  const int bin = a.multi[blockIdx.x];
  const int c0 = a.bin_chunk0[bin], nb = a.bin_nchunk[bin];
  const int bx = bin % a.TX, by = bin / a.TX;
  for (int e = threadIdx.x; e < kTile * kTile; e += 256) {
    float2 s = czero();
    for (int q = 0; q < nb; ++q) s = cadd(s, a.scratch[(size_t)(c0 + q) * (kTile * kTile) + e]);
    const int yy = e / kTile, xx = e % kTile;
    const int gy = by * kTile + yy, gx = bx * kTile + xx;
    if (gy < a.L && gx < a.L) a.grid[(size_t)gy * a.L + gx] = s;
  }
}

// --------------------------------------------------------- interpolation
// One workgroup per chunk of a bin: stage the bin plus its (w - 1)-cell halo
// of the fine grid in LDS, then every primary record gathers its w x w taps.
constexpr int kInterpThreads = 256;

template <int W>
__global__ void __launch_bounds__(kInterpThreads) k_interp(InterpArgs a) {
  constexpr int RS = kTile + W - 1;
  __shared__ float2 sg[RS * RS];
  const int cid = blockIdx.x;
  if (cid >= a.nchunks[0]) return;
  const int4 ch = a.chunks[cid];
  const int bin = ch.x, start = ch.y, n = ch.z;
  const int bx = bin % a.TX, by = bin / a.TX;
  for (int e = threadIdx.x; e < RS * RS; e += kInterpThreads) {
    const int yy = e / RS, xx = e % RS;
    const int gy = by * kTile + yy, gx = bx * kTile + xx;
    sg[e] = (gy < a.L && gx < a.L) ? a.grid[(size_t)gy * a.L + gx] : czero();
  }
  __syncthreads();
  for (int r = threadIdx.x; r < n; r += kInterpThreads) {
    const BinRec rec = a.recs[start + r];
    if (!rec_primary(rec.packed)) continue;
    const int lx = rec_lx(rec.packed), ly = rec_ly(rec.packed);
    float wx[W];
#pragma unroll
    for (int m = 0; m < W; ++m) wx[m] = es_kernel(rec.dx + (float)m, a.two_over_w, a.beta);
    float accr = 0.f, acci = 0.f;
#pragma unroll
    for (int my = 0; my < W; ++my) {
      const float wy = es_kernel(rec.dy + (float)my, a.two_over_w, a.beta);
      const float2* row = sg + (ly + my) * RS + lx;
      float rr = 0.f, ri = 0.f;
#pragma unroll
      for (int mx = 0; mx < W; ++mx) {
        const float2 v = row[mx];
        rr += v.x * wx[mx];
        ri += v.y * wx[mx];
      }
      accr += wy * rr;
      acci += wy * ri;
    }
    a.out[rec.idx] = make_float2(accr, acci);
  }
}

// --------------------------------------------------------------- launchers
static int grid_for(int64_t n, int threads) {
  int64_t b = (n + threads - 1) / threads;
  if (b > 65535 * 4) b = 65535 * 4;
  return (int)(b < 1 ? 1 : b);
}

hipError_t launch_fill_i32(int* p, int v, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256)), dim3(256), 0, st, p, v, n);
  return hipGetLastError();
}

hipError_t launch_bin_count(const double* x, const double* y, int64_t M, BinGeom g, int* counts,
                            int* bad, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bin_count, dim3(grid_for(M, 256)), dim3(256), 0, st, x, y, M, g, counts, bad);
  return hipGetLastError();
}

hipError_t launch_bin_scan(const int* counts, int T, int* cursor, int4* sp_chunks, int* sp_first,
                           int* sp_n, int* multi, int4* ip_chunks, int* nch, hipStream_t st) {
  hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(kScanThreads), 0, st, counts, T, cursor, sp_chunks,
                     sp_first, sp_n, multi, ip_chunks, nch);
  return hipGetLastError();
}

hipError_t launch_bin_scatter(const double* x, const double* y, int64_t M, BinGeom g, int* cursor,
                              BinRec* recs, hipStream_t st) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bin_scatter, dim3(grid_for(M, 256)), dim3(256), 0, st, x, y, M, g, cursor, recs);
  return hipGetLastError();
}

#define NUASM_DISPATCH_W(w, CALL)                                                   \
  switch (w) {                                                                      \
    case 2: CALL(2); break;                                                         \
    case 3: CALL(3); break;                                                         \
    case 4: CALL(4); break;                                                         \
    case 5: CALL(5); break;                                                         \
    case 6: CALL(6); break;                                                         \
    case 7: CALL(7); break;                                                         \
    case 8: CALL(8); break;                                                         \
    case 9: CALL(9); break;                                                         \
    case 10: CALL(10); break;                                                       \
    case 11: CALL(11); break;                                                       \
    case 12: CALL(12); break;                                                       \
    case 13: CALL(13); break;                                                       \
    case 14: CALL(14); break;                                                       \
    case 15: CALL(15); break;                                                       \
    case 16: CALL(16); break;                                                       \
    default: return hipErrorInvalidValue;                                           \
  }

hipError_t launch_spread(int w, const SpreadArgs& a, int grid, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
#define CALL(W) hipLaunchKernelGGL(k_spread<W>, dim3(grid), dim3(kSpreadThreads), 0, st, a)
  NUASM_DISPATCH_W(w, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_spread_reduce(const SpreadReduceArgs& a, int grid, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_spread_reduce, dim3(grid), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_interp(int w, const InterpArgs& a, int grid, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
#define CALL(W) hipLaunchKernelGGL(k_interp<W>, dim3(grid), dim3(kInterpThreads), 0, st, a)
  NUASM_DISPATCH_W(w, CALL)
#undef CALL
  return hipGetLastError();
}

}  // namespace nuasm
