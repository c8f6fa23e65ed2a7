// Non-uniform side of the pipelines on gfx950: coordinate normalisation and
// binning (the conversion of Fig. 1 into fine-grid cells), LDS-tiled
// spreading (gridding of the type-1 sum, Eq. 7) and LDS-tiled interpolation
// (the type-2 sum, Eq. 8).
//
// Fine-grid coordinates: the window is N''/2 cells of pitch g N'/N'' (the
// plan's pixels when N'' = N'), two fine cells each, and a point at x metres
// sits at tau = 2 x inv_g + tau0 support cells (tau0 = N''/2 + 8: that
// raster's pixel 0; BinGeom holds inv_g and tau0).
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

// Counting sort of (point, bin) pairs without global atomics on hot bins.
// The points are cut into G contiguous ranges of at most kBinPoints points,
// one workgroup each.  Pass 1 counts the range's pairs per bin in LDS (two
// 16-bit counters per word: a range has fewer than 65536 points, and a point
// adds at most 1 to a bin) and writes its histogram row hist[g][*].  A column
// scan turns hist into per-(range, bin) offsets; the bin scan adds the bin
// bases.  Pass 2 re-derives the pairs and ranks them inside (range, bin) with
// LDS counters, so every slot is written exactly once.
constexpr int kBinThreads = 1024;
constexpr int kScatterCursorBytes = 64 * 1024;  // LDS for 32-bit scatter cursors (up to 16384 bins)
constexpr int kBinBatch = 4;  // points per thread whose coordinates are loaded together

__device__ __forceinline__ unsigned lds_bump16(unsigned* sh, int b) {
  const int sft = (b & 1) * 16;
  return (atomicAdd(&sh[b >> 1], 1u << sft) >> sft) & 0xffffu;
}

// Histogram rows have T + 1 entries: entry T counts the range's points that
// are outside the window (they get no record).
__global__ void __launch_bounds__(kBinThreads)
k_bin_hist(const double* __restrict__ x, const double* __restrict__ y, int64_t M, BinGeom g, int ppw,
           uint16_t* __restrict__ hist) {
  extern __shared__ unsigned sh[];
  const int T = g.TX * g.TX, TW = (T + 2) / 2;
  for (int e = threadIdx.x; e < TW; e += kBinThreads) sh[e] = 0u;
  __syncthreads();
  const int64_t j0 = (int64_t)blockIdx.x * ppw;
  const int64_t j1 = min(M, j0 + ppw);
  for (int64_t jb = j0; jb < j1; jb += kBinThreads * kBinBatch) {
    double xv[kBinBatch], yv[kBinBatch];  // all loads of a batch in flight together
#pragma unroll
    for (int q = 0; q < kBinBatch; ++q) {
      const int64_t j = jb + threadIdx.x + q * kBinThreads;
      xv[q] = j < j1 ? x[j] : 0.0;
      yv[q] = j < j1 ? y[j] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kBinBatch; ++q) {
      const int64_t j = jb + threadIdx.x + q * kBinThreads;
      if (j >= j1) continue;
      const PointCells pc = point_cells(xv[q], yv[q], g);
      if (!pc.ok) {
        lds_bump16(sh, T);
        continue;
      }
      const int bx0 = pc.i0x / kTile, bx1 = (pc.i0x + g.w - 1) / kTile;
      const int by0 = pc.i0y / kTile, by1 = (pc.i0y + g.w - 1) / kTile;
      for (int by = by0; by <= by1; ++by)
        for (int bx = bx0; bx <= bx1; ++bx) lds_bump16(sh, by * g.TX + bx);
    }
  }
  __syncthreads();
  uint16_t* row = hist + (size_t)blockIdx.x * (T + 1);
  for (int b = threadIdx.x; b <= T; b += kBinThreads) row[b] = (uint16_t)((sh[b >> 1] >> ((b & 1) * 16)) & 0xffffu);
}

// Scan over the bins, run by one workgroup: first record of every bin (written to
// `cursor`, the bin bases the scatter adds), and the chunk tables.  Spreading
// needs a chunk for every bin (empty bins write zeros); interpolation only for
// non-empty bins.  A bin with more than so.sp_chunk (so.ip_chunk) records is
// split into several spreading (interpolation) chunks; for spreading those bins are
// listed in `multi` for the reduction, and their chunks get consecutive slots
// of the partial-tile scratch (nch[5] slots in all).  Both chunk tables are ordered by the
// size of their bin, largest first (17 size classes, a bin's chunks kept
// together), so that the dispatcher starts the longest workgroups first.
// counts[T] (one past the bins) is the number of points outside the window;
// it is copied to nch[4].  Each thread owns a contiguous run of bins; the
// block-wide exclusive scan is two wave-shuffle scans around one LDS step.
constexpr int kScanThreads = 1024;
constexpr int kScanRegs = 8;  // bins per thread kept in registers
constexpr int kSizeClasses = 17;

// size class of a bin's chunks of at most `chunk` records: 16 for bins of at
// least one full chunk, else 16 c / chunk
__device__ __forceinline__ int size_class(int c, int chunk) {
  return c >= chunk ? kSizeClasses - 1 : (c * (kSizeClasses - 1)) / chunk;
}

__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// `counts` is written by other workgroups of the same launch (see
// k_bin_colscan), so it is read through a plain pointer.
__device__ __forceinline__ void bin_scan_body(const int* counts, int T, const BinScanOut& so) {
  int* __restrict__ cursor = so.cursor;
  int4* __restrict__ sp_chunks = so.sp_chunks;
  int* __restrict__ sp_first = so.sp_first;
  int* __restrict__ sp_n = so.sp_n;
  int* __restrict__ multi = so.multi;
  int4* __restrict__ ip_chunks = so.ip_chunks;
  int* __restrict__ nch = so.nch;
  const int spc = so.sp_chunk, ipc = so.ip_chunk;
  constexpr int NW = kScanThreads / 64;
  __shared__ int wsum[5][NW];
  __shared__ int cls_n[2][kSizeClasses], cls_base[2][kSizeClasses];  // spreading, interpolation
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid < 2 * kSizeClasses) cls_n[tid / kSizeClasses][tid % kSizeClasses] = 0;
  const int per = (T + kScanThreads - 1) / kScanThreads;
  const int b0 = min(T, tid * per), b1 = min(T, b0 + per);
  int cr[kScanRegs];
#pragma unroll
  for (int q = 0; q < kScanRegs; ++q) cr[q] = (b0 + q < b1) ? counts[b0 + q] : 0;
  __syncthreads();  // cls_n cleared
  int acc[5] = {0, 0, 0, 0, 0};  // records, spread chunks, interp chunks, multi bins, split-bin chunks
  for (int q = 0; q < per; ++q) {
    const int b = b0 + q;
    const bool valid = b < b1;
    int c = 0;
#pragma unroll
    for (int r = 0; r < kScanRegs; ++r)
      if (r == q) c = cr[r];
    if (q >= kScanRegs && valid) c = counts[b];
    const int nsp = !valid ? 0 : c > spc ? (c + spc - 1) / spc : 1;
    const int nip = (c + ipc - 1) / ipc;
    acc[0] += c;
    acc[1] += nsp;
    acc[2] += nip;
    acc[3] += nsp > 1 ? 1 : 0;
    acc[4] += nsp > 1 ? nsp : 0;
    if (nsp > 0) atomicAdd(&cls_n[0][size_class(c, spc)], nsp);
    if (nip > 0) atomicAdd(&cls_n[1][size_class(c, ipc)], nip);
  }
  int incl[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    incl[k] = wave_incl_scan(acc[k], lane);
    if (lane == 63) wsum[k][wv] = incl[k];
  }
  __syncthreads();
  if (wv == 0) {
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const int v = lane < NW ? wsum[k][lane] : 0;
      const int w = wave_incl_scan(v, lane);
      if (lane < NW) wsum[k][lane] = w - v;  // exclusive wave bases
    }
  }
  if (tid < 2) {  // chunk bases of the size classes, largest class first
    int run = 0;
    for (int k = kSizeClasses - 1; k >= 0; --k) {
      cls_base[tid][k] = run;
      run += cls_n[tid][k];
    }
  }
  __syncthreads();
  int run[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) run[k] = wsum[k][wv] + incl[k] - acc[k];
  for (int q = 0; q < per; ++q) {
    const int b = b0 + q;
    const bool valid = b < b1;
    int c = 0;
#pragma unroll
    for (int r = 0; r < kScanRegs; ++r)
      if (r == q) c = cr[r];
    if (q >= kScanRegs && valid) c = counts[b];
    const int nsp = !valid ? 0 : c > spc ? (c + spc - 1) / spc : 1;
    const int nip = (c + ipc - 1) / ipc;
    if (!valid) continue;
    const int first = atomicAdd(&cls_base[0][size_class(c, spc)], nsp);
    const int ifirst = nip > 0 ? atomicAdd(&cls_base[1][size_class(c, ipc)], nip) : 0;
    cursor[b] = run[0];
    sp_first[b] = first;
    sp_n[b] = nsp;
    // .w: the chunk's partial-tile slot when the bin is split, else -1
    for (int r = 0; r < nsp; ++r)
      sp_chunks[first + r] =
          make_int4(b, run[0] + r * spc, min(spc, c - r * spc), nsp > 1 ? run[4] + r : -1);
    for (int r = 0; r < nip; ++r)
      ip_chunks[ifirst + r] = make_int4(b, run[0] + r * ipc, min(ipc, c - r * ipc), nip);
    if (nsp > 1) multi[run[3]] = b;
    run[0] += c;
    run[1] += nsp;
    run[2] += nip;
    run[3] += nsp > 1 ? 1 : 0;
    run[4] += nsp > 1 ? nsp : 0;
  }
  if (tid == kScanThreads - 1) {
    nch[0] = run[1];
    nch[1] = run[2];
    nch[2] = run[0];
    nch[3] = run[3];
    nch[4] = counts[T];
    nch[5] = run[4];
  }
}

// Column scan: off[g][b] = sum_{g' < g} hist[g'][b], total[b] = sum_g hist[g][b].
// A workgroup takes 64 consecutive bins (one per lane) and splits the G
// ranges over its 16 waves.  The last workgroup to finish (counted in `done`,
// which it resets to zero) then runs the bin scan over the totals; the
// counter is bumped after a release fence and read back before an acquire
// fence, so every workgroup's totals are visible to it.  No workgroup waits
// for another.
constexpr int kColWaves = 16;
static_assert(64 * kColWaves == kScanThreads, "the last column-scan workgroup runs the bin scan");

__global__ void __launch_bounds__(64 * kColWaves)
k_bin_colscan(const uint16_t* __restrict__ hist, int G, int T, int* __restrict__ off, int* total,
              BinScanOut so, int* __restrict__ done) {
  // T here is the row length (bins + 1)
  __shared__ int part[kColWaves][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int b = blockIdx.x * 64 + lane;
  const int per = (G + kColWaves - 1) / kColWaves;
  const int g0 = min(G, wv * per), g1 = min(G, g0 + per);
  int s = 0;
  if (b < T) {
#pragma unroll 8
    for (int gg = g0; gg < g1; ++gg) s += hist[(size_t)gg * T + b];
  }
  part[wv][lane] = s;
  __syncthreads();
  int base = 0;
  for (int q = 0; q < wv; ++q) base += part[q][lane];
  if (b < T) {
    int run = base;
#pragma unroll 8
    for (int gg = g0; gg < g1; ++gg) {
      const int h = hist[(size_t)gg * T + b];
      off[(size_t)gg * T + b] = run;
      run += h;
    }
    if (wv == kColWaves - 1) total[b] = run;
  }
  // the totals come from the last wave only: it releases them and bumps the
  // counter; in the last workgroup it also acquires the others' totals for
  // the whole workgroup (one CU, one L2), which the barrier then orders
  // before every wave's reads
  __shared__ int last;
  if (wv == kColWaves - 1) {
    __threadfence();
    if (lane == 0) {
      const bool l = atomicAdd(done, 1) == (int)gridDim.x - 1;
      if (l) __threadfence();
      last = l;
    }
  }
  __syncthreads();
  if (!last) return;
  bin_scan_body(total, T - 1, so);
  if (threadIdx.x == 0) *done = 0;
}

// CURSORS: the workgroup's write cursors bin_base[b] + off[g][b] are staged in
// LDS once and bumped there (one LDS atomic per record, no global loads);
// otherwise 16-bit LDS ranks are added to the two global tables per record
// (for supports with too many bins to stage 32-bit cursors).
template <bool CURSORS>
__global__ void __launch_bounds__(kBinThreads)
k_bin_scatter(const double* __restrict__ x, const double* __restrict__ y, int64_t M, BinGeom g, int ppw,
              const int* __restrict__ off, const int* __restrict__ bin_base, BinRec* __restrict__ recs) {
  extern __shared__ unsigned sh[];
  const int T = g.TX * g.TX, TW = (T + 1) / 2;
  const int* myoff = off + (size_t)blockIdx.x * (T + 1);
  if (CURSORS) {
    for (int b = threadIdx.x; b < T; b += kBinThreads) sh[b] = (unsigned)(bin_base[b] + myoff[b]);
  } else {
    for (int e = threadIdx.x; e < TW; e += kBinThreads) sh[e] = 0u;
  }
  __syncthreads();
  const int64_t j0 = (int64_t)blockIdx.x * ppw;
  const int64_t j1 = min(M, j0 + ppw);
  for (int64_t jb = j0; jb < j1; jb += kBinThreads * kBinBatch) {
    double xv[kBinBatch], yv[kBinBatch];
#pragma unroll
    for (int q = 0; q < kBinBatch; ++q) {
      const int64_t j = jb + threadIdx.x + q * kBinThreads;
      xv[q] = j < j1 ? x[j] : 0.0;
      yv[q] = j < j1 ? y[j] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kBinBatch; ++q) {
      const int64_t j = jb + threadIdx.x + q * kBinThreads;
      if (j >= j1) continue;
      const PointCells pc = point_cells(xv[q], yv[q], g);
      if (!pc.ok) continue;
      const int bx0 = pc.i0x / kTile, bx1 = (pc.i0x + g.w - 1) / kTile;
      const int by0 = pc.i0y / kTile, by1 = (pc.i0y + g.w - 1) / kTile;
      for (int by = by0; by <= by1; ++by)
        for (int bx = bx0; bx <= bx1; ++bx) {
          const int b = by * g.TX + bx;
          const int slot = CURSORS ? (int)atomicAdd(&sh[b], 1u)
                                   : bin_base[b] + myoff[b] + (int)lds_bump16(sh, b);
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
}

// Deterministic mode: the same counting sort with a stable scatter, so that
// the records of every bin are in point order whatever the timing of the
// workgroups.  A range holds at most kDetPoints points, one per thread; the
// range's records are compacted (a block scan of the per-point counts) and
// keyed (bin, 4 p + k) for the k-th bin of its p-th point, sorted by a
// bitonic network in LDS, and a record's slot is its bin's base plus the
// range's offset in the bin plus its index in the run of its bin (found by a
// max-scan of the run starts).
constexpr int kDetPoints = kBinThreads;  // 1024
constexpr int kDetRecs = 4 * kDetPoints;
constexpr int kDetRecBits = 12;          // 4 p + k < 2^12
static_assert(kDetRecs == 1 << kDetRecBits, "record ids fill the low key bits");
static_assert(kDetPoints == kBinPointsStable, "ranges of the stable scatter");

template <int NTH>
__device__ __forceinline__ void bitonic_sort_u32(unsigned* k, int np) {
  for (int kk = 2; kk <= np; kk <<= 1)
    for (int j = kk >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < np; i += NTH) {
        const int l = i ^ j;
        if (l > i) {
          const unsigned a = k[i], c = k[l];
          if ((a > c) == ((i & kk) == 0)) {
            k[i] = c;
            k[l] = a;
          }
        }
      }
      __syncthreads();
    }
}

__global__ void __launch_bounds__(kBinThreads)
k_bin_scatter_det(const double* __restrict__ x, const double* __restrict__ y, int64_t M, BinGeom g, int ppw,
                  const int* __restrict__ off, const int* __restrict__ bin_base, BinRec* __restrict__ recs) {
  constexpr int NW = kBinThreads / 64;
  __shared__ unsigned key[kDetRecs];
  __shared__ int slot_of[kDetRecs];  // by record id 4 p + k
  __shared__ int wsum[NW], wmax[NW];
  const int T = g.TX * g.TX;
  const int* myoff = off + (size_t)blockIdx.x * (T + 1);
  const int64_t j0 = (int64_t)blockIdx.x * ppw;
  const int np = (int)(min(M, j0 + ppw) - j0);  // <= kDetPoints (checked by the launcher)
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  PointCells pc = point_cells(t < np ? x[j0 + t] : 0.0, t < np ? y[j0 + t] : 0.0, g);
  if (t >= np) pc.ok = false;
  const int bx0 = pc.i0x / kTile, nbx = (pc.i0x + g.w - 1) / kTile - bx0 + 1;
  const int by0 = pc.i0y / kTile, nby = (pc.i0y + g.w - 1) / kTile - by0 + 1;
  const int nrec = pc.ok ? nbx * nby : 0;
  // compaction: exclusive block scan of the per-point record counts
  const int incl = wave_incl_scan(nrec, lane);
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  int base = incl - nrec, total = 0;
  for (int w2 = 0; w2 < NW; ++w2) {
    if (w2 < wv) base += wsum[w2];
    total += wsum[w2];
  }
  int E = 2;
  while (E < total) E <<= 1;
  {
    int o = base;
    for (int k = 0; k < 4; ++k) {
      const int kx = k & 1, ky = k >> 1;
      if (!pc.ok || kx >= nbx || ky >= nby) continue;
      key[o++] = ((unsigned)((by0 + ky) * g.TX + bx0 + kx) << kDetRecBits) | (unsigned)(4 * t + k);
    }
  }
  for (int i = total + t; i < E; i += kBinThreads) key[i] = 0xffffffffu;
  __syncthreads();
  bitonic_sort_u32<kBinThreads>(key, E);
  // run starts: start(i) = max over i' <= i of (i' if a bin's run begins at
  // i'); each thread scans a contiguous block of the sorted keys
  const int per = (E + kBinThreads - 1) / kBinThreads;
  const int i0 = min(E, t * per), i1 = min(E, i0 + per);
  int run = -1;
  for (int i = i0; i < i1; ++i)
    if (i == 0 || (key[i] >> kDetRecBits) != (key[i - 1] >> kDetRecBits)) run = i;
  int rmax = run;
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(rmax, o, 64);
    if (lane >= o) rmax = max(rmax, v);
  }
  if (lane == 63) wmax[wv] = rmax;
  __syncthreads();
  int before = -1;  // latest run start before this thread's block
  for (int w2 = 0; w2 < wv; ++w2) before = max(before, wmax[w2]);
  {
    const int up = __shfl_up(rmax, 1, 64);
    if (lane > 0) before = max(before, up);
  }
  run = before;
  for (int i = i0; i < i1 && i < total; ++i) {
    const unsigned kv = key[i];
    const int b = (int)(kv >> kDetRecBits);
    if (i == 0 || b != (int)(key[i - 1] >> kDetRecBits)) run = i;
    slot_of[kv & (kDetRecs - 1)] = bin_base[b] + myoff[b] + (i - run);
  }
  __syncthreads();
  for (int k = 0; k < 4; ++k) {
    const int kx = k & 1, ky = k >> 1;
    if (!pc.ok || kx >= nbx || ky >= nby) continue;
    const int bx = bx0 + kx, by = by0 + ky;
    const int lx = pc.i0x - bx * kTile, ly = pc.i0y - by * kTile;
    BinRec r;
    r.packed = (lx & 0xff) | ((ly & 0xff) << 8) | ((k == 0) ? (1 << 16) : 0);
    r.dx = pc.dx;
    r.dy = pc.dy;
    r.idx = (int32_t)(j0 + t);
    recs[slot_of[4 * t + k]] = r;
  }
}

// ------------------------------------------------------------- spreading
// Gather form, no atomics on the grid.  One workgroup per chunk of a bin.  A
// sub-batch of the chunk's records is counting-sorted in LDS by first-tap
// cell (first taps range over [-(w-1), 31]^2 relative to the bin), with the
// kernel weights of every record staged next to it (zero-padded by one entry
// on both sides).  Thread t owns a 2 x 2 block of the 32 x 32 bin in
// registers and walks only the records whose w x w footprint covers it: first
// taps in a (w+1) x (w+1) window, i.e. w+1 contiguous runs of the sorted
// order, taken two runs at a time.  Every grid cell is then written once.  A
// bin split into several chunks writes per-chunk partial tiles that
// k_spread_reduce sums in chunk order.
constexpr int kSpreadThreads = 256;

template <int W>
struct SpreadCfg {
  static constexpr int SB = spread_subbatch(W);  // records per LDS sub-batch (4 workgroups per CU at w = 7)
  static constexpr int RS = kTile + W - 1;       // first-tap cells per axis
  static constexpr int NC = RS * RS;
  static constexpr int WP = W + 2;               // padded weights, d = -1 .. w
  static_assert(kSpreadChunk == spread_nsub(W, false) * SB, "the default chunk is a whole number of sub-batches");
};

// 16-bit counters packed two per LDS word (a sub-batch has at most 448
// records): returns the count before the increment.
__device__ __forceinline__ int lds_bump16s(unsigned short* cnt, int k) {
  const int sft = (k & 1) * 16;
  return (int)((atomicAdd(reinterpret_cast<unsigned*>(cnt) + (k >> 1), 1u << sft) >> sft) & 0xffffu);
}

template <int W, int NSUB>
__global__ void __launch_bounds__(kSpreadThreads) k_spread(SpreadArgs a) {
  // NSUB: sub-batches per chunk (the chunk tables hold at most NSUB * SB
  // records per chunk)
  using Cfg = SpreadCfg<W>;
  constexpr int SB = Cfg::SB, RS = Cfg::RS, NC = Cfg::NC, WP = Cfg::WP, NT = kSpreadThreads;
  constexpr int PER = (SB + NT - 1) / NT;  // records per thread per sub-batch
  __shared__ float2 sc[SB];
  __shared__ float swx[SB][WP];
  __shared__ float swy[SB][WP];
  __shared__ int slx[SB];
  __shared__ __align__(4) unsigned short soff[(NC + 2) & ~1];  // cell counts, then offsets
  const int cid = blockIdx.x;
  if (cid >= a.nchunks[0]) return;
  const int4 ch = a.chunks[cid];
  const int bin = ch.x, start = ch.y, n = ch.z, slot = ch.w;
  const int t = threadIdx.x;
  const int x0 = 2 * (t & 15), y0 = 2 * (t >> 4);
  const float blog = a.beta * 1.4426950408889634f;
  // every record of the chunk and its value, loaded up front
  BinRec rl[NSUB][PER];
  float2 cv[NSUB][PER];
#pragma unroll
  for (int sb = 0; sb < NSUB; ++sb)
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int r = sb * SB + t + q * NT;
      if (t + q * NT < SB && r < n) rl[sb][q] = a.recs[start + r];
    }
#pragma unroll
  for (int sb = 0; sb < NSUB; ++sb)
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int r = sb * SB + t + q * NT;
      cv[sb][q] = (t + q * NT < SB && r < n) ? a.vals[rl[sb][q].idx] : czero();
    }
  float2 a00 = czero(), a01 = czero(), a10 = czero(), a11 = czero();
#pragma unroll
  for (int sb = 0; sb < NSUB; ++sb) {
    const int b0 = sb * SB;
    if (b0 >= n) break;
    const int nsb = min(SB, n - b0);
    for (int e = t; e <= NC; e += NT) soff[e] = 0;
    __syncthreads();
    int key[PER], rank[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int r = t + q * NT;
      key[q] = 0;
      rank[q] = 0;
      if (r < nsb) {
        key[q] = (rec_ly(rl[sb][q].packed) + W - 1) * RS + rec_lx(rl[sb][q].packed) + W - 1;
        rank[q] = lds_bump16s(soff, key[q]);
      }
    }
    __syncthreads();
    if (t < 64) {  // exclusive scan of the cell counts by one wave
      constexpr int per = (NC + 63) / 64;
      const int s0 = min(NC, t * per), s1 = min(NC, s0 + per);
      int acc = 0;
      for (int e = s0; e < s1; ++e) acc += soff[e];
      int incl = acc;
      for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o, 64);
        if (t >= o) incl += v;
      }
      int run = incl - acc;
      for (int e = s0; e < s1; ++e) {
        const int c = soff[e];
        soff[e] = run;
        run += c;
      }
      if (t == 63) soff[NC] = run;
    }
    __syncthreads();
    if (a.stable) {
      // deterministic mode: ranks in position order.  The positions are
      // placed at the atomic ranks (in the weight array, not yet in use); a
      // record's stable rank counts the lower positions in its cell's run.
      static_assert(SB * 2 <= (int)sizeof(swy), "stable-rank scratch");
      unsigned short* spos = reinterpret_cast<unsigned short*>(&swy[0][0]);
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int r = t + q * NT;
        if (r < nsb) spos[soff[key[q]] + rank[q]] = (unsigned short)r;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int r = t + q * NT;
        if (r < nsb) {
          const int s0 = soff[key[q]], s1 = soff[key[q] + 1];
          int below = 0;
          for (int i = s0; i < s1; ++i) below += spos[i] < r ? 1 : 0;
          rank[q] = below;  // rank inside the run, in position order
        }
      }
      __syncthreads();  // before the staging below overwrites the scratch
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int r = t + q * NT;
      if (r < nsb) {
        const BinRec& rc = rl[sb][q];
        const int slot = soff[key[q]] + rank[q];
        sc[slot] = cv[sb][q];
        slx[slot] = rec_lx(rc.packed);
        swx[slot][0] = 0.f;
        swy[slot][0] = 0.f;
        swx[slot][W + 1] = 0.f;
        swy[slot][W + 1] = 0.f;
#pragma unroll
        for (int m = 0; m < W; ++m) {
          swx[slot][m + 1] = es_kernel_fast(rc.dx + (float)m, a.two_over_w, blog);
          swy[slot][m + 1] = es_kernel_fast(rc.dy + (float)m, a.two_over_w, blog);
        }
      }
    }
    __syncthreads();
    // candidates: first taps in rows y0-(w-1) .. y0+1 and columns x0-(w-1) ..
    // x0+1, i.e. w+1 contiguous runs of the sorted order.  Runs are walked in
    // pairs as one sequence (positions 0 .. la-1 in run k, then run k+1), two
    // candidates per step, so a wave steps as often as its longest pair needs
    // rather than its longest run twice.
#pragma unroll
    for (int k = 0; k <= W; k += 2) {
      const int rowA = x0 + (y0 + k) * RS;  // soff index of run k: (ly + w - 1) * RS + x0, ly = y0 - (w-1) + k
      const int ra = soff[rowA], la = soff[rowA + W + 1] - ra;
      int rb = 0, lb = 0;
      if (k + 1 <= W) {
        rb = soff[rowA + RS];
        lb = soff[rowA + RS + W + 1] - rb;
      }
      const int n = la + lb;
      const int shift = rb - la;  // position p >= la lies at record rb + (p - la)
      for (int q = 0; q < n; q += 2) {
        const bool inA = q < la, two = q + 1 < n, inA2 = q + 1 < la;
        const int r = inA ? ra + q : shift + q;
        const int r2 = !two ? r : (inA2 ? ra + q + 1 : shift + q + 1);
        const int dya = inA ? W - k : W - k - 1;  // index of wy for output row y0
        // the second candidate, when there is none, repeats the first (so
        // every read stays inside the staged rows) and is masked by a zero value
        const int dyb = !two ? dya : (inA2 ? W - k : W - k - 1);
        const int dxa = x0 - slx[r] + 1, dxb = x0 - slx[r2] + 1;
        const float wa0 = swx[r][dxa], wa1 = swx[r][dxa + 1];
        const float wb0 = swx[r2][dxb], wb1 = swx[r2][dxb + 1];
        const float ya0 = swy[r][dya], ya1 = swy[r][dya + 1];
        const float yb0 = swy[r2][dyb], yb1 = swy[r2][dyb + 1];
        const float2 ca = sc[r];
        float2 cb = sc[r2];
        if (!two) cb = czero();
        {
          const float p0r = ca.x * ya0, p0i = ca.y * ya0, p1r = ca.x * ya1, p1i = ca.y * ya1;
          a00.x += p0r * wa0;
          a00.y += p0i * wa0;
          a01.x += p0r * wa1;
          a01.y += p0i * wa1;
          a10.x += p1r * wa0;
          a10.y += p1i * wa0;
          a11.x += p1r * wa1;
          a11.y += p1i * wa1;
        }
        {
          const float p0r = cb.x * yb0, p0i = cb.y * yb0, p1r = cb.x * yb1, p1i = cb.y * yb1;
          a00.x += p0r * wb0;
          a00.y += p0i * wb0;
          a01.x += p0r * wb1;
          a01.y += p0i * wb1;
          a10.x += p1r * wb0;
          a10.y += p1i * wb0;
          a11.x += p1r * wb1;
          a11.y += p1i * wb1;
        }
      }
    }
    __syncthreads();
  }
  if (slot < 0) {
    const int bx = bin % a.TX, by = bin / a.TX;
    const int gx = bx * kTile + x0, gy = by * kTile + y0;
    float2* g = a.grid;
    if (gy < a.L) {
      if (gx < a.L) g[(size_t)gy * a.L + gx] = a00;
      if (gx + 1 < a.L) g[(size_t)gy * a.L + gx + 1] = a01;
    }
    if (gy + 1 < a.L) {
      if (gx < a.L) g[(size_t)(gy + 1) * a.L + gx] = a10;
      if (gx + 1 < a.L) g[(size_t)(gy + 1) * a.L + gx + 1] = a11;
    }
  } else {
    float2* part = a.scratch + (size_t)slot * (kTile * kTile);
    part[y0 * kTile + x0] = a00;
    part[y0 * kTile + x0 + 1] = a01;
    part[(y0 + 1) * kTile + x0] = a10;
    part[(y0 + 1) * kTile + x0 + 1] = a11;
  }
}

// Sum the partial tiles of every multi-chunk bin, in chunk order (the bin's
// chunks hold consecutive scratch slots, the first one's in its table entry).
__global__ void __launch_bounds__(256) k_spread_reduce(SpreadReduceArgs a) {
  if ((int)blockIdx.x >= a.nmulti[0]) return;
  const int bin = a.multi[blockIdx.x];
  const int c0 = a.bin_chunk0[bin], nb = a.bin_nchunk[bin];
  const int slot0 = a.chunks[c0].w;
  const int bx = bin % a.TX, by = bin / a.TX;
  for (int e = threadIdx.x; e < kTile * kTile; e += 256) {
    float2 s = czero();
    for (int q = 0; q < nb; ++q) s = cadd(s, a.scratch[(size_t)(slot0 + q) * (kTile * kTile) + e]);
    const int yy = e / kTile, xx = e % kTile;
    const int gy = by * kTile + yy, gx = bx * kTile + xx;
    if (gy < a.L && gx < a.L) a.grid[(size_t)gy * a.L + gx] = s;
  }
}

// Scatter form: one workgroup per chunk of a bin accumulates every record's
// w x w taps into an LDS tile with native float atomic adds (ds_add_f32), one
// plane for the real and one for the imaginary parts.  The tile is the bin
// padded by w - 1 cells on every side, so that the taps of a record whose
// first tap lies up to w - 1 cells before the bin (a duplicate recorded in
// this bin) land in the padding without a bounds test; only the 32 x 32
// interior is written out.  Tap (my, mx) of a record is at a compile-time
// offset my * TS + mx from the record's first tap, so each add is one LDS
// instruction with an immediate offset.  The order of the additions into a
// cell is not fixed (deterministic mode uses the gather form).
template <int W>
struct SpreadLdsCfg {
  static constexpr int TS = kTile + 2 * (W - 1);  // padded tile side
  static constexpr int NT = 256;
  static constexpr int B = 2;                     // records per thread in flight
};

template <int W>
__global__ void __launch_bounds__(SpreadLdsCfg<W>::NT) k_spread_lds(SpreadArgs a) {
  using Cfg = SpreadLdsCfg<W>;
  constexpr int TS = Cfg::TS, NT = Cfg::NT, B = Cfg::B;
  __shared__ float sre[TS * TS];
  __shared__ float sim[TS * TS];
  const int cid = blockIdx.x;
  if (cid >= a.nchunks[0]) return;
  const int4 ch = a.chunks[cid];
  const int bin = ch.x, start = ch.y, n = ch.z, slot = ch.w;
  const int t = threadIdx.x;
  for (int e = t; e < TS * TS; e += NT) {
    sre[e] = 0.f;
    sim[e] = 0.f;
  }
  __syncthreads();
  const float blog = a.beta * 1.4426950408889634f;
  for (int r0 = 0; r0 < n; r0 += NT * B) {
    BinRec rl[B];
    float2 cv[B];
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const int r = r0 + t + q * NT;
      rl[q].packed = 0;
      rl[q].dx = rl[q].dy = 0.f;
      rl[q].idx = -1;
      if (r < n) rl[q] = a.recs[start + r];
    }
#pragma unroll
    for (int q = 0; q < B; ++q) cv[q] = rl[q].idx >= 0 ? a.vals[rl[q].idx] : czero();
#pragma unroll
    for (int q = 0; q < B; ++q) {
      if (rl[q].idx < 0) continue;
      const int base = (rec_ly(rl[q].packed) + W - 1) * TS + rec_lx(rl[q].packed) + W - 1;
      float wx[W];
#pragma unroll
      for (int m = 0; m < W; ++m) wx[m] = es_kernel_fast(rl[q].dx + (float)m, a.two_over_w, blog);
#pragma unroll
      for (int my = 0; my < W; ++my) {
        const float wy = es_kernel_fast(rl[q].dy + (float)my, a.two_over_w, blog);
        const float cr = cv[q].x * wy, ci = cv[q].y * wy;
        float* pr = sre + base + my * TS;
        float* pi = sim + base + my * TS;
#pragma unroll
        for (int mx = 0; mx < W; ++mx) {
          atomicAdd(pr + mx, cr * wx[mx]);
          atomicAdd(pi + mx, ci * wx[mx]);
        }
      }
    }
  }
  __syncthreads();
  const int bx = bin % a.TX, by = bin / a.TX;
  for (int e = t; e < kTile * kTile; e += NT) {
    const int yy = e / kTile, xx = e % kTile;
    const int s = (yy + W - 1) * TS + xx + W - 1;
    const float2 v = make_float2(sre[s], sim[s]);
    if (slot < 0) {
      const int gy = by * kTile + yy, gx = bx * kTile + xx;
      if (gy < a.L && gx < a.L) a.grid[(size_t)gy * a.L + gx] = v;
    } else {
      a.scratch[(size_t)slot * (kTile * kTile) + e] = v;
    }
  }
}

// --------------------------------------------------------- interpolation
// One workgroup per chunk of a bin: stage the bin plus its (w - 1)-cell halo
// of the fine grid in LDS; each primary record of the chunk (first tap inside
// the bin) gathers its w x w taps from it and writes its caller-order slot.
// Records are taken kInterpBatch per thread at a time so that their loads are
// in flight together.
constexpr int kInterpThreads = 256;
constexpr int kInterpBatch = 4;
// (launch bound: at least 5 waves per SIMD, i.e. at most 96 VGPRs)

template <int W>
__global__ void __launch_bounds__(kInterpThreads, 5) k_interp(InterpArgs a) {
  constexpr int RS = kTile + W - 1;
  constexpr int NT = kInterpThreads, B = kInterpBatch;
  __shared__ float2 sg[RS * RS];
  const int cid = blockIdx.x;
  if (cid >= a.nchunks[0]) return;
  const int4 ch = a.chunks[cid];
  const int bin = ch.x, start = ch.y, n = ch.z;
  const int bx = bin % a.TX, by = bin / a.TX;
  const int t = threadIdx.x;
  for (int e = t; e < RS * RS; e += NT) {
    const int yy = e / RS, xx = e % RS;
    const int gy = by * kTile + yy, gx = bx * kTile + xx;
    sg[e] = (gy < a.L && gx < a.L) ? a.grid[(size_t)gy * a.L + gx] : czero();
  }
  __syncthreads();
  const float blog = a.beta * 1.4426950408889634f;
  for (int r0 = 0; r0 < n; r0 += NT * B) {
    BinRec rl[B];
#pragma unroll
    for (int q = 0; q < B; ++q) {
      const int r = r0 + t + q * NT;
      rl[q].packed = 0;  // not primary
      if (r < n) rl[q] = a.recs[start + r];
    }
#pragma unroll
    for (int q = 0; q < B; ++q) {
      if (!rec_primary(rl[q].packed)) continue;
      const int lx = rec_lx(rl[q].packed), ly = rec_ly(rl[q].packed);
      float wx[W];
#pragma unroll
      for (int m = 0; m < W; ++m) wx[m] = es_kernel_fast(rl[q].dx + (float)m, a.two_over_w, blog);
      float accr = 0.f, acci = 0.f;
#pragma unroll
      for (int my = 0; my < W; ++my) {
        const float wy = es_kernel_fast(rl[q].dy + (float)my, a.two_over_w, blog);
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
      a.out[rl[q].idx] = make_float2(accr, acci);
    }
  }
}

// Device wall-clock stamp (constant-rate counter), for per-plane latency.
__global__ void k_stamp(long long* __restrict__ out) {
  if (threadIdx.x == 0) *out = wall_clock64();
}

// --------------------------------------------------------------- launchers
hipError_t launch_stamp(long long* out, hipStream_t st) {
  hipLaunchKernelGGL(k_stamp, dim3(1), dim3(64), 0, st, out);
  return hipGetLastError();
}

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

static hipError_t bin_lds_attr(const void* k, int bytes) {
  if (bytes > 64 * 1024) return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  return hipSuccess;
}

hipError_t launch_bin_hist(const double* x, const double* y, int64_t M, BinGeom g, int ppw, int G,
                           uint16_t* hist, hipStream_t st) {
  if (G <= 0) return hipSuccess;
  const int T = g.TX * g.TX, bytes = ((T + 2) / 2) * 4;
  hipError_t e = bin_lds_attr((const void*)k_bin_hist, bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bin_hist, dim3(G), dim3(kBinThreads), bytes, st, x, y, M, g, ppw, hist);
  return hipGetLastError();
}

hipError_t launch_bin_colscan(const uint16_t* hist, int G, int T, int* off, int* total, const BinScanOut& so,
                              int* done, hipStream_t st) {
  const int cols = T + 1;
  hipLaunchKernelGGL(k_bin_colscan, dim3((cols + 63) / 64), dim3(64 * kColWaves), 0, st, hist, G, cols, off,
                     total, so, done);
  return hipGetLastError();
}

hipError_t launch_bin_scatter(const double* x, const double* y, int64_t M, BinGeom g, int ppw, int G,
                              const int* off, const int* bin_base, BinRec* recs, bool stable, hipStream_t st) {
  if (G <= 0) return hipSuccess;
  const int T = g.TX * g.TX;
  if (stable) {
    if (ppw > kDetPoints) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bin_scatter_det, dim3(G), dim3(kBinThreads), 0, st, x, y, M, g, ppw, off, bin_base,
                       recs);
    return hipGetLastError();
  }
  if (T * 4 <= kScatterCursorBytes) {
    hipLaunchKernelGGL(k_bin_scatter<true>, dim3(G), dim3(kBinThreads), T * 4, st, x, y, M, g, ppw, off, bin_base,
                       recs);
  } else {
    const int bytes = ((T + 1) / 2) * 4;
    hipError_t e = bin_lds_attr((const void*)k_bin_scatter<false>, bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bin_scatter<false>, dim3(G), dim3(kBinThreads), bytes, st, x, y, M, g, ppw, off, bin_base,
                       recs);
  }
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

hipError_t launch_spread(int w, bool small_chunks, const SpreadArgs& a, int grid, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
#define CALL(W)                                                                                          \
  {                                                                                                      \
    if (small_chunks)                                                                                    \
      hipLaunchKernelGGL((k_spread<W, spread_nsub(W, true)>), dim3(grid), dim3(kSpreadThreads), 0, st, a);  \
    else                                                                                                 \
      hipLaunchKernelGGL((k_spread<W, spread_nsub(W, false)>), dim3(grid), dim3(kSpreadThreads), 0, st, a); \
  }
  NUASM_DISPATCH_W(w, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_spread_lds(int w, const SpreadArgs& a, int grid, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
#define CALL(W) hipLaunchKernelGGL(k_spread_lds<W>, dim3(grid), dim3(SpreadLdsCfg<W>::NT), 0, st, a)
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
