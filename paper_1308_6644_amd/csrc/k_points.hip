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
#include "group.h"
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
__device__ __forceinline__ void bin_hist_body(const BinArgs& a, int bid, int) {
  const double* __restrict__ x = a.x;
  const double* __restrict__ y = a.y;
  const int64_t M = a.M;
  const BinGeom& g = a.g;
  const int ppw = a.ppw;
  uint16_t* __restrict__ hist = a.hist;
  extern __shared__ unsigned sh[];
  const int T = g.TX * g.TX, TW = (T + 2) / 2;
  const int64_t j0 = (int64_t)bid * ppw;
  const int64_t j1 = min(M, j0 + ppw);
  double xv[kBinBatch], yv[kBinBatch];  // all loads of a batch in flight together
  // positions clamped into the range (never empty), so that no load sits
  // behind a branch; points past its end are skipped where they are used
  auto load = [&](int64_t jb) {
#pragma unroll
    for (int q = 0; q < kBinBatch; ++q) {
      const int64_t j = min(jb + threadIdx.x + q * kBinThreads, j1 - 1);
      xv[q] = x[j];
      yv[q] = y[j];
    }
  };
  load(j0);  // the first batch in flight while the counters are cleared
  for (int e = threadIdx.x; e < TW; e += kBinThreads) sh[e] = 0u;
  __syncthreads();
  for (int64_t jb = j0; jb < j1; jb += kBinThreads * kBinBatch) {
    if (jb != j0) load(jb);
#pragma unroll
    for (int q = 0; q < kBinBatch; ++q) {
      const int64_t j = jb + threadIdx.x + q * kBinThreads;
      if (j >= j1) continue;
      const PointCells pc = point_cells(xv[q], yv[q], g);
      if (!pc.ok) {
        lds_bump16(sh, T);
        continue;
      }
      // every bin the taps touch, or only the first tap's (interpolation only)
      const int bx0 = pc.i0x >> g.tile_log, bx1 = g.primary_only ? bx0 : (pc.i0x + g.w - 1) >> g.tile_log;
      const int by0 = pc.i0y >> g.tile_log, by1 = g.primary_only ? by0 : (pc.i0y + g.w - 1) >> g.tile_log;
      for (int by = by0; by <= by1; ++by)
        for (int bx = bx0; bx <= bx1; ++bx) lds_bump16(sh, by * g.TX + bx);
    }
  }
  __syncthreads();
  uint16_t* row = hist + (size_t)bid * (T + 1);
  for (int b = threadIdx.x; b <= T; b += kBinThreads) row[b] = (uint16_t)((sh[b >> 1] >> ((b & 1) * 16)) & 0xffffu);
}

// Column scan and bin scan (two launches).  The column scan gives
// off[g][b] = sum_{g' < g} hist[g'][b] and the bin totals (records per bin;
// entry T of the rows counts the points outside the window).  The bin scan
// turns the totals into the first record of every bin (`cursor`, the bin bases
// the scatter adds) and the chunk tables.  Spreading needs a chunk for every
// bin (empty bins write zeros); interpolation only for non-empty bins.  A bin
// with more than so.sp_chunk (so.ip_chunk) records is split into several
// spreading (interpolation) chunks; for spreading those bins are listed in
// `multi` for the reduction, and their chunks get consecutive slots of the
// partial-tile scratch (nch[5] slots in all).  Both chunk tables are ordered by
// the size class of their bin, largest first (a bin's chunks kept together,
// bins in index order inside a class), so that the dispatcher starts the
// longest workgroups first.
//
// Column scan: a workgroup owns 64 consecutive bins (a lane each) and splits
// the G ranges over its 16 waves; its last wave, holding the totals, also
// scans its 64 bins: exclusive prefixes of the records, of the split bins, of
// their slots and of the chunks of each size class, stored per bin, and the
// workgroup's sums of the same quantities.  Bin scan: one workgroup per
// column-scan workgroup reduces those sums to its own exclusive prefix and to
// the totals, and writes its 64 bins' entries.  No workgroup of either launch
// waits for another.
constexpr int kColWaves = 16;
constexpr int kColThreads = 64 * kColWaves;
constexpr int kClasses = 4;       // chunk size classes per table
constexpr int kColRegs = 16;      // ranges per wave held in registers (G <= 256)
constexpr int kScanThreads = 256;
// per-workgroup sums: records, split bins, slots, then the chunks of each
// class of the spreading and of the interpolation table
constexpr int kWgRec = 0, kWgMulti = 1, kWgSlot = 2, kWgSp = 3, kWgIp = 3 + kClasses;
constexpr int kWgVals = 3 + 2 * kClasses;  // 11
static_assert(kWgVals <= kBinPre, "per-bin prefixes fit the table row");

// size class of a bin of c records split into chunks of at most `chunk`:
// 3 for a full chunk, 2 for at least half, 1 for at least an eighth, else 0
__device__ __forceinline__ int size_class(int c, int chunk) {
  return c >= chunk ? 3 : 2 * c >= chunk ? 2 : 8 * c >= chunk ? 1 : 0;
}

__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int spread_chunks(int c, int spc) { return c > spc ? (c + spc - 1) / spc : 1; }

__device__ __forceinline__ void bin_colscan_body(const ColscanArgs& a, int bid, int) {
  const uint16_t* __restrict__ hist = a.hist;
  const int G = a.G, T = a.T;  // T: bins; rows of hist and off have T + 1 entries
  int* __restrict__ off = a.off;
  int* total = a.total;
  const BinScanOut& so = a.so;
  const int R = T + 1;
  __shared__ int part[kColWaves][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int b = bid * 64 + lane;
  const int per = (G + kColWaves - 1) / kColWaves;
  const int g0 = min(G, wv * per), g1 = min(G, g0 + per);
  int s = 0;
  if (per <= kColRegs) {
    // one pass: the wave's rows held in registers
    int h[kColRegs];
#pragma unroll
    for (int q = 0; q < kColRegs; ++q) h[q] = (b < R && g0 + q < g1) ? hist[(size_t)(g0 + q) * R + b] : 0;
#pragma unroll
    for (int q = 0; q < kColRegs; ++q) s += h[q];
    part[wv][lane] = s;
    __syncthreads();
    int run = 0;
    for (int q = 0; q < wv; ++q) run += part[q][lane];
    if (b < R) {
#pragma unroll
      for (int q = 0; q < kColRegs; ++q) {
        if (g0 + q < g1) off[(size_t)(g0 + q) * R + b] = run;
        run += h[q];
      }
      if (wv == kColWaves - 1) total[b] = run;
    }
  } else {
    if (b < R) {
#pragma unroll 8
      for (int gg = g0; gg < g1; ++gg) s += hist[(size_t)gg * R + b];
    }
    part[wv][lane] = s;
    __syncthreads();
    int run = 0;
    for (int q = 0; q < wv; ++q) run += part[q][lane];
    if (b < R) {
#pragma unroll 8
      for (int gg = g0; gg < g1; ++gg) {
        const int hv = hist[(size_t)gg * R + b];
        off[(size_t)gg * R + b] = run;
        run += hv;
      }
      if (wv == kColWaves - 1) total[b] = run;
    }
  }
  if (wv != kColWaves - 1) return;
  // the workgroup's 64 bins: per-bin exclusive prefixes and the sums
  int c = 0;
  if (b < T) {
    c = part[0][lane];
    for (int q = 1; q < kColWaves; ++q) c += part[q][lane];
  }
  const bool valid = b < T;
  const int nsp = valid ? spread_chunks(c, so.sp_chunk) : 0;
  const int nip = (c + so.ip_chunk - 1) / so.ip_chunk;
  const int ksp = size_class(c, so.sp_chunk), kip = size_class(c, so.ip_chunk);
  int v[kWgVals];
  v[kWgRec] = c;
  v[kWgMulti] = nsp > 1 ? 1 : 0;
  v[kWgSlot] = nsp > 1 ? nsp : 0;
#pragma unroll
  for (int k = 0; k < kClasses; ++k) {
    v[kWgSp + k] = ksp == k ? nsp : 0;
    v[kWgIp + k] = kip == k ? nip : 0;
  }
  int pre[kWgVals];
#pragma unroll
  for (int i = 0; i < kWgVals; ++i) {
    const int inc = wave_incl_scan(v[i], lane);
    pre[i] = inc - v[i];
    if (lane == 63) so.wg_sum[(size_t)bid * kBinPre + i] = inc;
  }
  if (valid) {
    int* bp = so.bin_pre + (size_t)b * kBinPre;
    bp[0] = pre[kWgRec];
    bp[1] = pre[kWgMulti];
    bp[2] = pre[kWgSlot];
    int psp = 0, pip = 0;
#pragma unroll
    for (int k = 0; k < kClasses; ++k) {
      if (ksp == k) psp = pre[kWgSp + k];
      if (kip == k) pip = pre[kWgIp + k];
    }
    bp[3] = psp;
    bp[4] = pip;
  }
}

// Bin scan: workgroup w (of the nbid column-scan workgroups) sums the
// column-scan sums of workgroups 0..w-1 (its prefix) and of all (the totals),
// wave v taking values v, v + 4, ..., and then its first wave writes the
// entries of bins 64 w .. 64 w + 63.  Workgroup 0 also writes the counts.
__device__ __forceinline__ void bin_scan_body(const ColscanArgs& a, int bid, int nbid) {
  const int T = a.T;
  const int* __restrict__ total = a.total;
  const BinScanOut& so = a.so;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int bb = bid * 64 + lane;
  __shared__ int wpre[kWgVals], tot[kWgVals];
  // the bin's own entries first, so that their latency overlaps the sums
  int c = 0, pre[5] = {0, 0, 0, 0, 0};
  if (wv == 0 && bb < T) {
    c = total[bb];
    const int* bp = so.bin_pre + (size_t)bb * kBinPre;
#pragma unroll
    for (int v = 0; v < 5; ++v) pre[v] = bp[v];
  }
  for (int i = wv; i < kWgVals; i += kScanThreads / 64) {
    int sp = 0, st = 0;
    for (int w0 = 0; w0 < nbid; w0 += 64) {
      const int w = w0 + lane;
      const int x = w < nbid ? so.wg_sum[(size_t)w * kBinPre + i] : 0;
      st += x;
      sp += w < bid ? x : 0;
    }
    sp = wave_sum(sp);
    st = wave_sum(st);
    if (lane == 0) {
      wpre[i] = sp;
      tot[i] = st;
    }
  }
  __syncthreads();
  if (wv != 0) return;
  if (bid == 0 && lane == 0) {
    int nsp_all = 0, nip_all = 0;
    for (int k = 0; k < kClasses; ++k) {
      nsp_all += tot[kWgSp + k];
      nip_all += tot[kWgIp + k];
    }
    so.nch[0] = nsp_all;
    so.nch[1] = nip_all;
    so.nch[2] = tot[kWgRec];
    so.nch[3] = tot[kWgMulti];
    so.nch[4] = total[T];
    so.nch[5] = tot[kWgSlot];
  }
  if (bb >= T) return;
  const int spc = so.sp_chunk, ipc = so.ip_chunk;
  const int nsp = spread_chunks(c, spc);
  const int nip = (c + ipc - 1) / ipc;
  const int ksp = size_class(c, spc), kip = size_class(c, ipc);
  // class bases, largest class first
  int bsp = 0, bip = 0;
#pragma unroll
  for (int k = kClasses - 1; k >= 0; --k) {
    if (k > ksp) bsp += tot[kWgSp + k];
    if (k > kip) bip += tot[kWgIp + k];
  }
  const int rec0 = wpre[kWgRec] + pre[0];
  const int first = bsp + wpre[kWgSp + ksp] + pre[3];
  const int ifirst = bip + wpre[kWgIp + kip] + pre[4];
  const int slot0 = wpre[kWgSlot] + pre[2];
  so.cursor[bb] = rec0;
  so.sp_first[bb] = first;
  so.sp_n[bb] = nsp;
  // .w: the chunk's partial-tile slot when the bin is split, else -1
  for (int r = 0; r < nsp; ++r)
    so.sp_chunks[first + r] = make_int4(bb, rec0 + r * spc, min(spc, c - r * spc), nsp > 1 ? slot0 + r : -1);
  for (int r = 0; r < nip; ++r)
    so.ip_chunks[ifirst + r] = make_int4(bb, rec0 + r * ipc, min(ipc, c - r * ipc), nip);
  if (nsp > 1) so.multi[wpre[kWgMulti] + pre[1]] = bb;
}

// CURSORS: the workgroup's write cursors bin_base[b] + off[g][b] are staged in
// LDS once and bumped there (one LDS atomic per record, no global loads);
// otherwise 16-bit LDS ranks are added to the two global tables per record
// (for supports with too many bins to stage 32-bit cursors).
template <bool CURSORS>
__device__ __forceinline__ void bin_scatter_body(const BinArgs& a, int bid, int) {
  const double* __restrict__ x = a.x;
  const double* __restrict__ y = a.y;
  const int64_t M = a.M;
  const BinGeom& g = a.g;
  const int ppw = a.ppw;
  const int* __restrict__ off = a.off;
  const int* __restrict__ bin_base = a.bin_base;
  BinRec* __restrict__ recs = a.recs;
  extern __shared__ unsigned sh[];
  const int T = g.TX * g.TX, TW = (T + 1) / 2;
  const int* myoff = off + (size_t)bid * (T + 1);
  const int64_t j0 = (int64_t)bid * ppw;
  const int64_t j1 = min(M, j0 + ppw);
  double xv[kBinBatch], yv[kBinBatch];
  // positions clamped into the range (never empty), so that no load sits
  // behind a branch; points past its end are skipped where they are used
  auto load = [&](int64_t jb) {
#pragma unroll
    for (int q = 0; q < kBinBatch; ++q) {
      const int64_t j = min(jb + threadIdx.x + q * kBinThreads, j1 - 1);
      xv[q] = x[j];
      yv[q] = y[j];
    }
  };
  load(j0);  // the first batch in flight with the cursor staging
  if (CURSORS) {
    // the loads of eight bins per thread in flight together (clamped
    // addresses), then the LDS writes; entry T is the cursor of the range's
    // points outside the window
    // Every load and LDS write is unconditional (no load behind a branch): an
    // entry past T is clamped to T and written, with the same value, by
    // several lanes.
    constexpr int NB = 8;
    int base[NB], o[NB];
    auto stage_load = [&](int b0) {
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int b = min(b0 + (int)threadIdx.x + u * kBinThreads, T);
        base[u] = bin_base[min(b, T - 1)];
        o[u] = myoff[b];
      }
    };
    auto stage_write = [&](int b0) {
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const int b = min(b0 + (int)threadIdx.x + u * kBinThreads, T);
        sh[b] = (unsigned)((b < T ? base[u] : 0) + o[u]);
      }
    };
    stage_load(0);
    // every load above (and the first coordinates) issued before any is used
    __builtin_amdgcn_sched_barrier(0);
    stage_write(0);
    for (int b0 = kBinThreads * NB; b0 <= T; b0 += kBinThreads * NB) {
      stage_load(b0);
      stage_write(b0);
    }
  } else {
    for (int e = threadIdx.x; e < TW; e += kBinThreads) sh[e] = 0u;
  }
  __syncthreads();
  for (int64_t jb = j0; jb < j1; jb += kBinThreads * kBinBatch) {
    if (jb != j0) load(jb);
#pragma unroll
    for (int q = 0; q < kBinBatch; ++q) {
      const int64_t j = jb + threadIdx.x + q * kBinThreads;
      if (j >= j1) continue;
      const PointCells pc = point_cells(xv[q], yv[q], g);
      if (!pc.ok) {
        // outside the window: no record; its index is listed for the NaN
        // outputs of a deferred range check
        const int r = CURSORS ? (int)atomicAdd(&sh[T], 1u) : myoff[T] + (int)lds_bump16(sh, T);
        a.rej_end[-1 - r] = (int)j;
        continue;
      }
      const int bx0 = pc.i0x >> g.tile_log, bx1 = g.primary_only ? bx0 : (pc.i0x + g.w - 1) >> g.tile_log;
      const int by0 = pc.i0y >> g.tile_log, by1 = g.primary_only ? by0 : (pc.i0y + g.w - 1) >> g.tile_log;
      for (int by = by0; by <= by1; ++by)
        for (int bx = bx0; bx <= bx1; ++bx) {
          const int b = by * g.TX + bx;
          const int slot = CURSORS ? (int)atomicAdd(&sh[b], 1u)
                                   : bin_base[b] + myoff[b] + (int)lds_bump16(sh, b);
          const int lx = pc.i0x - (bx << g.tile_log), ly = pc.i0y - (by << g.tile_log);
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

__device__ __forceinline__ void bin_scatter_det_body(const BinArgs& a, int bid, int) {
  const double* __restrict__ x = a.x;
  const double* __restrict__ y = a.y;
  const int64_t M = a.M;
  const BinGeom& g = a.g;
  const int ppw = a.ppw;
  const int* __restrict__ off = a.off;
  const int* __restrict__ bin_base = a.bin_base;
  BinRec* __restrict__ recs = a.recs;
  constexpr int NW = kBinThreads / 64;
  __shared__ unsigned key[kDetRecs];
  __shared__ int slot_of[kDetRecs];  // by record id 4 p + k
  __shared__ int wsum[NW], wmax[NW];
  __shared__ int nrej;
  const int T = g.TX * g.TX;
  const int* myoff = off + (size_t)bid * (T + 1);
  const int64_t j0 = (int64_t)bid * ppw;
  const int np = (int)(min(M, j0 + ppw) - j0);  // <= kDetPoints (checked by the launcher)
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  if (t == 0) nrej = 0;
  PointCells pc = point_cells(t < np ? x[j0 + t] : 0.0, t < np ? y[j0 + t] : 0.0, g);
  const bool rejected = t < np && !pc.ok;  // outside the window: listed for NaN outputs
  if (t >= np) pc.ok = false;
  const int bx0 = pc.i0x >> g.tile_log, nbx = g.primary_only ? 1 : ((pc.i0x + g.w - 1) >> g.tile_log) - bx0 + 1;
  const int by0 = pc.i0y >> g.tile_log, nby = g.primary_only ? 1 : ((pc.i0y + g.w - 1) >> g.tile_log) - by0 + 1;
  const int nrec = pc.ok ? nbx * nby : 0;
  // compaction: exclusive block scan of the per-point record counts
  const int incl = wave_incl_scan(nrec, lane);
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  if (rejected) a.rej_end[-1 - (myoff[T] + atomicAdd(&nrej, 1))] = (int)(j0 + t);
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
    const int lx = pc.i0x - (bx << g.tile_log), ly = pc.i0y - (by << g.tile_log);
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
__device__ __forceinline__ void spread_body(const SpreadArgs& a, int bid, int) {
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
  const int cid = bid;
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

// ----------------------------------------------- spreading on the matrix cores
// The spreading of one bin is a sum of outer products: cell (y, x) receives
// sum_j c_j wy_j(y) wx_j(x) over the bin's records j, where wy_j, wx_j are the
// record's kernel weights (zero outside its w taps).  For a 16 x 16 quarter of
// the bin that is D = A B with A[y][j] = c_j wy_j(y) and B[j][x] = wx_j(x): a
// contraction over the record index, which v_mfma_f32_16x16x4f32 evaluates
// four records at a time (float32 products and sums; the real and imaginary
// parts of c in two accumulators).  Each of the workgroup's four waves owns a
// quarter and walks, in groups of four, the records of the sub-batch whose
// footprint meets it (lists built with wave ballots, in record order, so the
// result does not depend on timing).  Operand lane l supplies A[i][k] and
// B[k][i] for record k = l / 16 of the group and row / column i = l % 16; the
// accumulator element e of lane l is D[4 (l / 16) + e][l % 16].
typedef float v4f __attribute__((ext_vector_type(4)));

struct __align__(16) MfmaRec {
  float cr, ci;  // the point's value
  int lxy;       // first tap relative to the bin origin: column (low 16 bits), row (high)
  int pad;
};

// Sub-batches of 256 records (one per thread), loaded one ahead: the LDS
// footprint (about 24 KB at w = 7) and the registers leave room for six
// workgroups per CU, which hide the load and LDS latencies.
constexpr int kMfmaSB = kSpreadThreads;

// What an empty chunk (a bin with no records, which still writes its zero
// tile) reads in place of its first record and that record's value: every
// load of the kernel stays unconditional and in bounds.
__device__ const BinRec kNoRecord = {0, 0.f, 0.f, 0};
__device__ const float2 kNoValue = {0.f, 0.f};

template <int W, int TILE>
__device__ __forceinline__ void spread_mfma_body(const SpreadArgs& a, int bid, int) {
  constexpr int SB = kMfmaSB, NWV = kSpreadThreads / 64;  // 4 waves
  constexpr int QS = TILE / 16, NQ = QS * QS;  // 16 x 16 quarter tiles of the bin
  constexpr int QPW = NQ / NWV;                // quarter tiles per wave: 1 (32 x 32 bins) or 4 (64 x 64)
  constexpr int NACC = QPW == 1 ? 2 : 1;       // accumulator pairs per quarter tile
  static_assert(NQ % NWV == 0, "whole quarter tiles per wave");
  // one LDS row per record: its MfmaRec, then its x weights and its y
  // weights, each with a zero on either side (tap m at 1 + m), so that an
  // operand is one read at a clamped tap index.  The lists hold row byte
  // offsets.  Record SB is a sentinel (zero value and weights) that pads the
  // lists to whole steps.
  constexpr int WP = W + 2, STEP = 4 * NACC;
  constexpr int RX = 4, RY = 4 + WP;                 // floats: x and y weights in a row
  constexpr int RSZ = (4 + 2 * WP + 3) / 4 * 4;      // row length, whole 16-byte units
  static_assert((SB + 1) * RSZ * 4 < 65536, "row offsets fit 16 bits");
  __shared__ __align__(16) float srow[(SB + 1) * RSZ];
  __shared__ unsigned short slist[NQ][SB + 2 * STEP];
  __shared__ int scnt[NWV][NQ];
  __shared__ int sbase[NWV][NQ];
  __shared__ int slen[NQ];
  const int cid = bid;
  // count and descriptor requested together (in bounds: the launch grid never
  // exceeds the table's capacity)
  const int nchunks = a.nchunks[0];
  const int4 ch = a.chunks[cid];
  // (bin, first record and count are never negative: testing them keeps the
  // descriptor's load ahead of the branch)
  if ((cid >= nchunks) | ((ch.x | ch.y | ch.z) < 0)) return;
  const int bin = ch.x, start = ch.y, n = ch.z, slot = ch.w;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const float blog = a.beta * 1.4426950408889634f;
  // the pads and the sentinel row (never written again: the staging below
  // writes only the record and the taps)
  for (int e = t; e < SB + 1; e += kSpreadThreads) {
    float* row = srow + e * RSZ;
    row[RX] = row[RX + W + 1] = row[RY] = row[RY + W + 1] = 0.f;
  }
  for (int e = t; e < RSZ; e += kSpreadThreads) srow[SB * RSZ + e] = 0.f;
  // the lane's operand row / column and record slot inside a group of four
  const int kk = lane >> 4, ii = lane & 15;
  v4f accr[QPW][NACC], acci[QPW][NACC];
#pragma unroll
  for (int u = 0; u < QPW; ++u)
#pragma unroll
    for (int h = 0; h < NACC; ++h) {
      accr[u][h] = v4f{0.f, 0.f, 0.f, 0.f};
      acci[u][h] = v4f{0.f, 0.f, 0.f, 0.f};
    }
  const unsigned long long below = (1ull << lane) - 1ull;
  // the thread's record of the first sub-batch and its value.  Every thread
  // loads, from a position clamped into the chunk, so that no load sits
  // behind a branch (a load whose result merges with a default at a branch
  // join is waited for at once, which would serialise the prefetch below).
  const int last = start + n - 1;
  const BinRec* rsrc = n > 0 ? a.recs + min(start + t, last) : &kNoRecord;
  BinRec rc = *rsrc;
  const float2* vsrc = n > 0 ? a.vals : &kNoValue;  // kNoRecord.idx = 0
  float2 cv = vsrc[rc.idx];
  for (int b0 = 0; b0 < n; b0 += SB) {
    const int nsb = min(SB, n - b0);
    const bool ok = t < nsb;
    // the next sub-batch's record, in flight while this one is staged; its
    // value is requested once the record has arrived (after the staging)
    const BinRec nx = a.recs[min(start + b0 + SB + t, last)];
    // stage: value, first tap, kernel weights; list the record under every
    // quarter tile its footprint meets
    int lx = 0, ly = 0;
    if (ok) {
      lx = rec_lx(rc.packed);
      ly = rec_ly(rc.packed);
      MfmaRec m;
      m.cr = cv.x;
      m.ci = cv.y;
      m.lxy = (lx & 0xffff) | (ly << 16);
      m.pad = 0;
      float* row = srow + t * RSZ;
      *reinterpret_cast<MfmaRec*>(row) = m;
#pragma unroll
      for (int mm = 0; mm < W; ++mm) {
        row[RX + 1 + mm] = es_kernel_fast(rc.dx + (float)mm, a.two_over_w, blog);
        row[RY + 1 + mm] = es_kernel_fast(rc.dy + (float)mm, a.two_over_w, blog);
      }
    }
    int rank[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int qx = 16 * (q % QS), qy = 16 * (q / QS);
      const bool meets = ok && lx <= qx + 15 && lx + W - 1 >= qx && ly <= qy + 15 && ly + W - 1 >= qy;
      const unsigned long long bal = __ballot(meets);
      rank[q] = meets ? __popcll(bal & below) : -1;
      if (lane == 0) scnt[wv][q] = __popcll(bal);
    }
    __syncthreads();
    // list bases: records of earlier waves first; each list padded with the
    // sentinel to a whole step
    if (t < NQ) {
      int run = 0;
      for (int w2 = 0; w2 < NWV; ++w2) {
        const int c2 = scnt[w2][t];
        sbase[w2][t] = run;
        run += c2;
      }
      const int padded = (run + STEP - 1) / STEP * STEP;
      for (int p = run; p < padded; ++p) slist[t][p] = (unsigned short)(SB * RSZ * 4);
      slen[t] = padded;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      if (rank[q] >= 0) slist[q][sbase[wv][q] + rank[q]] = (unsigned short)(t * RSZ * 4);
    __syncthreads();
    const float2 nv = a.vals[nx.idx];
    // the wave's quarter tiles: groups of four listed records, NACC groups
    // per step into NACC accumulator pairs (independent matrix operations,
    // loads in flight together)
#pragma unroll
    for (int u = 0; u < QPW; ++u) {
      const int q = wv * QPW + u;
      const int sx0 = 16 * (q % QS), sy0 = 16 * (q / QS);
      const int len = __builtin_amdgcn_readfirstlane(slen[q]);  // uniform: a scalar loop
      const int oy = sy0 + ii + 1, ox = sx0 + ii + 1;
      const char* base = reinterpret_cast<const char*>(srow);
      // the list entries of the next step are read one step ahead (the list
      // has room for the reads past its end; those values go unused)
      int off[NACC];
#pragma unroll
      for (int h = 0; h < NACC; ++h) off[h] = slist[q][4 * h + kk];
      for (int g = 0; g < len; g += STEP) {
        const char* rp[NACC];
#pragma unroll
        for (int h = 0; h < NACC; ++h) {
          rp[h] = base + off[h];
          off[h] = slist[q][g + STEP + 4 * h + kk];
        }
        MfmaRec m[NACC];
#pragma unroll
        for (int h = 0; h < NACC; ++h) m[h] = *reinterpret_cast<const MfmaRec*>(rp[h]);
#pragma unroll
        for (int h = 0; h < NACC; ++h) {
          const int mlx = (int)(short)(m[h].lxy & 0xffff), mly = m[h].lxy >> 16;
          // tap index of this row / column, clamped onto a zero pad outside
          const int ty = min(max(oy - mly, 0), W + 1);
          const int tx = min(max(ox - mlx, 0), W + 1);
          const float* wr = reinterpret_cast<const float*>(rp[h]);
          const float ay = wr[RY + ty];
          const float bx = wr[RX + tx];
          accr[u][h] = __builtin_amdgcn_mfma_f32_16x16x4f32(m[h].cr * ay, bx, accr[u][h], 0, 0, 0);
          acci[u][h] = __builtin_amdgcn_mfma_f32_16x16x4f32(m[h].ci * ay, bx, acci[u][h], 0, 0, 0);
        }
      }
    }
    __syncthreads();
    rc = nx;
    cv = nv;
  }
  // accumulator element e of lane l: quarter-tile row 4 (l / 16) + e, column l % 16
  const int bx = bin % a.TX, by = bin / a.TX;
#pragma unroll
  for (int u = 0; u < QPW; ++u) {
    const int q = wv * QPW + u;
    const int sx0 = 16 * (q % QS), sy0 = 16 * (q / QS);
    v4f r = accr[u][0], i = acci[u][0];
#pragma unroll
    for (int h = 1; h < NACC; ++h) {
      r += accr[u][h];
      i += acci[u][h];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int yy = sy0 + 4 * kk + e, xx = sx0 + ii;
      const float2 v = make_float2(r[e], i[e]);
      if (slot < 0) {
        const int gy = by * TILE + yy, gx = bx * TILE + xx;
        if (gy < a.L && gx < a.L) a.grid[(size_t)gy * a.L + gx] = v;
      } else {
        a.scratch[(size_t)slot * (TILE * TILE) + yy * TILE + xx] = v;
      }
    }
  }
}

// Sum the partial tiles of every multi-chunk bin, in chunk order (the bin's
// chunks hold consecutive scratch slots, the first one's in its table entry).
// Each workgroup sums 256 cells of one bin, a cell per thread:
// (tile / 16)^2 workgroups per bin.  The partial tiles are read four at a
// time (loads in flight together) and added in chunk order.
__device__ __forceinline__ void spread_reduce_body(const SpreadReduceArgs& a, int bid, int) {
  const int tl = a.tile_log, tile = 1 << tl, cells = tile * tile;
  const int parts = cells >> 8;
  const int mb = bid / parts, part = bid - mb * parts;
  if (mb >= a.nmulti[0]) return;
  const int bin = a.multi[mb];
  const int c0 = a.bin_chunk0[bin], nb = a.bin_nchunk[bin];
  const int slot0 = a.chunks[c0].w;
  const int bx = bin % a.TX, by = bin / a.TX;
  const int e = (part << 8) + threadIdx.x;
  const float2* p = a.scratch + (size_t)slot0 * cells + e;
  float2 s = czero();
  int q = 0;
  for (; q + 4 <= nb; q += 4) {
    const float2 v0 = p[(size_t)q * cells], v1 = p[(size_t)(q + 1) * cells];
    const float2 v2 = p[(size_t)(q + 2) * cells], v3 = p[(size_t)(q + 3) * cells];
    s = cadd(cadd(cadd(cadd(s, v0), v1), v2), v3);
  }
  for (; q < nb; ++q) s = cadd(s, p[(size_t)q * cells]);
  const int yy = e >> tl, xx = e & (tile - 1);
  const int gy = (by << tl) + yy, gx = (bx << tl) + xx;
  if (gy < a.L && gx < a.L) a.grid[(size_t)gy * a.L + gx] = s;
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

template <int W, int TILE>
__device__ __forceinline__ void interp_body(const InterpArgs& a, int bid, int nbid) {
  constexpr int RS = TILE + W - 1;
  constexpr int NT = kInterpThreads, B = kInterpBatch;
  __shared__ float2 sg[RS * RS];
  const int cid = bid;
  // the chunk count and the descriptor requested together (the launch grid
  // never exceeds the table's capacity, so the read is in bounds even for a
  // workgroup beyond the count, which leaves)
  const int nchunks = a.nchunks[0];
  const int4 ch = a.chunks[cid];
  const int nrej = a.nrej[0];
  // points outside the window (a deferred range check; they have no
  // records): NaN at their outputs, strided over every workgroup
  for (int i = bid * kInterpThreads + (int)threadIdx.x; i < nrej; i += nbid * kInterpThreads)
    a.out[a.rej_end[-1 - i]] = make_float2(__builtin_nanf(""), __builtin_nanf(""));
  // (bin, first record and count are never negative: testing them keeps the
  // descriptor's load ahead of the branch)
  if ((cid >= nchunks) | ((ch.x | ch.y | ch.z) < 0)) return;
  const int bin = ch.x, start = ch.y, n = ch.z;
  const int bx = bin % a.TX, by = bin / a.TX;
  const int t = threadIdx.x;
  // the first batch of records, in flight with the staging below (positions
  // clamped into the chunk, which is never empty; validity is checked on use)
  BinRec rl[B];
#pragma unroll
  for (int q = 0; q < B; ++q) rl[q] = a.recs[start + min(t + q * NT, n - 1)];
  {
    // every load of the staging first (clamped addresses, values selected
    // afterwards), then the LDS writes: one memory latency, not one per
    // element.  The writes are unconditional (no load is moved behind a
    // branch): a clamped element is written by several lanes, with one value.
    constexpr int NS = (RS * RS + NT - 1) / NT;
    float2 v[NS];
    int e[NS];
#pragma unroll
    for (int u = 0; u < NS; ++u) {
      e[u] = min(t + u * NT, RS * RS - 1);
      const int gy = by * TILE + e[u] / RS, gx = bx * TILE + e[u] % RS;
      v[u] = a.grid[(size_t)min(gy, a.L - 1) * a.L + min(gx, a.L - 1)];
      if (gy >= a.L || gx >= a.L) v[u] = czero();
    }
#pragma unroll
    for (int u = 0; u < NS; ++u) sg[e[u]] = v[u];
  }
  __syncthreads();
  const float blog = a.beta * 1.4426950408889634f;
  for (int r0 = 0; r0 < n; r0 += NT * B) {
    if (r0 > 0) {
#pragma unroll
      for (int q = 0; q < B; ++q) rl[q] = a.recs[start + min(r0 + t + q * NT, n - 1)];
    }
#pragma unroll
    for (int q = 0; q < B; ++q) {
      if (r0 + t + q * NT >= n || !rec_primary(rl[q].packed)) continue;
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


hipError_t launch_bin_hist(const double* x, const double* y, int64_t M, BinGeom g, int ppw, int G,
                           uint16_t* hist, hipStream_t st) {
  const int T = g.TX * g.TX, bytes = ((T + 2) / 2) * 4;
  BinArgs a{};
  a.x = x;
  a.y = y;
  a.M = M;
  a.g = g;
  a.ppw = ppw;
  a.hist = hist;
  return launch_or_record<BinArgs, bin_hist_body, kBinThreads>(a, G, bytes, st);
}

int bin_scan_workgroups(int T) { return (T + 1 + 63) / 64; }

hipError_t launch_bin_colscan(const uint16_t* hist, int G, int T, int* off, int* total, const BinScanOut& so,
                              hipStream_t st) {
  const ColscanArgs a{hist, G, T, off, total, so};
  return launch_or_record<ColscanArgs, bin_colscan_body, kColThreads>(a, bin_scan_workgroups(T), 0, st);
}

hipError_t launch_bin_scan(int T, const int* total, const BinScanOut& so, hipStream_t st) {
  const ColscanArgs a{nullptr, 0, T, nullptr, const_cast<int*>(total), so};
  return launch_or_record<ColscanArgs, bin_scan_body, kScanThreads>(a, bin_scan_workgroups(T), 0, st);
}

hipError_t launch_bin_scatter(const double* x, const double* y, int64_t M, BinGeom g, int ppw, int G,
                              const int* off, const int* bin_base, BinRec* recs, int* rej_end, bool stable,
                              hipStream_t st) {
  if (G <= 0) return hipSuccess;
  const int T = g.TX * g.TX;
  BinArgs a{};
  a.x = x;
  a.y = y;
  a.M = M;
  a.g = g;
  a.ppw = ppw;
  a.off = off;
  a.bin_base = bin_base;
  a.recs = recs;
  a.rej_end = rej_end;
  if (stable) {
    if (ppw > kDetPoints) return hipErrorInvalidValue;
    return launch_or_record<BinArgs, bin_scatter_det_body, kBinThreads>(a, G, 0, st);
  }
  if ((T + 1) * 4 <= kScatterCursorBytes)
    return launch_or_record<BinArgs, bin_scatter_body<true>, kBinThreads>(a, G, (T + 1) * 4, st);
  return launch_or_record<BinArgs, bin_scatter_body<false>, kBinThreads>(a, G, ((T + 1) / 2) * 4, st);
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
#define CALL(W)                                                                                               \
  {                                                                                                           \
    if (small_chunks)                                                                                         \
      return launch_or_record<SpreadArgs, spread_body<W, spread_nsub(W, true)>, kSpreadThreads>(a, grid, 0, st); \
    return launch_or_record<SpreadArgs, spread_body<W, spread_nsub(W, false)>, kSpreadThreads>(a, grid, 0, st);  \
  }
  NUASM_DISPATCH_W(w, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

hipError_t launch_spread_mfma(int w, int tile, const SpreadArgs& a, int grid, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  // any chunk size: sub-batches of 256 records
#define CALL(W)                                                                                           \
  {                                                                                                       \
    if (tile == 64) return launch_or_record<SpreadArgs, spread_mfma_body<W, 64>, kSpreadThreads>(a, grid, 0, st); \
    return launch_or_record<SpreadArgs, spread_mfma_body<W, 32>, kSpreadThreads>(a, grid, 0, st);           \
  }
  NUASM_DISPATCH_W(w, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

hipError_t launch_spread_reduce(const SpreadReduceArgs& a, int grid, hipStream_t st) {
  return launch_or_record<SpreadReduceArgs, spread_reduce_body, 256>(a, grid, 0, st);
}

hipError_t launch_interp(int w, int tile, const InterpArgs& a, int grid, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  // at least five waves per SIMD: at most 96 VGPRs
#define CALL(W)                                                                                         \
  {                                                                                                     \
    if (tile == 64) return launch_or_record<InterpArgs, interp_body<W, 64>, kInterpThreads, 5>(a, grid, 0, st); \
    return launch_or_record<InterpArgs, interp_body<W, 32>, kInterpThreads, 5>(a, grid, 0, st);           \
  }
  NUASM_DISPATCH_W(w, CALL)
#undef CALL
  return hipErrorInvalidValue;
}

}  // namespace nuasm
