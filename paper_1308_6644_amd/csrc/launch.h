// Internal interface between the host plan code and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"

namespace nuasm {

constexpr int kTile = 32;        // default fine cells per bin side (32 or 64)
constexpr int kPad = 8;          // support margin: taps reach w/2 <= 8 cells past the window
constexpr int kChunk = 2048;       // default max records per interpolation workgroup
constexpr int kSpreadChunk = 1792; // default max records per spreading workgroup
// Spreading chunk sizes the kernel is instantiated for: whole sub-batches of
// 448 records (w <= 8) or 256 (w > 8); `small` is about half the default.
__host__ __device__ constexpr int spread_subbatch(int w) { return w <= 8 ? 448 : 256; }
__host__ __device__ constexpr int spread_nsub(int w, bool small) {
  return small ? (w <= 8 ? 2 : 4) : (w <= 8 ? 4 : 7);
}
constexpr int kMaxW = 16;

// Geometry of the fine-grid support and of the uniform planes.
struct GridGeom {
  int N, Np, nf;   // plane side, N' = 2N, fine grid nf = 2 N''
  int Npf;         // spectral grid N'': N', or a power of two >= 32 covering the band of Eq. 4
  int L, s0;       // support side N'' + 2*kPad, first support row/column in the fine grid
  int kxlo, kxhi;  // inclusive band of Eq. 4, index units
  int kylo, kyhi;
  int Nin;         // side of the uniform input of the type-2 pipeline (N, or N' for the type-1 adjoint)
  int crop;        // type-1 pipeline writes only the central N x N
};

// Everything the fused spectral kernels need to form D(kx) D(ky) H(k) R(k).
struct Spectral {
  int tf;          // 0 = ASM (Eq. 4), 1 = Fresnel (Eq. 5)
  int phase_fp64;  // ASM phase in float64 (1) or float32 (0)
  int conj;        // apply conj(H) (adjoint)
  float scale;     // N'^-2
  // ASM: cycles = c0 + ax kx + ay ky - zl (1 - sqrt(1 - t)), t = ql2 k^2,
  // with zl = z / l, ql2 = (l df)^2 and c0 = z / l reduced mod 1
  double c0, ax, ay, zl, ql2;
  // float32 variant: cycles = axf kx + ayf ky + zf sqrt(inv_lam2f - qf k^2)
  float axf, ayf, qf, zf, inv_lam2f;
  const float2* fre_x;  // Fresnel: A * H_x(k), index k + N'/2
  const float2* fre_y;  // Fresnel: H_y(k), index k + N'/2
  const float* dinv;    // 1 / psihat(k), index k + N'/2
};

// The non-uniform plane in fine-grid units: N''/2 raster pixels of pitch
// g N'/N'' across the window (the plan's own pixels when N'' = N').
struct BinGeom {
  int N;            // raster pixels across the window, N''/2
  double inv_g;     // 1 / raster pitch, N'' / (N' g)
  double half_n;    // N''/4: the window's half-width in raster pixels (range check)
  double tau0;      // support coordinate of raster pixel 0: N''/2 + kPad
  int w;            // kernel width
  int L;            // support side
  int TX;           // bins per axis
  int tile_log;     // log2 of the bin side in fine cells (5 or 6)
  int primary_only; // one record per point, in the bin of its first tap (interpolation only)
};

// Arguments of the row and column passes of the grid pipelines.
struct RowArgs {
  const float2* in;
  float2* out;
  GridGeom g;
  const float* dinv;   // deconvolution weights (row passes that apply them)
  const float2* tw;    // twiddle tables
};
struct ColArgs {
  const float2* in;
  float2* out;
  GridGeom g;
  Spectral sp;
  const float2* tw;
};

// Outputs of the bin scan (bin bases, chunk tables and their counts).
struct BinScanOut {
  int* cursor;       // first record of each bin
  int4* sp_chunks;   // spreading chunks (bin, first record, count, partial-tile slot or -1)
  int* sp_first;     // first spreading chunk of each bin
  int* sp_n;         // spreading chunks of each bin
  int* multi;        // bins with several spreading chunks
  int4* ip_chunks;   // interpolation chunks
  int* nch;          // spread chunks, interp chunks, records, multi bins, points out of range,
                     // partial-tile slots of split bins
  int* bin_pre;      // [T][kBinPre] per-bin prefixes inside the bin's column-scan workgroup
  int* wg_sum;       // [bin_scan_workgroups(T)][kBinPre] that workgroup's sums
  int sp_chunk;      // max records per spreading chunk
  int ip_chunk;      // max records per interpolation chunk
};
constexpr int kBinPre = 12;  // ints per row of bin_pre / wg_sum
int bin_scan_workgroups(int T);  // workgroups of the column scan over T bins

struct ColscanArgs {
  const uint16_t* hist;
  int G, T;                // ranges, bins
  int* off;
  int* total;
  BinScanOut so;
};

// Arguments of the binning kernels (histogram, scatter).
struct BinArgs {
  const double* x;
  const double* y;
  int64_t M;
  BinGeom g;
  int ppw;                 // points per binning workgroup
  uint16_t* hist;          // histogram rows (histogram pass)
  const int* off;          // per-range offsets (scatter)
  const int* bin_base;     // first record of each bin (scatter)
  BinRec* recs;            // records (scatter)
  int* rej_end;            // one past the end of the record buffer: the caller
                           // indices of points outside the window are stored
                           // downwards from here (scatter; the records, at
                           // most four per accepted point, never reach them)
};

// Outputs of the points outside the window (deferred range check) set to NaN.

struct SpreadArgs {
  const BinRec* recs;
  const int4* chunks;     // (bin, first record, count, partial-tile slot or -1)
  const int* nchunks;     // device count of valid chunks (element 0)
  float2* scratch;        // partial tiles of split bins, one per slot
  const float2* vals;     // point values, caller order
  float2* grid;           // L x L support
  int L, TX;
  float two_over_w, beta;
  int stable;             // deterministic mode: records ranked in position order
};

struct SpreadReduceArgs {
  const int4* chunks;     // spreading chunk table (slot of a chunk in .w)
  const int* multi;       // multi-chunk bins
  const int* nmulti;      // their count
  const int* bin_chunk0;  // first chunk of each bin
  const int* bin_nchunk;  // chunks of each bin
  const float2* scratch;
  float2* grid;
  int L, TX;
  int tile_log;           // log2 of the bin side
};

struct InterpArgs {
  const BinRec* recs;
  const int4* chunks;
  const int* nchunks;
  const float2* grid;
  float2* out;            // caller order
  const int* rej_end;     // end of the list of points outside the window (indices stored downwards)
  const int* nrej;        // their count (0 once a synchronised set_points has accepted every point)
  int L, TX;
  float two_over_w, beta;
};

// A non-uniform plane that is a uniform grid (scaled diffraction): nx x ny
// points, point [b][a] at (cx + (a - nx/2) pitch, cy + (b - ny/2) pitch)
// metres (integer division).  Its fine-grid taps follow the same rule as a
// binned point's (tau = 2 x inv_g + tau0 as in BinGeom, first tap
// ceil(tau - w/2)), so the separable kernels apply the weights the generic
// spreading and interpolation would.
struct GridPts {
  int nx, ny;
  double pitch, cx, cy;
  double inv_g;     // as BinGeom
  double half_n;
  double tau0;
  int L;            // support side
  float two_over_w, beta_log2e;
  int ty0, nrows;   // support rows the interpolation's x pass produces
};

// ---- launchers (return hipGetLastError() of the launch) -------------------
hipError_t launch_fill_i32(int* p, int v, int64_t n, hipStream_t st);
// counting sort of (point, bin) pairs: hist -> colscan -> scan -> scatter
constexpr int kBinPointsMax = 65535;  // points per binning workgroup (16-bit LDS counters)
constexpr int kBinPointsStable = 1024;  // the same in deterministic mode (stable scatter in LDS)
// hist rows and offset rows have T + 1 entries (entry T: points outside the window)
hipError_t launch_bin_hist(const double* x, const double* y, int64_t M, BinGeom g, int ppw, int G,
                           uint16_t* hist, hipStream_t st);
// column scan + bin scan (T bins; hist / off rows of T + 1 entries)
hipError_t launch_bin_colscan(const uint16_t* hist, int G, int T, int* off, int* total, const BinScanOut& so,
                              hipStream_t st);
hipError_t launch_bin_scan(int T, const int* total, const BinScanOut& so, hipStream_t st);
hipError_t launch_bin_scatter(const double* x, const double* y, int64_t M, BinGeom g, int ppw, int G,
                              const int* off, const int* bin_base, BinRec* recs, int* rej_end, bool stable,
                              hipStream_t st);
hipError_t launch_spread(int w, bool small_chunks, const SpreadArgs& a, int grid, hipStream_t st);
// the same spreading as sums of outer products on the matrix cores
hipError_t launch_spread_mfma(int w, int tile, const SpreadArgs& a, int grid, hipStream_t st);
hipError_t launch_spread_reduce(const SpreadReduceArgs& a, int grid, hipStream_t st);
hipError_t launch_interp(int w, int tile, const InterpArgs& a, int grid, hipStream_t st);
// separable interpolation at a grid: support (L x L) -> R (nrows x nx) -> out (ny x nx)
hipError_t launch_grid_interp(int w, const float2* fine, float2* R, float2* out, const GridPts& p, hipStream_t st);
// separable spreading of grid values (ny x nx) -> S (ny x L) -> support (L x L)
hipError_t launch_grid_spread(int w, const float2* vals, float2* S, float2* fine, const GridPts& p, hipStream_t st);

// type-1 pipeline: fine support (L x L) -> rows -> fused columns -> rows -> plane
// (row passes over the fine grid take log2 N'', the column pass both sizes)
hipError_t launch_t1_rows(int logNp, const float2* fine, float2* T, GridGeom g, const float* dinv,
                          const float2* tw, hipStream_t st);
hipError_t launch_t1_cols(int logNpf, int logNp, const float2* T, float2* V, GridGeom g, Spectral sp,
                          const float2* tw, hipStream_t st);
hipError_t launch_t1_rows_inv(int logNp, const float2* V, float2* out, GridGeom g, const float2* tw,
                              hipStream_t st);
// type-2 pipeline: plane (Nin x Nin) -> rows -> fused columns -> fine rows (L x L)
hipError_t launch_t2_rows(int logNp, const float2* u1, float2* T, GridGeom g, const float* dinv,
                          const float2* tw, hipStream_t st);
hipError_t launch_t2_cols(int logNpf, int logNp, const float2* T, float2* V, GridGeom g, Spectral sp,
                          const float2* tw, hipStream_t st);
hipError_t launch_t2_rows_inv(int logNp, const float2* V, float2* fine, GridGeom g, const float2* tw,
                              hipStream_t st);
// type-3 column pass: source support rows (after launch_t1_rows) -> FFT ->
// transfer function and deconvolutions -> inverse FFT -> destination support
// rows (for launch_t2_rows_inv)
hipError_t launch_t3_cols(int logNp, const float2* T, float2* V, GridGeom g, Spectral sp,
                          const float2* tw, hipStream_t st);

// Rayleigh-Sommerfeld direct summation (Eq. 10): constants of one propagation
struct RsConst {
  double ox, oy;     // offset o added to the destination points, metres
  double inv_z2;     // 1 / z^2
  double inv_lz;     // 1 / (l |z|)
  double c0;         // |z| / l reduced to [-1/2, 1/2]
  double inv_2pi;    // 1 / (2 pi)
  float a3;          // z / |z|^3
  float ak;          // k z / z^2, k = 2 pi / l
};
hipError_t launch_rs_direct(const double* x1, const double* y1, const float2* c, int64_t M1, const double* x2,
                            const double* y2, int64_t M2, const RsConst& k, float2* out, hipStream_t st);

hipError_t launch_stamp(long long* out, hipStream_t st);
hipError_t launch_transfer_table(const GridGeom& g, const Spectral& sp, float2* out, hipStream_t st);
hipError_t launch_fresnel_axis(int Np, double g, double two_lam_z, double o, double2 amp,
                               float2* out, hipStream_t st);
hipError_t launch_fft_rows(int logn, int64_t batch, int sign, const float2* in, float2* out,
                           const float2* tw, hipStream_t st);

// Twiddle tables: for length n = 2^logn (1 <= logn <= kMaxLogN) the table
// tw[m] = exp(-2 pi i m / n), m < n, starts at element n of one buffer.
constexpr int kMaxLogN = 14;
__host__ __device__ inline const float2* tw_for(const float2* all, int logn) { return all + (1 << logn); }

}  // namespace nuasm
