/*
 * nuasm.h -- non-uniform sampled angular-spectrum (ASM) and Fresnel
 * diffraction on one AMD Instinct MI355X (gfx950).
 *
 * Operators (Shimobaba et al., arXiv 1308.6644):
 *
 *   NU-ASM_1 / NU-FRE_1 (Eq. 6, type-1 sum of Eq. 7): complex samples c_j at
 *     non-uniform source points p_j -> uniform N' x N' destination plane,
 *       u2[n] = N'^-2 sum_{k in K^2} H(k) F(k) exp(2 pi i k.n / N'),
 *       F(k)  = sum_j c_j exp(-2 pi i df k.p_j),   df = 1/(N' g).
 *   NU-ASM_2 / NU-FRE_2 (Eq. 9, type-2 sum of Eq. 8): uniform N x N source
 *     u1 -> complex samples at non-uniform destination points q_j,
 *       u2_j = N'^-2 sum_{k in K^2} H(k) U(k) exp(2 pi i df k.q_j),
 *       U(k) = sum_m u1[m] exp(-2 pi i k.m / N').
 *   NU-ASM_3 / NU-FRE_3 (the third type, stated after Eq. 9 as the
 *     combination of the first two): complex samples c_i at non-uniform
 *     source points p_i -> complex samples at non-uniform destination points
 *     q_j, both in the same N g window,
 *       u2_j = N'^-2 sum_{k in K^2} H(k) F(k) exp(2 pi i df k.q_j),
 *     with F the type-1 sum above; N' and g are the destination's (the paper
 *     names no intermediate grid).
 *
 *   N' = 2N (zero padding against circular wrap, the passage after Eq. 5),
 *   K = {-N'/2, ..., N'/2 - 1}, g is the pitch of the uniform plane
 *   (Delta_2 for type 1, Delta_1 for type 2, as stated under Eqs. 6 and 9;
 *   Delta_2 for type 3).
 *   H is the shifted band-limited ASM transfer function (Eq. 4) or the
 *   Fresnel transfer function (Eq. 5, the DFT of the impulse response
 *   sampled on the centred N' x N' grid with area element g^2).
 *
 * Layouts: complex values are complex64, interleaved (re, im).  Planes are
 * row-major with x fastest and centred: element [b][a] of an N' x N' plane is
 * the sample at n = (a - N'/2, b - N'/2), i.e. at global position n g + o;
 * element [b][a] of an N x N plane is pixel (a - N/2, b - N/2).  Point
 * coordinates are FP64 metres in the plane's local frame (window centre at
 * 0); they must satisfy -N g/2 <= x, y <= N g/2 (up to 1e-9 pixel of
 * rounding slack; such points are clamped onto the edge).
 *
 * Threading and streams: a plan is not thread-safe; use one plan per stream.
 * All device work of a call is enqueued on the plan's HIP stream.  execute()
 * never synchronises the host.  set_points() synchronises once (a 4-byte
 * readback) to report out-of-range points, unless the plan was created with
 * NUASM_DEFER_RANGE_CHECK, in which case nuasm_check_points() reports it.
 * Under a deferred check, points outside the window (or with NaN
 * coordinates) take no part in the operator: every output slot of such a
 * point (type-2 and type-3 destinations, type-1 adjoint values) is NaN, and a
 * type-1 result is the sum over the other points only, so a result is not to
 * be used unless nuasm_check_points() returns NUASM_OK.
 *
 * Errors: every call returns nuasm_status; nothing throws across the ABI.
 * nuasm_last_error() gives a thread-local human-readable detail of the most
 * recent failure on the calling thread.
 */
#ifndef NUASM_H
#define NUASM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NUASM_OK = 0,
  NUASM_ERR_INVALID_ARG = 1,   /* bad parameter, null pointer, wrong plan type */
  NUASM_ERR_OUT_OF_RANGE = 2,  /* a point lies outside the N g window */
  NUASM_ERR_NOT_READY = 3,     /* execute before a successful set_points */
  NUASM_ERR_UNSUPPORTED = 4,   /* N not a power of two in [16, 4096], ... */
  NUASM_ERR_NO_DEVICE = 5,     /* no HIP device visible */
  NUASM_ERR_ALLOC = 6,         /* device or pinned-host allocation failed */
  NUASM_ERR_HIP = 7,           /* a HIP runtime call failed */
  NUASM_STATUS_MAX = 0x7fffffff /* not a status: widens the type's range so
                                   that any value 0..INT32_MAX a caller passes
                                   to nuasm_status_string is a valid one */
} nuasm_status;

enum { NUASM_TYPE_1 = 1, NUASM_TYPE_2 = 2, NUASM_TYPE_3 = 3 };
enum { NUASM_TF_ASM = 0, NUASM_TF_FRESNEL = 1 };
/* Rect of Eq. 4: full grid; limited = aliasing-free band of the shifted ASM
 * (per axis |o - z f / sqrt(1/lambda^2 - f^2)| <= N g, edges inclusive);
 * explicit = caller's centre band_c and width band_w in frequency-index
 * units, |k - c| <= w/2.  Fresnel plans ignore the band. */
enum { NUASM_BAND_FULL = 0, NUASM_BAND_LIMITED = 1, NUASM_BAND_EXPLICIT = 2 };

/* params.flags */
#define NUASM_OUT_CROP_N        0x1u  /* type 1: write only the central N x N */
#define NUASM_DEFER_RANGE_CHECK 0x2u  /* set_points does not synchronise */
#define NUASM_FULL_FINE_GRID    0x4u  /* keep the fine grid at 2 N' even when the
                                         band of Eq. 4 would allow a smaller one */
#define NUASM_DETERMINISTIC     0x8u  /* bitwise-reproducible results: binning
                                         keeps every bin's records in point
                                         order (a stable scatter; ranges of at
                                         most 1024 points) and spreading ranks
                                         each sub-batch stably, so every sum
                                         runs in one order on every run, in
                                         every plan and batch */
#define NUASM_FORWARD_ONLY      0x10u /* type 2 only: the points are binned for
                                         interpolation alone, one record per
                                         point (in the bin of its first tap)
                                         instead of one per bin its taps touch;
                                         nuasm_execute_adjoint (which spreads)
                                         returns NUASM_ERR_UNSUPPORTED */

typedef struct {
  int32_t type;        /* NUASM_TYPE_1, NUASM_TYPE_2 or NUASM_TYPE_3 */
  int32_t tf;          /* NUASM_TF_ASM or NUASM_TF_FRESNEL */
  int32_t band;        /* NUASM_BAND_* (ASM only) */
  int32_t phase_fp64;  /* 1 (default): ASM phase in float64; 0: float32 */
  int64_t N;           /* plane side in pixels; N' = 2N; power of two, 16..4096 */
  double lambda;       /* wavelength, metres (> 0) */
  double z;            /* propagation distance, metres; < 0 back-propagates;
                          must be != 0 for Fresnel */
  double ox, oy;       /* off-axis offset o of Eq. 4, metres */
  double d1, d2;       /* source / destination pitch, metres; the uniform
                          plane's pitch is used: d2 for type 1, d1 for type 2;
                          type 3 uses d2 */
  double band_c[2];    /* NUASM_BAND_EXPLICIT: band centre (c_m, c_n), index units */
  double band_w[2];    /* NUASM_BAND_EXPLICIT: band width  (w_m, w_n), index units */
  double tol;          /* spreading-kernel tolerance, 1e-12 .. 1e-2 */
  uint32_t flags;      /* NUASM_OUT_CROP_N (type 1 only) | NUASM_DEFER_RANGE_CHECK |
                          NUASM_FULL_FINE_GRID | NUASM_DETERMINISTIC |
                          NUASM_FORWARD_ONLY (type 2 only) */
  uint32_t reserved;   /* must be 0 */
} nuasm_params;

typedef struct {
  int64_t N, Np, nf;          /* plane side, N' = 2N, fine grid nf = 2 N'' (N'' = Npf) */
  int64_t L;                  /* side of the stored fine-grid support, N'' + 16 */
  int32_t w;                  /* spreading-kernel width in fine cells */
  float beta;                 /* exponential-of-semicircle shape parameter */
  int32_t tile;               /* fine cells per bin side (nuasm_tuning.bin_tile) */
  int32_t tiles;              /* number of bins */
  int32_t kx_lo, kx_hi;       /* inclusive band of Eq. 4 in index units */
  int32_t ky_lo, ky_hi;
  int64_t in_elems, out_elems;/* complex elements of execute()'s in / out
                                 (for the current point count) */
  int64_t M;                  /* points of the last set_points (0 if none) */
  size_t device_bytes;        /* device memory the plan holds */
  int64_t M_dest;             /* type 3: points of the last set_dest_points */
  int32_t spread_chunk;       /* records per spreading workgroup (tuning) */
  int32_t interp_chunk;       /* records per interpolation workgroup (tuning) */
  int32_t bin_range_points;   /* points per binning workgroup for M (tuning) */
  int32_t Npf;                /* spectral grid N'': N', or, when the band of Eq. 4
                                 is narrow, the smallest power of two >= max(32,
                                 N'/8) whose centred index set holds the band;
                                 the fine grid is 2 N'' */
} nuasm_plan_info;

/* Launch-shape tuning of a plan (see nuasm_plan_set_tuning); 0 = default. */
typedef struct {
  int32_t spread_chunk;       /* max records per spreading workgroup: 0 = 1792;
                                 a value below 1792 selects the small size
                                 (896 records for w <= 8, 1024 above) */
  int32_t interp_chunk;       /* max records per interpolation workgroup: 0 = 2048,
                                 else 256 .. 65536 */
  int32_t bin_range_points;   /* points per binning workgroup: 0 = automatic
                                 (max(4096, M/256), at most 65535), else 1024 .. 65535 */
  int32_t spread_method;      /* 0 = automatic (matrix cores), 1 = register gather
                                 (each output cell sums the records covering it on
                                 the vector ALUs), 2 = matrix cores (each quarter
                                 bin as sums of outer products on v_mfma_f32 units).
                                 Both are float32 and reproducible in
                                 deterministic mode */
  int32_t bin_tile;           /* bin side in fine cells: 0 = 32, else 32 or 64
                                 (64: fewer records per point -- a point is
                                 recorded in every bin its w x w taps touch --
                                 and 16 times fewer bins, but larger spreading
                                 and interpolation workgroups; matrix-core
                                 spreading only) */
} nuasm_tuning;

typedef struct nuasm_plan_s* nuasm_plan;

/* Fill *p with defaults: type 1, ASM, full band, float64 phase, tol 1e-6. */
nuasm_status nuasm_params_default(nuasm_params* p);

/* Create a plan on the current HIP device for operator Eq. 6 (type 1),
 * Eq. 9 (type 2) or their combination (type 3) with transfer function Eq. 4
 * or Eq. 5.  hip_stream is a hipStream_t (NULL = default stream); it is
 * borrowed, not owned.  Builds the plan tables on the device (twiddles,
 * deconvolution weights, Fresnel axis transforms).  On failure *out is set
 * to NULL. */
nuasm_status nuasm_plan_create(const nuasm_params* p, void* hip_stream, nuasm_plan* out);

/* Release every resource of the plan.  NULL-safe.  Synchronises the plan's
 * stream first. */
nuasm_status nuasm_plan_destroy(nuasm_plan plan);

/* Change the stream later calls are enqueued on (borrowed).  Work the plan
 * has already enqueued on its previous stream (plan tables, a binning, an
 * execute) is ordered before anything later enqueued on the new one: an event
 * recorded on the old stream is waited on by the new stream, without blocking
 * the host.  The previous stream must still be valid when this is called. */
nuasm_status nuasm_plan_set_stream(nuasm_plan plan, void* hip_stream);

nuasm_status nuasm_plan_get_info(nuasm_plan plan, nuasm_plan_info* info);

/* Set the plan's launch shapes (chunk sizes of the spreading and
 * interpolation workgroups, points per binning workgroup), e.g. from an
 * autotuner's cache.  Results do not depend on them beyond float32
 * summation order.  Binned point sets must be bound again afterwards
 * (execute returns NUASM_ERR_NOT_READY until then); grids stay bound. */
nuasm_status nuasm_plan_set_tuning(nuasm_plan plan, const nuasm_tuning* t);

/* Caller-owned workspace (e.g. memory from a framework's caching allocator).
 * nuasm_plan_workspace_bytes: bytes a workspace needs so that every point set
 * of the plan (type 3: each of the two) can hold M_max points, for the plan's
 * current tuning: the two grid buffers of the pipelines of Eqs. 6 and 9 and
 * the point-count-dependent buffers of the binning (records, chunk tables,
 * per-range histograms, partial tiles of split bins).  0 <= M_max < 2^29.
 * nuasm_plan_set_workspace: carve those buffers from the device memory `dev`
 * (256-byte aligned, `bytes` long, caller-owned: it must stay valid and
 * otherwise unused until the plan is destroyed or given another workspace).
 * The plan frees its own copies of them and from then on allocates none of
 * them; its capacity becomes the largest point count per set that fits, and
 * set_points with more points returns NUASM_ERR_INVALID_ARG.  dev = NULL goes
 * back to plan-owned memory.  Binned point sets must be bound again
 * afterwards (execute returns NUASM_ERR_NOT_READY until then).  Small
 * T-sized bin arrays, the plan's tables and the buffers of a grid bound with
 * nuasm_set_grid_points stay plan-owned (nuasm_plan_info.device_bytes counts
 * what the plan itself holds).  A nuasm_plan_set_tuning that changes the sizes
 * carves the workspace again (and fails, keeping the old tuning, if the new
 * minimum does not fit).  Synchronises the plan's stream.  Errors:
 * NUASM_ERR_INVALID_ARG (misaligned, or below the minimum for 1024 points). */
nuasm_status nuasm_plan_workspace_bytes(nuasm_plan plan, int64_t M_max, size_t* bytes);
nuasm_status nuasm_plan_set_workspace(nuasm_plan plan, void* dev, size_t bytes);

/* Coordinate normalisation and binning of the non-uniform plane (Fig. 1 and
 * the text around Eqs. 7-9): M points x_dev[M], y_dev[M] (device FP64
 * metres) are converted once to fine-grid cells and offsets and sorted into
 * bins.  The arrays are read on the plan's stream and may be freed once the
 * stream has passed this call; the plan keeps its own sorted copy.  Returns
 * NUASM_ERR_OUT_OF_RANGE (and leaves the plan not ready) if any point is
 * outside the window or not finite.  M = 0 is allowed.  For a type-3 plan
 * these are the source points p_i. */
nuasm_status nuasm_set_points(nuasm_plan plan, int64_t M, const double* x_dev, const double* y_dev);

/* Type 3 only: bind the destination points q_j, with the same conventions,
 * range check and synchronisation as nuasm_set_points (NUASM_ERR_INVALID_ARG
 * for other plan types).  Each point set keeps its own buffers, so either
 * can be rebound without touching the other. */
nuasm_status nuasm_set_dest_points(nuasm_plan plan, int64_t M, const double* x_dev, const double* y_dev);

/* Scaled diffraction (the introduction's scaled ASM / Fresnel, which NU-ASM
 * generalises): bind a uniform nx x ny grid of pitch `pitch` metres centred
 * at (cx, cy) as a point set -- which = 0 for the plan's points (type 3: the
 * source), 1 for a type-3 plan's destination.  Point [b][a] of the grid sits
 * at (cx + (a - nx/2) pitch, cy + (b - ny/2) pitch) (integer division) and
 * the point-side arrays of execute / execute_adjoint are [ny][nx] in that
 * order.  The whole grid must lie in the window [-N g/2, N g/2]^2
 * (NUASM_ERR_OUT_OF_RANGE otherwise, checked on the host, nothing enqueued).
 * Such a set needs no binning: spreading and interpolation run as two
 * separable 1-D passes each (the stage timers record two launches under
 * NUASM_STAGE_SPREAD / NUASM_STAGE_INTERP).  May allocate a workspace of
 * max(rows reached x nx, ny x L) complex values; never synchronises
 * otherwise.  nx, ny <= 2^18, nx ny <= 2^30. */
nuasm_status nuasm_set_grid_points(nuasm_plan plan, int32_t which, int64_t nx, int64_t ny, double pitch, double cx,
                                   double cy);

/* With NUASM_DEFER_RANGE_CHECK: synchronise and report whether the last
 * set_points (and, for type 3, set_dest_points) saw out-of-range points
 * (NUASM_ERR_OUT_OF_RANGE) or not. */
nuasm_status nuasm_check_points(nuasm_plan plan);

/* Apply the operator.  Type 1: in_dev = c[M], out_dev = u2[N'][N'] (or
 * [N][N] with NUASM_OUT_CROP_N).  Type 2: in_dev = u1[N][N], out_dev = u2[M]
 * in the caller's point order.  Type 3: in_dev = c[M] (source order),
 * out_dev = u2[M_dest] (destination order).  Device pointers, complex64,
 * caller-owned, non-overlapping. */
nuasm_status nuasm_execute(nuasm_plan plan, const void* in_dev, void* out_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): nuasm_execute
 * exactly, except that the partial tiles of bins split over several spreading
 * workgroups go to a static device array of the library (2048 tiles of 32 x 32
 * complex64, 16 MiB per device, held until the process ends) instead of the
 * plan's own scratch, and no stage-timing events are recorded.  Calls no
 * hipMalloc / hipFree or any other allocating routine: every other buffer was
 * sized when the plan was created and its points bound.  The array is shared
 * by every call on a device and keeps the last call's contents; every tile a
 * call reads is written earlier in that call, so nothing needs clearing, but
 * calls whose work overlaps on one device (two streams, two threads) race on
 * it.  Returns NUASM_ERR_UNSUPPORTED, enqueuing nothing, if the bound points
 * may need more tiles than the array holds (the exact need is known when
 * set_points synchronised; with NUASM_DEFER_RANGE_CHECK a bound of
 * 8 M / spread_chunk tiles is used), and the errors of nuasm_execute. */
nuasm_status nuasm_execute_noalloc(nuasm_plan plan, const void* in_dev, void* out_dev);

/* Apply the adjoint (conjugate transpose) of the plan's operator, derived
 * from Eqs. 6 and 9 by reversing every step and conjugating H.  Type 1:
 * in_dev = v[N'][N'], out_dev = w[M].  Type 2: in_dev = w[M], out_dev =
 * u1'[N][N] (NUASM_ERR_UNSUPPORTED for a NUASM_FORWARD_ONLY plan).  Type 3:
 * in_dev = w[M_dest], out_dev = c'[M] (the type-3 operator from the
 * destination to the source points with conj H). */
nuasm_status nuasm_execute_adjoint(nuasm_plan plan, const void* in_dev, void* out_dev);

/* Write the transfer function exactly as the fused spectral kernel applies
 * it, H(k) of Eq. 4 or Eq. 5 times its Rect, as complex64 [N'][N'] centred
 * ([b][a] holds k = (a - N'/2, b - N'/2)), to out_dev.  For testing. */
nuasm_status nuasm_debug_transfer(nuasm_plan plan, void* out_dev);

/* Copy the records of a bound point set (which = 0; 1 for a type-3 plan's
 * destination) in the order the point kernels read them, and the number of
 * records of every bin, for testing.  recs_out_dev: device buffer of rec_cap
 * 16-byte records {int32 packed: bits 0-7 and 8-15 the first tap's column and
 * row relative to the bin origin (int8), bit 16 set in the bin that holds
 * the first tap; float dx, dy: first tap minus the point, fine cells; int32
 * the point's index}; bins are consecutive, row-major.  counts_out_dev:
 * device int32[tiles] (nuasm_plan_info.tiles).  *n_records receives the total.
 * Synchronises the plan's stream.  NUASM_ERR_NOT_READY unless the set holds
 * binned points; NUASM_ERR_INVALID_ARG if rec_cap is below the total. */
nuasm_status nuasm_debug_records(nuasm_plan plan, int32_t which, void* recs_out_dev, int64_t rec_cap,
                                 int32_t* counts_out_dev, int64_t* n_records);

/* Spreading alone, for testing: the values vals_dev (complex64, one per point
 * of the bound set `which`) spread with the plan's kernel onto the fine-grid
 * support, copied to grid_out_dev as complex64 [L][L] (nuasm_plan_info.L;
 * support cell (i, j) of a point's taps as the binning defines them).
 * Enqueued on the plan's stream.  NUASM_ERR_NOT_READY unless the set is
 * bound. */
nuasm_status nuasm_debug_spread(nuasm_plan plan, int32_t which, const void* vals_dev, void* grid_out_dev);

/* Interpolation alone, for testing: the support grid grid_dev (complex64
 * [L][L]) interpolated with the plan's kernel at the points of the bound set
 * `which`, into out_dev (complex64, one per point, caller order).  Enqueued on
 * the plan's stream.  NUASM_ERR_NOT_READY unless the set is bound. */
nuasm_status nuasm_debug_interp(nuasm_plan plan, int32_t which, const void* grid_dev, void* out_dev);

/* Plain batched 1-D FFT with the library's Stockham kernels, for testing:
 * `batch` (< 2^31) contiguous rows of length n (power of two, 32..16384),
 * complex64, forward (sign = -1) or unnormalised inverse (sign = +1), out of
 * place. */
nuasm_status nuasm_debug_fft(int64_t n, int64_t batch, int32_t sign, const void* in_dev,
                             void* out_dev, void* hip_stream);

/* Rayleigh-Sommerfeld diffraction by direct summation (Eq. 10, the paper's
 * accuracy reference), O(M1 M2):
 *   u2_j = 1/(2 pi) sum_i c_i (z/r)(1 - i k r) exp(i k r) / r^2,
 *   r = sqrt(|q_j + o - p_i|^2 + z^2),  k = 2 pi / lambda,
 * for M1 source points p_i = (x1, y1) with complex weights c_i that carry
 * each sample's area element (u1 g^2 for a uniform grid of pitch g) and M2
 * destination points q_j = (x2, y2).  Coordinates are device FP64 metres,
 * c and out device complex64 (caller-owned; out[M2] in destination order).
 * The phase is formed in FP64 (error ~1e-11 cycles), amplitudes and the
 * sums in FP32 with FP64 accumulation every 64 sources.  z != 0 (its sign
 * enters as the z/r factor of Eq. 10; r depends on z^2).  Plan-less:
 * enqueued on hip_stream (NULL = default stream), allocates nothing,
 * never synchronises.  M1 = 0 writes zeros; M2 = 0 does nothing. */
nuasm_status nuasm_rs_direct(int64_t M1, const double* x1_dev, const double* y1_dev, const void* c_dev,
                             int64_t M2, const double* x2_dev, const double* y2_dev, double lambda, double z,
                             double ox, double oy, void* out_dev, void* hip_stream);

/* Per-kernel device timing with HIP events recorded on the plan's stream
 * around each kernel launch (off by default).  Stages, one kernel each: */
#define NUASM_STAGE_BIN_HIST 0     /* set_points: per-range bin histograms */
#define NUASM_STAGE_BIN_COLSCAN 1  /* set_points: offsets across ranges, per-bin prefixes */
#define NUASM_STAGE_BIN_SCAN 2     /* set_points: bin bases and chunk tables */
#define NUASM_STAGE_BIN_SCATTER 3  /* set_points: records into bin order */
#define NUASM_STAGE_SPREAD 4       /* spreading */
#define NUASM_STAGE_SPREAD_REDUCE 5 /* sum of split bins' partial tiles */
#define NUASM_STAGE_T1_ROWS 6      /* type-1 pipeline: fine rows, FFT */
#define NUASM_STAGE_T1_COLS 7      /* type-1 pipeline: fused column pass */
#define NUASM_STAGE_T1_ROWS_INV 8  /* type-1 pipeline: inverse row FFT */
#define NUASM_STAGE_T2_ROWS 9      /* type-2 pipeline: plane rows, FFT */
#define NUASM_STAGE_T2_COLS 10     /* type-2 pipeline: fused column pass */
#define NUASM_STAGE_T2_ROWS_INV 11 /* type-2 pipeline: fine rows, inverse FFT */
#define NUASM_STAGE_INTERP 12      /* interpolation */
#define NUASM_STAGE_T3_COLS 13     /* type-3 pipeline: fused column pass (between
                                      T1_ROWS and T2_ROWS_INV) */
#define NUASM_NUM_STAGES 14
nuasm_status nuasm_plan_set_timing(nuasm_plan plan, int32_t enable);
/* Synchronise on the recorded events, add each stage's elapsed milliseconds
 * and launch count into ms[NUASM_NUM_STAGES] / launches[NUASM_NUM_STAGES]
 * (caller-owned host arrays, accumulated into, not overwritten) and forget
 * the recorded events. */
nuasm_status nuasm_plan_read_timing(nuasm_plan plan, double* ms, int64_t* launches);

/* ------------------------------------------------------------ batches
 * Many independent planes (each its own N, type, transfer function, z, point
 * count) run as one HIP graph: the binning and the operator of every plane
 * are captured once as grouped stage launches (see nuasm_batch_set_grouped)
 * and replayed by each run.  For
 * callers that propagate many planes per step (a batch of holograms, a
 * focal stack).  Plans inside a batch always defer their range checks.
 * Type-3 planes are not batched (nuasm_batch_create returns
 * NUASM_ERR_UNSUPPORTED). */
typedef struct nuasm_batch_s* nuasm_batch;

/* params[P]; hip_stream is borrowed.  On failure *out is NULL. */
nuasm_status nuasm_batch_create(int32_t P, const nuasm_params* params, void* hip_stream, nuasm_batch* out);
nuasm_status nuasm_batch_destroy(nuasm_batch batch);  /* NULL-safe */
/* One-shot run of every plane p: bin M[p] points x[p], y[p] (device FP64
 * metres) and apply the operator to in[p] -> out[p] (device complex64, shapes
 * as for nuasm_execute).  The first call with a given set of pointers and
 * counts records the graph (and runs it); later calls with the same arguments
 * only launch it.  Never synchronises the host then.  In the grouped form a
 * call with other buffers but the same counts keeps the recorded graph: it
 * waits for the graph's last run, rewrites the per-stage argument tables and
 * launches (any other change records the graph again). */
nuasm_status nuasm_batch_run(nuasm_batch batch, const int64_t* M, const double* const* x,
                             const double* const* y, const void* const* in, void* const* out);
/* The same work in two steps, for many operator runs on points bound once
 * (the iterations of a hologram optimisation over many planes): binning of
 * every plane's points (M[p], x[p], y[p] as above), recorded as one graph on
 * first use, then the operators of every plane (in[p] -> out[p]) recorded as
 * another.  Each graph is recorded again only when its arguments change
 * (execute_many's also when a plane's point count changed).  execute_many
 * returns NUASM_ERR_NOT_READY until every plane has points (and again after
 * nuasm_batch_set_tuning).  Never synchronise the host once recorded. */
nuasm_status nuasm_set_points_many(nuasm_batch batch, const int64_t* M, const double* const* x,
                                   const double* const* y);
nuasm_status nuasm_execute_many(nuasm_batch batch, const void* const* in, void* const* out);
/* Same as nuasm_batch_create. */
nuasm_status nuasm_plan_many_create(int32_t P, const nuasm_params* params, void* hip_stream, nuasm_batch* out);
/* Tuning of one plane of a batch (as nuasm_plan_set_tuning) and the number
 * of parallel graph branches of the per-plane form (1 .. min(4, P); default
 * the maximum), e.g. from an autotuner.  Either drops the recorded graphs; the
 * next run records them again. */
nuasm_status nuasm_batch_set_tuning(nuasm_batch batch, int32_t plane, const nuasm_tuning* t);
nuasm_status nuasm_batch_set_branches(nuasm_batch batch, int32_t branches);
/* How a batch's graphs are recorded.  grouped = 1 (default): grouped stage
 * launches -- every stage (binning histogram, column scan, scatter, spreading,
 * split-bin reduction, the row and column passes, interpolation) is one
 * launch per kernel instantiation covering every plane that has it, each
 * workgroup finding its plane's arguments in a per-stage descriptor table;
 * the type-1 planes' binning and operator run on one graph branch, the
 * type-2 planes' grid passes, binning and interpolation on another (each
 * stage grouped over the planes of its branch).  grouped = 0:
 * every plane's own launch sequence on one of `branches` parallel branches.
 * Drops the recorded graphs. */
nuasm_status nuasm_batch_set_grouped(nuasm_batch batch, int32_t grouped);
/* Synchronise; *bad_plane = index of the first plane with out-of-range
 * points in the last run, or -1. */
nuasm_status nuasm_batch_check_points(nuasm_batch batch, int32_t* bad_plane);
/* Completion stamps for nuasm_batch_plane_times (enabled = 1, the default)
 * or none (0): each stamp is one small launch on its graph branch after the
 * launch that completes its planes (in the grouped form one stamp serves
 * every plane a grouped launch completes), plus one at the start.  A change
 * drops the recorded graphs. */
nuasm_status nuasm_batch_set_plane_times(nuasm_batch batch, int32_t enabled);
/* Synchronise; ms[p] = device wall-clock time from the start of the last
 * recorded-graph launch (run, set_points_many or execute_many) to the
 * completion of plane p (caller-owned host array of P floats).  A plane with
 * no launch (no points, type 2 with nothing to do) completes at 0.
 * NUASM_ERR_NOT_READY when stamps are off or no recorded graph has run since
 * the graphs were last dropped. */
nuasm_status nuasm_batch_plane_times(nuasm_batch batch, float* ms);
/* How often a batch has recorded a graph, and how often it has only
 * rewritten a grouped graph's argument tables for new buffers (see
 * nuasm_batch_run), since it was created.  For testing. */
nuasm_status nuasm_debug_batch_graphs(nuasm_batch batch, int64_t* recorded, int64_t* refreshed);

const char* nuasm_status_string(nuasm_status s);
const char* nuasm_last_error(void);

/* Testing aid: make the k-th device or pinned-host allocation the library
 * attempts from now on fail as if memory had run out (NUASM_ERR_ALLOC from
 * the call that needed it), then allocate normally again; k = 0 turns it off.
 * The environment variable NUASM_FAIL_ALLOC=k does the same when the library
 * is first used.  Every failing call leaves its plan or batch destroyable
 * (and a plan whose set_points failed usable after a later successful one). */
nuasm_status nuasm_debug_fail_alloc(int64_t k);

/* Testing aid: the bytes of device memory and of pinned host memory the
 * library holds at this moment (every plan, batch and per-device table), so
 * that a test can check that a call sequence gave back all it allocated. */
nuasm_status nuasm_debug_live_bytes(int64_t* device_bytes, int64_t* host_bytes);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int32_t nuasm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NUASM_H */
