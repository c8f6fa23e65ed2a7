// Host side of libnuasm: parameter validation, plan tables, workspace, and
// the C-ABI entry points declared in include/nuasm.h.  Every step of the
// operators runs in the gfx950 kernels of k_fft.hip and k_points.hip; the
// host only derives sizes and constants, builds the small float64 plan tables
// and enqueues launches on the plan's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "group.h"
#include "launch.h"
#include "nuasm.h"

using namespace nuasm;

namespace {

thread_local std::string g_last_error;

nuasm_status fail(nuasm_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

nuasm_status hip_fail(hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return fail(NUASM_ERR_ALLOC, m);
  return fail(NUASM_ERR_HIP, m);
}

#define HIP_TRY(expr, what)                     \
  do {                                          \
    hipError_t e_ = (expr);                     \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

constexpr double kPi = 3.14159265358979323846264338327950288;

// ------------------------------------------------ allocation-failure injection
// Testing aid: with NUASM_FAIL_ALLOC=k in the environment (or after
// nuasm_debug_fail_alloc(k)), the k-th device or pinned-host allocation the
// library attempts from then on fails as if memory had run out (1-based; 0 or
// unset: never).  Every allocation of the library goes through dev_malloc /
// host_malloc.
std::atomic<int64_t> g_fail_at{-1};  // allocations left before the failing one; < 0: off
std::once_flag g_fail_env_once;

void read_fail_env() {
  std::call_once(g_fail_env_once, [] {
    const char* v = std::getenv("NUASM_FAIL_ALLOC");
    if (v && *v) {
      const long long k = std::atoll(v);
      if (k > 0) g_fail_at.store(k - 1);
    }
  });
}

bool inject_alloc_failure() {
  read_fail_env();
  int64_t left = g_fail_at.load();
  while (left >= 0) {
    if (g_fail_at.compare_exchange_weak(left, left - 1)) return left == 0;
  }
  return false;
}

// Every live allocation of the library with its size (device and pinned
// host apart), so that a test can check that what a call sequence allocated
// was all given back (nuasm_debug_live_bytes).  Frees go through dev_free /
// host_free.
std::mutex g_live_mutex;
std::unordered_map<void*, size_t> g_live[2];  // 0: device, 1: pinned host
int64_t g_live_bytes[2] = {0, 0};

void live_add(int kind, void* p, size_t bytes) {
  std::lock_guard<std::mutex> lk(g_live_mutex);
  g_live[kind][p] = bytes;
  g_live_bytes[kind] += (int64_t)bytes;
}

void live_remove(int kind, void* p) {
  std::lock_guard<std::mutex> lk(g_live_mutex);
  auto it = g_live[kind].find(p);
  if (it == g_live[kind].end()) return;
  g_live_bytes[kind] -= (int64_t)it->second;
  g_live[kind].erase(it);
}

hipError_t dev_malloc(void** p, size_t bytes) {
  if (inject_alloc_failure()) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  const hipError_t e = hipMalloc(p, bytes);
  if (e == hipSuccess) live_add(0, *p, bytes);
  return e;
}

hipError_t host_malloc(void** p, size_t bytes) {
  if (inject_alloc_failure()) {
    *p = nullptr;
    return hipErrorOutOfMemory;
  }
  const hipError_t e = hipHostMalloc(p, bytes, hipHostMallocDefault);
  if (e == hipSuccess) live_add(1, *p, bytes);
  return e;
}

hipError_t dev_free(void* p) {
  if (!p) return hipSuccess;
  live_remove(0, p);
  return hipFree(p);
}

hipError_t host_free(void* p) {
  if (!p) return hipSuccess;
  live_remove(1, p);
  return hipHostFree(p);
}

// ------------------------------------------------------- twiddle tables
// One table per device: for n = 2^l, tw[n + m] = exp(-2 pi i m / n).
std::mutex g_tw_mutex;
float2* g_tw[64] = {nullptr};

nuasm_status twiddles_for_device(int dev, const float2** out) {
  std::lock_guard<std::mutex> lk(g_tw_mutex);
  if (dev < 0 || dev >= 64) return fail(NUASM_ERR_UNSUPPORTED, "device ordinal >= 64");
  if (!g_tw[dev]) {
    const int total = 2 << kMaxLogN;
    std::vector<float2> h(total);
    h[0] = make_float2(0.f, 0.f);
    h[1] = make_float2(0.f, 0.f);
    for (int l = 1; l <= kMaxLogN; ++l) {
      const int n = 1 << l;
      for (int m = 0; m < n; ++m) {
        const double a = -2.0 * kPi * (double)m / (double)n;
        h[n + m] = make_float2((float)std::cos(a), (float)std::sin(a));
      }
    }
    float2* d = nullptr;
    HIP_TRY(dev_malloc((void**)&d, sizeof(float2) * total), "hipMalloc(twiddles)");
    hipError_t e = hipMemcpy(d, h.data(), sizeof(float2) * total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)dev_free(d);
      return hip_fail(e, "hipMemcpy(twiddles)");
    }
    g_tw[dev] = d;
  }
  *out = g_tw[dev];
  return NUASM_OK;
}

// ------------------------------------------------------ kernel transform
// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// 1 / psihat(k) for k in K, where psihat(k) = int psi(d) exp(-2 pi i k d / nf) dd
// over |d| <= w/2 (psi even, so a cosine transform), by Gauss-Legendre.
std::vector<float> deconvolution_table(int Np, int nf, int w, double beta) {
  std::vector<double> gx, gw;
  gauss_legendre(64, gx, gw);
  const double half = 0.5 * w;
  std::vector<float> out(Np);
  for (int a = 0; a < Np; ++a) {
    const int k = a - Np / 2;
    double s = 0.0;
    for (size_t i = 0; i < gx.size(); ++i) {
      const double d = 0.5 * (gx[i] + 1.0) * half;  // [0, w/2]
      const double t = d / half;
      const double psi = std::exp(beta * (std::sqrt(std::max(0.0, 1.0 - t * t)) - 1.0));
      s += gw[i] * 0.5 * half * psi * std::cos(2.0 * kPi * k * d / nf);
    }
    out[a] = (float)(1.0 / (2.0 * s));
  }
  return out;
}

// --------------------------------------------------------------- Eq. 4 band
// Per axis, frequencies whose transfer-function phase has local spatial
// frequency within the window: |o - z f / sqrt(1/l^2 - f^2)| <= S, S = N g.
// Inverting u = z f / s(f): f = sign(z) u / (l sqrt(z^2 + u^2)).
void band_axis(double lam, double z, double o, double S, double df, int Np, int* lo, int* hi) {
  const int kmin = -Np / 2, kmax = Np / 2 - 1;
  if (z == 0.0) {
    if (std::fabs(o) <= S) {
      *lo = kmin;
      *hi = kmax;
    } else {
      *lo = 1;
      *hi = 0;
    }
    return;
  }
  auto gam = [&](double t) { return t / (lam * std::sqrt(z * z + t * t)); };
  double flo, fhi;
  if (z > 0.0) {
    flo = gam(o - S);
    fhi = gam(o + S);
  } else {
    flo = -gam(o + S);
    fhi = -gam(o - S);
  }
  const double klo = std::ceil(flo / df), khi = std::floor(fhi / df);
  *lo = (int)std::max<double>(klo, kmin);
  *hi = (int)std::min<double>(khi, kmax);
}

}  // namespace

// ------------------------------------------------------------------- plan
// One bound point set: its records in bin order, the counting-sort state and
// the chunk tables of the spreading and interpolation kernels.
struct PointSet {
  int* counts = nullptr;     // records per bin
  int* cursor = nullptr;     // first record of each bin
  uint16_t* hist = nullptr;  // [G][T] per-range bin counts
  int* hoff = nullptr;       // [G][T] per-range offsets inside each bin
  int64_t hist_rows = 0;
  int* sp_first = nullptr;
  int* sp_n = nullptr;
  int* multi = nullptr;
  int* bin_pre = nullptr;    // [T][kBinPre] bin-scan prefixes
  int* wg_sum = nullptr;     // [column-scan workgroups][kBinPre] their sums
  int* nch = nullptr;  // [8]: chunk and record counts [0..3], points out of range [4], split-bin slots [5]
  int4* sp_chunks = nullptr;
  int4* ip_chunks = nullptr;
  int64_t chunk_cap = 0;
  BinRec* recs = nullptr;
  int64_t rec_cap = 0;  // points the record buffer is sized for
  float2* scratch = nullptr;  // partial tiles of split bins
  int64_t scratch_chunks = 0;  // tiles it holds
  size_t scratch_bytes = 0;
  int* host_stat = nullptr;  // pinned [8]
  int64_t M = 0;
  bool ready = false;
  bool synced = false;
  int exact_sp = 0, exact_ip = 0, exact_multi = 0, exact_slots = 0;
  // a uniform grid bound with nuasm_set_grid_points (no records, no binning)
  bool grid = false;
  GridPts gp{};
  float2* gbuf = nullptr;  // separable passes' intermediate rows
  int64_t gbuf_cap = 0;
};

struct nuasm_plan_s {
  nuasm_params p{};
  hipStream_t stream = nullptr;
  hipEvent_t handoff = nullptr;  // orders a new stream after the previous one
  int device = 0;
  int logNp = 0;
  int logNpf = 0;  // spectral grid N'' (the fine grid is 2 N'')
  int w = 0;
  float beta = 0.f;
  GridGeom geom{};
  BinGeom bgeom{};
  Spectral spec{};
  int T = 0, TX = 0;
  int tile = kTile;          // bin side in fine cells (32 or 64)
  int tile_log = 5;
  const float2* tw = nullptr;
  // device memory
  float2* gridA = nullptr;
  float2* gridB = nullptr;
  float* dinv = nullptr;     // 1/psihat(k), k in K'' (N'' entries)
  float* dinv_np = nullptr;  // the same at column k + N'/2 of an N'-wide row (zero outside K''),
                             // for the type-2 row pass; == dinv when N'' = N'
  float2* fre = nullptr;  // [2][Np]
  // point sets: [0] the plan's points (type 3: the source), [1] type 3's destination
  PointSet ps[2];
  // tuning (nuasm_plan_set_tuning): chunk sizes and binning ranges
  bool sp_small = false;  // spreading chunks of about half the default size
  int sp_chunk = kSpreadChunk;
  int ip_chunk = kChunk;
  int bin_ppw = 0;        // points per binning workgroup, 0 = automatic
  int sp_method = 0;      // spreading: 0 automatic, 1 register gather, 2 matrix cores
  int nsets = 1;
  size_t bytes = 0;          // device memory the plan allocated itself
  // caller-owned workspace (nuasm_plan_set_workspace): the two grids and the
  // point-count-dependent buffers of every point set are carved from it
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int64_t ws_cap = 0;        // points per set the workspace holds
  // set only during nuasm_execute_noalloc: the device's static partial-tile
  // array replaces the point sets' own scratch
  float2* scratch_override = nullptr;
  // stage timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_stage;          // stage of each recorded (start, end) pair
  std::vector<hipEvent_t> ev_pairs;   // start0, end0, start1, end1, ...
  int64_t grid_elems = 0;
  bool ready() const {
    for (int i = 0; i < nsets; ++i)
      if (!ps[i].ready) return false;
    return true;
  }
};

namespace {

template <typename T>
hipError_t dalloc(nuasm_plan_s* pl, T** p, size_t n) {
  hipError_t e = dev_malloc((void**)p, sizeof(T) * std::max<size_t>(n, 1));
  if (e == hipSuccess) pl->bytes += sizeof(T) * std::max<size_t>(n, 1);
  return e;
}

void release(nuasm_plan_s* pl) {
  auto f = [](void* p) {
    if (p) (void)dev_free(p);
  };
  // buffers carved from a caller's workspace are not the plan's to free
  auto fo = [&](void* p) {
    if (!pl->ws) f(p);
  };
  fo(pl->gridA);
  fo(pl->gridB);
  if (pl->dinv_np != pl->dinv) f(pl->dinv_np);
  f(pl->dinv);
  f(pl->fre);
  for (PointSet& q : pl->ps) {
    f(q.counts);
    f(q.cursor);
    f(q.sp_first);
    f(q.sp_n);
    f(q.multi);
    f(q.bin_pre);
    f(q.wg_sum);
    f(q.nch);
    fo(q.sp_chunks);
    fo(q.ip_chunks);
    fo(q.recs);
    fo(q.scratch);
    fo(q.hist);
    fo(q.hoff);
    f(q.gbuf);
    if (q.host_stat) (void)host_free(q.host_stat);
    q = PointSet{};
  }
  if (pl->handoff) (void)hipEventDestroy(pl->handoff);
  pl->handoff = nullptr;
  for (hipEvent_t e : pl->ev_pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : pl->ev_pairs) (void)hipEventDestroy(e);
  pl->ev_pool.clear();
  pl->ev_pairs.clear();
}

hipEvent_t take_event(nuasm_plan_s* pl) {
  if (!pl->ev_pool.empty()) {
    hipEvent_t e = pl->ev_pool.back();
    pl->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets the launches of one stage with events when timing is on.
struct StageScope {
  nuasm_plan_s* pl;
  int stage;
  hipEvent_t start = nullptr;
  StageScope(nuasm_plan_s* p, int s) : pl(p), stage(s) {
    // a batch collecting launches for grouped execution: tag them, time nothing
    if (LaunchRecorder* r = active_recorder()) {
      r->stage = s;
      return;
    }
    if (!pl->timing) return;
    start = take_event(pl);
    if (start) (void)hipEventRecord(start, pl->stream);
  }
  ~StageScope() {
    if (!start) return;
    hipEvent_t end = take_event(pl);
    if (!end) {
      pl->ev_pool.push_back(start);
      return;
    }
    (void)hipEventRecord(end, pl->stream);
    pl->ev_pairs.push_back(start);
    pl->ev_pairs.push_back(end);
    pl->ev_stage.push_back(stage);
  }
};

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// Deterministic mode: stable binning scatter and stable ranks in spreading.
bool stable_bins(const nuasm_plan_s* pl) { return (pl->p.flags & NUASM_DETERMINISTIC) != 0; }

// Pitch of the plan's grid: the uniform plane's (d2 for type 1, d1 for type
// 2); type 3 takes the destination's, d2.
double plane_pitch(const nuasm_params* p) { return p->type == NUASM_TYPE_2 ? p->d1 : p->d2; }

nuasm_status validate(const nuasm_params* p) {
  if (!p) return fail(NUASM_ERR_INVALID_ARG, "params is NULL");
  if (p->type != NUASM_TYPE_1 && p->type != NUASM_TYPE_2 && p->type != NUASM_TYPE_3)
    return fail(NUASM_ERR_INVALID_ARG, "type must be 1, 2 or 3");
  if (p->tf != NUASM_TF_ASM && p->tf != NUASM_TF_FRESNEL) return fail(NUASM_ERR_INVALID_ARG, "tf must be ASM or FRESNEL");
  if (p->band < NUASM_BAND_FULL || p->band > NUASM_BAND_EXPLICIT) return fail(NUASM_ERR_INVALID_ARG, "bad band mode");
  if (p->phase_fp64 != 0 && p->phase_fp64 != 1) return fail(NUASM_ERR_INVALID_ARG, "phase_fp64 must be 0 or 1");
  if (!is_pow2(p->N) || p->N < 16 || p->N > 4096)
    return fail(NUASM_ERR_UNSUPPORTED, "N must be a power of two in [16, 4096]");
  if (!(p->lambda > 0.0) || !std::isfinite(p->lambda)) return fail(NUASM_ERR_INVALID_ARG, "lambda must be > 0");
  if (!std::isfinite(p->z)) return fail(NUASM_ERR_INVALID_ARG, "z must be finite");
  if (!std::isfinite(p->ox) || !std::isfinite(p->oy)) return fail(NUASM_ERR_INVALID_ARG, "offset must be finite");
  const double g = plane_pitch(p);
  if (!(g > 0.0) || !std::isfinite(g)) return fail(NUASM_ERR_INVALID_ARG, "pitch of the uniform plane must be > 0");
  if (p->type == NUASM_TYPE_3 && (p->flags & NUASM_OUT_CROP_N))
    return fail(NUASM_ERR_INVALID_ARG, "NUASM_OUT_CROP_N applies to type 1 only");
  if (p->tf == NUASM_TF_FRESNEL && p->z == 0.0) return fail(NUASM_ERR_INVALID_ARG, "Fresnel needs z != 0");
  if (!(p->tol >= 1e-12 && p->tol <= 1e-2)) return fail(NUASM_ERR_INVALID_ARG, "tol must be in [1e-12, 1e-2]");
  if (p->flags &
      ~(NUASM_OUT_CROP_N | NUASM_DEFER_RANGE_CHECK | NUASM_FULL_FINE_GRID | NUASM_DETERMINISTIC | NUASM_FORWARD_ONLY))
    return fail(NUASM_ERR_INVALID_ARG, "unknown flag bits");
  if ((p->flags & NUASM_FORWARD_ONLY) && p->type != NUASM_TYPE_2)
    return fail(NUASM_ERR_INVALID_ARG, "NUASM_FORWARD_ONLY applies to type 2 only");
  if (p->reserved != 0) return fail(NUASM_ERR_INVALID_ARG, "reserved must be 0");
  if (p->band == NUASM_BAND_EXPLICIT) {
    for (int i = 0; i < 2; ++i)
      if (!std::isfinite(p->band_c[i]) || !(p->band_w[i] >= 0.0))
        return fail(NUASM_ERR_INVALID_ARG, "explicit band needs finite centre and width >= 0");
  }
  return NUASM_OK;
}

// Binning workgroups: contiguous ranges of ppw points (automatic: at least
// 4096, at most kBinPointsMax, and about 256 ranges for large M; or the
// tuned count; at most kBinPointsStable in deterministic mode).
void bin_ranges(int64_t M, int fixed, bool stable, int* ppw, int* G) {
  int64_t p = fixed > 0 ? fixed : std::max<int64_t>(4096, (M + 255) / 256);
  p = std::min<int64_t>(p, stable ? kBinPointsStable : kBinPointsMax);
  *ppw = (int)p;
  *G = (int)((M + p - 1) / p);
}

// T-sized bin arrays and counters of one point set (at plan creation).
nuasm_status alloc_point_set(nuasm_plan_s* pl, PointSet& q) {
  HIP_TRY(dalloc(pl, &q.counts, (size_t)pl->T + 1), "hipMalloc(bins)");
  HIP_TRY(dalloc(pl, &q.cursor, (size_t)pl->T), "hipMalloc(bins)");
  HIP_TRY(dalloc(pl, &q.sp_first, (size_t)pl->T), "hipMalloc(bins)");
  HIP_TRY(dalloc(pl, &q.sp_n, (size_t)pl->T), "hipMalloc(bins)");
  HIP_TRY(dalloc(pl, &q.multi, (size_t)pl->T), "hipMalloc(bins)");
  HIP_TRY(dalloc(pl, &q.bin_pre, (size_t)pl->T * kBinPre), "hipMalloc(bins)");
  HIP_TRY(dalloc(pl, &q.wg_sum, (size_t)bin_scan_workgroups(pl->T) * kBinPre), "hipMalloc(bins)");
  HIP_TRY(dalloc(pl, &q.nch, (size_t)8), "hipMalloc(counters)");
  HIP_TRY(host_malloc((void**)&q.host_stat, sizeof(int) * 8), "hipHostMalloc(status)");
  HIP_TRY(launch_fill_i32(q.nch, 0, 8, pl->stream), "launch fill");
  return NUASM_OK;
}

// Sizes of the point-count-dependent buffers of one point set sized for `cap`
// points (each rounded up to 256 bytes): records (at most 4 per point), the
// two chunk tables, the per-range histograms and offsets, and the partial
// tiles of split bins (the bound of scratch_tiles_needed).
size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

struct PointLayout {
  int64_t cap = 0, chunk_cap = 0, hist_rows = 0, tiles = 0;
  size_t recs = 0, chunks = 0, hist = 0, hoff = 0, scratch = 0;
  size_t total() const { return recs + 2 * chunks + hist + hoff + scratch; }
};

PointLayout point_layout(const nuasm_plan_s* pl, int64_t cap) {
  PointLayout L;
  L.cap = std::max<int64_t>(cap, 1024);
  int ppw = 0, G = 0;
  bin_ranges(L.cap, pl->bin_ppw, stable_bins(pl), &ppw, &G);
  L.hist_rows = std::max(G, 1);
  L.chunk_cap = pl->T + (4 * L.cap) / std::min(pl->sp_chunk, pl->ip_chunk) + 1;  // covers both chunk tables
  L.tiles = std::max<int64_t>(1, std::min<int64_t>(L.chunk_cap, (8 * L.cap) / pl->sp_chunk + 1));
  L.recs = round256(sizeof(BinRec) * 4 * (size_t)L.cap);
  L.chunks = round256(sizeof(int4) * (size_t)L.chunk_cap);
  L.hist = round256(sizeof(uint16_t) * (size_t)L.hist_rows * (pl->T + 1));
  L.hoff = round256(sizeof(int) * (size_t)L.hist_rows * (pl->T + 1));
  L.scratch = round256(sizeof(float2) * (size_t)pl->tile * pl->tile * (size_t)L.tiles);
  return L;
}

size_t grid_bytes(const nuasm_plan_s* pl) { return round256(sizeof(float2) * (size_t)pl->grid_elems); }

size_t workspace_bytes_for(const nuasm_plan_s* pl, int64_t cap) {
  return 2 * grid_bytes(pl) + (size_t)pl->nsets * point_layout(pl, cap).total();
}

// Point the grids and every point set's buffers into the caller's workspace
// (sized for pl->ws_cap points per set).
void carve_workspace(nuasm_plan_s* pl) {
  char* p = pl->ws;
  const size_t gb = grid_bytes(pl);
  pl->gridA = (float2*)p;
  pl->gridB = (float2*)(p + gb);
  p += 2 * gb;
  const PointLayout L = point_layout(pl, pl->ws_cap);
  for (int i = 0; i < pl->nsets; ++i) {
    PointSet& q = pl->ps[i];
    q.recs = (BinRec*)p;
    p += L.recs;
    q.sp_chunks = (int4*)p;
    p += L.chunks;
    q.ip_chunks = (int4*)p;
    p += L.chunks;
    q.hist = (uint16_t*)p;
    p += L.hist;
    q.hoff = (int*)p;
    p += L.hoff;
    q.scratch = (float2*)p;
    q.scratch_bytes = L.scratch;
    p += L.scratch;
    q.rec_cap = L.cap;
    q.chunk_cap = L.chunk_cap;
    q.hist_rows = L.hist_rows;
    q.scratch_chunks = L.tiles;
  }
}

// Free the plan-owned grids and point buffers (not a caller's workspace).
void free_owned_buffers(nuasm_plan_s* pl) {
  auto f = [&](void* p, size_t b) {
    if (p && !pl->ws) {
      (void)dev_free(p);
      pl->bytes -= b;
    }
  };
  f(pl->gridA, sizeof(float2) * pl->grid_elems);
  f(pl->gridB, sizeof(float2) * pl->grid_elems);
  pl->gridA = pl->gridB = nullptr;
  for (int i = 0; i < pl->nsets; ++i) {
    PointSet& q = pl->ps[i];
    f(q.recs, sizeof(BinRec) * 4 * q.rec_cap);
    f(q.sp_chunks, sizeof(int4) * q.chunk_cap);
    f(q.ip_chunks, sizeof(int4) * q.chunk_cap);
    f(q.hist, sizeof(uint16_t) * q.hist_rows * (pl->T + 1));
    f(q.hoff, sizeof(int) * q.hist_rows * (pl->T + 1));
    f(q.scratch, q.scratch_bytes);
    q.recs = nullptr;
    q.sp_chunks = q.ip_chunks = nullptr;
    q.hist = nullptr;
    q.hoff = nullptr;
    q.scratch = nullptr;
    q.rec_cap = q.chunk_cap = q.hist_rows = q.scratch_chunks = 0;
    q.scratch_bytes = 0;
    if (!q.grid) q.ready = false;
  }
}

// Bind the caller's workspace `dev` of `bytes` bytes (NULL: go back to
// plan-owned memory).  The capacity is the largest point count per set whose
// buffers fit; binned point sets must be bound again.
nuasm_status bind_workspace(nuasm_plan_s* pl, void* dev, size_t bytes) {
  if (dev && ((uintptr_t)dev & 255)) return fail(NUASM_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (!dev && !pl->ws) return NUASM_OK;  // already plan-owned
  int64_t cap = 0;
  if (dev) {
    const size_t need = workspace_bytes_for(pl, 1024);
    if (bytes < need) {
      char buf[160];
      std::snprintf(buf, sizeof(buf), "workspace of %zu bytes is below this plan's minimum of %zu bytes", bytes,
                    need);
      return fail(NUASM_ERR_INVALID_ARG, buf);
    }
    int64_t lo = 1024, hi = (int64_t)INT32_MAX / 4;  // 4 records per point must fit in int32
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo + 1) / 2;
      if (workspace_bytes_for(pl, mid) <= bytes) lo = mid;
      else hi = mid - 1;
    }
    cap = lo;
  }
  HIP_TRY(hipStreamSynchronize(pl->stream), "hipStreamSynchronize");
  free_owned_buffers(pl);
  pl->ws = (char*)dev;
  pl->ws_bytes = dev ? bytes : 0;
  pl->ws_cap = cap;
  if (dev) {
    carve_workspace(pl);
    return NUASM_OK;
  }
  HIP_TRY(dalloc(pl, &pl->gridA, (size_t)pl->grid_elems), "hipMalloc(gridA)");
  HIP_TRY(dalloc(pl, &pl->gridB, (size_t)pl->grid_elems), "hipMalloc(gridB)");
  return NUASM_OK;
}

// Free the T-sized bin arrays of a point set (before the bin tile changes).
void free_bin_arrays(nuasm_plan_s* pl, PointSet& q) {
  const size_t T = (size_t)pl->T;
  auto f = [&](void* p, size_t b) {
    if (p) {
      (void)dev_free(p);
      pl->bytes -= b;
    }
  };
  f(q.counts, sizeof(int) * (T + 1));
  f(q.cursor, sizeof(int) * T);
  f(q.sp_first, sizeof(int) * T);
  f(q.sp_n, sizeof(int) * T);
  f(q.multi, sizeof(int) * T);
  f(q.bin_pre, sizeof(int) * T * kBinPre);
  f(q.wg_sum, sizeof(int) * (size_t)bin_scan_workgroups(pl->T) * kBinPre);
  f(q.nch, sizeof(int) * 8);
  q.counts = q.cursor = q.sp_first = q.sp_n = q.multi = q.bin_pre = q.wg_sum = q.nch = nullptr;
  if (q.host_stat) (void)host_free(q.host_stat);
  q.host_stat = nullptr;
}

// The bin side and everything that follows from it (bins per axis, the
// binning geometry).
void set_tile(nuasm_plan_s* pl, int tile) {
  pl->tile = tile;
  pl->tile_log = tile == 64 ? 6 : 5;
  pl->TX = (pl->geom.L + tile - 1) / tile;
  pl->T = pl->TX * pl->TX;
  pl->bgeom.TX = pl->TX;
  pl->bgeom.tile_log = pl->tile_log;
}

nuasm_status ensure_points_capacity(nuasm_plan_s* pl, PointSet& q, int64_t M) {
  if (pl->ws) {
    if (M <= q.rec_cap) return NUASM_OK;
    char buf[160];
    std::snprintf(buf, sizeof(buf), "%lld points exceed the workspace's capacity of %lld points per set",
                  (long long)M, (long long)q.rec_cap);
    return fail(NUASM_ERR_INVALID_ARG, buf);
  }
  if (M <= q.rec_cap && q.recs) return NUASM_OK;
  const int64_t cap = std::max<int64_t>(M, 1024);
  if (cap * 4 > (int64_t)INT32_MAX) return fail(NUASM_ERR_UNSUPPORTED, "too many points (4 M must fit in int32)");
  HIP_TRY(hipStreamSynchronize(pl->stream), "hipStreamSynchronize");
  if (q.recs) {
    (void)dev_free(q.recs);
    pl->bytes -= sizeof(BinRec) * 4 * q.rec_cap;
    q.recs = nullptr;
  }

  if (q.sp_chunks) {
    (void)dev_free(q.sp_chunks);
    (void)dev_free(q.ip_chunks);
    pl->bytes -= 2 * sizeof(int4) * q.chunk_cap;
    q.sp_chunks = q.ip_chunks = nullptr;
  }
  if (q.scratch) {
    (void)dev_free(q.scratch);
    pl->bytes -= q.scratch_bytes;
    q.scratch = nullptr;
    q.scratch_chunks = 0;
    q.scratch_bytes = 0;
  }
  if (q.hist) {
    (void)dev_free(q.hist);
    (void)dev_free(q.hoff);
    pl->bytes -= (sizeof(uint16_t) + sizeof(int)) * q.hist_rows * (pl->T + 1);
    q.hist = nullptr;
    q.hoff = nullptr;
  }
  q.rec_cap = 0;
  {
    int ppw = 0, G = 0;
    bin_ranges(cap, pl->bin_ppw, stable_bins(pl), &ppw, &G);
    q.hist_rows = std::max(G, 1);
    HIP_TRY(dalloc(pl, &q.hist, (size_t)q.hist_rows * (pl->T + 1)), "hipMalloc(bin histograms)");
    HIP_TRY(dalloc(pl, &q.hoff, (size_t)q.hist_rows * (pl->T + 1)), "hipMalloc(bin offsets)");
  }
  HIP_TRY(dalloc(pl, &q.recs, (size_t)(4 * cap)), "hipMalloc(records)");
  q.chunk_cap = pl->T + (4 * cap) / std::min(pl->sp_chunk, pl->ip_chunk) + 1;  // covers both chunk tables
  HIP_TRY(dalloc(pl, &q.sp_chunks, (size_t)q.chunk_cap), "hipMalloc(chunks)");
  HIP_TRY(dalloc(pl, &q.ip_chunks, (size_t)q.chunk_cap), "hipMalloc(chunks)");
  q.rec_cap = cap;
  return NUASM_OK;
}

// Partial tiles the split bins of a bound set may need: the exact count once
// a set_points has synchronised, else a bound.  A split bin holds c > chunk
// records in ceil(c / chunk) < 2 c / chunk chunks, and there are at most 4 M
// records, so fewer than 8 M / chunk slots are ever used.
int64_t scratch_tiles_needed(const nuasm_plan_s* pl, const PointSet& q) {
  if (q.synced) return q.exact_slots;
  return std::min<int64_t>(q.chunk_cap, (8 * q.M) / pl->sp_chunk + 1);
}

nuasm_status ensure_scratch(nuasm_plan_s* pl, PointSet& q) {
  const int64_t need = std::max<int64_t>(scratch_tiles_needed(pl, q), 1);
  if (q.scratch && need <= q.scratch_chunks) return NUASM_OK;
  // a workspace holds the bound for its capacity, which covers every M <= it
  if (pl->ws) return fail(NUASM_ERR_INVALID_ARG, "split-bin scratch exceeds the workspace");
  if (q.scratch) {
    HIP_TRY(hipStreamSynchronize(pl->stream), "hipStreamSynchronize");
    (void)dev_free(q.scratch);
    pl->bytes -= q.scratch_bytes;
    q.scratch = nullptr;
    q.scratch_chunks = 0;
    q.scratch_bytes = 0;
  }
  HIP_TRY(dalloc(pl, &q.scratch, (size_t)need * pl->tile * pl->tile), "hipMalloc(spread scratch)");
  q.scratch_chunks = need;
  q.scratch_bytes = sizeof(float2) * (size_t)need * pl->tile * pl->tile;
  return NUASM_OK;
}

// The point-set status read back from the device: points outside the
// window (nch[4]).
nuasm_status point_status(const PointSet& q, int which) {
  if (q.host_stat[4] != 0) {
    char buf[160];
    std::snprintf(buf, sizeof(buf), "%d point(s) outside the window [-N g/2, N g/2]^2 or not finite%s",
                  q.host_stat[4], which == 1 ? " (destination points)" : "");
    return fail(NUASM_ERR_OUT_OF_RANGE, buf);
  }
  return NUASM_OK;
}

// Grid sizes of the point kernels: the exact chunk counts once a set_points
// has synchronised, else upper bounds (surplus workgroups exit at once).
int sp_grid(const nuasm_plan_s* pl, const PointSet& q) {
  return q.synced ? q.exact_sp : (int)std::min<int64_t>(q.chunk_cap, pl->T + (4 * q.M) / pl->sp_chunk + 1);
}
int ip_grid(const nuasm_plan_s* pl, const PointSet& q) {
  return q.synced ? q.exact_ip : (int)std::min<int64_t>(q.chunk_cap, pl->T + (4 * q.M) / pl->ip_chunk + 1);
}
int multi_grid(const nuasm_plan_s* pl, const PointSet& q) {
  return q.synced ? q.exact_multi : (int)std::min<int64_t>(pl->T, (4 * q.M) / pl->sp_chunk + 1);
}

// The rejected points' indices are stored downwards from the end of the
// record buffer (capacity four records per point; the records of the
// accepted points, at most four each, never reach them).
int* rej_end(const PointSet& q) { return reinterpret_cast<int*>(q.recs + 4 * q.rec_cap); }

// Coordinate normalisation and binning of one point set (three launches).
nuasm_status bind_points(nuasm_plan_s* pl, PointSet& q, int64_t M, const double* x, const double* y) {
  if (M < 0) return fail(NUASM_ERR_INVALID_ARG, "M < 0");
  if (M > 0 && (!x || !y)) return fail(NUASM_ERR_INVALID_ARG, "coordinate pointer is NULL");
  q.ready = false;
  q.grid = false;
  nuasm_status s = ensure_points_capacity(pl, q, M);
  if (s != NUASM_OK) return s;
  hipStream_t st = pl->stream;
  {
    int ppw = 0, G = 0;
    bin_ranges(M, pl->bin_ppw, stable_bins(pl), &ppw, &G);
    if (M > 0) {
      StageScope sc(pl, NUASM_STAGE_BIN_HIST);
      HIP_TRY(launch_bin_hist(x, y, M, pl->bgeom, ppw, G, q.hist, st), "launch bin_hist");
    }
    {
      // column scan, then bin scan; with no points (G = 0) they write zero
      // totals and empty-bin chunk tables
      const BinScanOut so{q.cursor, q.sp_chunks, q.sp_first, q.sp_n, q.multi, q.ip_chunks, q.nch,
                          q.bin_pre, q.wg_sum, pl->sp_chunk, pl->ip_chunk};
      {
        StageScope sc(pl, NUASM_STAGE_BIN_COLSCAN);
        HIP_TRY(launch_bin_colscan(q.hist, M > 0 ? G : 0, pl->T, q.hoff, q.counts, so, st), "launch bin_colscan");
      }
      StageScope sc(pl, NUASM_STAGE_BIN_SCAN);
      HIP_TRY(launch_bin_scan(pl->T, q.counts, so, st), "launch bin_scan");
    }
    StageScope sc(pl, NUASM_STAGE_BIN_SCATTER);
    HIP_TRY(launch_bin_scatter(x, y, M, pl->bgeom, ppw, G, q.hoff, q.cursor, q.recs, rej_end(q), stable_bins(pl),
                               st),
            "launch bin_scatter");
  }
  q.M = M;
  q.synced = false;
  if (pl->p.flags & NUASM_DEFER_RANGE_CHECK) {
    q.ready = true;
    return NUASM_OK;
  }
  HIP_TRY(hipMemcpyAsync(q.host_stat, q.nch, sizeof(int) * 6, hipMemcpyDeviceToHost, st), "hipMemcpyAsync");
  HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
  {
    const nuasm_status ps = point_status(q, &q == &pl->ps[1] ? 1 : 0);
    if (ps != NUASM_OK) return ps;
  }
  q.exact_sp = q.host_stat[0];
  q.exact_ip = q.host_stat[1];
  q.exact_multi = q.host_stat[3];
  q.exact_slots = q.host_stat[5];
  q.synced = true;
  q.ready = true;
  return NUASM_OK;
}

// Bind a uniform nx x ny grid of the given pitch centred at (cx, cy) as a
// point set: no device work, the separable kernels derive every tap from the
// grid index.  Host-side range check of the grid's extreme points.
nuasm_status bind_grid(nuasm_plan_s* pl, PointSet& q, int64_t nx, int64_t ny, double pitch, double cx,
                       double cy) {
  if (nx < 0 || ny < 0) return fail(NUASM_ERR_INVALID_ARG, "grid sizes must be >= 0");
  if (!(pitch > 0.0) || !std::isfinite(pitch) || !std::isfinite(cx) || !std::isfinite(cy))
    return fail(NUASM_ERR_INVALID_ARG, "grid pitch must be > 0 and the centre finite");
  if (nx > (1 << 18) || ny > (1 << 18) || nx * ny > ((int64_t)1 << 30))
    return fail(NUASM_ERR_UNSUPPORTED, "grid larger than 2^18 per side or 2^30 points");
  q.ready = false;
  const double g = plane_pitch(&pl->p);
  const double half = 0.5 * (double)pl->geom.N + 1e-9;  // pixels, with the binning's rounding slack
  if (nx > 0 && ny > 0) {
    const double xs[2] = {cx + (double)(0 - nx / 2) * pitch, cx + (double)(nx - 1 - nx / 2) * pitch};
    const double ys[2] = {cy + (double)(0 - ny / 2) * pitch, cy + (double)(ny - 1 - ny / 2) * pitch};
    for (int i = 0; i < 2; ++i)
      if (!(std::fabs(xs[i] / g) <= half) || !(std::fabs(ys[i] / g) <= half))
        return fail(NUASM_ERR_OUT_OF_RANGE, "grid extends outside the window [-N g/2, N g/2]^2");
  }
  GridPts& p = q.gp;
  p.nx = (int)nx;
  p.ny = (int)ny;
  p.pitch = pitch;
  p.cx = cx;
  p.cy = cy;
  p.inv_g = pl->bgeom.inv_g;
  p.half_n = pl->bgeom.half_n;
  p.tau0 = pl->bgeom.tau0;
  p.L = pl->geom.L;
  p.two_over_w = 2.0f / (float)pl->w;
  p.beta_log2e = pl->beta * 1.4426950408889634f;
  // support rows the interpolation's taps reach, two rows of margin against
  // the rounding of the host's and the device's tap positions
  p.ty0 = 0;
  p.nrows = 0;
  if (nx > 0 && ny > 0) {
    auto tap = [&](int64_t k) {
      const double t = 2.0 * ((cy + (double)(k - ny / 2) * pitch) * p.inv_g) + p.tau0;
      return (int)std::ceil(t - 0.5 * pl->w);
    };
    const int lo = std::max(0, tap(0) - 2);
    const int hi = std::min(p.L, tap(ny - 1) + pl->w + 2);
    p.ty0 = lo;
    p.nrows = std::max(0, hi - lo);
  }
  const int64_t need = std::max<int64_t>((int64_t)p.nrows * nx, ny * (int64_t)p.L);
  if (need > q.gbuf_cap) {
    HIP_TRY(hipStreamSynchronize(pl->stream), "hipStreamSynchronize");
    if (q.gbuf) {
      (void)dev_free(q.gbuf);
      pl->bytes -= sizeof(float2) * q.gbuf_cap;
      q.gbuf = nullptr;
      q.gbuf_cap = 0;
    }
    HIP_TRY(dalloc(pl, &q.gbuf, (size_t)need), "hipMalloc(grid passes)");
    q.gbuf_cap = need;
  }
  q.grid = true;
  q.M = nx * ny;
  q.synced = true;
  q.ready = true;
  return NUASM_OK;
}

// Spreading of one point set's values onto the fine support (gridA).
nuasm_status run_spread(nuasm_plan_s* pl, PointSet& q, const float2* vals) {
  hipStream_t st = pl->stream;
  if (q.grid) {
    StageScope sc(pl, NUASM_STAGE_SPREAD);
    HIP_TRY(launch_grid_spread(pl->w, vals, q.gbuf, pl->gridA, q.gp, st), "launch grid_spread");
    return NUASM_OK;
  }
  float2* scratch = pl->scratch_override;
  if (!scratch) {
    nuasm_status s = ensure_scratch(pl, q);
    if (s != NUASM_OK) return s;
    scratch = q.scratch;
  }
  {
    StageScope sc(pl, NUASM_STAGE_SPREAD);
    SpreadArgs sa{};
    sa.recs = q.recs;
    sa.stable = stable_bins(pl) ? 1 : 0;
    sa.chunks = q.sp_chunks;
    sa.nchunks = q.nch + 0;
    sa.scratch = scratch;
    sa.vals = vals;
    sa.grid = pl->gridA;
    sa.L = pl->geom.L;
    sa.TX = pl->TX;
    sa.two_over_w = 2.0f / (float)pl->w;
    sa.beta = pl->beta;
    if (pl->sp_method == 1)
      HIP_TRY(launch_spread(pl->w, pl->sp_small, sa, sp_grid(pl, q), st), "launch spread");
    else
      HIP_TRY(launch_spread_mfma(pl->w, pl->tile, sa, sp_grid(pl, q), st), "launch spread_mfma");
  }
  {
    StageScope sc(pl, NUASM_STAGE_SPREAD_REDUCE);
    SpreadReduceArgs ra{};
    ra.chunks = q.sp_chunks;
    ra.multi = q.multi;
    ra.nmulti = q.nch + 3;
    ra.bin_chunk0 = q.sp_first;
    ra.bin_nchunk = q.sp_n;
    ra.scratch = scratch;
    ra.grid = pl->gridA;
    ra.L = pl->geom.L;
    ra.TX = pl->TX;
    ra.tile_log = pl->tile_log;
    const int parts = (pl->tile / 16) * (pl->tile / 16);  // 256 cells per workgroup
    HIP_TRY(launch_spread_reduce(ra, multi_grid(pl, q) * parts, st), "launch spread_reduce");
  }
  return NUASM_OK;
}

// Interpolation of the fine support `grid` at one point set's points.
nuasm_status run_interp(nuasm_plan_s* pl, PointSet& q, const float2* grid, float2* out) {
  if (q.M == 0) return NUASM_OK;
  StageScope sc(pl, NUASM_STAGE_INTERP);
  if (q.grid) {
    HIP_TRY(launch_grid_interp(pl->w, grid, q.gbuf, out, q.gp, pl->stream), "launch grid_interp");
    return NUASM_OK;
  }
  InterpArgs ia{};
  ia.recs = q.recs;
  ia.chunks = q.ip_chunks;
  ia.nchunks = q.nch + 1;
  ia.grid = grid;
  ia.out = out;
  // a deferred range check may have left points without records; the kernel
  // writes NaN at their outputs (a synchronised set_points refuses such
  // points, so their count is then 0)
  ia.rej_end = rej_end(q);
  ia.nrej = q.nch + 4;
  ia.L = pl->geom.L;
  ia.TX = pl->TX;
  ia.two_over_w = 2.0f / (float)pl->w;
  ia.beta = pl->beta;
  HIP_TRY(launch_interp(pl->w, pl->tile, ia, ip_grid(pl, q), pl->stream), "launch interp");
  return NUASM_OK;
}

// type-1 pipeline: values at the points -> N' x N' (or N x N) plane
nuasm_status run_type1_pipeline(nuasm_plan_s* pl, PointSet& q, const float2* vals, float2* out, bool conj,
                                bool crop) {
  hipStream_t st = pl->stream;
  nuasm_status s = run_spread(pl, q, vals);
  if (s != NUASM_OK) return s;
  GridGeom g = pl->geom;
  g.crop = crop ? 1 : 0;
  Spectral sp = pl->spec;
  sp.conj = conj ? 1 : 0;
  {
    StageScope sc(pl, NUASM_STAGE_T1_ROWS);
    HIP_TRY(launch_t1_rows(pl->logNpf, pl->gridA, pl->gridB, g, pl->dinv, pl->tw, st), "launch t1_rows");
  }
  {
    StageScope sc(pl, NUASM_STAGE_T1_COLS);
    HIP_TRY(launch_t1_cols(pl->logNpf, pl->logNp, pl->gridB, pl->gridA, g, sp, pl->tw, st), "launch t1_cols");
  }
  {
    StageScope sc(pl, NUASM_STAGE_T1_ROWS_INV);
    HIP_TRY(launch_t1_rows_inv(pl->logNp, pl->gridA, out, g, pl->tw, st), "launch t1_rows_inv");
  }
  return NUASM_OK;
}

// type-2 pipeline: Nin x Nin plane -> values at the points
nuasm_status run_type2_pipeline(nuasm_plan_s* pl, PointSet& q, const float2* plane, int Nin, float2* out,
                                bool conj) {
  hipStream_t st = pl->stream;
  GridGeom g = pl->geom;
  g.Nin = Nin;
  g.crop = 0;
  Spectral sp = pl->spec;
  sp.conj = conj ? 1 : 0;
  {
    StageScope sc(pl, NUASM_STAGE_T2_ROWS);
    HIP_TRY(launch_t2_rows(pl->logNp, plane, pl->gridB, g, pl->dinv_np, pl->tw, st), "launch t2_rows");
  }
  {
    StageScope sc(pl, NUASM_STAGE_T2_COLS);
    HIP_TRY(launch_t2_cols(pl->logNpf, pl->logNp, pl->gridB, pl->gridA, g, sp, pl->tw, st), "launch t2_cols");
  }
  {
    StageScope sc(pl, NUASM_STAGE_T2_ROWS_INV);
    HIP_TRY(launch_t2_rows_inv(pl->logNpf, pl->gridA, pl->gridB, g, pl->tw, st), "launch t2_rows_inv");
  }
  return run_interp(pl, q, pl->gridB, out);
}

// type-3 pipeline: values at the points of `src` -> values at the points of
// `dst`: spreading, the type-1 row pass, the fused type-3 column pass, the
// type-2 inverse row pass, interpolation.
nuasm_status run_type3_pipeline(nuasm_plan_s* pl, PointSet& src, PointSet& dst, const float2* vals,
                                float2* out, bool conj) {
  if (dst.M == 0) return NUASM_OK;
  hipStream_t st = pl->stream;
  nuasm_status s = run_spread(pl, src, vals);
  if (s != NUASM_OK) return s;
  GridGeom g = pl->geom;
  g.crop = 0;
  Spectral sp = pl->spec;
  sp.conj = conj ? 1 : 0;
  {
    StageScope sc(pl, NUASM_STAGE_T1_ROWS);
    HIP_TRY(launch_t1_rows(pl->logNpf, pl->gridA, pl->gridB, g, pl->dinv, pl->tw, st), "launch t1_rows");
  }
  {
    StageScope sc(pl, NUASM_STAGE_T3_COLS);
    HIP_TRY(launch_t3_cols(pl->logNpf, pl->gridB, pl->gridA, g, sp, pl->tw, st), "launch t3_cols");
  }
  {
    StageScope sc(pl, NUASM_STAGE_T2_ROWS_INV);
    HIP_TRY(launch_t2_rows_inv(pl->logNpf, pl->gridA, pl->gridB, g, pl->tw, st), "launch t2_rows_inv");
  }
  return run_interp(pl, dst, pl->gridB, out);
}

}  // namespace

// ================================================================== C ABI
extern "C" {

int32_t nuasm_version(void) { return 10100; }

const char* nuasm_status_string(nuasm_status s) {
  switch (s) {
    case NUASM_OK: return "NUASM_OK";
    case NUASM_ERR_INVALID_ARG: return "NUASM_ERR_INVALID_ARG";
    case NUASM_ERR_OUT_OF_RANGE: return "NUASM_ERR_OUT_OF_RANGE";
    case NUASM_ERR_NOT_READY: return "NUASM_ERR_NOT_READY";
    case NUASM_ERR_UNSUPPORTED: return "NUASM_ERR_UNSUPPORTED";
    case NUASM_ERR_NO_DEVICE: return "NUASM_ERR_NO_DEVICE";
    case NUASM_ERR_ALLOC: return "NUASM_ERR_ALLOC";
    case NUASM_ERR_HIP: return "NUASM_ERR_HIP";
    default: break;
  }
  return "NUASM_UNKNOWN_STATUS";
}

const char* nuasm_last_error(void) { return g_last_error.c_str(); }

nuasm_status nuasm_debug_live_bytes(int64_t* device_bytes, int64_t* host_bytes) {
  if (!device_bytes || !host_bytes) return fail(NUASM_ERR_INVALID_ARG, "output pointer is NULL");
  std::lock_guard<std::mutex> lk(g_live_mutex);
  *device_bytes = g_live_bytes[0];
  *host_bytes = g_live_bytes[1];
  return NUASM_OK;
}

nuasm_status nuasm_debug_fail_alloc(int64_t k) {
  if (k < 0) return fail(NUASM_ERR_INVALID_ARG, "k must be >= 0");
  read_fail_env();  // the environment first, so that this call wins
  g_fail_at.store(k > 0 ? k - 1 : -1);
  return NUASM_OK;
}

nuasm_status nuasm_params_default(nuasm_params* p) {
  if (!p) return fail(NUASM_ERR_INVALID_ARG, "params is NULL");
  std::memset(p, 0, sizeof(*p));
  p->type = NUASM_TYPE_1;
  p->tf = NUASM_TF_ASM;
  p->band = NUASM_BAND_FULL;
  p->phase_fp64 = 1;
  p->N = 1024;
  p->lambda = 633e-9;
  p->z = 0.01;
  p->d1 = p->d2 = 4e-6;
  p->tol = 1e-6;
  return NUASM_OK;
}

nuasm_status nuasm_plan_create(const nuasm_params* p, void* hip_stream, nuasm_plan* out) {
  if (!out) return fail(NUASM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  nuasm_status s = validate(p);
  if (s != NUASM_OK) return s;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return fail(NUASM_ERR_NO_DEVICE, "no HIP device visible");
  }
  nuasm_plan_s* pl = new (std::nothrow) nuasm_plan_s();
  if (!pl) return fail(NUASM_ERR_ALLOC, "host allocation failed");
  pl->p = *p;
  pl->stream = (hipStream_t)hip_stream;
  auto bail = [&](nuasm_status st) {
    release(pl);
    delete pl;
    return st;
  };
  if (hipGetDevice(&pl->device) != hipSuccess) return bail(fail(NUASM_ERR_HIP, "hipGetDevice failed"));
  const int N = (int)p->N, Np = 2 * N;
  int logNp = 0;
  while ((1 << logNp) < Np) ++logNp;
  pl->logNp = logNp;
  const double g = plane_pitch(p);
  const double df = 1.0 / (Np * g);
  // kernel width from the tolerance: w = ceil(log10(1/tol)) + 1, beta = 2.30 w
  int w = (int)std::ceil(-std::log10(p->tol) - 1e-9) + 1;
  w = std::max(2, std::min(kMaxW, w));
  pl->w = w;
  pl->beta = (float)(2.30 * w);
  GridGeom& G = pl->geom;
  G.N = N;
  G.Np = Np;
  G.Nin = N;
  G.crop = (p->flags & NUASM_OUT_CROP_N) ? 1 : 0;
  const int kmin = -Np / 2, kmax = Np / 2 - 1;
  G.kxlo = G.kylo = kmin;
  G.kxhi = G.kyhi = kmax;
  if (p->tf == NUASM_TF_ASM && p->band == NUASM_BAND_LIMITED) {
    band_axis(p->lambda, p->z, p->ox, N * g, df, Np, &G.kxlo, &G.kxhi);
    band_axis(p->lambda, p->z, p->oy, N * g, df, Np, &G.kylo, &G.kyhi);
  } else if (p->tf == NUASM_TF_ASM && p->band == NUASM_BAND_EXPLICIT) {
    int b[4];
    for (int i = 0; i < 2; ++i) {
      b[2 * i] = (int)std::max<double>(std::ceil(p->band_c[i] - 0.5 * p->band_w[i]), kmin);
      b[2 * i + 1] = (int)std::min<double>(std::floor(p->band_c[i] + 0.5 * p->band_w[i]), kmax);
    }
    G.kxlo = b[0];
    G.kxhi = b[1];
    G.kylo = b[2];
    G.kyhi = b[3];
  }

  // Spectral grid N'': the smallest power of two (>= 32, >= N'/8) whose index
  // set K'' = [-N''/2, N''/2) holds the band of Eq. 4 on both axes; N' for a
  // full band, for Fresnel, or with NUASM_FULL_FINE_GRID.  The non-uniform
  // sums keep their accuracy on the smaller fine grid 2 N'' (same
  // oversampling, same kernel) because no mode outside the band is needed;
  // the fine cells become N'/N'' times wider.
  {
    int need = 0;
    if (G.kxlo <= G.kxhi && G.kylo <= G.kyhi)
      need = 2 * std::max(std::max(-G.kxlo, G.kxhi + 1), std::max(-G.kylo, G.kyhi + 1));
    int lpf = 5;
    while ((1 << lpf) < need) ++lpf;
    lpf = std::max(lpf, logNp - 3);
    if (lpf > logNp || (p->flags & NUASM_FULL_FINE_GRID)) lpf = logNp;
    pl->logNpf = lpf;
  }
  const int Npf = 1 << pl->logNpf, nf = 2 * Npf;
  const int L = Npf + 2 * kPad;
  pl->TX = (L + pl->tile - 1) / pl->tile;
  pl->T = pl->TX * pl->TX;
  G.Npf = Npf;
  G.nf = nf;
  G.L = L;
  G.s0 = Npf / 2 - kPad;

  // the non-uniform plane in fine-cell units: N'' / 2 cells of N'/N'' pixels
  // across the window, pixel 0 of that coarser raster at support cell N''/2 + 8
  BinGeom& B = pl->bgeom;
  B.N = Npf / 2;
  B.inv_g = (double)Npf / ((double)Np * g);
  B.half_n = 0.25 * Npf;
  B.tau0 = (double)(Npf / 2 + kPad);
  B.w = w;
  B.L = L;
  B.TX = pl->TX;
  B.tile_log = pl->tile_log;
  B.primary_only = (p->flags & NUASM_FORWARD_ONLY) ? 1 : 0;

  Spectral& S = pl->spec;
  S.tf = p->tf == NUASM_TF_FRESNEL ? 1 : 0;
  S.phase_fp64 = p->phase_fp64;
  S.conj = 0;
  S.scale = (float)(1.0 / ((double)Np * (double)Np));
  {
    const double zl = p->z / p->lambda;
    S.c0 = zl - std::nearbyint(zl);
    S.ax = df * p->ox;
    S.ay = df * p->oy;
    S.zl = zl;
    S.ql2 = (p->lambda * df) * (p->lambda * df);
    S.axf = (float)S.ax;
    S.ayf = (float)S.ay;
    S.qf = (float)(df * df);
    S.zf = (float)p->z;
    S.inv_lam2f = (float)(1.0 / (p->lambda * p->lambda));
  }

  s = twiddles_for_device(pl->device, &pl->tw);
  if (s != NUASM_OK) return bail(s);
  // the fine support, and the N' x N' intermediates of the column passes
  pl->grid_elems = std::max<int64_t>((int64_t)L * L, (int64_t)Np * Np);
  hipError_t e;
  if ((e = dalloc(pl, &pl->gridA, (size_t)pl->grid_elems)) != hipSuccess) return bail(hip_fail(e, "hipMalloc(gridA)"));
  if ((e = dalloc(pl, &pl->gridB, (size_t)pl->grid_elems)) != hipSuccess) return bail(hip_fail(e, "hipMalloc(gridB)"));
  if ((e = dalloc(pl, &pl->dinv, (size_t)Npf)) != hipSuccess) return bail(hip_fail(e, "hipMalloc(dinv)"));
  pl->dinv_np = pl->dinv;
  if (Npf != Np && (e = dalloc(pl, &pl->dinv_np, (size_t)Np)) != hipSuccess)
    return bail(hip_fail(e, "hipMalloc(dinv)"));
  pl->nsets = p->type == NUASM_TYPE_3 ? 2 : 1;
  for (int i = 0; i < pl->nsets; ++i) {
    s = alloc_point_set(pl, pl->ps[i]);
    if (s != NUASM_OK) return bail(s);
  }
  {
    std::vector<float> dv = deconvolution_table(Npf, nf, w, (double)pl->beta);
    if ((e = hipMemcpyAsync(pl->dinv, dv.data(), sizeof(float) * Npf, hipMemcpyHostToDevice, pl->stream)) != hipSuccess)
      return bail(hip_fail(e, "hipMemcpy(dinv)"));
    std::vector<float> dn;
    if (Npf != Np) {
      dn.assign(Np, 0.f);
      for (int a = 0; a < Npf; ++a) dn[a - Npf / 2 + Np / 2] = dv[a];
      if ((e = hipMemcpyAsync(pl->dinv_np, dn.data(), sizeof(float) * Np, hipMemcpyHostToDevice, pl->stream)) !=
          hipSuccess)
        return bail(hip_fail(e, "hipMemcpy(dinv)"));
    }
    if ((e = hipStreamSynchronize(pl->stream)) != hipSuccess) return bail(hip_fail(e, "hipStreamSynchronize"));
  }
  S.dinv = pl->dinv;
  if (S.tf == 1) {
    if ((e = dalloc(pl, &pl->fre, (size_t)2 * Np)) != hipSuccess) return bail(hip_fail(e, "hipMalloc(fresnel)"));
    // A = g^2 exp(2 pi i z/l) / (i l z), folded into the x table
    const double cyc = S.c0;
    const double mag = g * g / (p->lambda * p->z);
    const double cr = std::cos(2.0 * kPi * cyc), ci = std::sin(2.0 * kPi * cyc);
    const double2 A = make_double2(mag * ci, -mag * cr);  // (cr + i ci) * mag / i
    const double2 one = make_double2(1.0, 0.0);
    const double two_lam_z = 2.0 * p->lambda * p->z;
    if ((e = launch_fresnel_axis(Np, g, two_lam_z, p->ox, A, pl->fre, pl->stream)) != hipSuccess)
      return bail(hip_fail(e, "launch fresnel_axis"));
    if ((e = launch_fresnel_axis(Np, g, two_lam_z, p->oy, one, pl->fre + Np, pl->stream)) != hipSuccess)
      return bail(hip_fail(e, "launch fresnel_axis"));
    S.fre_x = pl->fre;
    S.fre_y = pl->fre + Np;
  }
  *out = pl;
  return NUASM_OK;
}

nuasm_status nuasm_plan_destroy(nuasm_plan pl) {
  if (!pl) return NUASM_OK;
  (void)hipStreamSynchronize(pl->stream);
  release(pl);
  delete pl;
  return NUASM_OK;
}

nuasm_status nuasm_plan_set_stream(nuasm_plan pl, void* hip_stream) {
  if (!pl) return fail(NUASM_ERR_INVALID_ARG, "plan is NULL");
  const hipStream_t ns = (hipStream_t)hip_stream;
  if (ns == pl->stream) return NUASM_OK;
  // what the plan enqueued on the old stream (its tables, a binning) must
  // finish before the new stream's work reads it
  if (!pl->handoff) HIP_TRY(hipEventCreateWithFlags(&pl->handoff, hipEventDisableTiming), "hipEventCreate");
  HIP_TRY(hipEventRecord(pl->handoff, pl->stream), "hipEventRecord");
  HIP_TRY(hipStreamWaitEvent(ns, pl->handoff, 0), "hipStreamWaitEvent");
  pl->stream = ns;
  return NUASM_OK;
}

nuasm_status nuasm_plan_get_info(nuasm_plan pl, nuasm_plan_info* info) {
  if (!pl || !info) return fail(NUASM_ERR_INVALID_ARG, "plan or info is NULL");
  std::memset(info, 0, sizeof(*info));
  info->N = pl->geom.N;
  info->Np = pl->geom.Np;
  info->nf = pl->geom.nf;
  info->L = pl->geom.L;
  info->w = pl->w;
  info->beta = pl->beta;
  info->tile = pl->tile;
  info->tiles = pl->T;
  info->kx_lo = pl->geom.kxlo;
  info->kx_hi = pl->geom.kxhi;
  info->ky_lo = pl->geom.kylo;
  info->ky_hi = pl->geom.kyhi;
  const int64_t plane = pl->geom.crop ? (int64_t)pl->geom.N * pl->geom.N : (int64_t)pl->geom.Np * pl->geom.Np;
  const int64_t M = pl->ps[0].M, M2 = pl->nsets > 1 ? pl->ps[1].M : 0;
  if (pl->p.type == NUASM_TYPE_1) {
    info->in_elems = M;
    info->out_elems = plane;
  } else if (pl->p.type == NUASM_TYPE_2) {
    info->in_elems = (int64_t)pl->geom.N * pl->geom.N;
    info->out_elems = M;
  } else {
    info->in_elems = M;
    info->out_elems = M2;
  }
  info->M = M;
  info->device_bytes = pl->bytes;
  info->M_dest = M2;
  info->Npf = pl->geom.Npf;
  info->spread_chunk = pl->sp_chunk;
  info->interp_chunk = pl->ip_chunk;
  {
    int ppw = 0, G = 0;
    bin_ranges(M, pl->bin_ppw, stable_bins(pl), &ppw, &G);
    info->bin_range_points = ppw;
  }
  return NUASM_OK;
}

nuasm_status nuasm_plan_set_tuning(nuasm_plan pl, const nuasm_tuning* t) {
  if (!pl || !t) return fail(NUASM_ERR_INVALID_ARG, "plan or tuning is NULL");
  if (t->spread_chunk < 0 || t->interp_chunk < 0 || t->bin_range_points < 0)
    return fail(NUASM_ERR_INVALID_ARG, "tuning fields must be >= 0");
  if (t->spread_method < 0 || t->spread_method > 2)
    return fail(NUASM_ERR_INVALID_ARG, "spread_method must be 0 (automatic), 1 (register gather) or 2 (matrix cores)");
  if (t->bin_tile != 0 && t->bin_tile != 32 && t->bin_tile != 64)
    return fail(NUASM_ERR_INVALID_ARG, "bin_tile must be 0 (32), 32 or 64");
  const int new_tile = t->bin_tile == 0 ? kTile : t->bin_tile;
  if (new_tile != kTile && t->spread_method == 1)
    return fail(NUASM_ERR_INVALID_ARG, "the register-gather spreading takes 32 x 32 bins only");
  if (t->interp_chunk != 0 && (t->interp_chunk < 256 || t->interp_chunk > 65536))
    return fail(NUASM_ERR_INVALID_ARG, "interp_chunk must be 0 or in [256, 65536]");
  if (t->bin_range_points != 0 && (t->bin_range_points < 1024 || t->bin_range_points > kBinPointsMax))
    return fail(NUASM_ERR_INVALID_ARG, "bin_range_points must be 0 or in [1024, 65535]");
  // spreading chunks come in the two sizes the kernels are built for; a
  // request below the default takes the small one
  const int small = spread_nsub(pl->w, true) * spread_subbatch(pl->w);
  struct Sizes {
    bool sp_small;
    int sp_chunk, ip_chunk, bin_ppw, sp_method, tile;
  };
  const Sizes old{pl->sp_small, pl->sp_chunk, pl->ip_chunk, pl->bin_ppw, pl->sp_method, pl->tile};
  Sizes nw;
  nw.sp_small = t->spread_chunk != 0 && t->spread_chunk < kSpreadChunk;
  nw.sp_chunk = nw.sp_small ? small : kSpreadChunk;
  nw.ip_chunk = t->interp_chunk != 0 ? t->interp_chunk : kChunk;
  nw.bin_ppw = t->bin_range_points;
  nw.sp_method = t->spread_method;
  nw.tile = new_tile;
  auto apply = [&](const Sizes& z) {
    pl->sp_small = z.sp_small;
    pl->sp_chunk = z.sp_chunk;
    pl->ip_chunk = z.ip_chunk;
    pl->bin_ppw = z.bin_ppw;
    pl->sp_method = z.sp_method;
    set_tile(pl, z.tile);
  };
  // a caller's workspace must hold the new sizes' minimum; else nothing changes
  if (pl->ws) {
    apply(nw);
    const size_t need = workspace_bytes_for(pl, 1024);
    apply(old);
    if (need > pl->ws_bytes) {
      char buf[200];
      std::snprintf(buf, sizeof(buf), "the workspace (%zu bytes) is below this tuning's minimum of %zu bytes",
                    pl->ws_bytes, need);
      return fail(NUASM_ERR_INVALID_ARG, buf);
    }
  }
  if (new_tile != old.tile) {
    // new bins: the T-sized arrays of every set are allocated again
    HIP_TRY(hipStreamSynchronize(pl->stream), "hipStreamSynchronize");
    for (int i = 0; i < pl->nsets; ++i) free_bin_arrays(pl, pl->ps[i]);
    apply(nw);
    for (int i = 0; i < pl->nsets; ++i) {
      const nuasm_status s = alloc_point_set(pl, pl->ps[i]);
      if (s != NUASM_OK) return s;
    }
  }
  apply(nw);
  // binned point sets must be bound again (their chunk tables and histogram
  // rows follow the old sizes); a set bound as a grid stays ready, but its
  // buffers are resized too at its next binning.  A caller's workspace is
  // carved again for the new sizes.
  if (pl->ws) return bind_workspace(pl, pl->ws, pl->ws_bytes);
  for (int i = 0; i < pl->nsets; ++i) {
    PointSet& q = pl->ps[i];
    q.rec_cap = 0;
    if (!q.grid) q.ready = false;
  }
  return NUASM_OK;
}

nuasm_status nuasm_plan_workspace_bytes(nuasm_plan pl, int64_t M_max, size_t* bytes) {
  if (!pl || !bytes) return fail(NUASM_ERR_INVALID_ARG, "plan or bytes is NULL");
  if (M_max < 0 || M_max > (int64_t)INT32_MAX / 4) return fail(NUASM_ERR_INVALID_ARG, "M_max must be in [0, 2^29)");
  *bytes = workspace_bytes_for(pl, M_max);
  return NUASM_OK;
}

nuasm_status nuasm_plan_set_workspace(nuasm_plan pl, void* dev, size_t bytes) {
  if (!pl) return fail(NUASM_ERR_INVALID_ARG, "plan is NULL");
  return bind_workspace(pl, dev, bytes);
}

nuasm_status nuasm_set_points(nuasm_plan pl, int64_t M, const double* x, const double* y) {
  if (!pl) return fail(NUASM_ERR_INVALID_ARG, "plan is NULL");
  return bind_points(pl, pl->ps[0], M, x, y);
}

nuasm_status nuasm_set_dest_points(nuasm_plan pl, int64_t M, const double* x, const double* y) {
  if (!pl) return fail(NUASM_ERR_INVALID_ARG, "plan is NULL");
  if (pl->p.type != NUASM_TYPE_3) return fail(NUASM_ERR_INVALID_ARG, "destination points belong to type-3 plans");
  return bind_points(pl, pl->ps[1], M, x, y);
}

nuasm_status nuasm_set_grid_points(nuasm_plan pl, int32_t which, int64_t nx, int64_t ny, double pitch, double cx,
                                   double cy) {
  if (!pl) return fail(NUASM_ERR_INVALID_ARG, "plan is NULL");
  if (which < 0 || which >= pl->nsets)
    return fail(NUASM_ERR_INVALID_ARG, "which must be 0 (or 1 for a type-3 plan's destination)");
  return bind_grid(pl, pl->ps[which], nx, ny, pitch, cx, cy);
}

nuasm_status nuasm_check_points(nuasm_plan pl) {
  if (!pl) return fail(NUASM_ERR_INVALID_ARG, "plan is NULL");
  for (int i = 0; i < pl->nsets; ++i) {
    PointSet& q = pl->ps[i];
    if (q.grid) continue;  // range-checked on the host when bound
    HIP_TRY(hipMemcpyAsync(q.host_stat, q.nch, sizeof(int) * 6, hipMemcpyDeviceToHost, pl->stream),
            "hipMemcpyAsync");
  }
  HIP_TRY(hipStreamSynchronize(pl->stream), "hipStreamSynchronize");
  for (int i = 0; i < pl->nsets; ++i) {
    PointSet& q = pl->ps[i];
    if (q.grid) continue;
    const nuasm_status ps = point_status(q, i);
    if (ps != NUASM_OK) {
      q.ready = false;
      return ps;
    }
  }
  return NUASM_OK;
}

namespace {
const char* not_ready_msg(const nuasm_plan_s* pl) {
  return pl->nsets > 1 ? "execute before successful set_points and set_dest_points"
                       : "execute before a successful set_points";
}
}  // namespace

nuasm_status nuasm_execute(nuasm_plan pl, const void* in, void* out) {
  if (!pl) return fail(NUASM_ERR_INVALID_ARG, "plan is NULL");
  if (!pl->ready()) return fail(NUASM_ERR_NOT_READY, not_ready_msg(pl));
  PointSet& q = pl->ps[0];
  if (pl->p.type == NUASM_TYPE_3) {
    PointSet& d = pl->ps[1];
    if ((!in && q.M > 0) || (!out && d.M > 0)) return fail(NUASM_ERR_INVALID_ARG, "in/out pointer is NULL");
    return run_type3_pipeline(pl, q, d, (const float2*)in, (float2*)out, false);
  }
  // the point-side array may be NULL only when there are no points
  const bool t1 = pl->p.type == NUASM_TYPE_1;
  const void* pts = t1 ? in : out;
  const void* plane = t1 ? out : in;
  if (!plane || (!pts && q.M > 0)) return fail(NUASM_ERR_INVALID_ARG, "in/out pointer is NULL");
  if (t1) return run_type1_pipeline(pl, q, (const float2*)in, (float2*)out, false, pl->geom.crop != 0);
  if (q.M == 0) return NUASM_OK;
  return run_type2_pipeline(pl, q, (const float2*)in, pl->geom.N, (float2*)out, false);
}

nuasm_status nuasm_execute_adjoint(nuasm_plan pl, const void* in, void* out) {
  if (!pl) return fail(NUASM_ERR_INVALID_ARG, "plan is NULL");
  if (!pl->ready()) return fail(NUASM_ERR_NOT_READY, not_ready_msg(pl));
  PointSet& q = pl->ps[0];
  if (pl->p.type == NUASM_TYPE_3) {
    PointSet& d = pl->ps[1];
    if ((!in && d.M > 0) || (!out && q.M > 0)) return fail(NUASM_ERR_INVALID_ARG, "in/out pointer is NULL");
    return run_type3_pipeline(pl, d, q, (const float2*)in, (float2*)out, true);
  }
  if (pl->p.flags & NUASM_FORWARD_ONLY)
    return fail(NUASM_ERR_UNSUPPORTED, "the plan was created NUASM_FORWARD_ONLY: its bins hold no records for spreading");
  const bool t1 = pl->p.type == NUASM_TYPE_1;
  const void* pts = t1 ? out : in;
  const void* plane = t1 ? in : out;
  if (!plane || (!pts && q.M > 0)) return fail(NUASM_ERR_INVALID_ARG, "in/out pointer is NULL");
  if (t1) {
    if (pl->geom.crop) return fail(NUASM_ERR_UNSUPPORTED, "adjoint of a cropped type-1 plan");
    if (q.M == 0) return NUASM_OK;
    return run_type2_pipeline(pl, q, (const float2*)in, pl->geom.Np, (float2*)out, true);
  }
  return run_type1_pipeline(pl, q, (const float2*)in, (float2*)out, true, true);
}

}  // extern "C"

// ------------------------------------------------ allocation-free execute
// Partial tiles of split bins for nuasm_execute_noalloc: one array per device
// in the library's code object, kStaticTiles tiles of 32 x 32 complex64
// (16 MiB), held until the process ends.  Host code never passes `scratch`
// itself to a kernel (on the host it is only a stand-in for the symbol): the
// device address comes from hipGetSymbolAddress, once per device.
constexpr int64_t kStaticTiles = 2048;
static __device__ __align__(256) float2 scratch[kStaticTiles * kTile * kTile];

namespace {
std::mutex g_static_mutex;
float2* g_static_ptr[64] = {nullptr};

// Device address of `scratch` on device `dev` (taken once, with that device
// current; the caller's current device is restored).
nuasm_status static_scratch_for_device(int dev, float2** out) {
  std::lock_guard<std::mutex> lk(g_static_mutex);
  if (dev < 0 || dev >= 64) return fail(NUASM_ERR_UNSUPPORTED, "device ordinal >= 64");
  if (!g_static_ptr[dev]) {
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur), "hipGetDevice");
    if (cur != dev) HIP_TRY(hipSetDevice(dev), "hipSetDevice");
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(NUASM_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_static_ptr[dev] = (float2*)ptr;
  }
  *out = g_static_ptr[dev];
  return NUASM_OK;
}
}  // namespace

extern "C" {

nuasm_status nuasm_execute_noalloc(nuasm_plan pl, const void* in, void* out) {
  if (!pl) return fail(NUASM_ERR_INVALID_ARG, "plan is NULL");
  if (!pl->ready()) return fail(NUASM_ERR_NOT_READY, not_ready_msg(pl));
  // the point set that is spread: the plan's points (type 1, and type 3's
  // sources); type 2 spreads nothing
  const PointSet& q = pl->ps[0];
  if (pl->p.type != NUASM_TYPE_2 && !q.grid) {
    // partial tiles of the plan's bin side, counted in 32 x 32 units
    const int64_t need = scratch_tiles_needed(pl, q) * (pl->tile / kTile) * (pl->tile / kTile);
    if (need > kStaticTiles) {
      char buf[256];
      std::snprintf(buf, sizeof(buf),
                    "split bins may need %lld partial 32 x 32 tiles, above the static scratch's %lld (bind the "
                    "points without NUASM_DEFER_RANGE_CHECK so that the exact count is known, or use nuasm_execute)",
                    (long long)need, (long long)kStaticTiles);
      return fail(NUASM_ERR_UNSUPPORTED, buf);
    }
  }
  float2* ptr = nullptr;
  nuasm_status s = static_scratch_for_device(pl->device, &ptr);
  if (s != NUASM_OK) return s;
  // no stage events either (creating one may allocate)
  const bool timing = pl->timing;
  pl->timing = false;
  pl->scratch_override = ptr;
  s = nuasm_execute(pl, in, out);
  pl->scratch_override = nullptr;
  pl->timing = timing;
  return s;
}

nuasm_status nuasm_plan_set_timing(nuasm_plan pl, int32_t enable) {
  if (!pl) return fail(NUASM_ERR_INVALID_ARG, "plan is NULL");
  pl->timing = enable != 0;
  return NUASM_OK;
}

nuasm_status nuasm_plan_read_timing(nuasm_plan pl, double* ms, int64_t* launches) {
  if (!pl || !ms || !launches) return fail(NUASM_ERR_INVALID_ARG, "NULL argument");
  if (!pl->ev_pairs.empty()) HIP_TRY(hipEventSynchronize(pl->ev_pairs.back()), "hipEventSynchronize");
  for (size_t i = 0; i < pl->ev_stage.size(); ++i) {
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, pl->ev_pairs[2 * i], pl->ev_pairs[2 * i + 1]), "hipEventElapsedTime");
    const int s = pl->ev_stage[i];
    ms[s] += t;
    launches[s] += 1;
  }
  for (hipEvent_t e : pl->ev_pairs) pl->ev_pool.push_back(e);
  pl->ev_pairs.clear();
  pl->ev_stage.clear();
  return NUASM_OK;
}

nuasm_status nuasm_debug_transfer(nuasm_plan pl, void* out) {
  if (!pl || !out) return fail(NUASM_ERR_INVALID_ARG, "plan or out is NULL");
  HIP_TRY(launch_transfer_table(pl->geom, pl->spec, (float2*)out, pl->stream), "launch transfer_table");
  return NUASM_OK;
}

nuasm_status nuasm_debug_records(nuasm_plan pl, int32_t which, void* recs_out, int64_t rec_cap, int32_t* counts_out,
                                 int64_t* n_records) {
  if (!pl || !recs_out || !counts_out || !n_records) return fail(NUASM_ERR_INVALID_ARG, "NULL argument");
  if (which < 0 || which >= pl->nsets) return fail(NUASM_ERR_INVALID_ARG, "which must be 0 (or 1 for type 3)");
  PointSet& q = pl->ps[which];
  if (!q.ready || q.grid) return fail(NUASM_ERR_NOT_READY, "the point set holds no binned points");
  HIP_TRY(hipMemcpyAsync(q.host_stat, q.nch, sizeof(int) * 6, hipMemcpyDeviceToHost, pl->stream), "hipMemcpyAsync");
  HIP_TRY(hipStreamSynchronize(pl->stream), "hipStreamSynchronize");
  const int64_t total = q.host_stat[2];
  *n_records = total;
  if (rec_cap < total) return fail(NUASM_ERR_INVALID_ARG, "rec_cap is below the number of records");
  if (total > 0)
    HIP_TRY(hipMemcpyAsync(recs_out, q.recs, sizeof(BinRec) * total, hipMemcpyDeviceToDevice, pl->stream),
            "hipMemcpyAsync");
  HIP_TRY(hipMemcpyAsync(counts_out, q.counts, sizeof(int) * pl->T, hipMemcpyDeviceToDevice, pl->stream),
          "hipMemcpyAsync");
  HIP_TRY(hipStreamSynchronize(pl->stream), "hipStreamSynchronize");
  return NUASM_OK;
}

nuasm_status nuasm_debug_spread(nuasm_plan pl, int32_t which, const void* vals, void* grid_out) {
  if (!pl || !grid_out) return fail(NUASM_ERR_INVALID_ARG, "plan or grid_out is NULL");
  if (which < 0 || which >= pl->nsets) return fail(NUASM_ERR_INVALID_ARG, "which must be 0 (or 1 for type 3)");
  PointSet& q = pl->ps[which];
  if (!q.ready) return fail(NUASM_ERR_NOT_READY, "the point set is not bound");
  if (!vals && q.M > 0) return fail(NUASM_ERR_INVALID_ARG, "vals is NULL");
  nuasm_status s = run_spread(pl, q, (const float2*)vals);
  if (s != NUASM_OK) return s;
  const size_t n = (size_t)pl->geom.L * pl->geom.L;
  HIP_TRY(hipMemcpyAsync(grid_out, pl->gridA, sizeof(float2) * n, hipMemcpyDeviceToDevice, pl->stream),
          "hipMemcpyAsync");
  return NUASM_OK;
}

nuasm_status nuasm_debug_interp(nuasm_plan pl, int32_t which, const void* grid, void* out) {
  if (!pl || !grid) return fail(NUASM_ERR_INVALID_ARG, "plan or grid is NULL");
  if (which < 0 || which >= pl->nsets) return fail(NUASM_ERR_INVALID_ARG, "which must be 0 (or 1 for type 3)");
  PointSet& q = pl->ps[which];
  if (!q.ready) return fail(NUASM_ERR_NOT_READY, "the point set is not bound");
  if (!out && q.M > 0) return fail(NUASM_ERR_INVALID_ARG, "out is NULL");
  return run_interp(pl, q, (const float2*)grid, (float2*)out);
}

nuasm_status nuasm_debug_fft(int64_t n, int64_t batch, int32_t sign, const void* in, void* out, void* stream) {
  if (!is_pow2(n) || n < 32 || n > (1 << kMaxLogN)) return fail(NUASM_ERR_UNSUPPORTED, "n must be 2^5..2^14");
  if (batch < 0 || (sign != -1 && sign != 1)) return fail(NUASM_ERR_INVALID_ARG, "bad batch or sign");
  if (batch > (int64_t)INT32_MAX) return fail(NUASM_ERR_UNSUPPORTED, "batch must be below 2^31");
  if (batch == 0) return NUASM_OK;
  if (!in || !out) return fail(NUASM_ERR_INVALID_ARG, "in/out pointer is NULL");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return fail(NUASM_ERR_NO_DEVICE, "no HIP device visible");
  }
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  const float2* tw = nullptr;
  nuasm_status s = twiddles_for_device(dev, &tw);
  if (s != NUASM_OK) return s;
  int logn = 0;
  while ((int64_t(1) << logn) < n) ++logn;
  HIP_TRY(launch_fft_rows(logn, batch, sign, (const float2*)in, (float2*)out, tw, (hipStream_t)stream),
          "launch fft_rows");
  return NUASM_OK;
}


nuasm_status nuasm_rs_direct(int64_t M1, const double* x1, const double* y1, const void* c, int64_t M2,
                             const double* x2, const double* y2, double lambda, double z, double ox, double oy,
                             void* out, void* stream) {
  if (M1 < 0 || M2 < 0) return fail(NUASM_ERR_INVALID_ARG, "point counts must be >= 0");
  if (M1 > 0 && (!x1 || !y1 || !c)) return fail(NUASM_ERR_INVALID_ARG, "source pointer is NULL");
  if (M2 > 0 && (!x2 || !y2 || !out)) return fail(NUASM_ERR_INVALID_ARG, "destination pointer is NULL");
  if (!(lambda > 0.0) || !std::isfinite(lambda)) return fail(NUASM_ERR_INVALID_ARG, "lambda must be > 0");
  if (!std::isfinite(z) || z == 0.0) return fail(NUASM_ERR_INVALID_ARG, "z must be finite and != 0");
  if (!std::isfinite(ox) || !std::isfinite(oy)) return fail(NUASM_ERR_INVALID_ARG, "offset must be finite");
  if ((M2 + 63) / 64 > (int64_t)INT32_MAX) return fail(NUASM_ERR_UNSUPPORTED, "too many destination points");
  if (M2 == 0) return NUASM_OK;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
    (void)hipGetLastError();
    return fail(NUASM_ERR_NO_DEVICE, "no HIP device visible");
  }
  const double az = std::fabs(z);
  const double zl = az / lambda;
  const double k = 2.0 * kPi / lambda;
  RsConst kc{};
  kc.ox = ox;
  kc.oy = oy;
  kc.inv_z2 = 1.0 / (z * z);
  kc.inv_lz = 1.0 / (lambda * az);
  kc.c0 = zl - std::nearbyint(zl);
  kc.inv_2pi = 1.0 / (2.0 * kPi);
  kc.a3 = (float)(z / (az * az * az));
  kc.ak = (float)(k * z / (z * z));
  HIP_TRY(launch_rs_direct(x1, y1, (const float2*)c, M1, x2, y2, M2, kc, (float2*)out, (hipStream_t)stream),
          "launch rs_direct");
  return NUASM_OK;
}

// ================================================================ batches
}  // extern "C"

// One grouped launch: the same kernel instantiation for every plane that has
// it in one stage, its planes' arguments in a device table.
struct GroupedStage {
  int stage = 0;
  hipError_t (*grouped)(const void*, const int*, int, int, size_t, hipStream_t) = nullptr;
  int n = 0;            // planes (table entries)
  int blocks = 0;       // blocks of all entries
  size_t lds = 0;       // the largest entry's dynamic LDS
  size_t tab_off = 0;   // entry table and block offsets inside the batch's table buffer
  size_t first_off = 0;
  std::vector<int> planes;
};

// One recorded graph of a batch and the arguments it was recorded with.
struct BatchGraph {
  hipGraphExec_t exec = nullptr;
  std::vector<const void*> key;
  bool grouped = false;
  std::vector<GroupedStage> stages;
  char* tables = nullptr;  // device: every grouped stage's entry table and block offsets
  size_t table_bytes = 0;
  std::vector<int64_t> M;    // the point counts it was recorded with
  std::vector<int> slot_of;  // plane -> its completion stamp in ts (0: finished at the start)
};

struct nuasm_batch_s {
  std::vector<nuasm_plan_s*> plans;
  hipStream_t stream = nullptr;  // caller's stream
  hipStream_t cap = nullptr;     // internal stream the graphs are recorded on (they run on `stream`)
  std::vector<hipStream_t> branch;
  int active = 0;              // branches in use (nuasm_batch_set_branches)
  std::vector<int> branch_of;  // plane -> branch
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  // one-shot (binning + operator), binning alone, operator alone
  BatchGraph g_run, g_bin, g_exec;
  bool grouped = true;         // grouped stage launches (nuasm_batch_set_grouped)
  bool stamps = true;          // completion stamps recorded (nuasm_batch_set_plane_times)
  long long* ts = nullptr;     // [P + 1] device wall-clock stamps: the start, then completions
  const BatchGraph* last = nullptr;  // the graph launched last
  int clock_khz = 0;
  int64_t recorded = 0, refreshed = 0;  // graph recordings; grouped tables rewritten in place
};

namespace {

constexpr int kBranches = 4;

void drop_graph(BatchGraph& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  g.exec = nullptr;
  g.key.clear();
  if (g.tables) (void)dev_free(g.tables);
  g.tables = nullptr;
  g.stages.clear();
  g.table_bytes = 0;
  g.M.clear();
  g.slot_of.clear();
  g.grouped = false;
}

void batch_release(nuasm_batch_s* b) {
  drop_graph(b->g_run);
  drop_graph(b->g_bin);
  drop_graph(b->g_exec);
  for (nuasm_plan_s* pl : b->plans) {
    if (!pl) continue;
    release(pl);
    delete pl;
  }
  for (hipStream_t s : b->branch) (void)hipStreamDestroy(s);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (hipEvent_t e : b->join) (void)hipEventDestroy(e);
  if (b->ts) (void)dev_free(b->ts);
}

}  // namespace

// Modelled GPU time of one plane (one-shot: binning + operator), in
// microseconds, from per-kernel timings of the N' = 2048, M = 2^20 workload on
// MI355X: the grid passes scale with the stored support L^2 (about 2.1e-5 us
// per cell for either type), binning with the points (5.2e-5 us each), and
// the point kernels with the points too: spreading with its reduction
// 7.4e-5 us per point, interpolation 3.8e-5.  Only the ratios matter.
static double plane_cost(const nuasm_plan_s* pl, int64_t M) {
  const double grid = 2.1e-5 * (double)pl->geom.L * (double)pl->geom.L;
  const double pts = (5.2e-5 + (pl->p.type == NUASM_TYPE_1 ? 7.4e-5 : 3.8e-5)) * (double)M;
  return 20.0 + grid + pts;
}

// Longest-processing-time assignment of the planes to the capture branches.
static void assign_branches(nuasm_batch_s* b, const std::vector<int64_t>& M) {
  const int P = (int)b->plans.size(), K = b->active;
  std::vector<double> work(P);
  std::vector<int> order(P);
  for (int p = 0; p < P; ++p) {
    work[p] = plane_cost(b->plans[p], M[p]);
    order[p] = p;
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return work[a] > work[c]; });
  std::vector<double> load(K, 0.0);
  for (int p : order) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    b->branch_of[p] = k;
    load[k] += work[p];
  }
}

// Pipeline order of the stages for grouped execution, and which chain each
// belongs to: the type-1 planes' binning, then the type-1 operator, on one
// branch; the type-2 grid passes (which need no points), the type-2 planes'
// binning and the interpolation on a second.  The type-2 planes' binning
// launches are told apart by a stage offset (kStageBinB) when they are
// collected, so that the two chains share nothing.
constexpr int kStageBinB = 100;
static const int kGroupOrderA[] = {NUASM_STAGE_BIN_HIST, NUASM_STAGE_BIN_COLSCAN, NUASM_STAGE_BIN_SCAN,
                                   NUASM_STAGE_BIN_SCATTER,
                                   NUASM_STAGE_SPREAD,   NUASM_STAGE_SPREAD_REDUCE, NUASM_STAGE_T1_ROWS,
                                   NUASM_STAGE_T1_COLS,  NUASM_STAGE_T1_ROWS_INV};
static const int kGroupOrderB[] = {NUASM_STAGE_T2_ROWS,
                                   NUASM_STAGE_T2_COLS,
                                   NUASM_STAGE_T2_ROWS_INV,
                                   kStageBinB + NUASM_STAGE_BIN_HIST,
                                   kStageBinB + NUASM_STAGE_BIN_COLSCAN,
                                   kStageBinB + NUASM_STAGE_BIN_SCAN,
                                   kStageBinB + NUASM_STAGE_BIN_SCATTER,
                                   NUASM_STAGE_INTERP};

// Collect every plane's launches (plane(pl, p) with the recorder active: host
// logic and allocations run, kernels are only recorded), group them by stage
// and kernel instantiation, and upload the grouped launches' tables.
template <typename F>
static nuasm_status batch_collect_host(nuasm_batch_s* b, F plane, std::vector<GroupedStage>& stages,
                                       std::vector<unsigned char>& host) {
  const int P = (int)b->plans.size();
  std::vector<LaunchRecorder> rec(P);
  for (int p = 0; p < P; ++p) {
    nuasm_plan_s* pl = b->plans[p];
    pl->stream = b->stream;
    pl->timing = false;
    active_recorder() = &rec[p];
    const nuasm_status s = plane(pl, p);
    active_recorder() = nullptr;
    if (s != NUASM_OK) return fail(s, "plane " + std::to_string(p) + ": " + g_last_error);
    if (pl->p.type == NUASM_TYPE_2)
      for (RecordedLaunch& L : rec[p].launches)
        if (L.stage == NUASM_STAGE_BIN_HIST || L.stage == NUASM_STAGE_BIN_COLSCAN || L.stage == NUASM_STAGE_BIN_SCAN ||
            L.stage == NUASM_STAGE_BIN_SCATTER)
          L.stage += kStageBinB;
  }
  // group: for each stage in pipeline order, one launch per instantiation
  std::vector<int> order(std::begin(kGroupOrderA), std::end(kGroupOrderA));
  order.insert(order.end(), std::begin(kGroupOrderB), std::end(kGroupOrderB));
  std::vector<std::vector<const RecordedLaunch*>> members;
  for (int stage : order) {
    std::vector<const void*> keys;
    for (int p = 0; p < P; ++p)
      for (const RecordedLaunch& L : rec[p].launches)
        if (L.stage == stage && std::find(keys.begin(), keys.end(), L.key) == keys.end()) keys.push_back(L.key);
    for (const void* key : keys) {
      GroupedStage gs;
      gs.stage = stage;
      std::vector<const RecordedLaunch*> mem;
      for (int p = 0; p < P; ++p)
        for (const RecordedLaunch& L : rec[p].launches)
          if (L.stage == stage && L.key == key) {
            mem.push_back(&L);
            gs.planes.push_back(p);
            gs.grouped = L.grouped;
            gs.lds = std::max(gs.lds, L.lds);
            gs.blocks += L.blocks;
          }
      gs.n = (int)mem.size();
      stages.push_back(gs);
      members.push_back(mem);
    }
  }
  // tables: entries (each stage's argument struct), then block offsets
  size_t bytes = 0;
  for (size_t i = 0; i < stages.size(); ++i) {
    GroupedStage& gs = stages[i];
    gs.tab_off = bytes;
    bytes = round256(bytes + (size_t)gs.n * members[i][0]->arg_bytes);
    gs.first_off = bytes;
    bytes = round256(bytes + sizeof(int) * (size_t)(gs.n + 1));
  }
  host.assign(std::max<size_t>(bytes, 1), 0);
  for (size_t i = 0; i < stages.size(); ++i) {
    const GroupedStage& gs = stages[i];
    int* first = (int*)(host.data() + gs.first_off);
    int run = 0;
    for (int e = 0; e < gs.n; ++e) {
      const RecordedLaunch& L = *members[i][e];
      std::memcpy(host.data() + gs.tab_off + (size_t)e * L.arg_bytes, L.args.data(), L.arg_bytes);
      first[e] = run;
      run += L.blocks;
    }
    first[gs.n] = run;
  }
  return NUASM_OK;
}

template <typename F>
static nuasm_status batch_collect(nuasm_batch_s* b, BatchGraph& g, F plane) {
  std::vector<unsigned char> host;
  nuasm_status s = batch_collect_host(b, plane, g.stages, host);
  if (s != NUASM_OK) return s;
  HIP_TRY(dev_malloc((void**)&g.tables, host.size()), "hipMalloc(grouped tables)");
  HIP_TRY(hipMemcpy(g.tables, host.data(), host.size(), hipMemcpyHostToDevice), "hipMemcpy(grouped tables)");
  g.table_bytes = host.size();
  return NUASM_OK;
}

// Same launches, tables laid out alike: a grouped graph recorded with one set
// of arguments runs with another once its tables hold the new entries.
static bool same_layout(const std::vector<GroupedStage>& a, const std::vector<GroupedStage>& b) {
  if (a.size() != b.size()) return false;
  for (size_t i = 0; i < a.size(); ++i)
    if (a[i].stage != b[i].stage || a[i].grouped != b[i].grouped || a[i].n != b[i].n || a[i].blocks != b[i].blocks ||
        a[i].lds != b[i].lds || a[i].tab_off != b[i].tab_off || a[i].first_off != b[i].first_off ||
        a[i].planes != b[i].planes)
      return false;
  return true;
}

// Enqueue the grouped launches of the two chains (stages in orderA on sA,
// orderB on sB), one stage of each in turn: the graph launches its nodes in
// recorded order, so neither chain's first kernels wait for the other chain's
// whole submission.  With stamps on, a launch that finishes planes (their
// last grouped launch) is followed by one completion stamp in the next free
// slot of ts, which g.slot_of maps them to.
static hipError_t enqueue_chains(nuasm_batch_s* b, BatchGraph& g, const int* orderA, int nA, hipStream_t sA,
                                 const int* orderB, int nB, hipStream_t sB, const std::vector<int>& last_stage_of) {
  hipError_t e = hipSuccess;
  int next_slot = 1;
  auto stage_launches = [&](int stage, hipStream_t st) {
    for (size_t i = 0; i < g.stages.size() && e == hipSuccess; ++i) {
      const GroupedStage& gs = g.stages[i];
      if (gs.stage != stage) continue;
      e = gs.grouped(g.tables + gs.tab_off, (const int*)(g.tables + gs.first_off), gs.n, gs.blocks, gs.lds, st);
      if (e != hipSuccess || !b->stamps) continue;
      bool finishes = false;
      for (int p : gs.planes)
        if (last_stage_of[p] == (int)i) {
          finishes = true;
          g.slot_of[p] = next_slot;
        }
      if (finishes) e = launch_stamp(b->ts + next_slot++, st);
    }
  };
  for (int k = 0; k < std::max(nA, nB) && e == hipSuccess; ++k) {
    if (k < nA) stage_launches(orderA[k], sA);
    if (k < nB && e == hipSuccess) stage_launches(orderB[k], sB);
  }
  return e;
}

// Launch graph g, or record it first when it is missing or was recorded with
// other arguments (key).  plane(pl, p) enqueues plane p's work on the plan's
// current stream.  Recording: one eager pass on the caller's stream (sizes every
// buffer and sets kernel attributes, so that the capture enqueues launches
// only), then the capture on the internal stream -- stamp, fork onto the
// branches, every plane on its branch followed by its completion stamp, join.
// The graph is launched on the caller's stream itself.
template <typename F>
static nuasm_status batch_launch(nuasm_batch_s* b, BatchGraph& g, const std::vector<const void*>& key,
                                 const std::vector<int64_t>& M, F plane) {
  const int P = (int)b->plans.size();
  auto launch = [&]() -> nuasm_status {
    // on the caller's stream itself: ordered with its other work, no event
    // hops between streams
    b->last = &g;
    HIP_TRY(hipGraphLaunch(g.exec, b->stream), "hipGraphLaunch");
    return NUASM_OK;
  };
  if (g.exec && key == g.key && g.grouped == b->grouped) return launch();
  if (g.exec && g.grouped && b->grouped && M == g.M) {
    // only buffers changed (the point counts, and so every size and grid, are
    // the ones recorded): collect the new arguments on the host and, when
    // the launches come out the same, rewrite the tables in place once the
    // graph's last run has finished, instead of recording again
    std::vector<GroupedStage> stages;
    std::vector<unsigned char> host;
    const nuasm_status s = batch_collect_host(b, plane, stages, host);
    for (nuasm_plan_s* pl : b->plans) pl->stream = b->stream;
    if (s != NUASM_OK) return s;
    if (same_layout(stages, g.stages) && host.size() == g.table_bytes) {
      HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
      HIP_TRY(hipMemcpy(g.tables, host.data(), host.size(), hipMemcpyHostToDevice), "hipMemcpy(grouped tables)");
      g.key = key;
      ++b->refreshed;
      return launch();
    }
  }
  if (g.exec || g.tables) {
    HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    drop_graph(g);
  }
  // eager pass on the caller's stream: sizes every buffer and sets kernel
  // attributes, so that the capture below enqueues launches only
  for (int p = 0; p < P; ++p) {
    nuasm_plan_s* pl = b->plans[p];
    pl->stream = b->stream;
    pl->timing = false;
    nuasm_status s = plane(pl, p);
    if (s != NUASM_OK) return fail(s, "plane " + std::to_string(p) + ": " + g_last_error);
  }
  HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  if (b->grouped) {
    g.grouped = true;
    nuasm_status s = batch_collect(b, g, plane);
    for (nuasm_plan_s* pl : b->plans) pl->stream = b->stream;
    if (s != NUASM_OK) {
      drop_graph(g);
      return s;
    }
  }
  if (!b->grouped) assign_branches(b, M);
  HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  nuasm_status st = NUASM_OK;
  // planes with no launch at all finish at the start (slot 0)
  g.slot_of.assign(P, 0);
  hipError_t e = b->stamps ? launch_stamp(b->ts, b->cap) : hipSuccess;
  if (e == hipSuccess) e = hipEventRecord(b->fork, b->cap);
  if (b->grouped) {
    // two independent chains: the type-1 planes (binning, operator) on branch
    // 0, the type-2 planes (grid passes, binning, interpolation) on branch 1
    std::vector<int> last(P, -1);
    for (size_t i = 0; i < g.stages.size(); ++i)
      for (int p : g.stages[i].planes) last[p] = (int)i;
    hipStream_t s0 = b->branch[0], s1 = b->branch[1];
    if (e == hipSuccess) e = hipStreamWaitEvent(s0, b->fork, 0);
    if (e == hipSuccess) e = hipStreamWaitEvent(s1, b->fork, 0);
    if (e == hipSuccess)
      e = enqueue_chains(b, g, kGroupOrderA, (int)(sizeof(kGroupOrderA) / sizeof(int)), s0, kGroupOrderB,
                         (int)(sizeof(kGroupOrderB) / sizeof(int)), s1, last);
    for (size_t k = 0; e == hipSuccess && k < 2; ++k) {
      e = hipEventRecord(b->join[k], b->branch[k]);
      if (e == hipSuccess) e = hipStreamWaitEvent(b->cap, b->join[k], 0);
    }
  } else {
    for (size_t k = 0; e == hipSuccess && k < (size_t)b->active; ++k)
      e = hipStreamWaitEvent(b->branch[k], b->fork, 0);
    for (int p = 0; e == hipSuccess && st == NUASM_OK && p < P; ++p) {
      nuasm_plan_s* pl = b->plans[p];
      pl->stream = b->branch[b->branch_of[p]];
      st = plane(pl, p);
      if (st == NUASM_OK && b->stamps) {
        g.slot_of[p] = 1 + p;
        e = launch_stamp(b->ts + 1 + p, pl->stream);
      }
    }
    for (size_t k = 0; e == hipSuccess && k < (size_t)b->active; ++k) {
      e = hipEventRecord(b->join[k], b->branch[k]);
      if (e == hipSuccess) e = hipStreamWaitEvent(b->cap, b->join[k], 0);
    }
  }
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(b->cap, &graph);
  for (nuasm_plan_s* pl : b->plans) pl->stream = b->stream;
  if (st != NUASM_OK || e != hipSuccess || e2 != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    drop_graph(g);
    if (st != NUASM_OK) return st;
    return hip_fail(e != hipSuccess ? e : e2, "graph capture");
  }
  e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    g.exec = nullptr;
    drop_graph(g);
    return hip_fail(e, "hipGraphInstantiate");
  }
  g.key = key;
  g.M = M;
  ++b->recorded;
  return launch();
}

extern "C" {

nuasm_status nuasm_batch_create(int32_t P, const nuasm_params* params, void* hip_stream, nuasm_batch* out) {
  if (!out) return fail(NUASM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (P <= 0 || !params) return fail(NUASM_ERR_INVALID_ARG, "need P > 0 plane parameters");
  nuasm_batch_s* b = new (std::nothrow) nuasm_batch_s();
  if (!b) return fail(NUASM_ERR_ALLOC, "host allocation failed");
  b->stream = (hipStream_t)hip_stream;
  auto bail = [&](nuasm_status st) {
    batch_release(b);
    delete b;
    return st;
  };
  for (int p = 0; p < P; ++p) {
    nuasm_params q = params[p];
    if (q.type == NUASM_TYPE_3) {
      batch_release(b);
      delete b;
      return fail(NUASM_ERR_UNSUPPORTED, "plane " + std::to_string(p) + ": type-3 plans are not batched");
    }
    q.flags |= NUASM_DEFER_RANGE_CHECK;
    nuasm_plan pl = nullptr;
    nuasm_status s = nuasm_plan_create(&q, hip_stream, &pl);
    if (s != NUASM_OK) {
      std::string m = "plane " + std::to_string(p) + ": " + g_last_error;
      b->plans.push_back(nullptr);
      batch_release(b);
      delete b;
      return fail(s, m);
    }
    b->plans.push_back(pl);
  }
  b->active = std::min(kBranches, (int)P);
  b->branch_of.assign(P, 0);
  hipError_t e;
  for (int k = 0; k < kBranches; ++k) {
    hipStream_t st = nullptr;
    if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess)
      return bail(hip_fail(e, "hipStreamCreate"));
    b->branch.push_back(st);
    hipEvent_t ev = nullptr;
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
      return bail(hip_fail(e, "hipEventCreate"));
    b->join.push_back(ev);
  }
  if ((e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming)) != hipSuccess)
    return bail(hip_fail(e, "hipEventCreate"));
  if ((e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking)) != hipSuccess)
    return bail(hip_fail(e, "hipStreamCreate"));
  if ((e = dev_malloc((void**)&b->ts, sizeof(long long) * (P + 1))) != hipSuccess)
    return bail(hip_fail(e, "hipMalloc(stamps)"));
  int dev = 0;
  (void)hipGetDevice(&dev);
  if ((e = hipDeviceGetAttribute(&b->clock_khz, hipDeviceAttributeWallClockRate, dev)) != hipSuccess)
    return bail(hip_fail(e, "hipDeviceGetAttribute(wall clock)"));
  *out = b;
  return NUASM_OK;
}

nuasm_status nuasm_plan_many_create(int32_t P, const nuasm_params* params, void* hip_stream, nuasm_batch* out) {
  return nuasm_batch_create(P, params, hip_stream, out);
}

nuasm_status nuasm_batch_destroy(nuasm_batch b) {
  if (!b) return NUASM_OK;
  (void)hipStreamSynchronize(b->stream);
  if (b->cap) (void)hipStreamSynchronize(b->cap);
  for (hipStream_t s : b->branch) (void)hipStreamSynchronize(s);
  batch_release(b);
  delete b;
  return NUASM_OK;
}

nuasm_status nuasm_batch_run(nuasm_batch b, const int64_t* M, const double* const* x, const double* const* y,
                             const void* const* in, void* const* out) {
  if (!b || !M || !x || !y || !in || !out) return fail(NUASM_ERR_INVALID_ARG, "NULL argument");
  const int P = (int)b->plans.size();
  std::vector<const void*> key;
  std::vector<int64_t> Ms(P);
  key.reserve(5 * P);
  for (int p = 0; p < P; ++p) {
    if (M[p] < 0) return fail(NUASM_ERR_INVALID_ARG, "M < 0");
    Ms[p] = M[p];
    key.push_back((const void*)(intptr_t)M[p]);
    key.push_back(x[p]);
    key.push_back(y[p]);
    key.push_back(in[p]);
    key.push_back(out[p]);
  }
  return batch_launch(b, b->g_run, key, Ms, [&](nuasm_plan_s* pl, int p) {
    nuasm_status s = nuasm_set_points(pl, M[p], x[p], y[p]);
    if (s != NUASM_OK) return s;
    return nuasm_execute(pl, in[p], out[p]);
  });
}

nuasm_status nuasm_set_points_many(nuasm_batch b, const int64_t* M, const double* const* x, const double* const* y) {
  if (!b || !M || !x || !y) return fail(NUASM_ERR_INVALID_ARG, "NULL argument");
  const int P = (int)b->plans.size();
  std::vector<const void*> key;
  std::vector<int64_t> Ms(P);
  key.reserve(3 * P);
  for (int p = 0; p < P; ++p) {
    if (M[p] < 0) return fail(NUASM_ERR_INVALID_ARG, "M < 0");
    Ms[p] = M[p];
    key.push_back((const void*)(intptr_t)M[p]);
    key.push_back(x[p]);
    key.push_back(y[p]);
  }
  return batch_launch(b, b->g_bin, key, Ms,
                      [&](nuasm_plan_s* pl, int p) { return nuasm_set_points(pl, M[p], x[p], y[p]); });
}

nuasm_status nuasm_execute_many(nuasm_batch b, const void* const* in, void* const* out) {
  if (!b || !in || !out) return fail(NUASM_ERR_INVALID_ARG, "NULL argument");
  const int P = (int)b->plans.size();
  std::vector<const void*> key;
  std::vector<int64_t> Ms(P);
  key.reserve(3 * P);
  for (int p = 0; p < P; ++p) {
    const nuasm_plan_s* pl = b->plans[p];
    if (!pl->ready()) return fail(NUASM_ERR_NOT_READY, "plane " + std::to_string(p) + ": execute_many before set_points_many");
    // launch grids follow the bound point counts, so they are part of the key
    Ms[p] = pl->ps[0].M;
    key.push_back((const void*)(intptr_t)Ms[p]);
    key.push_back(in[p]);
    key.push_back(out[p]);
  }
  return batch_launch(b, b->g_exec, key, Ms, [&](nuasm_plan_s* pl, int p) { return nuasm_execute(pl, in[p], out[p]); });
}

namespace {
// Drop the recorded graphs so that the next runs record them again.
nuasm_status batch_invalidate(nuasm_batch_s* b) {
  HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  drop_graph(b->g_run);
  drop_graph(b->g_bin);
  drop_graph(b->g_exec);
  return NUASM_OK;
}
}  // namespace

nuasm_status nuasm_batch_set_tuning(nuasm_batch b, int32_t plane, const nuasm_tuning* t) {
  if (!b || !t) return fail(NUASM_ERR_INVALID_ARG, "batch or tuning is NULL");
  if (plane < 0 || plane >= (int32_t)b->plans.size()) return fail(NUASM_ERR_INVALID_ARG, "plane index out of range");
  nuasm_status s = batch_invalidate(b);
  if (s != NUASM_OK) return s;
  return nuasm_plan_set_tuning(b->plans[plane], t);
}

nuasm_status nuasm_batch_set_branches(nuasm_batch b, int32_t branches) {
  if (!b) return fail(NUASM_ERR_INVALID_ARG, "batch is NULL");
  if (branches < 1 || branches > std::min<int32_t>(kBranches, (int32_t)b->plans.size()))
    return fail(NUASM_ERR_INVALID_ARG, "branches must be in [1, min(4, planes)]");
  nuasm_status s = batch_invalidate(b);
  if (s != NUASM_OK) return s;
  b->active = branches;
  return NUASM_OK;
}

nuasm_status nuasm_batch_set_grouped(nuasm_batch b, int32_t grouped) {
  if (!b) return fail(NUASM_ERR_INVALID_ARG, "batch is NULL");
  if (grouped != 0 && grouped != 1) return fail(NUASM_ERR_INVALID_ARG, "grouped must be 0 or 1");
  nuasm_status s = batch_invalidate(b);
  if (s != NUASM_OK) return s;
  b->grouped = grouped != 0;
  return NUASM_OK;
}

nuasm_status nuasm_batch_check_points(nuasm_batch b, int32_t* bad_plane) {
  if (!b || !bad_plane) return fail(NUASM_ERR_INVALID_ARG, "NULL argument");
  HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  *bad_plane = -1;
  for (size_t p = 0; p < b->plans.size(); ++p) {
    nuasm_plan_s* pl = b->plans[p];
    PointSet& q = pl->ps[0];
    HIP_TRY(hipMemcpy(q.host_stat, q.nch, sizeof(int) * 6, hipMemcpyDeviceToHost), "hipMemcpy");
    const nuasm_status ps = point_status(q, 0);
    if (ps != NUASM_OK) {
      *bad_plane = (int32_t)p;
      return fail(ps, "plane " + std::to_string(p) + ": " + g_last_error);
    }
  }
  return NUASM_OK;
}

nuasm_status nuasm_debug_batch_graphs(nuasm_batch b, int64_t* recorded, int64_t* refreshed) {
  if (!b || !recorded || !refreshed) return fail(NUASM_ERR_INVALID_ARG, "NULL argument");
  *recorded = b->recorded;
  *refreshed = b->refreshed;
  return NUASM_OK;
}

nuasm_status nuasm_batch_set_plane_times(nuasm_batch b, int32_t enabled) {
  if (!b) return fail(NUASM_ERR_INVALID_ARG, "batch is NULL");
  if (enabled != 0 && enabled != 1) return fail(NUASM_ERR_INVALID_ARG, "enabled must be 0 or 1");
  if (b->stamps == (enabled != 0)) return NUASM_OK;
  nuasm_status s = batch_invalidate(b);
  if (s != NUASM_OK) return s;
  b->stamps = enabled != 0;
  b->last = nullptr;
  return NUASM_OK;
}

nuasm_status nuasm_batch_plane_times(nuasm_batch b, float* ms) {
  if (!b || !ms) return fail(NUASM_ERR_INVALID_ARG, "NULL argument");
  if (!b->stamps) return fail(NUASM_ERR_NOT_READY, "plane times are off (nuasm_batch_set_plane_times)");
  if (!b->last || !b->last->exec) return fail(NUASM_ERR_NOT_READY, "no recorded graph has run");
  HIP_TRY(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  const size_t P = b->plans.size();
  std::vector<long long> h(P + 1);
  HIP_TRY(hipMemcpy(h.data(), b->ts, sizeof(long long) * (P + 1), hipMemcpyDeviceToHost), "hipMemcpy");
  const std::vector<int>& slot = b->last->slot_of;
  for (size_t p = 0; p < P; ++p) ms[p] = (float)((double)(h[slot[p]] - h[0]) / (double)b->clock_khz);
  return NUASM_OK;
}

}  // extern "C"

namespace nuasm {
LaunchRecorder*& active_recorder() {
  static thread_local LaunchRecorder* r = nullptr;
  return r;
}
}  // namespace nuasm
