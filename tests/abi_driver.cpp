// Drives the C ABI of libnuasm from a host program built with host-side
// AddressSanitizer and UndefinedBehaviorSanitizer (the kernels are not
// instrumented).
//
//   abi_driver cpu   argument validation, status strings and the paths that
//                    need no device (plan creation reports NUASM_ERR_NO_DEVICE
//                    when none is visible)
//   abi_driver gpu   every operator's life cycle -- plans of the three types,
//                    a caller-owned workspace, a batch in one and two steps --
//                    with the k-th device or pinned allocation failing
//                    (nuasm_debug_fail_alloc), for every k up to the number a
//                    clean run makes: each failure must come back as
//                    NUASM_ERR_ALLOC from the call that allocated, every
//                    object must then destroy cleanly, and the memory the
//                    library holds (nuasm_debug_live_bytes) must return to
//                    where it started
//
// Prints one line per check group and "ABI_DRIVER_OK" at the end; any failed
// check prints its line and exits with status 1.  Leaks of host memory and
// memory errors are the sanitizers' to report.
//
// The driver ends with an explicit leak check and _exit: the ROCm runtime's
// own teardown at normal exit frees device memory through the sanitizer's
// device allocator after the runtime it depends on has been unloaded, which
// stops the sanitizer on an internal check that says nothing about this
// program.
#include <hip/hip_runtime.h>
#include <sanitizer/lsan_interface.h>
#include <unistd.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "nuasm.h"

static int g_fail = 0;

#define CHECK(cond)                                                       \
  do {                                                                    \
    if (!(cond)) {                                                        \
      std::printf("CHECK FAILED %s:%d: %s (last error: %s)\n", __FILE__, \
                  __LINE__, #cond, nuasm_last_error());                   \
      g_fail = 1;                                                         \
      return;                                                             \
    }                                                                     \
  } while (0)

static void cpu_checks(bool have_device) {
  nuasm_params p;
  CHECK(nuasm_params_default(nullptr) == NUASM_ERR_INVALID_ARG);
  CHECK(nuasm_params_default(&p) == NUASM_OK);
  for (int s = 0; s <= 7; ++s)
    CHECK(std::strcmp(nuasm_status_string((nuasm_status)s), "NUASM_UNKNOWN_STATUS") != 0);
  CHECK(std::strcmp(nuasm_status_string((nuasm_status)8), "NUASM_UNKNOWN_STATUS") == 0);
  CHECK(nuasm_last_error() != nullptr);
  nuasm_plan pl = (nuasm_plan)0x1;
  CHECK(nuasm_plan_create(nullptr, nullptr, &pl) == NUASM_ERR_INVALID_ARG && pl == nullptr);
  CHECK(nuasm_plan_create(&p, nullptr, nullptr) == NUASM_ERR_INVALID_ARG);
  nuasm_params bad = p;
  bad.N = 100;
  pl = (nuasm_plan)0x1;
  CHECK(nuasm_plan_create(&bad, nullptr, &pl) == NUASM_ERR_UNSUPPORTED && pl == nullptr);
  bad = p;
  bad.tol = 0.5;
  CHECK(nuasm_plan_create(&bad, nullptr, &pl) == NUASM_ERR_INVALID_ARG && pl == nullptr);
  bad = p;
  bad.band = NUASM_BAND_EXPLICIT;
  bad.band_w[0] = -1.0;
  CHECK(nuasm_plan_create(&bad, nullptr, &pl) == NUASM_ERR_INVALID_ARG && pl == nullptr);
  // calls on a NULL plan
  CHECK(nuasm_plan_destroy(nullptr) == NUASM_OK);
  CHECK(nuasm_set_points(nullptr, 1, nullptr, nullptr) == NUASM_ERR_INVALID_ARG);
  CHECK(nuasm_execute(nullptr, nullptr, nullptr) == NUASM_ERR_INVALID_ARG);
  CHECK(nuasm_execute_adjoint(nullptr, nullptr, nullptr) == NUASM_ERR_INVALID_ARG);
  CHECK(nuasm_execute_noalloc(nullptr, nullptr, nullptr) == NUASM_ERR_INVALID_ARG);
  size_t bytes = 0;
  CHECK(nuasm_plan_workspace_bytes(nullptr, 10, &bytes) == NUASM_ERR_INVALID_ARG);
  CHECK(nuasm_plan_set_workspace(nullptr, nullptr, 0) == NUASM_ERR_INVALID_ARG);
  nuasm_tuning t{};
  t.spread_method = 3;
  CHECK(nuasm_plan_set_tuning(nullptr, &t) == NUASM_ERR_INVALID_ARG);
  nuasm_plan_info info;
  CHECK(nuasm_plan_get_info(nullptr, &info) == NUASM_ERR_INVALID_ARG);
  // batches
  nuasm_batch b = (nuasm_batch)0x1;
  CHECK(nuasm_batch_create(0, &p, nullptr, &b) == NUASM_ERR_INVALID_ARG && b == nullptr);
  CHECK(nuasm_batch_destroy(nullptr) == NUASM_OK);
  int64_t M = 1;
  const double* xs[1] = {nullptr};
  const void* ins[1] = {nullptr};
  void* outs[1] = {nullptr};
  CHECK(nuasm_set_points_many(nullptr, &M, xs, xs) == NUASM_ERR_INVALID_ARG);
  CHECK(nuasm_execute_many(nullptr, ins, outs) == NUASM_ERR_INVALID_ARG);
  CHECK(nuasm_batch_run(nullptr, &M, xs, xs, ins, outs) == NUASM_ERR_INVALID_ARG);
  CHECK(nuasm_batch_set_grouped(nullptr, 1) == NUASM_ERR_INVALID_ARG);
  // plan-less entry points
  CHECK(nuasm_debug_fft(100, 1, -1, nullptr, nullptr, nullptr) == NUASM_ERR_UNSUPPORTED);
  CHECK(nuasm_debug_fft(64, 1, 2, nullptr, nullptr, nullptr) == NUASM_ERR_INVALID_ARG);
  CHECK(nuasm_rs_direct(-1, nullptr, nullptr, nullptr, 0, nullptr, nullptr, 5e-7, 0.01, 0, 0, nullptr,
                        nullptr) == NUASM_ERR_INVALID_ARG);
  CHECK(nuasm_rs_direct(0, nullptr, nullptr, nullptr, 0, nullptr, nullptr, 5e-7, 0.0, 0, 0, nullptr,
                        nullptr) == NUASM_ERR_INVALID_ARG);
  CHECK(nuasm_debug_fail_alloc(-1) == NUASM_ERR_INVALID_ARG);
  int64_t db = -1, hb = -1;
  CHECK(nuasm_debug_live_bytes(nullptr, &hb) == NUASM_ERR_INVALID_ARG);
  CHECK(nuasm_debug_live_bytes(&db, &hb) == NUASM_OK && db >= 0 && hb >= 0);
  CHECK(nuasm_debug_fail_alloc(0) == NUASM_OK);
  // a valid plan: no device -> NUASM_ERR_NO_DEVICE; else a full life cycle
  pl = (nuasm_plan)0x1;
  const nuasm_status s = nuasm_plan_create(&p, nullptr, &pl);
  if (!have_device) {
    CHECK(s == NUASM_ERR_NO_DEVICE && pl == nullptr);
    b = (nuasm_batch)0x1;
    CHECK(nuasm_batch_create(1, &p, nullptr, &b) == NUASM_ERR_NO_DEVICE && b == nullptr);
  } else {
    CHECK(s == NUASM_OK && pl != nullptr);
    CHECK(nuasm_execute(pl, nullptr, nullptr) == NUASM_ERR_NOT_READY);
    CHECK(nuasm_plan_destroy(pl) == NUASM_OK);
  }
  std::printf("cpu checks done (device visible: %d)\n", (int)have_device);
}

// ---------------------------------------------------------------- gpu mode
struct DevArrays {
  double *x = nullptr, *y = nullptr;
  float* c = nullptr;    // complex64 values / planes (interleaved floats)
  float* out = nullptr;
  float* ws = nullptr;   // a caller-owned workspace
};

static nuasm_params params(int type, int N, double z, int tf) {
  nuasm_params p;
  nuasm_params_default(&p);
  p.type = type;
  p.N = N;
  p.z = z;
  p.tf = tf;
  p.band = tf == NUASM_TF_ASM ? NUASM_BAND_LIMITED : NUASM_BAND_FULL;
  p.d1 = p.d2 = 4e-6;
  p.lambda = 633e-9;
  p.flags = NUASM_DEFER_RANGE_CHECK;
  return p;
}

// One run of every life cycle; returns the first non-OK status (NUASM_OK if
// all passed).  Objects are destroyed on every path.
static nuasm_status scenario(const DevArrays& d, int64_t M, size_t ws_bytes) {
  nuasm_status first = NUASM_OK;
  auto note = [&](nuasm_status s) {
    if (first == NUASM_OK && s != NUASM_OK) first = s;
    return s == NUASM_OK;
  };
  // type 1 and type 2 plans: bind, apply, adjoint
  for (int type = 1; type <= 2; ++type) {
    nuasm_params p = params(type, 64, 0.01, type == 1 ? NUASM_TF_ASM : NUASM_TF_FRESNEL);
    nuasm_plan pl = nullptr;
    if (note(nuasm_plan_create(&p, nullptr, &pl)) && note(nuasm_set_points(pl, M, d.x, d.y))) {
      note(nuasm_execute(pl, d.c, d.out));
      note(nuasm_execute_adjoint(pl, type == 1 ? d.out : d.c, type == 1 ? d.c : d.out));
      note(nuasm_execute_noalloc(pl, d.c, d.out));
    }
    nuasm_plan_destroy(pl);
  }
  // type 3 with a grid-bound destination
  {
    nuasm_params p = params(3, 64, 0.02, NUASM_TF_ASM);
    nuasm_plan pl = nullptr;
    if (note(nuasm_plan_create(&p, nullptr, &pl)) && note(nuasm_set_points(pl, M, d.x, d.y)) &&
        note(nuasm_set_grid_points(pl, 1, 40, 30, 3e-6, 0.0, 0.0)))
      note(nuasm_execute(pl, d.c, d.out));
    nuasm_plan_destroy(pl);
  }
  // a caller-owned workspace, then back to plan-owned memory
  {
    nuasm_params p = params(1, 64, 0.01, NUASM_TF_ASM);
    nuasm_plan pl = nullptr;
    size_t need = 0;
    if (note(nuasm_plan_create(&p, nullptr, &pl)) && note(nuasm_plan_workspace_bytes(pl, M, &need))) {
      if (need <= ws_bytes && note(nuasm_plan_set_workspace(pl, d.ws, ws_bytes)) &&
          note(nuasm_set_points(pl, M, d.x, d.y)))
        note(nuasm_execute(pl, d.c, d.out));
      if (note(nuasm_plan_set_workspace(pl, nullptr, 0)) && note(nuasm_set_points(pl, M, d.x, d.y)))
        note(nuasm_execute(pl, d.c, d.out));
    }
    nuasm_plan_destroy(pl);
  }
  // a batch: one-shot run, then points and operators in two steps, both forms
  {
    nuasm_params ps[3] = {params(1, 64, 0.01, NUASM_TF_ASM), params(2, 64, 0.02, NUASM_TF_FRESNEL),
                          params(1, 64, 0.05, NUASM_TF_FRESNEL)};
    nuasm_batch b = nullptr;
    const int64_t Ms[3] = {M, M, M / 2};
    const double* xs[3] = {d.x, d.x, d.x};
    const double* ys[3] = {d.y, d.y, d.y};
    const void* ins[3] = {d.c, d.c, d.c};
    void* outs[3] = {d.out, d.out, d.out};
    if (note(nuasm_batch_create(3, ps, nullptr, &b))) {
      for (int grouped = 1; grouped >= 0; --grouped) {
        if (!note(nuasm_batch_set_grouped(b, grouped))) break;
        if (!note(nuasm_batch_run(b, Ms, xs, ys, ins, outs))) break;
        if (!note(nuasm_set_points_many(b, Ms, xs, ys))) break;
        if (!note(nuasm_execute_many(b, ins, outs))) break;
      }
    }
    nuasm_batch_destroy(b);
  }
  (void)hipDeviceSynchronize();
  return first;
}

static void gpu_checks() {
  const int64_t M = 3000;
  DevArrays d;
  std::vector<double> hx(M), hy(M);
  for (int64_t j = 0; j < M; ++j) {  // points inside the 64 x 4 um window
    hx[j] = 1.2e-4 * std::sin(0.37 * (double)j);
    hy[j] = 1.2e-4 * std::cos(0.91 * (double)j);
  }
  const size_t plane = 128 * 128 * 2;  // the largest complex64 array the scenario uses, in floats
  const size_t ws_bytes = (size_t)64 << 20;
  CHECK(hipMalloc((void**)&d.x, sizeof(double) * M) == hipSuccess);
  CHECK(hipMalloc((void**)&d.y, sizeof(double) * M) == hipSuccess);
  CHECK(hipMalloc((void**)&d.c, sizeof(float) * plane) == hipSuccess);
  CHECK(hipMalloc((void**)&d.out, sizeof(float) * plane) == hipSuccess);
  CHECK(hipMalloc((void**)&d.ws, ws_bytes) == hipSuccess);
  CHECK(hipMemcpy(d.x, hx.data(), sizeof(double) * M, hipMemcpyHostToDevice) == hipSuccess);
  CHECK(hipMemcpy(d.y, hy.data(), sizeof(double) * M, hipMemcpyHostToDevice) == hipSuccess);
  CHECK(hipMemset(d.c, 0, sizeof(float) * plane) == hipSuccess);
  // a clean run first (also allocates the library's per-device tables)
  CHECK(nuasm_debug_fail_alloc(0) == NUASM_OK);
  CHECK(scenario(d, M, ws_bytes) == NUASM_OK);
  size_t free0 = 0, total = 0;
  CHECK(hipMemGetInfo(&free0, &total) == hipSuccess);
  int64_t dev0 = 0, host0 = 0;
  CHECK(nuasm_debug_live_bytes(&dev0, &host0) == NUASM_OK);
  int failures = 0, k = 1;
  for (; k <= 400; ++k) {
    CHECK(nuasm_debug_fail_alloc(k) == NUASM_OK);
    const nuasm_status s = scenario(d, M, ws_bytes);
    if (s == NUASM_OK) break;  // fewer than k allocations: every one has failed once
    if (s != NUASM_ERR_ALLOC) {
      std::printf("k = %d: first failure %s (%s), expected NUASM_ERR_ALLOC\n", k, nuasm_status_string(s),
                  nuasm_last_error());
      g_fail = 1;
      return;
    }
    ++failures;
  }
  CHECK(nuasm_debug_fail_alloc(0) == NUASM_OK);
  CHECK(k <= 400);
  CHECK(scenario(d, M, ws_bytes) == NUASM_OK);  // and everything works again
  size_t free1 = 0;
  CHECK(hipMemGetInfo(&free1, &total) == hipSuccess);
  int64_t dev1 = 0, host1 = 0;
  CHECK(nuasm_debug_live_bytes(&dev1, &host1) == NUASM_OK);
  std::printf("gpu: %d injected allocation failures, each reported and cleaned up; library-held device "
              "bytes %lld -> %lld, pinned host bytes %lld -> %lld; device free memory %zu -> %zu bytes "
              "(the runtime's own pools may move it)\n", failures, (long long)dev0, (long long)dev1,
              (long long)host0, (long long)host1, free0, free1);
  // every allocation the library made during the failures was given back
  CHECK(dev1 == dev0 && host1 == host0);
  hipFree(d.x);
  hipFree(d.y);
  hipFree(d.c);
  hipFree(d.out);
  hipFree(d.ws);
}

// Runs the leak check after a clean run; "ABI_DRIVER_OK" is printed only if
// it finds nothing.
static int finish(int code) {
  if (code == 0) {
    if (__lsan_do_recoverable_leak_check() != 0) {
      std::printf("leaks reported\n");
      code = 1;
    } else {
      std::printf("ABI_DRIVER_OK\n");
    }
  }
  std::fflush(stdout);
  std::fflush(stderr);
  _exit(code);
}

int main(int argc, char** argv) {
  std::setvbuf(stdout, nullptr, _IONBF, 0);
  const char* mode = argc > 1 ? argv[1] : "cpu";
  int ndev = 0;
  const bool have_device = hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0;
  if (!have_device) (void)hipGetLastError();
  if (std::strcmp(mode, "cpu") == 0) {
    cpu_checks(have_device);
  } else if (std::strcmp(mode, "gpu") == 0) {
    if (!have_device) {
      std::printf("gpu mode needs a device\n");
      return finish(2);
    }
    cpu_checks(true);
    if (!g_fail) gpu_checks();
  } else {
    std::printf("usage: abi_driver cpu|gpu\n");
    return finish(2);
  }
  if (g_fail) return finish(1);
  std::printf("checks passed\n");
  return finish(0);
}
