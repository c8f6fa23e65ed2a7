// Grouped launches: one launch of a kernel instantiation covering the work of
// many planes.  Every pipeline kernel is a __device__ body taking its
// arguments as one struct plus its (virtual) block index and block count;
// k_plain runs one plane's launch, k_grouped many planes' launches of the same
// instantiation at once, each block finding its plane's entry in a table by
// the block offsets (first[e] = first block of entry e, first[n] = total).
// While a recorder is active (a batch collecting its planes' work), the
// launchers append the launch to it instead of running it.
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

namespace nuasm {

struct RecordedLaunch {
  int stage;        // NUASM_STAGE_* the launch belongs to
  const void* key;  // the kernel instantiation (address of its plain kernel)
  hipError_t (*grouped)(const void* tab, const int* first, int n, int blocks, size_t lds, hipStream_t st);
  int blocks;
  size_t lds;
  size_t arg_bytes;
  std::vector<unsigned char> args;
};

struct LaunchRecorder {
  int stage = -1;
  std::vector<RecordedLaunch> launches;
};

// The calling thread's active recorder (null: launch normally).
LaunchRecorder*& active_recorder();

template <typename Args, void (*Body)(const Args&, int, int), int NT, int MINW = 1>
__global__ void __launch_bounds__(NT, MINW) k_plain(Args a) {
  Body(a, (int)blockIdx.x, (int)gridDim.x);
}

template <typename Args, void (*Body)(const Args&, int, int), int NT, int MINW = 1>
__global__ void __launch_bounds__(NT, MINW) k_grouped(const Args* __restrict__ tab, const int* __restrict__ first, int n) {
  const int b = (int)blockIdx.x;
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const Args a = tab[lo];
  Body(a, b - first[lo], first[lo + 1] - first[lo]);
}

template <typename Args, void (*Body)(const Args&, int, int), int NT, int MINW = 1>
hipError_t launch_grouped(const void* tab, const int* first, int n, int blocks, size_t lds, hipStream_t st) {
  hipLaunchKernelGGL((k_grouped<Args, Body, NT, MINW>), dim3(blocks), dim3(NT), lds, st, (const Args*)tab, first, n);
  return hipGetLastError();
}

// Dynamic LDS above 64 KB must be allowed per kernel: both forms.
template <typename Args, void (*Body)(const Args&, int, int), int NT, int MINW = 1>
hipError_t allow_lds(size_t lds) {
  if (lds <= 64 * 1024) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)k_plain<Args, Body, NT, MINW>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_grouped<Args, Body, NT, MINW>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

// Run one plane's launch, or record it for a grouped launch.
template <typename Args, void (*Body)(const Args&, int, int), int NT, int MINW = 1>
hipError_t launch_or_record(const Args& a, int blocks, size_t lds, hipStream_t st) {
  if (blocks <= 0) return hipSuccess;
  hipError_t e = allow_lds<Args, Body, NT, MINW>(lds);
  if (e != hipSuccess) return e;
  if (LaunchRecorder* r = active_recorder()) {
    RecordedLaunch L;
    L.stage = r->stage;
    L.key = (const void*)k_plain<Args, Body, NT, MINW>;
    L.grouped = &launch_grouped<Args, Body, NT, MINW>;
    L.blocks = blocks;
    L.lds = lds;
    L.arg_bytes = sizeof(Args);
    L.args.resize(sizeof(Args));
    std::memcpy(L.args.data(), &a, sizeof(Args));
    r->launches.push_back(std::move(L));
    return hipSuccess;
  }
  hipLaunchKernelGGL((k_plain<Args, Body, NT, MINW>), dim3(blocks), dim3(NT), lds, st, a);
  return hipGetLastError();
}

}  // namespace nuasm
