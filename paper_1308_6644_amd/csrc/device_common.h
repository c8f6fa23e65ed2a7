// Device helpers shared by the gfx950 kernels: complex arithmetic, the
// register-level DFT butterflies, the LDS Stockham FFT, and the
// exponential-of-semicircle spreading kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nuasm {

// ------------------------------------------------------------ complex math
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 czero() { return make_float2(0.f, 0.f); }

// exp(2 pi i x) for x in [-1/2, 1/2] cycles from the hardware sine and cosine,
// which take their argument in revolutions (v_sin_f32 / v_cos_f32; measured
// error below 1.3e-7 over that range, against 5.5e-8 for sincospif).
__device__ __forceinline__ float2 cis_rev(float x) {
  return make_float2(__builtin_amdgcn_cosf(x), __builtin_amdgcn_sinf(x));
}

// cos / sin of 2 pi m / 16 for m = 0..8 (exact decimal expansions)
__device__ __forceinline__ float cos16(int m) {
  switch (m) {
    case 0: return 1.0f;
    case 1: return 0.92387953251128675613f;
    case 2: return 0.70710678118654752440f;
    case 3: return 0.38268343236508977173f;
    case 4: return 0.0f;
    case 5: return -0.38268343236508977173f;
    case 6: return -0.70710678118654752440f;
    case 7: return -0.92387953251128675613f;
    default: return -1.0f;
  }
}
__device__ __forceinline__ float sin16(int m) { return cos16(m < 4 ? 4 - m : m - 4) * (m <= 8 ? 1.f : -1.f); }

// v * exp(DIR * 2 pi i m / 16), m compile-time after unrolling.
template <int DIR>
__device__ __forceinline__ float2 rot16(int m, float2 v) {
  if (m == 0) return v;
  if (m == 4) return DIR < 0 ? make_float2(v.y, -v.x) : make_float2(-v.y, v.x);
  const float c = cos16(m);
  const float s = DIR < 0 ? -sin16(m) : sin16(m);
  return make_float2(c * v.x - s * v.y, c * v.y + s * v.x);
}

// In-register DFT of length R (R = 1, 2, 4, 8, 16), natural order in and out,
// kernel exp(DIR * 2 pi i j k / R).  Radix-2 decimation in time.
template <int R, int DIR>
struct Dft {
  static __device__ __forceinline__ void run(float2* x) {
    float2 e[R / 2], o[R / 2];
#pragma unroll
    for (int i = 0; i < R / 2; ++i) {
      e[i] = x[2 * i];
      o[i] = x[2 * i + 1];
    }
    Dft<R / 2, DIR>::run(e);
    Dft<R / 2, DIR>::run(o);
#pragma unroll
    for (int k = 0; k < R / 2; ++k) {
      const float2 t = rot16<DIR>(k * (16 / R), o[k]);
      x[k] = cadd(e[k], t);
      x[k + R / 2] = csub(e[k], t);
    }
  }
};
template <int DIR>
struct Dft<2, DIR> {
  static __device__ __forceinline__ void run(float2* x) {
    const float2 a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};
template <int DIR>
struct Dft<1, DIR> {
  static __device__ __forceinline__ void run(float2*) {}
};

// LDS index with one pad slot per 16 complex elements: breaks the stride-16
// bank pattern of the first Stockham pass.
__host__ __device__ constexpr int pidx(int e) { return e + (e >> 4); }
__host__ __device__ constexpr int lds_elems(int n) { return n + (n >> 4) + 1; }

// Two-level twiddle table for length N = 2^LOGN, held in LDS:
// hi[i] = exp(-2 pi i 64 i / N) for i < HI, lo[j] = exp(-2 pi i j / N) for
// j < 64, so exp(-2 pi i m / N) = hi[m >> 6] * lo[m & 63] for every m < N
// (one complex product, about one float32 ulp).  Staging it costs SIZE
// entries instead of N and keeps twiddles out of global memory.
template <int LOGN>
struct Tw2 {
  static constexpr int N = 1 << LOGN;
  static constexpr int HI = N >= 64 ? N / 64 : 1;
  static constexpr int SIZE = HI + 64;
};

// Fill dst[0 .. Tw2::SIZE) from the global table tw[m] = exp(-2 pi i m / N).
template <int LOGN, int NT>
__device__ __forceinline__ void load_tw2(float2* __restrict__ dst, const float2* __restrict__ tw) {
  using T = Tw2<LOGN>;
  for (int e = threadIdx.x; e < T::SIZE; e += NT)
    dst[e] = e < T::HI ? tw[(e * 64) & (T::N - 1)] : tw[(e - T::HI) & (T::N - 1)];
}

template <int LOGN>
__device__ __forceinline__ float2 tw2_get(const float2* __restrict__ t, int m) {
  return cmul(t[m >> 6], t[Tw2<LOGN>::HI + (m & 63)]);
}

// No-op input / output / hook for the passes below.
struct NoIO {
  __device__ __forceinline__ float2 operator()(int, int) const { return czero(); }
  __device__ __forceinline__ void operator()(int, int, float2) const {}
  __device__ __forceinline__ void operator()() const {}
};

// One radix-R Stockham pass over C interleaved transforms of length N held in
// LDS (element t of transform c at pidx(t * C + c)), NT threads.  P is the
// product of the radices of the earlier passes.  tw is the LDS two-level
// twiddle table of length N (see Tw2).
//
// LOAD: the inputs come from ld(t, c) instead of LDS (first pass only, P = 1:
// the kernel's global load feeds the butterflies directly, and no barrier is
// needed before the LDS writes).  STORE: the outputs, in natural order at
// this point (last pass, P R = N), go to st(t, c, v) instead of LDS, and
// post() runs after them, before the closing barrier.
template <int LOGN, int C, int NT, int DIR, int R, int P, bool LOAD, bool STORE, class Ld, class St, class Post>
__device__ __forceinline__ void stockham_pass_io(float2* __restrict__ s, const float2* __restrict__ tw, int tid,
                                                 const Ld& ld, const St& st, const Post& post) {
  constexpr int N = 1 << LOGN;
  constexpr int NR = N / R;
  constexpr int NB = C * NR;
  constexpr int PER = (NB + NT - 1) / NT;
  constexpr int TWS = N / (P * R);
  static_assert(!LOAD || P == 1, "only the first pass reads from the loader");
  static_assert(!STORE || P * R == N, "only the last pass writes to the store");
  float2 x[PER][R];
  float2 w[PER][R];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int b = tid + q * NT;
    if (NB % NT == 0 || b < NB) {
      const int c = b % C, i = b / C;
      const int k = i & (P - 1);
      if constexpr (LOAD) {
#pragma unroll
        for (int j = 0; j < R; ++j) x[q][j] = ld(i + j * NR, c);
      } else if constexpr ((NR * C) % 16 == 0) {
        // inputs NR * C elements apart: one padded address and constant
        // offsets when the stride is a whole number of pad groups
        const int p0 = pidx(i * C + c);
#pragma unroll
        for (int j = 0; j < R; ++j) x[q][j] = s[p0 + j * pidx(NR * C)];
      } else {
#pragma unroll
        for (int j = 0; j < R; ++j) x[q][j] = s[pidx((i + j * NR) * C + c)];
      }
      if (P > 1) {
        // w^j, w = exp(-2 pi i k TWS / N): one table lookup, then a power
        // tree (each w^j a few products away from the table value)
        w[q][1] = tw2_get<LOGN>(tw, k * TWS);
#pragma unroll
        for (int j = 2; j < R; ++j) {
          const int hb = 1 << (31 - __builtin_clz(j));
          w[q][j] = hb == j ? cmul(w[q][j / 2], w[q][j / 2]) : cmul(w[q][hb], w[q][j - hb]);
        }
      }
    }
  }
  if constexpr (!LOAD) __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int b = tid + q * NT;
    if (NB % NT == 0 || b < NB) {
      const int c = b % C, i = b / C;
      const int k = i & (P - 1);
      if (P > 1) {
#pragma unroll
        for (int j = 1; j < R; ++j) {
          float2 t = w[q][j];
          if (DIR > 0) t.y = -t.y;
          x[q][j] = cmul(x[q][j], t);
        }
      }
      Dft<R, DIR>::run(x[q]);
      const int base = (i - k) * R + k;
      if constexpr (STORE) {
#pragma unroll
        for (int j = 0; j < R; ++j) st(base + j * P, c, x[q][j]);
      } else if constexpr ((P * C) % 16 == 0) {
        const int p0 = pidx(base * C + c);
#pragma unroll
        for (int j = 0; j < R; ++j) s[p0 + j * pidx(P * C)] = x[q][j];
      } else {
#pragma unroll
        for (int j = 0; j < R; ++j) s[pidx((base + j * P) * C + c)] = x[q][j];
      }
    }
  }
  if constexpr (STORE) post();
  __syncthreads();
}

template <int LOGN, int C, int NT, int DIR, int R, int P>
__device__ __forceinline__ void stockham_pass(float2* __restrict__ s, const float2* __restrict__ tw, int tid) {
  stockham_pass_io<LOGN, C, NT, DIR, R, P, false, false>(s, tw, tid, NoIO{}, NoIO{}, NoIO{});
}

// Radix-8 passes (a radix-4 or radix-2 tail) from P on, REM bits left; the
// first one may read from the loader and the last one write to the store.
template <int LOGN, int C, int NT, int DIR, int P, int REM, bool LOAD, bool STORE>
struct FftPassesIO {
  template <class Ld, class St, class Post>
  static __device__ __forceinline__ void run(float2* s, const float2* tw, int tid, const Ld& ld, const St& st,
                                             const Post& post) {
    constexpr int LR = REM >= 3 ? 3 : REM;
    constexpr int R = 1 << LR;
    constexpr bool LAST = REM == LR;
    stockham_pass_io<LOGN, C, NT, DIR, R, P, LOAD, STORE && LAST>(s, tw, tid, ld, st, post);
    FftPassesIO<LOGN, C, NT, DIR, P * R, REM - LR, false, STORE>::run(s, tw, tid, ld, st, post);
  }
};
template <int LOGN, int C, int NT, int DIR, int P, bool LOAD, bool STORE>
struct FftPassesIO<LOGN, C, NT, DIR, P, 0, LOAD, STORE> {
  template <class Ld, class St, class Post>
  static __device__ __forceinline__ void run(float2*, const float2*, int, const Ld&, const St&, const Post&) {}
};

template <int LOGN, int C, int NT, int DIR, int P, int REM>
struct FftPasses {
  static __device__ __forceinline__ void run(float2* s, const float2* tw, int tid) {
    FftPassesIO<LOGN, C, NT, DIR, P, REM, false, false>::run(s, tw, tid, NoIO{}, NoIO{}, NoIO{});
  }
};

// FFT of C interleaved transforms of length 2^LOGN whose first pass reads
// ld(t, c) (LOAD) and whose last pass hands the outputs, in natural order, to
// st(t, c, v) and then runs post() (STORE); the passes in between use LDS as
// fft_lds does.  Entered by all NT threads; with LOAD the twiddle table only
// has to be in LDS by the end of the first pass (which has no twiddles), so
// its staging needs no barrier of its own.  Ends with a barrier.
template <int LOGN, int C, int NT, int DIR, bool LOAD, bool STORE, class Ld, class St, class Post>
__device__ __forceinline__ void fft_io(float2* s, const float2* tw, int tid, const Ld& ld, const St& st,
                                       const Post& post) {
  FftPassesIO<LOGN, C, NT, DIR, 1, LOGN, LOAD, STORE>::run(s, tw, tid, ld, st, post);
}

// Unnormalised in-LDS FFT of C interleaved transforms of length 2^LOGN,
// kernel exp(DIR * 2 pi i t k / N).  tw is the LDS two-level twiddle table of
// that length.  Must be entered by all NT threads after the data and the
// table are in LDS and a barrier; ends with a barrier.
template <int LOGN, int C, int NT, int DIR>
__device__ __forceinline__ void fft_lds(float2* s, const float2* tw) {
  FftPasses<LOGN, C, NT, DIR, 1, LOGN>::run(s, tw, (int)threadIdx.x);
}

// The same transform with the thread index passed in.  A kernel that runs
// two transforms of one length passes an opaque copy (opaque_tid) to the
// second, so that the compiler recomputes its LDS addresses instead of
// keeping the first transform's live across the code in between.
template <int LOGN, int C, int NT, int DIR>
__device__ __forceinline__ void fft_lds(float2* s, const float2* tw, int tid) {
  FftPasses<LOGN, C, NT, DIR, 1, LOGN>::run(s, tw, tid);
}

__device__ __forceinline__ int opaque_tid() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// ------------------------------------------------- spreading kernel (ES)
// psi(d) = exp(beta (sqrt(1 - (2d/w)^2) - 1)) for |d| <= w/2, 0 outside
// (Barnett, Magland and af Klinteberg, SIAM J. Sci. Comput. 2019).
__device__ __forceinline__ float es_kernel(float d, float two_over_w, float beta) {
  const float t = d * two_over_w;
  const float r = 1.0f - t * t;
  return r > 0.0f ? expf(beta * (sqrtf(r) - 1.0f)) : 0.0f;
}

// es_kernel with the hardware exp2 and square root (v_exp_f32, v_sqrt_f32):
// absolute error below 3e-8 of the kernel's peak value 1.
__device__ __forceinline__ float es_kernel_fast(float d, float two_over_w, float beta_log2e) {
  const float t = d * two_over_w;
  const float r = 1.0f - t * t;
  return r > 0.0f ? __builtin_amdgcn_exp2f(beta_log2e * (__builtin_amdgcn_sqrtf(r) - 1.0f)) : 0.0f;
}

// Bin record: one (point, bin) pair.  lx, ly: first tap relative to the bin
// origin (int8 each), bit 16: the bin holds the point's first tap; dx, dy:
// offset of the first tap from the point in fine cells; idx: caller's point
// index.
struct __align__(16) BinRec {
  int32_t packed;
  float dx, dy;
  int32_t idx;
};

__device__ __forceinline__ int rec_lx(int32_t p) { return (int)(int8_t)(p & 0xff); }
__device__ __forceinline__ int rec_ly(int32_t p) { return (int)(int8_t)((p >> 8) & 0xff); }
__device__ __forceinline__ bool rec_primary(int32_t p) { return (p >> 16) & 1; }

// blockIdx -> work index such that consecutive work items land on the same
// XCD (the dispatcher deals workgroups round-robin over the 8 XCDs, each with
// its own L2).  `count` must be the grid size.
__device__ __forceinline__ int xcd_remap(int bid, int count) {
  constexpr int XCD = 8;
  const int per = count / XCD;
  if (per == 0 || bid >= per * XCD) return bid;
  return (bid % XCD) * per + bid / XCD;
}

}  // namespace nuasm
