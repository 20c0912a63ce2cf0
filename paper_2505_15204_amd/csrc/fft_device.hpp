// fft_device.hpp — FP32 complex inverse FFT building blocks for gfx950 (wave64, LDS).
//
// The inverse transform of Section 4 (Eq. 5) with the + sign that Eq. 4's exp(-i2pi(ul+vm))
// implies: X[j] = sum_k x[k] exp(+2 pi i j k / N), unnormalised.
//
// Formulation: self-sorting (Stockham) decimation in time with radix-16 stages and one
// smaller final radix (2, 4 or 8). A transform of length N is done by T = N/16 threads; each
// thread holds 16 values in registers, so the butterflies run in VGPRs and every stage costs
// one pass through LDS. Stage s with radix r and span Ns (product of earlier radices) reads
// element b + m*N/r (b = butterfly, m < r), multiplies by w^(k m) with w = exp(2 pi i/(Ns r)),
// k = b mod Ns, does an r-point DFT and writes element (b - k) r + k + m Ns. The output is in
// natural order. Twiddles are FP32 values rounded from FP64 ones, stored per stage (the
// twiddle table layout below) so that the lanes of a wave, which differ in k, read different
// LDS banks.
//
// LDS layout of one transform: element e lives at pad(e) = e + e/16, so the stride-16 writes
// of the first stage spread over the banks; a transform occupies padded_len(N) float2.
#pragma once

#include <hip/hip_runtime.h>

namespace blink {

// ---------------------------------------------------------------- complex helpers
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 mul_i(float2 a) { return make_float2(-a.y, a.x); }   // i a
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

__host__ __device__ constexpr int pad_index(int e) { return e + (e >> 4); }
// Column stride in float2: the padded length plus one so that neighbouring columns start on
// different banks (the transposing store reads one element from each of S columns).
__host__ __device__ constexpr int padded_len(int n) { return n + (n >> 4) + 1; }

// ---------------------------------------------------------------- small inverse DFTs
__device__ __forceinline__ void dft2(float2* v) {
  float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

__device__ __forceinline__ void dft4(float2* v) {
  float2 a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
  float2 b0 = cadd(v[1], v[3]), b1 = mul_i(csub(v[1], v[3]));
  v[0] = cadd(a0, b0);
  v[2] = csub(a0, b0);
  v[1] = cadd(a1, b1);
  v[3] = csub(a1, b1);
}

// exp(+2 pi i e / 16) constants
#define BLINK_C16 0.92387953251128674f   // cos(pi/8)
#define BLINK_S16 0.38268343236508977f   // sin(pi/8)
#define BLINK_R2 0.70710678118654752f    // sqrt(1/2)

__device__ __forceinline__ void dft8(float2* v) {
  float2 e[4] = {v[0], v[2], v[4], v[6]};
  float2 o[4] = {v[1], v[3], v[5], v[7]};
  dft4(e);
  dft4(o);
  o[1] = make_float2(BLINK_R2 * (o[1].x - o[1].y), BLINK_R2 * (o[1].x + o[1].y));    // * e^{i pi/4}
  o[2] = mul_i(o[2]);                                                               // * e^{i pi/2}
  o[3] = make_float2(-BLINK_R2 * (o[3].x + o[3].y), BLINK_R2 * (o[3].x - o[3].y));   // * e^{i 3pi/4}
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = cadd(e[k], o[k]);
    v[k + 4] = csub(e[k], o[k]);
  }
}

// 16 = 4 x 4: inner DFT4 over n1 of x[4 n1 + n2], twiddle w16^(n2 k1), outer DFT4 over n2.
__device__ __forceinline__ void dft16(float2* v) {
  float2 a[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    a[n2][0] = v[n2];
    a[n2][1] = v[n2 + 4];
    a[n2][2] = v[n2 + 8];
    a[n2][3] = v[n2 + 12];
    dft4(a[n2]);
  }
  const float2 w1 = make_float2(BLINK_C16, BLINK_S16);
  const float2 w2 = make_float2(BLINK_R2, BLINK_R2);
  const float2 w3 = make_float2(BLINK_S16, BLINK_C16);
  const float2 w6 = make_float2(-BLINK_R2, BLINK_R2);
  const float2 w9 = make_float2(-BLINK_C16, -BLINK_S16);
  a[1][1] = cmul(a[1][1], w1);
  a[1][2] = cmul(a[1][2], w2);
  a[1][3] = cmul(a[1][3], w3);
  a[2][1] = cmul(a[2][1], w2);
  a[2][2] = mul_i(a[2][2]);
  a[2][3] = cmul(a[2][3], w6);
  a[3][1] = cmul(a[3][1], w3);
  a[3][2] = cmul(a[3][2], w6);
  a[3][3] = cmul(a[3][3], w9);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
    dft4(b);
    v[k1] = b[0];
    v[k1 + 4] = b[1];
    v[k1 + 8] = b[2];
    v[k1 + 12] = b[3];
  }
}

template <int RAD>
__device__ __forceinline__ void dft(float2* v) {
  if constexpr (RAD == 2) dft2(v);
  else if constexpr (RAD == 4) dft4(v);
  else if constexpr (RAD == 8) dft8(v);
  else if constexpr (RAD == 16) dft16(v);
  else static_assert(RAD == 2 || RAD == 4 || RAD == 8 || RAD == 16, "unsupported radix");
}

// ---------------------------------------------------------------- twiddle table layout
// Twiddle table of one size N, by stage (generated in FP64 and rounded to FP32 on the device):
//   A[16 m + k]      = exp(+2 pi i k m / (16 R1)),  k < 16, m < R1   second stage (span 16)
//   D[t]             = exp(+2 pi i t / 16),         t < 16           16-point DFT entries
//   B[256 m + k]     = exp(+2 pi i k m / N),        k < 256, m < R2  third stage (span 256), N >= 512
// with D = A + 256 and B = A + 272. For one m the lanes of a wave read consecutive k: distinct
// LDS banks, and one cache line per 16 values when the table is read from global memory.
constexpr int kTwA = 16 * 16 + 16;
__host__ __device__ constexpr int tw_size(int logn) { return kTwA + (logn >= 9 ? (1 << logn) : 0); }

template <int NS>
__device__ __forceinline__ float2 stage_twiddle(const float2* __restrict__ tw, int k, int m) {
  static_assert(NS == 16 || NS == 256, "twiddled stages have span 16 or 256");
  if constexpr (NS == 16) return tw[m * 16 + k];
  else return tw[kTwA + m * 256 + k];
}
__device__ __forceinline__ float2 dft16_entry(const float2* __restrict__ tw, int t) { return tw[256 + t]; }

// ---------------------------------------------------------------- plan
template <int LOGN>
struct FftPlan {
  static_assert(LOGN >= 3 && LOGN <= 12, "grid sizes 8 .. 4096");
  static constexpr int N = 1 << LOGN;
  static constexpr int R = (LOGN >= 4) ? 16 : N;                 // values per thread
  static constexpr int T = N / R;                                // threads per transform
  static constexpr int NST = (LOGN <= 4) ? 1 : (LOGN <= 8 ? 2 : 3);
  static constexpr int R0 = R;
  static constexpr int R1 = (NST >= 2) ? (LOGN >= 8 ? 16 : N / 16) : 1;
  static constexpr int R2 = (NST >= 3) ? N / 256 : 1;
  static constexpr int NP = padded_len(N);
};

// One stage's twiddles and butterflies on the registers of one thread.
// Slot q*RAD + m holds element (tid + q*T) + m*N/RAD.
template <int N, int R, int T, int NS, int RAD>
__device__ __forceinline__ void stage_compute(float2 (&v)[R], int tid, const float2* __restrict__ tw) {
  constexpr int Q = R / RAD;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    if constexpr (NS > 1) {
      const int b = tid + q * T;
      const int k = b & (NS - 1);
#pragma unroll
      for (int m = 1; m < RAD; ++m) v[q * RAD + m] = cmul(v[q * RAD + m], stage_twiddle<NS>(tw, k, m));
    }
    dft<RAD>(&v[q * RAD]);
  }
}

template <int T, int NS, int RAD>
__device__ __forceinline__ int stage_out_index(int tid, int q, int m) {
  const int b = tid + q * T;
  const int k = b & (NS - 1);
  return (b - k) * RAD + k + m * NS;
}

// pad(e + c) = pad(e) + c + c/16 whenever c is a multiple of 16, so the addresses of one
// thread's loads and stores are one computed base plus compile-time offsets where the strides
// allow it.
__host__ __device__ constexpr int pad_offset(int c) { return c + c / 16; }

template <int N, int R, int T, int NS, int RAD>
__device__ __forceinline__ void stage_store_lds(const float2 (&v)[R], float2* buf, int tid) {
  constexpr int Q = R / RAD;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int b = tid + q * T;
    const int k = b & (NS - 1);
    const int base = (b - k) * RAD + k;
    if constexpr (NS % 16 == 0) {
      const int pb = pad_index(base);
#pragma unroll
      for (int m = 0; m < RAD; ++m) buf[pb + pad_offset(m * NS)] = v[q * RAD + m];
    } else if constexpr (NS == 1 && RAD == 16) {
      const int pb = 17 * b;                         // pad(16 b + m) = 17 b + m for m < 16
#pragma unroll
      for (int m = 0; m < RAD; ++m) buf[pb + m] = v[q * RAD + m];
    } else {
#pragma unroll
      for (int m = 0; m < RAD; ++m) buf[pad_index(base + m * NS)] = v[q * RAD + m];
    }
  }
}

template <int N, int R, int T, int RAD>
__device__ __forceinline__ void stage_load_lds(float2 (&v)[R], const float2* buf, int tid) {
  constexpr int Q = R / RAD;
  constexpr int STEP = N / RAD;
  if constexpr (STEP % 16 == 0 && T % 16 == 0) {
    const int pb = pad_index(tid);
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int m = 0; m < RAD; ++m) v[q * RAD + m] = buf[pb + pad_offset(q * T + m * STEP)];
  } else {
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int m = 0; m < RAD; ++m) v[q * RAD + m] = buf[pad_index(tid + q * T + m * STEP)];
  }
}

// Synchronisation between two LDS passes of the transforms. When the T threads of a transform
// lie within one wavefront (T <= 64 with transforms at multiples of T), only that wavefront reads
// what it wrote: the LDS unit performs one wavefront's instructions in issue order, so fences at
// wavefront scope (which keep the compiler from moving memory operations across) replace the
// workgroup barrier, and the wavefronts of a workgroup are free to run their LDS passes and
// butterflies out of step. Larger transforms span wavefronts and take the workgroup barrier.
template <int T>
__device__ __forceinline__ void stage_sync() {
  if constexpr (T <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Full inverse FFT of one transform per group of T threads.
// On entry v[m] holds element tid + m*T (the first stage's input order); `buf` is this
// transform's padded LDS buffer and `tw` the twiddle table of N in the layout above (LDS or
// global). Every thread of the block must call this (it contains block barriers); threads with
// active == false take part in the barriers only and touch no memory. The passes between stages
// are separated by stage_sync, so the caller's last LDS writes before the call must already be
// visible to the transform's threads, and the caller separates a later reuse of buf by other
// threads with a barrier of its own. On return the caller's `sink(e, value)` has been called for
// every output element e this thread owns (natural order, each element exactly once across the T
// threads); when the last stage writes back to LDS instead (ToLds = true) the result is in buf at
// pad(e) and the block is synchronised.
template <int LOGN, bool ToLds, class Sink>
__device__ __forceinline__ void fft_inverse(float2 (&v)[FftPlan<LOGN>::R], float2* buf,
                                            const float2* __restrict__ tw, int tid, Sink sink,
                                            bool active = true) {
  using P = FftPlan<LOGN>;
  constexpr int N = P::N, R = P::R, T = P::T;
  if (active) stage_compute<N, R, T, 1, P::R0>(v, tid, tw);
  if constexpr (P::NST == 1) {
    if constexpr (ToLds) {
      stage_sync<T>();
      if (active) stage_store_lds<N, R, T, 1, P::R0>(v, buf, tid);
      __syncthreads();
    } else {
      if (active) {
#pragma unroll
        for (int m = 0; m < P::R0; ++m) sink(stage_out_index<T, 1, P::R0>(tid, 0, m), v[m]);
      }
    }
  } else {
    stage_sync<T>();                       // the caller's loads of buf are complete
    if (active) stage_store_lds<N, R, T, 1, P::R0>(v, buf, tid);
    stage_sync<T>();
    if (active) {
      stage_load_lds<N, R, T, P::R1>(v, buf, tid);
      stage_compute<N, R, T, P::R0, P::R1>(v, tid, tw);
    }
    constexpr int Q1 = R / P::R1;
    if constexpr (P::NST == 2) {
      if constexpr (ToLds) {
        stage_sync<T>();
        if (active) stage_store_lds<N, R, T, P::R0, P::R1>(v, buf, tid);
        __syncthreads();
      } else {
        if (active) {
#pragma unroll
          for (int q = 0; q < Q1; ++q)
#pragma unroll
            for (int m = 0; m < P::R1; ++m) sink(stage_out_index<T, P::R0, P::R1>(tid, q, m), v[q * P::R1 + m]);
        }
      }
    } else {
      stage_sync<T>();
      if (active) stage_store_lds<N, R, T, P::R0, P::R1>(v, buf, tid);
      stage_sync<T>();
      constexpr int NS2 = P::R0 * P::R1;
      if (active) {
        stage_load_lds<N, R, T, P::R2>(v, buf, tid);
        stage_compute<N, R, T, NS2, P::R2>(v, tid, tw);
      }
      constexpr int Q2 = R / P::R2;
      if constexpr (ToLds) {
        stage_sync<T>();
        if (active) stage_store_lds<N, R, T, NS2, P::R2>(v, buf, tid);
        __syncthreads();
      } else {
        if (active) {
#pragma unroll
          for (int q = 0; q < Q2; ++q)
#pragma unroll
            for (int m = 0; m < P::R2; ++m) sink(stage_out_index<T, NS2, P::R2>(tid, q, m), v[q * P::R2 + m]);
        }
      }
    }
  }
}

}  // namespace blink
