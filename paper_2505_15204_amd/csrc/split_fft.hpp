// split_fft.hpp — the precision form of the inverse FFT: radix-16 stages as gfx950 matrix-core
// (MFMA) products in FP16 or BF16 with hi + lo split operands and FP32 accumulation.
//
// Same transform as fft_device.hpp (X[j] = sum_k x[k] exp(+2 pi i j k / N), Section 4, Eq. 5) and
// the same self-sorting radix-16 stage order, so the LDS layout between stages is unchanged.
// What differs is how one radix-16 butterfly is evaluated: the 16-point inverse DFT is the real
// 32 x 32 matrix M that maps interleaved (re, im) inputs to interleaved outputs,
//     M[2j][2q] = cos a,  M[2j][2q+1] = -sin a,  M[2j+1][2q] = sin a,  M[2j+1][2q+1] = cos a,
// a = 2 pi (j q mod 16) / 16, and 32 butterflies at a time form the 32 x 32 right-hand side of
// two v_mfma_f32_32x32x16 products (K = 16 reals each). Every FP32 operand x is split into
// hi = round(x) and lo = round(x - hi) in the 16-bit type (FP16 data: hi rounded toward zero,
// lo to nearest; otherwise both to nearest), and the product is
//     M x ~ M_lo x_hi + M_hi x_lo + M_hi x_hi        (the lo * lo term is dropped)
// accumulated in FP32: about 21 significant bits for FP16 (11 + 11), 16 for BF16 (8 + 8).
// Twiddle multiplications between stages, and a final radix-2/4/8 stage where N is not a power
// of 16, stay in FP32 on the vector ALUs. The reduced-precision study is left open by the paper
// (Section 10, future work); this is one design for it.
//
// FP16 range: the inputs of a task (the columns of a strip, or the row pairs of a row block; up
// to N = 1024 those of one wave, which holds whole transforms) are scaled by one power of two so
// that their largest real or imaginary part lies in [32, 64). A
// radix-16 stage with unit-modulus twiddles grows that bound by at most 16 sqrt(2) = 2^4.5, so
// the inputs of the third radix-16 stage stay below 2^15 and no 16-bit operand overflows; the
// outputs are multiplied back by the exact inverse power of two. BF16 has the FP32 exponent
// range and needs no scaling.
//
// Wave layout of the MFMA products (v_mfma_f32_32x32x16_{f16,bf16}, wave64): with n = lane % 32
// and g = lane / 32, lane (n, g) holds row n of A and column n of B for k = 8 g .. 8 g + 7, and
// rows 8 (v / 4) + 4 g + v % 4 (v < 16) of column n of the FP32 result. Butterfly 64 w + 32 h + n
// of a stage (wave w, batch h < 2) is column n of batch h; lane (n, g) loads its complex inputs
// 4 g .. 4 g + 3 and 8 + 4 g .. 8 + 4 g + 3 and receives its outputs 4 t' + 2 g + {0, 1}, t' < 4.
// A block of W waves covers 64 W butterflies per stage, one per thread as in the FP32 form;
// the block size must be a multiple of 64 because the matrix operand A is spread over the
// whole wave.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "fft_device.hpp"

namespace blink {

enum : int { kPrecFp32 = 0, kPrecSplitF16 = 1, kPrecSplitBf16 = 2 };

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int PREC>
struct Split;

template <>
struct Split<kPrecSplitF16> {
  using elem = _Float16;
  using vec = f16x8;
  static __device__ __forceinline__ f32x16 mma(vec a, vec b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

template <>
struct Split<kPrecSplitBf16> {
  using elem = __bf16;
  using vec = bf16x8;
  static __device__ __forceinline__ f32x16 mma(vec a, vec b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

// hi = x rounded to nearest even in the 16-bit type, lo = (x - hi) rounded the same way.
template <int PREC>
__device__ __forceinline__ void split_value(float x, typename Split<PREC>::elem& hi, typename Split<PREC>::elem& lo) {
  using E = typename Split<PREC>::elem;
  hi = (E)x;
  lo = (E)(x - (float)hi);
}

// The A operands (hi and lo, for K blocks 0 and 1) of one lane: row n of M, columns 16 kb + 8 g + e,
// from the 16-point DFT entries of a twiddle table (stage-ordered twiddle layout). They depend only on the lane,
// so they are computed once per context (make_dft_operands) into a table of 4 x 16 bytes per lane
// and precision: {hi kb 0, hi kb 1, lo kb 0, lo kb 1}.
template <int PREC>
struct DftOperands {
  typename Split<PREC>::vec hi[2], lo[2];
};

constexpr int kDftOpsPerPrec = 64 * 4;   // uint4 per precision

template <int PREC>
__device__ __forceinline__ DftOperands<PREC> dft16_operands_for_lane(const float2* __restrict__ tw, int lane) {
  DftOperands<PREC> F;
  const int n = lane & 31, g = lane >> 5;
  const int j = n >> 1, p = n & 1;
#pragma unroll
  for (int kb = 0; kb < 2; ++kb) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int q = 8 * kb + 4 * g + (e >> 1), r = e & 1;
      const float2 w = dft16_entry(tw, (j * q) & 15);
      const float f = (p == 0) ? (r == 0 ? w.x : -w.y) : (r == 0 ? w.y : w.x);
      typename Split<PREC>::elem h, l;
      split_value<PREC>(f, h, l);
      F.hi[kb][e] = h;
      F.lo[kb][e] = l;
    }
  }
  return F;
}

// Writes the operand table of one precision (64 lanes) from a twiddle table.
template <int PREC>
__device__ void make_dft_operands(const float2* __restrict__ tw, uint4* ops, int lane) {
  const DftOperands<PREC> F = dft16_operands_for_lane<PREC>(tw, lane);
  uint4* o = ops + (PREC - 1) * kDftOpsPerPrec + lane * 4;
  o[0] = __builtin_bit_cast(uint4, F.hi[0]);
  o[1] = __builtin_bit_cast(uint4, F.hi[1]);
  o[2] = __builtin_bit_cast(uint4, F.lo[0]);
  o[3] = __builtin_bit_cast(uint4, F.lo[1]);
}

// This lane's operands from the table (four 16-byte loads).
template <int PREC>
__device__ __forceinline__ DftOperands<PREC> dft16_operands(const uint4* __restrict__ ops) {
  const uint4* o = ops + (PREC - 1) * kDftOpsPerPrec + (threadIdx.x & 63) * 4;
  DftOperands<PREC> F;
  F.hi[0] = __builtin_bit_cast(typename Split<PREC>::vec, o[0]);
  F.hi[1] = __builtin_bit_cast(typename Split<PREC>::vec, o[1]);
  F.lo[0] = __builtin_bit_cast(typename Split<PREC>::vec, o[2]);
  F.lo[1] = __builtin_bit_cast(typename Split<PREC>::vec, o[3]);
  return F;
}

// What the split form needs besides the data: the workgroup's LDS word for the FP16 maximum and
// the context's DFT operand table (global memory).
struct SplitCtx {
  unsigned* s_max = nullptr;
  const uint4* ops = nullptr;
};

// FP16 split of one complex value: hi = (re, im) rounded toward zero to FP16 (one packed word),
// lo = the exact remainders x - hi rounded to nearest FP16, which the compiler forms with fused
// mixed-precision operations on the halves of hi. hi + lo carries about 21 bits of x. (Written
// without inline assembly so that the compiler sees every register the matrix core reads.)
__device__ __forceinline__ void split_f16_pair(float re, float im, uint32_t& hi, uint32_t& lo) {
  typedef __fp16 h2 __attribute__((ext_vector_type(2)));
  typedef _Float16 f2 __attribute__((ext_vector_type(2)));
  const h2 h = __builtin_amdgcn_cvt_pkrtz(re, im);
  const f2 hf = __builtin_bit_cast(f2, h);
  f2 l;
  l[0] = (_Float16)(re - (float)hf[0]);
  l[1] = (_Float16)(im - (float)hf[1]);
  hi = __builtin_bit_cast(uint32_t, h);
  lo = __builtin_bit_cast(uint32_t, l);
}

// One batch of 32 radix-16 butterflies: x[4 kb + i] is this lane's complex input 8 kb + 4 g + i.
// Returns the FP32 result; output t (< 8) of this lane is complex 4 (t / 2) + 2 g + t % 2,
// at (r[2 t], r[2 t + 1]).
template <int PREC>
__device__ __forceinline__ f32x16 dft16_mfma(const float2 (&x)[8], const DftOperands<PREC>& F) {
  using S = Split<PREC>;
  typename S::vec bhi[2], blo[2];
  if constexpr (PREC == kPrecSplitF16) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      u32x4 h, l;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        uint32_t hw, lw;
        split_f16_pair(x[4 * kb + i].x, x[4 * kb + i].y, hw, lw);
        h[i] = hw;
        l[i] = lw;
      }
      bhi[kb] = __builtin_bit_cast(typename S::vec, h);
      blo[kb] = __builtin_bit_cast(typename S::vec, l);
    }
  } else {
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        typename S::elem h, l;
        split_value<PREC>(x[4 * kb + i].x, h, l);
        bhi[kb][2 * i] = h;
        blo[kb][2 * i] = l;
        split_value<PREC>(x[4 * kb + i].y, h, l);
        bhi[kb][2 * i + 1] = h;
        blo[kb][2 * i + 1] = l;
      }
    }
  }
  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.f;
  // small terms first
#pragma unroll
  for (int kb = 0; kb < 2; ++kb) {
    acc = S::mma(F.lo[kb], bhi[kb], acc);
    acc = S::mma(F.hi[kb], blo[kb], acc);
  }
#pragma unroll
  for (int kb = 0; kb < 2; ++kb) acc = S::mma(F.hi[kb], bhi[kb], acc);
  return acc;
}

__device__ __forceinline__ int split_in_q(int g, int i) { return (i < 4) ? 4 * g + i : 8 + 4 * g + (i - 4); }
__device__ __forceinline__ int split_out_j(int g, int t) { return 4 * (t >> 1) + 2 * g + (t & 1); }

// Largest |re| or |im| over the block. *s_max must be 0 and visible to every thread on entry
// (set before an earlier barrier); it keeps the maximum afterwards. Contains a block barrier.
__device__ __forceinline__ float block_max_abs(float m, unsigned* s_max) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(s_max, __float_as_uint(m));
  __syncthreads();
  return __uint_as_float(*s_max);
}

// Largest |re| or |im| over the wave (no LDS word, no barrier): m >= 0, so its bits order as an
// unsigned integer. A DPP reduction leaves the row maxima in lanes 15, 31, 47, 63 (row_shr 1, 2,
// 4 and 8, the last two on the upper banks), then row_bcast 15 and 31 fold the rows into lane 63,
// which is read back as a scalar. Lanes whose DPP source is masked keep their own value.
__device__ __forceinline__ float wave_max_abs(float m) {
  int v = __float_as_int(m);
  auto step = [](int x, int y) { return (int)max((unsigned)x, (unsigned)y); };
  v = step(v, __builtin_amdgcn_update_dpp(v, v, 0x111, 0xf, 0xf, false));   // row_shr:1
  v = step(v, __builtin_amdgcn_update_dpp(v, v, 0x112, 0xf, 0xf, false));   // row_shr:2
  v = step(v, __builtin_amdgcn_update_dpp(v, v, 0x114, 0xf, 0xe, false));   // row_shr:4
  v = step(v, __builtin_amdgcn_update_dpp(v, v, 0x118, 0xf, 0xc, false));   // row_shr:8
  v = step(v, __builtin_amdgcn_update_dpp(v, v, 0x142, 0xa, 0xf, false));   // row_bcast:15
  v = step(v, __builtin_amdgcn_update_dpp(v, v, 0x143, 0xc, 0xf, false));   // row_bcast:31
  return __int_as_float(__builtin_amdgcn_readlane(v, 63));
}

// Power of two that brings a maximum magnitude mx into [32, 64).
__device__ __forceinline__ int f16_scale_exponent(float mx) {
  if (!(mx > 0.f) || !isfinite(mx)) return 0;
  int e;
  (void)frexpf(mx, &e);                 // mx = f 2^e, f in [0.5, 1)
  e = 6 - e;
  return e < -126 ? -126 : (e > 126 ? 126 : e);
}

// Complete inverse FFT of `ntrans` transforms of length N = 2^LOGN (LOGN >= 4) held by one block.
// Transform c lives at buf + c * NP (padded, natural order) between stages. The first stage's
// inputs come from buf (FromBuf) or from load(c, e); the outputs go to sink(c, e, value), or,
// with ToLds, back into buf at pad(e) with the block synchronised on return. Every thread of the block calls this; the
// block size is a multiple of 64 and at least ntrans * N / 16. `tw` is the twiddle table of N in
// the stage-ordered twiddle layout (visible to the block on entry); sp.s_max as for block_max_abs (FP16 only)
// and sp.ops the DFT operand table.
//
// Up to N = 1024 (N / 16 <= 64 butterflies per stage) every butterfly and every thread of the
// FP32 stage of transform c lies in wave 64 c / (N / 16): each wave owns whole transforms, so the
// stages exchange data through LDS within the wave only and are ordered by stage_sync's
// wavefront-scope fences instead of workgroup barriers, and the FP16 scale is taken per wave
// (every transform of a wave shares one power of two). Larger N spread a transform over several
// waves and use workgroup barriers.
template <int LOGN, int PREC, bool ToLds, bool FromBuf, class Load, class Sink>
__device__ __forceinline__ void fft_inverse_split(float2* buf, int ntrans, const float2* __restrict__ tw, Load load,
                                                  Sink sink, SplitCtx sp) {
  using P = FftPlan<LOGN>;
  static_assert(LOGN >= 4, "the split form needs at least one radix-16 stage");
  static_assert(PREC == kPrecSplitF16 || PREC == kPrecSplitBf16, "split precision");
  constexpr int N = P::N, T = P::T, NP = P::NP, NB = N / 16;
  const DftOperands<PREC> F = dft16_operands<PREC>(sp.ops);
  const int lane = threadIdx.x & 63, n = lane & 31, g = lane >> 5, w = threadIdx.x >> 6;
  const int total = ntrans * NB;
  constexpr bool WAVE_LOCAL = NB <= 64;   // T == NB: stage_sync<T> orders within the wave

  // The butterfly of batch h of this lane, and whether it exists. A lane without one gets
  // butterfly 0 (which always exists), so its loads need no branch (their values are discarded):
  // loads under a branch would each wait for their data before the next is issued.
  auto bfly = [&](int h, int& c, int& b) {
    const int beta = 64 * w + 32 * h + n;
    const bool exists = beta < total;
    const int bs = exists ? beta : 0;
    c = bs / NB;
    b = bs % NB;
    return exists;
  };
  // LDS address of input i of butterfly b of transform c (element b + q NB, q = split_in_q(g, i)):
  // one base plus a compile-time offset when NB is a multiple of 16.
  auto in_addr = [&](int c, int b, int i) {
    if constexpr (NB % 16 == 0) {
      const int qoff = i < 4 ? i : i + 4;
      return c * NP + pad_index(b) + pad_offset(4 * NB) * g + pad_offset(qoff * NB);
    } else {
      return c * NP + pad_index(b + split_in_q(g, i) * NB);
    }
  };
  // Emits the outputs of one MFMA stage with span NS; `last` stages go to the sink (or LDS).
  // Output t is element base + j NS with j = 2 g + jc(t), jc(t) = 4 (t / 2) + t % 2.
  auto emit = [&](const f32x16& r, int c, int b, bool act, auto ns_tag, auto last_tag, float u) {
    constexpr int NS = decltype(ns_tag)::value;
    constexpr bool LAST = decltype(last_tag)::value;
    static_assert(NS == 1 || NS % 16 == 0, "stage spans are 1, 16 or 256");
    if (!act) return;
    const int k = b & (NS - 1);
    const int base = (b - k) * 16 + k;
    const int abase = NS == 1 ? c * NP + 17 * b + 2 * g : c * NP + pad_index(base) + pad_offset(2 * NS) * g;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int jc = 4 * (t >> 1) + (t & 1);
      const int off = NS == 1 ? jc : pad_offset(jc * NS);
      float2 val = make_float2(r[2 * t], r[2 * t + 1]);
      if constexpr (LAST) {
        val = cscale(val, u);
        if constexpr (ToLds) buf[abase + off] = val;
        else sink(c, base + (2 * g + jc) * NS, val);
      } else {
        buf[abase + off] = val;
      }
    }
  };

  // ---- stage 0: radix 16, span 1, inputs from load()
  float2 x[2][8];
  bool act[2];
  int cc[2], bb[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    act[h] = bfly(h, cc[h], bb[h]);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      if constexpr (FromBuf) x[h][i] = buf[in_addr(cc[h], bb[h], i)];
      else x[h][i] = load(cc[h], bb[h] + split_in_q(g, i) * NB);
      if (!act[h]) x[h][i] = make_float2(0.f, 0.f);
    }
  }
  float u = 1.f;
  if constexpr (PREC == kPrecSplitF16) {
    float m = 0.f;
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int i = 0; i < 8; ++i) m = fmaxf(m, fmaxf(fabsf(x[h][i].x), fabsf(x[h][i].y)));
    int e;
    if constexpr (WAVE_LOCAL) {
      e = f16_scale_exponent(wave_max_abs(m));
      stage_sync<T>();                   // every load of buf is done before the in-place stores
    } else {
      e = f16_scale_exponent(block_max_abs(m, sp.s_max));   // also: every load of buf is done
    }
    const float s = ldexpf(1.f, e);
    u = ldexpf(1.f, -e);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int i = 0; i < 8; ++i) x[h][i] = cscale(x[h][i], s);
  } else {
    stage_sync<T>();                        // every load of buf is done before the in-place stores
  }
  using One = std::integral_constant<int, 1>;
  constexpr bool ONE_STAGE = (P::NST == 1);
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const f32x16 r = dft16_mfma<PREC>(x[h], F);
    emit(r, cc[h], bb[h], act[h], One{}, std::integral_constant<bool, ONE_STAGE>{}, u);
  }
  if constexpr (ONE_STAGE) {
    if constexpr (ToLds) __syncthreads();
    return;
  } else {
    stage_sync<T>();
    // ---- later stages
    auto mfma_stage = [&](auto ns_tag, auto last_tag) {
      constexpr int NS = decltype(ns_tag)::value;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        act[h] = bfly(h, cc[h], bb[h]);
        const int k = bb[h] & (NS - 1);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int q = split_in_q(g, i);
          float2 v = buf[in_addr(cc[h], bb[h], i)];
          if (!act[h]) v = make_float2(0.f, 0.f);
          x[h][i] = cmul(v, stage_twiddle<NS>(tw, k, q));
        }
      }
      stage_sync<T>();
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const f32x16 r = dft16_mfma<PREC>(x[h], F);
        emit(r, cc[h], bb[h], act[h], ns_tag, last_tag, u);
      }
    };
    auto valu_stage = [&](auto ns_tag, auto rad_tag) {
      // final small-radix stage in FP32, one thread per group of 16 elements as in fft_inverse
      constexpr int NS = decltype(ns_tag)::value, RAD = decltype(rad_tag)::value;
      const int c = threadIdx.x / T, lt = threadIdx.x % T;
      const bool active = c < ntrans;
      float2 v[16];
      if (active) {
        stage_load_lds<N, 16, T, RAD>(v, buf + c * NP, lt);
        stage_compute<N, 16, T, NS, RAD>(v, lt, tw);
      }
      if constexpr (ToLds) stage_sync<T>();
      if (active) {
        constexpr int Q = 16 / RAD;
#pragma unroll
        for (int qq = 0; qq < Q; ++qq)
#pragma unroll
          for (int m = 0; m < RAD; ++m) {
            const int e = stage_out_index<T, NS, RAD>(lt, qq, m);
            const float2 val = cscale(v[qq * RAD + m], u);
            if constexpr (ToLds) buf[c * NP + pad_index(e)] = val;
            else sink(c, e, val);
          }
      }
      if constexpr (ToLds) __syncthreads();
    };
    using B0 = std::integral_constant<bool, false>;
    using B1 = std::integral_constant<bool, true>;
    using S16 = std::integral_constant<int, 16>;
    if constexpr (P::NST == 2) {
      if constexpr (P::R1 == 16) {
        mfma_stage(S16{}, B1{});
        if constexpr (ToLds) __syncthreads();
      } else {
        valu_stage(S16{}, std::integral_constant<int, P::R1>{});
      }
    } else {
      mfma_stage(S16{}, B0{});
      stage_sync<T>();
      using S256 = std::integral_constant<int, 256>;
      if constexpr (P::R2 == 16) {
        mfma_stage(S256{}, B1{});
        if constexpr (ToLds) __syncthreads();
      } else {
        valu_stage(S256{}, std::integral_constant<int, P::R2>{});
      }
    }
  }
}

}  // namespace blink
