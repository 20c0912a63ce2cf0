// kernels.hpp — the FFT kernels of the batched path as templates over the precision form, and
// their variant dispatch. kernels.hip instantiates the FP32 form; split.hip is compiled once per
// split precision (FP16, BF16) and instantiates that one, so the three build in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include "conv_device.hpp"
#include "imaging_device.hpp"
#include "launch.hpp"

namespace blink {

// ---------------------------------------------------------------- configuration
// Largest strip width (columns per workgroup) of the fused column kernel that fits 1024 threads
// and the 160 KB of LDS (strip buffer, twiddle table, strip offsets and, for uniform weighting,
// counts).
template <int LOGN, bool UNIFORM>
struct ColSmax {
  using P = FftPlan<LOGN>;
  static constexpr int N = P::N;
  static constexpr int per_col = P::NP * 8 + (UNIFORM ? N * 4 : 0);
  static constexpr int avail = kLdsBytes - tw_size(LOGN) * 8 - (N / 2 + 1) * 4 - 1024;
  static constexpr int value = pow2_floor(cmin(cmin(N / 2, 1024 / P::T), avail / per_col));
};

// Tunable variants are compiled for N >= 256: strip widths Smax, Smax/2, Smax/4 and 1, 2, 4, 8
// row-pair transforms per workgroup. Smaller grids get one variant each.
constexpr int kTunedLogn = 8;

template <int LOGN>
struct GridCfg {
  static constexpr int N = 1 << LOGN;
  static constexpr int S = pow2_floor(cmin(N, (128 * 1024) / (N * 12)));
  static constexpr int THREADS = 256;
};

// A row variant fits when TPB transforms of N padded points plus the twiddle table fit in LDS.
template <int LOGN, int TPB>
struct RowFits {
  static constexpr bool value = TPB >= 1 && TPB * FftPlan<LOGN>::T <= 1024 && TPB <= (1 << LOGN) / 2 &&
                                TPB * FftPlan<LOGN>::NP * 8 + tw_size(LOGN) * 8 <= kLdsBytes;
};

template <int LOGN>
struct RowDefault {
  using P = FftPlan<LOGN>;
  static constexpr int value = cmin(P::N / 2, (256 / P::T) > 0 ? 256 / P::T : 1);
};

// Workgroup size for `work` FFT threads: exact for FP32, whole waves for the split forms.
__host__ __device__ constexpr int fft_block(int work, int prec) {
  return prec == kPrecFp32 ? work : ((work + 63) / 64) * 64;
}

// ---------------------------------------------------------------- fused grid + column FFT
template <int LOGN, int S, bool UNIFORM, int PREC>
__global__ __launch_bounds__(fft_block(S * FftPlan<LOGN>::T, PREC)) void k_grid_colfft(ColArgs a,
                                                                                        const float2* __restrict__ twg) {
  using P = FftPlan<LOGN>;
  constexpr int N = P::N, NP = P::NP;
  constexpr int NT = fft_block(S * FftPlan<LOGN>::T, PREC), TW = tw_size(LOGN);
  __shared__ float2 sbuf[S * NP];
  __shared__ float2 stw[TW];
  __shared__ unsigned scnt[UNIFORM ? S * N : 1];
  __shared__ int s_off[(N / 2) / S + 1];
  __shared__ int s_tmp;
  __shared__ unsigned s_max;
  // blockIdx.x = slot of the image in this launch's group; the image is img0 + slot in the chunk.
  // The workgroup takes the strips blockIdx.y, blockIdx.y + gridDim.y, ... of that image.
  const int slot = blockIdx.x, img = a.img0 + slot;
  const int tcl = img / a.P;
  const int nstrips = (N / 2) / S;
  // Strips at or beyond the column extent hold no placement: their columns of H are zero, and the
  // row pass reads them as zero without loading them, so they are neither transformed nor stored.
  const int live = a.ext ? a.ext[tcl] / S : nstrips;
  if ((int)blockIdx.y >= live) return;   // uniform over the workgroup
  for (int i = threadIdx.x; i < TW; i += NT) stw[i] = twg[i];   // visible after the task's first barrier
  const int* so = a.strip_off + (size_t)tcl * (nstrips + 1);
  for (int i = threadIdx.x; i <= nstrips; i += NT) s_off[i] = so[i];   // visible after the task's first barrier
  grid_colfft_strips<LOGN, S, UNIFORM, PREC, NT, kColPrefetch>(
      a.vis + (size_t)img * a.B, a.plc + (size_t)tcl * 2 * a.B, s_off, blockIdx.y, gridDim.y, live,
      a.B > 0 ? live : 0, a.shift != 0,
      a.H + (size_t)slot * N * (N / 2), a.occ + img, stw, sbuf, scnt, &s_tmp, SplitCtx{&s_max, a.dft_ops});
}

// ---------------------------------------------------------------- fused conv gridding + column FFT
template <int LOGN, int S, int PREC>
__global__ __launch_bounds__(fft_block(S * FftPlan<LOGN>::T, PREC)) void k_grid_colfft_conv(
    ColArgs a, ConvSpec cs, const float2* __restrict__ twg) {
  using P = FftPlan<LOGN>;
  constexpr int N = P::N, NP = P::NP;
  constexpr int NT = fft_block(S * FftPlan<LOGN>::T, PREC), TW = tw_size(LOGN);
  constexpr int NB = N >> conv_log_band(LOGN);   // row bands per column
  __shared__ float2 sbuf[S * NP];
  __shared__ float2 stw[TW];
  __shared__ int s_boff[NB + 2];
  __shared__ unsigned s_max;
  const int slot = blockIdx.x, img = a.img0 + slot, strip = blockIdx.y;
  const int tcl = img / a.P;
  const int nstrips = (N / 2) / S;
  // strips past the column extent receive no tap; the row pass reads their columns as zero
  if (a.ext && strip >= a.ext[tcl] / S) return;   // uniform over the workgroup
  for (int i = threadIdx.x; i < TW; i += NT) stw[i] = twg[i];   // visible after the task's first barrier
  const int* so = a.strip_off + (size_t)tcl * (nstrips * NB + 1) + (size_t)strip * NB;
  const ConvRec* rec = reinterpret_cast<const ConvRec*>(a.plc) + (size_t)tcl * a.rec_stride;
  grid_colfft_conv_task<LOGN, S, PREC, NT>(a.vis + (size_t)img * a.B, rec, so, s_boff, strip, a.shift != 0,
                                           cs, a.H + (size_t)slot * N * (N / 2), stw, sbuf,
                                           SplitCtx{&s_max, a.dft_ops});
}

// ---------------------------------------------------------------- dense grid column FFT
template <int LOGN, int PREC>
__global__ __launch_bounds__(fft_block(ColSmax<LOGN, false>::value * FftPlan<LOGN>::T, PREC)) void k_dense_colfft(
    const float2* __restrict__ grids, int shift, float2* __restrict__ H, const float2* __restrict__ twg,
    const uint4* __restrict__ ops) {
  using P = FftPlan<LOGN>;
  constexpr int N = P::N, T = P::T, S = ColSmax<LOGN, false>::value, NP = P::NP, mask = N - 1;
  constexpr int TW = tw_size(LOGN);
  constexpr bool SPLIT = PREC != kPrecFp32 && LOGN >= 4;
  __shared__ float2 sbuf[S * NP];
  __shared__ float2 stw[TW];
  __shared__ unsigned s_max;
  const int img = blockIdx.x, strip = blockIdx.y;
  const float2* G = grids + (size_t)img * N * N;
  for (int i = threadIdx.x; i < TW; i += blockDim.x) stw[i] = twg[i];
  if (threadIdx.x == 0) s_max = 0u;
  // Hermitian part Gh[kv][ku] = (G[kv][ku] + conj G[-kv][-ku]) / 2; column 0 packs
  // Gh[.][0] + i Gh[.][N/2], whose transforms are both real.
  for (int i = threadIdx.x; i < S * N; i += blockDim.x) {
    const int kv = i / S, c = i % S, ku = strip * S + c;
    const int mkv = (N - kv) & mask;
    const float2 g1 = G[(size_t)kv * N + ku];
    const float2 g2 = G[(size_t)mkv * N + ((N - ku) & mask)];
    float2 h = make_float2(0.5f * (g1.x + g2.x), 0.5f * (g1.y - g2.y));
    if (ku == 0) {
      const float2 n1 = G[(size_t)kv * N + N / 2];
      const float2 n2 = G[(size_t)mkv * N + N / 2];
      const float2 hn = make_float2(0.5f * (n1.x + n2.x), 0.5f * (n1.y - n2.y));
      h = make_float2(h.x - hn.y, h.y + hn.x);
    }
    if (shift && ((kv + ku) & 1)) {
      h.x = -h.x;
      h.y = -h.y;
    }
    sbuf[c * NP + pad_index(kv)] = h;
  }
  __syncthreads();
  if constexpr (SPLIT) {
    fft_inverse_split<LOGN, PREC, true, true>(
        sbuf, S, stw, [&](int c, int e) { return sbuf[c * NP + pad_index(e)]; }, [](int, int, float2) {},
        SplitCtx{&s_max, ops});
  } else {
    const bool active = (int)threadIdx.x < S * T;
    const int col = active ? (int)threadIdx.x / T : 0, lt = (int)threadIdx.x % T;
    float2* cb = sbuf + col * NP;
    float2 v[P::R];
    if (active) stage_load_lds<N, P::R, T, P::R0>(v, cb, lt);
    fft_inverse<LOGN, true>(v, cb, stw, lt, [](int, float2) {}, active);
  }
  float2* Hi = H + (size_t)img * N * (N / 2);
  for (int i = threadIdx.x; i < S * N; i += blockDim.x) {
    const int y = i / S, c = i % S;
    Hi[(size_t)y * (N / 2) + strip * S + c] = sbuf[c * NP + pad_index(y)];
  }
}

// ---------------------------------------------------------------- row pass
// Transform j of block (img, blk) handles rows y1 = 2 r, y2 = 2 r + 1 (r = blk*TPB + j).
// Z[e] = Hf1[e] + i Hf2[e] where Hf is the Hermitian extension of the stored half row:
// Hf[0] = Re H[0], Hf[N/2] = Im H[0], Hf[e] = H[e] (0 < e < N/2), Hf[e] = conj H[N-e].
// The inverse FFT of Z is I1 + i I2 with both rows real.
__device__ __forceinline__ double image_weight(const RowArgs& a, int img) {
  if (a.wmode == kWeightUser) return a.w_user ? a.w_user[img] : 1.0;
  if (a.wmode == kWeightNatural) return 2.0 * (double)a.n_kept[img / a.P];
  return (double)a.occ[img];
}

template <int LOGN, int TPB, int PREC>
__global__ __launch_bounds__(fft_block(TPB * FftPlan<LOGN>::T, PREC)) void k_row_c2r(RowArgs a,
                                                                                      const float2* __restrict__ twg) {
  using P = FftPlan<LOGN>;
  constexpr int N = P::N, NP = P::NP;
  // Every form reads its twiddles from the global table (cached in L1): without a copy in LDS a
  // workgroup of a few transforms leaves room for many workgroups per compute unit (the split
  // forms, with their LDS copy, took 3.9 ms per 1536 images at 1024^2; 3.7 ms without).
  __shared__ float2 sbuf[TPB * NP];
  __shared__ unsigned s_max;
  const int slot = blockIdx.x, img = a.img0 + slot;
  const float2* stw = twg;
  const double W = image_weight(a, img);
  if (a.weight_sum && blockIdx.y == 0 && threadIdx.x == 0) a.weight_sum[img] = W;
  const int ext = a.ext ? a.ext[img / a.P] : N / 2;
  row_task<LOGN, TPB, PREC>(a.H + (size_t)slot * N * (N / 2), blockIdx.y, inverse_weight(W),
                            a.images + (size_t)slot * N * N, stw, sbuf, SplitCtx{&s_max, a.dft_ops}, a.corr, ext);
}

// ---------------------------------------------------------------- dispatch
template <template <int> class F, class... Args>
static hipError_t by_logn(int logn, Args... args) {
  switch (logn) {
    case 3: return F<3>::run(args...);
    case 4: return F<4>::run(args...);
    case 5: return F<5>::run(args...);
    case 6: return F<6>::run(args...);
    case 7: return F<7>::run(args...);
    case 8: return F<8>::run(args...);
    case 9: return F<9>::run(args...);
    case 10: return F<10>::run(args...);
    case 11: return F<11>::run(args...);
    case 12: return F<12>::run(args...);
    default: return hipErrorInvalidValue;
  }
}

template <int PREC>
struct ForPrec {
  template <int LOGN, int S, bool U>
  static hipError_t col_one(const ColArgs* a, int n_img, const float2* tw, hipStream_t s) {
    if constexpr (S >= 1) {
      const int nstrips = ((1 << LOGN) / 2) / S, loop = a->col_loop > 1 ? a->col_loop : 1;
      dim3 grid(n_img, (nstrips + loop - 1) / loop);
      k_grid_colfft<LOGN, S, U, PREC><<<grid, fft_block(S * FftPlan<LOGN>::T, PREC), 0, s>>>(*a, tw);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }

  template <int LOGN, bool U>
  static hipError_t col_variant(const ColArgs* a, int n_img, int S, const float2* tw, hipStream_t s) {
    constexpr int SM = ColSmax<LOGN, U>::value;
    if (S == SM) return col_one<LOGN, SM, U>(a, n_img, tw, s);
    if constexpr (LOGN >= kTunedLogn) {
      if (S == SM / 2) return col_one<LOGN, SM / 2, U>(a, n_img, tw, s);
      if (S == SM / 4) return col_one<LOGN, SM / 4, U>(a, n_img, tw, s);
    }
    return hipErrorInvalidValue;
  }

  template <int LOGN>
  struct ColL {
    static hipError_t run(const ColArgs* a, int n_img, int S, const float2* tw, hipStream_t s) {
      return a->uniform ? col_variant<LOGN, true>(a, n_img, S, tw, s) : col_variant<LOGN, false>(a, n_img, S, tw, s);
    }
  };

  template <int LOGN>
  struct ConvL {
    static hipError_t run(const ColArgs* a, int n_img, ConvSpec cs, const float2* tw, hipStream_t s) {
      constexpr int S = ColSmax<LOGN, false>::value;
      dim3 grid(n_img, ((1 << LOGN) / 2) / S);
      k_grid_colfft_conv<LOGN, S, PREC><<<grid, fft_block(S * FftPlan<LOGN>::T, PREC), 0, s>>>(*a, cs, tw);
      return hipGetLastError();
    }
  };

  template <int LOGN>
  struct DenseL {
    static hipError_t run(const float2* g, int n_img, int shift, float2* H, const float2* tw, const uint4* ops,
                          hipStream_t s) {
      constexpr int N = 1 << LOGN;
      constexpr int S = ColSmax<LOGN, false>::value;
      dim3 grid(n_img, (N / 2) / S);
      k_dense_colfft<LOGN, PREC><<<grid, fft_block(S * FftPlan<LOGN>::T, PREC), 0, s>>>(g, shift, H, tw, ops);
      return hipGetLastError();
    }
  };

  template <int LOGN, int TPB>
  static hipError_t row_one(const RowArgs* a, int n_img, const float2* tw, hipStream_t s) {
    if constexpr (RowFits<LOGN, TPB>::value) {
      dim3 grid(n_img, ((1 << LOGN) / 2) / TPB);
      k_row_c2r<LOGN, TPB, PREC><<<grid, fft_block(TPB * FftPlan<LOGN>::T, PREC), 0, s>>>(*a, tw);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }

  template <int LOGN>
  struct RowL {
    static hipError_t run(const RowArgs* a, int n_img, int tpb, const float2* tw, hipStream_t s) {
      if constexpr (LOGN >= kTunedLogn) {
        switch (tpb) {
          case 1: return row_one<LOGN, 1>(a, n_img, tw, s);
          case 2: return row_one<LOGN, 2>(a, n_img, tw, s);
          case 4: return row_one<LOGN, 4>(a, n_img, tw, s);
          case 8: return row_one<LOGN, 8>(a, n_img, tw, s);
          default: return hipErrorInvalidValue;
        }
      } else {
        if (tpb != RowDefault<LOGN>::value) return hipErrorInvalidValue;
        return row_one<LOGN, RowDefault<LOGN>::value>(a, n_img, tw, s);
      }
    }
  };

  static hipError_t grid_colfft(const ColArgs& a, int n_img, int strip, const float2* tw, hipStream_t s) {
    if (n_img <= 0) return hipSuccess;
    return by_logn<ColL>(a.logn, &a, n_img, strip, tw, s);
  }
  static hipError_t dense_colfft(const float2* grids, int n_img, int logn, int shift, float2* H, const float2* tw,
                                 const uint4* ops, hipStream_t s) {
    if (n_img <= 0) return hipSuccess;
    return by_logn<DenseL>(logn, grids, n_img, shift, H, tw, ops, s);
  }
  static hipError_t row_c2r(const RowArgs& a, int n_img, int tpb, const float2* tw, hipStream_t s) {
    if (n_img <= 0) return hipSuccess;
    return by_logn<RowL>(a.logn, &a, n_img, tpb, tw, s);
  }
  static hipError_t grid_colfft_conv(const ColArgs& a, int n_img, ConvSpec cs, const float2* tw, hipStream_t s) {
    if (n_img <= 0) return hipSuccess;
    return by_logn<ConvL>(a.logn, &a, n_img, cs, tw, s);
  }
};

template <int PREC>
hipError_t PrecLaunch<PREC>::grid_colfft(const ColArgs& a, int n_img, int strip, const float2* tw, hipStream_t s) {
  return ForPrec<PREC>::grid_colfft(a, n_img, strip, tw, s);
}
template <int PREC>
hipError_t PrecLaunch<PREC>::dense_colfft(const float2* grids, int n_img, int logn, int shift, float2* H,
                                          const float2* tw, const uint4* ops, hipStream_t s) {
  return ForPrec<PREC>::dense_colfft(grids, n_img, logn, shift, H, tw, ops, s);
}
template <int PREC>
hipError_t PrecLaunch<PREC>::row_c2r(const RowArgs& a, int n_img, int tpb, const float2* tw, hipStream_t s) {
  return ForPrec<PREC>::row_c2r(a, n_img, tpb, tw, s);
}
template <int PREC>
hipError_t PrecLaunch<PREC>::grid_colfft_conv(const ColArgs& a, int n_img, int width, float beta, const float2* tw,
                                              hipStream_t s) {
  return ForPrec<PREC>::grid_colfft_conv(a, n_img, ConvSpec{width, beta}, tw, s);
}

static_assert(kPrecFp32 == BLINK_PREC_FP32 && kPrecSplitF16 == BLINK_PREC_SPLIT_F16 &&
                  kPrecSplitBf16 == BLINK_PREC_SPLIT_BF16,
              "device precision tags match the C ABI");

}  // namespace blink
