// staged.hpp — the staged form of the uneven-batch path: the batched path's fused column kernel
// and row kernel applied to one chunk of same-size images of an uneven batch (the descriptor pass
// in persistent.hip builds the chunks), with the batched path's variants (strip width, row
// block). staged.hip builds them once per precision form, in an object of their own.
#pragma once

#include "kernels.hpp"

namespace blink {

// ---------------------------------------------------------------- uneven batches, staged form
// The batched kernels' work on one chunk of an uneven batch: up to `slots` images of one grid size
// whose half spectra share the chunk buffer. Image slot blockIdx.x of chunk {logn, first, count}
// is the image at position first + slot of the descriptor pass's order; its placements, strip
// offsets, counts and column extent are indexed by that position and its half spectrum sits at
// slot N^2/2 in the chunk buffer. Workgroups of slots past the chunk's count (or of an empty
// chunk) return at once.
template <int LOGN, int S, bool UNIFORM, int PREC>
__global__ __launch_bounds__(fft_block(S * FftPlan<LOGN>::T, PREC)) void k_chunk_colfft(DescArgs a, int chunk,
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
  const int4 c = a.chunks[chunk];
  const int slot = blockIdx.x;
  if (c.x != LOGN || slot >= c.z) return;   // uniform over the workgroup
  const int q = c.y + slot;
  const int nstrips = (N / 2) / S;
  const int live = a.ext[q] / S;            // strips past the column extent hold no placement
  if ((int)blockIdx.y >= live) return;
  const blink_image_desc d = a.desc[a.order[q]];
  for (int i = threadIdx.x; i < TW; i += NT) stw[i] = twg[i];   // visible after the strips' first barrier
  const int* so = a.strip_off + (size_t)q * a.strip_stride;
  for (int i = threadIdx.x; i <= nstrips; i += NT) s_off[i] = so[i];
  grid_colfft_strips<LOGN, S, UNIFORM, PREC, NT, kColPrefetch>(
      a.vis + d.vis_offset, a.plc + (size_t)q * 2 * a.max_b, s_off, blockIdx.y, gridDim.y, live,
      d.n_baselines > 0 ? live : 0, a.shift != 0, a.H + (size_t)slot * N * (N / 2), a.occ + q, stw, sbuf, scnt,
      &s_tmp, SplitCtx{&s_max, a.dft_ops});
}

template <int LOGN, int TPB, int PREC>
__global__ __launch_bounds__(fft_block(TPB * FftPlan<LOGN>::T, PREC)) void k_chunk_row(DescArgs a, int chunk,
                                                                                        const float2* __restrict__ twg) {
  using P = FftPlan<LOGN>;
  constexpr int N = P::N, NP = P::NP;
  __shared__ float2 sbuf[TPB * NP];        // twiddles from the global table, as in k_row_c2r
  __shared__ unsigned s_max;
  const int4 c = a.chunks[chunk];
  const int slot = blockIdx.x;
  if (c.x != LOGN || slot >= c.z) return;
  const int q = c.y + slot;
  const int img = a.order[q];
  const float2* stw = twg;
  const double W = a.weighting ? (double)a.occ[q] : 2.0 * (double)a.kept[q];
  if (a.weight_sum && blockIdx.y == 0 && threadIdx.x == 0) a.weight_sum[img] = W;
  row_task<LOGN, TPB, PREC>(a.H + (size_t)slot * N * (N / 2), blockIdx.y, inverse_weight(W),
                            a.images + a.desc[img].image_offset, stw, sbuf, SplitCtx{&s_max, a.dft_ops}, nullptr,
                            a.ext[q]);
}

template <int PREC>
struct StagedFor {
  template <int LOGN, int S, bool U>
  static hipError_t chunk_col_one(const DescArgs* a, int chunk, int col_loop, int slots, hipStream_t s) {
    if constexpr (S >= 1) {
      const int nstrips = ((1 << LOGN) / 2) / S, loop = col_loop > 1 ? col_loop : 1;
      dim3 grid(slots, (nstrips + loop - 1) / loop);
      k_chunk_colfft<LOGN, S, U, PREC><<<grid, fft_block(S * FftPlan<LOGN>::T, PREC), 0, s>>>(*a, chunk, a->tw[LOGN]);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }

  template <int LOGN, bool U>
  static hipError_t chunk_col_variant(const DescArgs* a, int chunk, int S, int col_loop, int slots, hipStream_t s) {
    constexpr int SM = ColSmax<LOGN, U>::value;
    if (S == SM) return chunk_col_one<LOGN, SM, U>(a, chunk, col_loop, slots, s);
    if constexpr (LOGN >= kTunedLogn) {
      if (S == SM / 2) return chunk_col_one<LOGN, SM / 2, U>(a, chunk, col_loop, slots, s);
      if (S == SM / 4) return chunk_col_one<LOGN, SM / 4, U>(a, chunk, col_loop, slots, s);
    }
    return hipErrorInvalidValue;
  }

  template <int LOGN>
  struct ChunkColL {
    static hipError_t run(const DescArgs* a, int chunk, int S, int col_loop, int slots, hipStream_t s) {
      return a->weighting ? chunk_col_variant<LOGN, true>(a, chunk, S, col_loop, slots, s)
                          : chunk_col_variant<LOGN, false>(a, chunk, S, col_loop, slots, s);
    }
  };

  template <int LOGN, int TPB>
  static hipError_t chunk_row_one(const DescArgs* a, int chunk, int slots, hipStream_t s) {
    if constexpr (RowFits<LOGN, TPB>::value) {
      dim3 grid(slots, ((1 << LOGN) / 2) / TPB);
      k_chunk_row<LOGN, TPB, PREC><<<grid, fft_block(TPB * FftPlan<LOGN>::T, PREC), 0, s>>>(*a, chunk, a->tw[LOGN]);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }

  template <int LOGN>
  struct ChunkRowL {
    static hipError_t run(const DescArgs* a, int chunk, int tpb, int slots, hipStream_t s) {
      if constexpr (LOGN >= kTunedLogn) {
        switch (tpb) {
          case 1: return chunk_row_one<LOGN, 1>(a, chunk, slots, s);
          case 2: return chunk_row_one<LOGN, 2>(a, chunk, slots, s);
          case 4: return chunk_row_one<LOGN, 4>(a, chunk, slots, s);
          case 8: return chunk_row_one<LOGN, 8>(a, chunk, slots, s);
          default: return hipErrorInvalidValue;
        }
      } else {
        if (tpb != RowDefault<LOGN>::value) return hipErrorInvalidValue;
        return chunk_row_one<LOGN, RowDefault<LOGN>::value>(a, chunk, slots, s);
      }
    }
  };

};

template <int PREC>
hipError_t StagedLaunch<PREC>::colfft(const DescArgs& a, int chunk, int logn, int strip, int col_loop, int slots,
                                      hipStream_t s) {
  if (slots <= 0) return hipSuccess;
  return by_logn<StagedFor<PREC>::template ChunkColL>(logn, &a, chunk, strip, col_loop, slots, s);
}

template <int PREC>
hipError_t StagedLaunch<PREC>::row(const DescArgs& a, int chunk, int logn, int tpb, int slots, hipStream_t s) {
  if (slots <= 0) return hipSuccess;
  return by_logn<StagedFor<PREC>::template ChunkRowL>(logn, &a, chunk, tpb, slots, s);
}

}  // namespace blink
