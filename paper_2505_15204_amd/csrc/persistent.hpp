// persistent.hpp — uneven batches: the persistent fused gridding + FFT kernel as a template over
// the precision form (Section 6.2.4: many channels and intervals gridded in parallel on one GPU
// and transformed all at once; here the images may differ in grid size and visibility count).
// persistent.hip builds the descriptor pass and the FP32 form; split.hip builds the split forms.
//
//   k_persistent     every workgroup repeatedly claims the next image of the order prepared by the
//                    descriptor pass and images it alone: nearest-cell binning into column strips,
//                    the fused gridding + column FFT strip by strip into the workgroup's own
//                    intermediate slot, then the row FFTs into the image
//
// Workgroups never wait for one another: the only shared state is the queue counter, so every
// workgroup finishes once the queue is empty, whatever the number of resident workgroups. The
// intermediate slot is written and read by the same workgroup, ordered by workgroup barriers.
#pragma once

#include <hip/hip_runtime.h>

#include "imaging_device.hpp"
#include "launch.hpp"

namespace blink {

// Strip width and row block of the persistent kernel for one grid size and block size: one
// transform per T = N/16 threads, as many as the block holds (at most N/2).
__host__ __device__ constexpr int fft_threads(int logn) { return logn >= 4 ? (1 << logn) / 16 : 1; }
__host__ __device__ constexpr int desc_cols(int logn, int block) {
  return cmin(block / fft_threads(logn), (1 << logn) / 2);
}

template <int BLOCK>
struct PersistLds {
  // float2 elements of the largest strip or row block over all grid sizes
  static constexpr int f2(int logn) { return desc_cols(logn, BLOCK) * padded_len(1 << logn); }
  static constexpr int max_f2() {
    int m = 0;
    for (int l = 3; l <= 12; ++l) m = f2(l) > m ? f2(l) : m;
    return m;
  }
  // strips of the largest count over all grid sizes (the strip offsets staged in LDS)
  static constexpr int max_strips() {
    int m = 0;
    for (int l = 3; l <= 12; ++l) {
      int c = (1 << l) / 2 / desc_cols(l, BLOCK);
      m = c > m ? c : m;
    }
    return m;
  }
  static constexpr int max_counts() {
    int m = 0;
    for (int l = 3; l <= 12; ++l) {
      int c = desc_cols(l, BLOCK) * (1 << l);
      m = c > m ? c : m;
    }
    return m;
  }
  // The largest twiddle table is staged in LDS when it fits beside the strip and counts of
  // uniform weighting; otherwise the jobs read the tables from global memory.
  static constexpr bool tw_in_lds = (max_f2() + tw_size(12)) * 8 + max_counts() * 4 + 1024 <= kLdsBytes;
};
static_assert(sizeof(BinShared) <= sizeof(float2) * PersistLds<512>::max_f2(), "binning scratch aliases the strip");

// ---------------------------------------------------------------- one image in one workgroup
// A job is a separate (non-inlined) function. Its pointer arguments carry their address space
// (global memory or LDS) in their types: through plain pointers every access in the job would be
// a flat instruction, which also waits on the LDS counter and needs 64-bit addresses per lane.
typedef __attribute__((address_space(1))) const float2 gc_float2;
typedef __attribute__((address_space(1))) const double gc_double;
typedef __attribute__((address_space(1))) const uint8_t gc_u8;
typedef __attribute__((address_space(1))) const uint4 gc_uint4;
typedef __attribute__((address_space(1))) int2 g_int2;
typedef __attribute__((address_space(1))) int g_int;
typedef __attribute__((address_space(1))) float2 g_float2;
typedef __attribute__((address_space(1))) float g_float;
typedef __attribute__((address_space(1))) int32_t g_i32;
typedef __attribute__((address_space(1))) double g_double;
typedef __attribute__((address_space(3))) float2 l_float2;
typedef __attribute__((address_space(3))) unsigned l_u32;
typedef __attribute__((address_space(3))) int l_int;

struct ImageJob {
  gc_float2* V;             // visibilities of the image
  gc_double* uvw;           // its baselines' uvw
  gc_u8* flags;             // its flags or null
  int B;
  double k;                 // cells per metre
  g_int2* plc;              // this workgroup's placement list
  g_int* off;               // this workgroup's strip offsets
  g_float2* H;              // this workgroup's intermediate slot
  g_float* out;             // the image
  g_i32* n_out;             // its out-of-grid count or null
  g_double* wsum;           // its weight sum or null
  int shift;
};

// The LDS arrays of the persistent kernel that a job uses.
struct JobLds {
  l_float2* sbuf;           // strip / row-block buffer (also the binning scratch)
  l_u32* scnt;              // uniform weighting's counts
  l_int* s_int;             // [0] block reduction word, [1] kept count, [2] occupancy
  l_u32* s_max;             // the split form's largest magnitude
  l_float2* stw;            // twiddle table copy (TWL)
  l_int* s_tw_logn;         // size whose table stw holds
  l_int* s_off;             // strip offsets
};

template <int S>
struct Log2 {
  static constexpr int value = S <= 1 ? 0 : 1 + Log2<S / 2>::value;
};
template <>
struct Log2<1> {
  static constexpr int value = 0;
};

// `tw` is the twiddle table of N in global memory; with TWL it is first copied to `stw` (LDS)
// unless the previous job of this workgroup had the same size (*s_tw_logn). The strips are
// gridded and transformed by the batched path's pipelined strip loop (grid_colfft_strips, every
// strip in turn) from the strip offsets copied to `s_off` (LDS, NBLK + 1 ints).
template <int LOGN, int BLOCK, bool UNIFORM, int PREC, bool TWL>
__device__ __noinline__ void image_job(ImageJob j, gc_float2* gtw, gc_uint4* gops, JobLds lds) {
  constexpr int N = 1 << LOGN;
  constexpr int S = desc_cols(LOGN, BLOCK);
  constexpr int NBLK = (N / 2) / S;         // column strips, and row blocks of S row pairs
  constexpr int LOGS = Log2<S>::value;
  static_assert((1 << LOGS) == S, "strip width is a power of two");
  const float2* tw = (const float2*)gtw;
  float2* sbuf = (float2*)lds.sbuf;
  unsigned* scnt = (unsigned*)lds.scnt;
  int* s_int = (int*)lds.s_int;
  float2* stw = (float2*)lds.stw;
  int* s_tw_logn = (int*)lds.s_tw_logn;
  int* s_off = (int*)lds.s_off;
  const SplitCtx sp{(unsigned*)lds.s_max, (const uint4*)gops};
  const float2* V = (const float2*)j.V;
  const double* uvw = (const double*)j.uvw;
  const uint8_t* flags = (const uint8_t*)j.flags;
  int2* plc = (int2*)j.plc;
  int* off = (int*)j.off;
  float2* H = (float2*)j.H;
  float* out = (float*)j.out;
  int32_t* n_out = (int32_t*)j.n_out;
  double* wsum = (double*)j.wsum;
  int* s_tmp = s_int;
  int* s_kept = s_int + 1;
  int* s_occ = s_int + 2;
  BinShared& bsh = *reinterpret_cast<BinShared*>(sbuf);
  if constexpr (TWL) {
    if (*s_tw_logn != LOGN) {           // the same value in every thread: a uniform branch
      for (int i = threadIdx.x; i < tw_size(LOGN); i += BLOCK) stw[i] = tw[i];
      __syncthreads();                  // every thread has read *s_tw_logn and the table is complete
      if (threadIdx.x == 0) *s_tw_logn = LOGN;
    }
    tw = stw;
  }
  bin_visibilities(uvw, flags, j.B, j.k, LOGN, LOGS, N / 2, plc, off, s_kept, n_out, nullptr, bsh);
  if (threadIdx.x == 0) *s_occ = 0;
  __syncthreads();                          // placement list and offsets complete; binning scratch free
  for (int i = threadIdx.x; i <= NBLK; i += BLOCK) s_off[i] = off[i];   // visible after the loop's first barrier
  grid_colfft_strips<LOGN, S, UNIFORM, PREC, BLOCK, kColPrefetch>(V, plc, s_off, 0, 1, NBLK, j.B > 0 ? NBLK : 0,
                                                                  j.shift != 0, H, s_occ, tw, sbuf, scnt, s_tmp, sp);
  const double W = UNIFORM ? (double)*s_occ : 2.0 * (double)*s_kept;
  if (wsum && threadIdx.x == 0) *wsum = W;
  const float scale = inverse_weight(W);
  for (int rb = 0; rb < NBLK; ++rb) {
    row_task<LOGN, S, PREC>(H, rb, scale, out, tw, sbuf, sp);
    __syncthreads();
  }
}

template <int BLOCK, bool UNIFORM, int PREC>
__global__ __launch_bounds__(BLOCK) void k_persistent(DescArgs a) {
  using L = PersistLds<BLOCK>;
  __shared__ float2 sbuf[L::max_f2()];
  __shared__ unsigned scnt[UNIFORM ? L::max_counts() : 1];
  __shared__ int s_int[4];
  __shared__ int s_next;
  __shared__ unsigned s_max;
  constexpr bool TWL = L::tw_in_lds;
  __shared__ float2 stw[TWL ? tw_size(12) : 1];
  __shared__ int s_tw_logn;
  __shared__ int s_off[L::max_strips() + 1];
  if (threadIdx.x == 0) s_tw_logn = -1;   // visible after the claim barrier below
  const size_t slot_elems = (size_t)1 << (2 * a.max_logn - 1);
  float2* H = a.H + (size_t)blockIdx.x * slot_elems;
  int2* plc = a.plc + (size_t)blockIdx.x * 2 * a.max_b;
  int* off = a.strip_off + (size_t)blockIdx.x * a.strip_stride;
  for (;;) {
    if (threadIdx.x == 0) s_next = atomicAdd(a.counter, 1);
    __syncthreads();
    const int q = s_next;
    __syncthreads();
    if (q >= a.n_img) break;
    const int img = a.order[q];
    if (!a.valid[img]) continue;
    const blink_image_desc d = a.desc[img];
    const int logn = 31 - __clz(d.grid_n);
    ImageJob j;
    j.V = (gc_float2*)(a.vis + d.vis_offset);
    j.uvw = (gc_double*)(a.uvw + 3 * d.uvw_offset);
    j.flags = a.flags ? (gc_u8*)(a.flags + d.flag_offset) : nullptr;
    j.B = d.n_baselines;
    j.k = (d.freq_hz / kSpeedOfLight) * ((double)d.grid_n * d.pixel_scale);
    j.plc = (g_int2*)plc;
    j.off = (g_int*)off;
    j.H = (g_float2*)H;
    j.out = (g_float*)(a.images + d.image_offset);
    j.n_out = a.n_out ? (g_i32*)(a.n_out + img) : nullptr;
    j.wsum = a.weight_sum ? (g_double*)(a.weight_sum + img) : nullptr;
    j.shift = a.shift;
    const JobLds lds{(l_float2*)sbuf, (l_u32*)scnt, (l_int*)s_int, (l_u32*)&s_max, (l_float2*)stw,
                     (l_int*)&s_tw_logn, (l_int*)s_off};
    gc_uint4* ops = (gc_uint4*)a.dft_ops;
    switch (logn) {
      case 3: image_job<3, BLOCK, UNIFORM, PREC, TWL>(j, (gc_float2*)a.tw[3], ops, lds); break;
      case 4: image_job<4, BLOCK, UNIFORM, PREC, TWL>(j, (gc_float2*)a.tw[4], ops, lds); break;
      case 5: image_job<5, BLOCK, UNIFORM, PREC, TWL>(j, (gc_float2*)a.tw[5], ops, lds); break;
      case 6: image_job<6, BLOCK, UNIFORM, PREC, TWL>(j, (gc_float2*)a.tw[6], ops, lds); break;
      case 7: image_job<7, BLOCK, UNIFORM, PREC, TWL>(j, (gc_float2*)a.tw[7], ops, lds); break;
      case 8: image_job<8, BLOCK, UNIFORM, PREC, TWL>(j, (gc_float2*)a.tw[8], ops, lds); break;
      case 9: image_job<9, BLOCK, UNIFORM, PREC, TWL>(j, (gc_float2*)a.tw[9], ops, lds); break;
      case 10: image_job<10, BLOCK, UNIFORM, PREC, TWL>(j, (gc_float2*)a.tw[10], ops, lds); break;
      case 11: image_job<11, BLOCK, UNIFORM, PREC, TWL>(j, (gc_float2*)a.tw[11], ops, lds); break;
      case 12: image_job<12, BLOCK, UNIFORM, PREC, TWL>(j, (gc_float2*)a.tw[12], ops, lds); break;
      default: break;
    }
  }
}

template <int PREC>
int PersistLaunch<PREC>::blocks_per_cu(int block, bool uniform) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  if (block == 512 && !uniform)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persistent<512, false, PREC>, 512, 0);
  if (block == 1024 && !uniform)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persistent<1024, false, PREC>, 1024, 0);
  if (block == 512 && uniform)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_persistent<512, true, PREC>, 512, 0);
  return e == hipSuccess ? n : 0;
}

template <int PREC>
hipError_t PersistLaunch<PREC>::launch(const DescArgs& a, int workgroups, hipStream_t s) {
  if (a.n_img <= 0) return hipSuccess;
  if (a.block == 512 && !a.weighting) k_persistent<512, false, PREC><<<workgroups, 512, 0, s>>>(a);
  else if (a.block == 1024 && !a.weighting) k_persistent<1024, false, PREC><<<workgroups, 1024, 0, s>>>(a);
  else if (a.block == 512 && a.weighting) k_persistent<512, true, PREC><<<workgroups, 512, 0, s>>>(a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace blink
