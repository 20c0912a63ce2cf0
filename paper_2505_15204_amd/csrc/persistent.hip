// persistent.hip — uneven batches: the descriptor pass and the FP32 form of the persistent
// kernel (persistent.hpp); the split precision forms are built in split.hip.
//
//   k_desc_prep      checks every descriptor against the caller's array lengths, orders the valid
//                    images by decreasing grid size (so the longest jobs start first) and resets
//                    the queue; for the staged form it also cuts the order into chunks
//   k_desc_bin       staged form: bins every valid image (one workgroup per image)
#include <hip/hip_runtime.h>

#include "persistent.hpp"

namespace blink {

// ---------------------------------------------------------------- descriptor pass
__global__ __launch_bounds__(1024) void k_desc_prep(DescArgs a) {
  __shared__ int s_bucket[17];     // images per log2 N (3..12), then their offsets
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  if (tid < 17) s_bucket[tid] = 0;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int i = tid; i < a.n_img; i += blockDim.x) {
    const blink_image_desc d = a.desc[i];
    const int n = d.grid_n;
    int logn = -1;
    if (n >= 8 && n <= (1 << a.max_logn) && (n & (n - 1)) == 0) logn = 31 - __clz(n);
    bool ok = logn >= 3;
    ok = ok && d.n_baselines >= 0 && d.n_baselines <= a.max_b;
    ok = ok && d.pixel_scale > 0.0 && isfinite(d.pixel_scale) && isfinite(d.freq_hz);
    ok = ok && d.vis_offset >= 0 && d.vis_offset + d.n_baselines <= a.vis_len;
    ok = ok && d.uvw_offset >= 0 && d.uvw_offset + d.n_baselines <= a.uvw_len;
    ok = ok && (!a.flags || (d.flag_offset >= 0 && d.flag_offset + d.n_baselines <= a.flags_len));
    ok = ok && d.image_offset >= 0 && d.image_offset + (int64_t)n * n <= a.images_len;
    a.valid[i] = ok ? 1 : 0;
    // bucket 0 holds the largest grids; invalid images go last (bucket 16)
    atomicAdd(&s_bucket[ok ? 12 - logn : 16], 1);
    if (!ok) s_bad = 1;
  }
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int b = 0; b < 17; ++b) {
      const int c = s_bucket[b];
      s_bucket[b] = run;
      run += c;
    }
    *a.counter = 0;
    *a.status = s_bad ? BLINK_DESC_BAD : 0;
  }
  __syncthreads();
  if (a.chunks) {
    // Staged form: the images of one bucket (one grid size) go in chunks of as many as the chunk
    // buffer holds, in that size's reserved range of the chunk table (staged_slots); the
    // remaining slots of the range get no images.
    __shared__ int s_first[10], s_count[10], s_cap[10], s_base[11];
    if (tid == 0) {
      int base = 0;
      for (int b = 0; b < 10; ++b) {
        const int logn = 12 - b;
        s_first[b] = s_bucket[b];
        s_count[b] = s_bucket[b + 1] - s_bucket[b];
        s_cap[b] = staged_capacity(logn, a.chunk_elems, a.n_img);
        s_base[b] = base;
        if (logn <= a.max_logn) base += staged_slots(logn, a.chunk_elems, a.n_img);
      }
      s_base[10] = base;
    }
    __syncthreads();
    for (int j = tid; j < a.max_chunks; j += blockDim.x) {
      int4 e = make_int4(0, 0, 0, 0);
      for (int b = 0; b < 10; ++b)
        if (j >= s_base[b] && j < s_base[b + 1]) {
          const int first = s_first[b] + (j - s_base[b]) * s_cap[b];
          const int left = s_first[b] + s_count[b] - first;
          e = make_int4(12 - b, first, left > 0 ? min(s_cap[b], left) : 0, 0);
        }
      a.chunks[j] = e;
    }
  }
  for (int i = tid; i < a.n_img; i += blockDim.x) {
    const int b = a.valid[i] ? 12 - (31 - __clz(a.desc[i].grid_n)) : 16;
    a.order[atomicAdd(&s_bucket[b], 1)] = i;
  }
}

// Staged form: workgroup q bins the image at position q of the order into strips of the column
// width the chunk kernels use for its size, into its own placement list and offsets.
__global__ __launch_bounds__(kBinThreads) void k_desc_bin(DescArgs a) {
  __shared__ BinShared sh;
  const int q = blockIdx.x;
  const int img = a.order[q];
  if (!a.valid[img]) return;                 // uniform over the workgroup
  const blink_image_desc d = a.desc[img];
  const int logn = 31 - __clz(d.grid_n);
  const int log_s = a.col_log_strip[logn];
  const double k = (d.freq_hz / kSpeedOfLight) * ((double)d.grid_n * d.pixel_scale);
  bin_visibilities(a.uvw + 3 * d.uvw_offset, a.flags ? a.flags + d.flag_offset : nullptr, d.n_baselines, k, logn,
                   log_s, d.grid_n / 2, a.plc + (size_t)q * 2 * a.max_b, a.strip_off + (size_t)q * a.strip_stride,
                   a.kept + q, a.n_out ? a.n_out + img : nullptr, nullptr, sh, a.ext + q);
  if (threadIdx.x == 0) a.occ[q] = 0;
}

hipError_t launch_desc_prep(const DescArgs& a, hipStream_t s) {
  k_desc_prep<<<1, 1024, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_desc_bin(const DescArgs& a, hipStream_t s) {
  if (a.n_img <= 0) return hipSuccess;
  k_desc_bin<<<a.n_img, kBinThreads, 0, s>>>(a);
  return hipGetLastError();
}

template struct PersistLaunch<BLINK_PREC_FP32>;

hipError_t launch_persistent(const DescArgs& a, int workgroups, int prec, hipStream_t s) {
  switch (prec) {
    case BLINK_PREC_FP32: return PersistLaunch<BLINK_PREC_FP32>::launch(a, workgroups, s);
    case BLINK_PREC_SPLIT_F16: return PersistLaunch<BLINK_PREC_SPLIT_F16>::launch(a, workgroups, s);
    case BLINK_PREC_SPLIT_BF16: return PersistLaunch<BLINK_PREC_SPLIT_BF16>::launch(a, workgroups, s);
    default: return hipErrorInvalidValue;
  }
}

int persistent_blocks_per_cu(int block, bool uniform, int prec) {
  switch (prec) {
    case BLINK_PREC_FP32: return PersistLaunch<BLINK_PREC_FP32>::blocks_per_cu(block, uniform);
    case BLINK_PREC_SPLIT_F16: return PersistLaunch<BLINK_PREC_SPLIT_F16>::blocks_per_cu(block, uniform);
    case BLINK_PREC_SPLIT_BF16: return PersistLaunch<BLINK_PREC_SPLIT_BF16>::blocks_per_cu(block, uniform);
    default: return 0;
  }
}

}  // namespace blink
