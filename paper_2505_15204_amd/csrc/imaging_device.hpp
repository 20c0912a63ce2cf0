// imaging_device.hpp — device building blocks shared by the batched kernels (kernels.hip) and the
// persistent uneven-batch kernel (persistent.hip): nearest-cell binning, LDS-private strip
// gridding fused with the column FFT, and the Hermitian-extended row FFT.
#pragma once

#include <hip/hip_runtime.h>

#include "fft_device.hpp"
#include "split_fft.hpp"

namespace blink {

constexpr int kLdsBytes = 160 * 1024;
constexpr double kSpeedOfLight = 299792458.0;
constexpr int kBinThreads = 1024;
constexpr int kMaxStrips = 4096;
// Fourth word of a raw buffer resource on gfx9-family chips (gfx950): 32-bit data format, no
// swizzle, no index stride; with it a load at or past the resource's byte size returns zero.
constexpr int kBufferRsrcWord3 = 0x00020000;

__host__ __device__ constexpr int pow2_floor(int x) {
  int p = 1;
  while (p * 2 <= x) p *= 2;
  return p;
}
__host__ __device__ constexpr int cmin(int a, int b) { return a < b ? a : b; }

// ---------------------------------------------------------------- block scan
// Exclusive scan of v[0..n) in place by the whole workgroup (blockDim a multiple of 64, at most
// 1024; n <= 8 * blockDim); v[n] receives the total. s_wave holds at least 17 ints.
__device__ inline void block_exclusive_scan(int* v, int n, int* s_wave) {
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, w = tid >> 6, nw = nt >> 6;
  const int per = (n + nt - 1) / nt;
  const int base = tid * per;
  int tsum = 0;
  for (int j = 0; j < per; ++j)
    if (base + j < n) tsum += v[base + j];
  int x = tsum;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) s_wave[w] = x;
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int i = 0; i < nw; ++i) {
      int t = s_wave[i];
      s_wave[i] = run;
      run += t;
    }
    s_wave[nw] = run;
  }
  __syncthreads();
  int excl = s_wave[w] + x - tsum;
  for (int j = 0; j < per; ++j) {
    if (base + j < n) {
      const int t = v[base + j];
      v[base + j] = excl;
      excl += t;
    }
  }
  if (tid == 0) v[n] = s_wave[nw];
  __syncthreads();
}

// ---------------------------------------------------------------- binning
// Nearest cell of one visibility (Section 6.2.4). Returns 1 when kept (and sets iu, iv), 0 when
// out of grid. k = (f/c)(N dl) cells per metre; iu = rint(u k), ties to even.
__device__ __forceinline__ int nearest_cell(double u, double v, double k, double half, int& iu, int& iv) {
  const double ru = rint(u * k);      // one IEEE double product, round half to even
  const double rv = rint(v * k);
  if (!(fabs(ru) < half && fabs(rv) < half)) return 0;   // NaN lands here too
  iu = (int)ru;
  iv = (int)rv;
  return 1;
}

struct BinShared {
  int cnt[kMaxStrips + 1];
  int wave[17];
  int red[3];
};

// Cell indices and the counting sort of one visibility set's placements into column strips of
// width 2^log_strip, keeping only columns ku < ku_limit. Writes the placement list plc (each
// record {kv*N + ku, b | conj<<31}), the strip offsets off[0..ku_limit>>log_strip], the kept and
// out-of-grid counts, and cell_idx[b] when non-null. When ext_out is non-null it receives the
// column extent: (index of the last strip holding a placement + 1) * 2^log_strip, 0 when no
// placement is kept; every column at or beyond it is zero in the grid. One workgroup (a multiple
// of 64 threads, at least 512 so that the strip count fits the scan).
__device__ inline void bin_visibilities(const double* __restrict__ uvw, const uint8_t* __restrict__ fl, int B,
                                        double k, int logn, int log_strip, int ku_limit, int2* __restrict__ plc,
                                        int* __restrict__ off, int* kept_out, int* nout_out,
                                        int32_t* __restrict__ cell_idx, BinShared& sh, int* ext_out = nullptr) {
  const int N = 1 << logn, mask = N - 1;
  const int nstrips = ku_limit >> log_strip;
  const double half = (double)(N / 2);
  for (int i = threadIdx.x; i <= nstrips; i += blockDim.x) sh.cnt[i] = 0;
  if (threadIdx.x < 3) sh.red[threadIdx.x] = 0;
  __syncthreads();
  int kept = 0, outside = 0;
  for (int b = threadIdx.x; b < B; b += blockDim.x) {
    int cell = -1;
    if (!(fl && fl[b])) {
      int iu, iv;
      if (nearest_cell(uvw[3 * b], uvw[3 * b + 1], k, half, iu, iv)) {
        const int ku1 = iu & mask, kv1 = iv & mask, ku2 = (-iu) & mask;
        cell = kv1 * N + ku1;
        ++kept;
        if (ku1 < ku_limit) atomicAdd(&sh.cnt[ku1 >> log_strip], 1);
        if (ku2 < ku_limit) atomicAdd(&sh.cnt[ku2 >> log_strip], 1);
      } else {
        cell = -2;
        ++outside;
      }
    }
    if (cell_idx) cell_idx[b] = cell;
  }
  if (kept) atomicAdd(&sh.red[0], kept);
  if (outside) atomicAdd(&sh.red[1], outside);
  __syncthreads();
  // the counts are read here before the scan's first barrier, after which it overwrites them
  if (ext_out)
    for (int i = threadIdx.x; i < nstrips; i += blockDim.x)
      if (sh.cnt[i] > 0) atomicMax(&sh.red[2], i + 1);
  block_exclusive_scan(sh.cnt, nstrips, sh.wave);
  for (int i = threadIdx.x; i <= nstrips; i += blockDim.x) off[i] = sh.cnt[i];
  if (threadIdx.x == 0) {
    *kept_out = sh.red[0];
    if (nout_out) *nout_out = sh.red[1];
  }
  __syncthreads();
  if (ext_out && threadIdx.x == 0) *ext_out = sh.red[2] << log_strip;
  for (int b = threadIdx.x; b < B; b += blockDim.x) {
    if (fl && fl[b]) continue;
    int iu, iv;
    if (!nearest_cell(uvw[3 * b], uvw[3 * b + 1], k, half, iu, iv)) continue;
    const int ku1 = iu & mask, kv1 = iv & mask;
    const int ku2 = (-iu) & mask, kv2 = (-iv) & mask;
    if (ku1 < ku_limit) {
      int pos = atomicAdd(&sh.cnt[ku1 >> log_strip], 1);
      plc[pos] = make_int2(kv1 * N + ku1, b);
    }
    if (ku2 < ku_limit) {
      int pos = atomicAdd(&sh.cnt[ku2 >> log_strip], 1);
      plc[pos] = make_int2(kv2 * N + ku2, (int)((unsigned)b | 0x80000000u));
    }
  }
}

// ---------------------------------------------------------------- scatter into an LDS strip
// Accumulates the placements [o0, o1) of strip `strip` into the LDS strip buffer (column c at
// sbuf[c*stride + pad(kv)] when PADDED, else sbuf[c*stride + kv]); V are the image's
// visibilities; the mirrored placement takes the conjugate; `modulate` applies (-1)^(ku+kv).
// place_one adds one placement record r (with its visibility v) to the strip.
template <int LOGN, int S, bool PADDED, bool COUNT>
__device__ __forceinline__ void place_one(int2 r, float2 val, int strip, int stride, bool modulate, float2* sbuf,
                                          unsigned* scnt) {
  constexpr int N = 1 << LOGN;
  const int kv = r.x >> LOGN, ku = r.x & (N - 1);
  if (r.y < 0) val.y = -val.y;
  if (modulate && ((kv + ku) & 1)) {
    val.x = -val.x;
    val.y = -val.y;
  }
  const int col = ku - strip * S;
  float2* dst = sbuf + col * stride + (PADDED ? pad_index(kv) : kv);
  atomicAdd(&dst->x, val.x);
  atomicAdd(&dst->y, val.y);
  if constexpr (COUNT) atomicAdd(&scnt[col * N + kv], 1u);
}

template <int LOGN, int S, bool PADDED, bool COUNT>
__device__ __forceinline__ void scatter_strip(const int2* __restrict__ plc, int o0, int o1,
                                              const float2* __restrict__ V, int strip, int stride,
                                              bool modulate, float2* sbuf, unsigned* scnt) {
  for (int i = o0 + (int)threadIdx.x; i < o1; i += blockDim.x) {
    const int2 r = plc[i];
    place_one<LOGN, S, PADDED, COUNT>(r, V[r.y & 0x7fffffff], strip, stride, modulate, sbuf, scnt);
  }
}

// Uniform weighting: cell mean; returns this thread's occupied-cell count (weighted). NT is the
// workgroup size (0: read blockDim). With CLEAR every count read is reset to zero behind the read.
template <int LOGN, int S, bool PADDED, int NT = 0, bool CLEAR = false>
__device__ __forceinline__ int uniform_divide(float2* sbuf, unsigned* scnt, int stride, int col_weight0,
                                              int col_weight) {
  constexpr int N = 1 << LOGN;
  const int nt = NT > 0 ? NT : (int)blockDim.x;
  int occ = 0;
  for (int i = threadIdx.x; i < S * N; i += nt) {
    const int col = i >> LOGN, kv = i & (N - 1);
    const unsigned n = scnt[i];
    if (n) {
      float2* p = sbuf + col * stride + (PADDED ? pad_index(kv) : kv);
      const float inv = 1.0f / (float)n;
      p->x *= inv;
      p->y *= inv;
      occ += (col == 0) ? col_weight0 : col_weight;
      if constexpr (CLEAR) scnt[i] = 0u;
    }
  }
  return occ;
}

// Adds one value per thread into *dst with a single global atomic per workgroup. *s_tmp is zero
// on entry and is zero again once the caller's next barrier has passed.
__device__ __forceinline__ void block_add_to_global(int val, int* s_tmp, int* dst) {
  if (val) atomicAdd(s_tmp, val);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (*s_tmp) atomicAdd(dst, *s_tmp);
    *s_tmp = 0;
  }
}

// ---------------------------------------------------------------- strip store
// The S transformed columns of a strip (column c at sbuf + c*NP, padded) into rows of the half
// spectrum: Hi[y][strip*S + c]. With REAL0, column 0 of strip 0 keeps only its real part (the
// transform of the Hermitian part of column 0; the imaginary slot is the Nyquist column's, empty).
// Thread t handles column t % S of rows t / S + j * NT / S, so when NT / S is a multiple of 16
// every address is one base plus compile-time steps. With ZERO every cell read is cleared behind
// the read (the cells at pad(y) of the S columns: all that gridding and the transforms use), so
// the strip buffer is zero for the next strip once the caller's following barrier has passed.
template <int LOGN, int S, int NT, bool REAL0 = true, bool ZERO = false>
__device__ __forceinline__ void store_strip(float2* sbuf, int strip, float2* __restrict__ Hi) {
  constexpr int N = 1 << LOGN, NP = padded_len(N), HALF = N / 2;
  if constexpr (NT % S == 0 && (NT / S) % 16 == 0 && (S * N) % NT == 0) {
    constexpr int RPI = NT / S, ITER = (S * N) / NT;
    const int c = (int)threadIdx.x % S, y0 = (int)threadIdx.x / S;
    float2* src = sbuf + c * NP + pad_index(y0);
    float2* dst = Hi + (size_t)y0 * HALF + strip * S + c;
    const bool real_only = REAL0 && strip == 0 && c == 0;
#pragma unroll
    for (int j = 0; j < ITER; ++j) {
      float2 val = src[pad_offset(j * RPI)];
      if constexpr (ZERO) src[pad_offset(j * RPI)] = make_float2(0.f, 0.f);
      if (real_only) val.y = 0.f;
      dst[(size_t)j * RPI * HALF] = val;
    }
  } else {
    for (int i = threadIdx.x; i < S * N; i += NT) {
      const int y = i / S, c = i % S;
      float2 val = sbuf[c * NP + pad_index(y)];
      if constexpr (ZERO) sbuf[c * NP + pad_index(y)] = make_float2(0.f, 0.f);
      if (REAL0 && strip == 0 && c == 0) val.y = 0.f;
      Hi[(size_t)y * HALF + strip * S + c] = val;
    }
  }
}

// ---------------------------------------------------------------- strip FFT + store
// The column transforms of a gridded LDS strip (S columns, padded) and their store into Hi; the
// block is synchronised before the store. REAL0 keeps only the real part of column 0 of strip 0
// (nearest-cell gridding leaves the Nyquist column empty); without it column 0 carries
// (column 0) + i (column N/2) as packed by the gridding.
template <int LOGN, int S, int PREC, int NT, bool REAL0, bool ZERO = false>
__device__ __forceinline__ void strip_fft_store(float2* sbuf, int strip, float2* __restrict__ Hi,
                                                const float2* __restrict__ tw, SplitCtx sp) {
  using P = FftPlan<LOGN>;
  constexpr int T = P::T, NP = P::NP;
  constexpr bool SPLIT = PREC != kPrecFp32 && LOGN >= 4;
  if constexpr (SPLIT) {
    fft_inverse_split<LOGN, PREC, true, true>(
        sbuf, S, tw, [&](int c, int e) { return sbuf[c * NP + pad_index(e)]; }, [](int, int, float2) {}, sp);
  } else {
    const bool active = (int)threadIdx.x < S * T;
    const int col = active ? (int)threadIdx.x / T : 0, lt = (int)threadIdx.x % T;
    float2* cb = sbuf + col * NP;
    float2 v[P::R];
    if (active) stage_load_lds<P::N, P::R, T, P::R0>(v, cb, lt);
    fft_inverse<LOGN, true>(v, cb, tw, lt, [](int, float2) {}, active);
  }
  store_strip<LOGN, S, NT, REAL0, ZERO>(sbuf, strip, Hi);
}

// ---------------------------------------------------------------- fused grid + column FFT of strips
// The strips strip0, strip0 + dstrip, ... (< nstrips) of one image. One strip is S half-spectrum
// columns: scatter the strip's placements into the zeroed LDS strip, (uniform) divide by counts
// and add the strip's occupied cells (column 0 once, columns 1..N/2-1 twice for their mirrors) to
// *occ_img, inverse FFT every column along v, and store the strip into Hi[y][strip*S + c]. Column
// 0 is stored as (Re of its transform, 0): the real part is the transform of the column's
// Hermitian part, and the Nyquist column is empty. `tw` is the twiddle table for N. PREC selects
// the FP32 butterflies or the split matrix-core form (split_fft.hpp), which needs a workgroup of
// whole waves (threads beyond S*T only join the barriers); `sp` holds that form's LDS word for
// the strip's largest magnitude and the DFT operand table. NT is the workgroup size.
//
// The global loads of the placements are software-pipelined across strips: the first PF*NT
// placement records of the strip after next and the visibilities of the next strip are requested
// before the current strip's column FFT and store, so they arrive while the workgroup computes
// and the scatter of the next strip starts from registers. Placements beyond the first PF*NT of a
// strip are loaded in the scatter. s_off (LDS, nstrips + 1 ints) holds the image's strip offsets,
// written by the caller before the first barrier.
//
// Every prefetch load of an existing strip is issued unconditionally (slots past the strip's end
// read record 0 and visibility 0 of the image, in bounds whenever B > 0) and whether a slot holds
// a placement is decided where it is consumed, from the strip offsets, so the loads are never
// folded into branches. With B = 0 (no visibilities, an empty placement list) nothing is
// requested: `pf_strips` is nstrips when B > 0, else 0.
// With the strip store one straight run of stores, the number of memory operations after each
// prefetch is fixed: consuming a prefetched value waits only for the loads before it, never for
// the previous strip's stores (the memory counter is in order), and those stores drain while the
// next strip is gridded and transformed.
// Placement records per thread that the strip loop requests one strip ahead.
constexpr int kColPrefetch = 2;

template <int PF>
struct StripPrefetch {
  int2 r[PF];       // placement records of slots threadIdx.x + j*NT of the strip
  float2 v[PF];     // their visibilities (requested by prefetch_vis)
};

template <int PF, int NT>
__device__ __forceinline__ bool prefetch_slot_used(const int* s_off, int strip, int nstrips, int j) {
  return strip < nstrips && s_off[strip] + (int)threadIdx.x + j * NT < s_off[strip + 1];
}

template <int PF, int NT>
__device__ __forceinline__ void prefetch_records(const int2* __restrict__ plc, const int* s_off, int strip,
                                                 int nstrips, StripPrefetch<PF>& p) {
  if (strip >= nstrips) return;   // nothing left to request (uniform over the workgroup)
#pragma unroll
  for (int j = 0; j < PF; ++j)
    p.r[j] = plc[prefetch_slot_used<PF, NT>(s_off, strip, nstrips, j) ? s_off[strip] + (int)threadIdx.x + j * NT : 0];
}

template <int PF, int NT>
__device__ __forceinline__ void prefetch_vis(const float2* __restrict__ V, const int* s_off, int strip, int nstrips,
                                             StripPrefetch<PF>& p) {
  if (strip >= nstrips) return;
#pragma unroll
  for (int j = 0; j < PF; ++j)
    p.v[j] = V[prefetch_slot_used<PF, NT>(s_off, strip, nstrips, j) ? (p.r[j].y & 0x7fffffff) : 0];
}

template <int LOGN, int S, bool UNIFORM, int PREC, int NT, int PF>
__device__ __forceinline__ void grid_colfft_strips(const float2* __restrict__ V, const int2* __restrict__ plc,
                                                   const int* s_off, int strip0, int dstrip, int nstrips,
                                                   int pf_strips, bool shift, float2* __restrict__ Hi, int* occ_img,
                                                   const float2* __restrict__ tw, float2* sbuf, unsigned* scnt,
                                                   int* s_tmp, SplitCtx sp = {}) {
  using P = FftPlan<LOGN>;
  constexpr int N = P::N, NP = P::NP;
  constexpr bool SPLIT = PREC != kPrecFp32 && LOGN >= 4;
  // The FP32 form clears the strip buffer (and the counts of uniform weighting) once here and then
  // behind the reads of each strip's store (store_strip with ZERO) and of the division by the
  // counts (uniform_divide with CLEAR), which saves the clearing passes and a barrier per strip.
  constexpr bool ZERO_IN_STORE = !SPLIT;
  StripPrefetch<PF> cur, nxt;
  if constexpr (ZERO_IN_STORE) {
#pragma unroll 4
    for (int i = threadIdx.x; i < S * NP; i += NT) sbuf[i] = make_float2(0.f, 0.f);
    if constexpr (UNIFORM)
      for (int i = threadIdx.x; i < S * N; i += NT) scnt[i] = 0u;
    if (threadIdx.x == 0) *s_tmp = 0;
  }
  __syncthreads();   // s_off is visible (and the strip buffer zero)
  prefetch_records<PF, NT>(plc, s_off, strip0, pf_strips, cur);
  prefetch_vis<PF, NT>(V, s_off, strip0, pf_strips, cur);
  prefetch_records<PF, NT>(plc, s_off, strip0 + dstrip, pf_strips, nxt);
  // Wait for the prologue's loads here (vmcnt(0) only): the loop then starts every strip with
  // the same loads in flight whether it comes from here or from the previous strip, so the waits
  // inside it count past the previous strip's stores instead of draining them.
  __builtin_amdgcn_s_waitcnt(0x0F70);
  for (int strip = strip0; strip < nstrips; strip += dstrip) {
    if constexpr (!ZERO_IN_STORE) {
#pragma unroll 4
      for (int i = threadIdx.x; i < S * NP; i += NT) sbuf[i] = make_float2(0.f, 0.f);
      if constexpr (UNIFORM)
        for (int i = threadIdx.x; i < S * N; i += NT) scnt[i] = 0u;
      if (threadIdx.x == 0) {
        *s_tmp = 0;
        if constexpr (SPLIT) *sp.s_max = 0u;
      }
      __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < PF; ++j)
      if (prefetch_slot_used<PF, NT>(s_off, strip, nstrips, j))
        place_one<LOGN, S, true, UNIFORM>(cur.r[j], cur.v[j], strip, NP, shift, sbuf, scnt);
    const int o1 = s_off[strip + 1];
    scatter_strip<LOGN, S, true, UNIFORM>(plc, cmin(s_off[strip] + PF * NT, o1), o1, V, strip, NP, shift, sbuf,
                                          scnt);
    __syncthreads();
    if constexpr (UNIFORM) {
      int occ = uniform_divide<LOGN, S, true, NT, ZERO_IN_STORE>(sbuf, scnt, NP, strip == 0 ? 1 : 2, 2);
      block_add_to_global(occ, s_tmp, occ_img);
      __syncthreads();
    }
    // requests for the next strips, answered during this strip's transform and store
#pragma unroll
    for (int j = 0; j < PF; ++j) cur.r[j] = nxt.r[j];
    prefetch_vis<PF, NT>(V, s_off, strip + dstrip, pf_strips, cur);
    prefetch_records<PF, NT>(plc, s_off, strip + 2 * dstrip, pf_strips, nxt);
    strip_fft_store<LOGN, S, PREC, NT, true, ZERO_IN_STORE>(sbuf, strip, Hi, tw, sp);
    __syncthreads();   // the store's reads (and clears) of the strip buffer are done before it is reused
  }
}

// ---------------------------------------------------------------- row task
// Row-pair transforms j < TPB of row block `rowblk` of one image: rows y1 = 2r, y2 = 2r + 1 with
// r = rowblk*TPB + j. Z[e] = Hf1[e] + i Hf2[e], where Hf is the Hermitian extension of a stored
// half row: Hf[0] = Re H[0], Hf[N/2] = Im H[0], Hf[e] = H[e] (0 < e < N/2), Hf[e] = conj H[N-e].
// The inverse FFT of Z is I1 + i I2 with both rows real; they are scaled by `scale` and stored.
// The caller makes `tw` visible to the whole workgroup before the FFT's first barrier. With a
// split PREC the workgroup is whole waves and `sp` is that form's context (as for the column
// task, consecutive calls are separated by a workgroup barrier). A non-null `corr` (N values)
// multiplies pixel (y, x) by corr[y] corr[x] (the convolutional path's grid correction).
// Pixels are written with non-temporal stores: nothing in the path reads them again, and keeping
// them out of the caches leaves the last-level cache to the half spectra that the launches of
// the image group read and write. H columns at or beyond `ext` hold no placement and the column
// pass does not write them: they are read as zero, without a memory access where the rows of a
// transform are uniform over the wavefront (buffer loads whose range ends at the extent), and
// otherwise from a column the other lanes read too, masked to zero afterwards. Either way the
// loads stay unconditional, so they are all in flight before the first wait.
__device__ __forceinline__ float2 hermitian_combine(float2 a, float2 b, int e, int HALF) {
  if (e == 0) return make_float2(a.x, b.x);
  if (e == HALF) return make_float2(a.y, b.y);
  if (e < HALF) return make_float2(a.x - b.y, a.y + b.x);
  return make_float2(a.x + b.y, b.x - a.y);
}

__device__ __forceinline__ int hermitian_index(int e, int HALF) {
  return (e < HALF) ? e : ((e == HALF) ? 0 : 2 * HALF - e);
}

__device__ __forceinline__ float2 masked(float2 a, unsigned keep) {
  return make_float2(__uint_as_float(__float_as_uint(a.x) & keep), __uint_as_float(__float_as_uint(a.y) & keep));
}

__device__ __forceinline__ float2 hermitian_pair(const float2* __restrict__ h1, const float2* __restrict__ h2, int e,
                                                 int N, int ext) {
  const int HALF = N / 2;
  const int idx = hermitian_index(e, HALF);
  const bool live = idx < ext;
  const int at = live ? idx : 0;
  const unsigned keep = 0u - (unsigned)live;
  return hermitian_combine(masked(h1[at], keep), masked(h2[at], keep), e, HALF);
}

// Buffer resource over the first `ext` columns of a stored half row (base and size uniform over
// the wavefront); a load past the size returns zero without touching memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t half_row_rsrc(const float2* row, int ext) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float2*>(row), (short)0, ext * (int)sizeof(float2),
                                           kBufferRsrcWord3);
}

__device__ __forceinline__ float2 half_row_load(__amdgpu_buffer_rsrc_t r, int idx) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, idx * (int)sizeof(float2), 0, 0));
}

// The first stage's inputs of the row-pair transform of rows 2r, 2r + 1 held by this thread:
// v[m] = Z[lt + T m], Z the Hermitian-extended pair (see row_task). Threads with active == false
// load nothing (the T = 64 form takes every lane of the wavefront, which is one transform).
template <int LOGN>
__device__ __forceinline__ void load_row_pair(const float2* __restrict__ H, int r, int lt, bool active, int ext,
                                              float2 (&v)[FftPlan<LOGN>::R]) {
  using P = FftPlan<LOGN>;
  constexpr int N = P::N, T = P::T, HALF = N / 2;
  const float2* h1 = H + (size_t)(2 * r) * HALF;
  const float2* h2 = h1 + HALF;
  if constexpr (T == 64) {
    // One wavefront per transform (N = 1024). Lane lt loads only its columns below N/2
    // (e = lt + 64 m, m < R/2) and takes the values of the columns above, Z[N - e], from lane
    // 64 - lt, which loaded column N - e's half-row entries as its own: one cross-lane read per
    // float (ds_bpermute, no memory access) instead of loading every entry twice.
    const int ru = __builtin_amdgcn_readfirstlane(r);
    const float2* g1 = H + (size_t)(2 * ru) * HALF;
    const __amdgpu_buffer_rsrc_t r1 = half_row_rsrc(g1, cmin(ext, HALF));
    const __amdgpu_buffer_rsrc_t r2 = half_row_rsrc(g1 + HALF, cmin(ext, HALF));
    constexpr int HR = P::R / 2;
    float2 zm[HR];                         // Z at N - e of this lane's columns e
    float2 a0 = make_float2(0.f, 0.f), b0 = a0;
#pragma unroll
    for (int m = 0; m < HR; ++m) {
      const int e = lt + m * T;
      const float2 a = half_row_load(r1, e), b = half_row_load(r2, e);
      v[m] = hermitian_combine(a, b, e, HALF);
      zm[m] = make_float2(a.x + b.y, b.x - a.y);
      if (m == 0) {
        a0 = a;
        b0 = b;
      }
    }
    const int src = ((T - lt) & (T - 1)) << 2;
#pragma unroll
    for (int m = HR; m < P::R; ++m) {
      const float2 z = zm[P::R - 1 - m];
      v[m] = make_float2(__int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(z.x))),
                         __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(z.y))));
    }
    if (lt == 0) {                         // columns N/2 and N - 64 m are this lane's own
      v[HR] = make_float2(a0.y, b0.y);
#pragma unroll
      for (int m = HR + 1; m < P::R; ++m) v[m] = zm[P::R - m];
    }
  } else if constexpr (T % 64 == 0) {
    // a transform spans whole wavefronts: its two rows are the same for every lane of one
    const int ru = __builtin_amdgcn_readfirstlane(r);
    const float2* g1 = H + (size_t)(2 * ru) * HALF;
    const __amdgpu_buffer_rsrc_t r1 = half_row_rsrc(g1, cmin(ext, HALF));
    const __amdgpu_buffer_rsrc_t r2 = half_row_rsrc(g1 + HALF, cmin(ext, HALF));
    if (active) {
#pragma unroll
      for (int m = 0; m < P::R; ++m) {
        const int e = lt + m * T, idx = hermitian_index(e, HALF);
        v[m] = hermitian_combine(half_row_load(r1, idx), half_row_load(r2, idx), e, HALF);
      }
    }
  } else if (active) {
#pragma unroll
    for (int m = 0; m < P::R; ++m) v[m] = hermitian_pair(h1, h2, lt + m * T, N, ext);
  }
}

template <int LOGN, int TPB, int PREC = kPrecFp32>
__device__ __forceinline__ void row_task(const float2* __restrict__ H, int rowblk, float scale, float* __restrict__ out,
                                         const float2* __restrict__ tw, float2* sbuf, SplitCtx sp = {},
                                         const float* __restrict__ corr = nullptr, int ext = 1 << 30) {
  using P = FftPlan<LOGN>;
  constexpr int N = P::N, T = P::T, NP = P::NP;
  if constexpr (PREC != kPrecFp32 && LOGN >= 4) {
    // Z of every transform is loaded as in the FP32 form (one transform per T threads) and staged
    // into the row buffer, from which the matrix-core stages read their operands.
    {
      const int j = (int)threadIdx.x / T, lt = (int)threadIdx.x % T;
      const bool active = j < TPB;
      float2 v[P::R];
      load_row_pair<LOGN>(H, rowblk * TPB + (active ? j : 0), lt, active, ext, v);
      if (threadIdx.x == 0) *sp.s_max = 0u;
      if (active) {
#pragma unroll
        for (int m = 0; m < P::R; ++m) sbuf[j * NP + pad_index(lt + m * T)] = v[m];
      }
    }
    __syncthreads();   // the staged rows and the caller's twiddle table are visible
    float* ob = out + (size_t)(2 * rowblk * TPB) * N;
    auto load = [](int, int) { return make_float2(0.f, 0.f); };   // unused: the inputs are in sbuf
    if (corr) {
      fft_inverse_split<LOGN, PREC, false, true>(sbuf, TPB, tw, load, [&](int c, int e, float2 z) {
        const int y1 = 2 * (rowblk * TPB + c);
        float* o1 = ob + (size_t)(2 * c) * N;
        const float cx = corr[e] * scale;
        __builtin_nontemporal_store(z.x * cx * corr[y1], &o1[e]);
        __builtin_nontemporal_store(z.y * cx * corr[y1 + 1], &o1[N + e]);
      }, sp);
    } else {
      fft_inverse_split<LOGN, PREC, false, true>(sbuf, TPB, tw, load, [&](int c, int e, float2 z) {
        float* o1 = ob + (size_t)(2 * c) * N;
        __builtin_nontemporal_store(z.x * scale, &o1[e]);
        __builtin_nontemporal_store(z.y * scale, &o1[N + e]);
      }, sp);
    }
  } else {
    const int j = (int)threadIdx.x / T, lt = (int)threadIdx.x % T;
    const bool active = j < TPB;
    const int r = rowblk * TPB + (active ? j : 0);
    float2 v[P::R];
    load_row_pair<LOGN>(H, r, lt, active, ext, v);
    __syncthreads();   // the caller's twiddle table is visible
    float* o1 = out + (size_t)(2 * r) * N;
    float* o2 = o1 + N;
    float2* buf = sbuf + (active ? j : 0) * NP;
    if (corr) {
      const float s1 = scale * corr[2 * r], s2 = scale * corr[2 * r + 1];
      fft_inverse<LOGN, false>(v, buf, tw, lt, [&](int e, float2 z) {
        const float cx = corr[e];
        __builtin_nontemporal_store(z.x * s1 * cx, &o1[e]);
        __builtin_nontemporal_store(z.y * s2 * cx, &o2[e]);
      }, active);
    } else {
      fft_inverse<LOGN, false>(v, buf, tw, lt, [&](int e, float2 z) {
        __builtin_nontemporal_store(z.x * scale, &o1[e]);
        __builtin_nontemporal_store(z.y * scale, &o2[e]);
      }, active);
    }
  }
}

__device__ __forceinline__ float inverse_weight(double W) {
  return (W > 0.0 && isfinite(W)) ? (float)(1.0 / W) : 0.f;
}

}  // namespace blink
