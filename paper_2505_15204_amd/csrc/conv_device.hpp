// conv_device.hpp — convolutional gridding for the fused path (a step beyond the paper: Section
// 6.2.4 places each visibility on its nearest cell with no convolution kernel and names a kernel
// as the planned remedy for aliasing; Section 10 lists it as work in progress).
//
// Kernel: the "exponential of semicircle" of Barnett, Magland and af Klinteberg (2019),
//     phi(z) = exp(beta (sqrt(1 - z^2) - 1)) for |z| < 1, else 0,   z = 2 d / W,
// applied separably in u and v for a cell offset d and a support of W cells. A kept visibility at
// cell position (x, y) = (u k, v k) (the same FP64 product and keep rule as nearest-cell
// gridding) adds phi(2 (ju - x)/W) phi(2 (jv - y)/W) V to every cell (ju, jv) with |ju - x| < W/2
// and |jv - y| < W/2, cells wrapping modulo N; conj(V) spreads the same way around (-x, -y).
// Natural weighting (W_sum = 2 x kept). The image is afterwards divided by c(X/N) c(Y/N), c the
// kernel's continuous Fourier transform (grid correction, applied in the row pass).
//
// Fused layout: the binning pass writes one 16-byte record per (placement, column strip it
// reaches); a record holds the first tap cell of each axis and its offset from the exact
// position, so the column pass can evaluate the taps of its own columns. The half-spectrum
// columns 0 .. N/2 - 1 are transformed; taps on column N/2 (the Nyquist column) are added to
// column 0 times i, whose transform is then (Re: column 0, Im: column N/2), both real because
// the spread grid is Hermitian by construction.
#pragma once

#include <hip/hip_runtime.h>

#include "imaging_device.hpp"

namespace blink {

constexpr int kConvMaxWidth = 16;

struct ConvRec {
  int cells;    // (ju0 + 32768) | (jv0 + 32768) << 16: first tap column and row (signed)
  int bconj;    // baseline | conj << 31
  float du0;    // ju0 - x
  float dv0;    // jv0 - y
};

struct ConvSpec {
  int width;    // W, support in cells (1 .. 16, < N/2)
  float beta;
};

__device__ __forceinline__ float es_weight(float d, float two_over_w, float beta) {
  const float z = d * two_over_w;
  const float q = 1.f - z * z;
  return q > 0.f ? __expf(beta * (sqrtf(q) - 1.f)) : 0.f;
}

// First tap cell j0 (the smallest integer with j0 - x > -W/2) and its offset, in FP64.
__device__ __forceinline__ int first_tap(double x, double h, double* d0) {
  double j = ceil(x - h);
  if (!(j - x > -h)) j += 1.0;
  *d0 = j - x;
  return (int)j;
}

// Strip of half-spectrum column ku for strips of width 2^log_strip: columns 0 .. N/2-1 map to
// their strip, the Nyquist column N/2 to strip 0, the rest (negative u) to -1.
__device__ __forceinline__ int conv_strip_of(int ku, int half_n, int log_strip) {
  if (ku < half_n) return ku >> log_strip;
  return ku == half_n ? 0 : -1;
}

// Calls f(strip) once for every strip the tap columns j0 .. j0+n-1 reach (each strip's columns
// are one contiguous run because W < N/2).
template <class F>
__device__ __forceinline__ void for_each_conv_strip(int j0, int n, int N, int log_strip, F f) {
  int prev = -2;
  for (int j = 0; j < n; ++j) {
    const int s = conv_strip_of((j0 + j) & (N - 1), N / 2, log_strip);
    if (s >= 0 && s != prev) f(s);
    prev = s;
  }
}

// Binning for convolutional gridding (one workgroup per visibility set): keep rule and counts as
// bin_visibilities, then one ConvRec per (placement, strip reached), counting-sorted by strip.
// rec holds at most 2 B (ceil(W / 2^log_strip) + 2) records; off[0..nstrips] gets the offsets.
__device__ inline void bin_visibilities_conv(const double* __restrict__ uvw, const uint8_t* __restrict__ fl, int B,
                                             double k, int logn, int log_strip, ConvSpec cs, ConvRec* __restrict__ rec,
                                             int* __restrict__ off, int* kept_out, int* nout_out, BinShared& sh,
                                             int* ext_out = nullptr) {
  const int N = 1 << logn;
  const int nstrips = (N / 2) >> log_strip;
  const double half = (double)(N / 2), h = 0.5 * cs.width;
  for (int i = threadIdx.x; i <= nstrips; i += blockDim.x) sh.cnt[i] = 0;
  if (threadIdx.x < 3) sh.red[threadIdx.x] = 0;
  __syncthreads();
  int kept = 0, outside = 0;
  // pass 1: counts per strip
  for (int b = threadIdx.x; b < B; b += blockDim.x) {
    if (fl && fl[b]) continue;
    const double x = uvw[3 * b] * k, y = uvw[3 * b + 1] * k;
    const double ru = rint(x), rv = rint(y);
    if (!(fabs(ru) < half && fabs(rv) < half)) {
      ++outside;
      continue;
    }
    ++kept;
    for (int m = 0; m < 2; ++m) {
      const double xs = m ? -x : x;
      double d0;
      const int j0 = first_tap(xs, h, &d0);
      int n = 0;
      while (n < cs.width && d0 + n < h) ++n;
      for_each_conv_strip(j0, n, N, log_strip, [&](int s) { atomicAdd(&sh.cnt[s], 1); });
    }
  }
  if (kept) atomicAdd(&sh.red[0], kept);
  if (outside) atomicAdd(&sh.red[1], outside);
  __syncthreads();
  // column extent: the end of the last strip any tap reaches (read before the scan's first barrier)
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
  // pass 2: records
  for (int b = threadIdx.x; b < B; b += blockDim.x) {
    if (fl && fl[b]) continue;
    const double x = uvw[3 * b] * k, y = uvw[3 * b + 1] * k;
    const double ru = rint(x), rv = rint(y);
    if (!(fabs(ru) < half && fabs(rv) < half)) continue;
    for (int m = 0; m < 2; ++m) {
      const double xs = m ? -x : x, ys = m ? -y : y;
      double du, dv;
      const int ju0 = first_tap(xs, h, &du);
      const int jv0 = first_tap(ys, h, &dv);
      int n = 0;
      while (n < cs.width && du + n < h) ++n;
      ConvRec r;
      r.cells = (int)((unsigned)(ju0 + 32768) | ((unsigned)(jv0 + 32768) << 16));
      r.bconj = (int)((unsigned)b | (m ? 0x80000000u : 0u));
      r.du0 = (float)du;
      r.dv0 = (float)dv;
      for_each_conv_strip(ju0, n, N, log_strip, [&](int s) { rec[atomicAdd(&sh.cnt[s], 1)] = r; });
    }
  }
}

// Spreads the records [o0, o1) of strip `strip` (S columns) into the LDS strip buffer (column c
// at sbuf[c*NP + pad(kv)]), with the (-1)^(ku+kv) modulation when `modulate`.
template <int LOGN, int S>
__device__ __forceinline__ void scatter_strip_conv(const ConvRec* __restrict__ rec, int o0, int o1,
                                                   const float2* __restrict__ V, int strip, bool modulate,
                                                   ConvSpec cs, float2* sbuf) {
  constexpr int N = 1 << LOGN, NP = padded_len(N), HALF = N / 2;
  const float h = 0.5f * cs.width, tw = 2.f / cs.width;
  const int c_lo = strip * S;
  for (int i = o0 + (int)threadIdx.x; i < o1; i += blockDim.x) {
    const ConvRec r = rec[i];
    const int b = r.bconj & 0x7fffffff;
    float2 val = V[b];
    if (r.bconj < 0) val.y = -val.y;
    const int ju0 = (int)((unsigned)r.cells & 0xffffu) - 32768, jv0 = (int)((unsigned)r.cells >> 16) - 32768;
    float wv[kConvMaxWidth];
    int nv = 0;
#pragma unroll
    for (int t = 0; t < kConvMaxWidth; ++t) {
      const float d = r.dv0 + t;
      const bool in = t < cs.width && d < h;
      wv[t] = in ? es_weight(d, tw, cs.beta) : 0.f;
      nv += in ? 1 : 0;
    }
    for (int j = 0; j < cs.width; ++j) {
      const float du = r.du0 + j;
      if (!(du < h)) break;
      const int ku = (ju0 + j) & (N - 1);
      int col;
      bool nyq = false;
      if (ku >= c_lo && ku < c_lo + S) col = ku - c_lo;
      else if (strip == 0 && ku == HALF) { col = 0; nyq = true; }
      else continue;
      const float wu = es_weight(du, tw, cs.beta);
      float2 cu = make_float2(val.x * wu, val.y * wu);
      if (nyq) cu = make_float2(-cu.y, cu.x);          // packed as i * column N/2
      float* base = &sbuf[col * NP].x;
#pragma unroll
      for (int t = 0; t < kConvMaxWidth; ++t) {   // unrolled: wv stays in registers
        if (t >= nv) break;
        const int kv = (jv0 + t) & (N - 1);
        float sx = cu.x * wv[t], sy = cu.y * wv[t];
        if (modulate && ((ku + kv) & 1)) {
          sx = -sx;
          sy = -sy;
        }
        float* p = base + 2 * pad_index(kv);
        atomicAdd(p, sx);
        atomicAdd(p + 1, sy);
      }
    }
  }
}

// The same with one wave per record: lane l takes tap (row l / 8, column l % 8) for W <= 8, or
// four passes over a 16 x 16 tap tile for larger W, so a record's taps are issued as one wave of
// independent LDS atomics. Needs a workgroup of whole waves (NT a multiple of 64).
template <int LOGN, int S, int NT>
__device__ __forceinline__ void scatter_strip_conv_waves(const ConvRec* __restrict__ rec, int o0, int o1,
                                                         const float2* __restrict__ V, int strip, bool modulate,
                                                         ConvSpec cs, float2* sbuf) {
  static_assert(NT % 64 == 0, "whole waves");
  constexpr int N = 1 << LOGN, NP = padded_len(N), HALF = N / 2, NW = NT / 64;
  const float h = 0.5f * cs.width, tw = 2.f / cs.width;
  const int c_lo = strip * S;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tile = cs.width <= 8 ? 8 : 16, passes = cs.width <= 8 ? 1 : 4;
  for (int i = o0 + wave; i < o1; i += NW) {
    const ConvRec r = rec[i];
    const int b = r.bconj & 0x7fffffff;
    float2 val = V[b];
    if (r.bconj < 0) val.y = -val.y;
    const int ju0 = (int)((unsigned)r.cells & 0xffffu) - 32768, jv0 = (int)((unsigned)r.cells >> 16) - 32768;
    for (int p = 0; p < passes; ++p) {
      const int t = p * 64 + lane;
      const int ti = t / tile, tj = t % tile;
      const float du = r.du0 + tj, dv = r.dv0 + ti;
      if (ti >= cs.width || tj >= cs.width || !(du < h) || !(dv < h)) continue;
      const int ku = (ju0 + tj) & (N - 1);
      int col;
      bool nyq = false;
      if (ku >= c_lo && ku < c_lo + S) col = ku - c_lo;
      else if (strip == 0 && ku == HALF) { col = 0; nyq = true; }
      else continue;
      const int kv = (jv0 + ti) & (N - 1);
      const float w = es_weight(du, tw, cs.beta) * es_weight(dv, tw, cs.beta);
      float sx = val.x * w, sy = val.y * w;
      if (nyq) {                                      // packed as i * column N/2
        const float t0 = sx;
        sx = -sy;
        sy = t0;
      }
      if (modulate && ((ku + kv) & 1)) {
        sx = -sx;
        sy = -sy;
      }
      float* q = &sbuf[col * NP + pad_index(kv)].x;
      atomicAdd(q, sx);
      atomicAdd(q + 1, sy);
    }
  }
}

// ---------------------------------------------------------------- fused conv gridding + column FFT
// One strip of S half-spectrum columns of one image: zero the LDS strip, spread the strip's
// records, transform the columns and store the strip into Hi (column 0 keeps the packed Nyquist
// column). NT is the workgroup size.
template <int LOGN, int S, int PREC, int NT>
__device__ __forceinline__ void grid_colfft_conv_task(const float2* __restrict__ V, const ConvRec* __restrict__ rec,
                                                      int o0, int o1, int strip, bool shift, ConvSpec cs,
                                                      float2* __restrict__ Hi, const float2* __restrict__ tw,
                                                      float2* sbuf, SplitCtx sp) {
  constexpr int NP = padded_len(1 << LOGN);
  constexpr bool SPLIT = PREC != kPrecFp32 && LOGN >= 4;
#pragma unroll 4
  for (int i = threadIdx.x; i < S * NP; i += NT) sbuf[i] = make_float2(0.f, 0.f);
  if constexpr (SPLIT) {
    if (threadIdx.x == 0) *sp.s_max = 0u;
  }
  __syncthreads();
  if constexpr (NT % 64 == 0) scatter_strip_conv_waves<LOGN, S, NT>(rec, o0, o1, V, strip, shift, cs, sbuf);
  else scatter_strip_conv<LOGN, S>(rec, o0, o1, V, strip, shift, cs, sbuf);
  __syncthreads();
  strip_fft_store<LOGN, S, PREC, NT, false>(sbuf, strip, Hi, tw, sp);
}

// Grid correction of one axis: corr[x] = 1 / c(X/N), X the signed offset of pixel x from the
// phase centre (x - N/2 when shifted, else x below N/2 and x - N above), with
// c(nu) = W * integral_0^{pi/2} exp(beta (cos t - 1)) cos(pi nu W sin t) cos t dt (the kernel's
// transform after d = (W/2) sin t), by composite Simpson's rule on 8192 intervals in FP64.
// One workgroup of 256 threads per pixel.
constexpr int kCorrIntervals = 8192;

__device__ inline void conv_correction_entry(float* corr, int N, int x, int width, double beta, int shift,
                                             double* s_part) {
  const int X = shift ? x - N / 2 : (x < N / 2 ? x : x - N);
  const double nu = (double)X / N;
  const double h = (M_PI / 2.0) / kCorrIntervals;
  double s = 0.0;
  for (int i = threadIdx.x; i <= kCorrIntervals; i += blockDim.x) {
    double st, ct;
    sincos(i * h, &st, &ct);
    const double f = exp(beta * (ct - 1.0)) * cos(M_PI * nu * width * st) * ct;
    const double w = (i == 0 || i == kCorrIntervals) ? 1.0 : ((i & 1) ? 4.0 : 2.0);
    s += w * f;
  }
  s_part[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s_part[threadIdx.x] += s_part[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double c = (double)width * s_part[0] * h / 3.0;
    corr[x] = (float)(1.0 / c);
  }
}

}  // namespace blink
