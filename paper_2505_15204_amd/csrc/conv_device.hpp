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
// reaches, and for 64 <= N <= 1024 row band of 16 rows it reaches); a record holds the first tap
// cell of each axis and its offset from the exact position, so the column pass can evaluate the
// taps of its own cells. With row bands the column pass spreads on the matrix cores: the taps of a
// band are a sum of outer products (row weights x column-weighted visibilities), four records
// per v_mfma_f32_16x16x4_f32; otherwise each tap is an LDS atomic add. The half-spectrum
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

// A padding record of the banded binning: baseline field all ones (no visibility is read) and
// offsets that put every tap outside the support.
constexpr ConvRec kConvPad = {(int)0x80008000u, -1, 1.0e30f, 1.0e30f};

struct ConvSpec {
  int width;    // W, support in cells (1 .. 16, < N/2)
  float beta;
};

// The kernel value in FP32. The exponent beta (sqrt(1 - z^2) - 1) is formed as
// -beta z^2 / (1 + sqrt(1 - z^2)), which has no cancellation near z = 0, so the hardware square
// root and reciprocal (each within about one unit in the last place) leave the exponent with a
// relative error of a few units, and the weight with a relative error below 1e-6 where it is
// above exp(-beta / 4).
__device__ __forceinline__ float es_weight(float d, float two_over_w, float beta) {
  const float z = d * two_over_w;
  const float z2 = z * z;
  const float q = 1.f - z2;
  return q > 0.f ? __expf(-beta * z2 * __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_sqrtf(q))) : 0.f;
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

// Row bands of the matrix-core spreading (spread_strip_conv_mfma): 16 rows, one tile of
// v_mfma_f32_16x16x4_f32, for 64 <= N <= 1024, where (column strips) x (bands) stays within the
// binning's counters and the column workgroup is whole waves. Other sizes keep one band, the
// whole column, and spread with LDS atomics per tap.
__host__ __device__ constexpr int conv_log_band(int logn) { return (logn >= 6 && logn <= 10) ? 4 : logn; }

// Calls f(band) once for every band of height 2^log_band >= 16 that the tap rows j0 .. j0+n-1
// (modulo N, n <= 16) reach: the bands of the first and the last row.
template <class F>
__device__ __forceinline__ void for_each_conv_band(int j0, int n, int N, int log_band, F f) {
  if (n <= 0) return;
  const int b0 = (j0 & (N - 1)) >> log_band, b1 = ((j0 + n - 1) & (N - 1)) >> log_band;
  f(b0);
  if (b1 != b0) f(b1);
}

// Number of taps j < W with d0 + j < h (d0 in (-h, 1 - h]): the integers below h - d0, which is
// exact in FP64 here.
__device__ __forceinline__ int conv_taps(double d0, double h, int width) {
  const int n = (int)ceil(h - d0);
  return n < width ? n : width;
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
// bin_visibilities, then one ConvRec per (placement, strip reached, row band reached),
// counting-sorted by bin = strip * nb + band with nb = N >> log_band bands per column
// (2 nstrips nb < kMaxStrips). rec holds at most conv_records_per_pair records; off[0..nbins]
// gets the offsets, so the records of strip s are off[s nb] .. off[(s + 1) nb]. With more than
// one band every bin is padded to a multiple of four records with kConvPad records (no tap, no
// visibility), so that the matrix-core spreading's groups of four never straddle two bands.
__device__ inline void bin_visibilities_conv(const double* __restrict__ uvw, const uint8_t* __restrict__ fl, int B,
                                             double k, int logn, int log_strip, int log_band, ConvSpec cs,
                                             ConvRec* __restrict__ rec, int* __restrict__ off, int* kept_out,
                                             int* nout_out, BinShared& sh, int* ext_out = nullptr) {
  const int N = 1 << logn;
  const int nstrips = (N / 2) >> log_strip, nb = N >> log_band, nbins = nstrips * nb;
  const double half = (double)(N / 2), h = 0.5 * cs.width;
  for (int i = threadIdx.x; i <= nbins; i += blockDim.x) sh.cnt[i] = 0;
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
      const double xs = m ? -x : x, ys = m ? -y : y;
      double du, dv;
      const int ju0 = first_tap(xs, h, &du);
      const int jv0 = first_tap(ys, h, &dv);
      const int nu = conv_taps(du, h, cs.width), nv = conv_taps(dv, h, cs.width);
      for_each_conv_strip(ju0, nu, N, log_strip, [&](int s) {
        for_each_conv_band(jv0, nv, N, log_band, [&](int bnd) { atomicAdd(&sh.cnt[s * nb + bnd], 1); });
      });
    }
  }
  if (kept) atomicAdd(&sh.red[0], kept);
  if (outside) atomicAdd(&sh.red[1], outside);
  __syncthreads();
  // column extent: the end of the last strip any tap reaches; the padding of each bin (kept in
  // cnt[nbins + 1 + i]) and the padded counts (read and written before the scan's first barrier)
  int* pad = sh.cnt + nbins + 1;
  for (int i = threadIdx.x; i < nbins; i += blockDim.x) {
    const int c = sh.cnt[i];
    if (ext_out && c > 0) atomicMax(&sh.red[2], i / nb + 1);
    const int p = nb > 1 ? (4 - (c & 3)) & 3 : 0;
    pad[i] = p;
    sh.cnt[i] = c + p;
  }
  __syncthreads();
  block_exclusive_scan(sh.cnt, nbins, sh.wave);
  for (int i = threadIdx.x; i <= nbins; i += blockDim.x) {
    const int o = sh.cnt[i];
    off[i] = o;
    if (i < nbins) {                       // the padding records open the bin
      for (int j = 0; j < pad[i]; ++j) rec[o + j] = kConvPad;
      sh.cnt[i] = o + pad[i];
    }
  }
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
      const int nu = conv_taps(du, h, cs.width), nv = conv_taps(dv, h, cs.width);
      ConvRec r;
      r.cells = (int)((unsigned)(ju0 + 32768) | ((unsigned)(jv0 + 32768) << 16));
      r.bconj = (int)((unsigned)b | (m ? 0x80000000u : 0u));
      r.du0 = (float)du;
      r.dv0 = (float)dv;
      for_each_conv_strip(ju0, nu, N, log_strip, [&](int s) {
        for_each_conv_band(jv0, nv, N, log_band, [&](int bnd) { rec[atomicAdd(&sh.cnt[s * nb + bnd], 1)] = r; });
      });
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

// Matrix-core spreading of one strip (S a multiple of 16 columns) from records binned by row
// band of 16 rows. The cells of band beta (rows 16 beta .. 16 beta + 15) receive the sum over the band's
// records r of wv_r(kv) * V_r wu_r(ku): the product of a 16 x R matrix of row weights and an
// R x S matrix of column-weighted visibilities, evaluated four records at a time with
// v_mfma_f32_16x16x4_f32 (FP32 products and sums) for the real and the imaginary parts. Lane
// l = 16 g + n supplies the row weight of row n and the value of column n of record g of the
// group, and receives rows 4 g + i (i < 4) of column n. Taps on the Nyquist column N/2 enter
// column 0 of strip 0 times i, as in the per-tap form.
//
// The bins are padded to groups of four, so a group lies in one band. Wave w takes the groups
// [w G / NW, (w + 1) G / NW) of the strip (G groups in all) and accumulates the groups of one band
// in registers. A band whose groups all lie in the wave's range is added to the LDS strip with a
// plain read-add-write when the wave leaves it; the first and the last band of the range can
// also hold groups of other waves, so their tiles stay in registers until the loop is over and
// are then added in turns with a workgroup barrier between turns: the waves whose ranges reach a
// band add their tiles of it in the order of their ranges (a wave's last band, when it differs
// from its first, begins inside its range, so the wave is that band's first contributor), and
// there are as many turns as the most waves that share one band (LDS float atomics, the
// alternative, cost several times a plain access and serialise where waves meet on a busy band).
// The (-1)^(ku + kv) modulation is a sign per cell, applied there. s_boff (LDS) holds the strip's
// NB + 1 band offsets into rec and, at s_boff[NB + 1], the turn count (zero on entry, visible).
// Every thread of the workgroup calls this.
constexpr int kConvBatch = 8;                  // groups whose records are requested together

template <int NB>
__device__ __forceinline__ void set_conv_bands(const int* __restrict__ so, int* s_boff) {
  for (int i = threadIdx.x; i <= NB; i += blockDim.x) s_boff[i] = so[i];
  if (threadIdx.x == 0) s_boff[NB + 1] = 0;   // the tile turns of spread_strip_conv_mfma
}

template <int LOGN, int S, int NT>
__device__ __forceinline__ void spread_strip_conv_mfma(const ConvRec* __restrict__ rec, int* s_boff,
                                                       const float2* __restrict__ V, int strip, bool modulate,
                                                       ConvSpec cs, float2* sbuf) {
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  constexpr int N = 1 << LOGN, NP = padded_len(N), NB = N >> conv_log_band(LOGN), CT = S / 16, NW = NT / 64;
  constexpr int GB = kConvBatch;
  static_assert(conv_log_band(LOGN) == 4 && S % 16 == 0 && NT % 64 == 0, "16-row bands, 16-column tiles, whole waves");
  const float h = 0.5f * cs.width, two_w = 2.f / cs.width;
  const int lane = threadIdx.x & 63, n = lane & 15, g = lane >> 4, wave = threadIdx.x >> 6;
  const int base = s_boff[0], ngroups = (s_boff[NB] - base) >> 2;
  const int q0 = (int)(((long long)ngroups * wave) / NW), q1 = (int)(((long long)ngroups * (wave + 1)) / NW);
  const bool active = q0 < q1;                // uniform over the wave
  // band of record i: the last band whose offset is at most i
  auto band_of = [&](int i) {
    int lo = 0, hi = NB;                      // s_boff[lo] <= i < s_boff[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_boff[mid] <= i) lo = mid;
      else hi = mid;
    }
    return lo;
  };
  const int first = active ? band_of(base + 4 * q0) : 0, last = active ? band_of(base + 4 * (q1 - 1)) : 0;
  int band = first;
  f32x4 acc[CT][2], acc_first[CT][2];
  auto clear = [&](f32x4 (&t)[CT][2]) {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int p = 0; p < 2; ++p) t[ct][p] = f32x4{0.f, 0.f, 0.f, 0.f};
  };
  auto flush = [&](int bnd, const f32x4 (&t)[CT][2]) {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int col = 16 * ct + n;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = 16 * bnd + 4 * g + q;
        float sx = t[ct][0][q], sy = t[ct][1][q];
        if (modulate && ((strip * S + col + row) & 1)) {
          sx = -sx;
          sy = -sy;
        }
        float2* p = &sbuf[col * NP + pad_index(row)];
        const float2 o = *p;
        *p = make_float2(o.x + sx, o.y + sy);
      }
    }
  };
  clear(acc);
  clear(acc_first);
  for (int qb = q0; qb < q1; qb += GB) {      // uniform over the wave
    // this lane's record of each group of the batch and its visibility, requested together
    ConvRec rr[GB];
    float2 vv[GB];
#pragma unroll
    for (int j = 0; j < GB; ++j) {
      const int q = qb + j < q1 ? qb + j : q0;
      rr[j] = rec[base + 4 * q + g];
    }
#pragma unroll
    for (int j = 0; j < GB; ++j) vv[j] = V[rr[j].bconj == -1 ? 0 : (rr[j].bconj & 0x7fffffff)];
#pragma unroll
    for (int j = 0; j < GB; ++j) {
      if (qb + j >= q1) break;                // uniform over the wave
      const int i0 = base + 4 * (qb + j);
      if (i0 >= s_boff[band + 1]) {           // the group opens a later band
        if (band == first) {
#pragma unroll
          for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int p = 0; p < 2; ++p) acc_first[ct][p] = acc[ct][p];
        } else {
          flush(band, acc);                   // a band of this wave alone
        }
        clear(acc);
        band = band_of(i0);
      }
      const ConvRec r = rr[j];
      const bool real = r.bconj != -1;
      float2 val = real ? vv[j] : make_float2(0.f, 0.f);
      if (r.bconj < 0) val.y = -val.y;
      const int ju0 = (int)((unsigned)r.cells & 0xffffu) - 32768, jv0 = (int)((unsigned)r.cells >> 16) - 32768;
      const int tv = (16 * band + n - jv0) & (N - 1);
      const float dv = r.dv0 + tv;
      const float a = (tv < cs.width && dv < h) ? es_weight(dv, two_w, cs.beta) : 0.f;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int ku = strip * S + 16 * ct + n;
        const int tu = (ku - ju0) & (N - 1);
        const float du = r.du0 + tu;
        const float wu = (tu < cs.width && du < h) ? es_weight(du, two_w, cs.beta) : 0.f;
        float wn = 0.f;
        if (ct == 0 && strip == 0 && n == 0) {  // column N/2, packed into column 0 times i
          const int tn = (N / 2 - ju0) & (N - 1);
          const float dn = r.du0 + tn;
          wn = (tn < cs.width && dn < h) ? es_weight(dn, two_w, cs.beta) : 0.f;
        }
        const float bre = val.x * wu - val.y * wn, bim = val.y * wu + val.x * wn;
        acc[ct][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bre, acc[ct][0], 0, 0, 0);
        acc[ct][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bim, acc[ct][1], 0, 0, 0);
      }
    }
  }
  // The first and the last band's tiles (acc holds the last). The turn of the first band's tile is
  // the number of earlier waves whose ranges reach that band (ranges are in wave order).
  int turn = 0;
  if (active) {
    const int gs = (s_boff[first] - base) >> 2;      // the band's first group
    for (int v = 0; v < wave; ++v) {
      const int a0 = (int)(((long long)ngroups * v) / NW), a1 = (int)(((long long)ngroups * (v + 1)) / NW);
      if (a0 < a1 && a1 > gs) ++turn;
    }
    if (lane == 0) atomicMax(&s_boff[NB + 1], turn + 1);
  }
  __syncthreads();
  const int turns = s_boff[NB + 1];
  for (int t = 0; t < turns; ++t) {
    if (t > 0) __syncthreads();
    if (active) {
      if (first != last) {
        if (t == turn) flush(first, acc_first);
        if (t == 0) flush(last, acc);
      } else if (t == turn) {
        flush(last, acc);
      }
    }
  }
}

// ---------------------------------------------------------------- fused conv gridding + column FFT
// One strip of S half-spectrum columns of one image: zero the LDS strip, spread the strip's
// records, transform the columns and store the strip into Hi (column 0 keeps the packed Nyquist
// column). NT is the workgroup size. so (global) holds the strip's NB + 1 band
// offsets into rec (NB = 1: one band); s_boff is NB + 2 ints of LDS.
template <int LOGN, int S, int PREC, int NT>
__device__ __forceinline__ void grid_colfft_conv_task(const float2* __restrict__ V, const ConvRec* __restrict__ rec,
                                                      const int* __restrict__ so, int* s_boff, int strip, bool shift,
                                                      ConvSpec cs, float2* __restrict__ Hi,
                                                      const float2* __restrict__ tw, float2* sbuf, SplitCtx sp) {
  constexpr int N = 1 << LOGN, NP = padded_len(N), NB = N >> conv_log_band(LOGN);
  constexpr bool SPLIT = PREC != kPrecFp32 && LOGN >= 4;
#pragma unroll 4
  for (int i = threadIdx.x; i < S * NP; i += NT) sbuf[i] = make_float2(0.f, 0.f);
  if constexpr (SPLIT) {
    if (threadIdx.x == 0) *sp.s_max = 0u;
  }
  set_conv_bands<NB>(so, s_boff);
  __syncthreads();
  if constexpr (NB > 1) spread_strip_conv_mfma<LOGN, S, NT>(rec, s_boff, V, strip, shift, cs, sbuf);
  else if constexpr (NT % 64 == 0) scatter_strip_conv_waves<LOGN, S, NT>(rec, s_boff[0], s_boff[1], V, strip, shift, cs, sbuf);
  else scatter_strip_conv<LOGN, S>(rec, s_boff[0], s_boff[1], V, strip, shift, cs, sbuf);
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
