// kernels.hip — gfx950 kernels of the batched dirty-imaging path.
//
//   k_twiddles       FP64 sincospi -> FP32 stage-ordered twiddle table
//   k_bin            cell indices (FP64 product + rint), flags, out-of-grid drop, counting sort
//                    of the placements into column strips (Section 6.2.4 gridding, one
//                    workgroup per (time, channel), shared by the polarisations)
//   k_grid_full      LDS-private strip grid -> complex grid in HBM (plain stores), counts
//   k_grid_colfft    LDS-private strip grid -> inverse FFT along v -> half-spectrum H
//   k_dense_colfft   Hermitian part of a dense grid -> inverse FFT along v -> H
//   k_row_c2r        two H rows -> Hermitian-extended inverse FFT along u -> two image rows,
//                    scaled by 1/W of the image (computed from the kept count or occupancy)
//   k_bin_conv, k_grid_colfft_conv, k_conv_correction
//                    the convolutional-gridding variant (conv_device.hpp)
//
// The dirty image is I = Re(IDFT2(G)) / W (Section 4, Eq. 5). The shift of Section 6.2.4 is
// folded into the input as the modulation (-1)^(ku + kv), which for even N moves the phase
// centre to pixel (N/2, N/2). Because the grid is Hermitian only the columns ku < N/2 are
// transformed along v; the row pass rebuilds the other half by symmetry, and H's column 0 packs
// the two real-valued columns ku = 0 (real part) and ku = N/2 (imaginary part).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace blink {

// ---------------------------------------------------------------- twiddles
// The stage-ordered table of one size N (fft_device.hpp): FP64 sincospi of an exact dyadic
// argument, rounded to FP32. Unused rows of A (m >= R1) hold zero.
__global__ void k_twiddles(float2* tw, int logn) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= tw_size(logn)) return;
  const int n = 1 << logn;
  const int r1 = logn <= 4 ? 1 : (logn >= 8 ? 16 : n / 16);
  long num = 0, den = 1;
  bool used = true;
  if (j < 256) {                      // A: row m, column k
    const int m = j / 16, k = j % 16;
    used = m < r1;
    num = (long)k * m;
    den = 16L * r1;
  } else if (j < kTwA) {              // D: 16-point DFT entries
    num = j - 256;
    den = 16;
  } else {                            // B: row m, column k
    const int m = (j - kTwA) / 256, k = (j - kTwA) % 256;
    num = (long)k * m;
    den = n;
  }
  double s = 0.0, c = 0.0;
  sincospi(2.0 * (double)(num % den) / (double)den, &s, &c);
  tw[j] = used ? make_float2((float)c, (float)s) : make_float2(0.f, 0.f);
}

int twiddle_table_size(int logn) { return tw_size(logn); }

// ---------------------------------------------------------------- split-form DFT operands
__global__ void k_dft_operands(const float2* __restrict__ tw, uint4* ops) {
  const int lane = threadIdx.x & 63;
  if (threadIdx.x < 64) make_dft_operands<kPrecSplitF16>(tw, ops, lane);
  else if (threadIdx.x < 128) make_dft_operands<kPrecSplitBf16>(tw, ops, lane);
}

hipError_t launch_dft_operands(const float2* tw, uint4* ops, hipStream_t s) {
  k_dft_operands<<<1, 128, 0, s>>>(tw, ops);
  return hipGetLastError();
}

hipError_t launch_twiddles(float2* tw, int logn, hipStream_t s) {
  const int n = tw_size(logn);
  k_twiddles<<<(n + 255) / 256, 256, 0, s>>>(tw, logn);
  return hipGetLastError();
}

// ---------------------------------------------------------------- binning
__global__ __launch_bounds__(kBinThreads) void k_bin(BinArgs a) {
  __shared__ BinShared sh;
  const int tcl = blockIdx.x;
  const long tc = (long)a.tc0 + tcl;
  const int t = (int)(tc / a.C), c = (int)(tc % a.C);
  const int N = 1 << a.logn;
  const int nstrips = a.ku_limit >> a.log_strip;
  const double k = (a.freq[c] / kSpeedOfLight) * ((double)N * a.pixel_scale);
  bin_visibilities(a.uvw + (size_t)t * a.B * 3, a.flags ? a.flags + (size_t)tc * a.B : nullptr, a.B, k, a.logn,
                   a.log_strip, a.ku_limit, a.plc + (size_t)tcl * 2 * a.B, a.strip_off + (size_t)tcl * (nstrips + 1),
                   a.n_kept + tcl, a.n_out ? a.n_out + tc : nullptr, a.cell_idx ? a.cell_idx + (size_t)tc * a.B : nullptr,
                   sh, a.ext ? a.ext + tcl : nullptr);
  if (threadIdx.x < a.P) a.occ[(size_t)tcl * a.P + threadIdx.x] = 0;
}

hipError_t launch_bin(const BinArgs& a, hipStream_t s) {
  if (a.Q <= 0) return hipSuccess;
  k_bin<<<a.Q, kBinThreads, 0, s>>>(a);
  return hipGetLastError();
}

// ---------------------------------------------------------------- convolutional binning
__global__ __launch_bounds__(kBinThreads) void k_bin_conv(BinArgs a, ConvSpec cs, int rec_stride) {
  __shared__ BinShared sh;
  const int tcl = blockIdx.x;
  const long tc = (long)a.tc0 + tcl;
  const int t = (int)(tc / a.C), c = (int)(tc % a.C);
  const int N = 1 << a.logn;
  const int nstrips = (N / 2) >> a.log_strip;
  const double k = (a.freq[c] / kSpeedOfLight) * ((double)N * a.pixel_scale);
  const int log_band = conv_log_band(a.logn), nb = N >> log_band;
  bin_visibilities_conv(a.uvw + (size_t)t * a.B * 3, a.flags ? a.flags + (size_t)tc * a.B : nullptr, a.B, k, a.logn,
                        a.log_strip, log_band, cs, reinterpret_cast<ConvRec*>(a.plc) + (size_t)tcl * rec_stride,
                        a.strip_off + (size_t)tcl * (nstrips * nb + 1), a.n_kept + tcl,
                        a.n_out ? a.n_out + tc : nullptr, sh, a.ext ? a.ext + tcl : nullptr);
}

// A placement's W < N/2 tap columns reach at most ceil(W / S) + 1 strips and its W <= 16 tap rows
// at most two 16-row bands; with bands every bin holds at most three padding records.
int conv_records_per_pair(int B, int width, int min_strip, int logn) {
  const bool banded = conv_log_band(logn) < logn;
  return 2 * B * ((width + min_strip - 1) / min_strip + 2) * (banded ? 2 : 1) +
         (banded ? 3 * conv_bins_per_pair(logn, min_strip) : 0);
}

int conv_bins_per_pair(int logn, int strip) { return ((1 << logn) / 2 / strip) * ((1 << logn) >> conv_log_band(logn)); }

hipError_t launch_bin_conv(const BinArgs& a, ConvParams cp, int rec_stride, hipStream_t s) {
  if (a.Q <= 0) return hipSuccess;
  k_bin_conv<<<a.Q, kBinThreads, 0, s>>>(a, ConvSpec{cp.width, (float)cp.beta}, rec_stride);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_conv_correction(float* corr, int n, int width, double beta, int shift) {
  __shared__ double s_part[256];
  conv_correction_entry(corr, n, blockIdx.x, width, beta, shift, s_part);
}

hipError_t launch_conv_correction(float* corr, int logn, ConvParams cp, int shift, hipStream_t s) {
  const int n = 1 << logn;
  k_conv_correction<<<n, 256, 0, s>>>(corr, n, cp.width, cp.beta, shift);
  return hipGetLastError();
}

template <int LOGN>
struct ConvStrip {
  static hipError_t run(int* out) {
    *out = ColSmax<LOGN, false>::value;
    return hipSuccess;
  }
};

int conv_strip_width(int logn) {
  int s = 0;
  return by_logn<ConvStrip>(logn, &s) == hipSuccess ? s : 0;
}

hipError_t launch_grid_colfft_conv(const ColArgs& a, int n_img, ConvParams cp, int prec, const float2* tw,
                                   hipStream_t s) {
  const float beta = (float)cp.beta;
  switch (prec) {
    case BLINK_PREC_FP32: return PrecLaunch<BLINK_PREC_FP32>::grid_colfft_conv(a, n_img, cp.width, beta, tw, s);
    case BLINK_PREC_SPLIT_F16:
      return PrecLaunch<BLINK_PREC_SPLIT_F16>::grid_colfft_conv(a, n_img, cp.width, beta, tw, s);
    case BLINK_PREC_SPLIT_BF16:
      return PrecLaunch<BLINK_PREC_SPLIT_BF16>::grid_colfft_conv(a, n_img, cp.width, beta, tw, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------- image averages
// Averages of images [T][C][P][N][N] over the axes in `axes` (1 time, 2 channel, 4 polarisation;
// Sections 7.2 and 7.3 average over time and over the band, the polarisation average of XX and YY
// is Stokes I). One thread per 4 consecutive pixels of one output image, FP64 sums.
// ---------------------------------------------------------------- visibility corrections
// Antenna pair (i, j), i > j, of baseline b = i (i - 1) / 2 + j: the lower-triangular order in
// which the correlation step stores visibilities (Section 6.2.2).
__device__ __forceinline__ void antenna_pair(long long b, int& i, int& j) {
  long long r = (long long)((1.0 + sqrt(1.0 + 8.0 * (double)b)) * 0.5);
  while (r * (r - 1) / 2 > b) --r;
  while ((r + 1) * r / 2 <= b) ++r;
  i = (int)r;
  j = (int)(b - r * (r - 1) / 2);
}

// One thread per (pair, baseline); the phase of the new phase centre is shared by the pols.
// Workgroup w covers baselines (w % nbx) * 256 .. of pair w / nbx.
__global__ __launch_bounds__(256) void k_correct_vis(CorrArgs a, int nbx) {
  const int q = (int)(blockIdx.x / (unsigned)nbx);
  const int b = (int)(blockIdx.x % (unsigned)nbx) * 256 + (int)threadIdx.x;
  if (b >= a.B) return;
  const long tc = (long)a.tc0 + q;
  const long t = tc / a.C, c = tc % a.C;
  const double* x = a.uvw + 3 * ((size_t)t * a.B + b);
  // geometric delay in turns (FP64), reduced exactly to [-1/2, 1/2]; the sine and cosine of the
  // reduced angle are taken in FP32 (|angle| <= pi, so their error is a few 1e-8)
  const double turns = (a.freq[c] / kSpeedOfLight) * (x[0] * a.l0 + x[1] * a.m0 + x[2] * a.n0m1);
  float snf, csf;
  sincospif((float)(2.0 * (turns - rint(turns))), &snf, &csf);
  const double sn = snf, cs = csf;
  int i = 0, j = 0;
  if (a.gains) antenna_pair(b, i, j);
  for (int p = 0; p < a.P; ++p) {
    const size_t at = ((size_t)q * a.P + p) * a.B + b;
    const float2 v = a.vis[at];
    double re = v.x, im = v.y;
    if (a.gains) {
      const float2 gi = a.gains[((size_t)c * a.P + p) * a.n_ant + i];
      const float2 gj = a.gains[((size_t)c * a.P + p) * a.n_ant + j];
      const double r1 = (double)gi.x * re - (double)gi.y * im, i1 = (double)gi.x * im + (double)gi.y * re;
      re = r1 * gj.x + i1 * gj.y;          // (r1 + i i1) conj(gj)
      im = i1 * gj.x - r1 * gj.y;
    }
    a.out[at] = make_float2((float)(re * cs - im * sn), (float)(re * sn + im * cs));
  }
}

hipError_t launch_correct_vis(const CorrArgs& a, hipStream_t s) {
  if (a.Q <= 0 || a.B <= 0) return hipSuccess;
  const long nbx = ((long)a.B + 255) / 256;
  if (nbx * a.Q > 0x7fffffffL) return hipErrorInvalidValue;
  k_correct_vis<<<(unsigned)(nbx * a.Q), 256, 0, s>>>(a, (int)nbx);
  return hipGetLastError();
}

// ---------------------------------------------------------------- de-dispersion
// out[k][t] = mean over c of in[t + delay[k][c]][c], four pixels per thread, FP64 sums in channel
// order (then one division by C and one rounding to float).
__global__ __launch_bounds__(256) void k_dedisperse(const float4* __restrict__ in, int C, long nn4,
                                                    const int* __restrict__ delays, int t_out,
                                                    float4* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn4) return;
  const int t = blockIdx.y, k = blockIdx.z;
  const int* dk = delays + (size_t)k * C;
  double sx = 0.0, sy = 0.0, sz = 0.0, sw = 0.0;
  for (int c = 0; c < C; ++c) {
    const float4 v = in[((size_t)(t + dk[c]) * C + c) * nn4 + i];
    sx += v.x;
    sy += v.y;
    sz += v.z;
    sw += v.w;
  }
  const double cd = (double)C;
  out[((size_t)k * t_out + t) * nn4 + i] = make_float4((float)(sx / cd), (float)(sy / cd), (float)(sz / cd),
                                                       (float)(sw / cd));
}

hipError_t launch_dedisperse(const float* in, int C, int logn, const int* delays, int n_dm, int t_out, float* out,
                             hipStream_t s) {
  const long nn4 = (1L << (2 * logn)) / 4;
  if (n_dm <= 0 || t_out <= 0) return hipSuccess;
  dim3 grid((unsigned)((nn4 + 255) / 256), (unsigned)t_out, (unsigned)n_dm);
  k_dedisperse<<<grid, 256, 0, s>>>((const float4*)in, C, nn4, delays, t_out, (float4*)out);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_image_average(const float4* __restrict__ in, int T, int C, int P, long nn4,
                                                       int axes, float4* __restrict__ out) {
  const int To = (axes & 1) ? 1 : T, Co = (axes & 2) ? 1 : C, Po = (axes & 4) ? 1 : P;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)To * Co * Po * nn4) return;
  const long img = gid / nn4, px = gid - img * nn4;
  const int po = (int)(img % Po), co = (int)((img / Po) % Co), to = (int)(img / ((long)Po * Co));
  const int t0 = (axes & 1) ? 0 : to, t1 = (axes & 1) ? T : to + 1;
  const int c0 = (axes & 2) ? 0 : co, c1 = (axes & 2) ? C : co + 1;
  const int p0 = (axes & 4) ? 0 : po, p1 = (axes & 4) ? P : po + 1;
  double ax = 0.0, ay = 0.0, az = 0.0, aw = 0.0;
  for (int t = t0; t < t1; ++t)
    for (int c = c0; c < c1; ++c)
      for (int p = p0; p < p1; ++p) {
        const float4 v = in[(((long)t * C + c) * P + p) * nn4 + px];
        ax += v.x;
        ay += v.y;
        az += v.z;
        aw += v.w;
      }
  const double inv = 1.0 / ((double)(t1 - t0) * (c1 - c0) * (p1 - p0));
  out[gid] = make_float4((float)(ax * inv), (float)(ay * inv), (float)(az * inv), (float)(aw * inv));
}

hipError_t launch_image_average(const float* in, int T, int C, int P, int logn, int axes, float* out, hipStream_t s) {
  const long nn4 = (1L << (2 * logn)) / 4;
  const long n_out = (long)((axes & 1) ? 1 : T) * ((axes & 2) ? 1 : C) * ((axes & 4) ? 1 : P) * nn4;
  if (n_out <= 0) return hipSuccess;
  k_image_average<<<(unsigned)((n_out + 255) / 256), 256, 0, s>>>((const float4*)in, T, C, P, nn4, axes,
                                                                    (float4*)out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- full grid (blink_grid)
template <int LOGN, bool UNIFORM>
__global__ __launch_bounds__(256) void k_grid_full(GridArgs a) {
  constexpr int N = 1 << LOGN;
  constexpr int S = GridCfg<LOGN>::S;
  __shared__ float2 sbuf[S * N];
  __shared__ unsigned scnt[S * N];
  __shared__ int s_tmp;
  const int img = blockIdx.x, strip = blockIdx.y;
  const int tcl = img / a.P, p = img - tcl * a.P;
  const int nstrips = N / S;
  for (int i = threadIdx.x; i < S * N; i += blockDim.x) {
    sbuf[i] = make_float2(0.f, 0.f);
    scnt[i] = 0u;
  }
  if (threadIdx.x == 0) s_tmp = 0;
  __syncthreads();
  const int* so = a.strip_off + (size_t)tcl * (nstrips + 1);
  scatter_strip<LOGN, S, false, true>(a.plc + (size_t)tcl * 2 * a.B, so[strip], so[strip + 1],
                                      a.vis + (size_t)img * a.B, strip, N, false, sbuf, scnt);
  __syncthreads();
  if constexpr (UNIFORM) {
    int occ = uniform_divide<LOGN, S, false>(sbuf, scnt, N, 1, 1);
    block_add_to_global(occ, &s_tmp, a.occ + img);
    __syncthreads();
  }
  float2* G = a.grids + (size_t)img * N * N;
  for (int i = threadIdx.x; i < S * N; i += blockDim.x) {
    const int kv = i / S, col = i % S;
    G[(size_t)kv * N + strip * S + col] = sbuf[col * N + kv];
  }
  if (a.counts && p == 0) {
    int32_t* cnt = a.counts + (size_t)tcl * N * N;
    for (int i = threadIdx.x; i < S * N; i += blockDim.x) {
      const int kv = i / S, col = i % S;
      cnt[(size_t)kv * N + strip * S + col] = (int32_t)scnt[col * N + kv];
    }
  }
}

// ---------------------------------------------------------------- weights
// Images img0 .. img0+n_img-1 of a chunk: W from the pair's kept count (natural) or the image's
// occupancy (uniform); inv_w and weight_sum are indexed by the chunk image index.
__global__ void k_image_weights(const int* n_kept, const int* occ, int uniform, int P, int img0, int n_img,
                                float* inv_w, double* weight_sum) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_img) return;
  const int i = img0 + j;
  const int W = uniform ? occ[i] : 2 * n_kept[i / P];
  if (inv_w) inv_w[i] = W > 0 ? (float)(1.0 / (double)W) : 0.f;
  if (weight_sum) weight_sum[i] = (double)W;
}

hipError_t launch_image_weights(const int* n_kept, const int* occ, int uniform, int P, int img0, int n_img,
                                float* inv_w, double* weight_sum, hipStream_t s) {
  if (n_img <= 0) return hipSuccess;
  k_image_weights<<<(n_img + 255) / 256, 256, 0, s>>>(n_kept, occ, uniform, P, img0, n_img, inv_w, weight_sum);
  return hipGetLastError();
}

// Strip-width and row-block options compiled for each size (largest first).
template <int LOGN>
struct Options {
  static hipError_t run(bool uniform, int* col, int* ncol, int* row, int* nrow, int* grid) {
    const int sm = uniform ? ColSmax<LOGN, true>::value : ColSmax<LOGN, false>::value;
    *ncol = 0;
    for (int k = 0; k < (LOGN >= kTunedLogn ? 3 : 1); ++k)
      if ((sm >> k) >= 1) col[(*ncol)++] = sm >> k;
    *nrow = 0;
    if (LOGN >= kTunedLogn) {
      if (RowFits<LOGN, 8>::value) row[(*nrow)++] = 8;
      if (RowFits<LOGN, 4>::value) row[(*nrow)++] = 4;
      if (RowFits<LOGN, 2>::value) row[(*nrow)++] = 2;
      if (RowFits<LOGN, 1>::value) row[(*nrow)++] = 1;
    } else {
      row[(*nrow)++] = RowDefault<LOGN>::value;
    }
    *grid = GridCfg<LOGN>::S;
    return hipSuccess;
  }
};

int col_strip_options(int logn, bool uniform, int* out) {
  int col[4], row[4], nc = 0, nr = 0, g = 0;
  if (by_logn<Options>(logn, uniform, col, &nc, row, &nr, &g) != hipSuccess) return 0;
  for (int i = 0; i < nc; ++i) out[i] = col[i];
  return nc;
}

int row_block_options(int logn, int* out) {
  int col[4], row[4], nc = 0, nr = 0, g = 0;
  if (by_logn<Options>(logn, false, col, &nc, row, &nr, &g) != hipSuccess) return 0;
  for (int i = 0; i < nr; ++i) out[i] = row[i];
  return nr;
}

int grid_strip_width(int logn) {
  int col[4], row[4], nc = 0, nr = 0, g = 0;
  (void)by_logn<Options>(logn, false, col, &nc, row, &nr, &g);
  return g;
}

template <int LOGN>
struct GridFullL {
  static hipError_t run(const GridArgs* a, hipStream_t s) {
    constexpr int N = 1 << LOGN;
    dim3 grid(a->Q * a->P, N / GridCfg<LOGN>::S);
    if (a->uniform) k_grid_full<LOGN, true><<<grid, GridCfg<LOGN>::THREADS, 0, s>>>(*a);
    else k_grid_full<LOGN, false><<<grid, GridCfg<LOGN>::THREADS, 0, s>>>(*a);
    return hipGetLastError();
  }
};

hipError_t launch_grid_full(const GridArgs& a, hipStream_t s) {
  if (a.Q <= 0) return hipSuccess;
  return by_logn<GridFullL>(a.logn, &a, s);
}

// ---------------------------------------------------------------- FFT launchers
template struct PrecLaunch<BLINK_PREC_FP32>;

hipError_t launch_grid_colfft(const ColArgs& a, int n_img, int strip, int prec, const float2* tw, hipStream_t s) {
  switch (prec) {
    case BLINK_PREC_FP32: return PrecLaunch<BLINK_PREC_FP32>::grid_colfft(a, n_img, strip, tw, s);
    case BLINK_PREC_SPLIT_F16: return PrecLaunch<BLINK_PREC_SPLIT_F16>::grid_colfft(a, n_img, strip, tw, s);
    case BLINK_PREC_SPLIT_BF16: return PrecLaunch<BLINK_PREC_SPLIT_BF16>::grid_colfft(a, n_img, strip, tw, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_dense_colfft(const float2* grids, int n_img, int logn, int shift, int prec, float2* H,
                               const float2* tw, const uint4* ops, hipStream_t s) {
  switch (prec) {
    case BLINK_PREC_FP32: return PrecLaunch<BLINK_PREC_FP32>::dense_colfft(grids, n_img, logn, shift, H, tw, ops, s);
    case BLINK_PREC_SPLIT_F16:
      return PrecLaunch<BLINK_PREC_SPLIT_F16>::dense_colfft(grids, n_img, logn, shift, H, tw, ops, s);
    case BLINK_PREC_SPLIT_BF16:
      return PrecLaunch<BLINK_PREC_SPLIT_BF16>::dense_colfft(grids, n_img, logn, shift, H, tw, ops, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_chunk_colfft(const DescArgs& a, int chunk, int logn, int strip, int col_loop, int slots, int prec,
                               hipStream_t s) {
  switch (prec) {
    case BLINK_PREC_FP32: return StagedLaunch<BLINK_PREC_FP32>::colfft(a, chunk, logn, strip, col_loop, slots, s);
    case BLINK_PREC_SPLIT_F16:
      return StagedLaunch<BLINK_PREC_SPLIT_F16>::colfft(a, chunk, logn, strip, col_loop, slots, s);
    case BLINK_PREC_SPLIT_BF16:
      return StagedLaunch<BLINK_PREC_SPLIT_BF16>::colfft(a, chunk, logn, strip, col_loop, slots, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_chunk_row(const DescArgs& a, int chunk, int logn, int tpb, int slots, int prec, hipStream_t s) {
  switch (prec) {
    case BLINK_PREC_FP32: return StagedLaunch<BLINK_PREC_FP32>::row(a, chunk, logn, tpb, slots, s);
    case BLINK_PREC_SPLIT_F16: return StagedLaunch<BLINK_PREC_SPLIT_F16>::row(a, chunk, logn, tpb, slots, s);
    case BLINK_PREC_SPLIT_BF16: return StagedLaunch<BLINK_PREC_SPLIT_BF16>::row(a, chunk, logn, tpb, slots, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_row_c2r(const RowArgs& a, int n_img, int tpb, int prec, const float2* tw, hipStream_t s) {
  switch (prec) {
    case BLINK_PREC_FP32: return PrecLaunch<BLINK_PREC_FP32>::row_c2r(a, n_img, tpb, tw, s);
    case BLINK_PREC_SPLIT_F16: return PrecLaunch<BLINK_PREC_SPLIT_F16>::row_c2r(a, n_img, tpb, tw, s);
    case BLINK_PREC_SPLIT_BF16: return PrecLaunch<BLINK_PREC_SPLIT_BF16>::row_c2r(a, n_img, tpb, tw, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace blink
