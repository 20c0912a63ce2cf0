// kernels.hip — gfx950 kernels of the batched dirty-imaging path.
//
//   k_twiddles       FP64 sincospi -> FP32 twiddle table
//   k_bin            cell indices (FP64 product + rint), flags, out-of-grid drop, counting sort
//                    of the placements into column strips (Section 6.2.4 gridding, one
//                    workgroup per (time, channel), shared by the polarisations)
//   k_grid_full      LDS-private strip grid -> complex grid in HBM (plain stores), counts
//   k_grid_colfft    LDS-private strip grid -> inverse FFT along v -> half-spectrum H
//   k_dense_colfft   Hermitian part of a dense grid -> inverse FFT along v -> H
//   k_row_c2r        two H rows -> Hermitian-extended inverse FFT along u -> two image rows,
//                    scaled by 1/W of the image (computed from the kept count or occupancy)
//
// The dirty image is I = Re(IDFT2(G)) / W (Section 4, Eq. 5). The shift of Section 6.2.4 is
// folded into the input as the modulation (-1)^(ku + kv), which for even N moves the phase
// centre to pixel (N/2, N/2). Because the grid is Hermitian only the columns ku < N/2 are
// transformed along v; the row pass rebuilds the other half by symmetry, and H's column 0 packs
// the two real-valued columns ku = 0 (real part) and ku = N/2 (imaginary part).
#include <hip/hip_runtime.h>

#include "imaging_device.hpp"
#include "launch.hpp"

namespace blink {

// ---------------------------------------------------------------- configuration
// Largest strip width (columns per workgroup) of the fused column kernel that fits 1024 threads
// and the 160 KB of LDS (strip buffer, twiddle table and, for uniform weighting, counts).
template <int LOGN, bool UNIFORM>
struct ColSmax {
  using P = FftPlan<LOGN>;
  static constexpr int N = P::N;
  static constexpr int per_col = P::NP * 8 + (UNIFORM ? N * 4 : 0);
  static constexpr int avail = kLdsBytes - N * 8 - 1024;
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
                                TPB * FftPlan<LOGN>::NP * 8 + (1 << LOGN) * 8 <= kLdsBytes;
};

template <int LOGN>
struct RowDefault {
  using P = FftPlan<LOGN>;
  static constexpr int value = cmin(P::N / 2, (256 / P::T) > 0 ? 256 / P::T : 1);
};

// ---------------------------------------------------------------- twiddles
__global__ void k_twiddles(float2* tw, int n) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s, c;
  sincospi(2.0 * (double)j / (double)n, &s, &c);   // exact argument: 2j/n is a dyadic rational
  tw[j] = make_float2((float)c, (float)s);
}

hipError_t launch_twiddles(float2* tw, int n, hipStream_t s) {
  k_twiddles<<<(n + 255) / 256, 256, 0, s>>>(tw, n);
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
                   sh);
  if (threadIdx.x < a.P) a.occ[(size_t)tcl * a.P + threadIdx.x] = 0;
}

hipError_t launch_bin(const BinArgs& a, hipStream_t s) {
  if (a.Q <= 0) return hipSuccess;
  k_bin<<<a.Q, kBinThreads, 0, s>>>(a);
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

// ---------------------------------------------------------------- fused grid + column FFT
template <int LOGN, int S, bool UNIFORM>
__global__ __launch_bounds__(S * FftPlan<LOGN>::T) void k_grid_colfft(ColArgs a, const float2* __restrict__ twg) {
  using P = FftPlan<LOGN>;
  constexpr int N = P::N, NP = P::NP;
  __shared__ float2 sbuf[S * NP];
  __shared__ float2 stw[N];
  __shared__ unsigned scnt[UNIFORM ? S * N : 1];
  __shared__ int s_tmp;
  // blockIdx.x = slot of the image in this launch's group; the image is img0 + slot in the chunk
  const int slot = blockIdx.x, img = a.img0 + slot, strip = blockIdx.y;
  const int tcl = img / a.P;
  const int nstrips = (N / 2) / S;
  for (int i = threadIdx.x; i < N; i += blockDim.x) stw[i] = twg[i];   // visible after the task's first barrier
  const int* so = a.strip_off + (size_t)tcl * (nstrips + 1);
  grid_colfft_task<LOGN, S, UNIFORM>(a.vis + (size_t)img * a.B, a.plc + (size_t)tcl * 2 * a.B, so[strip], so[strip + 1],
                                     strip, a.shift != 0, a.H + (size_t)slot * N * (N / 2), a.occ + img, stw, sbuf, scnt,
                                     &s_tmp);
}

// ---------------------------------------------------------------- dense grid column FFT
template <int LOGN>
__global__ __launch_bounds__((ColSmax<LOGN, false>::value * FftPlan<LOGN>::T)) void k_dense_colfft(
    const float2* __restrict__ grids, int shift, float2* __restrict__ H, const float2* __restrict__ twg) {
  using P = FftPlan<LOGN>;
  constexpr int N = P::N, T = P::T, S = ColSmax<LOGN, false>::value, NP = P::NP, mask = N - 1;
  __shared__ float2 sbuf[S * NP];
  __shared__ float2 stw[N];
  const int img = blockIdx.x, strip = blockIdx.y;
  const float2* G = grids + (size_t)img * N * N;
  for (int i = threadIdx.x; i < N; i += blockDim.x) stw[i] = twg[i];
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
  const int col = threadIdx.x / T, lt = threadIdx.x % T;
  float2* cb = sbuf + col * NP;
  float2 v[P::R];
#pragma unroll
  for (int m = 0; m < P::R; ++m) v[m] = cb[pad_index(lt + m * T)];
  fft_inverse<LOGN, true>(v, cb, stw, lt, [](int, float2) {});
  float2* Hi = H + (size_t)img * N * (N / 2);
  for (int i = threadIdx.x; i < S * N; i += blockDim.x) {
    const int y = i / S, c = i % S;
    Hi[(size_t)y * (N / 2) + strip * S + c] = sbuf[c * NP + pad_index(y)];
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

template <int LOGN, int TPB>
__global__ __launch_bounds__(TPB * FftPlan<LOGN>::T) void k_row_c2r(RowArgs a, const float2* __restrict__ twg) {
  using P = FftPlan<LOGN>;
  constexpr int N = P::N, NP = P::NP;
  __shared__ float2 sbuf[TPB * NP];
  __shared__ float2 stw[N];
  const int slot = blockIdx.x, img = a.img0 + slot;
  for (int i = threadIdx.x; i < N; i += blockDim.x) stw[i] = twg[i];   // visible after row_task's barrier
  const double W = image_weight(a, img);
  if (a.weight_sum && blockIdx.y == 0 && threadIdx.x == 0) a.weight_sum[img] = W;
  row_task<LOGN, TPB>(a.H + (size_t)slot * N * (N / 2), blockIdx.y, inverse_weight(W),
                      a.images + (size_t)slot * N * N, stw, sbuf);
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

template <int LOGN, int S, bool U>
static hipError_t col_one(const ColArgs* a, int n_img, const float2* tw, hipStream_t s) {
  if constexpr (S >= 1) {
    dim3 grid(n_img, ((1 << LOGN) / 2) / S);
    k_grid_colfft<LOGN, S, U><<<grid, S * FftPlan<LOGN>::T, 0, s>>>(*a, tw);
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

hipError_t launch_grid_colfft(const ColArgs& a, int n_img, int strip, const float2* tw, hipStream_t s) {
  if (n_img <= 0) return hipSuccess;
  return by_logn<ColL>(a.logn, &a, n_img, strip, tw, s);
}

template <int LOGN>
struct DenseL {
  static hipError_t run(const float2* g, int n_img, int shift, float2* H, const float2* tw, hipStream_t s) {
    constexpr int N = 1 << LOGN;
    constexpr int S = ColSmax<LOGN, false>::value;
    dim3 grid(n_img, (N / 2) / S);
    k_dense_colfft<LOGN><<<grid, S * FftPlan<LOGN>::T, 0, s>>>(g, shift, H, tw);
    return hipGetLastError();
  }
};

hipError_t launch_dense_colfft(const float2* grids, int n_img, int logn, int shift, float2* H,
                               const float2* tw, hipStream_t s) {
  if (n_img <= 0) return hipSuccess;
  return by_logn<DenseL>(logn, grids, n_img, shift, H, tw, s);
}

template <int LOGN, int TPB>
static hipError_t row_one(const RowArgs* a, int n_img, const float2* tw, hipStream_t s) {
  if constexpr (RowFits<LOGN, TPB>::value) {
    dim3 grid(n_img, ((1 << LOGN) / 2) / TPB);
    k_row_c2r<LOGN, TPB><<<grid, TPB * FftPlan<LOGN>::T, 0, s>>>(*a, tw);
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

hipError_t launch_row_c2r(const RowArgs& a, int n_img, int tpb, const float2* tw, hipStream_t s) {
  if (n_img <= 0) return hipSuccess;
  return by_logn<RowL>(a.logn, &a, n_img, tpb, tw, s);
}

}  // namespace blink
