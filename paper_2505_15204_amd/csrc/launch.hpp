// launch.hpp — host-side launchers of the imaging kernels (internal to libblink.so).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

#include "blink.h"

namespace blink {

// Compiled variants per grid size (largest first); each returns the number written to `out` (<= 4).
int col_strip_options(int logn, bool uniform, int* out);   // columns per workgroup of the fused kernel
int row_block_options(int logn, int* out);                 // row-pair transforms per workgroup
int grid_strip_width(int logn);                            // full-grid gridding kernel

// FP32 stage-ordered twiddle table of N = 2^logn (tw_size(logn) float2, layout in
// fft_device.hpp), generated in FP64 on the device.
hipError_t launch_twiddles(float2* tw, int logn, hipStream_t s);
int twiddle_table_size(int logn);   // float2 elements
// The split forms' DFT operand table (uint4 [2][64][4]) from the twiddle table of any N.
hipError_t launch_dft_operands(const float2* tw, uint4* ops, hipStream_t s);
constexpr int kDftOpsCount = 2 * 64 * 4;   // uint4 elements

// Cell indices and strip-binned placement lists, one workgroup per (time, channel) pair.
// Pairs tc0 .. tc0+Q-1 of the [T][C] batch. Placements with column >= ku_limit are dropped
// from the list (the half-spectrum path only needs ku < N/2).
struct BinArgs {
  const double* uvw;        // [T][B][3]
  const double* freq;       // [C]
  const uint8_t* flags;     // [T][C][B] or null
  int tc0, Q, C, B, logn, log_strip, ku_limit, P;
  double pixel_scale;
  int2* plc;                // [Q][2B]
  int* strip_off;           // [Q][nstrips+1]
  int* n_kept;              // [Q]
  int* occ;                 // [Q][P], zeroed here
  int32_t* cell_idx;        // [T][C][B] or null (global)
  int32_t* n_out;           // [T][C] or null (global)
  int* ext;                 // [Q] or null: half-spectrum columns [0, ext) hold every placement (whole strips)
};
hipError_t launch_bin(const BinArgs& a, hipStream_t s);

// Full complex grids (unshifted) plus counts for blink_grid.
struct GridArgs {
  const float2* vis;        // chunk base: [Q][P][B]
  const int2* plc;
  const int* strip_off;
  int Q, P, B, logn, uniform;
  float2* grids;            // chunk base: [Q][P][N][N]
  int32_t* counts;          // chunk base: [Q][N][N] or null
  int* occ;                 // [Q][P]
};
hipError_t launch_grid_full(const GridArgs& a, hipStream_t s);

// Fused gridding + column (v) FFT of the half spectrum ku < N/2 into H [img][N][N/2].
// One launch covers images img0 .. img0+n_img-1 of the chunk; image img0+j uses H slot j.
struct ColArgs {
  const float2* vis;        // chunk base: [Q][P][B]
  const int2* plc;
  const int* strip_off;
  int Q, P, B, logn, uniform, shift, img0;
  float2* H;                // [n_img][N][N/2]
  int* occ;                 // [Q][P]
  const uint4* dft_ops;     // DFT operand table of the split forms
  int rec_stride;           // convolutional path: records per (t,c) pair (plc holds ConvRec)
  int col_loop;             // strips each column workgroup takes in turn (<= 1: one strip each)
  const int* ext;           // [Q] or null: only strips below ext[pair] / S are gridded and stored
};
// `prec` selects the FFT form: BLINK_PREC_FP32 or a split matrix-core precision.
hipError_t launch_grid_colfft(const ColArgs& a, int n_img, int strip, int prec, const float2* tw, hipStream_t s);

// Column FFT of the Hermitian part of dense grids into H (blink_ifft2d).
hipError_t launch_dense_colfft(const float2* grids, int n_img, int logn, int shift, int prec, float2* H,
                               const float2* tw, const uint4* dft_ops, hipStream_t s);

// Per-image 1/W (and W as double) from kept counts (natural) or occupancy (uniform).
hipError_t launch_image_weights(const int* n_kept, const int* occ, int uniform, int P, int img0, int n_img,
                                float* inv_w, double* weight_sum, hipStream_t s);
// Row (u) pass: Hermitian-extended complex FFT of two H rows at a time, real part * 1/W.
// A launch covers chunk images img0 .. img0+n_img-1; image img0+j reads H slot j and writes
// images + j*N*N. W comes from the caller (wmode user; null = 1), from 2 x the pair's kept count
// (natural) or from the image's occupancy (uniform); weight_sum (chunk base) receives W if non-null.
enum { kWeightUser = 0, kWeightNatural = 1, kWeightUniform = 2 };
struct RowArgs {
  const float2* H;
  float* images;
  int logn, P, img0, wmode;
  const double* w_user;     // chunk base, [n] or null
  const int* n_kept;        // [Q]
  const int* occ;           // [Q][P]
  double* weight_sum;       // chunk base or null
  const uint4* dft_ops;     // DFT operand table of the split forms
  const float* corr;        // grid correction 1/c per pixel index [N], or null
  const int* ext;           // [Q] or null: H columns at or beyond ext[pair] are read as zero
};
hipError_t launch_row_c2r(const RowArgs& a, int n_img, int tpb, int prec, const float2* tw, hipStream_t s);

// ---------------------------------------------------------------- convolutional gridding
// Separable exponential-of-semicircle kernel of `width` cells (conv_device.hpp).
struct ConvParams {
  int width;
  double beta;
};
// Records per (t,c) pair the convolutional binning may write for strips of width >= min_strip.
int conv_records_per_pair(int B, int width, int min_strip, int logn);
// (column strips) x (row bands) of one (t,c) pair's convolutional binning (its offsets hold one more).
int conv_bins_per_pair(int logn, int strip);
hipError_t launch_bin_conv(const BinArgs& a, ConvParams cp, int rec_stride, hipStream_t s);
// Fused convolutional gridding + column FFT (strip width: the largest compiled for natural weighting).
hipError_t launch_grid_colfft_conv(const ColArgs& a, int n_img, ConvParams cp, int prec, const float2* tw,
                                   hipStream_t s);
int conv_strip_width(int logn);
// corr[x] = 1 / c(X/N) for x < N (FP64 quadrature, stored as FP32).
hipError_t launch_conv_correction(float* corr, int logn, ConvParams cp, int shift, hipStream_t s);

// Visibility corrections before gridding (Section 6.2.3) for pairs tc0 .. tc0+Q-1 of the
// [T][C] batch: out[q][p][b] = J[c][p][i] V[q][p][b] conj(J[c][p][j]) exp(+2 pi i (f_c/c)
// (u l0 + v m0 + w (n0 - 1))) with (i, j) the antenna pair of baseline b (i > j,
// b = i (i - 1) / 2 + j): delay and products in FP64, the sine and cosine in FP32 after an exact
// reduction of the delay to [-1/2, 1/2] turn, rounded once to complex64.
struct CorrArgs {
  const float2* vis;        // chunk base [Q][P][B]
  const double* uvw;        // [T][B][3]
  const double* freq;       // [C]
  const float2* gains;      // [C][P][n_ant] or null (all 1)
  int tc0, Q, C, P, B, n_ant;
  double l0, m0, n0m1;      // n0m1 = sqrt(1 - l0^2 - m0^2) - 1
  float2* out;              // [Q][P][B]
};
hipError_t launch_correct_vis(const CorrArgs& a, hipStream_t s);

// Correlator (Section 4, Eq. 3; Section 6.2.2): volt complex int8 [S][F][A][2 pols] (re, im);
// vis complex64 [T][C][pol_mode][B] (B = A (A - 1) / 2, b = i (i - 1) / 2 + j, i > j; products
// XX, XY, YX, YY for pol_mode 4, XX, YY for 2), autos complex64 [T][C][A][4] or null;
// T = S / n_int, C = F / n_favg. The caller has checked 4 <= A <= 256, A % 4 == 0, the
// divisibility, n_int n_favg <= 65535 and T, C <= 65535.
struct CorrelateArgs {
  const int8_t* volt;
  int S, F, A, n_int, n_favg, pol_mode;
  int n_slabs;              // ceil(2A / 32)
  int C, T, n_groups;       // set by the launcher
  float2* vis;
  float2* autos;
};
size_t correlate_lds_bytes(int A);
hipError_t launch_correlate(const CorrelateArgs& a, hipStream_t s);

// De-dispersion: out [n_dm][t_out][N][N] = mean over c of in[t + delays[k][c]][c] for images
// in [T][C][N][N]; delays (device, [n_dm][C]) are checked by the caller (0 <= d <= T - t_out),
// t_out and n_dm <= 65535.
hipError_t launch_dedisperse(const float* in, int C, int logn, const int* delays, int n_dm, int t_out, float* out,
                             hipStream_t s);

// Averages of images [T][C][P][N][N] over the axes in `axes` (1 time, 2 channel, 4 pol).
hipError_t launch_image_average(const float* in, int T, int C, int P, int logn, int axes, float* out, hipStream_t s);

struct DescArgs;

// The staged form of the uneven-batch path (staged.hip, one object per precision): the fused
// column kernel and the row kernel of one chunk (images of one grid size 2^logn, at most `slots`
// of them) with strip width `strip` and `tpb` row-pair transforms.
template <int PREC>
struct StagedLaunch {
  static hipError_t colfft(const DescArgs& a, int chunk, int logn, int strip, int col_loop, int slots, hipStream_t s);
  static hipError_t row(const DescArgs& a, int chunk, int logn, int tpb, int slots, hipStream_t s);
};
extern template struct StagedLaunch<BLINK_PREC_FP32>;
extern template struct StagedLaunch<BLINK_PREC_SPLIT_F16>;
extern template struct StagedLaunch<BLINK_PREC_SPLIT_BF16>;

// The same three launchers for one precision form; FP32 is built in kernels.hip, each split
// precision in its own object from split.hip.
template <int PREC>
struct PrecLaunch {
  static hipError_t grid_colfft(const ColArgs& a, int n_img, int strip, const float2* tw, hipStream_t s);
  static hipError_t dense_colfft(const float2* grids, int n_img, int logn, int shift, float2* H, const float2* tw,
                                 const uint4* dft_ops, hipStream_t s);
  static hipError_t row_c2r(const RowArgs& a, int n_img, int tpb, const float2* tw, hipStream_t s);
  static hipError_t grid_colfft_conv(const ColArgs& a, int n_img, int width, float beta, const float2* tw,
                                     hipStream_t s);
};
extern template struct PrecLaunch<BLINK_PREC_FP32>;
extern template struct PrecLaunch<BLINK_PREC_SPLIT_F16>;
extern template struct PrecLaunch<BLINK_PREC_SPLIT_BF16>;

// ---------------------------------------------------------------- uneven batches (persistent.hip)
struct DescArgs {
  const blink_image_desc* desc;
  int n_img;
  const float2* vis;
  int64_t vis_len;
  const double* uvw;
  int64_t uvw_len;                 // baselines
  const uint8_t* flags;
  int64_t flags_len;
  int max_b, max_logn, weighting, shift, block;
  float* images;
  int64_t images_len;
  double* weight_sum;              // [n_img] or null
  int32_t* n_out;                  // [n_img] or null
  int32_t* status;                 // [1] (caller's or workspace)
  // workspace
  int* valid;                      // [n_img] 1 if the descriptor passed the checks
  int* order;                      // [n_img] processing order (largest grids first)
  int* counter;                    // [1] next position in `order`
  int2* plc;                       // [workgroups][2 max_b]
  int* strip_off;                  // [workgroups][strip_stride]
  int strip_stride;
  float2* H;                       // [workgroups][max_n * max_n / 2]
  const float2* tw[13];            // twiddle tables per log2 N
  const uint4* dft_ops;            // DFT operand table of the split forms
  // staged form (plc, strip_off and H above then hold per-image placements and offsets, indexed
  // by position in `order`, and the chunk buffer)
  int4* chunks;                    // [max_chunks] {log2 N, first position in order, images, 0}; null: persistent form
  int max_chunks;
  int64_t chunk_elems;             // float2 elements of the chunk buffer (a multiple of the largest image's)
  int* kept;                       // [n_img] kept visibilities, by position
  int* occ;                        // [n_img] occupied cells (uniform weighting), by position
  int* ext;                        // [n_img] column extent, by position
  int col_log_strip[13];           // per log2 N: log2 of the column kernel's strip width
};
// Staged form: the chunk table reserves, for each grid size 2^logn <= the batch's largest, the
// chunk slots that n_img images of that size could fill (largest size first), so that the host
// can launch each slot's kernels for its size without reading the table back.
__host__ __device__ inline int staged_capacity(int logn, int64_t chunk_elems, int n_img) {
  const int64_t c = chunk_elems >> (2 * logn - 1);
  return (int)(c < (int64_t)n_img ? (c > 0 ? c : 1) : (n_img > 0 ? n_img : 1));
}
__host__ __device__ inline int staged_slots(int logn, int64_t chunk_elems, int n_img) {
  const int cap = staged_capacity(logn, chunk_elems, n_img);
  return n_img > 0 ? (n_img + cap - 1) / cap : 0;
}
hipError_t launch_desc_prep(const DescArgs& a, hipStream_t s);
hipError_t launch_persistent(const DescArgs& a, int workgroups, int prec, hipStream_t s);
// Resident workgroups of the persistent kernel per CU (0 if the configuration is not compiled).
int persistent_blocks_per_cu(int block, bool uniform, int prec);
// Staged form: binning of every image (one workgroup each, strips of the column width that
// `a.block` threads give), then per chunk a column launch and a row launch over `workgroups`.
hipError_t launch_desc_bin(const DescArgs& a, hipStream_t s);
hipError_t launch_chunk_colfft(const DescArgs& a, int chunk, int logn, int strip, int col_loop, int slots, int prec,
                               hipStream_t s);
hipError_t launch_chunk_row(const DescArgs& a, int chunk, int logn, int tpb, int slots, int prec, hipStream_t s);

// The persistent kernel of one precision form (FP32 in persistent.hip, split forms in split.hip).
template <int PREC>
struct PersistLaunch {
  static hipError_t launch(const DescArgs& a, int workgroups, hipStream_t s);
  static int blocks_per_cu(int block, bool uniform);
};
extern template struct PersistLaunch<BLINK_PREC_FP32>;
extern template struct PersistLaunch<BLINK_PREC_SPLIT_F16>;
extern template struct PersistLaunch<BLINK_PREC_SPLIT_BF16>;

}  // namespace blink
