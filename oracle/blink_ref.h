/*
 * blink_ref — plain, slow, obviously correct FP64 CPU oracle for batched dirty imaging.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or call this
 * library: only the tests, the package's smoke check and the benchmark's CPU-baseline
 * leg use it. It shares no code, header, table or constant with the HIP library.
 *
 * What it computes (BLINK, arXiv 2505.15204):
 *   - Section 4, Eq. 4: visibilities sample S(u,v) = FT of the sky with kernel exp(-i2pi(ul+vm)).
 *   - Section 4, Eq. 5 and Section 6.2.4: each visibility is placed, with no convolution
 *     kernel, on the regular N x N grid cell of its (u,v) ("gridding"); natural weighting
 *     gives every baseline the same weight; the dirty image is the inverse 2D FFT of the
 *     grid, shifted so the phase centre is in the middle.
 *   - Section 6.1: visibilities and images are 32-bit floats; this oracle widens them to
 *     double exactly and computes everything in IEEE double (no FMA contraction).
 *
 * Readings where the paper is silent (each one is listed with its reason in the design notes):
 *   cell size      1/(N*dl) wavelengths, so k = (f/c)*(N*dl) cells per metre, in that order;
 *   rounding       iu = nearbyint(u*k), ties to even, on that single double product;
 *   out of grid    kept only if |iu| < N/2 and |iv| < N/2 (strict; NaN counts as outside);
 *   Hermitian      every kept visibility V at (iu,iv) also contributes conj(V) at (-iu,-iv);
 *   linear cell    (iv mod N)*N + (iu mod N), corner origin;
 *   weighting      natural: G = sum of placements, W = number of placements;
 *                  uniform: G = mean of the placements in the cell, W = number of occupied cells;
 *   image          I[y][x] = Re( sum_{kv,ku} G[kv][ku] exp(+2 pi i (ku X + kv Y)/N) ) / W,
 *                  X = x - N/2, Y = y - N/2 when shifted (X = x, Y = y otherwise); W = 0 gives 0;
 *   flags          a flagged (t,c,b) is dropped before weighting, for every polarisation.
 *
 * Layouts: complex values are interleaved (re, im) pairs. vis is complex64 [T][C][P][B];
 * uvw is double [T][B][3] metres; freq is double [C]; flags are uint8 [T][C][B] (1 = flagged,
 * NULL = none); grids are complex double [N][N] row-major (row = v index); images are double
 * [N][N] (row = y = m direction, column = x = l direction).
 *
 * Return codes: 0 success, 1 invalid argument (N not a power of two in [2, 16384], negative
 * sizes, NULL required pointer), 2 out of memory. Nothing is written on an argument error.
 */
#ifndef BLINK_REF_H
#define BLINK_REF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Cells per metre for one channel: k = (f / c) * (N * dl), c = 299792458 m/s. */
double blink_ref_cells_per_metre(double freq_hz, int grid_n, double pixel_scale);

/* Nearest-cell gridding of one (time, channel) for P polarisations.
 * vis: complex64 [P][B]; flags: uint8 [B] or NULL; uvw: double [B][3].
 * grid: out complex double [P][N][N]; counts: out int32 [N][N] (placements per cell) or NULL;
 * cell_idx: out int32 [B] (linear cell of the (iu,iv) placement, -1 flagged, -2 out of grid) or NULL;
 * weight_sum: out W (same for every polarisation); n_out: out number of out-of-grid visibilities. */
int blink_ref_grid(const float *vis, const uint8_t *flags, const double *uvw, int P, int B,
                   double freq_hz, int grid_n, double pixel_scale, int weighting,
                   double *grid, int32_t *counts, int32_t *cell_idx,
                   double *weight_sum, int32_t *n_out);

/* In-place unnormalised inverse DFT of length n (power of two): X[j] <- sum_k X[k] exp(+2 pi i jk/n).
 * Iterative radix-2 decimation-in-time with bit-reversed input order. */
int blink_ref_ifft1d(double *data, int n);

/* Dirty image of one complex grid [N][N]: I = Re(IDFT2(G)) / W, optionally shifted.
 * weight_sum <= 0 or not finite gives an all-zero image. imag_max (may be NULL) receives
 * max |Im| / W over the image, for the realness check. */
int blink_ref_ifft2d(const double *grid, int grid_n, double weight_sum, int shift,
                     double *image, double *imag_max);

/* Whole path over a batch: images [T][C][P][N][N] double, weight_sum [T][C][P] (or NULL),
 * n_out [T][C] (or NULL), cell_idx [T][C][B] (or NULL), counts [T][C][N][N] (or NULL).
 * OpenMP over (t,c) with n_threads threads (<= 0: the OpenMP default). */
int blink_ref_image_batch(const float *vis, const uint8_t *flags, const double *uvw,
                          const double *freq_hz, int T, int C, int P, int B, int grid_n,
                          double pixel_scale, int weighting, int shift, double *images,
                          double *weight_sum, int32_t *n_out, int32_t *cell_idx,
                          int32_t *counts, int n_threads);

/* The same with complex double visibilities [T][C][P][B] (e.g. blink_ref_correct_vis output). */
int blink_ref_image_batch_c128(const double *vis, const uint8_t *flags, const double *uvw,
                               const double *freq_hz, int T, int C, int P, int B, int grid_n,
                               double pixel_scale, int weighting, int shift, double *images,
                               double *weight_sum, int32_t *n_out, int32_t *cell_idx,
                               int32_t *counts, int n_threads);

/* Direct Fourier transform of one (time, channel): the dirty image of Section 4 (Eq. 4 inverted on
 * the sampled (u, v), Eq. 5) summed baseline by baseline, with no grid and no FFT. Keep rule and
 * natural weighting as in blink_ref_grid (W = 2 x kept); each kept visibility and its Hermitian
 * mirror contribute
 *   I[p][y][x] += 2 Re( V[p][b] exp(+2 pi i (a_b X + c_b Y) / N) ) / W,
 * X = x - N/2, Y = y - N/2 when shifted (X = x, Y = y otherwise), where (a_b, c_b) is the nearest
 * cell (nearbyint(u k), nearbyint(v k)) when snap != 0 (the gridded image's value, reached by a
 * different route) and the exact position (u k, v k) in cells when snap == 0 (the ungridded
 * transform). vis complex64 [P][B]; image out double [P][N][N]; W = 0 gives a zero image. */
int blink_ref_dft(const float *vis, const uint8_t *flags, const double *uvw, int P, int B,
                  double freq_hz, int grid_n, double pixel_scale, int snap, int shift,
                  double *image, double *weight_sum, int32_t *n_out);

/* Visibility corrections before gridding (Section 6.2.3): for baseline b = (i, j), i > j,
 * b = i (i - 1) / 2 + j, and channel c with frequency f,
 *   V' = J[c][p][i] V conj(J[c][p][j]) exp(+2 pi i (f/c) (u l0 + v m0 + w (n0 - 1))),
 * n0 = sqrt(1 - l0^2 - m0^2), (u, v, w) = uvw[t][b] in metres. A source at direction cosines
 * (l0, m0) then has zero phase (it appears at the phase centre). gains: complex64 [C][P][n_ant]
 * or NULL (all 1; n_ant ignored); with gains, B must equal n_ant (n_ant - 1) / 2.
 * l0^2 + m0^2 < 1. vis complex64 [T][C][P][B]; out complex double [T][C][P][B]. */
int blink_ref_correct_vis(const float *vis, const double *uvw, const double *freq_hz, int T, int C,
                          int P, int B, const float *gains, int n_ant, double l0, double m0,
                          double *out);

/* Convolutional gridding (beyond the paper's nearest-cell placement, Section 6.2.4; the paper plans
 * a gridding kernel against aliasing, Section 10). Kernel: phi(z) = exp(beta (sqrt(1 - z^2) - 1))
 * for |z| < 1 ("exponential of semicircle", Barnett, Magland & af Klinteberg 2019), z = 2 d / W for
 * a cell offset d, support W cells, applied separably; a kept visibility V at cell position
 * (x, y) = (u k, v k) adds phi(2 (ju - x)/W) phi(2 (jv - y)/W) V to every cell (ju, jv) with
 * |ju - x| < W/2 and |jv - y| < W/2 (cells wrap modulo N), and conj(V) likewise around (-x, -y).
 * The keep rule is the nearest-cell one; natural weighting only (W_sum = 2 x kept). The image
 * is Re(IDFT2(G)) / W_sum / (c(X/N) c(Y/N)), c the kernel's continuous Fourier transform. */
double blink_ref_es_kernel(double z, double beta);
/* c(nu) = integral_{|d| < W/2} phi(2 d / W) cos(2 pi nu d) dd (composite Simpson, 4096 intervals). */
double blink_ref_es_transform(double nu, int width, double beta);
/* grid: out complex double [P][N][N]; width 1..16 (< N), beta >= 0. */
int blink_ref_grid_conv(const float *vis, const uint8_t *flags, const double *uvw, int P, int B,
                        double freq_hz, int grid_n, double pixel_scale, int width, double beta,
                        double *grid, double *weight_sum, int32_t *n_out);
/* corr[x] = c(X/N), X the signed offset of pixel x from the phase centre. */
int blink_ref_conv_correction(int grid_n, int width, double beta, int shift, double *corr);
/* Whole convolutional path over a batch (layouts as blink_ref_image_batch). */
int blink_ref_image_batch_conv(const float *vis, const uint8_t *flags, const double *uvw,
                               const double *freq_hz, int T, int C, int P, int B, int grid_n,
                               double pixel_scale, int width, double beta, int shift, double *images,
                               double *weight_sum, int32_t *n_out, int n_threads);

/* Image averages (Sections 7.2, 7.3): images float [T][C][P][N][N]; every axis set in `axes`
 * (1 time, 2 channel, 4 polarisation) is averaged, the others kept; out double [T'][C'][P'][N][N].
 * Over P = 2 (XX, YY) the polarisation average is Stokes I. */
int blink_ref_image_average(const float *images, int T, int C, int P, int grid_n, int axes, double *out);

/* Correlation (Section 4, Eq. 3; Section 6.2.2): volt complex int8 (re, im) [S][F][A][2 pols];
 * T = S / n_int integration intervals, C = F / n_favg output channels (both must divide).
 * vis: out complex64 [T][C][P][B], B = A (A - 1) / 2 cross baselines (i, j), i > j,
 * b = i (i - 1) / 2 + j; P = 4 products (XX, XY, YX, YY) for pol_mode 4, or P = 2 (XX, YY) for
 * pol_mode 2; V = (sum over the n_int samples and n_favg channels of x_{i,p} conj(x_{j,q}))
 * / (n_int n_favg), the sums exact in int64, the division in double, rounded once to float.
 * autos: out complex64 [T][C][A][4] (products XX, XY, YX, YY of each antenna with itself) or NULL. */
int blink_ref_correlate(const int8_t *volt, int S, int F, int A, int n_int, int n_favg, int pol_mode,
                        float *vis, float *autos);

/* Incoherent de-dispersion (the FRB search the images feed; Sections 1, 3, 10, Table 1).
 * delays [n_dm][C] = nearbyint(4148.808 s MHz^2 cm^3/pc x dm x (f^-2 - f_ref^-2) / dt), f in MHz,
 * f_ref the highest channel frequency; out [n_dm][t_out][N][N] (double) = mean over c of
 * images[t + delay(c)][c] for images float [T][C][N][N]; every t_out + delay must be <= T. */
int blink_ref_dispersion_delays(const double *freq_hz, int C, double dt_s, const double *dm, int n_dm,
                                int32_t *delays);
int blink_ref_dedisperse(const float *images, int T, int C, int grid_n, const int32_t *delays, int n_dm,
                         int t_out, double *out);

/* Number of threads blink_ref_image_batch would use for n_threads <= 0. */
int blink_ref_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
