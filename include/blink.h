/*
 * blink.h — C ABI of libblink.so: batched dirty imaging on one MI355X (gfx950) GPU.
 *
 * Method (BLINK, arXiv 2505.15204):
 *   Section 4, Eq. 4   visibilities sample the Fourier transform of the sky with kernel
 *                      exp(-i 2 pi (u l + v m)); so the image side uses the + sign.
 *   Section 4, Eq. 5   the dirty image is the inverse 2D FFT of the visibilities placed on a
 *                      regular N x N grid ("gridding").
 *   Section 6.2.4      gridding puts each visibility on the cell of its (u,v) with no
 *                      convolution kernel, natural weighting by default; many fine channels and
 *                      integration intervals are gridded in parallel on one GPU and all grids go
 *                      through one batched inverse 2D FFT; the phase centre is then shifted from
 *                      the corner to the middle of the image.
 *   Section 6.1        visibilities and images are 32-bit floating point.
 *
 * Readings of what the paper leaves open (the same ones the test oracle uses):
 *   cell size      1/(N dl) wavelengths: k = (f / c) * (N * dl) cells per metre, evaluated in
 *                  IEEE double in that order (c = 299792458 m/s);
 *   rounding       iu = rint(u * k), iv = rint(v * k) on one double product, ties to even;
 *   out of grid    a visibility is kept only if |iu| < N/2 and |iv| < N/2 (NaN is outside);
 *   Hermitian      a kept visibility V at (iu, iv) also places conj(V) at (-iu, -iv);
 *   weighting      natural: the cell holds the sum of its placements, W = number of placements;
 *                  uniform: the cell holds their mean, W = number of occupied cells;
 *   image          I[y][x] = Re( sum_{kv,ku} G[kv][ku] exp(+2 pi i (ku X + kv Y) / N) ) / W,
 *                  X = x - N/2, Y = y - N/2 when shifted, X = x, Y = y otherwise; W <= 0 gives 0;
 *   flags          a flagged (time, channel, baseline) is dropped for every polarisation.
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers into memory the caller owns (e.g. torch tensors);
 *     inputs are never modified, outputs are fully overwritten. Layouts are C order:
 *       vis       blink_cf32 [T][C][P][B]   (same bytes as complex64)
 *       flags     uint8      [T][C][B]      1 = flagged, NULL = nothing flagged
 *       uvw_m     double     [T][B][3]      metres; w is ignored (coplanar)
 *       freq_hz   double     [C]
 *       grids     blink_cf32 [T][C][P][N][N] row = v index, corner origin, unshifted
 *       images    float      [T][C][P][N][N] row = y (m direction), column = x (l direction)
 *   - Work is queued on `hip_stream` (a hipStream_t; NULL = the null stream) and is complete
 *     after that stream is synchronised. No entry point synchronises with the host.
 *   - The caller provides `workspace` (device memory, 256-byte aligned) of `workspace_bytes`;
 *     the library never allocates device memory in these calls. Use the *_workspace_size
 *     queries. blink_image_batch processes (t, c) pairs in chunks, so any workspace at least as
 *     large as the query for T = 1, C = 1 is accepted.
 *   - Calls that share a context or a workspace must not run concurrently; a context belongs to
 *     one host thread at a time.
 *   - Errors: every entry point returns a blink_status. Argument and size errors are detected on
 *     the host before anything is queued, and then nothing is written. blink_last_error()
 *     describes the last failure on a context. Nothing is thrown across the ABI.
 */
#ifndef BLINK_H
#define BLINK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct blink_ctx_s *blink_ctx;

typedef struct {
    float re, im;
} blink_cf32;

typedef enum {
    BLINK_OK = 0,
    BLINK_ERR_ARG = 1,    /* NULL required pointer, negative size, unknown enum value, NULL ctx */
    BLINK_ERR_SIZE = 2,   /* grid_n not a power of two in [8, 4096], workspace too small, sizes overflow */
    BLINK_ERR_NOMEM = 3,  /* a context allocation failed */
    BLINK_ERR_HIP = 4,    /* the HIP runtime reported an error, or the device is not gfx950 */
    BLINK_ERR_STATE = 5   /* the context is unusable after an earlier HIP error */
} blink_status;

enum { BLINK_WEIGHT_NATURAL = 0, BLINK_WEIGHT_UNIFORM = 1 };
/* FFT precision forms (the `precision` argument). The paper computes in 32-bit floating point
 * (Section 6.1) and names reduced precision as future work (Section 10):
 *   BLINK_PREC_FP32        radix-16 butterflies in FP32 on the vector ALUs;
 *   BLINK_PREC_SPLIT_F16   radix-16 stages as matrix-core (MFMA) products of FP16 operands split
 *                          into hi + lo (3 products, FP32 accumulation; a power-of-two scale per
 *                          strip or row block keeps FP16 in range);
 *   BLINK_PREC_SPLIT_BF16  the same with BF16 operands (no scaling needed).
 * Gridding, weights, twiddle multiplications and any radix-2/4/8 stage stay in FP32 in every
 * form; for N = 8 (no radix-16 stage) the split forms equal FP32. */
enum { BLINK_PREC_FP32 = 0, BLINK_PREC_SPLIT_F16 = 1, BLINK_PREC_SPLIT_BF16 = 2 };

#define BLINK_MIN_GRID 8
#define BLINK_MAX_GRID 4096

/* Library version as major*10000 + minor*100 + patch. */
int blink_version(void);

/* Static description of a status code. Never NULL. */
const char *blink_status_string(blink_status s);

/* Create a context on HIP device `hip_device`: checks that it is a gfx950 device and builds
 * the FP32 twiddle tables (generated in FP64 on the device). *out receives the handle.
 * Returns BLINK_ERR_HIP when no such device exists. */
blink_status blink_create(blink_ctx *out, int hip_device);

/* Release a context and its device tables. NULL is accepted. */
blink_status blink_destroy(blink_ctx ctx);

/* Text of the last error recorded on ctx ("" if none; a static message for NULL). */
const char *blink_last_error(blink_ctx ctx);

/* Workspace bytes for blink_grid over T time steps, C channels and B baselines on an N grid. */
blink_status blink_grid_workspace_size(int T, int C, int B, int grid_n, size_t *bytes);

/* Workspace bytes for blink_ifft2d over n_img grids of side grid_n. */
blink_status blink_ifft2d_workspace_size(int n_img, int grid_n, int precision, size_t *bytes);

/* Workspace bytes for blink_image_batch to process all T*C (time, channel) pairs in one chunk. */
blink_status blink_image_batch_workspace_size(int T, int C, int P, int B, int grid_n,
                                              int weighting, int precision, size_t *bytes);

/* One problem of one entry point, for the single workspace query blink_workspace_size. The
 * fields an entry point does not take are ignored. */
enum {
    BLINK_ENTRY_GRID = 0,                  /* T, C, B, grid_n */
    BLINK_ENTRY_IFFT2D = 1,                /* n_img, grid_n, precision */
    BLINK_ENTRY_IMAGE_BATCH = 2,           /* T, C, P, B, grid_n, weighting, precision */
    BLINK_ENTRY_IMAGE_BATCH_CORRECTED = 3, /* T, C, P, B, grid_n, weighting, precision */
    BLINK_ENTRY_IMAGE_BATCH_CONV = 4,      /* T, C, P, B, grid_n, kernel_width, precision */
    BLINK_ENTRY_IMAGE_BATCH_DESC = 5,      /* n_img, max_baselines, grid_n (the largest), workgroups */
    BLINK_ENTRY_DEDISPERSE = 6             /* C, n_dm */
};
typedef struct {
    int entry;                 /* BLINK_ENTRY_* */
    int T, C, P, B;            /* time steps, channels, polarisations, baselines */
    int n_img;                 /* grids (ifft2d) or described images (desc) */
    int grid_n;                /* N; for desc the largest N */
    int weighting, precision;  /* BLINK_WEIGHT_*, BLINK_PREC_* */
    int kernel_width;          /* conv: support W in cells */
    int max_baselines;         /* desc: most visibilities of one image */
    int workgroups;            /* desc: persistent workgroups (0 = the query's default, 512) */
    int n_dm;                  /* dedisperse: trial dispersion measures */
} blink_problem;

/* Workspace bytes of the entry point p->entry for problem *p: the same value as that entry
 * point's *_workspace_size query. ctx may be NULL. BLINK_ERR_ARG for a NULL p or bytes or an
 * unknown entry, otherwise the per-entry query's status. */
blink_status blink_workspace_size(blink_ctx ctx, const blink_problem *p, size_t *bytes);

/* Gridding only (Section 6.2.4; Section 4 Eq. 5). Places every unflagged, in-grid visibility
 * and its Hermitian mirror on the nearest cell of an N x N grid per (t, c, p).
 *   grids      out [T][C][P][N][N], natural: cell sums; uniform: cell means
 *   counts     out int32 [T][C][N][N] placements per cell (shared by the P pols), or NULL
 *   weight_sum out double [T][C][P] W of each image, or NULL
 *   cell_idx   out int32 [T][C][B]: (iv mod N)*N + (iu mod N) of the (iu, iv) placement,
 *              -1 if flagged, -2 if out of grid; or NULL
 *   n_out      out int32 [T][C]: visibilities dropped as out of grid, or NULL
 * pixel_scale is the image pixel size in direction-cosine units (radians, small angle). */
blink_status blink_grid(blink_ctx ctx, const blink_cf32 *vis, const uint8_t *flags,
                        const double *uvw_m, const double *freq_hz, int T, int C, int P, int B,
                        int grid_n, double pixel_scale, int weighting, blink_cf32 *grids,
                        int32_t *counts, double *weight_sum, int32_t *cell_idx, int32_t *n_out,
                        void *workspace, size_t workspace_bytes, void *hip_stream);

/* Batched dirty images of given grids (Section 4 Eq. 5; Section 6.2.4 shift):
 * images[i] = Re(IDFT2(grids[i])) / weight_sum[i], with the phase centre moved to (N/2, N/2)
 * when shift != 0. weight_sum may be NULL (W = 1); W <= 0 gives an all-zero image. Any complex
 * grid is accepted: its Hermitian part is transformed, which is what the real part needs. */
blink_status blink_ifft2d(blink_ctx ctx, const blink_cf32 *grids, const double *weight_sum,
                          int n_img, int grid_n, int precision, int shift, float *images,
                          void *workspace, size_t workspace_bytes, void *hip_stream);

/* The whole hot path, fused: gridding and inverse 2D FFT of every (t, c, p) image
 * (Section 6.2.4). The full complex grid is never materialised. Outputs:
 *   images     out float [T][C][P][N][N]
 *   weight_sum out double [T][C][P] or NULL
 *   n_out      out int32 [T][C] or NULL */
blink_status blink_image_batch(blink_ctx ctx, const blink_cf32 *vis, const uint8_t *flags,
                               const double *uvw_m, const double *freq_hz, int T, int C, int P,
                               int B, int grid_n, double pixel_scale, int weighting,
                               int precision, int shift, float *images, double *weight_sum,
                               int32_t *n_out, void *workspace, size_t workspace_bytes,
                               void *hip_stream);

/* ---------------------------------------------------------------- no-allocation variant
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): blink_image_batch with the same arguments, outputs and
 * results, minus the workspace. Its scratch memory is a fixed device array of
 * BLINK_STATIC_SCRATCH_BYTES inside the library (each GPU that the library runs on holds one
 * copy until the process ends), so the call allocates nothing and takes no kernel timing. The
 * (t, c) pairs are chunked to fit that array: a problem whose single (t, c) pair needs more
 * (blink_image_batch_workspace_size with T = C = 1 above the limit, e.g. N = 4096) is rejected
 * with BLINK_ERR_SIZE before anything is queued. Every call on one GPU shares that GPU's array,
 * from any context: calls that overlap on one GPU (on different streams or host threads) race and
 * must be serialised by the caller. Nothing in the array needs to start at zero. */
#define BLINK_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

blink_status blink_image_batch_noalloc(blink_ctx ctx, const blink_cf32 *vis, const uint8_t *flags,
                                       const double *uvw_m, const double *freq_hz, int T, int C,
                                       int P, int B, int grid_n, double pixel_scale, int weighting,
                                       int precision, int shift, float *images, double *weight_sum,
                                       int32_t *n_out, void *hip_stream);

/* ---------------------------------------------------------------- visibility corrections
 * The corrections the paper applies to the correlator output before imaging (Section 6.2.3):
 * calibration solutions per antenna, then the geometric correction that moves the phase centre to
 * the pointing direction (done in the imager, where (u, v, w) are known). Cable-length
 * corrections are per-antenna phases and go into the same per-antenna factors. For baseline
 * b = (i, j), i > j, b = i (i - 1) / 2 + j (the lower-triangular order of the correlation step,
 * Section 6.2.2, without autocorrelations) and channel c of frequency f:
 *   V' = J[c][p][i] V conj(J[c][p][j]) exp(+2 pi i (f / 299792458) (u l0 + v m0 + w (n0 - 1))),
 * n0 = sqrt(1 - l0^2 - m0^2), (u, v, w) the baseline's uvw_m[t][b] in metres. A source at
 * direction cosines (l0, m0) then has zero phase and images at the phase centre; the cells stay
 * those of the uncorrected (u, v) (no re-projection of the baselines). */
typedef struct blink_corrections {
    const blink_cf32 *gains;   /* device complex64 [C][P][n_ant] per-antenna factors J, or NULL (all 1) */
    int n_ant;                 /* antennas; with gains, B must equal n_ant (n_ant - 1) / 2 */
    double l0, m0;             /* new phase centre, direction cosines; l0^2 + m0^2 < 1 (0, 0: none) */
} blink_corrections;

/* Workspace bytes for blink_image_batch_corrected (blink_image_batch's, plus one chunk of
 * corrected visibilities). */
blink_status blink_image_batch_corrected_workspace_size(int T, int C, int P, int B, int grid_n,
                                                        int weighting, int precision, size_t *bytes);

/* blink_image_batch on the corrected visibilities V' above: a correction pass per chunk writes
 * V' into the workspace (delay and products in FP64, the rotation's sine and cosine in FP32 after
 * an exact reduction to one turn, the result rounded once to complex64), and the gridding of
 * blink_image_batch reads it in place of vis. corr is a host pointer (NULL: no corrections, the
 * result is blink_image_batch's); its gains are device memory. ERR_ARG when B does not match
 * n_ant with gains, or l0^2 + m0^2 >= 1. Same outputs, plans and workspace rules otherwise. */
blink_status blink_image_batch_corrected(blink_ctx ctx, const blink_cf32 *vis, const uint8_t *flags,
                                         const double *uvw_m, const double *freq_hz, int T, int C,
                                         int P, int B, int grid_n, double pixel_scale, int weighting,
                                         int precision, int shift, const blink_corrections *corr,
                                         float *images, double *weight_sum, int32_t *n_out,
                                         void *workspace, size_t workspace_bytes, void *hip_stream);

/* ---------------------------------------------------------------- correlation
 * The step before the corrections (Section 6.2.2; Section 4, Eq. 3): the conjugate
 * multiply-accumulate of every pair of fine-channelised antenna voltages, averaged over an
 * integration interval and over the fine channels of an output channel, written in the layout
 * blink_image_batch reads.
 *   volt     device complex int8 (re, im bytes) [S samples][F fine channels][A antennas][2 pols]
 *   vis      out complex64 [T][C][pol_mode][B]: T = S / n_int, C = F / n_favg,
 *            B = A (A - 1) / 2 cross baselines (i, j), i > j, b = i (i - 1) / 2 + j; products
 *            XX, XY, YX, YY (pol_mode 4) or XX, YY (pol_mode 2, directly imageable with P = 2)
 *   autos    out complex64 [T][C][A][4] (XX, XY, YX, YY of each antenna with itself) or NULL
 * V = (sum over the n_int samples and n_favg channels of x_{i,p} conj(x_{j,q})) / (n_int n_favg):
 * the sums are exact (int32 on the matrix cores), the division is done in FP64 and rounded once,
 * so the result is exactly the rounded mean. Requires volt 16-byte aligned, 4 <= A <= 256 with
 * A % 4 == 0, n_int | S,
 * n_favg | F, n_int n_favg <= 65535 (keeps the sums in int32), T and C <= 65535; otherwise
 * ERR_ARG. No workspace. */
blink_status blink_correlate(blink_ctx ctx, const int8_t *volt, int S, int F, int A, int n_int,
                             int n_favg, int pol_mode, blink_cf32 *vis, blink_cf32 *autos,
                             void *hip_stream);

/* ---------------------------------------------------------------- convolutional gridding
 * A step beyond the paper, which places visibilities on their nearest cell with no convolution
 * kernel (Section 6.2.4) and names a gridding kernel against aliasing as planned work (Sections 7
 * and 10). Here each kept visibility (same keep rule, natural weighting) is spread over the cells
 * within W/2 of its exact position (x, y) = (u k, v k) with the separable weights
 * phi(2 (ju - x)/W) phi(2 (jv - y)/W), phi(z) = exp(beta (sqrt(1 - z^2) - 1)) for |z| < 1 (the
 * "exponential of semicircle" kernel of Barnett, Magland & af Klinteberg, 2019); conj(V) spreads
 * around (-x, -y); cells wrap modulo N. The image is Re(IDFT2(G)) / W_sum divided by
 * c(X/N) c(Y/N), c(nu) = integral of phi(2d/W) cos(2 pi nu d) dd (the kernel's Fourier transform),
 * X, Y the pixel offsets from the phase centre. kernel_width is 1..16 and below N/2, kernel_beta
 * 0..100 (e.g. W = 8, beta = 2.3 W). Same layouts, workspace rules and outputs as
 * blink_image_batch; plans: the natural-weighting plan's row block and group. */
blink_status blink_image_batch_conv_workspace_size(int T, int C, int P, int B, int grid_n,
                                                   int kernel_width, int precision, size_t *bytes);
blink_status blink_image_batch_conv(blink_ctx ctx, const blink_cf32 *vis, const uint8_t *flags,
                                    const double *uvw_m, const double *freq_hz, int T, int C,
                                    int P, int B, int grid_n, double pixel_scale, int kernel_width,
                                    double kernel_beta, int precision, int shift, float *images,
                                    double *weight_sum, int32_t *n_out, void *workspace,
                                    size_t workspace_bytes, void *hip_stream);

/* ---------------------------------------------------------------- image averages
 * The paper averages its dirty images over time and over the band (Section 7.2: a long-exposure
 * image over all seconds and the 30.72 MHz band; Section 7.3: all channels of each 20 ms bin).
 * blink_image_average averages images float [T][C][P][N][N] (device) over every axis set in
 * `axes` and keeps the others: out float [T'][C'][P'][N][N] with T' = 1 if averaged over time,
 * else T (likewise C', P'). Averaging P = 2 (XX, YY) gives Stokes I = (XX + YY) / 2. Sums are
 * FP64; out must not overlap images. */
enum { BLINK_AVG_TIME = 1, BLINK_AVG_CHANNEL = 2, BLINK_AVG_POL = 4 };
blink_status blink_image_average(blink_ctx ctx, const float *images, int T, int C, int P, int grid_n,
                                 int axes, float *out, void *hip_stream);

/* ---------------------------------------------------------------- de-dispersion
 * The first step of the FRB search the images feed (Sections 1, 3 and 10; Table 1: DM up to 600
 * pc cm^-3, tens of seconds of dispersive delay over the band): incoherent de-dispersion of image
 * cubes. A pulse of dispersion measure DM reaches channel frequency f later than the highest
 * channel f_ref by 4148.808 s MHz^2 cm^3/pc x DM x (f^-2 - f_ref^-2) (frequencies in MHz; the
 * cold-plasma dispersion constant), rounded to whole time steps of dt seconds.
 *
 * blink_dispersion_delays (host only): delays [n_dm][C] int32 of the trial DMs dm[n_dm] >= 0 for
 * channel frequencies freq_hz[C] (Hz) and step dt_s > 0. */
blink_status blink_dispersion_delays(const double *freq_hz, int C, double dt_s, const double *dm, int n_dm,
                                     int32_t *delays);

/* Workspace bytes of blink_dedisperse for C channels and n_dm trials (the delay table). */
blink_status blink_dedisperse_workspace_size(int C, int n_dm, size_t *bytes);

/* out[k][t] = mean over channels c of images[t + delays[k][c]][c], t < t_out, for device images
 * float [T][C][N][N] (e.g. a Stokes I cube from blink_image_average) and device out float
 * [n_dm][t_out][N][N]. delays is a HOST array [n_dm][C] (blink_dispersion_delays); every delay
 * must satisfy 0 <= d <= T - t_out, else ERR_ARG before any device work. The table is copied
 * into the workspace (hipMemcpyAsync from the host array; the call returns once it is staged).
 * Sums are FP64 in channel order, divided by C and rounded once. grid_n a power of two 8 .. 4096;
 * n_dm, t_out <= 65535. */
blink_status blink_dedisperse(blink_ctx ctx, const float *images, int T, int C, int grid_n,
                              const int32_t *delays, int n_dm, int t_out, float *out, void *workspace,
                              size_t workspace_bytes, void *hip_stream);

/* ---------------------------------------------------------------- uneven batches
 * Section 6.2.4 grids many fine channels and integration intervals in parallel on one GPU and
 * transforms all grids at once. blink_image_batch_desc does this for images that differ in grid
 * size and visibility count: every image is described by one blink_image_desc (device memory).
 * A descriptor pass checks the descriptors and orders the images largest grid first; then one of
 * two forms (blink_set_desc_form) images them:
 *   BLINK_DESC_PERSISTENT  one persistent fused kernel whose workgroups claim images from a queue
 *                          and image each one alone (binning, gridding + column FFT, row FFT)
 *                          through a per-workgroup intermediate slot;
 *   BLINK_DESC_STAGED      one launch bins every image; then, per chunk of images of one grid size
 *                          whose half spectra fit a 256 MiB buffer (sized for the last-level
 *                          cache), a column launch and a row launch of blink_image_batch's fused
 *                          column and row kernels for that size, reading each image's visibilities
 *                          and output offset from its descriptor.
 * In both, workgroups never wait for each other (the staged launches are ordered by the stream). */
#define BLINK_DESC_PERSISTENT 0
#define BLINK_DESC_STAGED 1
typedef struct {
    int64_t vis_offset;    /* first visibility of the image in vis (blink_cf32 elements) */
    int64_t uvw_offset;    /* first baseline of the image in uvw_m (baselines: uvw_m + 3*uvw_offset) */
    int64_t flag_offset;   /* first flag of the image in flags (ignored when flags is NULL) */
    int64_t image_offset;  /* first pixel of the image in images (float elements) */
    double freq_hz;        /* channel frequency */
    double pixel_scale;    /* direction-cosine units per pixel */
    int32_t n_baselines;   /* B of this image, 0 <= B <= max_baselines */
    int32_t grid_n;        /* power of two in [8, max_grid_n] */
    int32_t reserved[2];   /* set to 0 */
} blink_image_desc;

/* Bits of the status word written by blink_image_batch_desc. */
#define BLINK_DESC_BAD 1       /* a descriptor was invalid or out of bounds; that image was skipped */

/* Workspace bytes for blink_image_batch_desc with n_img images of at most max_baselines
 * visibilities and grid side at most max_grid_n, enough for either form: the persistent form run
 * by `workgroups` workgroups (each owns one intermediate slot of max_grid_n^2/2 complex values)
 * and the staged form (placements of every image, 16 B per baseline, and the chunk buffer). */
blink_status blink_desc_workspace_size(int n_img, int max_baselines, int max_grid_n, int workgroups,
                                       size_t *bytes);

/* Images described by desc[0..n_img) (device array). vis_len, uvw_len (baselines), flags_len and
 * images_len give the element counts of the caller's arrays; every descriptor is checked against
 * them on the device and an invalid one only sets BLINK_DESC_BAD (its image is left untouched).
 * weighting, precision (any BLINK_PREC_* form) and shift apply to the whole batch. Outputs: images at each image_offset; weight_sum
 * double [n_img] and n_out int32 [n_img] (either may be NULL); status int32 [1] (may be NULL)
 * receives the BLINK_DESC_* bits. Uses the context's descriptor form and plan
 * (blink_set_desc_form, blink_set_desc_plan); the persistent form reduces the number of
 * workgroups to the slots the workspace holds, the staged form returns BLINK_ERR_SIZE when the
 * workspace is smaller than its layout. Capturable into a hipGraph (no allocation, copy or
 * memset is issued). */
blink_status blink_image_batch_desc(blink_ctx ctx, const blink_image_desc *desc, int n_img,
                                    const blink_cf32 *vis, int64_t vis_len, const double *uvw_m,
                                    int64_t uvw_len, const uint8_t *flags, int64_t flags_len,
                                    int max_baselines, int max_grid_n, int weighting, int precision,
                                    int shift, float *images, int64_t images_len,
                                    double *weight_sum, int32_t *n_out, int32_t *status,
                                    void *workspace, size_t workspace_bytes, void *hip_stream);

/* Persistent-form plan: block_threads (512 or 1024; uniform weighting uses 512) and the number of
 * workgroups (0 = as many as are resident on the device). */
blink_status blink_get_desc_plan(blink_ctx ctx, int *block_threads, int *workgroups);
blink_status blink_set_desc_plan(blink_ctx ctx, int block_threads, int workgroups);
/* Descriptor-path form: BLINK_DESC_STAGED (the default) or BLINK_DESC_PERSISTENT. The staged form
 * takes each grid size's execution plan of blink_image_batch (strip width, strips per workgroup,
 * row block); block_threads and workgroups apply to the persistent form. */
blink_status blink_get_desc_form(blink_ctx ctx, int *form);
blink_status blink_set_desc_form(blink_ctx ctx, int form);

/* Autotuner of the descriptor plan: times both forms (the staged one when the workspace holds it),
 * block sizes and workgroup counts on the caller's batch (same arguments as
 * blink_image_batch_desc) and keeps the fastest, form included. Synchronises. */
blink_status blink_autotune_desc(blink_ctx ctx, const blink_image_desc *desc, int n_img,
                                 const blink_cf32 *vis, int64_t vis_len, const double *uvw_m,
                                 int64_t uvw_len, const uint8_t *flags, int64_t flags_len,
                                 int max_baselines, int max_grid_n, int weighting, int precision,
                                 int shift, float *images, int64_t images_len, double *weight_sum,
                                 int32_t *n_out, int32_t *status, void *workspace,
                                 size_t workspace_bytes, void *hip_stream, int *block_threads,
                                 int *workgroups, double *best_ms);

/* A captured hipGraph of one blink_image_batch_desc call (same arguments, same buffers). Launch
 * replays it on any stream; descriptor and input contents may change between launches within the
 * maxima given at capture. */
typedef struct blink_graph_s *blink_graph;
blink_status blink_graph_create_desc(blink_ctx ctx, const blink_image_desc *desc, int n_img,
                                     const blink_cf32 *vis, int64_t vis_len, const double *uvw_m,
                                     int64_t uvw_len, const uint8_t *flags, int64_t flags_len,
                                     int max_baselines, int max_grid_n, int weighting,
                                     int precision, int shift, float *images, int64_t images_len,
                                     double *weight_sum, int32_t *n_out, int32_t *status,
                                     void *workspace, size_t workspace_bytes, blink_graph *out);
blink_status blink_graph_launch(blink_graph graph, void *hip_stream);
blink_status blink_graph_destroy(blink_graph graph);

/* ---------------------------------------------------------------- execution plans and autotuning
 * Not part of the method: how blink_image_batch schedules its kernels for one grid size,
 * weighting and precision form (each has its own plan; blink_ifft2d uses the row_block of the
 * natural-weighting plan of its precision). A plan never changes results beyond rounding order.
 * Fields:
 *   col_strip  columns of the half spectrum per workgroup of the fused gridding + column FFT kernel
 *   row_block  row-pair transforms per workgroup of the row FFT kernel
 *   group      images per column/row launch pair (0 = as many as the workspace holds, at most 256
 *              with the queried workspace); small groups keep the intermediates in the last-level
 *              cache between the two passes.
 *   col_loop   strips each workgroup of the fused gridding + column FFT kernel takes in turn
 *              (1 .. 64; 1 = one strip per workgroup). Above 1 the workgroup requests the next
 *              strips' placements while it transforms and stores the current one. */

/* Compiled options for grid_n and weighting (the same for every precision form): up to 4 strip
 * widths and 4 row blocks each. */
blink_status blink_plan_options(int grid_n, int weighting, int *col_strips, int *n_col,
                                int *row_blocks, int *n_row);

/* Current plan of a context (a default until set or tuned). */
blink_status blink_get_plan(blink_ctx ctx, int grid_n, int weighting, int precision,
                            int *col_strip, int *row_block, int *group, int *col_loop);

/* Set a plan; col_strip and row_block must be compiled options, group >= 0, 1 <= col_loop <= 64. */
blink_status blink_set_plan(blink_ctx ctx, int grid_n, int weighting, int precision,
                            int col_strip, int row_block, int group, int col_loop);

/* Autotuner: runs blink_image_batch on the caller's problem (same arguments) for every compiled
 * (col_strip, row_block) pair and group sizes 16, 24, 32, 48, 64, 96, 128, 256 with col_loop 1,
 * then every group with col_loop 2, 4, .. 16 and the strip width and row block of the fastest of
 * those; times each with hipEvents on hip_stream and keeps the fastest as the context's plan for
 * (grid_n, weighting, precision). Synchronises with the host. On return
 * `images` etc. hold a valid result, and col_strip, row_block, group, col_loop and best_ms (any
 * may be NULL) describe the choice. */
blink_status blink_autotune_image_batch(blink_ctx ctx, const blink_cf32 *vis, const uint8_t *flags,
                                        const double *uvw_m, const double *freq_hz, int T, int C,
                                        int P, int B, int grid_n, double pixel_scale, int weighting,
                                        int precision, int shift, float *images, double *weight_sum,
                                        int32_t *n_out, void *workspace, size_t workspace_bytes,
                                        void *hip_stream, int *col_strip, int *row_block,
                                        int *group, int *col_loop, double *best_ms);

/* ---------------------------------------------------------------- kernel timing
 * Not part of the method: per-kernel timing for measurement. While enabled, every kernel launch
 * of the entry points above is bracketed by a pair of hipEvents recorded on the caller's stream.
 * Kernel ids: */
enum {
    BLINK_KERNEL_BIN = 0,          /* cell indices + strip binning, one workgroup per (t, c) */
    BLINK_KERNEL_GRID = 1,         /* full-grid gridding (blink_grid) */
    BLINK_KERNEL_GRID_COLFFT = 2,  /* fused gridding + column FFT (blink_image_batch) */
    BLINK_KERNEL_DENSE_COLFFT = 3, /* column FFT of dense grids (blink_ifft2d) */
    BLINK_KERNEL_WEIGHTS = 4,      /* per-image 1/W */
    BLINK_KERNEL_ROW_FFT = 5,      /* row FFT, real part, 1/W, image store */
    BLINK_KERNEL_DESC_PREP = 6,    /* descriptor checks and image order (uneven batches) */
    BLINK_KERNEL_PERSISTENT = 7,   /* persistent fused binning + gridding + FFT (uneven batches) */
    BLINK_KERNEL_CONV_CORRECTION = 8, /* grid-correction table of the convolutional path */
    BLINK_KERNEL_AVERAGE = 9,      /* image averages (blink_image_average) */
    BLINK_KERNEL_CORRECT = 10,     /* visibility corrections (blink_image_batch_corrected) */
    BLINK_KERNEL_CORRELATE = 11,   /* correlator (blink_correlate) */
    BLINK_KERNEL_DEDISPERSE = 12,  /* de-dispersion (blink_dedisperse) */
    BLINK_KERNEL_COUNT = 13
};

/* Enable (nonzero) or disable timing; either way the recorded launches are discarded. */
blink_status blink_profile_enable(blink_ctx ctx, int enable);

/* Sum of the recorded durations (ms) and the number of launches of one kernel id since timing
 * was enabled. Waits for the recorded events to complete (a host synchronisation). */
blink_status blink_profile_read(blink_ctx ctx, int kernel, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif
