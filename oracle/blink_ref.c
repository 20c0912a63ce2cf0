/*
 * blink_ref.c — FP64 CPU oracle for batched dirty imaging (test infrastructure only).
 *
 * The definitions and the readings of the paper it follows are stated in blink_ref.h.
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (no fast-math).
 */
#include "blink_ref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define SPEED_OF_LIGHT 299792458.0

static int is_pow2(int n) { return n >= 2 && n <= 16384 && (n & (n - 1)) == 0; }

static int mod_n(int a, int n) { int r = a % n; return r < 0 ? r + n : r; }

/* Section 4, Eq. 5: the grid has N cells per side; with pixel scale dl the image spans N*dl in
 * direction cosine, so a cell is 1/(N dl) wavelengths wide and u metres are u f / c wavelengths.
 * The product is evaluated as (f / c) * (N * dl). */
double blink_ref_cells_per_metre(double freq_hz, int grid_n, double pixel_scale)
{
    double cycles_per_metre = freq_hz / SPEED_OF_LIGHT;
    double cells_per_wavelength = (double)grid_n * pixel_scale;
    return cycles_per_metre * cells_per_wavelength;
}

/* Section 6.2.4: nearest-cell placement with no convolution kernel; natural weighting by default.
 * Hermitian completion: the visibility of baseline (i,j) at (u,v) implies conj(V) at (-u,-v).
 * The visibilities come either as complex64 (vis32) or as complex double (vis64). */
static int grid_one(const float *vis32, const double *vis64, const uint8_t *flags, const double *uvw,
                    int P, int B, double freq_hz, int grid_n, double pixel_scale, int weighting,
                    double *grid, int32_t *counts, int32_t *cell_idx,
                    double *weight_sum, int32_t *n_out)
{
    if (!is_pow2(grid_n) || P < 1 || B < 0 || !(vis32 || vis64) || !uvw || !grid || !weight_sum || !n_out)
        return 1;
    if (weighting != 0 && weighting != 1)
        return 1;
    const int N = grid_n;
    const size_t NN = (size_t)N * N;
    int32_t *cnt = (int32_t *)calloc(NN, sizeof(int32_t));
    if (!cnt)
        return 2;
    memset(grid, 0, sizeof(double) * 2 * NN * (size_t)P);

    const double k = blink_ref_cells_per_metre(freq_hz, N, pixel_scale);
    const double half = (double)(N / 2);
    int32_t outside = 0;
    int64_t kept = 0;
    for (int b = 0; b < B; ++b) {
        if (flags && flags[b]) {
            if (cell_idx) cell_idx[b] = -1;
            continue;
        }
        double xu = uvw[3 * (size_t)b + 0] * k;   /* one IEEE double product each */
        double xv = uvw[3 * (size_t)b + 1] * k;
        double ru = nearbyint(xu);                /* round half to even */
        double rv = nearbyint(xv);
        if (!(fabs(ru) < half && fabs(rv) < half)) {
            if (cell_idx) cell_idx[b] = -2;
            ++outside;
            continue;
        }
        int iu = (int)ru, iv = (int)rv;
        size_t c1 = (size_t)mod_n(iv, N) * N + mod_n(iu, N);
        size_t c2 = (size_t)mod_n(-iv, N) * N + mod_n(-iu, N);
        if (cell_idx) cell_idx[b] = (int32_t)c1;
        cnt[c1] += 1;
        cnt[c2] += 1;
        ++kept;
        for (int p = 0; p < P; ++p) {
            const size_t at = 2 * ((size_t)p * B + b);
            double re = vis64 ? vis64[at] : (double)vis32[at];
            double im = vis64 ? vis64[at + 1] : (double)vis32[at + 1];
            double *g = grid + 2 * NN * (size_t)p;
            g[2 * c1] += re;
            g[2 * c1 + 1] += im;
            g[2 * c2] += re;
            g[2 * c2 + 1] -= im;
        }
    }

    double W;
    if (weighting == 0) {
        W = 2.0 * (double)kept;
    } else {
        int64_t occupied = 0;
        for (size_t c = 0; c < NN; ++c) {
            if (cnt[c] == 0) continue;
            ++occupied;
            for (int p = 0; p < P; ++p) {
                double *g = grid + 2 * NN * (size_t)p;
                g[2 * c] /= (double)cnt[c];
                g[2 * c + 1] /= (double)cnt[c];
            }
        }
        W = (double)occupied;
    }
    if (counts) memcpy(counts, cnt, sizeof(int32_t) * NN);
    *weight_sum = W;
    *n_out = outside;
    free(cnt);
    return 0;
}

int blink_ref_grid(const float *vis, const uint8_t *flags, const double *uvw, int P, int B,
                   double freq_hz, int grid_n, double pixel_scale, int weighting,
                   double *grid, int32_t *counts, int32_t *cell_idx,
                   double *weight_sum, int32_t *n_out)
{
    if (!vis) return 1;
    return grid_one(vis, NULL, flags, uvw, P, B, freq_hz, grid_n, pixel_scale, weighting, grid, counts,
                    cell_idx, weight_sum, n_out);
}

/* Section 4: the dirty image as the direct inverse transform of the samples, one baseline at a
 * time; the kept set and W follow the nearest-cell rules of grid_one. */
int blink_ref_dft(const float *vis, const uint8_t *flags, const double *uvw, int P, int B,
                  double freq_hz, int grid_n, double pixel_scale, int snap, int shift,
                  double *image, double *weight_sum, int32_t *n_out)
{
    if (!is_pow2(grid_n) || P < 1 || B < 0 || (B > 0 && (!vis || !uvw)) || !image || !weight_sum || !n_out)
        return 1;
    const int N = grid_n;
    const size_t NN = (size_t)N * N;
    memset(image, 0, sizeof(double) * NN * (size_t)P);
    const double k = blink_ref_cells_per_metre(freq_hz, N, pixel_scale);
    const double half = (double)(N / 2);
    const double two_pi = 2.0 * M_PI;
    int64_t kept = 0;
    int32_t outside = 0;
    for (int b = 0; b < B; ++b) {
        if (flags && flags[b])
            continue;
        double xu = uvw[3 * (size_t)b + 0] * k;
        double xv = uvw[3 * (size_t)b + 1] * k;
        double ru = nearbyint(xu), rv = nearbyint(xv);
        if (!(fabs(ru) < half) || !(fabs(rv) < half)) {     /* NaN is outside too */
            ++outside;
            continue;
        }
        ++kept;
        const double a = snap ? ru : xu;
        const double c = snap ? rv : xv;
        for (int p = 0; p < P; ++p) {
            const double re = (double)vis[2 * ((size_t)p * B + b)];
            const double im = (double)vis[2 * ((size_t)p * B + b) + 1];
            double *img = image + NN * (size_t)p;
            for (int y = 0; y < N; ++y) {
                const double Y = shift ? (double)(y - N / 2) : (double)y;
                for (int x = 0; x < N; ++x) {
                    const double X = shift ? (double)(x - N / 2) : (double)x;
                    const double phase = two_pi * (a * X + c * Y) / (double)N;
                    img[(size_t)y * N + x] += 2.0 * (re * cos(phase) - im * sin(phase));
                }
            }
        }
    }
    const double W = (double)(2 * kept);    /* the kept visibilities and their mirrors */
    for (size_t i = 0; i < NN * (size_t)P; ++i)
        image[i] = W > 0.0 ? image[i] / W : 0.0;
    *weight_sum = W;
    *n_out = outside;
    return 0;
}

/* Textbook iterative radix-2 decimation-in-time FFT with the + sign of the inverse transform
 * (the image side of Eq. 4's exp(-i2pi(ul+vm))). Twiddles cos/sin(2 pi j / n) from libm. */
int blink_ref_ifft1d(double *a, int n)
{
    if (!is_pow2(n) && n != 1) return 1;
    if (!a) return 1;
    if (n == 1) return 0;
    /* bit-reversal permutation */
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double tr = a[2 * i], ti = a[2 * i + 1];
            a[2 * i] = a[2 * j]; a[2 * i + 1] = a[2 * j + 1];
            a[2 * j] = tr; a[2 * j + 1] = ti;
        }
    }
    for (int len = 2; len <= n; len <<= 1) {
        int h = len / 2;
        for (int k = 0; k < h; ++k) {
            double ang = 2.0 * M_PI * (double)k / (double)len;
            double wr = cos(ang), wi = sin(ang);
            for (int i = 0; i < n; i += len) {
                double *x = a + 2 * (i + k), *y = a + 2 * (i + k + h);
                double tr = wr * y[0] - wi * y[1];
                double ti = wr * y[1] + wi * y[0];
                y[0] = x[0] - tr; y[1] = x[1] - ti;
                x[0] = x[0] + tr; x[1] = x[1] + ti;
            }
        }
    }
    return 0;
}

/* Eq. 5 and Section 6.2.4: dirty image = inverse 2D FFT of the grid (rows, then columns),
 * then the shift that moves the phase centre from the corner to the middle, then the real
 * part, normalised by the weight sum so a 1 Jy source at the phase centre peaks at 1. */
int blink_ref_ifft2d(const double *grid, int grid_n, double weight_sum, int shift,
                     double *image, double *imag_max)
{
    if (!is_pow2(grid_n) || !grid || !image) return 1;
    const int N = grid_n;
    const size_t NN = (size_t)N * N;
    if (!(weight_sum > 0.0) || !isfinite(weight_sum)) {
        memset(image, 0, sizeof(double) * NN);
        if (imag_max) *imag_max = 0.0;
        return 0;
    }
    double *work = (double *)malloc(sizeof(double) * 2 * NN);
    double *col = (double *)malloc(sizeof(double) * 2 * (size_t)N);
    if (!work || !col) { free(work); free(col); return 2; }
    memcpy(work, grid, sizeof(double) * 2 * NN);
    for (int r = 0; r < N; ++r)                 /* along u (x) */
        blink_ref_ifft1d(work + 2 * (size_t)r * N, N);
    for (int c = 0; c < N; ++c) {               /* along v (y) */
        for (int r = 0; r < N; ++r) {
            col[2 * r] = work[2 * ((size_t)r * N + c)];
            col[2 * r + 1] = work[2 * ((size_t)r * N + c) + 1];
        }
        blink_ref_ifft1d(col, N);
        for (int r = 0; r < N; ++r) {
            work[2 * ((size_t)r * N + c)] = col[2 * r];
            work[2 * ((size_t)r * N + c) + 1] = col[2 * r + 1];
        }
    }
    const double inv = 1.0 / weight_sum;
    double im_max = 0.0;
    const int s = shift ? N / 2 : 0;
    for (int y = 0; y < N; ++y) {
        int ry = (y + s) % N;                   /* fftshift: output y holds raw (y - N/2) mod N */
        for (int x = 0; x < N; ++x) {
            int rx = (x + s) % N;
            const double *w = work + 2 * ((size_t)ry * N + rx);
            image[(size_t)y * N + x] = w[0] * inv;
            double ai = fabs(w[1] * inv);
            if (ai > im_max) im_max = ai;
        }
    }
    if (imag_max) *imag_max = im_max;
    free(work);
    free(col);
    return 0;
}

int blink_ref_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int image_batch(const float *vis32, const double *vis64, const uint8_t *flags, const double *uvw,
                       const double *freq_hz, int T, int C, int P, int B, int grid_n,
                       double pixel_scale, int weighting, int shift, double *images,
                       double *weight_sum, int32_t *n_out, int32_t *cell_idx,
                       int32_t *counts, int n_threads)
{
    if (!is_pow2(grid_n) || T < 0 || C < 0 || P < 1 || B < 0) return 1;
    if (!(vis32 || vis64) || !uvw || !freq_hz || !images) return 1;
    if (weighting != 0 && weighting != 1) return 1;
    const int N = grid_n;
    const size_t NN = (size_t)N * N;
    const long n_tc = (long)T * C;
    int err = 0;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads) reduction(max : err)
#endif
    for (long tc = 0; tc < n_tc; ++tc) {
        const long t = tc / C, c = tc % C;
        double *grid = (double *)malloc(sizeof(double) * 2 * NN * (size_t)P);
        if (!grid) { err = 2; continue; }
        double W = 0.0;
        int32_t nout = 0;
        const size_t at = 2 * (size_t)tc * P * B;
        int rc = grid_one(vis32 ? vis32 + at : NULL, vis64 ? vis64 + at : NULL,
                          flags ? flags + (size_t)tc * B : NULL, uvw + 3 * (size_t)t * B, P, B, freq_hz[c],
                          N, pixel_scale, weighting, grid, counts ? counts + (size_t)tc * NN : NULL,
                          cell_idx ? cell_idx + (size_t)tc * B : NULL, &W, &nout);
        for (int p = 0; rc == 0 && p < P; ++p) {
            rc = blink_ref_ifft2d(grid + 2 * NN * (size_t)p, N, W, shift,
                                  images + ((size_t)tc * P + p) * NN, NULL);
            if (weight_sum) weight_sum[(size_t)tc * P + p] = W;
        }
        if (n_out) n_out[tc] = nout;
        if (rc > err) err = rc;
        free(grid);
    }
    return err;
}

int blink_ref_image_batch(const float *vis, const uint8_t *flags, const double *uvw,
                          const double *freq_hz, int T, int C, int P, int B, int grid_n,
                          double pixel_scale, int weighting, int shift, double *images,
                          double *weight_sum, int32_t *n_out, int32_t *cell_idx,
                          int32_t *counts, int n_threads)
{
    if (!vis) return 1;
    return image_batch(vis, NULL, flags, uvw, freq_hz, T, C, P, B, grid_n, pixel_scale, weighting, shift,
                       images, weight_sum, n_out, cell_idx, counts, n_threads);
}

int blink_ref_image_batch_c128(const double *vis, const uint8_t *flags, const double *uvw,
                               const double *freq_hz, int T, int C, int P, int B, int grid_n,
                               double pixel_scale, int weighting, int shift, double *images,
                               double *weight_sum, int32_t *n_out, int32_t *cell_idx,
                               int32_t *counts, int n_threads)
{
    if (!vis) return 1;
    return image_batch(NULL, vis, flags, uvw, freq_hz, T, C, P, B, grid_n, pixel_scale, weighting, shift,
                       images, weight_sum, n_out, cell_idx, counts, n_threads);
}

/* ------------------------------------------------------------------------------------------
 * Visibility corrections before gridding (Section 6.2.3): calibration
 * solutions applied per antenna, then the geometric correction that moves the phase centre to the
 * pointing direction (the paper does that step in the imager, where (u, v, w) are known). Cable
 * length corrections are per-antenna phases and enter through the same per-antenna factors.
 * Baseline b is the cross pair (i, j), i > j, b = i (i - 1) / 2 + j: the lower-triangular order
 * in which the correlation step stores visibilities (Section 6.2.2), without autocorrelations.
 * ------------------------------------------------------------------------------------------ */
int blink_ref_correct_vis(const float *vis, const double *uvw, const double *freq_hz, int T, int C,
                          int P, int B, const float *gains, int n_ant, double l0, double m0,
                          double *out)
{
    if (T < 0 || C < 0 || P < 1 || B < 0 || !vis || !uvw || !freq_hz || !out) return 1;
    if (gains && (n_ant < 2 || (long)n_ant * (n_ant - 1) / 2 != B)) return 1;
    if (!(l0 * l0 + m0 * m0 < 1.0)) return 1;
    const double n0 = sqrt(1.0 - l0 * l0 - m0 * m0);
    /* antenna pair of every baseline, in baseline order */
    int *ant_i = (int *)malloc(sizeof(int) * (size_t)(B > 0 ? B : 1));
    int *ant_j = (int *)malloc(sizeof(int) * (size_t)(B > 0 ? B : 1));
    if (!ant_i || !ant_j) { free(ant_i); free(ant_j); return 2; }
    if (gains) {
        int b = 0;
        for (int i = 1; i < n_ant; ++i)
            for (int j = 0; j < i; ++j, ++b) { ant_i[b] = i; ant_j[b] = j; }
    }
    for (int t = 0; t < T; ++t) {
        for (int c = 0; c < C; ++c) {
            const double cycles_per_metre = freq_hz[c] / SPEED_OF_LIGHT;
            for (int b = 0; b < B; ++b) {
                const double *x = uvw + 3 * ((size_t)t * B + b);
                /* geometric delay of the new phase centre, in turns: (f/c)(u l0 + v m0 + w (n0 - 1)) */
                const double turns = cycles_per_metre * (x[0] * l0 + x[1] * m0 + x[2] * (n0 - 1.0));
                const double rot_re = cos(2.0 * M_PI * turns), rot_im = sin(2.0 * M_PI * turns);
                for (int p = 0; p < P; ++p) {
                    const size_t at = 2 * ((((size_t)t * C + c) * P + p) * B + b);
                    double re = (double)vis[at], im = (double)vis[at + 1];
                    if (gains) {
                        /* J_i V conj(J_j) */
                        const float *gi = gains + 2 * (((size_t)c * P + p) * n_ant + ant_i[b]);
                        const float *gj = gains + 2 * (((size_t)c * P + p) * n_ant + ant_j[b]);
                        const double ar = gi[0], ai = gi[1], br = gj[0], bi = -(double)gj[1];
                        const double r1 = ar * re - ai * im, i1 = ar * im + ai * re;
                        re = r1 * br - i1 * bi;
                        im = r1 * bi + i1 * br;
                    }
                    out[at] = re * rot_re - im * rot_im;
                    out[at + 1] = re * rot_im + im * rot_re;
                }
            }
        }
    }
    free(ant_i);
    free(ant_j);
    return 0;
}

/* ------------------------------------------------------------------------------------------
 * Convolutional gridding (a step beyond the paper: Section 6.2.4 places visibilities with no
 * convolution kernel and names one as a planned improvement against aliasing; Section 10 lists
 * it as work in progress). The kernel is the "exponential of semicircle" of Barnett, Magland and
 * af Klinteberg (2019): phi(z) = exp(beta (sqrt(1 - z^2) - 1)) for |z| < 1, else 0, applied
 * separably in u and v with z = 2 d / W for a cell offset d and a support of W cells. The
 * image is divided by the kernel's continuous Fourier transform at each pixel (grid correction).
 * ------------------------------------------------------------------------------------------ */

double blink_ref_es_kernel(double z, double beta)
{
    if (!(fabs(z) < 1.0)) return 0.0;
    return exp(beta * (sqrt(1.0 - z * z) - 1.0));
}

/* c(nu) = integral over |d| < W/2 of phi(2d/W) cos(2 pi nu d) dd. With d = (W/2) sin(theta)
 * the integrand is smooth: c(nu) = W * integral_0^{pi/2} exp(beta (cos t - 1)) cos(pi nu W sin t)
 * cos t dt, evaluated by composite Simpson's rule on 4096 intervals. */
double blink_ref_es_transform(double nu, int width, double beta)
{
    const int M = 4096;
    const double h = (M_PI / 2.0) / M;
    double s = 0.0;
    for (int i = 0; i <= M; ++i) {
        double t = i * h;
        double f = exp(beta * (cos(t) - 1.0)) * cos(M_PI * nu * width * sin(t)) * cos(t);
        double w = (i == 0 || i == M) ? 1.0 : ((i % 2) ? 4.0 : 2.0);
        s += w * f;
    }
    return (double)width * s * h / 3.0;
}

/* One visibility value spread over the cells j (integers with |j - x| < W/2) of each axis with
 * weights phi(2 (j - x) / W); cells wrap modulo N. */
static void spread(double *g, int N, double xu, double xv, int width, double beta, double re, double im)
{
    const double h = 0.5 * width;
    int ju0 = (int)ceil(xu - h), jv0 = (int)ceil(xv - h);
    for (int jv = jv0; jv < xv + h; ++jv) {
        if (!(fabs(jv - xv) < h)) continue;
        double wv = blink_ref_es_kernel(2.0 * (jv - xv) / width, beta);
        for (int ju = ju0; ju < xu + h; ++ju) {
            if (!(fabs(ju - xu) < h)) continue;
            double w = wv * blink_ref_es_kernel(2.0 * (ju - xu) / width, beta);
            size_t c = (size_t)mod_n(jv, N) * N + mod_n(ju, N);
            g[2 * c] += w * re;
            g[2 * c + 1] += w * im;
        }
    }
}

int blink_ref_grid_conv(const float *vis, const uint8_t *flags, const double *uvw, int P, int B,
                        double freq_hz, int grid_n, double pixel_scale, int width, double beta,
                        double *grid, double *weight_sum, int32_t *n_out)
{
    if (!is_pow2(grid_n) || P < 1 || B < 0 || !vis || !uvw || !grid || !weight_sum || !n_out)
        return 1;
    if (width < 1 || width > 16 || !(beta >= 0.0) || !isfinite(beta) || width >= grid_n) return 1;
    const int N = grid_n;
    const size_t NN = (size_t)N * N;
    memset(grid, 0, sizeof(double) * 2 * NN * (size_t)P);
    const double k = blink_ref_cells_per_metre(freq_hz, N, pixel_scale);
    const double half = (double)(N / 2);
    int32_t outside = 0;
    int64_t kept = 0;
    for (int b = 0; b < B; ++b) {
        if (flags && flags[b]) continue;
        double xu = uvw[3 * (size_t)b + 0] * k;
        double xv = uvw[3 * (size_t)b + 1] * k;
        double ru = nearbyint(xu), rv = nearbyint(xv);
        if (!(fabs(rv) < half && fabs(ru) < half)) {   /* the nearest-cell keep rule */
            ++outside;
            continue;
        }
        ++kept;
        for (int p = 0; p < P; ++p) {
            const float *v = vis + 2 * ((size_t)p * B + b);
            double re = (double)v[0], im = (double)v[1];
            double *g = grid + 2 * NN * (size_t)p;
            spread(g, N, xu, xv, width, beta, re, im);      /* V at (u, v) */
            spread(g, N, -xu, -xv, width, beta, re, -im);   /* conj V at (-u, -v) */
        }
    }
    *weight_sum = 2.0 * (double)kept;
    *n_out = outside;
    return 0;
}

/* Grid correction of one axis: corr[x] = c(X / N) for pixel x, X its signed offset from the phase
 * centre (x - N/2 when shifted, else x for x < N/2 and x - N above). */
int blink_ref_conv_correction(int grid_n, int width, double beta, int shift, double *corr)
{
    if (!is_pow2(grid_n) || !corr || width < 1 || width > 16 || !(beta >= 0.0)) return 1;
    const int N = grid_n;
    for (int x = 0; x < N; ++x) {
        int X = shift ? x - N / 2 : (x < N / 2 ? x : x - N);
        corr[x] = blink_ref_es_transform((double)X / N, width, beta);
    }
    return 0;
}

int blink_ref_image_batch_conv(const float *vis, const uint8_t *flags, const double *uvw,
                               const double *freq_hz, int T, int C, int P, int B, int grid_n,
                               double pixel_scale, int width, double beta, int shift, double *images,
                               double *weight_sum, int32_t *n_out, int n_threads)
{
    if (!is_pow2(grid_n) || T < 0 || C < 0 || P < 1 || B < 0) return 1;
    if (!vis || !uvw || !freq_hz || !images) return 1;
    const int N = grid_n;
    const size_t NN = (size_t)N * N;
    double *corr = (double *)malloc(sizeof(double) * (size_t)N);
    if (!corr) return 2;
    if (blink_ref_conv_correction(N, width, beta, shift, corr)) { free(corr); return 1; }
    const long n_tc = (long)T * C;
    int err = 0;
#ifdef _OPENMP
    if (n_threads <= 0) n_threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads) reduction(max : err)
#endif
    for (long tc = 0; tc < n_tc; ++tc) {
        const long t = tc / C, c = tc % C;
        double *grid = (double *)malloc(sizeof(double) * 2 * NN * (size_t)P);
        if (!grid) { err = 2; continue; }
        double W = 0.0;
        int32_t nout = 0;
        int rc = blink_ref_grid_conv(vis + 2 * (size_t)tc * P * B, flags ? flags + (size_t)tc * B : NULL,
                                     uvw + 3 * (size_t)t * B, P, B, freq_hz[c], N, pixel_scale, width, beta,
                                     grid, &W, &nout);
        for (int p = 0; rc == 0 && p < P; ++p) {
            double *img = images + ((size_t)tc * P + p) * NN;
            rc = blink_ref_ifft2d(grid + 2 * NN * (size_t)p, N, W, shift, img, NULL);
            for (int y = 0; rc == 0 && y < N; ++y)
                for (int x = 0; x < N; ++x) img[(size_t)y * N + x] /= corr[x] * corr[y];
            if (weight_sum) weight_sum[(size_t)tc * P + p] = W;
        }
        if (n_out) n_out[tc] = nout;
        if (rc > err) err = rc;
        free(grid);
    }
    free(corr);
    return err;
}

/* ------------------------------------------------------------------------------------------
 * Image averages (Sections 7.2 and 7.3: images are averaged over time and over the band, e.g.
 * all channels of one time bin). images [T][C][P][N][N] float; each axis selected in `axes`
 * (1 time, 2 channel, 4 polarisation) is averaged (its extent becomes 1), the others are kept:
 * out [T'][C'][P'][N][N] double. Over P = 2 (XX, YY) this is Stokes I = (XX + YY) / 2.
 * ------------------------------------------------------------------------------------------ */
int blink_ref_image_average(const float *images, int T, int C, int P, int grid_n, int axes, double *out)
{
    if (!images || !out || T < 1 || C < 1 || P < 1 || grid_n < 1 || axes < 0 || axes > 7) return 1;
    const size_t NN = (size_t)grid_n * grid_n;
    const int To = (axes & 1) ? 1 : T, Co = (axes & 2) ? 1 : C, Po = (axes & 4) ? 1 : P;
    const double count = (double)((axes & 1) ? T : 1) * ((axes & 2) ? C : 1) * ((axes & 4) ? P : 1);
    memset(out, 0, sizeof(double) * NN * (size_t)To * Co * Po);
    for (int t = 0; t < T; ++t)
        for (int c = 0; c < C; ++c)
            for (int p = 0; p < P; ++p) {
                int to = (axes & 1) ? 0 : t, co = (axes & 2) ? 0 : c, po = (axes & 4) ? 0 : p;
                const float *src = images + (((size_t)t * C + c) * P + p) * NN;
                double *dst = out + (((size_t)to * Co + co) * Po + po) * NN;
                for (size_t i = 0; i < NN; ++i) dst[i] += (double)src[i];
            }
    const size_t total = NN * (size_t)To * Co * Po;
    for (size_t i = 0; i < total; ++i) out[i] /= count;
    return 0;
}

/* ------------------------------------------------------------------------------------------
 * Correlation (Section 4, Eq. 3; Section 6.2.2): the conjugate multiply-accumulate of every
 * pair of fine-channelised antenna voltages, averaged over an integration interval and over the
 * fine channels of an output channel. Voltages are complex int8 (re, im) in the layout
 * [S samples][F fine channels][A antennas][2 polarisations]; visibility (i, j), i > j, of
 * polarisations (p, q) is mean(x_{i,p} conj(x_{j,q})) over n_int samples and n_favg channels.
 * ------------------------------------------------------------------------------------------ */
int blink_ref_correlate(const int8_t *volt, int S, int F, int A, int n_int, int n_favg, int pol_mode,
                        float *vis, float *autos)
{
    if (S < 0 || F < 0 || A < 2 || n_int < 1 || n_favg < 1 || !volt || !vis) return 1;
    if (S % n_int != 0 || F % n_favg != 0) return 1;
    if (pol_mode != 2 && pol_mode != 4) return 1;
    const int T = S / n_int, C = F / n_favg, P = pol_mode;
    const long B = (long)A * (A - 1) / 2;
    const double count = (double)n_int * (double)n_favg;
    for (int t = 0; t < T; ++t) {
        for (int c = 0; c < C; ++c) {
            for (int i = 0; i < A; ++i) {
                for (int j = 0; j <= i; ++j) {
                    for (int p = 0; p < 2; ++p) {
                        for (int q = 0; q < 2; ++q) {
                            int64_t sre = 0, sim = 0;
                            for (int s = t * n_int; s < (t + 1) * n_int; ++s) {
                                for (int f = c * n_favg; f < (c + 1) * n_favg; ++f) {
                                    const int8_t *xi = volt + ((((size_t)s * F + f) * A + i) * 2 + p) * 2;
                                    const int8_t *xj = volt + ((((size_t)s * F + f) * A + j) * 2 + q) * 2;
                                    /* x_i conj(x_j) */
                                    sre += (int64_t)xi[0] * xj[0] + (int64_t)xi[1] * xj[1];
                                    sim += (int64_t)xi[1] * xj[0] - (int64_t)xi[0] * xj[1];
                                }
                            }
                            const float re = (float)((double)sre / count), im = (float)((double)sim / count);
                            if (i == j) {
                                if (autos) {
                                    float *o = autos + 2 * ((((size_t)t * C + c) * A + i) * 4 + 2 * p + q);
                                    o[0] = re;
                                    o[1] = im;
                                }
                                continue;
                            }
                            int pp;
                            if (P == 4) pp = 2 * p + q;
                            else if (p == q) pp = p;
                            else continue;
                            const long b = (long)i * (i - 1) / 2 + j;
                            float *o = vis + 2 * ((((size_t)t * C + c) * P + pp) * B + b);
                            o[0] = re;
                            o[1] = im;
                        }
                    }
                }
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------------------------
 * Incoherent de-dispersion of image cubes (the FRB search that the images feed, Sections 1, 3 and
 * 10; Table 1 gives a DM of 600 pc cm^-3 and tens of seconds of dispersive delay over the MWA
 * band). A pulse of dispersion measure DM reaches channel frequency f later than the highest
 * channel f_ref by k_DM DM (f^-2 - f_ref^-2), k_DM = 4148.808 s MHz^2 cm^3 / pc (the cold-plasma
 * dispersion constant; frequencies in MHz). In samples of length dt the delay is rounded to the
 * nearest integer; the de-dispersed image at output step t is the mean over channels of the
 * channel images at steps t + delay(c).
 * ------------------------------------------------------------------------------------------ */
#define K_DM_S_MHZ2 4148.808

int blink_ref_dispersion_delays(const double *freq_hz, int C, double dt_s, const double *dm, int n_dm,
                                int32_t *delays)
{
    if (C < 1 || n_dm < 0 || !(dt_s > 0.0) || !freq_hz || (n_dm > 0 && (!dm || !delays))) return 1;
    double f_ref = freq_hz[0];
    for (int c = 1; c < C; ++c)
        if (freq_hz[c] > f_ref) f_ref = freq_hz[c];
    const double ref_mhz = f_ref / 1.0e6;
    for (int k = 0; k < n_dm; ++k) {
        if (!(dm[k] >= 0.0)) return 1;
        for (int c = 0; c < C; ++c) {
            const double f_mhz = freq_hz[c] / 1.0e6;
            const double delay_s = K_DM_S_MHZ2 * dm[k] * (1.0 / (f_mhz * f_mhz) - 1.0 / (ref_mhz * ref_mhz));
            delays[(size_t)k * C + c] = (int32_t)nearbyint(delay_s / dt_s);
        }
    }
    return 0;
}

int blink_ref_dedisperse(const float *images, int T, int C, int grid_n, const int32_t *delays, int n_dm,
                         int t_out, double *out)
{
    if (T < 0 || C < 1 || grid_n < 1 || n_dm < 0 || t_out < 0 || !images || (n_dm > 0 && (!delays || !out)))
        return 1;
    const size_t NN = (size_t)grid_n * grid_n;
    for (int k = 0; k < n_dm; ++k)
        for (int c = 0; c < C; ++c) {
            const int32_t d = delays[(size_t)k * C + c];
            if (d < 0 || (long)t_out + d > T) return 1;
        }
    for (int k = 0; k < n_dm; ++k) {
        for (int t = 0; t < t_out; ++t) {
            double *o = out + ((size_t)k * t_out + t) * NN;
            for (size_t i = 0; i < NN; ++i) o[i] = 0.0;
            for (int c = 0; c < C; ++c) {
                const int ts = t + delays[(size_t)k * C + c];
                const float *in = images + ((size_t)ts * C + c) * NN;
                for (size_t i = 0; i < NN; ++i) o[i] += (double)in[i];
            }
            for (size_t i = 0; i < NN; ++i) o[i] /= (double)C;
        }
    }
    return 0;
}
