/*
 * FP64 CPU oracle for the discrete Fourier transform -- TEST INFRASTRUCTURE.
 * Only tests, the smoke check and the benchmark's CPU-baseline leg use it; the
 * GPU library never links or calls it.  See oracle.h for the conventions.
 *
 * Two independent routes to the same numbers:
 *   1. oracle_dft: the defining sum, O(N^2), every angle 2*pi*((j*k) mod N)/N
 *      evaluated with libm cos/sin in double (no table, no recursion).
 *   2. oracle_fft: the Cooley-Tukey recursion the paper describes (section
 *      III-A): a length-N DFT is assembled from p interleaved DFTs of length
 *      N/p.  The paper uses p = 2 throughout (radix-2 decimation in time);
 *      here p is the smallest prime factor of N, so powers of two recurse
 *      exactly as radix-2 DIT and 7-smooth lengths use p in {3, 5, 7} where
 *      needed.  A length whose smallest prime factor exceeds 7 is summed
 *      directly.  Combination step, for k = 0..N-1 with m = N/p:
 *          X[k] = sum_{r=0}^{p-1} w_N^{(r k) mod N} * Y_r[k mod m],
 *      where Y_r is the length-m DFT of x[r], x[r+p], x[r+2p], ...
 *      Twiddles w_N^t come from one table per top-level N, each entry computed
 *      directly with cos/sin (no recurrence); a sub-problem of length n reads
 *      w_n^t = w_N^{t N/n}.
 * The inverse uses the identity  ifft(x) = conj(fft(conj(x))) / N.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double re, im;
} cplx;

static const double TWO_PI = 6.283185307179586476925286766559;

static inline cplx cmul(cplx a, cplx b) {
    cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    return r;
}

static int64_t smallest_prime_factor(int64_t n) {
    for (int64_t p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

/* w_N^t = exp(-2 pi i t / N) for t in [0, N) */
static cplx *make_table(int64_t n) {
    cplx *tab = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!tab) return NULL;
    for (int64_t t = 0; t < n; ++t) {
        double ang = -TWO_PI * ((double)t / (double)n);
        tab[t].re = cos(ang);
        tab[t].im = sin(ang);
    }
    return tab;
}

/*
 * Length-n DFT of x[0], x[stride], ..., x[(n-1)*stride] into out[0..n).
 * tab holds w_{n*tstride}^t, so w_n^t = tab[t * tstride].
 * tmp is scratch of n elements, disjoint from out.
 */
static void fft_rec(const cplx *x, int64_t stride, int64_t n, cplx *out,
                    cplx *tmp, const cplx *tab, int64_t tstride) {
    if (n == 1) {
        out[0] = x[0];
        return;
    }
    int64_t p = smallest_prime_factor(n);
    if (p > 7) {
        for (int64_t k = 0; k < n; ++k) {
            cplx acc = {0.0, 0.0};
            for (int64_t j = 0; j < n; ++j) {
                cplx t = cmul(x[j * stride], tab[((j * k) % n) * tstride]);
                acc.re += t.re;
                acc.im += t.im;
            }
            out[k] = acc;
        }
        return;
    }
    int64_t m = n / p;
    /* Y_r = DFT_m of the r-th interleaved subsequence, stored at tmp + r*m;
     * each child uses its own slice of `out` as scratch. */
    for (int64_t r = 0; r < p; ++r)
        fft_rec(x + r * stride, stride * p, m, tmp + r * m, out + r * m, tab,
                tstride * p);
    for (int64_t k = 0; k < n; ++k) {
        cplx acc = {0.0, 0.0};
        for (int64_t r = 0; r < p; ++r) {
            cplx t = cmul(tab[((r * k) % n) * tstride], tmp[r * m + (k % m)]);
            acc.re += t.re;
            acc.im += t.im;
        }
        out[k] = acc;
    }
}

/* One signal: x (double pairs) -> y; tab = make_table(n); tmp of n elements. */
static void fft_one(const cplx *x, cplx *y, int64_t n, const cplx *tab,
                    cplx *tmp, cplx *conj_buf, int inverse) {
    if (!inverse) {
        fft_rec(x, 1, n, y, tmp, tab, 1);
        return;
    }
    for (int64_t j = 0; j < n; ++j) {
        conj_buf[j].re = x[j].re;
        conj_buf[j].im = -x[j].im;
    }
    fft_rec(conj_buf, 1, n, y, tmp, tab, 1);
    double s = 1.0 / (double)n;
    for (int64_t k = 0; k < n; ++k) {
        y[k].re = y[k].re * s;
        y[k].im = -y[k].im * s;
    }
}

int oracle_threads(int threads) {
#ifdef _OPENMP
    return threads > 0 ? threads : omp_get_max_threads();
#else
    (void)threads;
    return 1;
#endif
}

int oracle_dft(const double *xd, double *yd, int64_t n, int inverse) {
    if (!xd || !yd || n <= 0) return -1;
    const cplx *x = (const cplx *)xd;
    cplx *y = (cplx *)yd;
    double sign = inverse ? 1.0 : -1.0;
    for (int64_t k = 0; k < n; ++k) {
        double sr = 0.0, si = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            int64_t t = (j * k) % n;
            double ang = sign * TWO_PI * ((double)t / (double)n);
            double c = cos(ang), s = sin(ang);
            sr += x[j].re * c - x[j].im * s;
            si += x[j].re * s + x[j].im * c;
        }
        if (inverse) {
            sr /= (double)n;
            si /= (double)n;
        }
        y[k].re = sr;
        y[k].im = si;
    }
    return 0;
}

int oracle_fft(const double *xd, double *yd, int64_t n, int inverse) {
    if (!xd || !yd || n <= 0) return -1;
    cplx *tab = make_table(n);
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *cb = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    int rc = -1;
    if (tab && tmp && cb) {
        fft_one((const cplx *)xd, (cplx *)yd, n, tab, tmp, cb, inverse);
        rc = 0;
    }
    free(tab);
    free(tmp);
    free(cb);
    return rc;
}

int oracle_fft_batch_f32(const float *x, double *yd, int64_t n, int64_t batch,
                         int inverse, int threads) {
    if (!x || !yd || n <= 0 || batch < 0) return -1;
    cplx *tab = make_table(n);
    if (!tab) return -1;
    int failed = 0;
#pragma omp parallel num_threads(oracle_threads(threads))
    {
        cplx *xin = (cplx *)malloc(sizeof(cplx) * (size_t)n);
        cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)n);
        cplx *cb = (cplx *)malloc(sizeof(cplx) * (size_t)n);
        if (!xin || !tmp || !cb) {
#pragma omp atomic write
            failed = 1;
        } else {
#pragma omp for schedule(static)
            for (int64_t b = 0; b < batch; ++b) {
                const float *src = x + 2 * b * n;
                for (int64_t j = 0; j < n; ++j) {
                    xin[j].re = (double)src[2 * j];
                    xin[j].im = (double)src[2 * j + 1];
                }
                fft_one(xin, (cplx *)yd + b * n, n, tab, tmp, cb, inverse);
            }
        }
        free(xin);
        free(tmp);
        free(cb);
    }
    free(tab);
    return failed ? -1 : 0;
}

int oracle_fft_ragged_f32(const float *x, double *yd, const int64_t *sizes,
                          const int64_t *offsets, int64_t count, int inverse,
                          int threads) {
    if (!x || !yd || !sizes || !offsets || count < 0) return -1;
    for (int64_t i = 0; i < count; ++i)
        if (sizes[i] <= 0 || offsets[i] < 0) return -1;
    int failed = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(oracle_threads(threads))
    for (int64_t i = 0; i < count; ++i) {
        int64_t n = sizes[i];
        cplx *tab = make_table(n);
        cplx *xin = (cplx *)malloc(sizeof(cplx) * (size_t)n);
        cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)n);
        cplx *cb = (cplx *)malloc(sizeof(cplx) * (size_t)n);
        if (!tab || !xin || !tmp || !cb) {
#pragma omp atomic write
            failed = 1;
        } else {
            const float *src = x + 2 * offsets[i];
            for (int64_t j = 0; j < n; ++j) {
                xin[j].re = (double)src[2 * j];
                xin[j].im = (double)src[2 * j + 1];
            }
            fft_one(xin, (cplx *)yd + offsets[i], n, tab, tmp, cb, inverse);
        }
        free(tab);
        free(xin);
        free(tmp);
        free(cb);
    }
    return failed ? -1 : 0;
}

int oracle_fft2d_f32(const float *x, double *yd, int64_t ny, int64_t nx,
                     int64_t batch, int inverse, int threads) {
    if (!x || !yd || ny <= 0 || nx <= 0 || batch < 0) return -1;
    cplx *tab_x = make_table(nx);
    cplx *tab_y = make_table(ny);
    if (!tab_x || !tab_y) {
        free(tab_x);
        free(tab_y);
        return -1;
    }
    int64_t big = nx > ny ? nx : ny;
    int nthr = oracle_threads(threads);
    int failed = 0;
    cplx *y = (cplx *)yd;
    for (int64_t b = 0; b < batch; ++b) {
        const float *img = x + 2 * b * ny * nx;
        cplx *out = y + b * ny * nx;
        /* rows: 1D forward transform of each row (conjugated input if inverse) */
#pragma omp parallel num_threads(nthr)
        {
            cplx *xin = (cplx *)malloc(sizeof(cplx) * (size_t)big);
            cplx *tmp = (cplx *)malloc(sizeof(cplx) * (size_t)big);
            cplx *col = (cplx *)malloc(sizeof(cplx) * (size_t)big);
            cplx *res = (cplx *)malloc(sizeof(cplx) * (size_t)big);
            if (!xin || !tmp || !col || !res) {
#pragma omp atomic write
                failed = 1;
            } else {
#pragma omp for schedule(static)
                for (int64_t r = 0; r < ny; ++r) {
                    const float *src = img + 2 * r * nx;
                    double sg = inverse ? -1.0 : 1.0;
                    for (int64_t j = 0; j < nx; ++j) {
                        xin[j].re = (double)src[2 * j];
                        xin[j].im = sg * (double)src[2 * j + 1];
                    }
                    fft_rec(xin, 1, nx, out + r * nx, tmp, tab_x, 1);
                }
                /* columns: explicit gather, 1D transform, scatter */
#pragma omp for schedule(static)
                for (int64_t c = 0; c < nx; ++c) {
                    for (int64_t r = 0; r < ny; ++r) col[r] = out[r * nx + c];
                    fft_rec(col, 1, ny, res, tmp, tab_y, 1);
                    for (int64_t r = 0; r < ny; ++r) out[r * nx + c] = res[r];
                }
            }
            free(xin);
            free(tmp);
            free(col);
            free(res);
        }
        if (inverse) {
            double s = 1.0 / ((double)nx * (double)ny);
            for (int64_t i = 0; i < nx * ny; ++i) {
                out[i].re = out[i].re * s;
                out[i].im = -out[i].im * s;
            }
        }
    }
    free(tab_x);
    free(tab_y);
    return failed ? -1 : 0;
}

int oracle_rel_l2_f32(const float *y, const double *ref, int64_t n,
                      int64_t batch, double *err, double *ref_norm,
                      int threads) {
    if (!y || !ref || !err || n <= 0 || batch < 0) return -1;
#pragma omp parallel for schedule(static) num_threads(oracle_threads(threads))
    for (int64_t b = 0; b < batch; ++b) {
        const float *yb = y + 2 * b * n;
        const double *rb = ref + 2 * b * n;
        double num = 0.0, den = 0.0;
        for (int64_t j = 0; j < 2 * n; ++j) {
            double d = (double)yb[j] - rb[j];
            num += d * d;
            den += rb[j] * rb[j];
        }
        err[b] = sqrt(num) / (den > 0.0 ? sqrt(den) : 1.0);
        if (ref_norm) ref_norm[b] = sqrt(den);
    }
    return 0;
}

/*
 * Circular convolution, straight from its definition.  Section III-A names
 * convolution and polynomial multiplication among the uses of the DFT; the
 * convolution theorem makes DFT(x conv h) = DFT(x) * DFT(h) bin by bin, which
 * is what a transform-based method computes.  Here no transform is used:
 *     y_b[j] = sum_{m=0}^{n-1} x_b[m] * h_b[(j - m) mod n],   j = 0..n-1,
 * accumulated in double, O(n^2) per signal.  h_b is filter b (h_dist complex
 * elements apart) or the single filter h when h_dist == 0.
 */
int oracle_circular_conv_f32(const float *x, const float *h, double *y, int64_t n,
                             int64_t batch, int64_t h_dist, int threads) {
    if (!x || !h || !y || n <= 0 || batch < 0 || h_dist < 0) return -1;
#pragma omp parallel for schedule(static) num_threads(oracle_threads(threads))
    for (int64_t b = 0; b < batch; ++b) {
        const float *xb = x + 2 * b * n;
        const float *hb = h + 2 * b * h_dist;
        double *yb = y + 2 * b * n;
        for (int64_t j = 0; j < n; ++j) {
            double sr = 0.0, si = 0.0;
            for (int64_t m = 0; m < n; ++m) {
                const int64_t t = ((j - m) % n + n) % n;
                const double xr = xb[2 * m], xi = xb[2 * m + 1];
                const double hr = hb[2 * t], hi = hb[2 * t + 1];
                sr += xr * hr - xi * hi;
                si += xr * hi + xi * hr;
            }
            yb[2 * j] = sr;
            yb[2 * j + 1] = si;
        }
    }
    return 0;
}

/*
 * Image block compression, section III-B of the paper: five steps, the first
 * three and the last data-parallel, the codebook made from the returned data.
 * The paper names the steps but prints no formula; the readings here are the
 * textbook ones (listed with the library's design notes):
 *
 *  (a) chroma + luminance: full-range BT.601 as in JFIF,
 *        Y  =       0.299    R + 0.587    G + 0.114    B
 *        Cb = 128 - 0.168736 R - 0.331264 G + 0.5      B
 *        Cr = 128 + 0.5      R - 0.418688 G - 0.081312 B
 *  (b) chroma scaled to a quarter of the pixels: the mean of each 2x2 square;
 *  (c) directional derivative of the luminance along its gradient, |grad Y|,
 *      from central differences (edge pixels replicated outward), and per 4x4
 *      block its mean (the block's activity), the block's mean luminance and
 *      its 16 deviations from that mean (raster order);
 *  (d) codebook: k-means (Lloyd's iteration) over the deviation vectors of
 *      the blocks whose activity is at least tau, started from the deviation
 *      vectors of the pattern blocks of rank floor(c P / k), c = 0..k-1 (P
 *      pattern blocks in raster order); a codeword left without blocks keeps
 *      its value; ties go to the lower codeword;
 *  (e) encoding: a block of activity below tau keeps its mean only (code 0),
 *      any other block its mean and 1 + the index of the nearest codeword in
 *      squared Euclidean distance.
 * Images are h x w pixels, h and w multiples of 4, RGB interleaved uint8.
 */
int oracle_img_ycc(const uint8_t *rgb, int64_t h, int64_t w, double *y, double *cb,
                   double *cr) {
    if (!rgb || !y || !cb || !cr || h <= 0 || w <= 0 || (h | w) & 1) return -1;
    double *fcb = (double *)malloc(sizeof(double) * h * w);
    double *fcr = (double *)malloc(sizeof(double) * h * w);
    if (!fcb || !fcr) {
        free(fcb);
        free(fcr);
        return -1;
    }
    for (int64_t i = 0; i < h * w; ++i) {
        const double r = rgb[3 * i], g = rgb[3 * i + 1], b = rgb[3 * i + 2];
        y[i] = 0.299 * r + 0.587 * g + 0.114 * b;
        fcb[i] = 128.0 - 0.168736 * r - 0.331264 * g + 0.5 * b;
        fcr[i] = 128.0 + 0.5 * r - 0.418688 * g - 0.081312 * b;
    }
    const int64_t h2 = h / 2, w2 = w / 2;
    for (int64_t r = 0; r < h2; ++r)
        for (int64_t c = 0; c < w2; ++c) {
            const int64_t p = 2 * r * w + 2 * c;
            cb[r * w2 + c] = 0.25 * (fcb[p] + fcb[p + 1] + fcb[p + w] + fcb[p + w + 1]);
            cr[r * w2 + c] = 0.25 * (fcr[p] + fcr[p + 1] + fcr[p + w] + fcr[p + w + 1]);
        }
    free(fcb);
    free(fcr);
    return 0;
}

int oracle_img_blocks(const double *y, int64_t h, int64_t w, double *mean, double *act,
                      double *dev) {
    if (!y || !mean || !act || !dev || h <= 0 || w <= 0 || (h | w) & 3) return -1;
    const int64_t bw = w / 4, bh = h / 4;
    for (int64_t br = 0; br < bh; ++br)
        for (int64_t bc = 0; bc < bw; ++bc) {
            const int64_t b = br * bw + bc;
            double s = 0.0, g = 0.0;
            for (int64_t i = 0; i < 4; ++i)
                for (int64_t j = 0; j < 4; ++j) {
                    const int64_t r = 4 * br + i, c = 4 * bc + j;
                    const int64_t cl = c > 0 ? c - 1 : 0, cr = c < w - 1 ? c + 1 : w - 1;
                    const int64_t ru = r > 0 ? r - 1 : 0, rd = r < h - 1 ? r + 1 : h - 1;
                    const double gx = 0.5 * (y[r * w + cr] - y[r * w + cl]);
                    const double gy = 0.5 * (y[rd * w + c] - y[ru * w + c]);
                    g += sqrt(gx * gx + gy * gy);
                    s += y[r * w + c];
                }
            mean[b] = s / 16.0;
            act[b] = g / 16.0;
            for (int64_t i = 0; i < 4; ++i)
                for (int64_t j = 0; j < 4; ++j)
                    dev[16 * b + 4 * i + j] = y[(4 * br + i) * w + 4 * bc + j] - mean[b];
        }
    return 0;
}

/* index of the nearest codeword (ties to the lower index) and, if margin is
 * not NULL, the gap between the second-nearest and the nearest distance */
static int nearest_codeword(const double *v, const double *cb, int k, double *margin) {
    int best = 0;
    double d1 = INFINITY, d2 = INFINITY;
    for (int c = 0; c < k; ++c) {
        double d = 0.0;
        for (int t = 0; t < 16; ++t) {
            const double e = v[t] - cb[16 * c + t];
            d += e * e;
        }
        if (d < d1) {
            d2 = d1;
            d1 = d;
            best = c;
        } else if (d < d2) {
            d2 = d;
        }
    }
    if (margin) *margin = d2 - d1;
    return best;
}

int oracle_img_kmeans(const double *dev, const double *act, int64_t nb, double tau, int k,
                      int iters, double *codebook, int64_t *npattern) {
    if (!dev || !act || !codebook || nb < 0 || k <= 0 || iters < 0) return -1;
    int64_t P = 0;
    for (int64_t b = 0; b < nb; ++b) P += act[b] >= tau;
    if (npattern) *npattern = P;
    for (int64_t i = 0; i < 16 * (int64_t)k; ++i) codebook[i] = 0.0;
    if (P == 0) return 0;
    int64_t *pat = (int64_t *)malloc(sizeof(int64_t) * P);
    double *sum = (double *)malloc(sizeof(double) * 16 * k);
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * k);
    if (!pat || !sum || !cnt) {
        free(pat);
        free(sum);
        free(cnt);
        return -1;
    }
    for (int64_t b = 0, q = 0; b < nb; ++b)
        if (act[b] >= tau) pat[q++] = b;
    for (int c = 0; c < k; ++c) {
        const int64_t src = pat[(int64_t)c * P / k];
        for (int t = 0; t < 16; ++t) codebook[16 * c + t] = dev[16 * src + t];
    }
    for (int it = 0; it < iters; ++it) {
        for (int64_t i = 0; i < 16 * (int64_t)k; ++i) sum[i] = 0.0;
        for (int c = 0; c < k; ++c) cnt[c] = 0;
        for (int64_t q = 0; q < P; ++q) {
            const double *v = dev + 16 * pat[q];
            const int c = nearest_codeword(v, codebook, k, NULL);
            for (int t = 0; t < 16; ++t) sum[16 * c + t] += v[t];
            cnt[c] += 1;
        }
        for (int c = 0; c < k; ++c)
            if (cnt[c] > 0)
                for (int t = 0; t < 16; ++t) codebook[16 * c + t] = sum[16 * c + t] / (double)cnt[c];
    }
    free(pat);
    free(sum);
    free(cnt);
    return 0;
}

int oracle_img_encode(const double *dev, const double *act, int64_t nb, double tau,
                      const double *codebook, int k, int32_t *code, double *margin) {
    if (!dev || !act || !codebook || !code || nb < 0 || k <= 0) return -1;
    for (int64_t b = 0; b < nb; ++b) {
        if (act[b] < tau) {
            code[b] = 0;
            if (margin) margin[b] = INFINITY;
            continue;
        }
        code[b] = 1 + nearest_codeword(dev + 16 * b, codebook, k, margin ? margin + b : NULL);
    }
    return 0;
}
