/*
 * FP64 CPU oracle for the discrete Fourier transform -- TEST INFRASTRUCTURE.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may link or call this code.  It shares nothing with the GPU
 * library: no headers, tables or helpers.  Its purpose is to be slow, plain
 * and obviously correct.
 *
 * What it computes (the paper, section III-A, names the DFT and the
 * Cooley-Tukey algorithm but prints no formula; the textbook definition is
 * used, with the sign and scaling conventions below):
 *   forward  X[k] = sum_{j=0}^{N-1} x[j] * w_N^{j k},      w_N = exp(-2 pi i / N)
 *   inverse  x[j] = (1/N) sum_{k=0}^{N-1} X[k] * w_N^{-j k}
 *   2D       separable product of the 1D forward transform over both axes;
 *            inverse scaled by 1/(N1*N2).
 *
 * Data: interleaved complex (re, im).  Inputs are float32 pairs (the
 * library's element type), upcast exactly to double; outputs are double pairs.
 * All functions return 0 on success, -1 on a bad argument or allocation
 * failure.  Threads: OpenMP over independent signals; `threads <= 0` means the
 * OpenMP default.
 */
#ifndef DP_ORACLE_H
#define DP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* O(N^2) DFT straight from the definition (angles reduced as integers mod N). */
int oracle_dft(const double *x, double *y, int64_t n, int inverse);

/* Recursive mixed-radix decimation-in-time Cooley-Tukey FFT (double in/out). */
int oracle_fft(const double *x, double *y, int64_t n, int inverse);

/* Batch of `batch` signals of length n, consecutive signals `n` apart.
 * x: float32 pairs, y: double pairs. */
int oracle_fft_batch_f32(const float *x, double *y, int64_t n, int64_t batch,
                         int inverse, int threads);

/* Ragged batch: signal i has length sizes[i] and starts at element offsets[i]
 * in both x and y. */
int oracle_fft_ragged_f32(const float *x, double *y, const int64_t *sizes,
                          const int64_t *offsets, int64_t count, int inverse,
                          int threads);

/* 2D transform of `batch` images of ny rows by nx columns (row-major, x
 * contiguous): 1D transform of every row, then of every column. */
int oracle_fft2d_f32(const float *x, double *y, int64_t ny, int64_t nx,
                     int64_t batch, int inverse, int threads);

/* Error metric of the parity tests: per-signal relative L2 distance
 * err[b] = ||y_b - ref_b||_2 / ||ref_b||_2 (the denominator taken as 1 when
 * ref_b is all zeros) of `batch` signals of n complex elements, y as float32
 * pairs (a transform's output), ref as double pairs (the oracle's).
 * ref_norm (may be NULL) receives ||ref_b||_2. */
int oracle_rel_l2_f32(const float *y, const double *ref, int64_t n,
                      int64_t batch, double *err, double *ref_norm,
                      int threads);

/* Circular convolution of `batch` signals of length n (consecutive signals n
 * apart) with filters h, from the definition:
 *   y_b[j] = sum_{m=0}^{n-1} x_b[m] h_b[(j - m) mod n]
 * h_b starts h_dist complex elements after h_{b-1} (h_dist = 0: one filter
 * for every signal).  x, h: float32 pairs; y: double pairs. */
int oracle_circular_conv_f32(const float *x, const float *h, double *y, int64_t n,
                             int64_t batch, int64_t h_dist, int threads);

/* Image block compression (section III-B), steps a-e; images h x w pixels,
 * RGB interleaved uint8, h and w multiples of 4 (see oracle.c for the
 * formulas).
 *   oracle_img_ycc:    Y (h x w), Cb and Cr averaged over 2x2 squares
 *                      ((h/2) x (w/2) each)
 *   oracle_img_blocks: per 4x4 block (raster order, (h/4) x (w/4) blocks):
 *                      mean luminance, activity (mean |grad Y|), 16
 *                      deviations from the mean
 *   oracle_img_kmeans: k codewords of 16 values from the deviation vectors of
 *                      the blocks with activity >= tau, after `iters` Lloyd
 *                      iterations; *npattern (may be NULL) = pattern blocks
 *   oracle_img_encode: code per block, 0 = mean only, else 1 + nearest
 *                      codeword; margin (may be NULL): second-nearest minus
 *                      nearest squared distance (infinity for code 0) */
int oracle_img_ycc(const uint8_t *rgb, int64_t h, int64_t w, double *y, double *cb,
                   double *cr);
int oracle_img_blocks(const double *y, int64_t h, int64_t w, double *mean, double *act,
                      double *dev);
int oracle_img_kmeans(const double *dev, const double *act, int64_t nb, double tau, int k,
                      int iters, double *codebook, int64_t *npattern);
int oracle_img_encode(const double *dev, const double *act, int64_t nb, double tau,
                      const double *codebook, int k, int32_t *code, double *margin);

/* Number of OpenMP threads a parallel region will use with `threads`. */
int oracle_threads(int threads);

#ifdef __cplusplus
}
#endif
#endif
