/*
 * dpfft -- batched complex-to-complex FFTs on one AMD MI355X (gfx950).
 *
 * The operation.  Section III-A of Cabellos, "Advanced Programming Platform
 * for efficient use of Data Parallel Hardware" (arXiv 1203.4938) offloads the
 * discrete Fourier transform of a stream of signals, computed by Cooley-Tukey
 * decimation, as a flow of many independent DFTs, one data-parallel work item
 * each (section II-A: one work item per element of the stream; the stream is
 * cut into chunks and re-joined in order).  This library computes the same
 * operation for a batch of signals:
 *
 *   forward (FFT_FORWARD)  X[k] = sum_{j=0}^{N-1} x[j] exp(-2 pi i j k / N)
 *   inverse (FFT_INVERSE)  x[j] = (1/N) sum_{k=0}^{N-1} X[k] exp(+2 pi i j k / N)
 *   rank 2 (images)        the product of the 1D transforms over both axes;
 *                          the inverse is scaled by 1/(N1 N2)
 *
 * for every signal of the batch, outputs in natural order.  The plan-once /
 * execute-many split mirrors the paper's run protocol (section II-D: a
 * program is uploaded once, receives an identifier, and is then run on many
 * input flows).
 *
 * Data.  Interleaved complex64: each element is two float32 (re, im).  All
 * data pointers passed to fft_exec are device pointers (hipMalloc'd, or torch
 * CUDA tensors) owned by the caller, at least 8-byte aligned.
 *
 * Streams.  fft_exec only enqueues work on the given HIP stream (NULL = the
 * default stream) and never synchronizes.  A plan is immutable once created;
 * executions of one plan on different streams may run concurrently if each
 * has its own workspace.
 *
 * Errors.  Every function returns fft_status_t.  Argument validation happens
 * before any device work and has no side effects.  fft_last_error() returns a
 * thread-local message describing the most recent failure on the calling
 * thread.
 */
#ifndef DPFFT_H
#define DPFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dpfft_plan_s *fft_plan_t; /* opaque, owned by the library */

typedef enum {
  FFT_OK = 0,
  FFT_E_INVALID = 1,     /* bad argument (NULL pointer, negative size, ...) */
  FFT_E_UNSUPPORTED = 2, /* valid request this library does not implement */
  FFT_E_NOMEM = 3,       /* device or host allocation failed */
  FFT_E_DEVICE = 4,      /* a HIP call or kernel launch failed */
  FFT_E_INTERNAL = 5     /* an internal consistency check failed */
} fft_status_t;

/* Direction: the sign of the exponent. */
#define FFT_FORWARD (-1)
#define FFT_INVERSE (+1)

/* Arithmetic of the transform. FP32: float32 butterflies everywhere.  The
 * *_MFMA forms run the DFT-16 stages as FP16/BF16 matrix products on the
 * matrix cores with FP32 accumulation; *_SPLIT forms split inputs and
 * twiddles into hi + lo pieces to recover FP32-level accuracy.  Lengths of
 * the matrix-core forms (rank 1, not ragged, complex): N = 256 (one pass of
 * 16 x 16), N = 65536 (both four-step passes of 256 points on the matrix
 * cores), and N = 256 N2 with N2 a power of two from 64 to 4096 (the
 * 256-point column pass on the matrix cores, the N2-point row pass in FP32);
 * other lengths return FFT_E_UNSUPPORTED. */
typedef enum {
  FFT_FP32 = 0,
  FFT_FP16_MFMA = 1,
  FFT_BF16_MFMA = 2,
  FFT_FP16_SPLIT = 3,
  FFT_BF16_SPLIT = 4,
  FFT_BF16_SPLIT3 = 5
} fft_precision_t;

/* Plan flags. */
#define FFT_F_INPLACE 1u     /* in == out is allowed */
#define FFT_F_NO_AUTOTUNE 2u /* ignore the autotune cache, use the heuristic plan */
#define FFT_F_GRAPH 4u       /* ragged plans: replay the launches as a HIP graph */
#define FFT_F_PER_SIZE 8u    /* ragged plans: one launch per distinct length instead of
                                the two persistent launches (the comparison baseline) */
#define FFT_F_REAL 16u       /* real samples (see "Real-input transforms" below) */
#define FFT_F_CONV 32u       /* the plan also runs fft_conv_exec (circular convolution) */

typedef struct {
  int32_t rank;     /* 1: batched 1D signals; 2: batched images */
  int64_t n[2];     /* rank 1: n[0] = N; rank 2: {ny, nx}, nx contiguous */
  int64_t batch;    /* number of transforms (ragged: number of signals) */
  int64_t dist;     /* elements between consecutive transforms; 0 = dense
                       (N for rank 1, ny*nx for rank 2); same for in and out */
  const int64_t *ragged_sizes;   /* rank 1 only, optional: per-signal N
                                    (then n[0] is ignored); host pointer,
                                    copied by fft_plan */
  const int64_t *ragged_offsets; /* optional with ragged_sizes: element offset
                                    of each signal; NULL = packed prefix sum */
  int32_t precision; /* fft_precision_t */
  uint32_t flags;    /* FFT_F_* */
} fft_desc_t;

/*
 * Real-input transforms (FFT_F_REAL).  The paper's image workload (section
 * III-B) transforms real greyscale pictures; a real signal's spectrum is
 * Hermitian, X[N-k] = conj X[k], so bins 0..N/2 determine it.
 *   forward: in  = N float32 samples per signal (rank 2: ny rows of nx),
 *            out = N/2 + 1 complex64 bins per signal (rank 2: ny rows of
 *                  nx/2 + 1 bins), X[k] as defined above, k = 0..N/2;
 *   inverse: in  = N/2 + 1 bins per signal (rank 2: ny x (nx/2 + 1)) of a
 *                  Hermitian spectrum, out = N float32 samples, scaled by 1/N
 *                  (rank 2: 1/(ny nx)).  Bins 0 and N/2 of a Hermitian
 *                  spectrum are real, and their imaginary parts are ignored
 *                  (rank 2: those of columns 0 and nx/2 once the column
 *                  transforms have been inverted, which are real for a
 *                  Hermitian 2D spectrum).
 * Signals (images) are packed back to back on both sides: dist must be 0.
 * Supported: FFT_FP32, rank 1 with N an even number in [2, 2^24] whose
 * prime factors are at most 7 (powers of two up to 32768: one launch per
 * direction; otherwise the N/2-point complex transform of the samples read
 * as N/2 complex pairs runs on launches of its own, one single pass or a
 * four-step pair, and one more launch pairs bin k with N/2 - k, with a
 * workspace of batch * N/2 complex64), rank 2 with nx an even number in
 * [2, 32768] and ny in [1, 16384], both with prime factors <= 7 (powers of
 * two: two launches per direction, the inverse with a workspace of batch *
 * ny * (nx/2 + 1) complex64; other sides: three, the rows of nx/2 pairs on
 * the runtime-radix kernels, the pairing, the columns, with that workspace
 * in both directions).  in != out.  Both buffers are device pointers owned
 * by the caller, 8-byte aligned.
 */

/*
 * Create a plan.  Validates *desc, factors each length into radices
 * {16, 8, 4, 2, 3, 5, 7}, chooses the kernels (single pass through LDS, or the
 * two-pass four-step decomposition for lengths that do not fit on chip, or the
 * MFMA DFT-16 form, or the ragged persistent kernel), builds the twiddle
 * tables in FP64 on the host, rounds them to the kernel precision and uploads
 * them (hipMalloc + copy; this call may synchronize the device).
 *   out        receives the handle (set to NULL on failure)
 *   desc       host pointer, read only during the call
 *   hip_stream stream used for the table uploads (NULL = default)
 * Supported: 1 <= N <= 2^24 with all prime factors <= 7 (FFT_E_UNSUPPORTED
 * otherwise); batch >= 0; rank 2 with each side <= 16384 and all prime
 * factors <= 7 (powers of two on the line kernels, other sides on the
 * runtime-radix kernels).
 */
fft_status_t fft_plan(fft_plan_t *out, const fft_desc_t *desc, void *hip_stream);

/*
 * Execute a plan: transform `in` into `out` (device pointers, interleaved
 * complex64, laid out as described by the plan's desc).  direction is
 * FFT_FORWARD or FFT_INVERSE (the inverse includes the 1/N scale).
 *   workspace  device buffer of at least fft_workspace_bytes(plan) bytes,
 *              owned by the caller; may be NULL when that size is 0
 *   hip_stream stream to enqueue on (NULL = default stream)
 * in == out requires FFT_F_INPLACE at plan time; partial overlap is undefined.
 * `in` is not modified unless in == out.  Asynchronous: returns after the
 * launches are enqueued.
 */
fft_status_t fft_exec(fft_plan_t plan, const void *in, void *out, int direction,
                      void *workspace, void *hip_stream);

/* Number of kernel launches one fft_exec of this plan enqueues (0 if plan is
 * NULL). */
int fft_plan_num_steps(fft_plan_t plan);

/* Enqueue only launches [first, first + count) of fft_exec (for timing one
 * kernel at a time and for tests).  Same arguments, ownership and errors as
 * fft_exec; FFT_E_INVALID if the range is outside [0, fft_plan_num_steps). */
fft_status_t fft_exec_steps(fft_plan_t plan, const void *in, void *out, int direction,
                            void *workspace, void *hip_stream, int first, int count);

/* Plan without touching the device: validation, factorization, kernel choice
 * and the bounds checks of fft_plan, then the plan description (as
 * fft_plan_describe) in buf.  Same status codes as fft_plan except that no
 * device error can occur. */
fft_status_t fft_plan_dry(const fft_desc_t *desc, char *buf, size_t len);

/* Autotune: build every compiled kernel variant the planner could use for
 * *desc (tile widths, persistent form, the four-step split and chunking of
 * power-of-two lengths, radix order of non-power-of-two lengths), time `reps`
 * forward executions of each on `hip_stream` with HIP
 * events on scratch buffers it allocates and frees, and record the fastest
 * for (architecture, shape, batch rounded down to a power of two, precision).
 * Later fft_plan calls for that key use it unless FFT_F_NO_AUTOTUNE is set.
 * If the environment variable DPFFT_TUNE_CACHE names a file, the record is
 * also written there as JSON and read back by later processes (a missing or
 * unreadable file is treated as empty).  A per-candidate report (one line per
 * candidate, then the choice) goes to `report` (may be NULL).  Synchronizes
 * the stream.  MFMA precision forms have nothing to tune (FFT_OK, report says
 * so).  Ragged descriptors are tuned per distinct length: radix order, single
 * pass in a 256- or 1024-thread workgroup or four-step, and the four-step
 * split, each timed on a batch of signals of that length alone (at least
 * 2^21 points); the fastest is recorded for (architecture, length) and used
 * by every later ragged plan containing that length. */
fft_status_t fft_autotune(const fft_desc_t *desc, void *hip_stream, int reps, char *report,
                          size_t len);

/*
 * Fused circular convolution (plans made with FFT_F_CONV).  Section III-A of
 * the paper names convolution and polynomial multiplication among the uses of
 * the DFT, and section IV names the data movement between chained instances
 * as the platform's inefficiency; this call chains forward transform,
 * product and inverse transform on chip.  For every signal b of the batch:
 *
 *   out_b[j] = sum_{m=0}^{N-1} in_b[m] h_b[(j - m) mod N]
 *            = IDFT( DFT(in_b) * H_b )[j]            (j = 0..N-1)
 *
 * where H_b = DFT(h_b) is the filter's spectrum in natural order, exactly as
 * fft_exec(plan, h, H, FFT_FORWARD, ...) stores it.  Polynomial products are
 * the special case of zero-padded coefficient vectors (N >= deg a + deg b + 1).
 *   in, out      device pointers, interleaved complex64, the plan's layout
 *                (dist); in == out requires FFT_F_INPLACE
 *   filter       device pointer to the spectra H_b, complex64; spectrum b
 *                starts filter_dist elements after spectrum b-1, and
 *                filter_dist = 0 means one spectrum shared by every signal;
 *                the caller guarantees (batch-1)*filter_dist + N elements
 *   workspace    at least fft_workspace_bytes(plan) bytes (N > 16384 only)
 * Supported: FFT_FP32, rank 1, N a power of two in [1, 2^24], not ragged,
 * not real.  N <= 16384 runs as one launch (one HBM read of in and H, one
 * write of out); longer N as three (the four-step column pass, a fused row
 * launch, the inverse column pass).  Errors: FFT_E_INVALID for a plan made
 * without FFT_F_CONV, NULL or misaligned pointers, a negative filter_dist or
 * one below N (checked before any launch); FFT_E_DEVICE for a failed launch.
 * Asynchronous on hip_stream, like fft_exec.
 */
fft_status_t fft_conv_exec(fft_plan_t plan, const void *in, const void *filter,
                           int64_t filter_dist, void *out, void *workspace, void *hip_stream);

/*
 * fft_exec for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same launches, with the plan's workspace taken from a device array the
 * library holds (64 MiB per GPU, kept until the process ends) instead of a
 * caller buffer.  Graph plans (FFT_F_GRAPH) launch their kernels directly
 * rather than instantiating a graph.  Calls no allocating routine.
 *   in, out, direction, hip_stream   as for fft_exec
 * Errors: as fft_exec, plus FFT_E_UNSUPPORTED when fft_workspace_bytes(plan)
 * exceeds 64 MiB (checked before any launch) and FFT_E_DEVICE when the
 * array's address cannot be looked up on the current device.  The array is
 * shared by every call on a GPU and keeps the last call's contents (no kernel
 * reads workspace it has not written in the same call); calls whose
 * executions overlap on one GPU race on it.
 */
fft_status_t fft_exec_noalloc(fft_plan_t plan, const void *in, void *out, int direction,
                              void *hip_stream);

/*
 * Image block compression, the paper's second workload (section III-B): a
 * lossy coder in five steps, named there without formulas (the readings are
 * the textbook ones):
 *   (a) luminance and chroma, full-range BT.601 as in JFIF:
 *         Y = 0.299 R + 0.587 G + 0.114 B,
 *         Cb = 128 - 0.168736 R - 0.331264 G + 0.5 B,
 *         Cr = 128 + 0.5 R - 0.418688 G - 0.081312 B;
 *   (b) chroma at a quarter of the pixels: the mean of each 2x2 square;
 *   (c) the directional derivative of the luminance along its gradient,
 *       |grad Y| by central differences with the edge pixels replicated, and
 *       per 4x4 block its mean (the block's activity), the block's mean
 *       luminance and its 16 deviations from that mean (raster order);
 *   (d) a codebook of k deviation vectors: Lloyd's k-means over the blocks of
 *       activity >= tau ("pattern blocks"), started from the pattern blocks of
 *       rank floor(c P / k), c = 0..k-1 (P pattern blocks in raster order), a
 *       codeword without blocks keeping its value, ties to the lower index;
 *   (e) codes: 0 for a block of activity below tau (its mean alone), else 1 +
 *       the index of the nearest codeword in squared Euclidean distance.
 * Every step runs on the GPU, independently per image of the batch.
 */
typedef struct {
  int32_t height, width; /* pixels, positive multiples of 4, at most 2^30 per image */
  int32_t batch;         /* images, 0..65535 */
  int32_t k;             /* codewords, 1..256 */
  int32_t iters;         /* Lloyd iterations, 0..10000 (0: the seeds) */
  float tau;             /* activity threshold of pattern blocks */
  uint32_t flags;        /* IMG_F_* (0: launch the kernels one by one) */
} img_desc_t;

/* img_compress: replay the launch sequence as a HIP graph.  A graph is
 * instantiated on the first call for a given (descriptor, buffers, stream,
 * device) and kept for later calls with the same arguments (the 8 most
 * recent are kept); it saves the gaps between the 4 + 2 iters + 1 dependent
 * launches, so it pays off when the same call repeats. */
#define IMG_F_GRAPH 1u

/* Outputs of img_compress: caller-owned device buffers, per image back to back.
 *   y        batch x height x width          float32, 16-byte aligned
 *   cb, cr   batch x height/2 x width/2      float32, 8-byte aligned
 *   mean,act batch x (height/4) x (width/4)  float32 (blocks in raster order)
 *   dev      batch x blocks x 16             float32, 16-byte aligned
 *   codebook batch x k x 16                  float32
 *   code     batch x blocks                  int32
 * (buffers without a stated alignment: 4-byte aligned) */
typedef struct {
  float *y, *cb, *cr, *mean, *act, *dev, *codebook;
  int32_t *code;
} img_out_t;

/* Device workspace img_compress needs for *desc (0 if desc is invalid). */
size_t img_workspace_bytes(const img_desc_t *desc);

/* Steps (a)-(e) for `batch` RGB images (device pointer, interleaved uint8,
 * batch x height x width x 3, 4-byte aligned: each thread reads its four
 * pixels as three 32-bit words).  workspace: img_workspace_bytes(desc) bytes,
 * 256-byte aligned, caller-owned.  Asynchronous on hip_stream.  Errors:
 * FFT_E_INVALID for a bad descriptor, NULL or misaligned buffers (checked
 * before any launch); FFT_E_UNSUPPORTED for images above 2^30 pixels;
 * FFT_E_DEVICE for a failed launch.  Every sum is taken in an order that does
 * not depend on scheduling, so the same inputs give the same output bits on
 * every call (with or without IMG_F_GRAPH). */
fft_status_t img_compress(const img_desc_t *desc, const uint8_t *rgb, const img_out_t *out,
                          void *workspace, void *hip_stream);

/* Step (e) alone: codes of the blocks given their deviation vectors (dev,
 * 16-byte aligned), activities and a codebook (layouts as in img_out_t). */
fft_status_t img_encode(const img_desc_t *desc, const float *dev, const float *act,
                        const float *codebook, int32_t *code, void *hip_stream);

/* Release a plan and its device tables.  fft_destroy(NULL) returns FFT_OK.
 * The caller must ensure no execution of the plan is still pending. */
fft_status_t fft_destroy(fft_plan_t plan);

/* Device workspace bytes fft_exec needs for this plan (0 = none). */
size_t fft_workspace_bytes(fft_plan_t plan);

/* Static string naming a status code. */
const char *fft_status_str(fft_status_t s);

/* Thread-local description of the last failure on this thread ("" if none). */
const char *fft_last_error(void);

/* Human-readable description of the plan (variant, radices, kernels, grid,
 * LDS bytes, HBM passes) written into buf (NUL-terminated, truncated to len).
 * Returns the number of characters the full description needs. */
size_t fft_plan_describe(fft_plan_t plan, char *buf, size_t len);

#ifdef __cplusplus
}
#endif
#endif /* DPFFT_H */
