// Matrix-core (MFMA) form of the 256-point line transform: argument block
// shared by the host planner and the device code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpfft {

// Precision forms of the DFT-16 products (values of fft_precision_t).
enum MfmaPrec : int {
  MP_FP16 = 1,        // x, W rounded to FP16
  MP_BF16 = 2,        // x, W rounded to BF16
  MP_FP16_SPLIT = 3,  // x = xh + xl*2^-11, W = Wh + Wl*2^-11 (FP16 pieces), 3 products
  MP_BF16_SPLIT = 4,  // same with BF16 pieces and 2^-8
  MP_BF16_SPLIT3 = 5  // x = xh + xm*2^-8 + xl*2^-16 (BF16), 6 products
};

// Pieces and their exponent step for each form.
constexpr int mfma_pieces(int prec) {
  return prec == MP_BF16_SPLIT3 ? 3 : (prec == MP_FP16_SPLIT || prec == MP_BF16_SPLIT) ? 2 : 1;
}
constexpr int mfma_piece_shift(int prec) { return (prec == MP_FP16 || prec == MP_FP16_SPLIT) ? 11 : 8; }

struct MfmaArgs {
  int64_t in_b, in_l, in_e;
  int64_t out_b, out_l, out_e;
  int64_t lines;
  int64_t tiles_per_batch;
  // per-lane A operands of the DFT-16 matrix: [piece][re/im][lane][8] 16-bit
  // values (FP16 or BF16 bit patterns), built on the host from FP64 values
  const uint16_t *amat;
  const float2 *tw16;   // w_256^{n2 k1}, 256 entries (row k1, column n2)
  const float2 *tw4_lo; // four-step twiddles of N, two-level
  const float2 *tw4_hi;
  int32_t tw4_shift;
  float scale;
  uint32_t flags;
};

// Kernel instance for (precision, map, omap, tw4, swap mode); nullptr if none.
const void *mfma_kernel(int prec, int map, int omap, bool tw4, int sw);

// Threads and lines per workgroup of the MFMA instances, and their LDS bytes.
constexpr int kMfmaThreads = 256;
constexpr int kMfmaLines = 16;
int mfma_lds_bytes(int prec);

}  // namespace dpfft
