// Real-input (R2C forward, C2R inverse) power-of-two line kernels: host view
// of the compiled instances.
#pragma once
#include <hip/hip_runtime.h>

namespace dpfft {

struct RealKernel {
  const void *fwd = nullptr;  // N reals -> N/2 + 1 bins
  const void *inv = nullptr;  // N/2 + 1 bins -> N reals (scaled by LineArgs::scale)
  int lines = 0;              // lines per workgroup
  int threads = 0;
  int lds_bytes = 0;
};

// Instance for the L-point complex core of an N = 2L real transform, with
// L a power of two in [1, 16384].  Both kernels take LineArgs with unit element
// stride; in_l/out_l count complex elements (L on the real side, L + 1 on
// the spectrum side) and tw4_lo holds w_N^k for k = 0..L-1.
bool real_kernel(int L, RealKernel *out);

// The pairing pass of a real transform whose L-point complex core runs as a
// separate (four-step) transform: thread k < L/2 + 1 of signal b combines
// elements k and L - k.  Forward: Z (L complex per signal, in place in the
// output) -> bins 0..L.  Inverse: bins 0..L -> the L complex values whose
// inverse transform, halved, holds the real samples in pairs.
struct RealPairArgs {
  int64_t in_b, out_b;      // complex elements between the signals of in and out
  int64_t L;                // N / 2
  int64_t batch;
  const float2 *lo, *hi;    // two-level table of w_N: w_N^e = hi[e >> shift] lo[e & mask]
  int32_t shift;
  int32_t pad;
};
const void *real_pair_kernel(bool inverse);

}  // namespace dpfft
