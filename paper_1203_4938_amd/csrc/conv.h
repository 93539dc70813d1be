// Fused circular convolution kernels: host view of the compiled instances.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace dpfft {

// Extra arguments of a convolution launch: the filter spectra, `h_b` complex
// elements apart per batch item (0 = one spectrum shared by every item), and
// for the four-step row form the column count of the spectrum matrix.
struct ConvArgs {
  const float2 *h;
  int64_t h_b;
  int64_t h_l;  // single pass: elements between the spectra of consecutive lines
};

struct ConvKernel {
  const void *fn = nullptr;
  int L = 0;
  int lines = 0;    // lines per workgroup
  int threads = 0;
  int lds_bytes = 0;
  int ept = 16;
  bool rows4 = false;  // four-step row form (spectrum read as a column tile, conj twiddle on store)
  bool preferred = false;
};

// Compiled instances for a line length L (single pass) or a four-step row
// length L (rows4); returns how many exist and fills up to `max`.
int list_conv_kernels(int L, bool rows4, ConvKernel *out, int max);

}  // namespace dpfft
