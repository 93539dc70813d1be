// Ragged batches: signals of different 7-smooth lengths packed back to back,
// transformed by one persistent launch that pulls work items from a queue.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpfft {

// A line length used by the items (a signal length, or a four-step factor).
struct RaggedSize {
  int32_t L, P, T, pitch, tw2_shift, pad;
  uint64_t codes;   // radices, 5 bits each
  int64_t tw2_off;  // two-level pass table of w_L in the plan's table buffer
};

enum : int32_t { RK_SINGLE = 0, RK_COLUMNS = 1, RK_ROWS = 2 };

// One work item: C lines handled by one workgroup.
//   RK_SINGLE : C whole signals of length sizes[size].L (one pass through LDS);
//               signal ids are siglist[sig .. sig + C)
//   RK_COLUMNS: columns [first, first + C) of four-step signal `sig`
//               (n1-point column FFTs and the twiddle w_N^{n2 k1}, into the
//               workspace)
//   RK_ROWS   : rows [first, first + C) of four-step signal `sig` (n2-point
//               FFTs, stored transposed into the output); waits until all
//               `need` column items of the signal have finished
struct RaggedItem {
  int32_t kind, size, C, sig, first, n1, n2, need, big, pad;
};

// Per four-step signal: workspace offset (elements) and its twiddle tables.
struct RaggedBig {
  int64_t ws_off;
  int64_t tw4_lo_off, tw4_hi_off;  // in the plan's table buffer
  int32_t tw4_shift, pad;
};

struct RaggedArgs {
  const RaggedSize *sizes;
  const RaggedItem *items;
  const int32_t *order;     // queue order of the items (persistent mode)
  const int32_t *siglist;
  const int64_t *offsets;   // element offset of every signal (input and output)
  const RaggedBig *bigs;
  const float2 *tables;     // base of the plan's table buffer
  float2 *ws;               // four-step intermediates
  uint32_t *state;          // [0] queue ticket, [1] error flag, [2 + b] done count of big b
  int32_t nitems;           // items in the queue (persistent) or in this launch (direct)
  int32_t first_item;       // direct mode: first item index of this launch
  int32_t direct;           // 1: item = first_item + blockIdx.x, no queue, no waits
  int32_t spin_limit;       // bound on the dependency wait (then the error flag is set)
};

// Kernel instances: forward / inverse.
const void *ragged_kernel(bool inverse);
const void *ragged_reset_kernel();

}  // namespace dpfft
