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
//               FFTs, stored transposed into the output); runs in the second
//               launch, after every column tile (`need` of them) has finished
struct RaggedItem {
  int32_t kind, size, C, sig, first, n1, n2, need, big;
  int32_t tw_lds;  // LDS element offset of the pass-twiddle table (after the tile data)
};

constexpr int kRaggedThreads = 256;      // workgroup size of the ragged kernel
constexpr int kRaggedLdsBytes = 39936;   // per workgroup: four fit in one CU's 160 KB

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
  uint32_t *state;          // [0], [2]: queue tickets of the two launches
  int32_t nitems;           // items in this launch's queue (persistent) or launch (direct)
  int32_t first_item;       // direct mode: first item index of this launch
  int32_t direct;           // 1: item = first_item + blockIdx.x, no queue
  int32_t ticket;           // persistent mode: index of this launch's ticket in `state`
};

// Kernel instances: forward / inverse.
const void *ragged_kernel(bool inverse);
const void *ragged_reset_kernel();

}  // namespace dpfft
