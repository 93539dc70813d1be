// Ragged batches: signals of different 7-smooth lengths packed back to back,
// transformed by two persistent launches over a list of work items.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpfft {

// One work item: C lines handled by one workgroup.  Every field the kernel
// needs is in the item itself (line length and radix plan, offsets, tables),
// so a workgroup starts an item after a single descriptor load.
//   RK_SINGLE : C whole signals of length L (one pass through LDS); the
//               element offsets of the signals are sigoff[off .. off + C)
//   RK_COLUMNS: columns [first, first + C) of a four-step signal at element
//               offset `off` (n1-point column FFTs and the twiddle w_N^{n2 k1},
//               into the workspace at ws_off)
//   RK_ROWS   : rows [first, first + C) of that signal (n2-point FFTs, stored
//               transposed into the output); runs in the second launch, after
//               every column item
enum : int32_t { RK_SINGLE = 0, RK_COLUMNS = 1, RK_ROWS = 2 };

struct RaggedItem {
  int32_t kind, C, first, n1, n2;
  int32_t tw_lds;      // LDS element offset of the pass-twiddle table (after the tile data)
  int32_t L, P, T, pitch, tw2_shift;  // line length of this item and its radix plan
  int32_t tw4_shift;
  int32_t ct;          // 1: the line length has compile-time instances (tw2_off then
                       // names its per-pass twiddle table instead of the two-level one)
  int32_t pad;
  uint64_t codes;      // radices, 5 bits each
  int64_t tw2_off;     // two-level pass table of w_L in the table buffer
  int64_t off;         // RK_SINGLE: first index into sigoff; else: the signal's element offset
  int64_t ws_off;      // four-step intermediate of the signal (elements into the workspace)
  int64_t tw4_lo_off, tw4_hi_off;  // four-step twiddle tables of the signal
};

constexpr int kRaggedThreads = 256;      // workgroup size of the ragged kernel
constexpr int kRaggedLdsBytes = 39936;   // per workgroup: four fit in one CU's 160 KB
// the instance for single-pass signals longer than a 256-thread workgroup takes
constexpr int kRaggedBigThreads = 1024;
constexpr int kRaggedBigLdsBytes = 160 * 1024;

// Kernel arguments besides the buffers (in, out, workspace, item list, signal
// offsets, table base), which the kernel takes as separate parameters; the
// pointer fields mirror them for the device helpers.
struct RaggedArgs {
  const RaggedItem *items;  // in execution order: the first launch's items, then the second's
  const int64_t *sigoff;    // element offsets of the signals of RK_SINGLE items
  const float2 *tables;     // base of the plan's table buffer
  float2 *ws;               // four-step intermediates
  int32_t first_item;       // first item of this launch
  int32_t nitems;           // items of this launch
  int32_t direct;           // 1: one item per workgroup; 0: workgroup w runs items w, w + grid, ...
  int32_t pad;
};

// Kernel instances: forward / inverse, 256 threads or (big) 1024 threads.
const void *ragged_kernel(bool inverse, bool big = false);

}  // namespace dpfft
