// Runtime-radix (mixed 2/3/4/5/7/8/9/16) Stockham transforms: argument blocks
// shared by the host planner and the device code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpfft {

constexpr int kMaxPasses = 12;

// Radix plan of one line length L = prod radix[p].  Thread j of a line owns
// butterflies b = j + T*q of every pass; T >= ceil(L/16) bounds the
// butterflies of a pass to ceil(16/R) per thread.
struct MixedPlan {
  int32_t L;
  int32_t P;                  // passes
  int32_t T;                  // threads per line
  int32_t C;                  // lines per workgroup
  int32_t radix[kMaxPasses];
  int32_t ns[kMaxPasses];     // product of the earlier radices
  int32_t tw2_shift;          // w_L^e = hi[e >> s] * lo[e & (2^s - 1)]
  int32_t pitch;              // LDS elements per line (ELEM_FAST layout)
  uint64_t codes;             // radix[p] in bits 5p..5p+4 (the device reads only this)
  int32_t tw_lds;             // LDS element offset of the pass-twiddle table
};

struct MixedArgs {
  MixedPlan mp;
  int64_t in_b, in_l, in_e;
  int64_t out_b, out_l, out_e;
  int64_t lines;             // lines per batch item
  int64_t tiles_per_batch;   // ceil(lines / C)
  const float2 *tw2;         // 2^s lo entries, then ceil(L / 2^s) hi entries
  const float2 *tw4_lo;      // four-step twiddles of N (two-level)
  const float2 *tw4_hi;
  int32_t tw4_shift;
  float scale;
  uint32_t flags;
};

// Host: radix sequence for a 7-smooth L.  order 0: 16s, then 8/4/2, then 7,
// 5, 9 (pairs of 3), 3; order 1: the odd radices first, then the powers of
// two.  Returns false if L has a prime factor above 7 or needs too many
// passes.
bool mixed_radices(int64_t L, MixedPlan *mp, int order = 0);

// Host: the kernel instance for (map, omap, tw4, swap mode); nullptr if none.
const void *mixed_kernel(int map, int omap, bool tw4, int sw);

// LDS elements of the tile data of a workgroup, and total LDS bytes (tile
// data plus the pass-twiddle table that follows it).
int mixed_tile_elems(const MixedPlan &mp, int map, int omap);
int mixed_lds_bytes(const MixedPlan &mp, int map, int omap);

}  // namespace dpfft
