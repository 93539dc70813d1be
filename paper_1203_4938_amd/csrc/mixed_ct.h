// Compile-time twins of the runtime-radix passes for the line lengths that
// dominate ragged batches.
//
// A ragged signal longer than one workgroup's LDS is a four-step transform
// whose line lengths lie near the square root of its length: for signals of
// 2^14 to 2^16 points, between about 125 and 256.  Those lines carry most of a
// log-uniform ragged batch's work (four in five of its point-passes).  For
// them the ragged kernel runs these instances, in which the radix sequence,
// the butterflies per thread, the twiddle table offsets and every index
// constant are known to the compiler, instead of the runtime-radix passes.
// The decomposition and the data layout are the runtime passes' own (same
// radix order, same threads per line, same LDS layout), so an item can take
// either path.  Pass twiddles come from a per-pass table held in LDS (entry
// (r-1) Ns + k of pass p is w_{Ns R}^{k r}), one LDS read each.
#pragma once
#include <utility>

#include "mixed_ct_plan.h"
#include "mixed_device.h"

namespace dpfft {

template <int L, int MAP>
__device__ __forceinline__ int ct_idx(int C, int c, int pos) {
  if constexpr (MAP == ELEM_FAST) {
    return c * CtPlan<L>::PITCH + pos + (pos >> 4);
  } else {
    const int u = pos * C + c;
    return u + (u >> 4);
  }
}

// Everything a compile-time tile needs at run time.  Pointers carry their
// address space (the tile function is not inlined), so LDS and global
// accesses compile to ds_* and global_* instructions.
struct CtArgs {
  const gcf *src;
  gcf *dst;
  gcf *dst2;
  const gcf *tw4_lo;
  const gcf *tw4_hi;
  int tw4_shift;
  int C, c, j, c2, j2;
  bool valid, valid2;
  uint32_t in_e, out_e, line;
  float scale;
};

// The first pass also stores this thread's entry `tv` of the pass-twiddle
// table (loaded by the caller before the tile's data loads) at twl[tid]
// once its data loads are issued; its closing barrier publishes the table.
template <int L, int PP, int MAP, int OMAP, bool TW4, int SW>
__device__ __forceinline__ void ct_pass(const CtArgs &a, lcf *lds, lcf *twl, cf tv) {
  using PL = CtPlan<L>;
  constexpr int R = PL::R(PP), NS = PL::NS(PP), M = L / R, T = PL::T;
  constexpr int QM = (M + T - 1) / T;
  constexpr bool FIRST = PP == 0, LAST = PP == PL::P - 1;
  constexpr int TWO = PL::TWO(PP);
  cf v[QM][R];
  bool act[QM];
#pragma unroll
  for (int q = 0; q < QM; ++q) {
    const int b = a.j + T * q;
    act[q] = a.valid && ((q + 1) * T <= M || b < M);
    if (!act[q]) continue;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if constexpr (FIRST)
        v[q][r] = ldc(a.src, (uint32_t)(b + r * M) * a.in_e);
      else
        v[q][r] = ldc(lds, ct_idx<L, MAP>(a.C, a.c, b + r * M));
    }
  }
  if constexpr (FIRST) {
    if ((int)threadIdx.x < PL::NTW) stc(twl, (int)threadIdx.x, tv);
  }
#pragma unroll
  for (int q = 0; q < QM; ++q) {
    if (!act[q]) continue;
    if constexpr ((SW & 1) && FIRST) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = cswap(v[q][r]);
    }
    if constexpr (NS > 1) {
      const int k = (a.j + T * q) % NS;
#pragma unroll
      for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], ldc(twl, TWO + (r - 1) * NS + k));
    }
    Dft<R>::run(v[q]);
  }
  if constexpr (!FIRST) __syncthreads();  // every read of this pass precedes the in-place writes
#pragma unroll
  for (int q = 0; q < QM; ++q) {
    if (!act[q]) continue;
    const int b = a.j + T * q;
    const int k = NS > 1 ? b % NS : 0;
    const int base = (b - k) * R + k;
    cf tw[R];
    if constexpr (TW4 && LAST) {
      // outputs k1 = b + r NS: w_N^{line k1} = A B^r, A = w_N^{line b}, B = w_N^{line NS}
      const uint32_t msk = (1u << a.tw4_shift) - 1u;
      const uint32_t ea = a.line * (uint32_t)b, eb = a.line * (uint32_t)NS;
      const cf A = cmul(ldc(a.tw4_hi, ea >> a.tw4_shift), ldc(a.tw4_lo, ea & msk));
      const cf B = cmul(ldc(a.tw4_hi, eb >> a.tw4_shift), ldc(a.tw4_lo, eb & msk));
      // B^r from repeated squares (depth <= 4), as the runtime passes form it
      cf Bp[R];
      Bp[0] = make_float2(1.0f, 0.0f);
      if constexpr (R > 1) Bp[1] = B;
#pragma unroll
      for (int r = 2; r < R; ++r) {
        int p2 = 1;
        while (2 * p2 <= r) p2 *= 2;
        Bp[r] = (r == p2) ? cmul(Bp[p2 / 2], Bp[p2 / 2]) : cmul(Bp[p2], Bp[r - p2]);
      }
      tw[0] = A;
#pragma unroll
      for (int r = 1; r < R; ++r) tw[r] = cmul(A, Bp[r]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int pos = base + r * NS;
      cf y = v[q][r];
      if constexpr (LAST) {
        if constexpr (TW4) y = cmul(y, tw[r]);
        if constexpr (SW & 2) y = cswap(cscale(y, a.scale));
        if constexpr (OMAP == MAP)
          stc(a.dst, (uint32_t)pos * a.out_e, y);
        else
          stc(lds, ct_idx<L, OMAP>(a.C, a.c, pos), y);
      } else {
        stc(lds, ct_idx<L, MAP>(a.C, a.c, pos), y);
      }
    }
  }
  if constexpr (!LAST || OMAP != MAP) __syncthreads();
}

template <int L, int MAP, int OMAP, bool TW4, int SW, int... PP>
__device__ __forceinline__ void ct_passes(const CtArgs &a, lcf *lds, lcf *twl, cf tv,
                                          std::integer_sequence<int, PP...>) {
  (ct_pass<L, PP, MAP, OMAP, TW4, SW>(a, lds, twl, tv), ...);
}

// One tile through every pass.  `tw` is the per-pass table in global memory,
// copied to LDS at twl (after the tile data) while the first pass (which has
// no twiddles) loads the tile; the barrier that ends that pass publishes it.
// The arguments travel as scalars (a structure passed to a function that is
// not inlined would live in scratch memory); the uniform ones are moved to
// scalar registers.
template <int L, int MAP, int OMAP, bool TW4, int SW>
__device__ __noinline__ void ct_tile(const gcf *src, gcf *dst, gcf *dst2, const gcf *tw4_lo,
                                    const gcf *tw4_hi, int tw4_shift, int C, int c, int j, int c2,
                                    int j2, bool valid, bool valid2, uint32_t in_e,
                                    uint32_t out_e, uint32_t line, float scale, lcf *lds,
                                    lcf *twl, const gcf *tw, int nthreads) {
  using PL = CtPlan<L>;
  CtArgs a;
  a.src = src;
  a.dst = dst;
  a.dst2 = dst2;
  a.tw4_lo = tw4_lo;
  a.tw4_hi = tw4_hi;
  a.tw4_shift = __builtin_amdgcn_readfirstlane(tw4_shift);
  a.C = __builtin_amdgcn_readfirstlane(C);
  a.c = c;
  a.j = j;
  a.c2 = c2;
  a.j2 = j2;
  a.valid = valid;
  a.valid2 = valid2;
  a.in_e = (uint32_t)__builtin_amdgcn_readfirstlane((int)in_e);
  a.out_e = (uint32_t)__builtin_amdgcn_readfirstlane((int)out_e);
  a.line = line;
  a.scale = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(scale)));
  nthreads = __builtin_amdgcn_readfirstlane(nthreads);
  // pass twiddles: entry tid is loaded now and stored by the first pass after
  // the data loads are issued; entries past the first nthreads are copied here
  for (int i = threadIdx.x + nthreads; i < PL::NTW; i += nthreads) stc(twl, i, ldc(tw, i));
  cf tv = make_float2(0.0f, 0.0f);
  if ((int)threadIdx.x < PL::NTW && (int)threadIdx.x < nthreads) tv = ldc(tw, threadIdx.x);
  ct_passes<L, MAP, OMAP, TW4, SW>(a, lds, twl, tv, std::make_integer_sequence<int, PL::P>{});
  if constexpr (OMAP != MAP) {
    if (a.valid2) {
#pragma unroll 4
      for (int i = a.j2; i < L; i += PL::T)
        stc(a.dst2, (uint32_t)i * a.out_e, ldc(lds, ct_idx<L, OMAP>(a.C, a.c2, i)));
    }
  }
}

}  // namespace dpfft
