// Device building blocks of the runtime-radix transforms, shared by the
// batched kernels and the ragged persistent kernel.
#pragma once
#include "fft_common.h"
#include "kernels.h"
#include "mixed.h"

namespace dpfft {

// Address-space-qualified element pointers: the pass functions below are not
// inlined, so their pointer arguments must carry the address space for the
// compiler to emit LDS (ds_*) and global (global_*) instructions rather than
// flat ones.
typedef float v2f __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) v2f lcf;  // LDS
typedef __attribute__((address_space(1))) v2f gcf;  // global memory

__device__ __forceinline__ lcf *as_lds(cf *p) { return (lcf *)p; }
__device__ __forceinline__ gcf *as_glb(cf *p) { return (gcf *)p; }
__device__ __forceinline__ const gcf *as_glb(const cf *p) { return (const gcf *)p; }

template <class P, class I>
__device__ __forceinline__ cf ldc(P *p, I i) {
  const v2f v = p[i];
  return make_float2(v.x, v.y);
}
template <class P, class I>
__device__ __forceinline__ void stc(P *p, I i, cf y) {
  v2f v;
  v.x = y.x;
  v.y = y.y;
  p[i] = v;
}

namespace {

__device__ __forceinline__ int midx_elem(int pitch, int c, int pos) {
  return c * pitch + pos + (pos >> 4);
}
__device__ __forceinline__ int midx_line(int C, int c, int pos) {
  const int u = pos * C + c;
  return u + (u >> 4);
}

__device__ __forceinline__ cf tw2_lookup(const lcf *t, int shift, uint32_t e) {
  const cf lo = ldc(t, e & ((1u << shift) - 1u));
  const cf hi = ldc(t, (1u << shift) + (e >> shift));
  return cmul(hi, lo);
}

// Pass twiddles w_L^{e1 r}, r = 1..R-1, into x[1..R-1] (multiplied in).  For
// R = 8 and 16 only r = 1, 2, 3 and the multiples of 4 are looked up; the
// others are products w^{4s} w^{l}, which halves the table reads.
template <int R>
__device__ __forceinline__ void apply_pass_twiddles(cf *x, const lcf *t, int shift, uint32_t e1) {
  if constexpr (R == 8 || R == 16) {
    cf wl[4], w4[R / 4];
#pragma unroll
    for (int l = 1; l < 4; ++l) wl[l] = tw2_lookup(t, shift, e1 * (uint32_t)l);
#pragma unroll
    for (int s = 1; s < R / 4; ++s) w4[s] = tw2_lookup(t, shift, e1 * (uint32_t)(4 * s));
#pragma unroll
    for (int r = 1; r < R; ++r) {
      const int s = r / 4, l = r % 4;
      const cf w = s == 0 ? wl[l] : (l == 0 ? w4[s] : cmul(w4[s], wl[l]));
      x[r] = cmul(x[r], w);
    }
  } else {
#pragma unroll
    for (int r = 1; r < R; ++r) x[r] = cmul(x[r], tw2_lookup(t, shift, e1 * (uint32_t)r));
  }
}

__device__ __forceinline__ cf tw4_lookup_m(const MixedArgs &a, uint32_t e) {
  const uint32_t lo = e & ((1u << a.tw4_shift) - 1u);
  const uint32_t hi = e >> a.tw4_shift;
  return cmul(a.tw4_hi[hi], a.tw4_lo[lo]);
}

}  // namespace

// One pass.  It is a separate (non-inlined) function per radix so that each
// radix gets its own register allocation; its context travels as plain
// scalars and address-space-qualified pointers.  `tw2` is the two-level
// table of w_L held in LDS.
// The first pass also copies the first `ntw` entries of the global table tw2g
// into tw2 (one per thread): their loads are issued before the tile's data
// loads and their LDS stores after them, so the copy adds no round trip of its
// own (the pass's closing barrier publishes the table to the later passes).
template <int MAP, int OMAP, bool TW4, int SW, int R>
__device__ __noinline__ void mixed_pass(const gcf *__restrict__ src, gcf *__restrict__ dst,
                                        lcf *lds, lcf *tw2, const gcf *__restrict__ tw2g, int ntw,
                                        const gcf *__restrict__ tw4_lo,
                                        const gcf *__restrict__ tw4_hi, int L, int T, int C,
                                        int pitch, int NS, int tw2_shift, int tw4_shift, int c,
                                        int j, bool valid, bool first, bool last, int64_t in_e,
                                        int64_t out_e, int64_t line, float scale) {
  // The shape arguments arrive in VGPRs (this is a call); they are the same in
  // every lane, so move them to SGPRs: the divisions and branches on them then
  // run once per wave on the scalar unit instead of on the VALU.
  L = __builtin_amdgcn_readfirstlane(L);
  T = __builtin_amdgcn_readfirstlane(T);
  C = __builtin_amdgcn_readfirstlane(C);
  pitch = __builtin_amdgcn_readfirstlane(pitch);
  NS = __builtin_amdgcn_readfirstlane(NS);
  tw2_shift = __builtin_amdgcn_readfirstlane(tw2_shift);
  tw4_shift = __builtin_amdgcn_readfirstlane(tw4_shift);
  first = __builtin_amdgcn_readfirstlane((int)first) != 0;
  last = __builtin_amdgcn_readfirstlane((int)last) != 0;
  // element strides and in-line offsets fit 32 bits (checked by the planner:
  // (L - 1) * stride < 2^31), so the per-element index math stays 32-bit
  const uint32_t ie = (uint32_t)__builtin_amdgcn_readfirstlane((int)in_e);
  const uint32_t oe = (uint32_t)__builtin_amdgcn_readfirstlane((int)out_e);
  scale = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(scale)));
  const int M = L / R;
  constexpr int QM = (16 + R - 1) / R;  // butterflies per thread (T >= L/16)
  auto li = [&](int m, int pos) {
    return m == ELEM_FAST ? midx_elem(pitch, c, pos) : midx_line(C, c, pos);
  };
  cf v[QM][R];
  bool act[QM];
  int kq[QM];
  // all loads of the pass first (one branch on the source for the whole
  // pass), so every butterfly's data is in flight before the first one is
  // computed
  // k = b mod NS for b = j + T q: one division per pass, then a step of
  // T mod NS (a scalar) and a conditional subtraction per butterfly
  {
    const int k0 = NS > 1 ? j % NS : 0;
    const int tstep = NS > 1 ? T % NS : 0;
    int k = k0;
#pragma unroll
    for (int q = 0; q < QM; ++q) {
      const int b = j + T * q;
      act[q] = valid && b < M;
      kq[q] = k;
      k += tstep;
      if (k >= NS) k -= NS;
    }
  }
  if (first) {
    ntw = __builtin_amdgcn_readfirstlane(ntw);
    const int tid = (int)threadIdx.x;
    cf tv = make_float2(0.0f, 0.0f);
    if (tid < ntw) tv = ldc(tw2g, tid);
#pragma unroll
    for (int q = 0; q < QM; ++q) {
      if (!act[q]) continue;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = ldc(src, (uint32_t)(j + T * q + r * M) * ie);
    }
    if (tid < ntw) stc(tw2, tid, tv);
  } else {
#pragma unroll
    for (int q = 0; q < QM; ++q) {
      if (!act[q]) continue;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = ldc(lds, li(MAP, j + T * q + r * M));
    }
  }
#pragma unroll
  for (int q = 0; q < QM; ++q) {
    if (!act[q]) continue;
    if ((SW & 1) && first) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = cswap(v[q][r]);
    }
    if (NS > 1) {
      const uint32_t step = (uint32_t)(L / (NS * R));
      apply_pass_twiddles<R>(v[q], tw2, tw2_shift, (uint32_t)kq[q] * step);
    }
    Dft<R>::run(v[q]);
  }
  if (!first) __syncthreads();  // every read of this pass precedes the in-place writes
#pragma unroll
  for (int q = 0; q < QM; ++q) {
    if (!act[q]) continue;
    const int b = j + T * q;
    const int k = kq[q];
    const int base = (b - k) * R + k;
    // Four-step twiddles of the last pass: its outputs are k1 = b + r*NS, so
    // w_N^{line k1} = A * B^r with A = w_N^{line b}, B = w_N^{line NS} (two
    // table lookups per butterfly) and B^r from a product tree of depth <= 4.
    cf tw[R];
    if (TW4 && last) {
      const uint32_t msk = (1u << tw4_shift) - 1u;
      const uint32_t ea = (uint32_t)line * (uint32_t)b, eb = (uint32_t)line * (uint32_t)NS;
      const cf A = cmul(ldc(tw4_hi, ea >> tw4_shift), ldc(tw4_lo, ea & msk));
      const cf B = cmul(ldc(tw4_hi, eb >> tw4_shift), ldc(tw4_lo, eb & msk));
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
      if (last) {
        if (TW4) y = cmul(y, tw[r]);
        if (SW & 2) y = cswap(cscale(y, scale));
        if (OMAP == MAP) {
          stc(dst, (uint32_t)pos * oe, y);
          continue;
        }
        stc(lds, li(OMAP, pos), y);
      } else {
        stc(lds, li(MAP, pos), y);
      }
    }
  }
  if (!last || OMAP != MAP) __syncthreads();
}

// One tile (up to C lines of length L) through every pass.  Thread (c, j)
// works on line c; src/dst are its line's base pointers.  With OMAP != MAP the
// last pass leaves the tile in LDS and thread (c2, j2) stores line c2 through
// dst2, coalesced in the output layout.
struct TileLine {
  const cf *src;
  cf *dst;
  int64_t in_e, out_e, line;
  int c, j;
  bool valid;
  cf *dst2;      // staged store: output base of line c2
  int c2, j2;
  bool valid2;
};

struct LineShape {
  int L, T, C, pitch, P, tw2_shift;
  uint64_t codes;
  const cf *tw2;  // two-level table of w_L in global memory (copied to LDS per tile)
  const cf *tw4_lo, *tw4_hi;
  int tw4_shift;
  float scale;
  int tw_lds;     // LDS element offset of the copied table (after the tile data)
};

// entries of the two-level table of w_L: 2^s lo entries and ceil(L / 2^s) hi
__host__ __device__ inline int tw2_entries(int L, int shift) {
  return (1 << shift) + (L + (1 << shift) - 1) / (1 << shift);
}

template <int MAP, int OMAP, bool TW4, int SW>
__device__ __forceinline__ void mixed_tile(const LineShape &sh, const TileLine &t, cf *lds,
                                           int nthreads) {
  if (sh.P == 0) {  // length 1: the transform is the identity, up to the swaps and the scale
    if (t.valid && t.j == 0) {
      cf y = t.src[0];
      if (SW & 1) y = cswap(y);
      if (SW & 2) y = cswap(cscale(y, sh.scale));
      t.dst[0] = y;
    }
    return;
  }
  // pass twiddles to LDS: the first pass copies one entry per thread (see
  // mixed_pass), entries past the first nthreads are copied here; the barrier
  // that ends the first pass publishes them before the second pass reads any
  lcf *twl = as_lds(lds) + sh.tw_lds;
  const int ntw = tw2_entries(sh.L, sh.tw2_shift);
  for (int i = threadIdx.x + nthreads; i < ntw; i += nthreads) stc(twl, i, sh.tw2[i]);
  const int ntw0 = ntw < nthreads ? ntw : nthreads;
  int ns = 1;
  for (int p = 0; p < sh.P; ++p) {
    const bool first = p == 0, last = p == sh.P - 1;
    const int R = (int)((sh.codes >> (5 * p)) & 31u);
#define PASS(RR)                                                                                 \
  mixed_pass<MAP, OMAP, TW4, SW, RR>(as_glb(t.src), as_glb(t.dst), as_lds(lds), twl,            \
                                     as_glb(sh.tw2), ntw0,                                       \
                                     as_glb(sh.tw4_lo), as_glb(sh.tw4_hi), sh.L, sh.T, sh.C,      \
                                     sh.pitch, ns, sh.tw2_shift, sh.tw4_shift, t.c, t.j, t.valid, \
                                     first, last, t.in_e, t.out_e, t.line, sh.scale)
    switch (R) {
      case 2: PASS(2); break;
      case 3: PASS(3); break;
      case 4: PASS(4); break;
      case 5: PASS(5); break;
      case 7: PASS(7); break;
      case 9: PASS(9); break;
      case 8: PASS(8); break;
      default: PASS(16); break;
    }
#undef PASS
    ns *= R;
  }
  if (OMAP != MAP && t.valid2) {
    for (int i = t.j2; i < sh.L; i += sh.T)
      t.dst2[(int64_t)i * t.out_e] =
          lds[OMAP == ELEM_FAST ? midx_elem(sh.pitch, t.c2, i) : midx_line(sh.C, t.c2, i)];
  }
}

}  // namespace dpfft
