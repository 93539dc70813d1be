// Device building blocks of the power-of-two Stockham line kernels: LDS
// layouts and exchanges, the radix passes, pass-twiddle sources, four-step
// twiddles and the tile data accesses.  Included by every translation unit
// that runs these passes (plain and persistent line kernels, real-input
// transforms, fused convolution).
#pragma once
#include <numeric>
#include <type_traits>

#include "fft_common.h"
#include "kernels.h"

namespace dpfft {

constexpr int kPadShift = 4;

// LDS layouts; one padding element every 2^PADSH entries breaks the power-of-
// two strides of the scatter writes across banks.
template <int L, int C, int MAP, int PADSH> struct Lds {
  static constexpr int PITCH = L + (L >> PADSH);
  static constexpr int SIZE = (MAP == ELEM_FAST) ? C * PITCH : (L * C + ((L * C) >> PADSH));
  __device__ __forceinline__ static int idx(int c, int pos) {
    if constexpr (MAP == ELEM_FAST) {
      return c * PITCH + pos + (pos >> PADSH);
    } else {
      int u = pos * C + c;
      return u + (u >> PADSH);
    }
  }
  // idx(c, pos + d) for an offset d that is constant once the caller's loop
  // is unrolled: d is split as d0 + d1 with d1's share of the flat index a
  // multiple of the padding period, so idx(c, pos + d1 + d0) = idx(c, pos + d0)
  // + d1's padded share exactly.  Offsets with the same d0 share one base, and
  // the rest folds into the LDS instruction's immediate offset.
  __device__ __forceinline__ static int idx_off(int c, int pos, int d) {
    constexpr int U = (MAP == ELEM_FAST) ? 1 : C;  // flat-index units per position
    constexpr int PER = 1 << PADSH;
    constexpr int P = PER / std::gcd(U, PER);      // smallest p with p * U % PER == 0
    const int d0 = d % P, d1u = (d - d0) * U;
    return idx(c, pos + d0) + d1u + (d1u >> PADSH);
  }
};

// Exchange through LDS: v[m] goes to slot wpos(m), then v[m] is reloaded from
// slot rpos(m) (complex pairs).  `TAIL` adds the barrier that protects the
// buffer against the next writer.
template <int E, bool TAIL, class WPos, class RPos>
__device__ __forceinline__ void lds_exchange(cf (&v)[E], cf *lds, WPos wpos, RPos rpos) {
#pragma unroll
  for (int m = 0; m < E; ++m) lds[wpos(m)] = v[m];
  __syncthreads();
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = lds[rpos(m)];
  if constexpr (TAIL) __syncthreads();
}

// One Stockham pass on the registers of thread (c, j).  Butterfly q of the
// thread is b = j + T*q; its inputs are v[q + r*QN] and its outputs are left
// in the same registers, then (unless this is the last pass) exchanged so that
// v[m] again holds element j + T*m.
// Pass twiddle sources: TwTable reads the per-pass table from global memory;
// TwLds2 rebuilds w_{Ns R}^{k r} = w_L^{k r L/(Ns R)} from the two-level table
// held in LDS (one product, no global load, so nothing waits behind a
// prefetch).
// tree<..>(): where a lookup costs more than a product, for radix 8, 16 and 32
// only w^r for r = 1, 2, 3 and the multiples of 4 are looked up and the
// others are formed as w^{4s} w^l (one product each).
struct TwTable {
  template <int TWO> static constexpr bool tree() { return false; }
  const cf *__restrict__ tw;
  template <int L, int TWO, int NS, int R>
  __device__ __forceinline__ cf get(int r, int k) const {
    return *(const cf *)((const char *)tw + ((uint32_t)(TWO + (r - 1) * NS + k) << 3));
  }
};
// TwLdsTable: the per-pass table itself, copied to LDS (one read per twiddle)
struct TwLdsTable {
  template <int TWO> static constexpr bool tree() { return false; }
  const cf *t;
  template <int L, int TWO, int NS, int R>
  __device__ __forceinline__ cf get(int r, int k) const {
    return t[TWO + (r - 1) * NS + k];
  }
};
struct TwLds2 {
  template <int TWO> static constexpr bool tree() { return true; }
  const cf *lo;
  const cf *hi;
  template <int L, int TWO, int NS, int R>
  __device__ __forceinline__ cf get(int r, int k) const {
    constexpr int S = tw2_shift(P2<L>::LG);
    const uint32_t e = (uint32_t)(k * r) * (uint32_t)(L / (NS * R));
    return cmul(hi[e >> S], lo[e & ((1u << S) - 1u)]);
  }
};
// TwLdsFirst: the first pass with twiddles (table offset 0) reads its own part
// of the per-pass table from LDS; the later passes use the two-level table.
struct TwLdsFirst {
  template <int TWO> static constexpr bool tree() { return TWO != 0; }
  const cf *first;
  TwLds2 rest;
  template <int L, int TWO, int NS, int R>
  __device__ __forceinline__ cf get(int r, int k) const {
    if constexpr (TWO == 0)
      return first[(r - 1) * NS + k];
    else
      return rest.template get<L, TWO, NS, R>(r, k);
  }
};

template <int L, int EPT, int C, int MAP, int P, class TW>
__device__ __forceinline__ void stockham_pass(cf (&v)[(P2<L, EPT>::E)], cf *lds, const TW &tw, int c,
                                              int j) {
  using G = P2<L, EPT>;
  constexpr int E = G::E, T = G::T, R = G::radix(P), NS = G::ns(P), QN = E / R;
  constexpr bool LAST = (P == G::NP - 1);
  constexpr int TWO = G::twoff(P);
  using LD = Lds<L, C, MAP, kPadShift>;
#pragma unroll
  for (int q = 0; q < QN; ++q) {
    const int b = j + T * q;
    cf x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = v[q + r * QN];
    if constexpr (NS > 1) {
      const int k = b & (NS - 1);
      if constexpr (TW::template tree<TWO>() && R >= 8) {
        cf wl[4], w4[R / 4];
#pragma unroll
        for (int l = 1; l < 4; ++l) wl[l] = tw.template get<L, TWO, NS, R>(l, k);
#pragma unroll
        for (int g = 1; g < R / 4; ++g) w4[g] = tw.template get<L, TWO, NS, R>(4 * g, k);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const int g = r / 4, l = r % 4;
          x[r] = cmul(x[r], g == 0 ? wl[l] : (l == 0 ? w4[g] : cmul(w4[g], wl[l])));
        }
      } else {
#pragma unroll
        for (int r = 1; r < R; ++r) x[r] = cmul(x[r], tw.template get<L, TWO, NS, R>(r, k));
      }
    }
    Dft<R>::run(x);
#pragma unroll
    for (int r = 0; r < R; ++r) v[q + r * QN] = x[r];
  }
  if constexpr (!LAST) {
    auto wpos = [&](int m) {
      const int q = m % QN, r = m / QN;
      if constexpr (T % NS == 0) {
        // k = b mod NS is the same for every butterfly of the thread
        const int k = j & (NS - 1);
        return LD::idx_off(c, (j - k) * R + k, T * q * R + r * NS);
      } else {
        const int b = j + T * q;
        const int k = b & (NS - 1);
        return LD::idx(c, (b - k) * R + k + r * NS);
      }
    };
    auto rpos = [&](int m) { return LD::idx_off(c, j, T * m); };
    lds_exchange<E, true>(v, lds, wpos, rpos);
  }
}

template <int L, int EPT, int C, int MAP, class TW, int... P>
__device__ __forceinline__ void all_passes(cf (&v)[(P2<L, EPT>::E)], cf *lds, const TW &tw, int c,
                                           int j, std::integer_sequence<int, P...>) {
  (stockham_pass<L, EPT, C, MAP, P>(v, lds, tw, c, j), ...);
}

template <int L, int EPT, int C, int MAP>
__device__ __forceinline__ void lane_map(int tid, int &c, int &j) {
  constexpr int T = P2<L, EPT>::T;
  if constexpr (MAP == ELEM_FAST) {
    c = tid / T;
    j = tid % T;
  } else {
    c = tid % C;
    j = tid / C;
  }
}

// w_N^e for 0 <= e < N from the two-level table: hi[e >> s] * lo[e & (2^s-1)]
__device__ __forceinline__ cf tw4_lookup(const LineArgs &a, uint32_t e) {
  const uint32_t lo = e & ((1u << a.tw4_shift) - 1u);
  const uint32_t hi = e >> a.tw4_shift;
  return cmul(a.tw4_hi[hi], a.tw4_lo[lo]);
}

// Four-step twiddles w_N^{n2 k1} for the elements k1 = j + T*m (m = 0..E-1)
// of column n2: with A = w_N^{n2 j} and B = w_N^{n2 T} (two table lookups
// each), w_N^{n2 (j + T m)} = A * B^m.  Writing m = 4s + l, the factor is
// (A B^l) * B^{4s}: the four A B^l come from B, B^2 = B B and B^3 = B^2 B, and
// B^{4s} is the product of the repeated squares B^4, B^8, B^16, ... picked by
// the bits of s.  No twiddle carries more than about seven roundings, and only
// a handful of complex values stay live next to the data.
template <int E>
__device__ __forceinline__ void tw4_apply_ab(cf (&v)[E], cf A, cf B) {
  if constexpr (E % 4 != 0) {
    cf w = A;
#pragma unroll
    for (int m = 0; m < E; ++m) {
      v[m] = cmul(v[m], w);
      if (m + 1 < E) w = cmul(w, B);
    }
  } else {
    constexpr int NG = E / 4;
    constexpr int NB = NG <= 1 ? 1 : (NG <= 2 ? 1 : (NG <= 4 ? 2 : (NG <= 8 ? 3 : 4)));
    const cf B2 = cmul(B, B);
    const cf Al[4] = {A, cmul(A, B), cmul(A, B2), cmul(A, cmul(B2, B))};
    cf Pw[NB];  // Pw[k] = B^(4 * 2^k)
    Pw[0] = cmul(B2, B2);
#pragma unroll
    for (int k = 1; k < NB; ++k) Pw[k] = cmul(Pw[k - 1], Pw[k - 1]);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      cf Q = make_float2(1.0f, 0.0f);
      bool have = false;
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        if ((g >> k) & 1) {
          Q = have ? cmul(Q, Pw[k]) : Pw[k];
          have = true;
        }
      }
#pragma unroll
      for (int l = 0; l < 4; ++l) v[4 * g + l] = cmul(v[4 * g + l], have ? cmul(Al[l], Q) : Al[l]);
    }
  }
}

// Global accesses of a column tile: a base address that is the same for the
// whole workgroup plus a 32-bit byte offset per lane (the plan keeps a column
// tile's span below 4 GiB), so the loads and stores take the scalar-base form
// with a single offset VGPR each.  Row tiles address each line from its own
// 64-bit base: their lines may be any distance apart.
// Tile data in HBM.  NT bit 0 marks the loads, bit 1 the stores nontemporal
// (streamed past the caches' usual allocation): 2-5% faster for the tiles
// whose rows move whole 128-byte segments both ways, slower for narrower
// column tiles and for some persistent kernels, so the registry sets it per
// instance from measurements.
typedef float f2v __attribute__((ext_vector_type(2)));
template <int NT>
__device__ __forceinline__ cf ld_data(const cf *p) {
  if constexpr (NT & 1) {
    const f2v r = __builtin_nontemporal_load((const f2v *)p);
    return make_float2(r.x, r.y);
  } else {
    return *p;
  }
}
template <int NT>
__device__ __forceinline__ void st_data(cf *p, cf v) {
  if constexpr (NT & 2) {
    const f2v r = {v.x, v.y};
    __builtin_nontemporal_store(r, (f2v *)p);
  } else {
    *p = v;
  }
}
template <int NT>
__device__ __forceinline__ cf ldg(const cf *base, uint32_t idx) {
  return ld_data<NT>((const cf *)((const char *)base + (idx << 3)));
}
template <int NT>
__device__ __forceinline__ void stg(cf *base, uint32_t idx, cf v) {
  st_data<NT>((cf *)((char *)base + (idx << 3)), v);
}

// LDS complex elements an instance needs (0 if it never exchanges)
template <int L, int C, int MAP, int OMAP>
constexpr int lds_pairs() {
  constexpr bool need = (P2<L>::NP > 1) || (OMAP != MAP);  // independent of EPT
  constexpr int a = Lds<L, C, MAP, kPadShift>::SIZE, b = Lds<L, C, OMAP, kPadShift>::SIZE;
  return need ? (a > b ? a : b) : 0;
}

// Pass twiddles of a persistent instance: the whole per-pass table when it
// fits in LDS next to the tile (taken for 16-element instances only: a
// 32-element tile of 512 or 1024 points has a single twiddle pass, which the
// first-pass table below covers, and the longer ones do not fit), else the
// two-level table (one more product per twiddle).
template <int L, int C, int MAP, int OMAP, int EPT>
constexpr bool pf_direct_tw() {
  return EPT == 16 && (lds_pairs<L, C, MAP, OMAP>() + P2<L>::twoff(P2<L>::NP)) * 8 <= 160 * 1024;
}
// Otherwise the two-level table, plus the first twiddle pass's own part of
// the per-pass table when that still fits.
template <int L, int EPT>
constexpr int pf_tw2_entries() {
  return (1 << tw2_shift(P2<L>::LG)) +
         ((L >> tw2_shift(P2<L>::LG)) > 0 ? (L >> tw2_shift(P2<L>::LG)) : 1);
}
template <int L, int EPT>
constexpr int pf_first_entries() {
  return P2<L, EPT>::NP > 1 ? P2<L, EPT>::twoff(2) : 0;
}
template <int L, int C, int MAP, int OMAP, int EPT>
constexpr bool pf_first_tw() {
  return !pf_direct_tw<L, C, MAP, OMAP, EPT>() && pf_first_entries<L, EPT>() > 0 &&
         (lds_pairs<L, C, MAP, OMAP>() + pf_tw2_entries<L, EPT>() + pf_first_entries<L, EPT>()) *
                 8 <= 160 * 1024;
}
template <int L, int C, int MAP, int OMAP, int EPT>
constexpr int pf_tw_entries() {
  if constexpr (pf_direct_tw<L, C, MAP, OMAP, EPT>()) {
    return P2<L>::twoff(P2<L>::NP) > 0 ? P2<L>::twoff(P2<L>::NP) : 1;
  } else if constexpr (pf_first_tw<L, C, MAP, OMAP, EPT>()) {
    return pf_tw2_entries<L, EPT>() + pf_first_entries<L, EPT>();
  } else {
    return pf_tw2_entries<L, EPT>();
  }
}

// Pass twiddles of a plain (one tile per workgroup) instance, copied to LDS
// when that costs no resident workgroup: the whole per-pass table, else (tiles
// without a re-tiling exchange) the first twiddle pass's part plus the
// two-level table, else the two-level table alone; otherwise they are read
// from the table in global memory.  Measured: 4-10% faster for the
// one-workgroup-per-CU column tiles and the 256-point four-step tiles; the
// two-level forms made the transposed-row tiles of 4096 9-15% slower (their
// LDS already carries three exchanges), hence the exclusion.  The copy is
// published by the barrier of the first exchange, which precedes the first
// pass with twiddles.
template <int L, int C, int MAP, int OMAP, int EPT, int NTH>
struct PlainTw {
  static constexpr int kLds = 160 * 1024;
  static constexpr int BASE = lds_pairs<L, C, MAP, OMAP>() * 8;
  static constexpr int WG0 = (BASE > 0 ? kLds / BASE : 64) < 2048 / NTH ? (BASE > 0 ? kLds / BASE : 64)
                                                                        : 2048 / NTH;
  static constexpr bool fits(int entries) {
    return BASE + entries * 8 <= kLds && kLds / (BASE + entries * 8) >= WG0;
  }
  static constexpr int DIRECT_N = EPT == 16 ? P2<L>::twoff(P2<L>::NP) : 0;
  static constexpr int N2L = pf_tw2_entries<L, EPT>();
  static constexpr int FIRST_N = pf_first_entries<L, EPT>();
  // 0: global table, 1: per-pass table, 2: first pass's table + two-level, 3: two-level
  static constexpr int MODE = P2<L, EPT>::NP < 2                        ? 0
                              : (DIRECT_N > 0 && fits(DIRECT_N))         ? 1
                              : OMAP != MAP                              ? 0
                              : (FIRST_N > 0 && fits(N2L + FIRST_N))     ? 2
                              : fits(N2L)                                ? 3
                                                                         : 0;
  static constexpr int NTW = MODE == 1 ? DIRECT_N : MODE == 2 ? N2L + FIRST_N : MODE == 3 ? N2L : 0;
  using type = std::conditional_t<
      MODE == 0, TwTable,
      std::conditional_t<MODE == 1, TwLdsTable, std::conditional_t<MODE == 2, TwLdsFirst, TwLds2>>>;
  __device__ static void fill(cf *twl, const LineArgs &a, int tid) {
    if constexpr (MODE == 1) {
      for (int i = tid; i < NTW; i += NTH) twl[i] = a.tw[i];
    } else if constexpr (MODE >= 2) {
      for (int i = tid; i < NTW; i += NTH) twl[i] = i < N2L ? a.tw2[i] : a.tw[i - N2L];
    }
  }
  __device__ static type make(const cf *twl, const LineArgs &a) {
    constexpr int NLO = 1 << tw2_shift(P2<L>::LG);
    if constexpr (MODE == 0) {
      return TwTable{a.tw};
    } else if constexpr (MODE == 1) {
      return TwLdsTable{twl};
    } else if constexpr (MODE == 2) {
      return TwLdsFirst{twl + N2L, TwLds2{twl, twl + NLO}};
    } else {
      return TwLds2{twl, twl + NLO};
    }
  }
};

}  // namespace dpfft
