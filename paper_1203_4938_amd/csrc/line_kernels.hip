// Power-of-two Stockham line kernels for gfx950.
//
// A workgroup transforms C "lines" (signals, matrix rows or matrix columns) of
// compile-time length L = 2^k.  Each line is owned by T = L/E threads that
// hold E = 16 (or 32) elements each in registers (thread j owns elements
// j + T*m).  Passes are radix 16 (32) with one smaller remainder pass last.
//
// Pass with radix R over butterflies b = 0..L/R-1 and span Ns (the product of
// the earlier radices), the self-sorting Stockham form of Cooley-Tukey
// (Stockham autosort; see e.g. Govindaraju et al., SC 2008):
//   inputs   x[b + r*L/R], r = 0..R-1
//   twiddle  x_r *= w_{Ns R}^{(b mod Ns) r}
//   DFT-R in registers
//   outputs  y[(b div Ns)*Ns*R + (b mod Ns) + r*Ns]
// so no bit reversal is ever needed.  Outputs of a pass go through LDS to the
// threads that need them next; the last pass's outputs land exactly in the
// registers holding j + T*m, which is also the coalesced order of the load,
// so the first load and the last store go straight between HBM and VGPRs.
//
// Twiddles of pass p >= 1 come from a per-length table built on the host in
// FP64: entry (r-1)*Ns + k holds w_{Ns R}^{k r}, consecutive k for
// consecutive lanes.  Where LDS has room next to the tile, the kernels copy
// it (or its first pass's part plus a two-level table of w_L) to LDS first.
#include "line_device.h"

namespace dpfft {

// SW bit 0: exchange re/im on load; bit 1: exchange on store (the inverse
// transform is swap(FFT(swap(x))), so the first launch of an inverse swaps on
// load and the last one on store).
//
// Addressing: an ELEM_FAST side has unit element stride (x_e == 1) and a
// LINE_FAST side has unit line stride (x_l == 1); the plan guarantees it.
template <int L, int C, int MAP, int OMAP, bool TW4, int SW, int EPT, int NT>
__global__ void __launch_bounds__(C * (P2<L, EPT>::T))
    k_lines(const cf *__restrict__ in, cf *__restrict__ out, LineArgs a) {
  using G = P2<L, EPT>;
  static_assert(C * G::T <= 1024, "a workgroup holds at most 1024 threads");
  constexpr int E = G::E, T = G::T;
  using LO = Lds<L, C, OMAP, kPadShift>;
  constexpr int NP = lds_pairs<L, C, MAP, OMAP>();
  __shared__ __align__(16) cf lds[NP > 0 ? NP : 1];

  const int tid = threadIdx.x;
  int c, j;
  lane_map<L, EPT, C, MAP>(tid, c, j);
  const uint32_t tile = !(a.flags & F_REMAP)  ? blockIdx.x
                        : (a.flags & F_ROUNDS) ? xcd_remap_rounds(blockIdx.x, gridDim.x, (a.flags & F_ROUNDS16) ? 4 : 5)
                                               : xcd_remap(blockIdx.x, gridDim.x);
  const int64_t bb = tile / a.tiles_per_batch;
  const int64_t line0 = (int64_t)(tile - bb * a.tiles_per_batch) * C;
  const int64_t line = line0 + c;
  const bool valid = line < a.lines;

  cf v[E];
  if (valid) {
    if constexpr (MAP == ELEM_FAST) {
      const cf *src = in + bb * a.in_b + (line0 + c) * a.in_l + j;
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = ld_data<NT>(src + T * m);
    } else {
      const cf *tin = in + bb * a.in_b + line0;
      const uint32_t es = (uint32_t)a.in_e;
      const uint32_t o = (uint32_t)c + (uint32_t)j * es;
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = ldg<NT>(tin, o + (uint32_t)(T * m) * es);
    }
    if constexpr (SW & 1) {
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = cswap(v[m]);
    }
  } else {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = make_float2(0.0f, 0.0f);
  }

  using PT = PlainTw<L, C, MAP, OMAP, EPT, C * G::T>;
  // Four-step twiddle bases.  Where two or more workgroups share a CU, their
  // table entries are loaded before the passes, so that the latency passes
  // behind them instead of before the stores (the 256-point column tiles of
  // a batch of 4096 transforms of 2^16 points: 3% faster).  The
  // one-workgroup-per-CU tiles gained nothing from it and load them after
  // the passes.  A lane past the last line reads the entries of line 0; it
  // stores nothing.
  constexpr bool TW4_EARLY = (NP + PT::NTW) * (int)sizeof(cf) * 2 <= PT::kLds;
  cf tAh, tAl, tBh, tBl;
  auto tw4_parts = [&]() {
    const uint32_t n2 = valid ? (uint32_t)line : 0u;
    const uint32_t msk = (1u << a.tw4_shift) - 1u;
    const uint32_t eA = n2 * (uint32_t)j, eB = n2 * (uint32_t)T;
    tAh = a.tw4_hi[eA >> a.tw4_shift];
    tAl = a.tw4_lo[eA & msk];
    tBh = a.tw4_hi[eB >> a.tw4_shift];
    tBl = a.tw4_lo[eB & msk];
  };
  if constexpr (TW4 && TW4_EARLY) tw4_parts();

  __shared__ cf twl[PT::NTW > 0 ? PT::NTW : 1];
  PT::fill(twl, a, tid);
  all_passes<L, EPT, C, MAP>(v, lds, PT::make(twl, a), c, j,
                             std::make_integer_sequence<int, G::NP>{});

  // epilogue in registers: four-step twiddle, inverse scale
  if constexpr (TW4) {
    if constexpr (!TW4_EARLY) tw4_parts();
    tw4_apply_ab<E>(v, cmul(tAh, tAl), cmul(tBh, tBl));
  }
  if constexpr (SW & 2) {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = cscale(v[m], a.scale);
  }
  int c2 = c, j2 = j;
  int64_t line2 = line;
  if constexpr (OMAP != MAP) {
    // re-tile through LDS so the store is coalesced in the output layout
    lane_map<L, EPT, C, OMAP>(tid, c2, j2);
    line2 = line0 + c2;
    auto wpos = [&](int m) { return LO::idx_off(c, j, T * m); };
    auto rpos = [&](int m) { return LO::idx_off(c2, j2, T * m); };
    lds_exchange<E, false>(v, lds, wpos, rpos);
  }
  if (line2 < a.lines) {
    if constexpr (SW & 2) {
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = cswap(v[m]);
    }
    if constexpr (OMAP == ELEM_FAST) {
      cf *dst = out + bb * a.out_b + line2 * a.out_l + j2;
#pragma unroll
      for (int m = 0; m < E; ++m) st_data<NT>(dst + T * m, v[m]);
    } else {
      cf *tout = out + bb * a.out_b + line0;
      const uint32_t es = (uint32_t)a.out_e;
      const uint32_t o = (uint32_t)c2 + (uint32_t)j2 * es;
#pragma unroll
      for (int m = 0; m < E; ++m) stg<NT>(tout, o + (uint32_t)(T * m) * es, v[m]);
    }
  }
}

// ---------------------------------------------------------------------------
// Persistent form for instances whose LDS buffer allows one workgroup per CU.
// A grid of resident workgroups loops over the tiles; while a tile is being
// transformed, the next tile's elements (and its four-step twiddle bases) are
// already in flight into a second register set, so the CU keeps HBM busy
// through the passes and barriers.  Pass twiddles come from LDS.  Each round
// of gridDim tiles is split so that every XCD sweeps a contiguous slice.
// ---------------------------------------------------------------------------
// A lane whose line lies past the last one of a ragged last tile loads the
// last line instead (and its results are never stored): no branch, so the
// loads of a prefetch land directly in the registers that hold them.
template <int L, int EPT, int C, int MAP, int NT>
__device__ __forceinline__ void load_tile(cf (&v)[(P2<L, EPT>::E)], const cf *__restrict__ in,
                                          const LineArgs &a, int64_t tile, int c, int j) {
  constexpr int E = P2<L, EPT>::E, T = P2<L, EPT>::T;
  const int64_t bb = tile / a.tiles_per_batch;
  const int64_t line0 = (tile - bb * a.tiles_per_batch) * C;
  const int64_t lc = line0 + c < a.lines ? c : a.lines - 1 - line0;
  if constexpr (MAP == ELEM_FAST) {
    const cf *src = in + bb * a.in_b + (line0 + lc) * a.in_l + j;
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = ld_data<NT>(src + T * m);
  } else {
    const cf *tin = in + bb * a.in_b + line0;
    const uint32_t es = (uint32_t)a.in_e;
    const uint32_t o = (uint32_t)lc + (uint32_t)j * es;
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = ldg<NT>(tin, o + (uint32_t)(T * m) * es);
  }
}

template <int L, int C, int MAP, int OMAP, bool TW4, int SW, int EPT, int NT>
__global__ void __launch_bounds__(C * (P2<L, EPT>::T))
    k_lines_pf(const cf *__restrict__ in, cf *__restrict__ out, LineArgs a) {
  using G = P2<L, EPT>;
  static_assert(C * G::T <= 1024, "a workgroup holds at most 1024 threads");
  constexpr int E = G::E, T = G::T, NTH = C * G::T;
  constexpr int S = tw2_shift(G::LG), NLO = 1 << S, NHI = (L >> S) > 0 ? (L >> S) : 1;
  using LO = Lds<L, C, OMAP, kPadShift>;
  constexpr int NPR = lds_pairs<L, C, MAP, OMAP>();
  __shared__ __align__(16) cf lds[NPR > 0 ? NPR : 1];
  constexpr bool DIRECT = pf_direct_tw<L, C, MAP, OMAP, EPT>();
  constexpr bool FIRST = pf_first_tw<L, C, MAP, OMAP, EPT>();
  constexpr int NTW = pf_tw_entries<L, C, MAP, OMAP, EPT>();
  constexpr int N2L = pf_tw2_entries<L, EPT>();
  __shared__ cf twl[NTW];
  if constexpr (DIRECT) {
    for (int i = threadIdx.x; i < NTW; i += NTH) twl[i] = a.tw[i];
  } else {
    // two-level table, then (FIRST) the first twiddle pass's part of a.tw
    for (int i = threadIdx.x; i < NTW; i += NTH) twl[i] = i < N2L ? a.tw2[i] : a.tw[i - N2L];
  }
  __syncthreads();
  using TWS = std::conditional_t<DIRECT, TwLdsTable, std::conditional_t<FIRST, TwLdsFirst, TwLds2>>;
  TWS tw;
  if constexpr (DIRECT) {
    tw = TwLdsTable{twl};
  } else if constexpr (FIRST) {
    tw = TwLdsFirst{twl + N2L, TwLds2{twl, twl + NLO}};
  } else {
    tw = TwLds2{twl, twl + NLO};
  }

  const int tid = threadIdx.x;
  int c, j;
  lane_map<L, EPT, C, MAP>(tid, c, j);
  const uint32_t Gd = gridDim.x, bid = blockIdx.x;
  const uint32_t slot = (Gd % 8u == 0u) ? (bid % 8u) * (Gd / 8u) + bid / 8u : bid;
  int64_t tile = slot;
  if (tile >= a.ntiles) return;

  // The prefetched tile is swapped (inverse) only when it becomes current, and
  // the four-step twiddle inputs of the next tile are loaded before its data:
  // every wait for an older load then leaves the prefetch in flight.
  cf v[E], vn[E];
  load_tile<L, EPT, C, MAP, NT>(v, in, a, tile, c, j);
  cf A = make_float2(1.f, 0.f), B = A;
  cf nAh = A, nAl = A, nBh = A, nBl = A;  // tw4 table entries of the next tile
  auto line_of = [&](int64_t t) {  // clamped like the loads of load_tile
    const int64_t bb = t / a.tiles_per_batch;
    const int64_t line = (t - bb * a.tiles_per_batch) * C + c;
    return line < a.lines ? line : a.lines - 1;
  };
  if constexpr (TW4) {
    const uint32_t n2 = (uint32_t)line_of(tile);
    A = tw4_lookup(a, n2 * (uint32_t)j);
    B = tw4_lookup(a, n2 * (uint32_t)T);
  }
  // Wait for the first tile here.  Otherwise the wait-count analysis merges
  // these loads, still pending at the loop entry, with the path on which no
  // prefetch is issued, and makes the first pass of every tile wait for the
  // prefetch of the next one as well (no overlap at all).
#pragma unroll
  for (int m = 0; m < E; ++m) pin_regs(v[m]);
  pin_regs(A);
  pin_regs(B);

  for (; tile < a.ntiles; tile += Gd) {
    // Keep the compiler from hoisting every pass's LDS addresses and twiddles
    // out of the tile loop: they would not fit next to the two register sets.
    asm volatile("" : "+v"(c), "+v"(j));
    // In the last round every workgroup prefetches the last tile once more
    // (L2 hits): an unconditional prefetch lets its loads land directly in
    // the registers of the next tile, where a branch around it makes the
    // compiler copy them, and wait for them, right after they are issued.
    const int64_t next = tile + Gd < a.ntiles ? tile + Gd : a.ntiles - 1;
    if constexpr (TW4) {
      const uint32_t n2 = (uint32_t)line_of(next);
      const uint32_t eA = n2 * (uint32_t)j, eB = n2 * (uint32_t)T;
      const uint32_t msk = (1u << a.tw4_shift) - 1u;
      nAh = a.tw4_hi[eA >> a.tw4_shift];
      nAl = a.tw4_lo[eA & msk];
      nBh = a.tw4_hi[eB >> a.tw4_shift];
      nBl = a.tw4_lo[eB & msk];
    }
    load_tile<L, EPT, C, MAP, NT>(vn, in, a, next, c, j);
    if constexpr (SW & 1) {
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = cswap(v[m]);
    }
    all_passes<L, EPT, C, MAP>(v, lds, tw, c, j, std::make_integer_sequence<int, G::NP>{});
    if constexpr (TW4) tw4_apply_ab<E>(v, A, B);
    if constexpr (SW & 2) {
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = cscale(v[m], a.scale);
    }
    const int64_t bb = tile / a.tiles_per_batch;
    const int64_t line0 = (tile - bb * a.tiles_per_batch) * C;
    int c2 = c, j2 = j;
    if constexpr (OMAP != MAP) {
      lane_map<L, EPT, C, OMAP>(tid, c2, j2);
      auto wpos = [&](int m) { return LO::idx_off(c, j, T * m); };
      auto rpos = [&](int m) { return LO::idx_off(c2, j2, T * m); };
      lds_exchange<E, true>(v, lds, wpos, rpos);
    }
    // Lanes past the last line of a ragged last tile hold that line's results
    // (they loaded it, with its twiddles) and store them once more to the same
    // addresses: identical values, and no branch around the stores.  With a
    // branch, the wait for the prefetch (on the copy below) would also wait
    // for the stores, which then could not drain during the next tile.
    const int64_t lc2 = line0 + c2 < a.lines ? c2 : a.lines - 1 - line0;
    if constexpr (SW & 2) {
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = cswap(v[m]);
    }
    if constexpr (OMAP == ELEM_FAST) {
      cf *dst = out + bb * a.out_b + (line0 + lc2) * a.out_l + j2;
#pragma unroll
      for (int m = 0; m < E; ++m) st_data<NT>(dst + T * m, v[m]);
    } else {
      cf *tout = out + bb * a.out_b + line0;
      const uint32_t es = (uint32_t)a.out_e;
      const uint32_t o = (uint32_t)lc2 + (uint32_t)j2 * es;
#pragma unroll
      for (int m = 0; m < E; ++m) stg<NT>(tout, o + (uint32_t)(T * m) * es, v[m]);
    }
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = vn[m];
    if constexpr (TW4) {
      A = cmul(nAh, nAl);
      B = cmul(nBh, nBl);
    }
  }
}

// ---------------------------------------------------------------------------
// Two sub-lines per line.  One radix-2 step in frequency (decimation in
// frequency) splits a line of L points into a[n] = x[n] + x[n + L/2] and
// b[n] = (x[n] - x[n + L/2]) w_L^n, n < L/2, whose L/2-point transforms are
// the even and the odd outputs: X[2k] = A[k], X[2k + 1] = B[k].  The two
// sub-lines then go through the Stockham passes one after the other, sharing
// an LDS buffer of half a tile, so two workgroups share a CU and overlap each
// other's loads, barriers and butterflies, while every row piece the tile
// reads or writes stays C x 8 bytes wide; the first sub-line's stores drain
// while the second one is transformed.  Thread j of a line holds elements
// j + T m (m < 2 ES, T = L / (2 ES)) with ES = 16 (radix-16 passes) or 8
// (radix-8 passes, twice the threads and half the registers): the pairs
// (m, m + ES) are the split's operands, and w_L^{j + T m} = w_L^j w_{2 ES}^m.
// ---------------------------------------------------------------------------
// Pass twiddles of a sub-line: its per-pass table in LDS where it fits next to
// the half tile for two workgroups per CU (else read from global memory).
template <int L, int C, int MAP, int OMAP, int ES>
constexpr int half_tw_entries() {
  constexpr int n = P2<L / 2, ES>::twoff(P2<L / 2, ES>::NP);
  return (n > 0 && (lds_pairs<L / 2, C, MAP, OMAP>() + n) * 8 <= 80 * 1024) ? n : 0;
}
template <int ES, int M>
__device__ __forceinline__ void half_split_one(cf &x, cf &y, cf wj) {
  const cf s = make_float2(x.x + y.x, x.y + y.y);
  const cf d = make_float2(x.x - y.x, x.y - y.y);
  x = s;
  y = cmul(mulw32<2 * ES, M>(d), wj);
}
template <int ES, int... M>
__device__ __forceinline__ void half_split(cf (&va)[ES], cf (&vb)[ES], cf wj,
                                           std::integer_sequence<int, M...>) {
  (half_split_one<ES, M>(va[M], vb[M], wj), ...);
}

template <int L, int C, int MAP, int OMAP, bool TW4, int SW, int NT, int ES>
__global__ void __launch_bounds__(C * L / (2 * ES))
    __attribute__((amdgpu_waves_per_eu(C * L / (2 * ES) / 128)))
    k_lines_half(const cf *__restrict__ in, cf *__restrict__ out, LineArgs a) {
  constexpr int H = L / 2;
  using G = P2<H, ES>;
  constexpr int E = G::E, T = G::T, NTH = C * T;
  static_assert(E == ES && T * 2 * ES == L, "ES elements of each sub-line per thread");
  static_assert(NTH <= 1024, "a workgroup holds at most 1024 threads");
  using LO = Lds<H, C, OMAP, kPadShift>;
  constexpr int NP = lds_pairs<H, C, MAP, OMAP>();
  __shared__ __align__(16) cf lds[NP > 0 ? NP : 1];

  const int tid = threadIdx.x;
  int c, j;
  lane_map<H, ES, C, MAP>(tid, c, j);
  const uint32_t tile = !(a.flags & F_REMAP)  ? blockIdx.x
                        : (a.flags & F_ROUNDS) ? xcd_remap_rounds(blockIdx.x, gridDim.x, (a.flags & F_ROUNDS16) ? 4 : 5)
                                               : xcd_remap(blockIdx.x, gridDim.x);
  const int64_t bb = tile / a.tiles_per_batch;
  const int64_t line0 = (int64_t)(tile - bb * a.tiles_per_batch) * C;
  const int64_t line = line0 + c;
  const bool valid = line < a.lines;

  cf va[E], vb[E];
  if (valid) {
    if constexpr (MAP == ELEM_FAST) {
      const cf *src = in + bb * a.in_b + line * a.in_l + j;
#pragma unroll
      for (int m = 0; m < E; ++m) va[m] = ld_data<NT>(src + T * m);
#pragma unroll
      for (int m = 0; m < E; ++m) vb[m] = ld_data<NT>(src + H + T * m);
    } else {
      const cf *tin = in + bb * a.in_b + line0;
      const uint32_t es = (uint32_t)a.in_e;
      const uint32_t o = (uint32_t)c + (uint32_t)j * es;
#pragma unroll
      for (int m = 0; m < E; ++m) va[m] = ldg<NT>(tin, o + (uint32_t)(T * m) * es);
#pragma unroll
      for (int m = 0; m < E; ++m) vb[m] = ldg<NT>(tin, o + (uint32_t)(H + T * m) * es);
    }
    if constexpr (SW & 1) {
#pragma unroll
      for (int m = 0; m < E; ++m) va[m] = cswap(va[m]), vb[m] = cswap(vb[m]);
    }
  } else {
#pragma unroll
    for (int m = 0; m < E; ++m) va[m] = vb[m] = make_float2(0.0f, 0.0f);
  }

  // w_L^j from the two-level table of w_L (j < T <= 2^S: a lo entry alone)
  constexpr int S = tw2_shift(P2<L>::LG);
  cf wj;
  if constexpr (T <= (1 << S)) {
    wj = a.tw2[j];
  } else {
    wj = cmul(a.tw2[(1 << S) + (j >> S)], a.tw2[j & ((1 << S) - 1)]);
  }

  constexpr int NTW = half_tw_entries<L, C, MAP, OMAP, ES>();
  __shared__ cf twl[NTW > 0 ? NTW : 1];
  if constexpr (NTW > 0) {
    for (int i = tid; i < NTW; i += NTH) twl[i] = a.tw[i];
  }
  using TWS = std::conditional_t<(NTW > 0), TwLdsTable, TwTable>;
  TWS tws;
  if constexpr (NTW > 0) {
    tws = TwLdsTable{twl};
  } else {
    tws = TwTable{a.tw};
  }

  half_split<ES>(va, vb, wj, std::make_integer_sequence<int, E>{});

  int c2 = c, j2 = j;
  if constexpr (OMAP != MAP) lane_map<H, ES, C, OMAP>(tid, c2, j2);
  const int64_t line2 = line0 + c2;
  // outputs of sub-line s: element j + T m holds X[2 (j + T m) + s]
  auto finish = [&](cf(&v)[E], const int s) {
    if constexpr (TW4) {
      const uint32_t n2 = valid ? (uint32_t)line : 0u;
      const uint32_t msk = (1u << a.tw4_shift) - 1u;
      const uint32_t eA = n2 * (uint32_t)(2 * j + s), eB = n2 * (uint32_t)(2 * T);
      const cf A = cmul(a.tw4_hi[eA >> a.tw4_shift], a.tw4_lo[eA & msk]);
      const cf B = cmul(a.tw4_hi[eB >> a.tw4_shift], a.tw4_lo[eB & msk]);
      tw4_apply_ab<E>(v, A, B);
    }
    if constexpr (SW & 2) {
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = cscale(v[m], a.scale);
    }
    if constexpr (OMAP != MAP) {
      // re-tile through LDS; the barrier after the reads frees the buffer
      // for the next sub-line
      auto wpos = [&](int m) { return LO::idx_off(c, j, T * m); };
      auto rpos = [&](int m) { return LO::idx_off(c2, j2, T * m); };
      lds_exchange<E, true>(v, lds, wpos, rpos);
    }
    if (line2 < a.lines) {
      if constexpr (SW & 2) {
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = cswap(v[m]);
      }
      if constexpr (OMAP == ELEM_FAST) {
        cf *dst = out + bb * a.out_b + line2 * a.out_l + 2 * j2 + s;
#pragma unroll
        for (int m = 0; m < E; ++m) st_data<NT>(dst + 2 * T * m, v[m]);
      } else {
        cf *tout = out + bb * a.out_b + line0;
        const uint32_t es = (uint32_t)a.out_e;
        const uint32_t o = (uint32_t)c2 + (uint32_t)(2 * j2 + s) * es;
#pragma unroll
        for (int m = 0; m < E; ++m) stg<NT>(tout, o + (uint32_t)(2 * T * m) * es, v[m]);
      }
    }
  };
  // The last exchange of a sub-line's passes ends with a barrier after its
  // reads, and so does the re-tiling, so the next sub-line may write LDS.
  all_passes<H, ES, C, MAP>(va, lds, tws, c, j, std::make_integer_sequence<int, G::NP>{});
  finish(va, 0);
  all_passes<H, ES, C, MAP>(vb, lds, tws, c, j, std::make_integer_sequence<int, G::NP>{});
  finish(vb, 1);
}

// ---------------------------------------------------------------------------
// registry of compiled instances
// ---------------------------------------------------------------------------
struct LineEntry {
  int L, C, map, omap;
  bool tw4;
  const void *fn[4];  // by SW; nullptr where not instantiated
  int threads;
  int lds;
  bool pf;
  bool pref;          // the planner's default for its shape (measured fastest)
  int ept;
  int sub = 1;        // sub-lines per line (2: k_lines_half)
};

#define KL(L_, C_, M_, O_, TW_, SW_) (const void *)&KFN<L_, C_, M_, O_, TW_, SW_, KEPT, KNT>
#define ENTRY(L_, C_, M_, O_, TW_, F0, F1, F2, F3)                                  \
  LineEntry{L_, C_, M_, O_, TW_, {F0, F1, F2, F3}, C_ * P2<L_, KEPT>::T,            \
            (int)sizeof(cf) * lds_pairs<L_, C_, M_, O_>() +                         \
                (int)sizeof(cf) * (KPF ? pf_tw_entries<L_, C_, M_, O_, KEPT>()        \
                                       : PlainTw<L_, C_, M_, O_, KEPT,                \
                                                 C_ * P2<L_, KEPT>::T>::NTW),         \
            KPF, KPREF, KEPT}

// rows: forward, inverse single pass (swap in+out), 2D row pass inverse (swap in)
#define ROW(L_, C_)                                                                          \
  ENTRY(L_, C_, ELEM_FAST, ELEM_FAST, false, KL(L_, C_, ELEM_FAST, ELEM_FAST, false, 0),   \
        KL(L_, C_, ELEM_FAST, ELEM_FAST, false, 1), nullptr,                                \
        KL(L_, C_, ELEM_FAST, ELEM_FAST, false, 3))
// 2D column pass: forward, inverse (swap out); the real-input 2D inverse runs
// its column pass first (swap in and out)
#define COL(L_, C_)                                                                          \
  ENTRY(L_, C_, LINE_FAST, LINE_FAST, false, KL(L_, C_, LINE_FAST, LINE_FAST, false, 0),   \
        nullptr, KL(L_, C_, LINE_FAST, LINE_FAST, false, 2),                                 \
        KL(L_, C_, LINE_FAST, LINE_FAST, false, 3))
// four-step first pass: forward, inverse (swap in)
#define COLTW(L_, C_)                                                                        \
  ENTRY(L_, C_, LINE_FAST, LINE_FAST, true, KL(L_, C_, LINE_FAST, LINE_FAST, true, 0),     \
        KL(L_, C_, LINE_FAST, LINE_FAST, true, 1), nullptr, nullptr)
// four-step second pass: forward, inverse (swap out)
#define ROWT(L_, C_)                                                                         \
  ENTRY(L_, C_, ELEM_FAST, LINE_FAST, false, KL(L_, C_, ELEM_FAST, LINE_FAST, false, 0),   \
        nullptr, KL(L_, C_, ELEM_FAST, LINE_FAST, false, 2), nullptr)

#define KFN k_lines
#define KPF false
#define KPREF false
#define KEPT 16
#define KNT 0
static const LineEntry kLineTable[] = {
    // batched rows (single-pass transforms, 2D row pass)
    ROW(1, 256), ROW(2, 256), ROW(4, 256), ROW(8, 256), ROW(16, 256), ROW(32, 128),
    ROW(64, 64), ROW(128, 32), ROW(256, 16), ROW(512, 8), ROW(1024, 4), ROW(1024, 8),
    ROW(2048, 4), ROW(4096, 1), ROW(4096, 2), ROW(8192, 1), ROW(16384, 1),
    // column tiles (2D column pass)
    COL(16, 64), COL(32, 32), COL(64, 16), COL(128, 16), COL(256, 16), COL(512, 16),
    COL(1024, 16), COL(1024, 8), COL(2048, 4), COL(2048, 8), COL(4096, 4),
    // column tiles with the four-step twiddle (first four-step pass)
    COLTW(64, 16), COLTW(128, 16), COLTW(256, 32), COLTW(512, 16),
    COLTW(1024, 16), COLTW(1024, 8), COLTW(2048, 4), COLTW(2048, 8), COLTW(4096, 4),
    // rows stored transposed (second four-step pass)
    ROWT(64, 16), ROWT(128, 16), ROWT(256, 32), ROWT(512, 16),
    ROWT(1024, 16), ROWT(1024, 8), ROWT(2048, 4), ROWT(2048, 8), ROWT(4096, 4),
};
// nontemporal tile data (rows of 2048, the 256 x 256 four-step): 2-4% faster
#undef KNT
#define KNT 3
static const LineEntry kLineTableNt[] = {
    ROW(2048, 2), COLTW(256, 16), ROWT(256, 16),
};
#undef KNT
#define KNT 0
#undef KEPT
#define KEPT 32
// 32 elements per thread without the persistent loop: two radix-32/16 passes
// for 512-point tiles instead of three.  The 2D column tiles of 512 are the
// default of their shape (4-5% faster); the others are opt-in for the tuner.
#undef KPREF
#define KPREF true
static const LineEntry kLineTable32Pref[] = {
    COL(512, 16),
};
#undef KPREF
#define KPREF false
static const LineEntry kLineTable32[] = {
    ROW(1024, 8), ROW(1024, 16), COLTW(512, 16), COLTW(512, 32), ROWT(512, 16), ROWT(512, 32),
};
#undef KFN
#undef KPF
#undef KEPT
#define KFN k_lines_pf
#define KPF true
#define KEPT 16
// Persistent instances, 16 elements per thread.  Rows of 4096, two per tile,
// are the default of their shape (3-4% faster than the plain 1-row tiles,
// nontemporal data 1% more); the others are opt-in (rows of 8192: 9% slower
// than the plain kernel once that reads its twiddles from LDS).
#undef KPREF
#define KPREF true
#undef KNT
#define KNT 3
static const LineEntry kLineTablePfPref[] = {
    ROW(4096, 2),
};
#undef KNT
#define KNT 0
#undef KPREF
#define KPREF false
static const LineEntry kLineTablePf[] = {
    ROW(8192, 1), ROW(16384, 1), COL(1024, 16), COLTW(1024, 16),
};
#undef KEPT
#define KEPT 32
// Persistent instances, 32 elements per thread (radix-32 passes: one pass and
// one exchange fewer than radix 16 for L = 2^10, 2^13 and 2^14), whose tiles
// fill the CU's LDS.  The defaults of their shapes, measured against the best
// other instance: rows of 16384 15% faster; rows of 1024, 16 per tile, 5%;
// 1024-point transposed rows 13%; 1024-point column tiles as fast as the
// plain ones.
#undef KPREF
#define KPREF true
static const LineEntry kLineTablePf32[] = {
    ROW(16384, 1), COL(1024, 16), COLTW(1024, 16), ROWT(1024, 16),
};
// rows of 1024 with nontemporal stores (2% faster)
#undef KNT
#define KNT 2
static const LineEntry kLineTablePf32Nts[] = {
    ROW(1024, 16),
};
#undef KPREF
#define KPREF false
// opt-in: 512-point column tiles of 32 with nontemporal data, and the others
// measured slower than the plain instances once those read their twiddles
// from LDS (512-point tiles of 32 lines by 5%, tiles of 2048 by 5-20%) or
// always (4096-point four-step tiles)
#undef KNT
#define KNT 3
static const LineEntry kLineTablePf32Nt[] = {
    COLTW(512, 32),
};
#undef KNT
#define KNT 0
static const LineEntry kLineTablePf32x[] = {
    ROW(8192, 1), COLTW(2048, 8), ROWT(2048, 8), COL(2048, 8), COLTW(512, 16), ROWT(512, 16),
    ROWT(512, 32), ROWT(4096, 4), COLTW(4096, 4),
};
#undef KFN
#undef KPF
#undef KPREF
#undef KEPT
#undef KNT

// Split-first instances (k_lines_half): half the LDS of the plain tile, two
// workgroups per CU.  The 1024-point column tiles of 16 are the default of
// their shape (2D 1024 x 1024 column pass 11% faster than the persistent
// 32-element tiles); the transposed rows of 1024 measured as fast as their
// default and are opt-in.  Measured and not kept: 16-element tiles of 2048
// (column tiles with and without the four-step twiddle, transposed rows:
// 1-4% slower, and 33% where the four-step twiddle spills registers at the
// 128-VGPR budget of two workgroups per CU), the same tiles with 8 elements
// of each sub-line per thread (1024 threads, radix-8 passes, 32 waves per CU:
// they spill at 64 registers and run 17-57% slower), 4096-point tiles of 4
// (spills, 35-70% slower) and the 1024-point four-step column tiles (5%
// slower than the persistent ones).
#define KH(L_, C_, M_, O_, TW_, SW_) (const void *)&k_lines_half<L_, C_, M_, O_, TW_, SW_, 0, KES>
#define HENTRY(L_, C_, M_, O_, TW_, F0, F1, F2, F3)                                        \
  LineEntry{L_, C_, M_, O_, TW_, {F0, F1, F2, F3}, C_ * L_ / (2 * KES),                     \
            (int)sizeof(cf) * lds_pairs<L_ / 2, C_, M_, O_>() +                              \
                (int)sizeof(cf) * half_tw_entries<L_, C_, M_, O_, KES>(),                     \
            false, KPREF, KES, 2}
#define HCOL(L_, C_)                                                                       \
  HENTRY(L_, C_, LINE_FAST, LINE_FAST, false, KH(L_, C_, LINE_FAST, LINE_FAST, false, 0), \
         nullptr, KH(L_, C_, LINE_FAST, LINE_FAST, false, 2),                               \
         KH(L_, C_, LINE_FAST, LINE_FAST, false, 3))
#define HROWT(L_, C_)                                                                      \
  HENTRY(L_, C_, ELEM_FAST, LINE_FAST, false, KH(L_, C_, ELEM_FAST, LINE_FAST, false, 0), \
         nullptr, KH(L_, C_, ELEM_FAST, LINE_FAST, false, 2), nullptr)
#define KES 16
#define KPREF true
static const LineEntry kLineTableHalfPref[] = {
    HCOL(1024, 16),
};
#undef KPREF
#define KPREF false
static const LineEntry kLineTableHalf[] = {
    HROWT(1024, 16),
};
#undef KES
#undef KPREF
#undef HCOL
#undef HROWT
#undef HENTRY
#undef KH

static void fill(const LineEntry &e, KernelInfo *out) {
  for (int i = 0; i < 4; ++i) out->fn_sw[i] = e.fn[i];
  out->fn = e.fn[0];
  out->threads = e.threads;
  out->lines = e.C;
  out->lds_bytes = e.lds;
  out->map = e.map;
  out->omap = e.omap;
  out->persistent = e.pf;
  out->preferred = e.pref;
  out->ept = e.ept;
  out->sub = e.sub;
}

template <class F>
static void for_each_entry(F f) {
  for (const auto &e : kLineTable) f(e);
  for (const auto &e : kLineTableNt) f(e);
  for (const auto &e : kLineTable32Pref) f(e);
  for (const auto &e : kLineTable32) f(e);
  for (const auto &e : kLineTablePfPref) f(e);
  for (const auto &e : kLineTablePf) f(e);
  for (const auto &e : kLineTablePf32) f(e);
  for (const auto &e : kLineTablePf32Nts) f(e);
  for (const auto &e : kLineTablePf32Nt) f(e);
  for (const auto &e : kLineTablePf32x) f(e);
  for (const auto &e : kLineTableHalfPref) f(e);
  for (const auto &e : kLineTableHalf) f(e);
}

uint64_t line_registry_digest() {
  // FNV-1a over every field the planner and the tuner read from an entry
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](int64_t v) {
    for (int b = 0; b < 8; ++b) {
      h ^= (uint64_t)((v >> (8 * b)) & 0xff);
      h *= 1099511628211ull;
    }
  };
  for_each_entry([&](const LineEntry &e) {
    mix(e.L), mix(e.C), mix(e.map), mix(e.omap), mix(e.tw4), mix(e.threads), mix(e.lds);
    mix(e.pf), mix(e.pref), mix(e.ept), mix(e.sub);
    for (int i = 0; i < 4; ++i) mix(e.fn[i] != nullptr);
  });
  return h;
}

int list_line_kernels(int L, int map, int omap, bool tw4, KernelInfo *out, int max) {
  int n = 0;
  for_each_entry([&](const LineEntry &e) {
    if (e.L == L && e.map == map && e.omap == omap && e.tw4 == tw4) {
      if (n < max) fill(e, &out[n]);
      ++n;
    }
  });
  return n;
}

}  // namespace dpfft
