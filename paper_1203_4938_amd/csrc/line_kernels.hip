// Power-of-two Stockham line kernels for gfx950.
//
// A workgroup transforms C "lines" (signals, matrix rows or matrix columns) of
// compile-time length L = 2^k.  Each line is owned by T = L/E threads that
// hold E = 16 elements each in registers (thread j owns elements j + T*m).
// Passes are radix 16 with one radix 2/4/8 remainder pass last.
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
// Twiddles of pass p >= 1 are read from a per-length table built on the host
// in FP64: entry (r-1)*Ns + k holds w_{Ns R}^{k r}, consecutive k for
// consecutive lanes.
#include "fft_common.h"
#include "kernels.h"

namespace dpfft {

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
};

template <int L, int C, int MAP, int PADSH, int P>
__device__ __forceinline__ void stockham_pass(cf (&v)[P2<L>::E], cf *lds,
                                              const cf *__restrict__ tw, int c, int j) {
  using G = P2<L>;
  constexpr int E = G::E, T = G::T, R = G::radix(P), NS = G::ns(P), QN = E / R;
  constexpr bool LAST = (P == G::NP - 1);
  constexpr int TWO = G::twoff(P);
  using LD = Lds<L, C, MAP, PADSH>;
#pragma unroll
  for (int q = 0; q < QN; ++q) {
    const int b = j + T * q;
    cf x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) x[r] = v[q + r * QN];
    const int k = b & (NS - 1);
    if constexpr (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) x[r] = cmul(x[r], tw[TWO + (r - 1) * NS + k]);
    }
    Dft<R>::run(x);
    if constexpr (LAST) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[q + r * QN] = x[r];
    } else {
      const int base = (b - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[LD::idx(c, base + r * NS)] = x[r];
    }
  }
  if constexpr (!LAST) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = lds[LD::idx(c, j + T * m)];
    __syncthreads();
  }
}

template <int L, int C, int MAP, int PADSH, int... P>
__device__ __forceinline__ void all_passes(cf (&v)[P2<L>::E], cf *lds, const cf *__restrict__ tw,
                                           int c, int j, std::integer_sequence<int, P...>) {
  (stockham_pass<L, C, MAP, PADSH, P>(v, lds, tw, c, j), ...);
}

template <int L, int C, int MAP>
__device__ __forceinline__ void lane_map(int tid, int &c, int &j) {
  constexpr int T = P2<L>::T;
  if constexpr (MAP == ELEM_FAST) {
    c = tid / T;
    j = tid % T;
  } else {
    c = tid % C;
    j = tid / C;
  }
}

// four-step twiddle w_N^e, e = line * i (< N), from the two-level table
__device__ __forceinline__ cf tw4_value(const LineArgs &a, int64_t e) {
  const int64_t lo = e & ((int64_t(1) << a.tw4_shift) - 1);
  const int64_t hi = e >> a.tw4_shift;
  return cmul(a.tw4_hi[hi], a.tw4_lo[lo]);
}

constexpr int kPadShift = 4;

template <int L, int C, int MAP, int OMAP, bool TW4>
__global__ void __launch_bounds__(C * P2<L>::T)
    k_lines(const cf *__restrict__ in, cf *__restrict__ out, LineArgs a) {
  using G = P2<L>;
  constexpr int E = G::E, T = G::T;
  constexpr bool NEED_LDS = (G::NP > 1) || (OMAP != MAP);
  using LI = Lds<L, C, MAP, kPadShift>;
  using LO = Lds<L, C, OMAP, kPadShift>;
  constexpr int LDS_SZ = NEED_LDS ? (LI::SIZE > LO::SIZE ? LI::SIZE : LO::SIZE) : 1;
  __shared__ cf lds[LDS_SZ];

  const int tid = threadIdx.x;
  int c, j;
  lane_map<L, C, MAP>(tid, c, j);
  const uint32_t tile = (a.flags & F_REMAP) ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
  const int64_t bb = tile / a.tiles_per_batch;
  const int64_t line0 = (int64_t)(tile - bb * a.tiles_per_batch) * C;
  const int64_t line = line0 + c;
  const bool valid = line < a.lines;

  cf v[E];
  if (valid) {
    const cf *src = in + bb * a.in_b + line * a.in_l;
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = src[(int64_t)(j + T * m) * a.in_e];
    if (a.flags & F_SWAP_IN) {
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = cswap(v[m]);
    }
  } else {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = make_float2(0.0f, 0.0f);
  }

  all_passes<L, C, MAP, kPadShift>(v, lds, a.tw, c, j, std::make_integer_sequence<int, G::NP>{});

  // epilogue: four-step twiddle and scale in registers
#pragma unroll
  for (int m = 0; m < E; ++m) {
    cf y = v[m];
    if constexpr (TW4) y = cmul(y, tw4_value(a, line * (int64_t)(j + T * m)));
    v[m] = cscale(y, a.scale);
  }
  const bool swap_out = (a.flags & F_SWAP_OUT) != 0;
  if constexpr (OMAP == MAP) {
    if (valid) {
      cf *dst = out + bb * a.out_b + line * a.out_l;
#pragma unroll
      for (int m = 0; m < E; ++m) {
        cf y = swap_out ? cswap(v[m]) : v[m];
        dst[(int64_t)(j + T * m) * a.out_e] = y;
      }
    }
  } else {
    // re-tile through LDS so the store is coalesced in the output layout
#pragma unroll
    for (int m = 0; m < E; ++m) lds[LO::idx(c, j + T * m)] = v[m];
    __syncthreads();
    int c2, j2;
    lane_map<L, C, OMAP>(tid, c2, j2);
    const int64_t line2 = line0 + c2;
    if (line2 < a.lines) {
      cf *dst = out + bb * a.out_b + line2 * a.out_l;
#pragma unroll
      for (int m = 0; m < E; ++m) {
        cf y = lds[LO::idx(c2, j2 + T * m)];
        if (swap_out) y = cswap(y);
        dst[(int64_t)(j2 + T * m) * a.out_e] = y;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// registry of compiled instances
// ---------------------------------------------------------------------------
struct LineEntry {
  int L, C, map, omap;
  bool tw4;
  const void *fn;
  int threads;
  int lds;
};

#define DP_LINE(L_, C_, M_, O_, TW_)                                                  \
  LineEntry{L_, C_, M_, O_, TW_, (const void *)&k_lines<L_, C_, M_, O_, TW_>,        \
            C_ * P2<L_>::T,                                                           \
            (int)sizeof(cf) *                                                         \
                (((P2<L_>::NP > 1) || (M_ != O_))                                     \
                     ? (Lds<L_, C_, M_, kPadShift>::SIZE > Lds<L_, C_, O_, kPadShift>::SIZE \
                            ? Lds<L_, C_, M_, kPadShift>::SIZE                        \
                            : Lds<L_, C_, O_, kPadShift>::SIZE)                       \
                     : 1)}

#define ROW(L_, C_) DP_LINE(L_, C_, ELEM_FAST, ELEM_FAST, false)
#define COL(L_, C_) DP_LINE(L_, C_, LINE_FAST, LINE_FAST, false)
#define COLTW(L_, C_) DP_LINE(L_, C_, LINE_FAST, LINE_FAST, true)
#define ROWT(L_, C_) DP_LINE(L_, C_, ELEM_FAST, LINE_FAST, false)

static const LineEntry kLineTable[] = {
    // batched rows (single-pass transforms, 2D row pass)
    ROW(1, 256), ROW(2, 256), ROW(4, 256), ROW(8, 256), ROW(16, 256), ROW(32, 128),
    ROW(64, 64), ROW(128, 32), ROW(256, 16), ROW(512, 8), ROW(1024, 4), ROW(2048, 2),
    ROW(4096, 1), ROW(4096, 2), ROW(8192, 1), ROW(16384, 1),
    // column tiles (2D column pass)
    COL(16, 64), COL(32, 32), COL(64, 16), COL(128, 16), COL(256, 16), COL(512, 16),
    COL(1024, 16), COL(1024, 8), COL(2048, 8), COL(4096, 4),
    // column tiles with the four-step twiddle (first four-step pass)
    COLTW(64, 16), COLTW(128, 16), COLTW(256, 16), COLTW(256, 32), COLTW(512, 16),
    COLTW(1024, 16), COLTW(1024, 8), COLTW(2048, 8), COLTW(4096, 4),
    // rows stored transposed (second four-step pass)
    ROWT(64, 16), ROWT(128, 16), ROWT(256, 16), ROWT(256, 32), ROWT(512, 16),
    ROWT(1024, 16), ROWT(1024, 8), ROWT(2048, 8), ROWT(4096, 4),
};

bool find_line_kernel(int L, int C, int map, int omap, bool tw4, KernelInfo *out) {
  for (const auto &e : kLineTable) {
    if (e.L == L && e.C == C && e.map == map && e.omap == omap && e.tw4 == tw4) {
      out->fn = e.fn;
      out->threads = e.threads;
      out->lines = e.C;
      out->lds_bytes = e.lds;
      return true;
    }
  }
  return false;
}

int best_line_c(int L, int map, int omap, bool tw4, int cmax) {
  int best = 0;
  for (const auto &e : kLineTable)
    if (e.L == L && e.map == map && e.omap == omap && e.tw4 == tw4 && e.C <= cmax && e.C > best)
      best = e.C;
  return best;
}

}  // namespace dpfft
