// Fused circular convolution: y = IDFT(DFT(x) * H) for every line, with H the
// DFT of the filter.  Section III-A of the paper names convolution and
// polynomial multiplication among the uses of the DFT, and section IV names
// the data movement between chained program instances as the platform's
// inefficiency; here the forward transform, the product with the filter
// spectrum and the inverse transform are one kernel, so a line makes a single
// round trip through HBM instead of three.
//
// Single pass (L <= 16384).  The line's Stockham passes leave X[j + T m] in
// the registers that loaded x[j + T m] (the natural order of the coalesced
// load); the product with H[j + T m] and the 1/L scale are applied in
// registers, and the inverse is the same forward passes run on swapped
// values (IDFT(Y) = swap(DFT(swap(Y))) / L).  The pass twiddles stay in LDS
// for both rounds.
//
// Four-step row form (N = N1 N2 > 16384).  The first launch is the forward
// column pass of the four-step (N1-point FFTs over n1, then w_N^{n2 k1}),
// leaving Y[k1][n2] in the workspace.  This kernel takes row k1 of Y: the
// N2-point forward FFT gives X[k1 + N1 k2] in its registers (k2 = j + T m),
// the product with H[k1 + N1 k2] / N follows, then the N2-point inverse over
// k2 and the factor w_N^{-k1 n2}, stored back in place as U[k1][n2].  The
// filter spectrum is read as a column tile of H viewed as an N2 x N1 matrix
// (C consecutive k1 per row segment, coalesced) and handed to the row lanes
// through LDS.  The last launch is the inverse N1-point column FFT over k1
// (for each n2), stored in natural order:
//   x[n1 N2 + n2] = sum_k1 w_N1^{-n1 k1} U[k1][n2].
#include "conv.h"
#include "line_device.h"

namespace dpfft {

// H[j + T m] * s, swapped: the product with the filter spectrum and the scale,
// entered in the swapped domain of the inverse passes
template <int E>
__device__ __forceinline__ void conv_product(cf (&v)[E], const cf (&h)[E], float s) {
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = cswap(cscale(cmul(v[m], h[m]), s));
}

template <int L, int C, int EPT>
__global__ void __launch_bounds__(C * (P2<L, EPT>::T))
    k_conv(const cf *__restrict__ in, cf *__restrict__ out, LineArgs a, ConvArgs f) {
  using G = P2<L, EPT>;
  static_assert(C * G::T <= 1024, "a workgroup holds at most 1024 threads");
  constexpr int E = G::E, T = G::T;
  constexpr int NP = lds_pairs<L, C, ELEM_FAST, ELEM_FAST>();
  __shared__ __align__(16) cf lds[NP > 0 ? NP : 1];
  using PT = PlainTw<L, C, ELEM_FAST, ELEM_FAST, EPT, C * G::T>;
  __shared__ cf twl[PT::NTW > 0 ? PT::NTW : 1];

  const int tid = threadIdx.x;
  int c, j;
  lane_map<L, EPT, C, ELEM_FAST>(tid, c, j);
  const int64_t line = (int64_t)blockIdx.x * C + c;
  const bool valid = line < a.lines;

  cf v[E];
  if (valid) {
    const cf *src = in + line * a.in_l + j;
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = src[T * m];
  } else {
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = make_float2(0.0f, 0.0f);
  }
  PT::fill(twl, a, tid);
  const auto tw = PT::make(twl, a);
  all_passes<L, EPT, C, ELEM_FAST>(v, lds, tw, c, j, std::make_integer_sequence<int, G::NP>{});

  // v[m] = X[j + T m]; the filter spectrum of this line (a lane past the last
  // line reads line 0's and stores nothing)
  cf h[E];
  {
    const cf *hp = f.h + (valid ? line : 0) * f.h_l + j;
#pragma unroll
    for (int m = 0; m < E; ++m) h[m] = hp[T * m];
  }
  conv_product<E>(v, h, a.scale);
  // the last forward pass left LDS free (its final exchange ended on a barrier)
  all_passes<L, EPT, C, ELEM_FAST>(v, lds, tw, c, j, std::make_integer_sequence<int, G::NP>{});
  if (valid) {
    cf *dst = out + line * a.out_l + j;
#pragma unroll
    for (int m = 0; m < E; ++m) dst[T * m] = cswap(v[m]);
  }
}

// Four-step row form: rows k1 of Y[k1][n2] (in place in the workspace), C
// consecutive rows per tile.  a.lines = N1 rows per batch item, a.in_b =
// a.out_b = N, a.in_l = a.out_l = N2; a.tw4_* is the two-level table of w_N;
// a.scale = 1/N.  f.h_b: elements between the spectra of consecutive batch
// items (0: shared); the spectrum X[k1 + N1 k2] of item b is at
// f.h + b f.h_b + k1 + N1 k2 (natural order, as the forward transform stores
// it).
template <int L, int C, int EPT>
__global__ void __launch_bounds__(C * (P2<L, EPT>::T))
    k_conv_rows(const cf *__restrict__ in, cf *__restrict__ out, LineArgs a, ConvArgs f) {
  using G = P2<L, EPT>;
  static_assert(C * G::T <= 1024, "a workgroup holds at most 1024 threads");
  constexpr int E = G::E, T = G::T;
  using LH = Lds<L, C, LINE_FAST, kPadShift>;  // the filter tile's transposition
  constexpr int NP = lds_pairs<L, C, ELEM_FAST, LINE_FAST>();
  __shared__ __align__(16) cf lds[NP];
  using PT = PlainTw<L, C, ELEM_FAST, ELEM_FAST, EPT, C * G::T>;
  __shared__ cf twl[PT::NTW > 0 ? PT::NTW : 1];

  const int tid = threadIdx.x;
  int c, j;
  lane_map<L, EPT, C, ELEM_FAST>(tid, c, j);
  int ch, jh;  // the same tile with lanes across the rows (filter reads)
  lane_map<L, EPT, C, LINE_FAST>(tid, ch, jh);
  const uint32_t tile = xcd_remap_rounds(blockIdx.x, gridDim.x);
  const int64_t bb = tile / a.tiles_per_batch;
  const int64_t line0 = (int64_t)(tile - bb * a.tiles_per_batch) * C;  // k1 of the tile's first row
  const int64_t N1 = a.lines;

  cf v[E];
  {
    const cf *src = in + bb * a.in_b + (line0 + c) * a.in_l + j;
#pragma unroll
    for (int m = 0; m < E; ++m) v[m] = src[T * m];
  }
  // filter spectrum: H[k1 + N1 k2], k1 = line0 + ch, k2 = jh + T m
  cf h[E];
  {
    const cf *hp = f.h + bb * f.h_b + line0 + ch + N1 * jh;
#pragma unroll
    for (int m = 0; m < E; ++m) h[m] = hp[N1 * (int64_t)(T * m)];
  }
  PT::fill(twl, a, tid);
  const auto tw = PT::make(twl, a);
  all_passes<L, EPT, C, ELEM_FAST>(v, lds, tw, c, j, std::make_integer_sequence<int, G::NP>{});

  // hand the filter tile to the row lanes
#pragma unroll
  for (int m = 0; m < E; ++m) lds[LH::idx_off(ch, jh, T * m)] = h[m];
  __syncthreads();
#pragma unroll
  for (int m = 0; m < E; ++m) h[m] = lds[LH::idx_off(c, j, T * m)];
  __syncthreads();  // the reads are done before the inverse passes write LDS

  conv_product<E>(v, h, a.scale);
  all_passes<L, EPT, C, ELEM_FAST>(v, lds, tw, c, j, std::make_integer_sequence<int, G::NP>{});
#pragma unroll
  for (int m = 0; m < E; ++m) v[m] = cswap(v[m]);
  // U[k1][n2] w_N^{-k1 n2}, n2 = j + T m: A = w_N^{-k1 j}, B = w_N^{-k1 T}
  {
    const uint32_t k1 = (uint32_t)(line0 + c);
    cf A = tw4_lookup(a, k1 * (uint32_t)j), B = tw4_lookup(a, k1 * (uint32_t)T);
    A.y = -A.y;
    B.y = -B.y;
    tw4_apply_ab<E>(v, A, B);
  }
  cf *dst = out + bb * a.out_b + (line0 + c) * a.out_l + j;
#pragma unroll
  for (int m = 0; m < E; ++m) dst[T * m] = v[m];
}

// ---------------------------------------------------------------------------
// registry
// ---------------------------------------------------------------------------
struct ConvEntry {
  int L, C, ept;
  bool rows4, pref;
  const void *fn;
  int threads, lds;
};

#define CV(L_, C_, EPT_, PREF_)                                                                \
  ConvEntry{L_, C_, EPT_, false, PREF_, (const void *)&k_conv<L_, C_, EPT_>, C_ * P2<L_, EPT_>::T, \
            (int)sizeof(cf) * (lds_pairs<L_, C_, ELEM_FAST, ELEM_FAST>() +                     \
                               PlainTw<L_, C_, ELEM_FAST, ELEM_FAST, EPT_,                     \
                                       C_ * P2<L_, EPT_>::T>::NTW)}
#define CR(L_, C_, EPT_, PREF_)                                                                   \
  ConvEntry{L_, C_, EPT_, true, PREF_, (const void *)&k_conv_rows<L_, C_, EPT_>,                 \
            C_ * P2<L_, EPT_>::T,                                                                 \
            (int)sizeof(cf) * (lds_pairs<L_, C_, ELEM_FAST, LINE_FAST>() +                        \
                               PlainTw<L_, C_, ELEM_FAST, ELEM_FAST, EPT_,                        \
                                       C_ * P2<L_, EPT_>::T>::NTW)}

// Single pass: 256 threads per workgroup up to L = 4096 (16 elements per
// thread), then one line per workgroup; 32-element forms (one pass fewer for
// L = 2^10, 2^13, 2^14) for the tuner.  Four-step rows: tiles of 16 rows
// (128-byte filter segments), 8 rows for N2 = 2048 and 4 for 4096.
static const ConvEntry kConvTable[] = {
    CV(1, 256, 16, true),    CV(2, 256, 16, true),    CV(4, 256, 16, true),
    CV(8, 256, 16, true),    CV(16, 256, 16, true),   CV(32, 128, 16, true),
    CV(64, 64, 16, true),    CV(128, 32, 16, true),   CV(256, 16, 16, true),
    CV(512, 8, 16, true),    CV(1024, 4, 16, true),   CV(2048, 2, 16, true),
    CV(4096, 1, 16, true),   CV(8192, 1, 16, true),   CV(16384, 1, 16, true),
    CV(1024, 8, 32, false),  CV(8192, 1, 32, false),  CV(16384, 1, 32, false),
    CR(128, 16, 16, true),   CR(256, 16, 16, true),   CR(512, 16, 16, true),
    CR(1024, 16, 16, true),  CR(2048, 8, 16, true),   CR(4096, 4, 16, true),
};
#undef CV
#undef CR

int list_conv_kernels(int L, bool rows4, ConvKernel *out, int max) {
  int n = 0;
  for (const auto &e : kConvTable) {
    if (e.L != L || e.rows4 != rows4) continue;
    if (n < max) {
      ConvKernel &k = out[n];
      k.fn = e.fn;
      k.L = e.L;
      k.lines = e.C;
      k.threads = e.threads;
      k.lds_bytes = e.lds;
      k.ept = e.ept;
      k.rows4 = e.rows4;
      k.preferred = e.pref;
    }
    ++n;
  }
  return n;
}

}  // namespace dpfft
