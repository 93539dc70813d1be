// 256-point line transforms with the DFT-16 stages on the matrix cores.
//
// A 256-point DFT is split as 16 x 16 (n = n2 + 16 n1, k = k1 + 16 k2):
//   stage 1: for each n2, a DFT-16 over n1          -> Y1[k1][n2]
//   twiddle: Y1[k1][n2] *= w_256^{n2 k1}            (FP32, on the vector ALUs)
//   stage 2: for each k1, a DFT-16 over n2          -> X[k1 + 16 k2]
// Each stage applies the 16x16 complex DFT matrix W to 16 vectors at once,
// written as a real product of a 16x32 matrix and a 32x16 matrix:
//   [Yr] = [Wr -Wi] [Xr]        A_re = [ cos | sin ]   (row i, column k)
//   [Yi]   [Wi  Wr] [Xi]        A_im = [-sin | cos ],  angle 2 pi i k / 16
// so a stage is one v_mfma_f32_16x16x32_{f16,bf16} for Yr and one for Yi,
// accumulating in FP32.  Operand layouts (64-wide wave, 16x16x32 shape):
//   A: lane l holds row (l & 15), k = 8 (l >> 4) + t, t = 0..7
//   B: lane l holds column (l & 15), k = 8 (l >> 4) + t
//   D: lane l holds column (l & 15), rows 4 (l >> 4) + t, t = 0..3
// (only the pairing of A and B k-slots matters for the sum, and both are
// built with the same convention).
//
// Split forms recover FP32 accuracy from 16-bit products.  With pieces
// x = xh + 2^-s xl (+ 2^-2s xll) and the same for W, scaled so every piece is
// a normal-range 16-bit number:
//   2 pieces: Y = Wh xh + 2^-s (Wh xl + Wl xh)                 (3 products)
//   3 pieces: Y = Wh xh + 2^-s (Wh xm + Wm xh)
//                       + 2^-2s (Wh xl + Wm xm + Wl xh)         (6 products)
// each group in its own FP32 accumulator (Ootomo and Yokota's scaled split for
// matrix units, SC 2022).  The W pieces are made on the host in FP64; the data
// pieces are made here with round-to-nearest-even conversions.
#include "fft_common.h"
#include "kernels.h"
#include "mfma.h"

namespace dpfft {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kPitch = 256 + 16 + 1;  // LDS pitch of a line (pad: one per 16, plus one)

// Tile data moves with the nontemporal hint: every tile row is a whole
// 128-byte segment or more, where it measured faster.
typedef float f2s __attribute__((ext_vector_type(2)));
__device__ __forceinline__ cf ld_stream(const cf *p) {
  const f2s r = __builtin_nontemporal_load((const f2s *)p);
  return make_float2(r.x, r.y);
}
__device__ __forceinline__ void st_stream(cf *p, cf v) {
  const f2s r = {v.x, v.y};
  __builtin_nontemporal_store(r, (f2s *)p);
}

__device__ __forceinline__ int tidx(int c, int pos) { return c * kPitch + pos + (pos >> 4); }

template <int PREC> struct Piece;
template <> struct Piece<MP_FP16> {
  typedef f16x8 vec;
  __device__ static _Float16 cvt(float x) { return (_Float16)x; }
  __device__ static float back(_Float16 h) { return (float)h; }
};
template <> struct Piece<MP_BF16> {
  typedef bf16x8 vec;
  __device__ static __bf16 cvt(float x) { return (__bf16)x; }
  __device__ static float back(__bf16 h) { return (float)h; }
};

template <int PREC> constexpr int base_of() {
  return (PREC == MP_FP16 || PREC == MP_FP16_SPLIT) ? MP_FP16 : MP_BF16;
}

template <int B>
__device__ __forceinline__ f32x4 mfma(typename Piece<B>::vec a, typename Piece<B>::vec b, f32x4 c) {
  if constexpr (B == MP_FP16)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// split eight FP32 values into NP 16-bit pieces (scaled by 2^s between pieces)
template <int PREC>
__device__ __forceinline__ void split8(const float (&x)[8],
                                       typename Piece<base_of<PREC>()>::vec (&p)[3]) {
  constexpr int B = base_of<PREC>(), NPC = mfma_pieces(PREC);
  constexpr float up = (float)(1 << mfma_piece_shift(PREC));
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    float r = x[t];
#pragma unroll
    for (int q = 0; q < NPC; ++q) {
      const auto h = Piece<B>::cvt(r);
      p[q][t] = h;
      // (r - h) * up, exact: the remainder has <= 24 - width bits and the
      // scale is a power of two.  As one fused multiply-add of the scaled
      // value, the conversion of an FP16 piece folds into a mixed-precision
      // FMA (one instruction fewer per piece).
      if (q + 1 < NPC) r = __builtin_fmaf(-Piece<B>::back(h), up, r * up);
    }
  }
}

// FP16 pieces have a 5-bit exponent: above 65504 they overflow, below 2^-14
// they lose bits, and a line's values can have any magnitude (the inputs of a
// four-step's second pass are up to 256 times the signal's).  The FP16 forms
// therefore scale each 256-point line by an exact power of two 2^-e that
// brings its largest magnitude into [1/2, 1) before stage 1, so stage 1's
// inputs are at most 1 and stage 2's (sums of 16 products with |w| <= 1)
// at most 16, and scale the FP32 results back by 2^e when they leave the
// registers.  Both scalings are exact, the pieces of every value at least
// 2^-35 times the line's largest stay exact to the form's precision, and the
// error stays relative to the line's own magnitude whatever the input range.
// BF16 pieces share FP32's exponent range and need no scaling.
//
// e is the exponent of the largest magnitude among the wave's 512 values (its
// line: the wave holds one line's B operand), the same in every lane: the
// largest of a lane's eight, then within each row of 16 lanes through DPP
// moves, then across the four rows through scalar reads.  Magnitudes are
// compared as their bit patterns (non-negative floats order like unsigned
// integers).
__device__ __forceinline__ uint32_t dpp_max(uint32_t m, int ctrl_id) {
  int v;
  switch (ctrl_id) {
    case 0: v = __builtin_amdgcn_mov_dpp((int)m, 0xB1, 0xF, 0xF, false); break;   // quad_perm 1,0,3,2
    case 1: v = __builtin_amdgcn_mov_dpp((int)m, 0x4E, 0xF, 0xF, false); break;   // quad_perm 2,3,0,1
    case 2: v = __builtin_amdgcn_mov_dpp((int)m, 0x141, 0xF, 0xF, false); break;  // row_half_mirror
    default: v = __builtin_amdgcn_mov_dpp((int)m, 0x140, 0xF, 0xF, false); break; // row_mirror
  }
  return m > (uint32_t)v ? m : (uint32_t)v;
}
__device__ __forceinline__ int line_exponent(const float (&x)[8]) {
  uint32_t m = 0;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const uint32_t b = __float_as_uint(x[t]) & 0x7fffffffu;
    m = m > b ? m : b;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) m = dpp_max(m, k);
  uint32_t r = (uint32_t)__builtin_amdgcn_readlane((int)m, 0);
#pragma unroll
  for (int row = 1; row < 4; ++row) {
    const uint32_t q = (uint32_t)__builtin_amdgcn_readlane((int)m, 16 * row);
    r = r > q ? r : q;
  }
  // frexp's exponent: m = f 2^e with f in [1/2, 1) (r = 0: no scaling)
  return r ? (int)(r >> 23) - 126 : 0;
}

// One DFT-16 stage: D = W X for the 16 vectors held in B layout.
template <int PREC>
__device__ __forceinline__ void dft16_stage(const typename Piece<base_of<PREC>()>::vec (&are)[3],
                                            const typename Piece<base_of<PREC>()>::vec (&aim)[3],
                                            const float (&xv)[8], f32x4 &dre, f32x4 &dim) {
  constexpr int B = base_of<PREC>(), NPC = mfma_pieces(PREC);
  constexpr float down = 1.0f / (float)(1 << mfma_piece_shift(PREC));
  typename Piece<B>::vec xp[3];
  split8<PREC>(xv, xp);
  const f32x4 z = {0.f, 0.f, 0.f, 0.f};
  f32x4 r0 = mfma<B>(are[0], xp[0], z);
  f32x4 i0 = mfma<B>(aim[0], xp[0], z);
  if constexpr (NPC >= 2) {
    f32x4 r1 = mfma<B>(are[0], xp[1], z);
    r1 = mfma<B>(are[1], xp[0], r1);
    f32x4 i1 = mfma<B>(aim[0], xp[1], z);
    i1 = mfma<B>(aim[1], xp[0], i1);
    if constexpr (NPC == 3) {
      f32x4 r2 = mfma<B>(are[0], xp[2], z);
      r2 = mfma<B>(are[1], xp[1], r2);
      r2 = mfma<B>(are[2], xp[0], r2);
      f32x4 i2 = mfma<B>(aim[0], xp[2], z);
      i2 = mfma<B>(aim[1], xp[1], i2);
      i2 = mfma<B>(aim[2], xp[0], i2);
      r1 = r1 + r2 * down;
      i1 = i1 + i2 * down;
    }
    r0 = r0 + r1 * down;
    i0 = i0 + i1 * down;
  }
  dre = r0;
  dim = i0;
}

}  // namespace

// C = 16 lines of 256 points per workgroup of 256 threads (4 waves, 4 lines
// each).  The tile is loaded coalesced into LDS, each wave runs the two MFMA
// stages of its lines, and the tile is stored coalesced.  The stage-1 result
// reaches the B layout of stage 2 through the line's own LDS region: a wave
// alone owns its lines, and an MFMA issues only once every lane's operands
// (the reads of the whole line) are in registers, so its results may
// overwrite the line.  Without a scratch buffer beside the tile four
// workgroups fit a CU instead of three: plain forms 4% faster, two-piece
// forms 1%, the three-piece form 2%.
template <int PREC, int MAP, int OMAP, bool TW4, int SW>
__global__ void __launch_bounds__(kMfmaThreads) k_mfma256(const cf *__restrict__ in,
                                                          cf *__restrict__ out, MfmaArgs a) {
  constexpr int B = base_of<PREC>(), NPC = mfma_pieces(PREC);
  constexpr int C = kMfmaLines;
  constexpr bool SCALED = B == MP_FP16;  // per-line power-of-two scaling
  __shared__ cf tile[C * kPitch];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t tileid = !(a.flags & F_REMAP)  ? blockIdx.x
                          : (a.flags & F_ROUNDS) ? xcd_remap_rounds(blockIdx.x, gridDim.x, (a.flags & F_ROUNDS16) ? 4 : 5)
                                                 : xcd_remap(blockIdx.x, gridDim.x);
  const int64_t bb = tileid / a.tiles_per_batch;
  const int64_t line0 = (tileid - bb * a.tiles_per_batch) * C;

  // A operands (DFT-16 matrix pieces) for this lane
  typename Piece<B>::vec are[3], aim[3];
#pragma unroll
  for (int q = 0; q < NPC; ++q) {
    const uint4 ur = *reinterpret_cast<const uint4 *>(a.amat + ((q * 2 + 0) * 64 + lane) * 8);
    const uint4 ui = *reinterpret_cast<const uint4 *>(a.amat + ((q * 2 + 1) * 64 + lane) * 8);
    are[q] = __builtin_bit_cast(typename Piece<B>::vec, ur);
    aim[q] = __builtin_bit_cast(typename Piece<B>::vec, ui);
  }
  const int col = lane & 15, g4 = lane >> 4;
  // inter-stage twiddles w_256^{n2 k1} for n2 = col, k1 = 4 g4 + t
  cf tw[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) tw[t] = a.tw16[(4 * g4 + t) * 16 + col];

  // four-step twiddle bases of the wave's lines l = l0 + u (u < C/4):
  // A_u = w_N^{l (col + 64 g4)} and S_u = w_N^{16 l}, multiplied out where
  // they are used.  Only the first line's bases are looked up; the others
  // follow as A_u = A_{u-1} D and S_u = S_{u-1} G with D = w_N^{col + 64 g4}
  // and G = w_N^{16} (at most three products each), so a lane reads two
  // scattered table pairs per tile instead of one per line.  The table
  // entries are loaded ahead of the tile, so they arrive with it.
  cf tw4e[8];  // A0 hi/lo, D hi/lo, S0 hi/lo, G hi/lo
  if constexpr (TW4) {
    const uint32_t m = (1u << a.tw4_shift) - 1u;
    const uint32_t l0 = (uint32_t)(line0 + wave * (C / 4));
    const uint32_t e[4] = {l0 * (uint32_t)(col + 64 * g4), (uint32_t)(col + 64 * g4), l0 * 16u, 16u};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      tw4e[2 * q] = a.tw4_hi[e[q] >> a.tw4_shift];
      tw4e[2 * q + 1] = a.tw4_lo[e[q] & m];
    }
  }

  // ---- load the tile (C lines x 256) coalesced, into LDS ----
  {
    const int c = MAP == ELEM_FAST ? tid >> 4 : tid & 15;
    const int j = MAP == ELEM_FAST ? tid & 15 : tid >> 4;
    const int64_t line = line0 + c;
    if (line < a.lines) {
      // per-line base, 32-bit element offsets (at most 255 x 256 elements)
      const cf *src = in + bb * a.in_b + line * a.in_l;
      const uint32_t es = (uint32_t)a.in_e;
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        cf v = ld_stream(src + (uint32_t)(j + 16 * m) * es);
        if (SW & 1) v = cswap(v);
        tile[tidx(c, j + 16 * m)] = v;
      }
    } else {
#pragma unroll
      for (int m = 0; m < 16; ++m) tile[tidx(c, j + 16 * m)] = make_float2(0.f, 0.f);
    }
  }
  __syncthreads();

  const int part = g4 >> 1, kb = 8 * (g4 & 1);
  cf A, S, Dw, Gw;  // bases of the current line and their steps
  if constexpr (TW4) {
    A = cmul(tw4e[0], tw4e[1]);
    Dw = cmul(tw4e[2], tw4e[3]);
    S = cmul(tw4e[4], tw4e[5]);
    Gw = cmul(tw4e[6], tw4e[7]);
  }
#pragma unroll
  for (int u = 0; u < C / 4; ++u) {
    const int c = wave * (C / 4) + u;
    // stage 1: vector n2 = col, element n1 = kb + t: x[n2 + 16 n1]
    float xv[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const cf v = tile[tidx(c, col + 16 * (kb + t))];
      xv[t] = part ? v.y : v.x;
    }
    int ex = 0;  // the line's scale 2^-ex (FP16 forms)
    if constexpr (SCALED) {
      ex = line_exponent(xv);
#pragma unroll
      for (int t = 0; t < 8; ++t) xv[t] = __builtin_amdgcn_ldexpf(xv[t], -ex);
    }
    f32x4 dre, dim;
    dft16_stage<PREC>(are, aim, xv, dre, dim);
    // D: column n2 = col, rows k1 = 4 g4 + t -> twiddle, to Y[k1][n2] at
    // position 16 k1 + n2 of the line (pitch 17 per k1 row)
    cf *scr = tile + c * kPitch;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const cf y = cmul(make_float2(dre[t], dim[t]), tw[t]);
      scr[(4 * g4 + t) * 17 + col] = y;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // stage 2: vector k1 = col, element n2 = kb + t
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const cf v = scr[col * 17 + kb + t];
      xv[t] = part ? v.y : v.x;
    }
    dft16_stage<PREC>(are, aim, xv, dre, dim);
    // D: column k1 = col, rows k2 = 4 g4 + t -> X[k1 + 16 k2] back into the line
    const int64_t line = line0 + c;
    cf y4[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) y4[t] = make_float2(dre[t], dim[t]);
    // the line's scale 2^ex goes back in with the four-step twiddle, or with
    // the inverse's 1/N, or on its own
    if constexpr (TW4) {
      // w_N^{line k}, k = col + 16 (4 g4 + t) = A S^t
      const cf S2 = cmul(S, S);
      cf As = A;
      if constexpr (SCALED) As = make_float2(__builtin_amdgcn_ldexpf(A.x, ex), __builtin_amdgcn_ldexpf(A.y, ex));
      y4[0] = cmul(y4[0], As);
      y4[1] = cmul(y4[1], cmul(As, S));
      y4[2] = cmul(y4[2], cmul(As, S2));
      y4[3] = cmul(y4[3], cmul(As, cmul(S2, S)));
      A = cmul(A, Dw);  // the next line's bases
      S = cmul(S, Gw);
    } else if constexpr (SCALED && !(SW & 2)) {
#pragma unroll
      for (int t = 0; t < 4; ++t)
        y4[t] = make_float2(__builtin_amdgcn_ldexpf(y4[t].x, ex), __builtin_amdgcn_ldexpf(y4[t].y, ex));
    }
    const float osc = (SCALED && !TW4) ? __builtin_amdgcn_ldexpf(a.scale, ex) : a.scale;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      cf y = y4[t];
      if (SW & 2) y = cswap(cscale(y, osc));
      tile[tidx(c, col + 16 * (4 * g4 + t))] = y;
    }
  }
  __syncthreads();

  // ---- store the tile coalesced in the output layout ----
  {
    const int c = OMAP == ELEM_FAST ? tid >> 4 : tid & 15;
    const int j = OMAP == ELEM_FAST ? tid & 15 : tid >> 4;
    const int64_t line = line0 + c;
    if (line < a.lines) {
      cf *dst = out + bb * a.out_b + line * a.out_l;
      const uint32_t es = (uint32_t)a.out_e;
#pragma unroll
      for (int m = 0; m < 16; ++m) st_stream(dst + (uint32_t)(j + 16 * m) * es, tile[tidx(c, j + 16 * m)]);
    }
  }
}

int mfma_lds_bytes(int) { return (int)sizeof(cf) * kMfmaLines * kPitch; }

const void *mfma_kernel(int prec, int map, int omap, bool tw4, int sw) {
#define MK2(P)                                                                                 \
  if (prec == P) {                                                                             \
    if (map == LINE_FAST && omap == LINE_FAST && tw4 && sw == 0)                               \
      return (const void *)&k_mfma256<P, LINE_FAST, LINE_FAST, true, 0>;                       \
    if (map == LINE_FAST && omap == LINE_FAST && tw4 && sw == 1)                               \
      return (const void *)&k_mfma256<P, LINE_FAST, LINE_FAST, true, 1>;                       \
    if (map == ELEM_FAST && omap == LINE_FAST && !tw4 && sw == 0)                              \
      return (const void *)&k_mfma256<P, ELEM_FAST, LINE_FAST, false, 0>;                      \
    if (map == ELEM_FAST && omap == LINE_FAST && !tw4 && sw == 2)                              \
      return (const void *)&k_mfma256<P, ELEM_FAST, LINE_FAST, false, 2>;                      \
    if (map == ELEM_FAST && omap == ELEM_FAST && !tw4 && sw == 0)                              \
      return (const void *)&k_mfma256<P, ELEM_FAST, ELEM_FAST, false, 0>;                      \
    if (map == ELEM_FAST && omap == ELEM_FAST && !tw4 && sw == 3)                              \
      return (const void *)&k_mfma256<P, ELEM_FAST, ELEM_FAST, false, 3>;                      \
  }
  MK2(MP_FP16)
  MK2(MP_BF16)
  MK2(MP_FP16_SPLIT)
  MK2(MP_BF16_SPLIT)
  MK2(MP_BF16_SPLIT3)
#undef MK2
  return nullptr;
}

}  // namespace dpfft
