// Runtime-radix Stockham line kernels (any 7-smooth length that fits LDS).
//
// Same data decomposition as the power-of-two kernels -- a workgroup owns C
// lines, T threads per line, passes in Stockham autosort order -- but the
// radix sequence is read at run time, so one compiled instance serves every
// length (the ragged batches use hundreds of them).  Because the element sets
// of consecutive passes differ when the radix changes, every pass reads its
// inputs from LDS (the first pass from HBM) and writes its outputs back to LDS
// (the last pass to HBM), in place, with a barrier between the reads and the
// writes.  Pass twiddles w_{Ns R}^{k r} = w_L^{k r L/(Ns R)} are rebuilt from a
// two-level table of w_L made in FP64 on the host.
#include "fft_common.h"
#include "kernels.h"
#include "mixed.h"

namespace dpfft {

namespace {

__device__ __forceinline__ int midx_elem(int pitch, int c, int pos) {
  return c * pitch + pos + (pos >> 4);
}
__device__ __forceinline__ int midx_line(int C, int c, int pos) {
  const int u = pos * C + c;
  return u + (u >> 4);
}

__device__ __forceinline__ cf tw2_lookup(const cf *__restrict__ t, int shift, uint32_t e) {
  const cf lo = t[e & ((1u << shift) - 1u)];
  const cf hi = t[(1u << shift) + (e >> shift)];
  return cmul(hi, lo);
}

__device__ __forceinline__ cf tw4_lookup_m(const MixedArgs &a, uint32_t e) {
  const uint32_t lo = e & ((1u << a.tw4_shift) - 1u);
  const uint32_t hi = e >> a.tw4_shift;
  return cmul(a.tw4_hi[hi], a.tw4_lo[lo]);
}

}  // namespace

// Per-thread and per-line context of a pass, as plain scalars: the pass is a
// separate (non-inlined) function per radix so that each gets its own
// register allocation, and scalars travel in registers rather than through
// the stack.
struct PassArgs {
  int L, T, C, pitch, NS, tw2_shift, tw4_shift, c, j;
  bool valid, first, last;
  int64_t in_e, out_e, line;
  float scale;
};

template <int MAP, int OMAP, bool TW4, int SW, int R>
__device__ __noinline__ void mixed_pass(const cf *__restrict__ src, cf *__restrict__ dst,
                                        cf *lds, const cf *__restrict__ tw2,
                                        const cf *__restrict__ tw4_lo,
                                        const cf *__restrict__ tw4_hi, int L, int T, int C,
                                        int pitch, int NS, int tw2_shift, int tw4_shift, int c,
                                        int j, bool valid, bool first, bool last, int64_t in_e,
                                        int64_t out_e, int64_t line, float scale) {
  const int M = L / R;
  constexpr int QM = (16 + R - 1) / R;  // butterflies per thread (T >= L/16)
  auto li = [&](int m, int pos) {
    return m == ELEM_FAST ? midx_elem(pitch, c, pos) : midx_line(C, c, pos);
  };
  cf v[QM][R];
  bool act[QM];
#pragma unroll
  for (int q = 0; q < QM; ++q) {
    const int b = j + T * q;
    act[q] = valid && b < M;
    if (!act[q]) continue;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int pos = b + r * M;
      cf y;
      if (first) {
        y = src[(int64_t)pos * in_e];
        if (SW & 1) y = cswap(y);
      } else {
        y = lds[li(MAP, pos)];
      }
      v[q][r] = y;
    }
    if (NS > 1) {
      const int k = b % NS;
      const uint32_t step = (uint32_t)(L / (NS * R));
#pragma unroll
      for (int r = 1; r < R; ++r)
        v[q][r] = cmul(v[q][r], tw2_lookup(tw2, tw2_shift, (uint32_t)(k * r) * step));
    }
    Dft<R>::run(v[q]);
  }
  if (!first) __syncthreads();  // every read of this pass precedes the in-place writes
#pragma unroll
  for (int q = 0; q < QM; ++q) {
    if (!act[q]) continue;
    const int b = j + T * q;
    const int k = b % NS;
    const int base = (b - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int pos = base + r * NS;
      cf y = v[q][r];
      if (last) {
        if (TW4) {
          const uint32_t e = (uint32_t)(line * pos);
          y = cmul(y, cmul(tw4_hi[e >> tw4_shift], tw4_lo[e & ((1u << tw4_shift) - 1u)]));
        }
        if (SW & 2) y = cswap(cscale(y, scale));
        if (OMAP == MAP) {
          dst[(int64_t)pos * out_e] = y;
          continue;
        }
        lds[li(OMAP, pos)] = y;
      } else {
        lds[li(MAP, pos)] = y;
      }
    }
  }
  if (!last || OMAP != MAP) __syncthreads();
}

template <int MAP, int OMAP, bool TW4, int SW>
__global__ void __launch_bounds__(1024) k_mixed(const cf *__restrict__ in, cf *__restrict__ out,
                                                MixedArgs a) {
  extern __shared__ cf lds[];
  const MixedPlan &mp = a.mp;
  const int tid = threadIdx.x;
  const int c = MAP == ELEM_FAST ? tid / mp.T : tid % mp.C;
  const int j = MAP == ELEM_FAST ? tid % mp.T : tid / mp.C;
  const uint32_t tile = (a.flags & F_REMAP) ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
  const int64_t bb = tile / a.tiles_per_batch;
  const int64_t line0 = (int64_t)(tile - bb * a.tiles_per_batch) * mp.C;
  const int64_t line = line0 + c;
  const bool valid = c < mp.C && line < a.lines;
  const cf *src = in + bb * a.in_b + line * a.in_l;
  cf *dst = out + bb * a.out_b + line * a.out_l;

  int ns = 1;
  for (int p = 0; p < mp.P; ++p) {
    const bool first = p == 0, last = p == mp.P - 1;
    const int R = (int)((mp.codes >> (5 * p)) & 31u);
#define PASS(RR)                                                                              \
  mixed_pass<MAP, OMAP, TW4, SW, RR>(src, dst, lds, a.tw2, a.tw4_lo, a.tw4_hi, mp.L, mp.T, mp.C, \
                                     mp.pitch, ns, mp.tw2_shift, a.tw4_shift, c, j, valid,     \
                                     first, last, a.in_e, a.out_e, line, a.scale)
    switch (R) {
      case 2: PASS(2); break;
      case 3: PASS(3); break;
      case 4: PASS(4); break;
      case 5: PASS(5); break;
      case 7: PASS(7); break;
      case 8: PASS(8); break;
      default: PASS(16); break;
    }
#undef PASS
    ns *= R;
  }
  if (OMAP != MAP) {
    // the last pass left the line in LDS (output layout); store it coalesced
    int c2, j2;
    if (OMAP == ELEM_FAST) {
      c2 = tid / mp.T;
      j2 = tid % mp.T;
    } else {
      c2 = tid % mp.C;
      j2 = tid / mp.C;
    }
    const int64_t line2 = line0 + c2;
    if (c2 < mp.C && line2 < a.lines) {
      cf *dst = out + bb * a.out_b + line2 * a.out_l;
      for (int i = j2; i < mp.L; i += mp.T)
        dst[(int64_t)i * a.out_e] =
            lds[OMAP == ELEM_FAST ? midx_elem(mp.pitch, c2, i) : midx_line(mp.C, c2, i)];
    }
  }
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
bool mixed_radices(int64_t L, MixedPlan *mp) {
  int64_t n = L;
  int np = 0;
  int cnt[17] = {};
  for (int p : {2, 3, 5, 7})
    while (n % p == 0) {
      n /= p;
      cnt[p]++;
    }
  if (n != 1) return false;
  auto push = [&](int r) {
    if (np >= kMaxPasses) return false;
    mp->radix[np++] = r;
    return true;
  };
  int twos = cnt[2];
  while (twos >= 4) {
    if (!push(16)) return false;
    twos -= 4;
  }
  if (twos == 3 && !push(8)) return false;
  if (twos == 2 && !push(4)) return false;
  if (twos == 1 && !push(2)) return false;
  for (int p : {7, 5, 3})
    for (int i = 0; i < cnt[p]; ++i)
      if (!push(p)) return false;
  mp->L = (int32_t)L;
  mp->P = np;
  int ns = 1;
  mp->codes = 0;
  for (int p = 0; p < np; ++p) {
    mp->ns[p] = ns;
    ns *= mp->radix[p];
    mp->codes |= (uint64_t)mp->radix[p] << (5 * p);
  }
  mp->T = (int32_t)((L + 15) / 16);
  int lg = 0;
  while ((int64_t(1) << lg) < L) ++lg;
  mp->tw2_shift = (lg + 1) / 2;
  mp->pitch = (int32_t)(L + (L >> 4) + 1);
  return true;
}

int mixed_lds_bytes(const MixedPlan &mp, int map, int omap) {
  auto need = [&](int m) {
    if (m == ELEM_FAST) return (int64_t)mp.C * mp.pitch;
    const int64_t u = (int64_t)mp.L * mp.C;
    return u + (u >> 4) + 1;
  };
  int64_t n = need(map);
  if (omap != map) n = n > need(omap) ? n : need(omap);
  return (int)(n * (int64_t)sizeof(cf));
}

const void *mixed_kernel(int map, int omap, bool tw4, int sw) {
#define MK(M, O, TW, S) \
  if (map == M && omap == O && tw4 == TW && sw == S) return (const void *)&k_mixed<M, O, TW, S>;
  // single-pass rows: forward, inverse (swap in+out), 2D row pass inverse (swap in)
  MK(ELEM_FAST, ELEM_FAST, false, 0)
  MK(ELEM_FAST, ELEM_FAST, false, 1)
  MK(ELEM_FAST, ELEM_FAST, false, 3)
  // column tiles: 2D column pass (fwd, inv = swap out), four-step first pass (fwd, swap in)
  MK(LINE_FAST, LINE_FAST, false, 0)
  MK(LINE_FAST, LINE_FAST, false, 2)
  MK(LINE_FAST, LINE_FAST, true, 0)
  MK(LINE_FAST, LINE_FAST, true, 1)
  // four-step second pass: rows stored transposed (fwd, swap out)
  MK(ELEM_FAST, LINE_FAST, false, 0)
  MK(ELEM_FAST, LINE_FAST, false, 2)
#undef MK
  return nullptr;
}

}  // namespace dpfft
