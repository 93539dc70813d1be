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
#include "mixed_device.h"

namespace dpfft {

template <int MAP, int OMAP, bool TW4, int SW>
__global__ void __launch_bounds__(1024) k_mixed(const cf *__restrict__ in, cf *__restrict__ out,
                                                MixedArgs a) {
  extern __shared__ cf lds[];
  const MixedPlan &mp = a.mp;
  const int tid = threadIdx.x;
  const uint32_t tile = (a.flags & F_REMAP) ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
  const int64_t bb = tile / a.tiles_per_batch;
  const int64_t line0 = (int64_t)(tile - bb * a.tiles_per_batch) * mp.C;
  LineShape sh{mp.L, mp.T, mp.C, mp.pitch, mp.P, mp.tw2_shift, mp.codes, a.tw2,
               a.tw4_lo, a.tw4_hi, a.tw4_shift, a.scale, mp.tw_lds};
  TileLine t;
  t.c = MAP == ELEM_FAST ? tid / mp.T : tid % mp.C;
  t.j = MAP == ELEM_FAST ? tid % mp.T : tid / mp.C;
  t.line = line0 + t.c;
  t.valid = tid < mp.C * mp.T && t.line < a.lines;
  t.src = in + bb * a.in_b + t.line * a.in_l;
  t.dst = out + bb * a.out_b + t.line * a.out_l;
  t.in_e = a.in_e;
  t.out_e = a.out_e;
  t.c2 = OMAP == ELEM_FAST ? tid / mp.T : tid % mp.C;
  t.j2 = OMAP == ELEM_FAST ? tid % mp.T : tid / mp.C;
  t.valid2 = tid < mp.C * mp.T && line0 + t.c2 < a.lines;
  t.dst2 = out + bb * a.out_b + (line0 + t.c2) * a.out_l;
  mixed_tile<MAP, OMAP, TW4, SW>(sh, t, lds, mp.C * mp.T);
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
bool mixed_radices(int64_t L, MixedPlan *mp, int order) {
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
  auto push_odd = [&]() {
    for (int p : {7, 5})
      for (int i = 0; i < cnt[p]; ++i)
        if (!push(p)) return false;
    // pairs of 3s as radix-9 passes (3 x 3 in registers): one LDS exchange
    // fewer per pair
    for (int i = 0; i < cnt[3] / 2; ++i)
      if (!push(9)) return false;
    if (cnt[3] % 2 && !push(3)) return false;
    return true;
  };
  if (order == 1 && !push_odd()) return false;
  int twos = cnt[2];
  while (twos >= 4) {
    if (!push(16)) return false;
    twos -= 4;
  }
  if (twos == 3 && !push(8)) return false;
  if (twos == 2 && !push(4)) return false;
  if (twos == 1 && !push(2)) return false;
  if (order != 1 && !push_odd()) return false;
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

int mixed_tile_elems(const MixedPlan &mp, int map, int omap) {
  auto need = [&](int m) {
    if (m == ELEM_FAST) return (int64_t)mp.C * mp.pitch;
    const int64_t u = (int64_t)mp.L * mp.C;
    return u + (u >> 4) + 1;
  };
  int64_t n = need(map);
  if (omap != map) n = n > need(omap) ? n : need(omap);
  return (int)n;
}

int mixed_lds_bytes(const MixedPlan &mp, int map, int omap) {
  return (mixed_tile_elems(mp, map, omap) + tw2_entries(mp.L, mp.tw2_shift)) * (int)sizeof(cf);
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
  MK(LINE_FAST, LINE_FAST, false, 3)
  MK(LINE_FAST, LINE_FAST, true, 0)
  MK(LINE_FAST, LINE_FAST, true, 1)
  // four-step second pass: rows stored transposed (fwd, swap out)
  MK(ELEM_FAST, LINE_FAST, false, 0)
  MK(ELEM_FAST, LINE_FAST, false, 2)
#undef MK
  return nullptr;
}

}  // namespace dpfft
