// Ragged-batch kernel.
//
// The work items of a ragged batch are self-contained: a group of whole
// single-pass signals, or a column or row tile of a long signal's four-step
// transform.  Each launch covers one list of items, largest first, with one
// workgroup per item dispatched by the hardware (a new workgroup starts as
// soon as one retires); the items are dealt to the XCDs in rounds so that a
// signal's neighbouring tiles run side by side in one L2 (ragged_slot).  The
// row tiles of a signal need every column tile of it, and publishing data
// from one workgroup to another inside a launch would take an agent-scope
// fence per tile (a write-back of the XCD's whole L2 on this chip), so the
// column tiles (with the single-pass signals of 256-thread workgroups) and
// the row tiles are two launches and the kernel boundary orders them.
// Single-pass signals too long for a 256-thread workgroup (up to 16384
// points: 16 elements per thread, 1024 threads, up to 160 KB of LDS) run in a
// third launch with the 1024-thread instance, which needs nothing from the
// other two.
//
// Optionally (persistent mode) a launch of resident workgroups walks its list
// with a static stride (workgroup w runs items w, w + grid, w + 2 grid, ...),
// fetching the descriptor of its next item while it works on the current one.
// The per-length baseline launches the kernel once per distinct length.
#include "mixed_ct.h"
#include "mixed_device.h"
#include "ragged.h"

namespace dpfft {

template <bool INV, int NTH>
__device__ __forceinline__ void ragged_item(const cf *__restrict__ in, cf *__restrict__ out,
                                            const RaggedArgs &a, const RaggedItem &d, cf *lds) {
  const int tid = threadIdx.x;
  LineShape sh{d.L, d.T, d.C, d.pitch, d.P, d.tw2_shift, d.codes, a.tables + d.tw2_off,
               nullptr, nullptr, 0, 1.0f, d.tw_lds};
  TileLine t;
  const bool in_tile = tid < d.C * d.T;

  if (d.kind == RK_SINGLE) {
    t.c = tid / d.T;
    t.j = tid % d.T;
    t.valid = in_tile;
    const int64_t off = in_tile ? a.sigoff[d.off + t.c] : 0;
    t.src = in + off;
    t.dst = out + off;
    t.in_e = t.out_e = 1;
    t.line = 0;
    t.valid2 = false;
    sh.scale = 1.0f / (float)d.L;
    mixed_tile<ELEM_FAST, ELEM_FAST, false, INV ? 3 : 0>(sh, t, lds, NTH);
  } else if (d.kind == RK_COLUMNS) {
    if constexpr (NTH == kRaggedThreads) {
      if (d.ct) {
        CtArgs ca{};
        ca.C = d.C;
        ca.c = tid % d.C;
        ca.j = tid / d.C;
        ca.valid = in_tile;
        const int64_t n2 = d.first + ca.c;
        ca.src = as_glb(in + d.off + n2);
        ca.dst = as_glb(a.ws + d.ws_off + n2);
        ca.in_e = ca.out_e = (uint32_t)d.n2;
        ca.line = (uint32_t)n2;
        ca.tw4_lo = as_glb(a.tables + d.tw4_lo_off);
        ca.tw4_hi = as_glb(a.tables + d.tw4_hi_off);
        ca.tw4_shift = d.tw4_shift;
        ca.scale = 1.0f;
        lcf *l = as_lds(lds);
        switch (d.L) {
#define CT_COL(LL)                                                                              \
  case LL:                                                                                      \
    ct_tile<LL, LINE_FAST, LINE_FAST, true, INV ? 1 : 0>(                                      \
        ca.src, ca.dst, ca.dst2, ca.tw4_lo, ca.tw4_hi, ca.tw4_shift, ca.C, ca.c, ca.j, ca.c2,   \
        ca.j2, ca.valid, ca.valid2, ca.in_e, ca.out_e, ca.line, ca.scale, l, l + d.tw_lds,     \
        as_glb(a.tables + d.tw2_off), NTH);                                                    \
    return;
          DPFFT_CT_LENGTHS(CT_COL)
#undef CT_COL
        }
      }
    }
    sh.tw4_lo = a.tables + d.tw4_lo_off;
    sh.tw4_hi = a.tables + d.tw4_hi_off;
    sh.tw4_shift = d.tw4_shift;
    t.c = tid % d.C;
    t.j = tid / d.C;
    t.valid = in_tile;
    const int64_t n2 = d.first + t.c;
    t.src = in + d.off + n2;
    t.dst = a.ws + d.ws_off + n2;
    t.in_e = t.out_e = d.n2;
    t.line = n2;
    t.valid2 = false;
    mixed_tile<LINE_FAST, LINE_FAST, true, INV ? 1 : 0>(sh, t, lds, NTH);
  } else {
    if constexpr (NTH == kRaggedThreads) {
      if (d.ct) {
        CtArgs ca{};
        ca.C = d.C;
        ca.c = tid / d.T;
        ca.j = tid % d.T;
        ca.valid = in_tile;
        const int64_t k1 = d.first + ca.c;
        ca.src = as_glb(a.ws + d.ws_off + k1 * d.n2);
        ca.in_e = 1;
        ca.out_e = (uint32_t)d.n1;
        ca.line = (uint32_t)k1;
        ca.c2 = tid % d.C;
        ca.j2 = tid / d.C;
        ca.valid2 = in_tile;
        ca.dst2 = as_glb(out + d.off + d.first + ca.c2);
        ca.scale = (float)(1.0 / ((double)d.n1 * (double)d.n2));
        lcf *l = as_lds(lds);
        switch (d.L) {
#define CT_ROW(LL)                                                                             \
  case LL:                                                                                     \
    ct_tile<LL, ELEM_FAST, LINE_FAST, false, INV ? 2 : 0>(                                    \
        ca.src, ca.dst, ca.dst2, ca.tw4_lo, ca.tw4_hi, ca.tw4_shift, ca.C, ca.c, ca.j, ca.c2, \
        ca.j2, ca.valid, ca.valid2, ca.in_e, ca.out_e, ca.line, ca.scale, l, l + d.tw_lds,   \
        as_glb(a.tables + d.tw2_off), NTH);                                                  \
    return;
          DPFFT_CT_LENGTHS(CT_ROW)
#undef CT_ROW
        }
      }
    }
    t.c = tid / d.T;
    t.j = tid % d.T;
    t.valid = in_tile;
    const int64_t k1 = d.first + t.c;
    t.src = a.ws + d.ws_off + k1 * d.n2;
    t.dst = nullptr;
    t.in_e = 1;
    t.out_e = d.n1;
    t.line = k1;
    t.c2 = tid % d.C;
    t.j2 = tid / d.C;
    t.valid2 = in_tile;
    t.dst2 = out + d.off + d.first + t.c2;
    sh.scale = (float)(1.0 / ((double)d.n1 * (double)d.n2));
    mixed_tile<ELEM_FAST, LINE_FAST, false, INV ? 2 : 0>(sh, t, lds, NTH);
  }
}

// Item of workgroup b in a launch of one workgroup per item.  Neighbouring
// items (the column or row tiles of one signal) read or write row pieces that
// share 128-byte lines, and workgroup ids are dealt round-robin over the 8
// XCDs, each with its own L2: in order, each XCD would fetch every shared
// line for its own piece.  So each round of 8 K ids gives XCD x the K
// consecutive items 8 K r + K x + k (k < K), which run side by side and share
// the lines in one L2; the rounds keep the largest-first order (and so every
// XCD's share of the work) intact.  Ids past the last whole round keep their
// own item.  K = 128 measured 1.3% faster on the 10,000-signal batch than
// K = 32 (K = 16: 1% slower, 64: 0.6% faster, 256: 0.2% faster).
__device__ __forceinline__ uint32_t ragged_slot(uint32_t b, uint32_t n) {
  constexpr uint32_t X = 8, K = 128;
  const uint32_t full = n / (X * K) * (X * K);
  if (b >= full) return b;
  const uint32_t x = b % X, p = b / X;
  return (p / K) * (X * K) + x * K + p % K;
}

// The buffers are separate restrict-qualified parameters so the compiler knows
// no store of the kernel reaches the item list, and reads the (uniform)
// descriptors through the scalar cache.
template <bool INV, int NTH>
__global__ void __launch_bounds__(NTH, NTH == kRaggedThreads ? 4 : 1)
    k_ragged(const cf *__restrict__ in, cf *__restrict__ out, cf *__restrict__ ws,
             const RaggedItem *__restrict__ item_list, const int64_t *__restrict__ sigoff,
             const cf *__restrict__ tables, RaggedArgs a) {
  extern __shared__ cf lds[];
  a.ws = ws;
  a.sigoff = sigoff;
  a.tables = tables;
  const RaggedItem *__restrict__ items = item_list + a.first_item;
  if (a.direct) {
    ragged_item<INV, NTH>(in, out, a, items[ragged_slot(blockIdx.x, gridDim.x)], lds);
    return;
  }
  // walk q = blockIdx.x, + gridDim.x, ...: with a grid that is a multiple of
  // 8, workgroup q mod gridDim sits on XCD q mod 8, so the same round mapping
  // as the direct mode keeps neighbouring items on one XCD
  const uint32_t n = (uint32_t)a.nitems;
  const bool remap = gridDim.x % 8u == 0u;
  int q = (int)blockIdx.x;
  if (q >= a.nitems) return;
  RaggedItem d = items[remap ? ragged_slot((uint32_t)q, n) : (uint32_t)q];
  for (;;) {
    const int qn = q + (int)gridDim.x;
    // the next descriptor is in flight while this item runs
    RaggedItem dn = d;
    if (qn < a.nitems) dn = items[remap ? ragged_slot((uint32_t)qn, n) : (uint32_t)qn];
    ragged_item<INV, NTH>(in, out, a, d, lds);
    if (qn >= a.nitems) break;
    __syncthreads();  // the next item reuses the LDS
    d = dn;
    q = qn;
  }
}

const void *ragged_kernel(bool inverse, bool big) {
  if (big)
    return inverse ? (const void *)&k_ragged<true, kRaggedBigThreads>
                   : (const void *)&k_ragged<false, kRaggedBigThreads>;
  return inverse ? (const void *)&k_ragged<true, kRaggedThreads>
                 : (const void *)&k_ragged<false, kRaggedThreads>;
}

}  // namespace dpfft
