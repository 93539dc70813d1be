// Persistent ragged-batch kernel.
//
// A launch of resident workgroups; each workgroup repeatedly takes a ticket
// from a device counter and runs the work item the ticket names (largest
// items first), until its queue is empty.  Signals too long for one
// workgroup are split into column-pass and row-pass tiles of a four-step
// transform.  The row tiles of a signal need every column tile of it, and
// publishing data from one workgroup to another inside a launch would take an
// agent-scope fence per tile (a write-back of the XCD's whole L2 on this
// chip), so the batch runs as two such launches back to back: the first
// drains the queue of single-pass items and column tiles, the second the
// queue of row tiles.  The kernel boundary orders them; nothing ever waits.
//
// In direct mode the kernel runs item first_item + blockIdx.x with no queue;
// the per-length baseline launches it once per distinct length.
#include "mixed_device.h"
#include "ragged.h"

namespace dpfft {

__global__ void k_ragged_reset(uint32_t *state, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    state[i] = 0u;
}

template <bool INV>
__global__ void __launch_bounds__(kRaggedThreads) k_ragged(const cf *__restrict__ in, cf *__restrict__ out,
                                                 RaggedArgs a) {
  extern __shared__ cf lds[];
  __shared__ int s_item;
  const int tid = threadIdx.x;
  for (int round = 0;; ++round) {
    int item;
    if (a.direct) {
      if (round > 0) break;
      item = a.first_item + (int)blockIdx.x;
    } else {
      if (tid == 0)
        s_item = (int)__hip_atomic_fetch_add(&a.state[a.ticket], 1u, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
      item = s_item;
      __syncthreads();
      if (item >= a.nitems) break;
      item = a.order[item];
    }
    const RaggedItem d = a.items[item];
    const RaggedSize z = a.sizes[d.size];
    LineShape sh{z.L, z.T, d.C, z.pitch, z.P, z.tw2_shift, z.codes, a.tables + z.tw2_off,
                 nullptr, nullptr, 0, 1.0f, d.tw_lds};
    TileLine t;
    const bool in_tile = tid < d.C * z.T;

    if (d.kind == RK_SINGLE) {
      t.c = tid / z.T;
      t.j = tid % z.T;
      t.valid = in_tile;
      const int64_t off = in_tile ? a.offsets[a.siglist[d.sig + t.c]] : 0;
      t.src = in + off;
      t.dst = out + off;
      t.in_e = t.out_e = 1;
      t.line = 0;
      t.valid2 = false;
      sh.scale = 1.0f / (float)z.L;
      mixed_tile<ELEM_FAST, ELEM_FAST, false, INV ? 3 : 0>(sh, t, lds, kRaggedThreads);
    } else if (d.kind == RK_COLUMNS) {
      const RaggedBig bg = a.bigs[d.big];
      sh.tw4_lo = a.tables + bg.tw4_lo_off;
      sh.tw4_hi = a.tables + bg.tw4_hi_off;
      sh.tw4_shift = bg.tw4_shift;
      t.c = tid % d.C;
      t.j = tid / d.C;
      t.valid = in_tile;
      const int64_t n2 = d.first + t.c;
      t.src = in + a.offsets[d.sig] + n2;
      t.dst = a.ws + bg.ws_off + n2;
      t.in_e = t.out_e = d.n2;
      t.line = n2;
      t.valid2 = false;
      mixed_tile<LINE_FAST, LINE_FAST, true, INV ? 1 : 0>(sh, t, lds, kRaggedThreads);
    } else {
      const RaggedBig bg = a.bigs[d.big];
      t.c = tid / z.T;
      t.j = tid % z.T;
      t.valid = in_tile;
      const int64_t k1 = d.first + t.c;
      t.src = a.ws + bg.ws_off + k1 * d.n2;
      t.dst = nullptr;
      t.in_e = 1;
      t.out_e = d.n1;
      t.line = k1;
      t.c2 = tid % d.C;
      t.j2 = tid / d.C;
      t.valid2 = in_tile;
      t.dst2 = out + a.offsets[d.sig] + d.first + t.c2;
      sh.scale = (float)(1.0 / ((double)d.n1 * (double)d.n2));
      mixed_tile<ELEM_FAST, LINE_FAST, false, INV ? 2 : 0>(sh, t, lds, kRaggedThreads);
    }
    __syncthreads();  // the next item reuses the LDS
  }
}

const void *ragged_kernel(bool inverse) {
  return inverse ? (const void *)&k_ragged<true> : (const void *)&k_ragged<false>;
}
const void *ragged_reset_kernel() { return (const void *)&k_ragged_reset; }

}  // namespace dpfft
