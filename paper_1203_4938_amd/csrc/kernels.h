// Host-visible descriptions of the device kernels: argument blocks and the
// registry that maps a kernel shape to its compiled instance.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpfft {

// Lane-to-data mapping of a line kernel.  ELEM_FAST: consecutive lanes walk
// along a line (rows, contiguous signals).  LINE_FAST: consecutive lanes walk
// across lines (column tiles of a row-major matrix).
enum : int { ELEM_FAST = 0, LINE_FAST = 1 };

enum : uint32_t {
  F_REMAP = 4u,     // XCD-aware workgroup -> tile order
  F_ROUNDS = 8u,    // with F_REMAP: the order in rounds of 256 tiles (xcd_remap_rounds)
  F_ROUNDS16 = 16u, // with F_ROUNDS: rounds of 128 tiles, 16 per XCD
};

// One launch of a line kernel: length-L transforms of `lines` lines per batch
// item; element (batch b, line l, index i) lives at
//   base + b*x_b + l*x_l + i*x_e   (in complex elements).
struct LineArgs {
  int64_t in_b, in_l, in_e;
  int64_t out_b, out_l, out_e;
  int64_t lines;           // lines per batch item
  int64_t tiles_per_batch; // ceil(lines / C)
  const float2 *tw;        // Stockham pass twiddles for length L
  const float2 *tw4_lo;    // four-step twiddles w_N^l, l < 2^tw4_shift
  const float2 *tw4_hi;    // four-step twiddles w_N^{h 2^tw4_shift}
  int32_t tw4_shift;
  float scale;             // applied to every output (1 or 1/N)
  uint32_t flags;
  const float2 *tw2;       // two-level pass table of w_L: 2^S lo entries, then L/2^S hi
  int64_t ntiles;          // tiles in the launch (persistent kernels loop over them)
};

// Radix plan of the power-of-two line kernels, shared by the device code and
// the host twiddle generator.  E elements per thread (EPT, or L if smaller;
// a multiple of every radix), T threads per line.  The main radix is EPT
// (16 or 32), followed by one smaller power-of-two remainder pass.
template <int L, int EPT = 16> struct P2 {
  static constexpr int lg() {
    int k = 0;
    while ((1 << k) < L) ++k;
    return k;
  }
  static constexpr int LG = lg();
  static constexpr int RB = EPT >= 32 ? 5 : EPT >= 16 ? 4 : 3;  // log2 of the main radix
  static constexpr int E = L >= EPT ? EPT : L;
  static constexpr int T = L / E;
  static constexpr int NP = (LG + RB - 1) / RB;
  static constexpr int radix(int p) { return (p < LG / RB) ? (1 << RB) : (1 << (LG % RB)); }
  static constexpr int ns(int p) {
    int s = 1;
    for (int i = 0; i < p; ++i) s *= radix(i);
    return s;
  }
  static constexpr int twoff(int p) {
    int o = 0;
    for (int i = 1; i < p; ++i) o += ns(i) * (radix(i) - 1);
    return o;
  }
};

// Split of the two-level pass-twiddle table of a length-L kernel: w_L^e =
// hi[e >> S] * lo[e & (2^S - 1)] with 2^S lo and L / 2^S hi entries.
constexpr int tw2_shift(int lg) { return (lg + 1) / 2; }

// Runtime twin of P2<L, EPT> for the host.
inline int pow2_rb(int ept) { return ept >= 32 ? 5 : ept >= 16 ? 4 : 3; }
inline int pow2_radix(int L, int p, int ept = 16) {
  int lg = 0;
  while ((1 << lg) < L) ++lg;
  const int rb = pow2_rb(ept);
  return (p < lg / rb) ? (1 << rb) : (1 << (lg % rb));
}
inline int pow2_passes(int L, int ept = 16) {
  int lg = 0;
  while ((1 << lg) < L) ++lg;
  const int rb = pow2_rb(ept);
  return (lg + rb - 1) / rb;
}

struct KernelInfo {
  const void *fn = nullptr;          // forward instance
  const void *fn_sw[4] = {};         // by swap mode: 1 = on load, 2 = on store, 3 = both
  int threads = 0;      // workgroup size
  int lines = 0;        // lines per workgroup (C)
  int lds_bytes = 0;    // static LDS of the instance
  int map = 0, omap = 0;
  bool persistent = false;  // loops over tiles; launch at most one grid of resident workgroups
  bool preferred = false;   // the planner's default for its shape (measured fastest)
  int ept = 16;             // elements per thread (sets the radix plan of the pass table)
  int sub = 1;              // sub-lines per line: 2 for the split-first instances, whose
                            // pass table is that of L / 2
};

// Power-of-two line kernels have compile-time length L and C lines per
// workgroup; tw4 = apply the four-step twiddle w_N^{line*i} before the store.
// All compiled instances for (L, map, omap, tw4); returns how many exist and
// fills up to `max` of them.
int list_line_kernels(int L, int map, int omap, bool tw4, KernelInfo *out, int max);

// Digest of the compiled line-kernel registry (shapes, tiles, variants): part
// of the tuning-cache key, so entries written by a build with other kernels
// are not applied.
uint64_t line_registry_digest();

}  // namespace dpfft
