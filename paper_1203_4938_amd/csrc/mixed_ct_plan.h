// Compile-time radix plans of the line lengths that have compile-time
// ragged instances (host and device).
#pragma once
#include <stdint.h>

namespace dpfft {

// The lengths: every 7-smooth number from 125 to 256 (the four-step line
// lengths of ragged signals of 2^14 to 2^16 points).
#define DPFFT_CT_LENGTHS(X)                                                                     \
  X(125) X(126) X(128) X(135) X(140) X(144) X(147) X(150) X(160) X(162) X(168) X(175) X(180) \
  X(189) X(192) X(196) X(200) X(210) X(216) X(224) X(225) X(240) X(243) X(245) X(250) X(252) \
  X(256)

namespace ctp {
constexpr int count(int L, int p) {
  int c = 0;
  while (L % p == 0) {
    L /= p;
    ++c;
  }
  return c;
}
// the runtime planner's order 0: 16s, then one 8/4/2, then 7s, 5s, pairs of
// 3s as 9s, a last 3
constexpr int radix_at(int L, int i) {
  const int c2 = count(L, 2), c3 = count(L, 3), c5 = count(L, 5), c7 = count(L, 7);
  int n = 0;
  for (int k = 0; k < c2 / 4; ++k, ++n)
    if (n == i) return 16;
  if (c2 % 4) {
    if (n == i) return 1 << (c2 % 4);
    ++n;
  }
  for (int k = 0; k < c7; ++k, ++n)
    if (n == i) return 7;
  for (int k = 0; k < c5; ++k, ++n)
    if (n == i) return 5;
  for (int k = 0; k < c3 / 2; ++k, ++n)
    if (n == i) return 9;
  if (c3 % 2) {
    if (n == i) return 3;
    ++n;
  }
  return 0;
}
constexpr int passes(int L) {
  int n = 0;
  while (radix_at(L, n)) ++n;
  return n;
}
}  // namespace ctp

template <int L> struct CtPlan {
  static constexpr int P = ctp::passes(L);
  static constexpr int R(int p) { return ctp::radix_at(L, p); }
  static constexpr int NS(int p) {
    int s = 1;
    for (int i = 0; i < p; ++i) s *= R(i);
    return s;
  }
  // offset of pass p's part of the per-pass twiddle table (p >= 1)
  static constexpr int TWO(int p) {
    int o = 0;
    for (int i = 1; i < p; ++i) o += (R(i) - 1) * NS(i);
    return o;
  }
  static constexpr int NTW = TWO(P) > 0 ? TWO(P) : 1;
  static constexpr int T = (L + 15) / 16;  // threads per line, as the runtime plan
  static constexpr int PITCH = L + (L >> 4) + 1;
  static constexpr uint64_t codes() {
    uint64_t c = 0;
    for (int p = 0; p < P; ++p) c |= (uint64_t)R(p) << (5 * p);
    return c;
  }
};

// Host: whether L has compile-time instances, and their radix codes.
inline bool ct_length(int L, uint64_t *codes) {
#define DPFFT_CT_CASE(LL)                 \
  if (L == LL) {                          \
    *codes = CtPlan<LL>::codes();         \
    return true;                          \
  }
  DPFFT_CT_LENGTHS(DPFFT_CT_CASE)
#undef DPFFT_CT_CASE
  return false;
}

}  // namespace dpfft
