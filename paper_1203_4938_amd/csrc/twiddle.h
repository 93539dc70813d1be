// Host twiddle tables, generated in FP64 and rounded once to the kernel type.
#pragma once
#include <stdint.h>

#include <complex>
#include <vector>

namespace dpfft {

// w_M^t = exp(-2 pi i t / M) in double, t reduced exactly modulo M first.
std::complex<double> omega(int64_t M, int64_t t);

// Stockham pass table for a power-of-two line kernel of length L with `ept`
// elements per thread (its radix plan, see P2): for each
// pass p >= 1 with radix R and span Ns, entries (r-1)*Ns + k = w_{Ns R}^{k r}
// for r = 1..R-1, k = 0..Ns-1, passes concatenated in order.
std::vector<std::complex<double>> stockham_table_pow2(int L, int ept = 16);

// Two-level four-step table for length N: lo[l] = w_N^l (l < 2^shift),
// hi[h] = w_N^{h 2^shift} (h < ceil(N / 2^shift)), so that
// w_N^e = hi[e >> shift] * lo[e & (2^shift - 1)].
void fourstep_tables(int64_t N, int shift, std::vector<std::complex<double>> &lo,
                     std::vector<std::complex<double>> &hi);

// Round a double to the nearest number with `p` significand bits and minimum
// normal exponent `emin` (ties to even; subnormals keep the quantum
// 2^(emin-p+1)).  FP16: p = 11, emin = -14.  BF16: p = 8, emin = -126.
double round_sig(double x, int p, int emin);
uint16_t fp16_bits(double exact);   // bit pattern of an FP16-representable value
uint16_t bf16_bits(double exact);   // bit pattern of a BF16-representable value

// Per-lane A operands of the DFT-16 matrix for the MFMA stages:
// [piece][re, im][lane 0..63][t 0..7] 16-bit patterns, where lane l, slot t
// holds row i = l & 15, column k = 8 (l >> 4) + t of
//   A_re = [cos | sin], A_im = [-sin | cos]  (angle 2 pi i k' / 16),
// split as w = hi + 2^-s mid + 2^-2s lo with every piece rounded in FP64.
std::vector<uint16_t> mfma_dft16_operands(int prec);

}  // namespace dpfft
