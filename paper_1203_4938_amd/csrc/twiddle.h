// Host twiddle tables, generated in FP64 and rounded once to the kernel type.
#pragma once
#include <stdint.h>

#include <complex>
#include <vector>

namespace dpfft {

// w_M^t = exp(-2 pi i t / M) in double, t reduced exactly modulo M first.
std::complex<double> omega(int64_t M, int64_t t);

// Stockham pass table for a power-of-two line kernel of length L: for each
// pass p >= 1 with radix R and span Ns, entries (r-1)*Ns + k = w_{Ns R}^{k r}
// for r = 1..R-1, k = 0..Ns-1, passes concatenated in order.
std::vector<std::complex<double>> stockham_table_pow2(int L);

// Two-level four-step table for length N: lo[l] = w_N^l (l < 2^shift),
// hi[h] = w_N^{h 2^shift} (h < ceil(N / 2^shift)), so that
// w_N^e = hi[e >> shift] * lo[e & (2^shift - 1)].
void fourstep_tables(int64_t N, int shift, std::vector<std::complex<double>> &lo,
                     std::vector<std::complex<double>> &hi);

}  // namespace dpfft
