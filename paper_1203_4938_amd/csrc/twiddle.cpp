// FP64 host twiddle generation.
#include "twiddle.h"

#include <cmath>

#include "kernels.h"

namespace dpfft {

std::complex<double> omega(int64_t M, int64_t t) {
  int64_t r = t % M;
  if (r < 0) r += M;
  // the angle is formed from the exactly reduced integer numerator, so its
  // only error is the double rounding of 2*pi*r/M (about 1e-16 relative)
  const double ang = -2.0 * M_PI * (static_cast<double>(r) / static_cast<double>(M));
  return {std::cos(ang), std::sin(ang)};
}

std::vector<std::complex<double>> stockham_table_pow2(int L) {
  std::vector<std::complex<double>> tab;
  const int np = pow2_passes(L);
  int ns = 1;
  for (int p = 0; p < np; ++p) {
    const int R = pow2_radix(L, p);
    if (p >= 1) {
      for (int r = 1; r < R; ++r)
        for (int k = 0; k < ns; ++k) tab.push_back(omega((int64_t)ns * R, (int64_t)k * r));
    }
    ns *= R;
  }
  if (tab.empty()) tab.push_back({1.0, 0.0});
  return tab;
}

void fourstep_tables(int64_t N, int shift, std::vector<std::complex<double>> &lo,
                     std::vector<std::complex<double>> &hi) {
  const int64_t B = int64_t(1) << shift;
  lo.resize(B);
  for (int64_t l = 0; l < B; ++l) lo[l] = omega(N, l);
  const int64_t H = (N + B - 1) / B;
  hi.resize(H);
  for (int64_t h = 0; h < H; ++h) hi[h] = omega(N, h * B);
}

}  // namespace dpfft
