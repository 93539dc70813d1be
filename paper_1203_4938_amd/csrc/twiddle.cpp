// FP64 host twiddle generation.
#include "twiddle.h"

#include <cmath>

#include <cstring>

#include "kernels.h"
#include "mfma.h"

namespace dpfft {

std::complex<double> omega(int64_t M, int64_t t) {
  int64_t r = t % M;
  if (r < 0) r += M;
  // the angle is formed from the exactly reduced integer numerator, so its
  // only error is the double rounding of 2*pi*r/M (about 1e-16 relative)
  const double ang = -2.0 * M_PI * (static_cast<double>(r) / static_cast<double>(M));
  return {std::cos(ang), std::sin(ang)};
}

std::vector<std::complex<double>> stockham_table_pow2(int L, int ept) {
  std::vector<std::complex<double>> tab;
  const int np = pow2_passes(L, ept);
  int ns = 1;
  for (int p = 0; p < np; ++p) {
    const int R = pow2_radix(L, p, ept);
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

double round_sig(double x, int p, int emin) {
  if (x == 0.0) return 0.0;
  int e = 0;
  std::frexp(x, &e);  // |x| in [2^(e-1), 2^e)
  int lead = e - 1;
  if (lead < emin) lead = emin;
  const double q = std::ldexp(1.0, lead - p + 1);
  return std::nearbyint(x / q) * q;  // default rounding mode: nearest, ties to even
}

uint16_t fp16_bits(double v) {
  const _Float16 h = (_Float16)v;  // exact: v is representable
  uint16_t b;
  std::memcpy(&b, &h, 2);
  return b;
}

uint16_t bf16_bits(double v) {
  const float f = (float)v;  // exact: a BF16 value is a float with 8 significant bits
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return (uint16_t)(u >> 16);
}

std::vector<uint16_t> mfma_dft16_operands(int prec) {
  const int np = mfma_pieces(prec), sh = mfma_piece_shift(prec);
  const bool half = (prec == MP_FP16 || prec == MP_FP16_SPLIT);
  const int p = half ? 11 : 8, emin = half ? -14 : -126;
  std::vector<uint16_t> out((size_t)np * 2 * 64 * 8);
  for (int reim = 0; reim < 2; ++reim)
    for (int lane = 0; lane < 64; ++lane)
      for (int t = 0; t < 8; ++t) {
        const int i = lane & 15, k = 8 * (lane >> 4) + t, kk = k & 15;
        const double ang = 2.0 * M_PI * (double)((i * kk) % 16) / 16.0;
        double w;
        if (reim == 0) w = k < 16 ? std::cos(ang) : std::sin(ang);
        else w = k < 16 ? -std::sin(ang) : std::cos(ang);
        double r = w;
        for (int q = 0; q < np; ++q) {
          const double piece = round_sig(r, p, emin);
          out[(((size_t)q * 2 + reim) * 64 + lane) * 8 + t] = half ? fp16_bits(piece) : bf16_bits(piece);
          r = (r - piece) * std::ldexp(1.0, sh);
        }
      }
  return out;
}

}  // namespace dpfft
