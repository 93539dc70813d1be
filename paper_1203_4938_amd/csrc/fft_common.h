// Device building blocks for the gfx950 FFT kernels: complex arithmetic and
// in-register DFTs of radix 2, 3, 4, 5, 7, 8, 16 and 32.
//
// Every DFT here is the forward transform X[k] = sum_j x[j] w_R^{jk} with
// w_R = exp(-2 pi i / R), computed in place in natural order.  The inverse
// transform is obtained by the kernels by exchanging real and imaginary parts
// on load and on store (swap(FFT(swap(x))) = conj(FFT(conj(x)))), so only the
// forward butterflies exist.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

namespace dpfft {

typedef float2 cf;

__device__ __forceinline__ cf cadd(cf a, cf b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cf csub(cf a, cf b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ cf cmul(cf a, cf b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ cf cscale(cf a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ cf cswap(cf a) { return make_float2(a.y, a.x); }
// An empty asm statement that reads and rewrites both halves: every load into
// them has to complete here, and the compiler keeps them in VGPRs.
__device__ __forceinline__ void pin_regs(cf &a) {
  float x = a.x, y = a.y;
  asm volatile("" : "+v"(x), "+v"(y));
  a = make_float2(x, y);
}
// multiply by -i
__device__ __forceinline__ cf mul_mi(cf a) { return make_float2(a.y, -a.x); }

// cos and sin of 2*pi*e/16 (e = 0..15), for the radix-16/8/4 internal twiddles
__device__ constexpr float kCos16[16] = {
    1.0f, 0.923879532511286756f, 0.707106781186547524f, 0.382683432365089772f,
    0.0f, -0.382683432365089772f, -0.707106781186547524f, -0.923879532511286756f,
    -1.0f, -0.923879532511286756f, -0.707106781186547524f, -0.382683432365089772f,
    0.0f, 0.382683432365089772f, 0.707106781186547524f, 0.923879532511286756f};
__device__ constexpr float kSin16[16] = {
    0.0f, 0.382683432365089772f, 0.707106781186547524f, 0.923879532511286756f,
    1.0f, 0.923879532511286756f, 0.707106781186547524f, 0.382683432365089772f,
    0.0f, -0.382683432365089772f, -0.707106781186547524f, -0.923879532511286756f,
    -1.0f, -0.923879532511286756f, -0.707106781186547524f, -0.382683432365089772f};

// x * w_R^E for a compile-time exponent, R a divisor of 16.  Multiples of
// pi/2 become swaps and negations; odd multiples of pi/4 use one shared
// product; the rest is a constant complex product.
template <int R, int E>
__device__ __forceinline__ cf mulw16(cf x) {
  static_assert(16 % R == 0, "radix must divide 16");
  constexpr int e = ((E % R) + R) % R * (16 / R);  // exponent in units of 2pi/16
  if constexpr (e == 0) {
    return x;
  } else if constexpr (e == 4) {
    return make_float2(x.y, -x.x);
  } else if constexpr (e == 8) {
    return make_float2(-x.x, -x.y);
  } else if constexpr (e == 12) {
    return make_float2(-x.y, x.x);
  } else if constexpr (e == 2) {  // (1 - i)/sqrt2
    constexpr float r = 0.707106781186547524f;
    return make_float2((x.x + x.y) * r, (x.y - x.x) * r);
  } else if constexpr (e == 6) {  // (-1 - i)/sqrt2
    constexpr float r = 0.707106781186547524f;
    return make_float2((x.y - x.x) * r, -(x.x + x.y) * r);
  } else if constexpr (e == 10) {  // (-1 + i)/sqrt2
    constexpr float r = 0.707106781186547524f;
    return make_float2(-(x.x + x.y) * r, (x.x - x.y) * r);
  } else if constexpr (e == 14) {  // (1 + i)/sqrt2
    constexpr float r = 0.707106781186547524f;
    return make_float2((x.x - x.y) * r, (x.x + x.y) * r);
  } else {
    constexpr float c = kCos16[e], s = kSin16[e];  // w = c - i s
    return make_float2(x.x * c + x.y * s, x.y * c - x.x * s);
  }
}

// cos and sin of 2*pi*e/32 for the odd e (the even ones are kCos16/kSin16)
__device__ constexpr float kCos32Odd[16] = {
    0.980785280403230449f,  0.831469612302545237f,  0.555570233019602225f,  0.195090322016128268f,
    -0.195090322016128268f, -0.555570233019602225f, -0.831469612302545237f, -0.980785280403230449f,
    -0.980785280403230449f, -0.831469612302545237f, -0.555570233019602225f, -0.195090322016128268f,
    0.195090322016128268f,  0.555570233019602225f,  0.831469612302545237f,  0.980785280403230449f};
__device__ constexpr float kSin32Odd[16] = {
    0.195090322016128268f,  0.555570233019602225f,  0.831469612302545237f,  0.980785280403230449f,
    0.980785280403230449f,  0.831469612302545237f,  0.555570233019602225f,  0.195090322016128268f,
    -0.195090322016128268f, -0.555570233019602225f, -0.831469612302545237f, -0.980785280403230449f,
    -0.980785280403230449f, -0.831469612302545237f, -0.555570233019602225f, -0.195090322016128268f};

// x * w_R^E for R a divisor of 32: even multiples of 2pi/32 go to mulw16,
// odd ones are a constant complex product (entry (e-1)/2 of the odd table).
template <int R, int E>
__device__ __forceinline__ cf mulw32(cf x) {
  static_assert(32 % R == 0, "radix must divide 32");
  constexpr int e = ((E % R) + R) % R * (32 / R);  // exponent in units of 2pi/32
  if constexpr (e % 2 == 0) {
    return mulw16<16, e / 2>(x);
  } else {
    constexpr float c = kCos32Odd[(e - 1) / 2], s = kSin32Odd[(e - 1) / 2];  // w = c - i s
    return make_float2(x.x * c + x.y * s, x.y * c - x.x * s);
  }
}

// x * w_9^E with w_9 = exp(-2 pi i / 9): cos and sin of 2*pi*e/9, e = 0..8
__device__ constexpr float kCos9[9] = {
    1.000000000000000000f, 0.766044443118978013f, 0.173648177666930414f, -0.500000000000000000f, -0.939692620785908317f,
    -0.939692620785908317f, -0.500000000000000000f, 0.173648177666930414f, 0.766044443118978013f};
__device__ constexpr float kSin9[9] = {
    0.000000000000000000f, 0.642787609686539252f, 0.984807753012208020f, 0.866025403784438708f, 0.342020143325668879f,
    -0.342020143325668879f, -0.866025403784438708f, -0.984807753012208020f, -0.642787609686539252f};
template <int E>
__device__ __forceinline__ cf mulw9(cf x) {
  constexpr int e = ((E % 9) + 9) % 9;
  if constexpr (e == 0) {
    return x;
  } else {
    constexpr float c = kCos9[e], s = kSin9[e];  // w = c - i s
    return make_float2(x.x * c + x.y * s, x.y * c - x.x * s);
  }
}

// ---------------------------------------------------------------------------
// power-of-two DFTs
// ---------------------------------------------------------------------------
__device__ __forceinline__ void dft2(cf &a, cf &b) {
  cf t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

// In-place DFT-4 of (a0, a1, a2, a3).
__device__ __forceinline__ void dft4(cf &a0, cf &a1, cf &a2, cf &a3) {
  cf t0 = cadd(a0, a2), t1 = csub(a0, a2);
  cf t2 = cadd(a1, a3), t3 = mul_mi(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

// DFT of R = R1*R2 points as R2 interleaved DFT-R1, twiddles w_R^{n2 k1},
// then R1 DFT-R2: with n = n2 + R2*n1 and k = k1 + R1*k2,
//   X[k1 + R1 k2] = sum_{n2} w_R2^{n2 k2} w_R^{n2 k1} sum_{n1} x[n2 + R2 n1] w_R1^{n1 k1}.
template <int R> struct Dft;

template <> struct Dft<1> {
  __device__ __forceinline__ static void run(cf *) {}
};
template <> struct Dft<2> {
  __device__ __forceinline__ static void run(cf *a) { dft2(a[0], a[1]); }
};
template <> struct Dft<4> {
  __device__ __forceinline__ static void run(cf *a) { dft4(a[0], a[1], a[2], a[3]); }
};

template <int R1, int R2, int N2 = 0>
__device__ __forceinline__ void twiddle_row(cf *b) {
  // b[k1] *= w_{R1 R2}^{N2 k1} for k1 = 1..R1-1 (compile-time unrolled)
  if constexpr (N2 > 0) {
    [&]<int... K>(std::integer_sequence<int, K...>) {
      if constexpr (16 % (R1 * R2) == 0)
        ((b[K] = mulw16<R1 * R2, N2 * K>(b[K])), ...);
      else if constexpr (R1 * R2 == 9)
        ((b[K] = mulw9<N2 * K>(b[K])), ...);
      else
        ((b[K] = mulw32<R1 * R2, N2 * K>(b[K])), ...);
    }(std::make_integer_sequence<int, R1>{});
  }
}

template <int R1, int R2>
__device__ __forceinline__ void dft_two_factor(cf *a) {
  constexpr int R = R1 * R2;
  cf b[R2][R1];
#pragma unroll
  for (int n2 = 0; n2 < R2; ++n2) {
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) b[n2][n1] = a[n2 + R2 * n1];
    Dft<R1>::run(b[n2]);
  }
  [&]<int... N2>(std::integer_sequence<int, N2...>) {
    (twiddle_row<R1, R2, N2>(b[N2]), ...);
  }(std::make_integer_sequence<int, R2>{});
#pragma unroll
  for (int k1 = 0; k1 < R1; ++k1) {
    cf c[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) c[n2] = b[n2][k1];
    Dft<R2>::run(c);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) a[k1 + R1 * k2] = c[k2];
  }
  (void)R;
}

template <> struct Dft<8> {
  __device__ __forceinline__ static void run(cf *a) { dft_two_factor<4, 2>(a); }
};
template <> struct Dft<16> {
  __device__ __forceinline__ static void run(cf *a) { dft_two_factor<4, 4>(a); }
};
template <> struct Dft<32> {
  __device__ __forceinline__ static void run(cf *a) { dft_two_factor<8, 4>(a); }
};

// ---------------------------------------------------------------------------
// odd prime DFTs: pair j with p-j.  With s_j = x_j + x_{p-j}, d_j = x_j - x_{p-j}
// (j = 1..(p-1)/2), c_m = cos(2 pi m/p), q_m = sin(2 pi m/p):
//   X_k     = x_0 + sum_j s_j c_{jk} - i sum_j d_j q_{jk}
//   X_{p-k} = x_0 + sum_j s_j c_{jk} + i sum_j d_j q_{jk}
// ---------------------------------------------------------------------------
template <int P> struct PrimeTrig;
template <> struct PrimeTrig<3> {
  static constexpr float c[3] = {1.0f, -0.5f, -0.5f};
  static constexpr float s[3] = {0.0f, 0.866025403784438647f, -0.866025403784438647f};
};
template <> struct PrimeTrig<5> {
  static constexpr float c[5] = {1.0f, 0.309016994374947424f, -0.809016994374947424f,
                                 -0.809016994374947424f, 0.309016994374947424f};
  static constexpr float s[5] = {0.0f, 0.951056516295153572f, 0.587785252292473129f,
                                 -0.587785252292473129f, -0.951056516295153572f};
};
template <> struct PrimeTrig<7> {
  static constexpr float c[7] = {1.0f, 0.623489801858733531f, -0.222520933956314404f,
                                 -0.900968867902419126f, -0.900968867902419126f,
                                 -0.222520933956314404f, 0.623489801858733531f};
  static constexpr float s[7] = {0.0f, 0.781831482468029809f, 0.974927912181823607f,
                                 0.433883739117558120f, -0.433883739117558120f,
                                 -0.974927912181823607f, -0.781831482468029809f};
};

template <int P>
__device__ __forceinline__ void dft_prime(cf *a) {
  constexpr int H = (P - 1) / 2;
  cf s[H + 1], d[H + 1];
#pragma unroll
  for (int j = 1; j <= H; ++j) {
    s[j] = cadd(a[j], a[P - j]);
    d[j] = csub(a[j], a[P - j]);
  }
  cf x0 = a[0];
  cf sum = x0;
#pragma unroll
  for (int j = 1; j <= H; ++j) sum = cadd(sum, s[j]);
#pragma unroll
  for (int k = 1; k <= H; ++k) {
    float re = x0.x, im = x0.y, pr = 0.0f, pi = 0.0f;
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      const int m = (j * k) % P;
      const float c = PrimeTrig<P>::c[m], q = PrimeTrig<P>::s[m];
      re += s[j].x * c;
      im += s[j].y * c;
      pr += d[j].x * q;
      pi += d[j].y * q;
    }
    // -i * (pr + i pi) = pi - i pr
    a[k] = make_float2(re + pi, im - pr);
    a[P - k] = make_float2(re - pi, im + pr);
  }
  a[0] = sum;
}

template <> struct Dft<3> {
  __device__ __forceinline__ static void run(cf *a) { dft_prime<3>(a); }
};
template <> struct Dft<5> {
  __device__ __forceinline__ static void run(cf *a) { dft_prime<5>(a); }
};
template <> struct Dft<7> {
  __device__ __forceinline__ static void run(cf *a) { dft_prime<7>(a); }
};
// DFT-9 as 3 x 3: two passes of 3 fewer through LDS for every pair of 3s
template <> struct Dft<9> {
  __device__ __forceinline__ static void run(cf *a) { dft_two_factor<3, 3>(a); }
};

// ---------------------------------------------------------------------------
// workgroup -> tile remapping that keeps consecutive tiles on one XCD.
// Consecutive workgroup ids are dispatched round-robin over the 8 XCDs, each
// with its own L2; tiles that share cache lines should share an L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t xcd_remap(uint32_t bid, uint32_t nblocks) {
  constexpr uint32_t X = 8;
  uint32_t full = nblocks / X * X;
  if (bid >= full) return bid;
  return (bid % X) * (nblocks / X) + bid / X;
}
// The same in rounds: each round of 8 K consecutive tiles gives every XCD K
// consecutive ones (K = 32: one per CU), so the tiles in flight sweep whole
// rows of the matrix together (DRAM page locality) while tiles sharing cache
// lines still share an L2.  Measured on the power-of-two line and MFMA
// kernels: 4-11% faster for the 256 x 256 four-step, the 4096-point column
// tiles of 2D images and the transposed-row tiles of 2048 and 4096.  K = 16
// (F_ROUNDS16, half a tile per CU in each round) is faster still for the
// 2048-point tiles of the 2^22 four-step, whose one workgroup per CU makes a
// round of 32 per XCD span a whole wave of the chip.  Falls back to xcd_remap
// when the grid is not a whole number of rounds.
__device__ __forceinline__ uint32_t xcd_remap_rounds(uint32_t bid, uint32_t nblocks,
                                                     uint32_t kshift = 5) {
  constexpr uint32_t X = 8;
  const uint32_t K = 1u << kshift;
  if (nblocks % (X * K) != 0) return xcd_remap(bid, nblocks);
  const uint32_t slot = bid / X;
  return (slot >> kshift) * (X * K) + (bid % X) * K + (slot & (K - 1));
}

}  // namespace dpfft
