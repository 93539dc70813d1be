// Real-input transforms of power-of-two length N = 2L (forward: N reals ->
// N/2 + 1 complex bins; inverse: N/2 + 1 bins of a Hermitian spectrum -> N
// reals), each through one L-point complex transform.
//
// Forward.  The N reals of a line, read as L complex values z[m] = x[2m] +
// i x[2m+1] (the same bytes, so the load is the complex kernels' load), go
// through the L-point Stockham passes: Z = DFT_L(z).  With Fe = DFT_L of the
// even samples and Fo = DFT_L of the odd ones,
//   Fe[k] = (Z[k] + conj Z[L-k]) / 2,   Fo[k] = (Z[k] - conj Z[L-k]) / (2i),
//   X[k]  = Fe[k] + w_N^k Fo[k]   (k = 0..L-1),   X[L] = Fe[0] - Fo[0],
// indices of Z taken mod L.  The pairing of k with L - k is one LDS exchange
// after the last pass.
//
// Inverse.  For real output, X[k + L] = conj X[L - k], so
//   Fe'[k] = X[k] + conj X[L-k],   Fo'[k] = (X[k] - conj X[L-k]) w_N^{-k}
// are twice the even and odd half-transforms, and z = IDFT_L(Fe' + i Fo') / 2
// holds x[2m] in its real and x[2m+1] in its imaginary part.  The kernel
// forms Fe' + i Fo' after one LDS exchange, runs the passes as swap(FFT(swap))
// and scales by 1/N (the caller's scale) on the store.  Bins 0 and L of a
// Hermitian spectrum are real; their imaginary parts are ignored.
#include "line_device.h"
#include "real.h"

namespace dpfft {

template <int L, int C, bool INV>
__global__ void __launch_bounds__(C * (P2<L>::T))
    k_real(const cf *__restrict__ in, cf *__restrict__ out, LineArgs a) {
  using G = P2<L>;
  constexpr int E = G::E, T = G::T;
  using LD = Lds<L, C, ELEM_FAST, kPadShift>;
  __shared__ __align__(16) cf lds[LD::SIZE];
  using PT = PlainTw<L, C, ELEM_FAST, ELEM_FAST, 16, C * G::T>;
  __shared__ cf twl[PT::NTW > 0 ? PT::NTW : 1];

  const int tid = threadIdx.x;
  int c, j;
  lane_map<L, 16, C, ELEM_FAST>(tid, c, j);
  const int64_t tile = blockIdx.x;
  const int64_t bb = tile / a.tiles_per_batch;
  const int64_t line = (tile - bb * a.tiles_per_batch) * C + c;
  const bool valid = line < a.lines;
  const cf *src = in + bb * a.in_b + line * a.in_l;
  cf *dst = out + bb * a.out_b + line * a.out_l;
  const cf *__restrict__ wn = a.tw4_lo;  // w_N^k, k = 0..L-1

  PT::fill(twl, a, tid);
  cf v[E];
  if constexpr (!INV) {
    if (valid) {
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = src[j + T * m];
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = make_float2(0.f, 0.f);
    }
    all_passes<L, 16, C, ELEM_FAST>(v, lds, PT::make(twl, a), c, j,
                                   std::make_integer_sequence<int, G::NP>{});
    // v[m] = Z[j + T m]; the last pass left the LDS buffer free
#pragma unroll
    for (int m = 0; m < E; ++m) lds[LD::idx_off(c, j, T * m)] = v[m];
    __syncthreads();
    cf X[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int k = j + T * m;
      const cf zr = lds[LD::idx(c, (L - k) & (L - 1))];
      const cf zk = v[m];
      const cf fe = make_float2(0.5f * (zk.x + zr.x), 0.5f * (zk.y - zr.y));
      // (Z[k] - conj Z[L-k]) / (2i)
      const cf fo = make_float2(0.5f * (zk.y + zr.y), -0.5f * (zk.x - zr.x));
      X[m] = cadd(fe, cmul(wn[k], fo));
    }
    if (valid) {
#pragma unroll
      for (int m = 0; m < E; ++m) dst[j + T * m] = X[m];
      if (j == 0) dst[L] = make_float2(v[0].x - v[0].y, 0.f);
    }
  } else {
    cf xl = make_float2(0.f, 0.f);
    if (valid) {
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = src[j + T * m];
      xl = src[L];
    } else {
#pragma unroll
      for (int m = 0; m < E; ++m) v[m] = make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int m = 0; m < E; ++m) lds[LD::idx_off(c, j, T * m)] = v[m];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < E; ++m) {
      const int k = j + T * m;
      cf xr = lds[LD::idx(c, (L - k) & (L - 1))];
      cf xk = v[m];
      if (m == 0 && j == 0) {
        // k = 0 pairs with bin L; both are real in a Hermitian spectrum
        xr = make_float2(xl.x, 0.f);
        xk.y = 0.f;
      }
      const cf fe = make_float2(xk.x + xr.x, xk.y - xr.y);
      const cf wc = wn[k];
      const cf d = cmul(make_float2(xk.x - xr.x, xk.y + xr.y), make_float2(wc.x, -wc.y));
      // Fe' + i Fo', entered swapped (the inverse is swap(FFT(swap)))
      v[m] = make_float2(fe.y + d.x, fe.x - d.y);
    }
    __syncthreads();  // the pairing reads are done before the passes write LDS
    all_passes<L, 16, C, ELEM_FAST>(v, lds, PT::make(twl, a), c, j,
                                   std::make_integer_sequence<int, G::NP>{});
    if (valid) {
#pragma unroll
      for (int m = 0; m < E; ++m) dst[j + T * m] = cswap(cscale(v[m], a.scale));
    }
  }
}

// Real transforms longer than one workgroup's LDS (N > 32768), or of even
// lengths that are not powers of two: the L-point complex transform of z runs
// as launches of its own (the four-step pair, or the runtime-radix single
// pass), and this pass pairs the elements k and L - k that the in-kernel form
// pairs through LDS.  With Fe[L-k] = conj Fe[k], Fo[L-k] = conj Fo[k] and w_N^{L-k} =
// -conj w_N^k, one twiddle serves both outputs of a pair:
//   X[k] = Fe[k] + w_N^k Fo[k],   X[L-k] = conj(Fe[k] - w_N^k Fo[k])
// (k = 0: X[L], from Z[0] alone; for even L, k = L/2 pairs with itself).  The inverse
// forms Fe' + i Fo' at k and L - k the same way (its conjugate halves) for the
// complex inverse, which holds the samples once scaled by 1/N.  A thread
// reads both elements of its pair before it writes them, so the pass would
// also be correct in place; in and out are not restrict-qualified.
template <bool INV>
__global__ void __launch_bounds__(256) k_real_pair(const cf *in, cf *out, RealPairArgs a) {
  const int64_t np = a.L / 2 + 1;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= np) return;
  const uint32_t msk = (1u << a.shift) - 1u;
  const cf w = cmul(a.hi[(uint32_t)k >> a.shift], a.lo[(uint32_t)k & msk]);  // w_N^k
  const int64_t kr = a.L - k;  // k = 0: bin L on the spectrum side, Z[0] on the other
  for (int64_t b = blockIdx.y; b < a.batch; b += gridDim.y) {
    const cf *src = in + b * a.in_b;
    cf *dst = out + b * a.out_b;
    if constexpr (!INV) {
      const cf zk = src[k], zr = src[kr == a.L ? 0 : kr];
      const cf fe = make_float2(0.5f * (zk.x + zr.x), 0.5f * (zk.y - zr.y));
      const cf fo = make_float2(0.5f * (zk.y + zr.y), -0.5f * (zk.x - zr.x));
      const cf t = cmul(w, fo);
      dst[k] = cadd(fe, t);
      if (kr != k) dst[kr] = make_float2(fe.x - t.x, t.y - fe.y);
    } else {
      cf xk = src[k], xr = src[kr];
      if (k == 0) {  // bins 0 and L of a Hermitian spectrum are real
        xk.y = 0.f;
        xr.y = 0.f;
      }
      const cf fe = make_float2(xk.x + xr.x, xk.y - xr.y);                   // X[k] + conj X[L-k]
      const cf fo = cmul(make_float2(xk.x - xr.x, xk.y + xr.y), make_float2(w.x, -w.y));
      dst[k] = make_float2(fe.x - fo.y, fe.y + fo.x);                        // Fe' + i Fo'
      if (k != 0 && kr != k) dst[kr] = make_float2(fe.x + fo.y, fo.x - fe.y);  // conj Fe' + i conj Fo'
    }
  }
}

const void *real_pair_kernel(bool inverse) {
  return inverse ? (const void *)&k_real_pair<true> : (const void *)&k_real_pair<false>;
}

struct RealEntry {
  int L, C;
  const void *fwd, *inv;
  int threads, lds;
};

#define RE(L_, C_)                                                                          \
  RealEntry{L_, C_, (const void *)&k_real<L_, C_, false>, (const void *)&k_real<L_, C_, true>, \
            C_ * P2<L_>::T,                                                                  \
            (int)sizeof(cf) * (Lds<L_, C_, ELEM_FAST, kPadShift>::SIZE +                     \
                               PlainTw<L_, C_, ELEM_FAST, ELEM_FAST, 16, C_ * P2<L_>::T>::NTW)}

// 256 threads per workgroup up to L = 4096, then one line per workgroup
static const RealEntry kRealTable[] = {
    RE(1, 256),  RE(2, 256),   RE(4, 256),  RE(8, 256),  RE(16, 256),
    RE(32, 128), RE(64, 64),   RE(128, 32), RE(256, 16), RE(512, 8),
    RE(1024, 4), RE(2048, 2),  RE(4096, 1), RE(8192, 1), RE(16384, 1),
};
#undef RE

bool real_kernel(int L, RealKernel *out) {
  for (const auto &e : kRealTable) {
    if (e.L == L) {
      out->fwd = e.fwd;
      out->inv = e.inv;
      out->lines = e.C;
      out->threads = e.threads;
      out->lds_bytes = e.lds;
      return true;
    }
  }
  return false;
}

}  // namespace dpfft
