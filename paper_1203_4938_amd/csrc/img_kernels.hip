// Image block compression (section III-B of the paper), five steps:
//   (a) RGB -> luminance Y and chroma Cb, Cr (full-range BT.601 as in JFIF)
//   (b) chroma at a quarter of the pixels (means of 2x2 squares)
//   (c) |grad Y| (central differences, edges replicated) and per 4x4 block
//       its mean (activity), the mean luminance and the 16 deviations
//   (d) k-means codebook of the deviation vectors of blocks with activity
//       >= tau (Lloyd's iteration from the pattern blocks of rank
//       floor(c P / k))
//   (e) per block: code 0 (mean only) or 1 + the nearest codeword.
// The paper runs (a)-(c) and (e) as data-parallel programs and (d) on the
// host; here every step is a kernel, so a batch of images is one sequence of
// launches on one stream with no host round trip.
//
// (a)-(c) are one pass over the pixels (k_img_front): a 64 x 16 pixel tile
// computes Y for itself and a one-pixel halo into LDS, writes Y and the
// quarter-size chroma, then four threads per block reduce its 16 pixels.
// The k-means and the encoding walk the blocks in groups of 256, one block
// per thread, the codebook in LDS; the cluster sums of a group go through
// LDS atomics into per-group partials that k_img_update adds up in a fixed
// order.
#include "fft_common.h"
#include "img.h"

namespace dpfft {

namespace {

__device__ __forceinline__ float luma(float r, float g, float b) {
  return 0.299f * r + 0.587f * g + 0.114f * b;
}
__device__ __forceinline__ float chroma_b(float r, float g, float b) {
  return 128.0f - 0.168736f * r - 0.331264f * g + 0.5f * b;
}
__device__ __forceinline__ float chroma_r(float r, float g, float b) {
  return 128.0f + 0.5f * r - 0.418688f * g - 0.081312f * b;
}

constexpr int HW = kImgTileW + 2, HH = kImgTileH + 2;  // tile with its halo

}  // namespace

// Y of pixel (gy, gx) clamped to the image (the replicated edge).
__device__ __forceinline__ float luma_at(const uint8_t *rgb, int64_t h, int64_t w, int64_t gy,
                                         int64_t gx) {
  gy = gy < 0 ? 0 : (gy >= h ? h - 1 : gy);
  gx = gx < 0 ? 0 : (gx >= w ? w - 1 : gx);
  const uint8_t *p = rgb + (gy * w + gx) * 3;
  return luma((float)p[0], (float)p[1], (float)p[2]);
}

// Thread (row ry, group g) of a tile owns the 4 pixels x0 + 4 g .. + 3 of row
// y0 + ry: their 12 bytes are three aligned 32-bit words (the width is a
// multiple of 4).  It writes their Y, keeps it in LDS with the tile's
// one-pixel halo, and leaves the Cb, Cr sums of its two horizontal pixel
// pairs in LDS for the 2 x 2 means.  Then four threads take each 4 x 4 block,
// one block row each, and add their row sums with lane shuffles.
__global__ void __launch_bounds__(kImgThreads) k_img_front(ImgArgs a) {
  static_assert(kImgTileW == 64 && kImgTileH == 16 && kImgThreads == 256, "tile shape");
  __shared__ float ys[HH * HW];
  __shared__ float2 cpart[kImgTileH][kImgTileW / 2];
  const int64_t img = blockIdx.y;
  const int64_t tiles_x = (a.w + kImgTileW - 1) / kImgTileW;
  const int64_t tx = blockIdx.x % tiles_x, ty = blockIdx.x / tiles_x;
  const int64_t x0 = tx * kImgTileW, y0 = ty * kImgTileH;
  const uint8_t *rgb = a.rgb + img * a.h * a.w * 3;
  float *Y = a.y + img * a.h * a.w;
  const int tid = threadIdx.x;

  // (a) luminance of the tile, (b) chroma sums of horizontal pairs
  {
    const int ry = tid / 16, g = tid % 16;
    const int64_t py = y0 + ry, px = x0 + 4 * g;
    float yv[4];
    if (py < a.h && px < a.w) {
      const uint32_t *p = reinterpret_cast<const uint32_t *>(rgb + (py * a.w + px) * 3);
      const uint32_t d0 = p[0], d1 = p[1], d2 = p[2];
      const float r[4] = {(float)(d0 & 255u), (float)(d0 >> 24), (float)((d1 >> 16) & 255u),
                          (float)((d2 >> 8) & 255u)};
      const float gg[4] = {(float)((d0 >> 8) & 255u), (float)(d1 & 255u), (float)(d1 >> 24),
                           (float)((d2 >> 16) & 255u)};
      const float bb[4] = {(float)((d0 >> 16) & 255u), (float)((d1 >> 8) & 255u), (float)(d2 & 255u),
                           (float)(d2 >> 24)};
      float cb[4], cr[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        yv[i] = luma(r[i], gg[i], bb[i]);
        cb[i] = chroma_b(r[i], gg[i], bb[i]);
        cr[i] = chroma_r(r[i], gg[i], bb[i]);
      }
      *reinterpret_cast<float4 *>(Y + py * a.w + px) = make_float4(yv[0], yv[1], yv[2], yv[3]);
      cpart[ry][2 * g] = make_float2(cb[0] + cb[1], cr[0] + cr[1]);
      cpart[ry][2 * g + 1] = make_float2(cb[2] + cb[3], cr[2] + cr[3]);
    } else {
      // past the image's last row or column: the replicated edge, for the
      // central differences of the blocks along it
#pragma unroll
      for (int i = 0; i < 4; ++i) yv[i] = luma_at(rgb, a.h, a.w, py, px + i);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) ys[(ry + 1) * HW + 4 * g + 1 + i] = yv[i];
  }
  // the halo: rows -1 and 16 of the tile, columns -1 and 64 (corners unused)
  if (tid < 2 * kImgTileW + 2 * kImgTileH) {
    int ly, lx;
    if (tid < 2 * kImgTileW) {
      ly = tid < kImgTileW ? 0 : HH - 1;
      lx = tid % kImgTileW + 1;
    } else {
      const int q = tid - 2 * kImgTileW;
      ly = q % kImgTileH + 1;
      lx = q < kImgTileH ? 0 : HW - 1;
    }
    ys[ly * HW + lx] = luma_at(rgb, a.h, a.w, y0 + ly - 1, x0 + lx - 1);
  }
  __syncthreads();
  // (b) chroma: means of 2 x 2 squares, two per thread of the first 128
  if (tid < kImgTileH / 2 * kImgTileW / 4) {
    const int rp = tid / 16, g = tid % 16;
    const int64_t py = y0 + 2 * rp, px = x0 + 4 * g;
    if (py < a.h && px < a.w) {
      const float2 u0 = cpart[2 * rp][2 * g], l0 = cpart[2 * rp + 1][2 * g];
      const float2 u1 = cpart[2 * rp][2 * g + 1], l1 = cpart[2 * rp + 1][2 * g + 1];
      const int64_t w2 = a.w / 2, o = img * (a.h / 2) * w2 + (py / 2) * w2 + px / 2;
      *reinterpret_cast<float2 *>(a.cb + o) = make_float2(0.25f * (u0.x + l0.x), 0.25f * (u1.x + l1.x));
      *reinterpret_cast<float2 *>(a.cr + o) = make_float2(0.25f * (u0.y + l0.y), 0.25f * (u1.y + l1.y));
    }
  }
  // (c) blocks: four threads per block (lanes 4 q .. 4 q + 3 of one wave)
  {
    const int blk = tid / 4, r = tid % 4;
    const int by = blk / (kImgTileW / 4), bx = blk % (kImgTileW / 4);
    const int ly = 4 * by + r + 1, lx0 = 4 * bx + 1;
    float v[4], s = 0.f, g = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int lx = lx0 + j;
      const float c = ys[ly * HW + lx];
      const float gx = 0.5f * (ys[ly * HW + lx + 1] - ys[ly * HW + lx - 1]);
      const float gyv = 0.5f * (ys[(ly + 1) * HW + lx] - ys[(ly - 1) * HW + lx]);
      g += __builtin_sqrtf(gx * gx + gyv * gyv);
      s += c;
      v[j] = c;
    }
    s += __shfl_xor(s, 1, 64);
    g += __shfl_xor(g, 1, 64);
    s += __shfl_xor(s, 2, 64);
    g += __shfl_xor(g, 2, 64);
    const int64_t gby = y0 / 4 + by, gbx = x0 / 4 + bx, bw = a.w / 4;
    if (gby < a.h / 4 && gbx < bw) {
      const float m = s * (1.0f / 16.0f);
      const int64_t b = img * a.nb + gby * bw + gbx;
      if (r == 0) {
        a.mean[b] = m;
        a.act[b] = g * (1.0f / 16.0f);
      }
      reinterpret_cast<float4 *>(a.dev + 16 * b)[r] = make_float4(v[0] - m, v[1] - m, v[2] - m, v[3] - m);
    }
  }
}

// (d) pattern blocks per group of 256 blocks
__global__ void __launch_bounds__(kImgBlocksPerGroup) k_img_count(ImgArgs a) {
  __shared__ int cnt;
  const int64_t img = blockIdx.y;
  const int64_t b = (int64_t)blockIdx.x * kImgBlocksPerGroup + threadIdx.x;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  const bool pat = b < a.nb && a.act[img * a.nb + b] >= a.tau;
  if (pat) atomicAdd(&cnt, 1);
  __syncthreads();
  if (threadIdx.x == 0) a.wgcount[img * a.groups + blockIdx.x] = cnt;
}

// Exclusive offsets of the groups' pattern blocks (one workgroup per image,
// sequential over chunks of 256 groups), the pattern count, and a zero
// codebook (codewords with no seed stay zero when no block is a pattern).
__global__ void __launch_bounds__(256) k_img_scan(ImgArgs a) {
  __shared__ int s[256];
  __shared__ int carry;
  const int64_t img = blockIdx.x;
  int32_t *wc = a.wgcount + img * a.groups;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < a.groups; base += 256) {
    const int i = base + threadIdx.x;
    const int v = i < a.groups ? wc[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < 256; d *= 2) {  // inclusive scan (Hillis-Steele)
      const int t = threadIdx.x >= d ? s[threadIdx.x - d] : 0;
      __syncthreads();
      s[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < a.groups) wc[i] = carry + s[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 255) carry += s[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.npat[img] = carry;
  for (int i = threadIdx.x; i < a.k * 16; i += 256) a.codebook[img * a.k * 16 + i] = 0.f;
}

// Seeds: codeword c takes the deviation vector of the pattern block of rank
// floor(c P / k); a block of rank r seeds every c with that floor.
__global__ void __launch_bounds__(kImgBlocksPerGroup) k_img_seed(ImgArgs a) {
  __shared__ int s[kImgBlocksPerGroup];
  const int64_t img = blockIdx.y;
  const int64_t b = (int64_t)blockIdx.x * kImgBlocksPerGroup + threadIdx.x;
  const bool pat = b < a.nb && a.act[img * a.nb + b] >= a.tau;
  s[threadIdx.x] = pat;
  __syncthreads();
  for (int d = 1; d < kImgBlocksPerGroup; d *= 2) {
    const int t = threadIdx.x >= d ? s[threadIdx.x - d] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  if (!pat) return;
  const int64_t P = a.npat[img];
  const int64_t rank = a.wgcount[img * a.groups + blockIdx.x] + s[threadIdx.x] - 1;
  const int64_t k = a.k;
  const int64_t c_lo = (rank * k + P - 1) / P, c_hi = ((rank + 1) * k + P - 1) / P;
  const float *src = a.dev + 16 * (img * a.nb + b);
  for (int64_t c = c_lo; c < c_hi && c < k; ++c)
    for (int t = 0; t < 16; ++t) a.codebook[(img * k + c) * 16 + t] = src[t];
}

// Nearest codeword of every pattern block (ties to the lower index).
// The squared distance |v - c|^2 = |v|^2 - 2 (v.c - |c|^2 / 2) is ranked by
// D_c = v.c - h_c with h_c = |c|^2 / 2, the same maximiser as the smallest
// distance in exact arithmetic.  The dot products of a wave's 64 blocks with
// all codewords are FP32 matrix products on the matrix cores
// (v_mfma_f32_16x16x4_f32, 16 codewords x 16 blocks x 4 components each, the
// accumulator started at -h_c): A = codebook rows, B = deviation vectors.
// Operand layout of the 16x16x4 FP32 product: lane l supplies A row (l & 15)
// and B column (l & 15) at k = l >> 4; it holds D column (l & 15), rows
// 4 (l >> 4) + r, r < 4.  Step s of the four takes component 4 (l >> 4) + s,
// so a lane's operands are one aligned float4 of a codeword and of a block.
// Each lane keeps the best of its rows in index order (strictly larger wins),
// then the four lanes of a column compare (value, index) pairs: the larger
// value, on equal values the lower index, as a plain scan would pick.
// A workgroup covers kImgAssignBlocks blocks in rounds of 256 (one per
// thread), so the codebook and h_c are staged in LDS once per 1024 blocks.
// ACC: the group's cluster sums.  In each round every pattern block takes a
// rank among its wave's blocks of the same code from the wave's own LDS
// counter (one atomic per block; no other wave touches it, so the ranks do
// not depend on how the waves are scheduled), the per-wave counts are
// scanned, the blocks' deviation vectors are scattered into (code, wave,
// rank) order, and the (cluster, component) sums are read off the contiguous
// runs and added, round after round, to the group's running sums (each entry
// owned by one thread, which reads back only its own writes): in LDS for up
// to kImgLdsSumK codewords, else in the group's partial in global memory,
// where they leave the LDS for more workgroups per CU.  One partial per 1024
// blocks.
// Otherwise the codes of every block are written.  The codebook and the
// group's work arrays sit in dynamic LDS sized for k.
typedef float img_f4 __attribute__((ext_vector_type(4)));

template <bool ACC>
__global__ void __launch_bounds__(kImgThreads) k_img_assign(ImgArgs a) {
  static_assert(kImgThreads % 64 == 0 && kImgAssignBlocks % kImgThreads == 0,
                "whole waves of blocks, whole rounds");
  extern __shared__ __align__(16) float img_lds[];
  const int k = a.k;
  float *cbk = img_lds;                          // k x 16
  float *hc = cbk + k * 16;                      // k: |c|^2 / 2
  float *sorted = hc + ((k + 3) & ~3);           // ACC: 256 x 16, in cluster order
  int *wcnt = (int *)(sorted + (ACC ? 16 * kImgThreads : 0));  // ACC: 4 x k per-wave counts
  int *off = wcnt + 4 * k;                       // ACC: k + 1 run offsets
  const bool lsum = k <= kImgLdsSumK;            // ACC: running sums in LDS
  float *gsum = (float *)(off + ((k + 4) & ~3)); // ACC, lsum: k x 17 running sums
  const int64_t img = blockIdx.y;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, col = lane & 15, g4 = lane >> 4;
  const float *gcb = a.codebook + img * (int64_t)k * 16;
  for (int i = tid; i < k * 16; i += kImgThreads) cbk[i] = gcb[i];
  if constexpr (ACC) {
    for (int i = tid; i < 4 * k; i += kImgThreads) wcnt[i] = 0;
  }
  __syncthreads();
  for (int c = tid; c < k; c += kImgThreads) {
    float h = 0.f;
#pragma unroll
    for (int t = 0; t < 16; ++t) h = __builtin_fmaf(cbk[16 * c + t], cbk[16 * c + t], h);
    hc[c] = 0.5f * h;
  }
  __syncthreads();
  float *part = a.part + (img * a.agroups + blockIdx.x) * (int64_t)k * 17;
  const int64_t base = (int64_t)blockIdx.x * kImgAssignBlocks;
  for (int rd = 0; rd < kImgAssignBlocks / kImgThreads; ++rd) {
    const int64_t r0 = base + (int64_t)rd * kImgThreads;  // the round's first block
    if (r0 >= a.nb) break;                                // uniform over the workgroup
    const int64_t b0 = r0 + (tid - lane);                 // the wave's first block
    const int64_t b = b0 + lane;
    const int64_t gb = img * a.nb + b;
    const bool in = b < a.nb;
    const bool pat = in && a.act[gb] >= a.tau;
    // B operands: block b0 + 16 nt + col, components 4 g4 .. 4 g4 + 3
    float4 vb[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int64_t bb = b0 + 16 * nt + col;
      vb[nt] = bb < a.nb ? reinterpret_cast<const float4 *>(a.dev + 16 * (img * a.nb + bb))[g4]
                         : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    float bv[4];
    int bi[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) bv[nt] = -3.4e38f, bi[nt] = 0;
    for (int m0 = 0; m0 < k; m0 += 16) {
      const int ca = m0 + col;  // this lane's A row
      const float4 va = ca < k ? reinterpret_cast<const float4 *>(cbk + 16 * ca)[g4]
                               : make_float4(0.f, 0.f, 0.f, 0.f);
      img_f4 init;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int cr = m0 + 4 * g4 + r;
        init[r] = cr < k ? -hc[cr] : -3.4e38f;
      }
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        img_f4 d = init;
        d = __builtin_amdgcn_mfma_f32_16x16x4f32(va.x, vb[nt].x, d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x4f32(va.y, vb[nt].y, d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x4f32(va.z, vb[nt].z, d, 0, 0, 0);
        d = __builtin_amdgcn_mfma_f32_16x16x4f32(va.w, vb[nt].w, d, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (d[r] > bv[nt]) {
            bv[nt] = d[r];
            bi[nt] = m0 + 4 * g4 + r;
          }
        }
      }
    }
    // the four lanes of a column (g4 = 0..3) hold interleaved rows: combine
    int best = 0;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
#pragma unroll
      for (int x = 16; x <= 32; x *= 2) {
        const float ov = __shfl_xor(bv[nt], x, 64);
        const int oi = __shfl_xor(bi[nt], x, 64);
        if (ov > bv[nt] || (ov == bv[nt] && oi < bi[nt])) {
          bv[nt] = ov;
          bi[nt] = oi;
        }
      }
      if (nt == g4) best = bi[nt];  // block b0 + 16 nt + col is this lane's own
    }
    if constexpr (ACC) {
      int *wc = wcnt;
      const int rank = pat ? atomicAdd(&wc[wave * k + best], 1) : 0;
      __syncthreads();
      if (tid < 64) {
        // exclusive scan of the k <= 256 counts by the first wave, four per lane
        int loc[4], run = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = 4 * tid + q;
          loc[q] = run;
          run += i < k ? wc[i] + wc[k + i] + wc[2 * k + i] + wc[3 * k + i] : 0;
        }
        int incl = run;
        for (int d = 1; d < 64; d *= 2) {
          const int o = __shfl_up(incl, d, 64);
          if (tid >= d) incl += o;
        }
        const int base_off = incl - run;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = 4 * tid + q;
          if (i < k) off[i] = base_off + loc[q];
        }
        if (tid == 63) off[k] = incl;
      }
      __syncthreads();
      if (pat) {
        // the block's own deviation vector (the B operands hold other blocks')
        int pos = off[best] + rank;
        for (int w = 0; w < wave; ++w) pos += wc[w * k + best];
        const float4 *src = reinterpret_cast<const float4 *>(a.dev + 16 * gb);
        float4 *dst = reinterpret_cast<float4 *>(sorted + 16 * pos);
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[q] = src[q];
      }
      __syncthreads();
      for (int i = tid; i < k * 17; i += kImgThreads) {
        const int c = i / 17, t = i % 17;
        const int q0 = off[c], q1 = off[c + 1];
        float sum;
        if (t == 16) {
          sum = (float)(q1 - q0);
        } else {
          sum = 0.f;
          for (int q = q0; q < q1; ++q) sum += sorted[16 * q + t];
        }
        float *acc = lsum ? gsum : part;
        acc[i] = rd == 0 ? sum : acc[i] + sum;
      }
      // other waves read this wave's counters only before the barrier above;
      // the wave clears them before its next round's atomics
      for (int i = lane; i < k; i += 64) wc[wave * k + i] = 0;
      // the next round's scan and scatter overwrite off and sorted only after
      // its first barrier, which every thread reaches after these reads
    } else {
      if (in) a.code[gb] = pat ? best + 1 : 0;
    }
  }
  if constexpr (ACC) {
    if (lsum)  // each entry was last written by the thread that copies it
      for (int i = tid; i < k * 17; i += kImgThreads) part[i] = gsum[i];
  }
}

// Dynamic LDS of k_img_assign for k codewords.
size_t img_assign_lds_bytes(int k, bool accumulate) {
  const size_t f = (size_t)k * 16 + (size_t)((k + 3) & ~3);
  return sizeof(float) *
         (f + (accumulate ? 16 * kImgThreads + 4 * (size_t)k + ((k + 4) & ~3) +
                                (k <= kImgLdsSumK ? 17 * (size_t)k : 0)
                          : 0));
}

// New codewords: one workgroup per (codeword blockIdx.x, image blockIdx.y).
// Thread i adds the partials of groups i, i + 256, ... in order, then the 256
// thread sums are added in a fixed tree, so the result does not depend on
// scheduling; a codeword without blocks keeps its value.
__global__ void __launch_bounds__(256) k_img_update(ImgArgs a) {
  __shared__ float red[17][256];
  const int64_t img = blockIdx.y;
  const int c = blockIdx.x, tid = threadIdx.x;
  const int64_t K17 = (int64_t)a.k * 17;
  const float *part = a.part + img * a.agroups * K17 + 17 * c;
  float s[17];
#pragma unroll
  for (int t = 0; t < 17; ++t) s[t] = 0.f;
  for (int g = tid; g < a.agroups; g += 256) {
    const float *p = part + g * K17;
#pragma unroll
    for (int t = 0; t < 17; ++t) s[t] += p[t];
  }
#pragma unroll
  for (int t = 0; t < 17; ++t) red[t][tid] = s[t];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (tid < st) {
#pragma unroll
      for (int t = 0; t < 17; ++t) red[t][tid] += red[t][tid + st];
    }
    __syncthreads();
  }
  if (tid < 16) {
    const float n = red[16][0];
    if (n > 0.f) a.codebook[(img * a.k + c) * 16 + tid] = red[tid][0] / n;
  }
}

const void *img_kernel_front() { return (const void *)&k_img_front; }
const void *img_kernel_count() { return (const void *)&k_img_count; }
const void *img_kernel_scan() { return (const void *)&k_img_scan; }
const void *img_kernel_seed() { return (const void *)&k_img_seed; }
const void *img_kernel_assign(bool accumulate) {
  return accumulate ? (const void *)&k_img_assign<true> : (const void *)&k_img_assign<false>;
}
const void *img_kernel_update() { return (const void *)&k_img_update; }

}  // namespace dpfft
