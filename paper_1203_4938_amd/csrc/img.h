// Image block compression: host view of the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpfft {

constexpr int kImgTileW = 64;         // pixels per front-end tile, x
constexpr int kImgTileH = 16;         // pixels per front-end tile, y
constexpr int kImgThreads = 256;
constexpr int kImgBlocksPerGroup = 256;  // 4x4 blocks per workgroup of the block-list kernels
constexpr int kImgAssignBlocks = 1024;   // 4x4 blocks per workgroup of the assignment
constexpr int kImgLdsSumK = 128;         // up to this k the assignment sums in LDS
constexpr int kImgMaxK = 256;

struct ImgArgs {
  const uint8_t *rgb;  // batch x h x w x 3
  float *y, *cb, *cr, *mean, *act, *dev, *codebook;
  int32_t *code;
  int32_t *wgcount;    // per image: per block group, pattern blocks (then their offsets)
  int32_t *npat;       // per image: pattern blocks
  float *part;         // per image, per assignment group: k x 17 partial sums and counts
  int64_t h, w;        // pixels
  int64_t nb;          // blocks per image ((h/4) (w/4))
  int32_t groups;      // block groups per image (ceil(nb / 256))
  int32_t agroups;     // assignment groups per image (ceil(nb / 1024))
  int32_t k;
  float tau;
};

// Kernel entry points, each launched with a grid of (tiles, groups,
// assignment groups or codewords, batch); k_img_assign takes
// img_assign_lds_bytes of dynamic LDS.
const void *img_kernel_front();
const void *img_kernel_count();
const void *img_kernel_scan();
const void *img_kernel_seed();
const void *img_kernel_assign(bool accumulate);
const void *img_kernel_update();
size_t img_assign_lds_bytes(int k, bool accumulate);

}  // namespace dpfft
