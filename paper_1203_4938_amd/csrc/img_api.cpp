// C ABI of the image block compression (section III-B): validation,
// workspace layout and the launch sequence.
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dpfft.h"
#include "img.h"
#include "internal.h"

using namespace dpfft;

namespace {

struct WsLayout {
  size_t wgcount = 0, npat = 0, part = 0, total = 0;
};

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

int64_t groups_of(const img_desc_t *d, int64_t per) {
  const int64_t nb = (int64_t)(d->height / 4) * (d->width / 4);
  return (nb + per - 1) / per;
}

WsLayout layout(const img_desc_t *d) {
  WsLayout L;
  const int64_t g = groups_of(d, kImgBlocksPerGroup), ga = groups_of(d, kImgAssignBlocks);
  const int64_t B = d->batch;
  L.wgcount = 0;
  L.npat = align256(L.wgcount + sizeof(int32_t) * B * g);
  L.part = align256(L.npat + sizeof(int32_t) * B);
  L.total = align256(L.part + sizeof(float) * B * ga * d->k * 17);
  return L;
}

fft_status_t check_desc(const img_desc_t *d) {
  if (!d) return fail(FFT_E_INVALID, "desc is NULL");
  if (d->height <= 0 || d->width <= 0 || (d->height % 4) || (d->width % 4))
    return fail(FFT_E_INVALID, "image sides must be positive multiples of 4");
  if ((int64_t)d->height * d->width > (int64_t(1) << 30))
    return fail(FFT_E_UNSUPPORTED, "images above 2^30 pixels");
  if (d->batch < 0 || d->batch > 65535) return fail(FFT_E_INVALID, "batch must be in [0, 65535]");
  if (d->k < 1 || d->k > kImgMaxK) return fail(FFT_E_INVALID, "k must be in [1, 256]");
  if (d->iters < 0 || d->iters > 10000) return fail(FFT_E_INVALID, "iters must be in [0, 10000]");
  if (!isfinite(d->tau)) return fail(FFT_E_INVALID, "tau must be finite");
  if (d->flags & ~IMG_F_GRAPH) return fail(FFT_E_INVALID, "unknown img flags");
  return FFT_OK;
}

bool misaligned(const void *p, uintptr_t a) { return ((uintptr_t)p & (a - 1)) != 0; }

ImgArgs args_of(const img_desc_t *d) {
  ImgArgs a{};
  a.h = d->height;
  a.w = d->width;
  a.nb = (a.h / 4) * (a.w / 4);
  a.groups = (int32_t)groups_of(d, kImgBlocksPerGroup);
  a.agroups = (int32_t)groups_of(d, kImgAssignBlocks);
  a.k = d->k;
  a.tau = d->tau;
  return a;
}

hipError_t launch(const void *fn, dim3 grid, int threads, ImgArgs &a, hipStream_t s,
                  size_t lds = 0) {
  void *kargs[] = {(void *)&a};
  return hipLaunchKernel(fn, grid, dim3(threads), kargs, lds, s);
}

struct Launch {
  const void *fn;
  dim3 grid;
  int threads;
  size_t lds;
};

// The launches of steps (a)-(e), in order: front end, pattern counts, their
// scan, seeds, iters x (assignment with cluster sums, codebook update), codes.
std::vector<Launch> sequence(const img_desc_t *d, const ImgArgs &a) {
  const unsigned B = (unsigned)d->batch;
  const int64_t tiles = ((a.w + kImgTileW - 1) / kImgTileW) * ((a.h + kImgTileH - 1) / kImgTileH);
  const dim3 gb((unsigned)a.groups, B), ga((unsigned)a.agroups, B), gu((unsigned)a.k, B);
  std::vector<Launch> v;
  v.push_back({img_kernel_front(), dim3((unsigned)tiles, B), kImgThreads, 0});
  v.push_back({img_kernel_count(), gb, kImgBlocksPerGroup, 0});
  v.push_back({img_kernel_scan(), dim3(B), 256, 0});
  v.push_back({img_kernel_seed(), gb, kImgBlocksPerGroup, 0});
  for (int it = 0; it < d->iters; ++it) {
    v.push_back({img_kernel_assign(true), ga, kImgThreads, img_assign_lds_bytes(a.k, true)});
    v.push_back({img_kernel_update(), gu, 256, 0});
  }
  v.push_back({img_kernel_assign(false), ga, kImgThreads, img_assign_lds_bytes(a.k, false)});
  return v;
}

// Instantiated graphs of the sequence, most recent first (IMG_F_GRAPH).
struct GraphKey {
  img_desc_t d;
  const void *ptr[11];
  hipStream_t stream;
  int device;
  bool operator==(const GraphKey &o) const {
    return d.height == o.d.height && d.width == o.d.width && d.batch == o.d.batch &&
           d.k == o.d.k && d.iters == o.d.iters && d.tau == o.d.tau &&
           std::equal(ptr, ptr + 11, o.ptr) && stream == o.stream && device == o.device;
  }
};
constexpr size_t kMaxImgGraphs = 8;
struct CachedGraph {
  GraphKey key;
  hipGraphExec_t exec;
  hipEvent_t done;  // recorded after every launch; an evicted graph waits on it
};
std::mutex g_mu;
std::vector<CachedGraph> g_graphs;

// launch a cached graph and record its completion (under g_mu, so that no
// other thread evicts it in between)
hipError_t launch_cached_locked(const CachedGraph &c, hipStream_t s) {
  hipError_t e = hipGraphLaunch(c.exec, s);
  if (e == hipSuccess) e = hipEventRecord(c.done, s);
  return e;
}

hipError_t run_graph(const GraphKey &key, const std::vector<Launch> &seq, ImgArgs &a,
                     hipStream_t s) {
  auto find = [&]() -> const CachedGraph * {
    for (size_t i = 0; i < g_graphs.size(); ++i)
      if (g_graphs[i].key == key) {
        std::rotate(g_graphs.begin(), g_graphs.begin() + i, g_graphs.begin() + i + 1);
        return &g_graphs[0];
      }
    return nullptr;
  };
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (const CachedGraph *c = find()) return launch_cached_locked(*c, s);
  }
  hipGraphExec_t exec = nullptr;
  {
    hipGraph_t g = nullptr;
    hipError_t e = hipGraphCreate(&g, 0);
    if (e != hipSuccess) return e;
    hipGraphNode_t prev = nullptr;
    for (const Launch &l : seq) {
      void *kargs[] = {(void *)&a};  // copied into the node
      hipKernelNodeParams p{};
      p.func = const_cast<void *>(l.fn);
      p.gridDim = l.grid;
      p.blockDim = dim3(l.threads);
      p.sharedMemBytes = (unsigned)l.lds;
      p.kernelParams = kargs;
      hipGraphNode_t node = nullptr;
      e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &p);
      if (e != hipSuccess) break;
      prev = node;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return e;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (const CachedGraph *other = find()) {  // built meanwhile by another thread
    (void)hipGraphExecDestroy(exec);
    return launch_cached_locked(*other, s);
  }
  hipEvent_t done = nullptr;
  hipError_t e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
  if (e == hipSuccess && g_graphs.size() >= kMaxImgGraphs) {
    // the evicted graph may still be running: wait for its last launch (the
    // event stays valid if the caller has destroyed the stream since)
    const CachedGraph &old = g_graphs.back();
    e = hipEventSynchronize(old.done);
    if (e == hipSuccess) {
      (void)hipGraphExecDestroy(old.exec);
      (void)hipEventDestroy(old.done);
      g_graphs.pop_back();
    }
  }
  if (e != hipSuccess) {
    (void)hipGraphExecDestroy(exec);
    if (done) (void)hipEventDestroy(done);
    return e;
  }
  g_graphs.insert(g_graphs.begin(), CachedGraph{key, exec, done});
  return launch_cached_locked(g_graphs.front(), s);
}

}  // namespace

extern "C" {

size_t img_workspace_bytes(const img_desc_t *desc) {
  if (check_desc(desc) != FFT_OK) return 0;
  return layout(desc).total;
}

fft_status_t img_compress(const img_desc_t *desc, const uint8_t *rgb, const img_out_t *out,
                          void *workspace, void *hip_stream) {
  fft_status_t st = check_desc(desc);
  if (st != FFT_OK) return st;
  if (!out) return fail(FFT_E_INVALID, "out is NULL");
  if (desc->batch == 0) return FFT_OK;
  if (!rgb || !out->y || !out->cb || !out->cr || !out->mean || !out->act || !out->dev ||
      !out->codebook || !out->code || !workspace)
    return fail(FFT_E_INVALID, "a buffer is NULL");
  if (misaligned(rgb, 4) || misaligned(out->y, 16) || misaligned(out->cb, 8) ||
      misaligned(out->cr, 8) || misaligned(out->mean, 4) || misaligned(out->act, 4) ||
      misaligned(out->dev, 16) || misaligned(out->codebook, 4) || misaligned(out->code, 4) ||
      misaligned(workspace, 256))
    return fail(FFT_E_INVALID,
                "misaligned buffer (y and dev 16 bytes, cb and cr 8, workspace 256, rgb and others 4)");
  const WsLayout L = layout(desc);
  ImgArgs a = args_of(desc);
  a.rgb = rgb;
  a.y = out->y;
  a.cb = out->cb;
  a.cr = out->cr;
  a.mean = out->mean;
  a.act = out->act;
  a.dev = out->dev;
  a.codebook = out->codebook;
  a.code = out->code;
  char *ws = (char *)workspace;
  a.wgcount = (int32_t *)(ws + L.wgcount);
  a.npat = (int32_t *)(ws + L.npat);
  a.part = (float *)(ws + L.part);
  hipStream_t s = (hipStream_t)hip_stream;
  const std::vector<Launch> seq = sequence(desc, a);
  hipError_t e = hipSuccess;
  if (desc->flags & IMG_F_GRAPH) {
    GraphKey key{};
    key.d = *desc;
    const void *ptrs[11] = {rgb, out->y, out->cb, out->cr, out->mean, out->act,
                            out->dev, out->codebook, out->code, workspace, nullptr};
    std::copy(ptrs, ptrs + 11, key.ptr);
    key.stream = s;
    e = hipGetDevice(&key.device);
    if (e == hipSuccess) e = run_graph(key, seq, a, s);
  } else {
    for (const Launch &l : seq) {
      e = launch(l.fn, l.grid, l.threads, a, s, l.lds);
      if (e != hipSuccess) break;
    }
  }
  if (e != hipSuccess) return fail(FFT_E_DEVICE, std::string("launch: ") + hipGetErrorString(e));
  return FFT_OK;
}

fft_status_t img_encode(const img_desc_t *desc, const float *dev, const float *act,
                        const float *codebook, int32_t *code, void *hip_stream) {
  fft_status_t st = check_desc(desc);
  if (st != FFT_OK) return st;
  if (desc->batch == 0) return FFT_OK;
  if (!dev || !act || !codebook || !code) return fail(FFT_E_INVALID, "a buffer is NULL");
  if (misaligned(dev, 16) || misaligned(act, 4) || misaligned(codebook, 4) || misaligned(code, 4))
    return fail(FFT_E_INVALID, "misaligned buffer (dev 16 bytes, others 4)");
  ImgArgs a = args_of(desc);
  a.dev = const_cast<float *>(dev);
  a.act = const_cast<float *>(act);
  a.codebook = const_cast<float *>(codebook);
  a.code = code;
  const hipError_t e = launch(img_kernel_assign(false), dim3((unsigned)a.agroups, (unsigned)desc->batch),
                              kImgThreads, a, (hipStream_t)hip_stream, img_assign_lds_bytes(a.k, false));
  if (e != hipSuccess) return fail(FFT_E_DEVICE, std::string("launch: ") + hipGetErrorString(e));
  return FFT_OK;
}

}  // extern "C"
