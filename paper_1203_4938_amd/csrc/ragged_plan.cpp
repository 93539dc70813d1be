// Plan builder and launcher of ragged batches.
#include <algorithm>
#include <cmath>
#include <complex>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <tuple>
#include <vector>

#include "internal.h"
#include "plan.h"
#include "ragged.h"
#include "twiddle.h"

namespace dpfft {

namespace {

constexpr int kRaggedThreads = 1024;
constexpr int kSpinLimit = 1 << 22;  // s_sleep(2) rounds: far above any real wait

struct GraphKey {
  const void *in;
  void *out, *ws;
  bool inverse;
  hipStream_t stream;
  bool operator<(const GraphKey &o) const {
    return std::tie(in, out, ws, inverse, stream) < std::tie(o.in, o.out, o.ws, o.inverse, o.stream);
  }
};

}  // namespace

struct RaggedStep : Step {
  RaggedArgs a{};
  size_t sizes_off = 0, items_off = 0, order_off = 0, siglist_off = 0, offsets_off = 0, bigs_off = 0;
  int nitems = 0, nbig = 0, nsizes = 0;
  int lds_bytes = 0, resident = 0;
  int64_t state_elems = 0;  // workspace float2 elements taken by the state words
  int64_t max_elem = -1;    // largest element index of in/out touched
  int64_t ws_elems = 0;     // workspace elements for four-step intermediates
  bool graph = false, per_size = false;
  std::vector<std::pair<int, int>> ranges;  // per-size mode: (first item, count)
  std::string summary;
  mutable std::mutex mu;
  mutable std::map<GraphKey, hipGraphExec_t> graphs;

  ~RaggedStep() override {
    for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
  }

  void bind(const float2 *tables) override {
    const char *base = reinterpret_cast<const char *>(tables);
    a.tables = tables;
    a.sizes = reinterpret_cast<const RaggedSize *>(base + sizes_off * sizeof(float2));
    a.items = reinterpret_cast<const RaggedItem *>(base + items_off * sizeof(float2));
    a.order = reinterpret_cast<const int32_t *>(base + order_off * sizeof(float2));
    a.siglist = reinterpret_cast<const int32_t *>(base + siglist_off * sizeof(float2));
    a.offsets = reinterpret_cast<const int64_t *>(base + offsets_off * sizeof(float2));
    a.bigs = reinterpret_cast<const RaggedBig *>(base + bigs_off * sizeof(float2));
    a.spin_limit = kSpinLimit;
  }

  RaggedArgs args_for(const ExecCtx &ctx) const {
    RaggedArgs r = a;
    r.state = reinterpret_cast<uint32_t *>(ctx.ws);
    r.ws = reinterpret_cast<float2 *>(ctx.ws) + state_elems;
    return r;
  }

  hipError_t launch_direct(const ExecCtx &ctx) const {
    RaggedArgs r = args_for(ctx);
    r.direct = 1;
    const void *fn = ragged_kernel(ctx.inverse);
    for (const auto &rg : ranges) {
      r.first_item = rg.first;
      r.nitems = rg.second;
      const float2 *s = (const float2 *)ctx.in;
      float2 *d = (float2 *)ctx.out;
      void *kargs[] = {(void *)&s, (void *)&d, (void *)&r};
      hipError_t e = hipLaunchKernel(fn, dim3((unsigned)rg.second), dim3(kRaggedThreads), kargs,
                                     (size_t)lds_bytes, ctx.stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }

  hipError_t launch_queue(const ExecCtx &ctx) const {
    RaggedArgs r = args_for(ctx);
    r.direct = 0;
    r.first_item = 0;
    r.nitems = nitems;
    int nstate = 2 + nbig;
    uint32_t *state = r.state;
    void *rargs[] = {(void *)&state, (void *)&nstate};
    hipError_t e = hipLaunchKernel(ragged_reset_kernel(), dim3(1), dim3(256), rargs, 0, ctx.stream);
    if (e != hipSuccess) return e;
    const float2 *s = (const float2 *)ctx.in;
    float2 *d = (float2 *)ctx.out;
    void *kargs[] = {(void *)&s, (void *)&d, (void *)&r};
    return hipLaunchKernel(ragged_kernel(ctx.inverse), dim3((unsigned)std::min(resident, nitems)),
                           dim3(kRaggedThreads), kargs, (size_t)lds_bytes, ctx.stream);
  }

  // The queue launch (state reset by a fill kernel, then the persistent
  // kernel) as a two-node graph, built once per (buffers, direction, stream).
  hipError_t launch_graph(const ExecCtx &ctx) const {
    GraphKey key{ctx.in, ctx.out, ctx.ws, ctx.inverse, ctx.stream};
    hipGraphExec_t exec = nullptr;
    {
      std::lock_guard<std::mutex> lk(mu);
      auto it = graphs.find(key);
      if (it != graphs.end()) exec = it->second;
    }
    if (!exec) {
      RaggedArgs r = args_for(ctx);
      r.direct = 0;
      r.first_item = 0;
      r.nitems = nitems;
      int nstate = 2 + nbig;
      uint32_t *state = r.state;
      const float2 *s = (const float2 *)ctx.in;
      float2 *d = (float2 *)ctx.out;
      void *rargs[] = {(void *)&state, (void *)&nstate};
      void *kargs[] = {(void *)&s, (void *)&d, (void *)&r};
      hipGraph_t g = nullptr;
      hipError_t e = hipGraphCreate(&g, 0);
      if (e != hipSuccess) return e;
      hipKernelNodeParams p0{};
      p0.func = const_cast<void *>(ragged_reset_kernel());
      p0.gridDim = dim3(1);
      p0.blockDim = dim3(256);
      p0.sharedMemBytes = 0;
      p0.kernelParams = rargs;
      hipKernelNodeParams p1{};
      p1.func = const_cast<void *>(ragged_kernel(ctx.inverse));
      p1.gridDim = dim3((unsigned)std::min(resident, nitems));
      p1.blockDim = dim3(kRaggedThreads);
      p1.sharedMemBytes = (unsigned)lds_bytes;
      p1.kernelParams = kargs;
      hipGraphNode_t n0 = nullptr, n1 = nullptr;
      e = hipGraphAddKernelNode(&n0, g, nullptr, 0, &p0);
      if (e == hipSuccess) e = hipGraphAddKernelNode(&n1, g, &n0, 1, &p1);
      if (e == hipSuccess) e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return e;
      std::lock_guard<std::mutex> lk(mu);
      auto it = graphs.find(key);
      if (it != graphs.end()) {
        (void)hipGraphExecDestroy(exec);
        exec = it->second;
      } else {
        graphs[key] = exec;
      }
    }
    return hipGraphLaunch(exec, ctx.stream);
  }

  hipError_t launch(const ExecCtx &ctx) const override {
    if (nitems == 0) return hipSuccess;
    if (per_size) return launch_direct(ctx);
    return graph ? launch_graph(ctx) : launch_queue(ctx);
  }

  std::string describe() const override { return summary; }

  void extent(int64_t &max_in, int64_t &max_out, int &src_id, int &dst_id) const override {
    max_in = max_out = max_elem;
    src_id = BUF_IN;
    dst_id = BUF_OUT;
  }

  bool valid() const override {
    return lds_bytes <= kLdsBytes && resident > 0 && ragged_kernel(false) && ragged_kernel(true);
  }
};

namespace {

// LDS elements a tile of `C` lines of this size needs in each layout
int64_t tile_lds(const MixedPlan &mp, int C, int map) {
  if (map == ELEM_FAST) return (int64_t)C * mp.pitch;
  const int64_t u = (int64_t)mp.L * C;
  return u + (u >> 4) + 1;
}

}  // namespace

}  // namespace dpfft

using namespace dpfft;

fft_status_t plan_ragged(dpfft_plan_s *P, const int64_t *sizes, const int64_t *offsets) {
  const int64_t count = P->batch;
  P->rsizes.assign(sizes, sizes + count);
  P->roffsets.resize(count);
  int64_t acc = 0;
  for (int64_t i = 0; i < count; ++i) {
    P->roffsets[i] = offsets ? offsets[i] : acc;
    acc += sizes[i];
  }
  int64_t max_elem = -1;
  for (int64_t i = 0; i < count; ++i) max_elem = std::max(max_elem, P->roffsets[i] + sizes[i] - 1);
  P->io_elems = max_elem + 1;

  auto st = std::make_unique<RaggedStep>();
  st->graph = (P->flags & FFT_F_GRAPH) != 0;
  st->per_size = (P->flags & FFT_F_PER_SIZE) != 0;
  st->max_elem = max_elem;

  std::vector<RaggedSize> rs;
  std::map<int64_t, int> size_idx;
  std::map<int64_t, MixedPlan> plans;
  auto size_of = [&](int64_t L) -> int {
    auto it = size_idx.find(L);
    if (it != size_idx.end()) return it->second;
    MixedPlan mp{};
    if (!mixed_radices(L, &mp)) return -1;
    RaggedSize z{};
    z.L = mp.L;
    z.P = mp.P;
    z.T = mp.T;
    z.pitch = mp.pitch;
    z.tw2_shift = mp.tw2_shift;
    z.codes = mp.codes;
    std::vector<std::complex<double>> lo, hi;
    fourstep_tables(L, mp.tw2_shift, lo, hi);
    lo.insert(lo.end(), hi.begin(), hi.end());
    z.tw2_off = (int64_t)P->tables.add(lo);
    rs.push_back(z);
    plans[L] = mp;
    return size_idx[L] = (int)rs.size() - 1;
  };

  std::map<int64_t, std::vector<int32_t>> by_size;
  for (int64_t i = 0; i < count; ++i) by_size[sizes[i]].push_back((int32_t)i);

  std::vector<RaggedItem> items;
  std::vector<int32_t> siglist;
  std::vector<RaggedBig> bigs;
  std::vector<int64_t> cost;
  int64_t lds_need = 1, ws = 0;
  int nbig_sizes = 0, nsingle_sizes = 0;
  auto lg = [](int64_t L) { return std::max(1.0, std::log2((double)L)); };

  for (const auto &kv : by_size) {
    const int64_t L = kv.first;
    const auto &sigs = kv.second;
    if (L <= kSinglePassMax) {
      const int zi = size_of(L);
      if (zi < 0) return fail(FFT_E_UNSUPPORTED, "no radix plan for ragged size " + std::to_string(L));
      const MixedPlan &mp = plans[L];
      int C = std::max(1, kRaggedThreads / mp.T);
      while (C > 1 && tile_lds(mp, C, ELEM_FAST) * (int64_t)sizeof(float2) > kLdsBytes) --C;
      const int first = (int)items.size();
      for (size_t s0 = 0; s0 < sigs.size(); s0 += C) {
        const int c = (int)std::min<size_t>(C, sigs.size() - s0);
        RaggedItem it{RK_SINGLE, zi, c, (int32_t)siglist.size(), 0, 0, 0, 0, -1, 0};
        for (int k = 0; k < c; ++k) siglist.push_back(sigs[s0 + k]);
        items.push_back(it);
        cost.push_back((int64_t)(c * L * lg(L)));
        lds_need = std::max(lds_need, tile_lds(mp, c, ELEM_FAST));
      }
      st->ranges.push_back({first, (int)items.size() - first});
      ++nsingle_sizes;
      continue;
    }
    // four-step: L = n1 * n2
    const int64_t n1 = split_factor(L), n2 = L / n1;
    if (n2 > kSinglePassMax)
      return fail(FFT_E_UNSUPPORTED, "no two-factor split of ragged size " + std::to_string(L));
    const int z1 = size_of(n1), z2 = size_of(n2);
    if (z1 < 0 || z2 < 0) return fail(FFT_E_UNSUPPORTED, "no radix plan for ragged size " + std::to_string(L));
    const MixedPlan &m1 = plans[n1], &m2 = plans[n2];
    int CA = std::min(16, kRaggedThreads / m1.T), CB = std::min(16, kRaggedThreads / m2.T);
    while (CA > 1 && tile_lds(m1, CA, LINE_FAST) * (int64_t)sizeof(float2) > kLdsBytes) --CA;
    while (CB > 1 && std::max(tile_lds(m2, CB, ELEM_FAST), tile_lds(m2, CB, LINE_FAST)) *
                             (int64_t)sizeof(float2) > kLdsBytes)
      --CB;
    std::vector<std::complex<double>> lo, hi;
    int lgL = 0;
    while ((int64_t(1) << lgL) < L) ++lgL;
    const int shift = (lgL + 1) / 2;
    fourstep_tables(L, shift, lo, hi);
    const int64_t lo_off = (int64_t)P->tables.add(lo), hi_off = (int64_t)P->tables.add(hi);
    const int first_cols = (int)items.size();
    std::vector<std::pair<int, int64_t>> big_of;  // (big index, need)
    for (int32_t s : sigs) {
      const int b = (int)bigs.size();
      bigs.push_back(RaggedBig{ws, lo_off, hi_off, shift, 0});
      ws += L;
      int need = 0;
      for (int64_t f = 0; f < n2; f += CA, ++need) {
        const int c = (int)std::min<int64_t>(CA, n2 - f);
        items.push_back(RaggedItem{RK_COLUMNS, z1, c, s, (int32_t)f, (int32_t)n1, (int32_t)n2, 0, b, 0});
        cost.push_back((int64_t)(c * n1 * lg(n1)));
        lds_need = std::max(lds_need, tile_lds(m1, c, LINE_FAST));
      }
      big_of.push_back({b, need});
    }
    st->ranges.push_back({first_cols, (int)items.size() - first_cols});
    const int first_rows = (int)items.size();
    size_t k = 0;
    for (int32_t s : sigs) {
      const int b = big_of[k].first;
      const int need = (int)big_of[k].second;
      ++k;
      for (int64_t f = 0; f < n1; f += CB) {
        const int c = (int)std::min<int64_t>(CB, n1 - f);
        items.push_back(RaggedItem{RK_ROWS, z2, c, s, (int32_t)f, (int32_t)n1, (int32_t)n2, need, b, 0});
        cost.push_back((int64_t)(c * n2 * lg(n2)));
        lds_need = std::max(lds_need, std::max(tile_lds(m2, c, ELEM_FAST), tile_lds(m2, c, LINE_FAST)));
      }
    }
    st->ranges.push_back({first_rows, (int)items.size() - first_rows});
    ++nbig_sizes;
  }

  // queue order: single-pass and column items by decreasing cost (largest
  // first keeps the tail short), then every row item, also by decreasing cost
  std::vector<int32_t> order(items.size());
  for (size_t i = 0; i < items.size(); ++i) order[i] = (int32_t)i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    const bool rx = items[x].kind == RK_ROWS, ry = items[y].kind == RK_ROWS;
    if (rx != ry) return !rx;
    return cost[x] > cost[y];
  });

  st->nitems = (int)items.size();
  st->nbig = (int)bigs.size();
  st->nsizes = (int)rs.size();
  st->lds_bytes = (int)(lds_need * (int64_t)sizeof(float2));
  st->resident = resident_for(st->lds_bytes, kRaggedThreads);
  if (rs.empty()) rs.push_back(RaggedSize{});
  if (items.empty()) items.push_back(RaggedItem{});
  if (siglist.empty()) siglist.push_back(0);
  if (bigs.empty()) bigs.push_back(RaggedBig{});
  if (order.empty()) order.push_back(0);
  st->sizes_off = P->tables.add_bytes(rs.data(), rs.size() * sizeof(RaggedSize));
  st->items_off = P->tables.add_bytes(items.data(), items.size() * sizeof(RaggedItem));
  st->order_off = P->tables.add_bytes(order.data(), order.size() * sizeof(int32_t));
  st->siglist_off = P->tables.add_bytes(siglist.data(), siglist.size() * sizeof(int32_t));
  st->offsets_off =
      P->tables.add_bytes(P->roffsets.data(), std::max<size_t>(1, P->roffsets.size()) * sizeof(int64_t));
  st->bigs_off = P->tables.add_bytes(bigs.data(), bigs.size() * sizeof(RaggedBig));

  const int64_t state_words = 2 + st->nbig;
  st->state_elems = ((state_words * 4 + 255) / 256) * 256 / (int64_t)sizeof(float2);
  st->ws_elems = ws;
  P->ws_bytes = (size_t)(st->state_elems + ws) * sizeof(float2);

  for (bool inv : {false, true})
    (void)hipFuncSetAttribute(ragged_kernel(inv), hipFuncAttributeMaxDynamicSharedMemorySize,
                              st->lds_bytes);

  std::ostringstream o;
  o << "ragged: " << count << " signals, " << nsingle_sizes << " single-pass lengths, "
    << nbig_sizes << " four-step lengths, " << st->nitems << " items, "
    << (st->per_size ? "one launch per length (" + std::to_string(st->ranges.size()) + " launches)"
                     : std::string("persistent queue, grid=") +
                           std::to_string(std::min(st->resident, st->nitems)))
    << (st->graph && !st->per_size ? " in a HIP graph" : "") << " threads=" << kRaggedThreads
    << " lds=" << st->lds_bytes << "B";
  st->summary = o.str();
  P->variant = st->per_size ? "ragged per-length launches" : "ragged persistent";
  P->steps.push_back(std::move(st));
  return FFT_OK;
}
