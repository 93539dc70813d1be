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
  int n_phase1 = 0;  // queue entries of the first launch; the rest belong to the second
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

  // the two persistent launches: (first queue entry, entries, ticket slot)
  void phase(int k, RaggedArgs &r) const {
    r.direct = 0;
    r.first_item = 0;
    if (k == 0) {
      r.order = a.order;
      r.nitems = n_phase1;
      r.ticket = 0;
    } else {
      r.order = a.order + n_phase1;
      r.nitems = nitems - n_phase1;
      r.ticket = 2;
    }
  }

  hipError_t launch_queue(const ExecCtx &ctx) const {
    RaggedArgs r = args_for(ctx);
    int nstate = 4;
    uint32_t *state = r.state;
    void *rargs[] = {(void *)&state, (void *)&nstate};
    hipError_t e = hipLaunchKernel(ragged_reset_kernel(), dim3(1), dim3(64), rargs, 0, ctx.stream);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
      phase(k, r);
      if (r.nitems == 0) continue;
      const float2 *s = (const float2 *)ctx.in;
      float2 *d = (float2 *)ctx.out;
      void *kargs[] = {(void *)&s, (void *)&d, (void *)&r};
      e = hipLaunchKernel(ragged_kernel(ctx.inverse), dim3((unsigned)std::min(resident, r.nitems)),
                          dim3(kRaggedThreads), kargs, (size_t)lds_bytes, ctx.stream);
    }
    return e;
  }

  // The queue launches (ticket reset by a fill kernel, then the two
  // persistent launches) as a three-node graph, built once per (buffers,
  // direction, stream).
  hipError_t launch_graph(const ExecCtx &ctx) const {
    GraphKey key{ctx.in, ctx.out, ctx.ws, ctx.inverse, ctx.stream};
    hipGraphExec_t exec = nullptr;
    {
      std::lock_guard<std::mutex> lk(mu);
      auto it = graphs.find(key);
      if (it != graphs.end()) exec = it->second;
    }
    if (!exec) {
      RaggedArgs r0 = args_for(ctx), r1 = args_for(ctx);
      phase(0, r0);
      phase(1, r1);
      int nstate = 4;
      uint32_t *state = r0.state;
      const float2 *s = (const float2 *)ctx.in;
      float2 *d = (float2 *)ctx.out;
      void *rargs[] = {(void *)&state, (void *)&nstate};
      void *k0[] = {(void *)&s, (void *)&d, (void *)&r0};
      void *k1[] = {(void *)&s, (void *)&d, (void *)&r1};
      hipGraph_t g = nullptr;
      hipError_t e = hipGraphCreate(&g, 0);
      if (e != hipSuccess) return e;
      hipKernelNodeParams pr{};
      pr.func = const_cast<void *>(ragged_reset_kernel());
      pr.gridDim = dim3(1);
      pr.blockDim = dim3(64);
      pr.kernelParams = rargs;
      hipGraphNode_t prev = nullptr;
      e = hipGraphAddKernelNode(&prev, g, nullptr, 0, &pr);
      void **kp[2] = {k0, k1};
      const RaggedArgs *rp[2] = {&r0, &r1};
      for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        if (rp[k]->nitems == 0) continue;
        hipKernelNodeParams p{};
        p.func = const_cast<void *>(ragged_kernel(ctx.inverse));
        p.gridDim = dim3((unsigned)std::min(resident, rp[k]->nitems));
        p.blockDim = dim3(kRaggedThreads);
        p.sharedMemBytes = (unsigned)lds_bytes;
        p.kernelParams = kp[k];
        hipGraphNode_t node = nullptr;
        e = hipGraphAddKernelNode(&node, g, &prev, 1, &p);
        prev = node;
      }
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
    return lds_bytes <= kRaggedLdsBytes && resident > 0 && ragged_kernel(false) &&
           ragged_kernel(true);
  }
};

namespace {

// LDS elements a tile of `C` lines of this size needs in each layout
int64_t tile_lds(const MixedPlan &mp, int C, int map) {
  if (map == ELEM_FAST) return (int64_t)C * mp.pitch;
  const int64_t u = (int64_t)mp.L * C;
  return u + (u >> 4) + 1;
}

int64_t tw_elems(const MixedPlan &mp) {
  return (1 << mp.tw2_shift) + (mp.L + (1 << mp.tw2_shift) - 1) / (1 << mp.tw2_shift);
}

constexpr int64_t kBudget = kRaggedLdsBytes / (int64_t)sizeof(float2);

// the largest length one ragged workgroup transforms in a single pass
bool fits_single(const MixedPlan &mp) {
  return mp.T <= kRaggedThreads && tile_lds(mp, 1, ELEM_FAST) + tw_elems(mp) <= kBudget;
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
    MixedPlan probe{};
    if (!mixed_radices(L, &probe))
      return fail(FFT_E_UNSUPPORTED, "no radix plan for ragged size " + std::to_string(L));
    if (fits_single(probe)) {
      const int zi = size_of(L);
      const MixedPlan &mp = plans[L];
      int C = std::max(1, kRaggedThreads / mp.T);
      while (C > 1 && tile_lds(mp, C, ELEM_FAST) + tw_elems(mp) > kBudget) --C;
      const int first = (int)items.size();
      for (size_t s0 = 0; s0 < sigs.size(); s0 += C) {
        const int c = (int)std::min<size_t>(C, sigs.size() - s0);
        const int64_t data = tile_lds(mp, c, ELEM_FAST);
        RaggedItem it{RK_SINGLE, zi, c, (int32_t)siglist.size(), 0, 0, 0, 0, -1, (int32_t)data};
        for (int k = 0; k < c; ++k) siglist.push_back(sigs[s0 + k]);
        items.push_back(it);
        cost.push_back((int64_t)(c * L * lg(L)));
        lds_need = std::max(lds_need, data + tw_elems(mp));
      }
      st->ranges.push_back({first, (int)items.size() - first});
      ++nsingle_sizes;
      continue;
    }
    // four-step: L = n1 * n2
    const int64_t n1 = split_factor(L), n2 = L / n1;
    const int z1 = size_of(n1), z2 = size_of(n2);
    if (z1 < 0 || z2 < 0) return fail(FFT_E_UNSUPPORTED, "no radix plan for ragged size " + std::to_string(L));
    const MixedPlan &m1 = plans[n1], &m2 = plans[n2];
    if (!fits_single(m1) || !fits_single(m2))
      return fail(FFT_E_UNSUPPORTED, "ragged size too long for two passes: " + std::to_string(L));
    int CA = std::max(1, kRaggedThreads / m1.T), CB = std::max(1, kRaggedThreads / m2.T);
    while (CA > 1 && tile_lds(m1, CA, LINE_FAST) + tw_elems(m1) > kBudget) --CA;
    auto rows_lds = [&](int c) { return std::max(tile_lds(m2, c, ELEM_FAST), tile_lds(m2, c, LINE_FAST)); };
    while (CB > 1 && rows_lds(CB) + tw_elems(m2) > kBudget) --CB;
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
        const int64_t data = tile_lds(m1, c, LINE_FAST);
        items.push_back(RaggedItem{RK_COLUMNS, z1, c, s, (int32_t)f, (int32_t)n1, (int32_t)n2, 0, b,
                                   (int32_t)data});
        cost.push_back((int64_t)(c * n1 * lg(n1)));
        lds_need = std::max(lds_need, data + tw_elems(m1));
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
        const int64_t data = rows_lds(c);
        items.push_back(RaggedItem{RK_ROWS, z2, c, s, (int32_t)f, (int32_t)n1, (int32_t)n2, need, b,
                                   (int32_t)data});
        cost.push_back((int64_t)(c * n2 * lg(n2)));
        lds_need = std::max(lds_need, data + tw_elems(m2));
      }
    }
    st->ranges.push_back({first_rows, (int)items.size() - first_rows});
    ++nbig_sizes;
  }

  // queue order: the first launch takes single-pass and column items, the
  // second the row items, each by decreasing cost (largest first keeps the
  // tail short)
  std::vector<int32_t> order(items.size());
  for (size_t i = 0; i < items.size(); ++i) order[i] = (int32_t)i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
    const bool rx = items[x].kind == RK_ROWS, ry = items[y].kind == RK_ROWS;
    if (rx != ry) return !rx;
    return cost[x] > cost[y];
  });

  st->nitems = (int)items.size();
  st->n_phase1 = 0;
  for (const auto &it : items)
    if (it.kind != RK_ROWS) ++st->n_phase1;
  st->nbig = (int)bigs.size();
  st->nsizes = (int)rs.size();
  st->lds_bytes = (int)(lds_need * (int64_t)sizeof(float2));
  st->resident = resident_for(st->lds_bytes, kRaggedThreads);
  if (rs.empty()) rs.push_back(RaggedSize{});
  if (items.empty()) items.push_back(RaggedItem{});
  if (lds_need * (int64_t)sizeof(float2) > kRaggedLdsBytes)
    return fail(FFT_E_INTERNAL, "ragged plan exceeds its LDS budget");
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

  const int64_t state_words = 4;
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
                     : std::string("persistent queues (") + std::to_string(st->n_phase1) + " + " +
                           std::to_string(st->nitems - st->n_phase1) + " items), grid=" +
                           std::to_string(std::min(st->resident, st->nitems)))
    << (st->graph && !st->per_size ? " in a HIP graph" : "") << " threads=" << kRaggedThreads
    << " lds=" << st->lds_bytes << "B";
  st->summary = o.str();
  P->variant = st->per_size ? "ragged per-length launches" : "ragged persistent";
  P->steps.push_back(std::move(st));
  return FFT_OK;
}
