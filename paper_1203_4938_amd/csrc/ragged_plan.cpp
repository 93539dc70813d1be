// Plan builder and launcher of ragged batches.
#include <stdio.h>

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
#include "mixed_ct_plan.h"
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
  bool operator==(const GraphKey &o) const {
    return std::tie(in, out, ws, inverse, stream) == std::tie(o.in, o.out, o.ws, o.inverse, o.stream);
  }
};

// Instantiated graphs a plan keeps, most recently used first.  A caller that
// rotates buffers gets a new graph per buffer set; beyond this many the
// least recently used one is released once its last launch has completed
// (an event recorded after every launch: it stays valid if the caller has
// destroyed the stream since).
constexpr size_t kMaxGraphs = 8;

struct CachedGraph {
  GraphKey key;
  hipGraphExec_t exec;
  hipEvent_t done;
};

}  // namespace

struct RaggedStep : Step {
  RaggedArgs a{};
  size_t items_off = 0, sigoff_off = 0;
  int nitems = 0;
  // items [0, n_big): single-pass signals of the 1024-thread instance (first
  // launch); [n_big, n_phase1): the other single-pass signals and the column
  // tiles (second launch); [n_phase1, nitems): the row tiles (third launch)
  int n_big = 0;
  int n_phase1 = 0;
  int lds_bytes = 0, resident = 0;
  int lds_big = 0, resident_big = 0;
  int64_t max_elem = -1;    // largest element index of in/out touched
  int64_t ws_elems = 0;     // workspace elements for four-step intermediates
  bool graph = false, per_size = false;
  bool persistent = false;  // resident workgroups walk the item lists
  struct Range {
    int first, count;
    bool big;
  };
  std::vector<Range> ranges;  // per-size mode: one launch each
  std::string summary;
  mutable std::mutex mu;
  mutable std::vector<CachedGraph> graphs;  // most recent first

  // (fft_destroy: no execution of the plan is pending)
  ~RaggedStep() override {
    for (auto &g : graphs) {
      (void)hipGraphExecDestroy(g.exec);
      (void)hipEventDestroy(g.done);
    }
  }

  hipError_t prepare() const override {
    // dynamic LDS above the default 64 KB needs an explicit opt-in per
    // function; the attribute belongs to the function, not to this plan, so it
    // is set to the class's budget (a plan needing less must not lower it
    // under another plan that needs more)
    for (bool inv : {false, true}) {
      hipError_t e = hipFuncSetAttribute(ragged_kernel(inv, false),
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         kRaggedLdsBytes);
      if (e == hipSuccess && n_big > 0)
        e = hipFuncSetAttribute(ragged_kernel(inv, true),
                                hipFuncAttributeMaxDynamicSharedMemorySize, kRaggedBigLdsBytes);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }

  // the cached graph for `key`, moved to the front (nullptr if none)
  const CachedGraph *find_graph_locked(const GraphKey &key) const {
    for (size_t i = 0; i < graphs.size(); ++i)
      if (graphs[i].key == key) {
        std::rotate(graphs.begin(), graphs.begin() + i, graphs.begin() + i + 1);
        return &graphs[0];
      }
    return nullptr;
  }

  // launch a cached graph and record its completion event (under mu, so that
  // no other thread evicts it in between)
  static hipError_t launch_cached_locked(const CachedGraph &c, hipStream_t s) {
    hipError_t e = hipGraphLaunch(c.exec, s);
    if (e == hipSuccess) e = hipEventRecord(c.done, s);
    return e;
  }

  void bind(const float2 *tables) override {
    const char *base = reinterpret_cast<const char *>(tables);
    a.tables = tables;
    a.items = reinterpret_cast<const RaggedItem *>(base + items_off * sizeof(float2));
    a.sigoff = reinterpret_cast<const int64_t *>(base + sigoff_off * sizeof(float2));
  }

  RaggedArgs args_for(const ExecCtx &ctx) const {
    RaggedArgs r = a;
    r.ws = reinterpret_cast<float2 *>(ctx.ws);
    return r;
  }

  hipError_t launch_direct(const ExecCtx &ctx) const {
    RaggedArgs r = args_for(ctx);
    r.direct = 1;
    for (const auto &rg : ranges) {
      r.first_item = rg.first;
      r.nitems = rg.count;
      const float2 *s = (const float2 *)ctx.in;
      float2 *d = (float2 *)ctx.out;
      void *kargs[] = {(void *)&s, (void *)&d, (void *)&r.ws, (void *)&r.items, (void *)&r.sigoff,
                       (void *)&r.tables, (void *)&r};
      hipError_t e = hipLaunchKernel(ragged_kernel(ctx.inverse, rg.big), dim3((unsigned)rg.count),
                                     dim3(rg.big ? kRaggedBigThreads : kRaggedThreads), kargs,
                                     (size_t)(rg.big ? lds_big : lds_bytes), ctx.stream);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }

  // the persistent launches: k = 0 over [0, n_big) with the 1024-thread
  // instance, k = 1 over [n_big, n_phase1), k = 2 over [n_phase1, nitems)
  // (not persistent: one workgroup per item, dispatched by the hardware)
  void phase(int k, RaggedArgs &r) const {
    r.direct = persistent ? 0 : 1;
    r.first_item = k == 0 ? 0 : k == 1 ? n_big : n_phase1;
    r.nitems = k == 0 ? n_big : k == 1 ? n_phase1 - n_big : nitems - n_phase1;
  }
  static bool big_phase(int k) { return k == 0; }
  unsigned grid_of(int k, const RaggedArgs &r) const {
    if (!persistent) return (unsigned)r.nitems;
    return (unsigned)std::min(big_phase(k) ? resident_big : resident, r.nitems);
  }
  unsigned threads_of(int k) const { return big_phase(k) ? kRaggedBigThreads : kRaggedThreads; }
  size_t lds_of(int k) const { return (size_t)(big_phase(k) ? lds_big : lds_bytes); }

  hipError_t launch_persistent(const ExecCtx &ctx) const {
    RaggedArgs r = args_for(ctx);
    hipError_t e = hipSuccess;
    for (int k = 0; k < 3 && e == hipSuccess; ++k) {
      phase(k, r);
      if (r.nitems == 0) continue;
      const float2 *s = (const float2 *)ctx.in;
      float2 *d = (float2 *)ctx.out;
      void *kargs[] = {(void *)&s, (void *)&d, (void *)&r.ws, (void *)&r.items, (void *)&r.sigoff,
                       (void *)&r.tables, (void *)&r};
      e = hipLaunchKernel(ragged_kernel(ctx.inverse, big_phase(k)), dim3(grid_of(k, r)),
                          dim3(threads_of(k)), kargs, lds_of(k), ctx.stream);
    }
    return e;
  }

  // The launches as a graph of up to three nodes, built once per (buffers,
  // direction, stream).
  hipError_t launch_graph(const ExecCtx &ctx) const {
    GraphKey key{ctx.in, ctx.out, ctx.ws, ctx.inverse, ctx.stream};
    {
      std::lock_guard<std::mutex> lk(mu);
      if (const CachedGraph *c = find_graph_locked(key)) return launch_cached_locked(*c, ctx.stream);
    }
    hipGraphExec_t exec = nullptr;
    {
      RaggedArgs rr[3] = {args_for(ctx), args_for(ctx), args_for(ctx)};
      const float2 *s = (const float2 *)ctx.in;
      float2 *d = (float2 *)ctx.out;
      void *kp[3][7];
      for (int k = 0; k < 3; ++k) {
        phase(k, rr[k]);
        void *v[7] = {(void *)&s, (void *)&d, (void *)&rr[k].ws, (void *)&rr[k].items,
                      (void *)&rr[k].sigoff, (void *)&rr[k].tables, (void *)&rr[k]};
        for (int i = 0; i < 7; ++i) kp[k][i] = v[i];
      }
      hipGraph_t g = nullptr;
      hipError_t e = hipGraphCreate(&g, 0);
      if (e != hipSuccess) return e;
      // The 1024-thread single-pass items share no data with the others, so
      // their node is a branch of its own that may run beside the column
      // launch; the row launch waits for the column launch only.
      hipGraphNode_t cols = nullptr;
      for (int k = 0; k < 3 && e == hipSuccess; ++k) {
        if (rr[k].nitems == 0) continue;
        hipKernelNodeParams p{};
        p.func = const_cast<void *>(ragged_kernel(ctx.inverse, big_phase(k)));
        p.gridDim = dim3(grid_of(k, rr[k]));
        p.blockDim = dim3(threads_of(k));
        p.sharedMemBytes = (unsigned)lds_of(k);
        p.kernelParams = kp[k];
        hipGraphNode_t node = nullptr;
        const bool dep = k == 2 && cols;
        e = hipGraphAddKernelNode(&node, g, dep ? &cols : nullptr, dep ? 1 : 0, &p);
        if (k == 1) cols = node;
      }
      if (e == hipSuccess) e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return e;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (const CachedGraph *other = find_graph_locked(key)) {  // built meanwhile by another thread
      (void)hipGraphExecDestroy(exec);
      return launch_cached_locked(*other, ctx.stream);
    }
    hipEvent_t done = nullptr;
    hipError_t e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
    if (e == hipSuccess && graphs.size() >= kMaxGraphs) {
      // the evicted graph may still be running: wait for its last launch
      const CachedGraph &old = graphs.back();
      e = hipEventSynchronize(old.done);
      if (e == hipSuccess) {
        (void)hipGraphExecDestroy(old.exec);
        (void)hipEventDestroy(old.done);
        graphs.pop_back();
      }
    }
    if (e != hipSuccess) {
      (void)hipGraphExecDestroy(exec);
      if (done) (void)hipEventDestroy(done);
      return e;
    }
    graphs.insert(graphs.begin(), CachedGraph{key, exec, done});
    return launch_cached_locked(graphs.front(), ctx.stream);
  }

  hipError_t launch(const ExecCtx &ctx) const override {
    if (nitems == 0) return hipSuccess;
    if (per_size) return launch_direct(ctx);
    return graph && ctx.graphs ? launch_graph(ctx) : launch_persistent(ctx);
  }

  std::string describe() const override { return summary; }

  void extent(int64_t &max_in, int64_t &max_out, int &src_id, int &dst_id) const override {
    max_in = max_out = max_elem;
    src_id = BUF_IN;
    dst_id = BUF_OUT;
  }

  bool valid() const override {
    return lds_bytes <= kRaggedLdsBytes && resident > 0 && lds_big <= kRaggedBigLdsBytes &&
           (n_big == 0 || resident_big > 0) && ragged_kernel(false) && ragged_kernel(true);
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
constexpr int64_t kBigBudget = kRaggedBigLdsBytes / (int64_t)sizeof(float2);

// the lengths one 256-thread ragged workgroup transforms in a single pass
bool fits_single(const MixedPlan &mp) {
  return mp.T <= kRaggedThreads && tile_lds(mp, 1, ELEM_FAST) + tw_elems(mp) <= kBudget;
}
// ... and one 1024-thread workgroup
bool fits_big(const MixedPlan &mp) {
  return mp.T <= kRaggedBigThreads && tile_lds(mp, 1, ELEM_FAST) + tw_elems(mp) <= kBigBudget;
}

}  // namespace

}  // namespace dpfft

using namespace dpfft;

std::string dpfft::ragged_tune_key(int64_t L) {
  // the ragged kernels' shape constants and the version of the choice format
  uint64_t h = 1469598103934665603ull;
  for (int64_t v : {(int64_t)kRaggedThreads, (int64_t)kRaggedLdsBytes, (int64_t)kRaggedBigThreads,
                    (int64_t)kRaggedBigLdsBytes, (int64_t)sizeof(RaggedItem), (int64_t)2}) {
    for (int b = 0; b < 8; ++b) {
      h ^= (uint64_t)((v >> (8 * b)) & 0xff);
      h *= 1099511628211ull;
    }
  }
  char reg[20];
  snprintf(reg, sizeof reg, "%016llx", (unsigned long long)h);
  return std::string("gfx950|k=") + reg + "|ragged|n=" + std::to_string(L);
}

// Column lengths n1 of the four-step splits of L whose two factors both fit
// one 256-thread ragged workgroup, nearest to sqrt(L) first (at most `max`).
static std::vector<int64_t> ragged_splits(int64_t L, int order, int max) {
  std::vector<std::pair<double, int64_t>> c;
  for (int64_t d = 2; d * 2 <= L; ++d) {
    if (L % d) continue;
    MixedPlan a{}, b{};
    if (!mixed_radices(d, &a, order) || !mixed_radices(L / d, &b, order)) continue;
    if (!fits_single(a) || !fits_single(b)) continue;
    c.push_back({std::fabs(std::log((double)d) - 0.5 * std::log((double)L)), d});
  }
  std::stable_sort(c.begin(), c.end());
  std::vector<int64_t> out;
  for (const auto &e : c) {
    if ((int)out.size() >= max) break;
    out.push_back(e.second);
  }
  return out;
}

// Forms of a ragged length that a choice may name: single pass in a 256- or
// a 1024-thread workgroup, four-step.
static bool ragged_form_fits(int64_t L, int order, int form) {
  MixedPlan mp{};
  if (!mixed_radices(L, &mp, order)) return false;
  if (form == 0) return fits_single(mp);
  if (form == 2) return fits_big(mp) && !fits_single(mp);
  return !ragged_splits(L, order, 1).empty();
}

// Choices worth timing for one ragged length: each radix order (the second
// only where it differs), each form that fits, and for the four-step the
// three splits nearest sqrt(L).
std::vector<std::string> dpfft::ragged_candidates(int64_t L) {
  std::vector<std::string> out;
  uint64_t codes0 = 0;
  for (int order : {0, 1}) {
    MixedPlan mp{};
    if (!mixed_radices(L, &mp, order)) continue;
    if (order == 0) codes0 = mp.codes;
    else if (mp.codes == codes0) continue;
    const std::string o = "o=" + std::to_string(order);
    if (ragged_form_fits(L, order, 0)) out.push_back(o + " f=0");
    if (ragged_form_fits(L, order, 2)) out.push_back(o + " f=2");
    for (int64_t n1 : ragged_splits(L, order, 3))
      out.push_back(o + " f=1 s=" + std::to_string(n1));
  }
  return out;
}

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
  {
    // One workgroup per item, dispatched by the hardware, measured 3-4%
    // faster on the 10,000-signal batch than resident workgroups walking the
    // item lists (a new workgroup starts as soon as one retires, where a
    // resident one waits for its own item's stores before the next item's
    // loads); DPFFT_FORCE_PLAN "p0=1" selects the persistent walk.
    const char *env = getenv("DPFFT_FORCE_PLAN");
    if (env && parse_override(env).p[0] == 1) st->persistent = true;
  }
  st->max_elem = max_elem;

  // radix plan and pass-twiddle table of each line length, built once
  struct LineInfo {
    MixedPlan mp;
    int64_t tw2_off;
    bool ct;          // compile-time instances exist for this radix plan
    int64_t ptab_off; // their per-pass twiddle table
    int64_t ptab_n;
  };
  // DPFFT_FORCE_PLAN "x=0": every line through the runtime-radix passes
  bool no_ct = false;
  if (const char *env = getenv("DPFFT_FORCE_PLAN")) no_ct = parse_override(env).ct == 0;
  std::map<std::pair<int64_t, int>, LineInfo> lines;
  auto line_of = [&](int64_t L, int order) -> const LineInfo * {
    auto it = lines.find({L, order});
    if (it != lines.end()) return &it->second;
    MixedPlan mp{};
    if (!mixed_radices(L, &mp, order)) return nullptr;
    std::vector<std::complex<double>> lo, hi;
    fourstep_tables(L, mp.tw2_shift, lo, hi);
    lo.insert(lo.end(), hi.begin(), hi.end());
    LineInfo li{mp, (int64_t)P->tables.add(lo), false, 0, 0};
    uint64_t codes = 0;
    if (L <= INT32_MAX && ct_length((int)L, &codes) && codes == mp.codes && !no_ct) {
      // per-pass table: pass p >= 1, entry (r-1) Ns + k = w_{Ns R}^{k r}
      std::vector<std::complex<double>> t;
      for (int p = 1; p < mp.P; ++p)
        for (int r = 1; r < mp.radix[p]; ++r)
          for (int k = 0; k < mp.ns[p]; ++k)
            t.push_back(omega((int64_t)mp.ns[p] * mp.radix[p], (int64_t)k * r));
      if (t.empty()) t.push_back({1.0, 0.0});
      li.ct = true;
      li.ptab_n = (int64_t)t.size();
      li.ptab_off = (int64_t)P->tables.add(t);
    }
    return &(lines[{L, order}] = li);
  };
  // a line's LDS twiddle entries: the per-pass table of a compile-time
  // instance (four-step lines), else the two-level table
  auto twn = [&](const LineInfo &li, bool four) { return four && li.ct ? li.ptab_n : tw_elems(li.mp); };
  auto item_for = [](int32_t kind, const LineInfo &li, int C, int64_t tw_lds) {
    RaggedItem it{};
    it.kind = kind;
    it.C = C;
    it.tw_lds = (int32_t)tw_lds;
    it.L = li.mp.L;
    it.P = li.mp.P;
    it.T = li.mp.T;
    it.pitch = li.mp.pitch;
    it.tw2_shift = li.mp.tw2_shift;
    it.codes = li.mp.codes;
    it.tw2_off = li.tw2_off;
    if (kind != RK_SINGLE && li.ct) {
      it.ct = 1;
      it.tw2_off = li.ptab_off;
    }
    return it;
  };

  std::map<int64_t, std::vector<int32_t>> by_size;
  for (int64_t i = 0; i < count; ++i) by_size[sizes[i]].push_back((int32_t)i);

  std::vector<RaggedItem> items;
  std::vector<char> isbig;
  std::vector<int64_t> sigoff;
  std::vector<int64_t> cost;
  int64_t lds_need = 1, lds_need_big = 1, ws = 0;
  int nbig_sizes = 0, nsingle_sizes = 0, nlarge_sizes = 0, ntuned = 0;
  auto lg = [](int64_t L) { return std::max(1.0, std::log2((double)L)); };

  for (const auto &kv : by_size) {
    const int64_t L = kv.first;
    const auto &sigs = kv.second;
    // per-length choices: the tuner's candidate, a forced plan, the tuning
    // cache, else the heuristic (256-thread single pass where it fits, then
    // the 1024-thread single pass, then the four-step with the split nearest
    // sqrt(L))
    const Override ov = read_ragged_override(L);
    if (!ov.empty()) ++ntuned;
    const int order = ov.order >= 0 ? ov.order : 0;
    MixedPlan probe{};
    if (!mixed_radices(L, &probe, order))
      return fail(FFT_E_UNSUPPORTED, "no radix plan for ragged size " + std::to_string(L));
    int form = ov.form;
    if (form < 0 || !ragged_form_fits(L, order, form))
      form = fits_single(probe) ? 0 : (ov.big != 0 && fits_big(probe)) ? 2 : 1;
    if (!ragged_form_fits(L, order, form))
      return fail(FFT_E_UNSUPPORTED, "ragged size " + std::to_string(L) + " fits no form");
    if (form == 0 || form == 2) {
      const bool big = form == 2;
      const LineInfo &li = *line_of(L, order);
      const MixedPlan &mp = li.mp;
      const int nth = big ? kRaggedBigThreads : kRaggedThreads;
      const int64_t budget = big ? kBigBudget : kBudget;
      int C = std::max(1, nth / mp.T);
      if (ov.c[0] > 0) C = std::min(C, ov.c[0]);
      while (C > 1 && tile_lds(mp, C, ELEM_FAST) + tw_elems(mp) > budget) --C;
      const int first = (int)items.size();
      for (size_t s0 = 0; s0 < sigs.size(); s0 += C) {
        const int c = (int)std::min<size_t>(C, sigs.size() - s0);
        const int64_t data = tile_lds(mp, c, ELEM_FAST);
        RaggedItem it = item_for(RK_SINGLE, li, c, data);
        it.off = (int64_t)sigoff.size();
        for (int k = 0; k < c; ++k) sigoff.push_back(P->roffsets[sigs[s0 + k]]);
        items.push_back(it);
        isbig.push_back(big);
        cost.push_back((int64_t)(c * L * lg(L)));
        (big ? lds_need_big : lds_need) = std::max(big ? lds_need_big : lds_need, data + tw_elems(mp));
      }
      st->ranges.push_back({first, (int)items.size() - first, big});
      ++(big ? nlarge_sizes : nsingle_sizes);
      continue;
    }
    // four-step: L = n1 * n2
    // the named split where it fits this length, else the one nearest sqrt(L)
    int64_t n1 = ragged_splits(L, order, 1)[0];
    if (ov.split > 0)
      for (int64_t d : ragged_splits(L, order, 64))
        if (d == ov.split) n1 = d;
    const int64_t n2 = L / n1;
    const LineInfo *l1 = line_of(n1, order), *l2 = line_of(n2, order);
    if (!l1 || !l2) return fail(FFT_E_UNSUPPORTED, "no radix plan for ragged size " + std::to_string(L));
    const MixedPlan &m1 = l1->mp, &m2 = l2->mp;
    int CA = std::max(1, kRaggedThreads / m1.T), CB = std::max(1, kRaggedThreads / m2.T);
    if (ov.c[0] > 0) CA = std::min(CA, ov.c[0]);
    if (ov.c[1] > 0) CB = std::min(CB, ov.c[1]);
    while (CA > 1 && tile_lds(m1, CA, LINE_FAST) + twn(*l1, true) > kBudget) --CA;
    auto rows_lds = [&](int c) { return std::max(tile_lds(m2, c, ELEM_FAST), tile_lds(m2, c, LINE_FAST)); };
    while (CB > 1 && rows_lds(CB) + twn(*l2, true) > kBudget) --CB;
    std::vector<std::complex<double>> lo, hi;
    int lgL = 0;
    while ((int64_t(1) << lgL) < L) ++lgL;
    const int shift = (lgL + 1) / 2;
    fourstep_tables(L, shift, lo, hi);
    const int64_t lo_off = (int64_t)P->tables.add(lo), hi_off = (int64_t)P->tables.add(hi);
    auto four = [&](RaggedItem it, int32_t s, int64_t ws_off, int64_t f) {
      it.first = (int32_t)f;
      it.n1 = (int32_t)n1;
      it.n2 = (int32_t)n2;
      it.off = P->roffsets[s];
      it.ws_off = ws_off;
      it.tw4_lo_off = lo_off;
      it.tw4_hi_off = hi_off;
      it.tw4_shift = shift;
      return it;
    };
    const int first_cols = (int)items.size();
    std::vector<int64_t> ws_of;
    for (int32_t s : sigs) {
      ws_of.push_back(ws);
      for (int64_t f = 0; f < n2; f += CA) {
        const int c = (int)std::min<int64_t>(CA, n2 - f);
        const int64_t data = tile_lds(m1, c, LINE_FAST);
        items.push_back(four(item_for(RK_COLUMNS, *l1, c, data), s, ws, f));
        isbig.push_back(0);
        cost.push_back((int64_t)(c * n1 * lg(n1)));
        lds_need = std::max(lds_need, data + twn(*l1, true));
      }
      ws += L;
    }
    st->ranges.push_back({first_cols, (int)items.size() - first_cols, false});
    const int first_rows = (int)items.size();
    for (size_t k = 0; k < sigs.size(); ++k) {
      for (int64_t f = 0; f < n1; f += CB) {
        const int c = (int)std::min<int64_t>(CB, n1 - f);
        const int64_t data = rows_lds(c);
        items.push_back(four(item_for(RK_ROWS, *l2, c, data), sigs[k], ws_of[k], f));
        isbig.push_back(0);
        cost.push_back((int64_t)(c * n2 * lg(n2)));
        lds_need = std::max(lds_need, data + twn(*l2, true));
      }
    }
    st->ranges.push_back({first_rows, (int)items.size() - first_rows, false});
    ++nbig_sizes;
  }

  st->nitems = (int)items.size();
  st->n_big = 0;
  st->n_phase1 = 0;
  for (size_t i = 0; i < items.size(); ++i) {
    if (isbig[i]) ++st->n_big;
    if (items[i].kind != RK_ROWS) ++st->n_phase1;
  }
  if (!st->per_size) {
    // execution order of the persistent launches: the 1024-thread single-pass
    // items, then the other single-pass and the column items, then the row
    // items, each group largest first (the static stride then hands every
    // workgroup a similar share and keeps the tail short)
    auto phase_of = [&](int32_t x) { return isbig[x] ? 0 : items[x].kind == RK_ROWS ? 2 : 1; };
    std::vector<int32_t> order(items.size());
    for (size_t i = 0; i < items.size(); ++i) order[i] = (int32_t)i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
      const int px = phase_of(x), py = phase_of(y);
      if (px != py) return px < py;
      return cost[x] > cost[y];
    });
    std::vector<RaggedItem> sorted;
    sorted.reserve(items.size());
    for (int32_t i : order) sorted.push_back(items[i]);
    items.swap(sorted);
  }
  st->lds_bytes = (int)(lds_need * (int64_t)sizeof(float2));
  st->resident = resident_for(st->lds_bytes, kRaggedThreads);
  st->lds_big = st->n_big ? (int)(lds_need_big * (int64_t)sizeof(float2)) : 0;
  st->resident_big = st->n_big ? resident_for(st->lds_big, kRaggedBigThreads) : 0;
  if (items.empty()) items.push_back(RaggedItem{});
  if (lds_need * (int64_t)sizeof(float2) > kRaggedLdsBytes ||
      (st->n_big && lds_need_big * (int64_t)sizeof(float2) > kRaggedBigLdsBytes))
    return fail(FFT_E_INTERNAL, "ragged plan exceeds its LDS budget");
  if (sigoff.empty()) sigoff.push_back(0);
  st->items_off = P->tables.add_bytes(items.data(), items.size() * sizeof(RaggedItem));
  st->sigoff_off = P->tables.add_bytes(sigoff.data(), sigoff.size() * sizeof(int64_t));
  st->ws_elems = ws;
  P->ws_bytes = (size_t)ws * sizeof(float2);


  std::ostringstream o;
  const int nl = (st->n_big > 0) + 1 + (st->nitems > st->n_phase1);
  o << "ragged: " << count << " signals, " << nsingle_sizes << " single-pass lengths, "
    << nlarge_sizes << " single-pass lengths of 1024 threads, " << nbig_sizes
    << " four-step lengths, " << ntuned << " lengths with tuned choices, " << st->nitems
    << " items, "
    << (st->per_size ? "one launch per length (" + std::to_string(st->ranges.size()) + " launches)"
                     : std::to_string(nl) + (st->persistent ? " persistent" : "") +
                           " launches (" + std::to_string(st->n_big) +
                           " + " + std::to_string(st->n_phase1 - st->n_big) + " + " +
                           std::to_string(st->nitems - st->n_phase1) + " items), " +
                           (st->persistent ? "grid=" + std::to_string(std::min(st->resident_big, st->n_big)) +
                                                 "/" + std::to_string(std::min(st->resident, st->nitems))
                                           : std::string("one workgroup per item")))
    << (st->graph && !st->per_size ? " in a HIP graph" : "") << " threads=" << kRaggedBigThreads
    << "/" << kRaggedThreads << " lds=" << st->lds_big << "/" << st->lds_bytes << "B";
  st->summary = o.str();
  P->variant = st->per_size ? "ragged per-length launches" : "ragged persistent";
  P->steps.push_back(std::move(st));
  return FFT_OK;
}
