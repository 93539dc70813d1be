// C ABI of dpfft: validation, plan construction and execution.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <sstream>
#include <string>

#include "internal.h"
#include "plan.h"
#include "twiddle.h"

using namespace dpfft;

namespace {
thread_local std::string g_last_error;
}

namespace dpfft {
fft_status_t fail(fft_status_t s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

int64_t split_factor(int64_t n) {
  int64_t best = 1;
  for (int64_t d = 1; d * d <= n; ++d)
    if (n % d == 0) best = d;
  return best;
}

namespace {
// compute units the plan being built sizes its persistent grids for (set by
// fft_plan from the current device; dry plans assume an MI355X's 256)
thread_local int t_cus = kDefaultCus;
}  // namespace

void set_plan_cus(int cus) { t_cus = cus > 0 ? cus : kDefaultCus; }

int device_cus() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
    return v;
  return kDefaultCus;
}

int resident_for(int lds_bytes, int threads) {
  const int cus = t_cus;
  int by_lds = lds_bytes ? kLdsBytes / lds_bytes : 8;
  int by_thr = 2048 / threads;
  return cus * std::max(1, std::min(by_lds, by_thr));
}
}  // namespace dpfft

namespace {

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

int ilog2(int64_t v) {
  int k = 0;
  while ((int64_t(1) << k) < v) ++k;
  return k;
}

// largest prime factor of n (1 for n == 1)
int64_t largest_prime_factor(int64_t n) {
  int64_t best = 1;
  for (int64_t p = 2; p * p <= n; ++p)
    while (n % p == 0) {
      best = p;
      n /= p;
    }
  return n > 1 ? n : best;
}


}  // namespace

// ---------------------------------------------------------------------------
// TableSet / steps
// ---------------------------------------------------------------------------
namespace dpfft {

static void align_tables(std::vector<float2> &h) {
  while (h.size() % 32) h.push_back(make_float2(0.f, 0.f));  // 256-byte alignment
}

size_t TableSet::add(const std::vector<std::complex<double>> &t) {
  align_tables(host);
  size_t off = host.size();
  for (const auto &w : t) host.push_back(make_float2((float)w.real(), (float)w.imag()));
  return off;
}

size_t TableSet::add_raw(const std::vector<float2> &t) {
  align_tables(host);
  size_t off = host.size();
  host.insert(host.end(), t.begin(), t.end());
  return off;
}

size_t TableSet::add_bytes(const void *p, size_t bytes) {
  align_tables(host);
  size_t off = host.size();
  size_t n = (bytes + sizeof(float2) - 1) / sizeof(float2);
  host.resize(off + n, make_float2(0.f, 0.f));
  memcpy(host.data() + off, p, bytes);
  return off;
}

void LineStep::bind(const float2 *tables) {
  a.tw = tables + tw_off;
  a.tw2 = tables + tw2_off;
  if (has_tw4) {
    a.tw4_lo = tables + tw4_lo_off;
    a.tw4_hi = tables + tw4_hi_off;
  }
}

int LineStep::inverse_sw() const { return (first ? 1 : 0) | (last ? 2 : 0); }

hipError_t LineStep::launch(const ExecCtx &ctx) const {
  LineArgs args = a;
  dim3 g = grid;
  if (k.persistent) g.x = (unsigned)std::min<int64_t>(a.ntiles, (int64_t)resident);
  const void *fn = k.fn_sw[0];
  if (ctx.inverse) {
    fn = k.fn_sw[inverse_sw()];
    if (last) args.scale = inv_scale;
  }
  const float2 *s = buf_c(ctx, src, src_off);
  float2 *d = buf_m(ctx, dst, dst_off);
  void *kargs[] = {(void *)&s, (void *)&d, (void *)&args};
  return hipLaunchKernel(fn, g, dim3(k.threads), kargs, 0, ctx.stream);
}

void LineStep::extent(int64_t &max_in, int64_t &max_out, int &src_id, int &dst_id) const {
  const int64_t nb = (int64_t)grid.x / a.tiles_per_batch;  // batch items covered by the grid
  const int64_t last_line = std::min<int64_t>(a.lines, a.tiles_per_batch * k.lines) - 1;
  max_in = src_off + (nb - 1) * a.in_b + last_line * a.in_l + (int64_t)(L - 1) * a.in_e;
  max_out = dst_off + (nb - 1) * a.out_b + last_line * a.out_l + (int64_t)(L - 1) * a.out_e;
  src_id = src;
  dst_id = dst;
}

bool LineStep::valid() const {
  // unit strides the kernel assumes, 32-bit in-line offsets, instances present
  const bool in_ok = k.map == ELEM_FAST ? a.in_e == 1 : a.in_l == 1;
  const bool out_ok = k.omap == ELEM_FAST ? a.out_e == 1 : a.out_l == 1;
  // a column tile's elements lie within 2^29 elements (32-bit byte offsets)
  // of its first column; row tiles address each line from its own base
  const int64_t C = k.lines;
  const int64_t span_in = k.map == LINE_FAST ? (C - 1) + (int64_t)(L - 1) * a.in_e : 0;
  const int64_t span_out = k.omap == LINE_FAST ? (C - 1) + (int64_t)(L - 1) * a.out_e : 0;
  const bool off_ok = span_in < (int64_t(1) << 29) && span_out < (int64_t(1) << 29);
  return in_ok && out_ok && off_ok && k.fn_sw[0] && k.fn_sw[inverse_sw()];
}

std::string LineStep::describe() const {
  std::ostringstream o;
  o << name << ": L=" << L << " C=" << k.lines << " threads=" << k.threads;
  if (k.persistent)
    o << " persistent tiles=" << a.ntiles << " grid<=" << resident;
  else
    o << " grid=" << grid.x;
  o << " lds=" << k.lds_bytes << "B";
  return o.str();
}

// ---- runtime-radix steps ----
void MixedStep::bind(const float2 *tables) {
  a.tw2 = tables + tw2_off;
  if (tw4) {
    a.tw4_lo = tables + tw4_lo_off;
    a.tw4_hi = tables + tw4_hi_off;
  }
}

hipError_t MixedStep::launch(const ExecCtx &ctx) const {
  MixedArgs args = a;
  const void *fn = fn_sw[0];
  if (ctx.inverse) {
    fn = fn_sw[inverse_sw()];
    if (last) args.scale = inv_scale;
  }
  const float2 *s = buf_c(ctx, src, 0);
  float2 *d = buf_m(ctx, dst, 0);
  void *kargs[] = {(void *)&s, (void *)&d, (void *)&args};
  return hipLaunchKernel(fn, grid, dim3(threads), kargs, (size_t)lds_bytes, ctx.stream);
}

void MixedStep::extent(int64_t &max_in, int64_t &max_out, int &src_id, int &dst_id) const {
  const int64_t nb = (int64_t)grid.x / a.tiles_per_batch;
  const int64_t last_line = std::min<int64_t>(a.lines, a.tiles_per_batch * a.mp.C) - 1;
  max_in = (nb - 1) * a.in_b + last_line * a.in_l + (int64_t)(a.mp.L - 1) * a.in_e;
  max_out = (nb - 1) * a.out_b + last_line * a.out_l + (int64_t)(a.mp.L - 1) * a.out_e;
  src_id = src;
  dst_id = dst;
}

hipError_t MixedStep::prepare() const {
  // dynamic LDS above the default 64 KB needs an explicit opt-in per function;
  // the attribute is the function's, so it is set to the whole LDS of a CU
  // (a plan needing less must not lower it under another plan)
  for (int sw = 0; sw < 4; ++sw)
    if (fn_sw[sw]) {
      const hipError_t e =
          hipFuncSetAttribute(fn_sw[sw], hipFuncAttributeMaxDynamicSharedMemorySize, kLdsBytes);
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

bool MixedStep::valid() const {
  // in-line element offsets travel to the passes as 32-bit values
  const int64_t span = (int64_t)(a.mp.L - 1) * std::max(a.in_e, a.out_e);
  return fn_sw[0] && fn_sw[inverse_sw()] && threads > 0 && threads <= 1024 &&
         threads == a.mp.C * a.mp.T && lds_bytes <= kLdsBytes && a.mp.T * 16 >= a.mp.L &&
         span < (int64_t(1) << 31);
}

std::string MixedStep::describe() const {
  std::ostringstream o;
  o << name << ": L=" << a.mp.L << " radices=";
  for (int p = 0; p < a.mp.P; ++p) o << (p ? "x" : "") << a.mp.radix[p];
  o << " C=" << a.mp.C << " threads=" << threads << " grid=" << grid.x << " lds=" << lds_bytes
    << "B";
  return o.str();
}

// ---- matrix-core steps ----
void MfmaStep::bind(const float2 *tables) {
  a.amat = reinterpret_cast<const uint16_t *>(tables + amat_off);
  a.tw16 = tables + tw16_off;
  if (tw4) {
    a.tw4_lo = tables + tw4_lo_off;
    a.tw4_hi = tables + tw4_hi_off;
  }
}

hipError_t MfmaStep::launch(const ExecCtx &ctx) const {
  MfmaArgs args = a;
  const void *fn = fn_sw[0];
  if (ctx.inverse) {
    fn = fn_sw[inverse_sw()];
    if (last) args.scale = inv_scale;
  }
  const float2 *s = buf_c(ctx, src, 0);
  float2 *d = buf_m(ctx, dst, 0);
  void *kargs[] = {(void *)&s, (void *)&d, (void *)&args};
  return hipLaunchKernel(fn, grid, dim3(kMfmaThreads), kargs, 0, ctx.stream);
}

void MfmaStep::extent(int64_t &max_in, int64_t &max_out, int &src_id, int &dst_id) const {
  const int64_t nb = (int64_t)grid.x / a.tiles_per_batch;
  const int64_t last_line = std::min<int64_t>(a.lines, a.tiles_per_batch * kMfmaLines) - 1;
  max_in = (nb - 1) * a.in_b + last_line * a.in_l + 255 * a.in_e;
  max_out = (nb - 1) * a.out_b + last_line * a.out_l + 255 * a.out_e;
  src_id = src;
  dst_id = dst;
}

bool MfmaStep::valid() const { return fn_sw[0] && fn_sw[inverse_sw()]; }

std::string MfmaStep::describe() const {
  static const char *names[] = {"fp32", "fp16", "bf16", "fp16_split", "bf16_split", "bf16_split3"};
  std::ostringstream o;
  o << name << ": L=256 (DFT-16 x DFT-16 on MFMA, " << names[prec] << ") C=" << kMfmaLines
    << " threads=" << kMfmaThreads << " grid=" << grid.x << " lds=" << mfma_lds_bytes(prec) << "B";
  return o.str();
}

// ---- real-input steps ----
void RealStep::bind(const float2 *tables) {
  a.tw = tables + tw_off;
  a.tw2 = tables + tw2_off;
  a.tw4_lo = tables + wn_off;
}

hipError_t RealStep::launch(const ExecCtx &ctx) const {
  const float2 *s = buf_c(ctx, src, 0);
  float2 *d = buf_m(ctx, dst, 0);
  LineArgs args = a;
  void *kargs[] = {(void *)&s, (void *)&d, (void *)&args};
  return hipLaunchKernel(inv ? k.inv : k.fwd, grid, dim3(k.threads), kargs, 0, ctx.stream);
}

void RealStep::extent(int64_t &max_in, int64_t &max_out, int &src_id, int &dst_id) const {
  const int64_t nb = (int64_t)grid.x / a.tiles_per_batch;
  const int64_t last_line = a.lines - 1;
  // the spectrum side holds L + 1 elements per line, the real side L pairs
  max_in = (nb - 1) * a.in_b + last_line * a.in_l + (inv ? L : L - 1);
  max_out = (nb - 1) * a.out_b + last_line * a.out_l + (inv ? L - 1 : L);
  src_id = src;
  dst_id = dst;
}

bool RealStep::valid() const {
  return k.fwd && k.inv && (int64_t)grid.x == a.tiles_per_batch * (grid.x / a.tiles_per_batch);
}

std::string RealStep::describe() const {
  std::ostringstream o;
  o << name << ": N=" << 2 * L << " (" << L << "-point complex core) C=" << k.lines
    << " threads=" << k.threads << " grid=" << grid.x << " lds=" << k.lds_bytes << "B";
  return o.str();
}

void RealPairStep::bind(const float2 *tables) {
  a.lo = tables + lo_off;
  a.hi = tables + hi_off;
}

hipError_t RealPairStep::launch(const ExecCtx &ctx) const {
  const float2 *s = buf_c(ctx, src, 0);
  float2 *d = buf_m(ctx, dst, 0);
  RealPairArgs args = a;
  void *kargs[] = {(void *)&s, (void *)&d, (void *)&args};
  const dim3 grid((unsigned)((a.L / 2 + 1 + 255) / 256), (unsigned)std::min<int64_t>(a.batch, 65535));
  return hipLaunchKernel(real_pair_kernel(inv), grid, dim3(256), kargs, 0, ctx.stream);
}

void RealPairStep::extent(int64_t &max_in, int64_t &max_out, int &src_id, int &dst_id) const {
  // forward: Z[0..L-1] in, bins 0..L out; inverse: bins 0..L in, L values out
  max_in = (a.batch - 1) * a.in_b + (inv ? a.L : a.L - 1);
  max_out = (a.batch - 1) * a.out_b + (inv ? a.L - 1 : a.L);
  src_id = src;
  dst_id = dst;
}

bool RealPairStep::valid() const {
  return a.L >= 1 && a.L / 2 + 1 <= int64_t(1) << 32 && real_pair_kernel(inv) != nullptr;
}

std::string RealPairStep::describe() const {
  std::ostringstream o;
  o << name << ": pairs k, L - k of L=" << a.L << " (N=" << 2 * a.L << ") batch=" << a.batch;
  return o.str();
}

}  // namespace dpfft

dpfft_plan_s::~dpfft_plan_s() {
  if (tables.dev) (void)hipFree(tables.dev);
}

// ---------------------------------------------------------------------------
// plan builders
// ---------------------------------------------------------------------------
namespace {

// Override in force for a plan being built (see internal.h for the sources).
thread_local const fft_desc_t *g_building = nullptr;
thread_local bool g_skip_cache = false;  // a plan rebuilt after its cached override failed
thread_local bool g_cache_used = false;  // the override in force came from the tuning cache

Override read_override() {
  if (const Override *t = tuner_override()) return *t;
  if (const char *env = getenv("DPFFT_FORCE_PLAN")) return parse_override(env);
  if (g_building && !g_skip_cache && !(g_building->flags & FFT_F_NO_AUTOTUNE)) {
    const std::string key = tune_key(g_building);
    std::string val;
    if (!key.empty() && tune_cache_lookup(key, &val)) {
      g_cache_used = true;
      return parse_override(val);
    }
  }
  return Override{};
}

}  // namespace

// Choices for one length of a ragged batch: the autotuner's candidate while
// it times candidates, else DPFFT_FORCE_PLAN, else the tuning-cache entry of
// that length (unless FFT_F_NO_AUTOTUNE), else none (the heuristic).
Override dpfft::read_ragged_override(int64_t L) {
  if (const Override *t = tuner_override()) return *t;
  if (const char *env = getenv("DPFFT_FORCE_PLAN")) return parse_override(env);
  if (g_building && !g_skip_cache && !(g_building->flags & FFT_F_NO_AUTOTUNE)) {
    std::string val;
    if (tune_cache_lookup(ragged_tune_key(L), &val)) {
      g_cache_used = true;
      return parse_override(val);
    }
  }
  return Override{};
}

namespace {

// Workgroups of a persistent instance that stay resident on the device.
int resident_workgroups(const KernelInfo &k) { return resident_for(k.lds_bytes, k.threads); }

// Heuristic choice among the compiled instances of a line kernel: an instance
// the registry marks as the measured default of its shape wins; otherwise the
// most resident waves per CU that the 160 KB LDS allows (counted up to 16),
// then for row tiles the smaller tile (more workgroups to overlap), for column
// tiles the wider tile (longer contiguous segments); the caller's cap on lines
// per tile applies to the heuristic choice only.  Other persistent
// instances and other instances with 32 elements per thread are opt-in
// (override or tuner).
bool choose_line(int L, int map, int omap, bool tw4, int cmax, int step, int64_t lines_total,
                 const Override &ov, KernelInfo *out) {
  KernelInfo cand[32];
  int n = list_line_kernels(L, map, omap, tw4, cand, 32);
  if (n > 32) n = 32;
  double best = -1;
  for (int i = 0; i < n; ++i) {
    const KernelInfo &k = cand[i];
    if (ov.c[step] >= 0 && k.lines != ov.c[step]) continue;
    if (ov.c[step] < 0 && k.lines > cmax && !k.preferred) continue;
    if (ov.p[step] >= 0 && (int)k.persistent != ov.p[step]) continue;
    if (ov.t[step] >= 0 && k.threads != ov.t[step]) continue;
    if (ov.h[step] >= 0 && k.sub != ov.h[step]) continue;
    if (ov.p[step] < 0 && k.persistent && !k.preferred) continue;
    // a persistent default pays off only where every resident workgroup gets
    // more than one tile (its prefetch needs a next tile); small batches take
    // the heuristic choice
    if (ov.p[step] < 0 && k.persistent &&
        (lines_total + k.lines - 1) / k.lines <= resident_workgroups(k))
      continue;
    if (ov.t[step] < 0 && k.ept != 16 && !k.preferred) continue;
    if (k.threads > 1024) continue;
    int by_lds = k.lds_bytes ? kLdsBytes / k.lds_bytes : 64;
    int by_thr = 2048 / k.threads;
    int wg = std::min(by_lds, by_thr);
    double waves = wg * (k.threads / 64.0);
    double tie = (map == LINE_FAST || omap == LINE_FAST) ? k.lines : 1.0 / k.lines;
    double score = std::min(waves, 16.0) * 1000 + tie * 10 + (k.preferred ? 1e6 : 0);
    if (score > best) {
      best = score;
      *out = k;
    }
  }
  return best >= 0;
}

std::unique_ptr<LineStep> make_line(dpfft_plan_s *P, const char *name, int L, int map, int omap,
                                    bool tw4, int cmax, int step, int64_t lines_total,
                                    const Override &ov) {
  auto s = std::make_unique<LineStep>();
  if (!choose_line(L, map, omap, tw4, cmax, step, lines_total, ov, &s->k)) return nullptr;
  s->L = L;
  s->name = name;
  s->tw_off = P->tables.add(stockham_table_pow2(L / s->k.sub, s->k.ept));
  s->a.scale = 1.0f;
  // two-level table of w_L (pass twiddles rebuilt in LDS by the kernels whose
  // LDS holds no per-pass table)
  {
    std::vector<std::complex<double>> lo, hi;
    const int sh = tw2_shift(ilog2(L));
    fourstep_tables(L, sh, lo, hi);
    lo.insert(lo.end(), hi.begin(), hi.end());
    s->tw2_off = P->tables.add(lo);
  }
  if (s->k.persistent) s->resident = resident_workgroups(s->k);
  return s;
}

}  // namespace

std::unique_ptr<LineStep> dpfft::make_line_step(dpfft_plan_s *P, const char *name, int L, int map,
                                                int omap, bool tw4, int cmax, int step,
                                                int64_t lines_total, const Override &ov) {
  return make_line(P, name, L, map, omap, tw4, cmax, step, lines_total, ov);
}

namespace {

// Two-pass plans over B transforms, `per` elements apart in the caller's
// buffers: run the pair of launches chunk by chunk, `k` transforms at a time,
// so the intermediate of a chunk (k transforms, reused by every chunk) can be
// read back from the memory-side cache instead of HBM.  Pass a reads from the
// input at chunk offset and writes the workspace (or the output, in place
// passes); pass b finishes into the output at chunk offset.
void push_chunked(dpfft_plan_s *P, std::unique_ptr<LineStep> a, std::unique_ptr<LineStep> b,
                  int64_t B, int64_t k, int64_t per) {
  if (k <= 0 || k >= B) {
    P->steps.push_back(std::move(a));
    P->steps.push_back(std::move(b));
    return;
  }
  for (int64_t c0 = 0; c0 < B; c0 += k) {
    const int64_t nb = std::min(k, B - c0);
    auto ac = std::make_unique<LineStep>(*a);
    auto bc = std::make_unique<LineStep>(*b);
    ac->grid = dim3((unsigned)(nb * ac->a.tiles_per_batch));
    ac->a.ntiles = ac->grid.x;
    bc->grid = dim3((unsigned)(nb * bc->a.tiles_per_batch));
    bc->a.ntiles = bc->grid.x;
    ac->src_off = c0 * per;
    if (ac->dst != BUF_WS) ac->dst_off = c0 * per;
    if (bc->src != BUF_WS) bc->src_off = c0 * per;
    bc->dst_off = c0 * per;
    P->steps.push_back(std::move(ac));
    P->steps.push_back(std::move(bc));
  }
}

// transforms per chunk: the override, else the whole batch at once
int64_t chunk_of(const Override &ov) { return ov.chunk > 0 ? ov.chunk : 0; }

// The two launches of an N-point power-of-two four-step over B signals,
// in_b and out_b elements apart in the caller's input and output: pass A
// reads the input (BUF_IN) into the workspace, pass B the workspace into the
// output (BUF_OUT); pass A takes the inverse's input swap, pass B its output
// swap and 1/N.
bool fourstep_steps(dpfft_plan_s *P, int64_t N, int64_t B, int64_t in_b, int64_t out_b,
                    const Override &ov, std::unique_ptr<LineStep> &a, std::unique_ptr<LineStep> &b) {
  // four-step: N = N1 * N2, x[n1*N2 + n2]; pass A: N1-point column FFTs
  // (stride N2) and twiddle w_N^{n2 k1} into the workspace Y[k1][n2]; pass B:
  // N2-point FFTs along the rows of Y, stored transposed: X[k1 + N1 k2].
  // Default split: N1 = N2 (or N2 = 2 N1).  For 2^22, 2048 x 2048 measured
  // 1.5% faster than 4096 x 1024 (and steadier) and 2% faster than
  // 1024 x 4096; the tuner tries all three (override s=).
  const int lg = ilog2(N);
  int lg1 = lg / 2;
  if (ov.split > 0 && ov.split < lg) lg1 = ov.split;
  const int N1 = 1 << lg1, N2 = 1 << (lg - lg1);
  a = make_line(P, "fourstep_columns", N1, LINE_FAST, LINE_FAST, true, 16, 0, B * N2, ov);
  b = make_line(P, "fourstep_rows_transposed", N2, ELEM_FAST, LINE_FAST, false, 16, 1, B * N1, ov);
  if (!a || !b) return false;
  const int CA = a->k.lines, CB = b->k.lines;
  std::vector<std::complex<double>> lo, hi;
  const int shift = (lg + 1) / 2;
  fourstep_tables(N, shift, lo, hi);
  a->has_tw4 = true;
  a->tw4_lo_off = P->tables.add(lo);
  a->tw4_hi_off = P->tables.add(hi);
  a->a.tw4_shift = shift;
  a->a.in_b = in_b;
  a->a.in_l = 1;
  a->a.in_e = N2;
  a->a.out_b = N;
  a->a.out_l = 1;
  a->a.out_e = N2;
  a->a.lines = N2;
  a->a.tiles_per_batch = N2 / CA;
  // tile order in rounds (xcd_remap_rounds) except for column tiles narrower
  // than 64 bytes, which measured 1-8% slower with it; rounds of 16 tiles per
  // XCD for the 2048 x 2048 split (measured faster than 32, 8 and 4; for the
  // other splits and the 2D column tiles of 2048, 32 is the fastest)
  const uint32_t r16 = N1 == 2048 && N2 == 2048 ? F_ROUNDS16 : 0u;
  a->a.flags = F_REMAP | (CA >= 8 ? F_ROUNDS | r16 : 0u);
  a->grid = dim3((unsigned)(B * a->a.tiles_per_batch));
  a->a.ntiles = a->grid.x;
  a->first = true;
  a->src = BUF_IN;
  a->dst = BUF_WS;

  b->a.in_b = N;
  b->a.in_l = N2;
  b->a.in_e = 1;
  b->a.out_b = out_b;
  b->a.out_l = 1;
  b->a.out_e = N1;
  b->a.lines = N1;
  b->a.tiles_per_batch = N1 / CB;
  b->a.flags = F_REMAP | F_ROUNDS | r16;
  b->grid = dim3((unsigned)(B * b->a.tiles_per_batch));
  b->a.ntiles = b->grid.x;
  b->last = true;
  b->inv_scale = (float)(1.0 / (double)N);
  b->src = BUF_WS;
  b->dst = BUF_OUT;
  return true;
}

fft_status_t plan_pow2_1d(dpfft_plan_s *P) {
  const int64_t N = P->n, B = P->batch, D = P->dist;
  const Override ov = read_override();
  if (N <= kSinglePassMax) {
    const int L = (int)N;
    auto s = make_line(P, "stockham_rows", L, ELEM_FAST, ELEM_FAST, false, 256, 0, B, ov);
    if (!s) return fail(FFT_E_INTERNAL, "no row kernel for L=" + std::to_string(L));
    const int C = s->k.lines;
    s->a.in_b = s->a.out_b = 0;
    s->a.in_l = s->a.out_l = D;
    s->a.in_e = s->a.out_e = 1;
    s->a.lines = B;
    s->a.tiles_per_batch = (B + C - 1) / C;
    s->grid = dim3((unsigned)s->a.tiles_per_batch);
    s->a.ntiles = s->grid.x;
    s->first = s->last = true;
    s->inv_scale = (float)(1.0 / (double)N);
    s->src = BUF_IN;
    s->dst = BUF_OUT;
    P->steps.push_back(std::move(s));
    P->variant = "single-pass";
    return FFT_OK;
  }
  std::unique_ptr<LineStep> a, b;
  if (!fourstep_steps(P, N, B, D, D, ov, a, b))
    return fail(FFT_E_UNSUPPORTED, "no four-step kernels for N=" + std::to_string(N));
  const int N1 = a->L, N2 = b->L;
  const int64_t k = chunk_of(ov);
  push_chunked(P, std::move(a), std::move(b), B, k, D);
  P->ws_bytes = (size_t)(k > 0 && k < B ? k : B) * (size_t)N * sizeof(float2);
  P->variant = "four-step " + std::to_string(N1) + "x" + std::to_string(N2) +
               (k > 0 && k < B ? " in chunks of " + std::to_string(k) : "");
  return FFT_OK;
}

fft_status_t plan_pow2_2d(dpfft_plan_s *P) {
  const int64_t NY = P->ny, NX = P->nx, B = P->batch, D = P->dist;
  const Override ov = read_override();
  // row pass: in -> out; column pass: in place on out (column tiles read and
  // written by the same workgroup, so no transpose and no workspace)
  auto r = make_line(P, "rows", (int)NX, ELEM_FAST, ELEM_FAST, false, 256, 0, B * NY, ov);
  auto c = make_line(P, "columns", (int)NY, LINE_FAST, LINE_FAST, false, 64, 1, B * NX, ov);
  if (!r || !c) return fail(FFT_E_UNSUPPORTED, "no 2D kernels for this shape");
  const int CR = r->k.lines, CC = c->k.lines;
  r->a.in_b = r->a.out_b = D;
  r->a.in_l = r->a.out_l = NX;
  r->a.in_e = r->a.out_e = 1;
  r->a.lines = NY;
  r->a.tiles_per_batch = (NY + CR - 1) / CR;
  r->grid = dim3((unsigned)(B * r->a.tiles_per_batch));
  r->a.ntiles = r->grid.x;
  r->first = true;
  r->src = BUF_IN;
  r->dst = BUF_OUT;
  c->a.in_b = c->a.out_b = D;
  c->a.in_l = c->a.out_l = 1;
  c->a.in_e = c->a.out_e = NX;
  c->a.lines = NX;
  c->a.tiles_per_batch = (NX + CC - 1) / CC;
  c->a.flags = F_REMAP | F_ROUNDS;
  c->grid = dim3((unsigned)(B * c->a.tiles_per_batch));
  c->a.ntiles = c->grid.x;
  c->last = true;
  c->inv_scale = (float)(1.0 / ((double)NX * (double)NY));
  c->src = BUF_OUT;
  c->dst = BUF_OUT;
  const int64_t k = chunk_of(ov);
  push_chunked(P, std::move(r), std::move(c), B, k, D);
  P->variant = std::string("2d rows+columns") +
               (k > 0 && k < B ? " in chunks of " + std::to_string(k) : "");
  return FFT_OK;
}

// A runtime-radix step over lines of length L, C lines per workgroup.
std::unique_ptr<MixedStep> make_mixed(dpfft_plan_s *P, const char *name, int64_t L, int map,
                                      int omap, bool tw4, int C) {
  auto s = std::make_unique<MixedStep>();
  const Override ov = read_override();
  if (!mixed_radices(L, &s->a.mp, ov.order > 0 ? ov.order : 0)) return nullptr;
  s->a.mp.C = C;
  s->map = map;
  s->omap = omap;
  s->tw4 = tw4;
  s->name = name;
  s->threads = C * s->a.mp.T;
  s->a.mp.tw_lds = mixed_tile_elems(s->a.mp, map, omap);
  s->lds_bytes = mixed_lds_bytes(s->a.mp, map, omap);
  for (int sw = 0; sw < 4; ++sw) s->fn_sw[sw] = mixed_kernel(map, omap, tw4, sw);
  std::vector<std::complex<double>> lo, hi;
  fourstep_tables(L, s->a.mp.tw2_shift, lo, hi);
  lo.insert(lo.end(), hi.begin(), hi.end());
  s->tw2_off = P->tables.add(lo);
  s->a.scale = 1.0f;
  return s;
}

// lines per workgroup: as many as keep the workgroup <= `thr` threads and the
// LDS within one CU's 160 KB, at least `cmin`
int mixed_lines(int64_t L, int map, int omap, int thr, int cmin) {
  MixedPlan mp{};
  if (!mixed_radices(L, &mp)) return 0;
  int C = std::max(cmin, thr / mp.T);
  while (C > 1) {
    mp.C = C;
    if (C * mp.T <= 1024 && mixed_lds_bytes(mp, map, omap) <= kLdsBytes) break;
    --C;
  }
  mp.C = C;
  if (C * mp.T > 1024 || mixed_lds_bytes(mp, map, omap) > kLdsBytes) return 0;
  return C;
}

// The two launches of an N-point 7-smooth four-step over B signals, in_b
// and out_b elements apart in the caller's input and output (pass A: input
// -> workspace with the twiddle; pass B: workspace -> output, transposed).
bool mixed_fourstep_steps(dpfft_plan_s *P, int64_t N, int64_t B, int64_t in_b, int64_t out_b,
                          std::unique_ptr<MixedStep> &a, std::unique_ptr<MixedStep> &b) {
  const int64_t N1 = split_factor(N), N2 = N / N1;
  if (N2 > kSinglePassMax) return false;
  const int CA = mixed_lines(N1, LINE_FAST, LINE_FAST, 1024, 1);
  const int CB = mixed_lines(N2, ELEM_FAST, LINE_FAST, 1024, 1);
  a = CA ? make_mixed(P, "mixed_fourstep_columns", N1, LINE_FAST, LINE_FAST, true, std::min(CA, 16))
         : nullptr;
  b = CB ? make_mixed(P, "mixed_fourstep_rows_transposed", N2, ELEM_FAST, LINE_FAST, false,
                      std::min(CB, 16))
         : nullptr;
  if (!a || !b) return false;
  std::vector<std::complex<double>> lo, hi;
  const int shift = (ilog2(N) + 1) / 2;
  fourstep_tables(N, shift, lo, hi);
  a->tw4_lo_off = P->tables.add(lo);
  a->tw4_hi_off = P->tables.add(hi);
  a->a.tw4_shift = shift;
  a->a.in_b = in_b;
  a->a.in_l = 1;
  a->a.in_e = N2;
  a->a.out_b = N;
  a->a.out_l = 1;
  a->a.out_e = N2;
  a->a.lines = N2;
  a->a.tiles_per_batch = (N2 + a->a.mp.C - 1) / a->a.mp.C;
  a->a.flags = F_REMAP;
  a->grid = dim3((unsigned)(B * a->a.tiles_per_batch));
  a->first = true;
  a->src = BUF_IN;
  a->dst = BUF_WS;
  b->a.in_b = N;
  b->a.in_l = N2;
  b->a.in_e = 1;
  b->a.out_b = out_b;
  b->a.out_l = 1;
  b->a.out_e = N1;
  b->a.lines = N1;
  b->a.tiles_per_batch = (N1 + b->a.mp.C - 1) / b->a.mp.C;
  b->a.flags = F_REMAP;
  b->grid = dim3((unsigned)(B * b->a.tiles_per_batch));
  b->last = true;
  b->inv_scale = (float)(1.0 / (double)N);
  b->src = BUF_WS;
  b->dst = BUF_OUT;
  return true;
}

// Images whose sides are 7-smooth but not both powers of two: the row pass
// (input -> output) and the column pass (column tiles in place on the
// output) on the runtime-radix kernels, one pass through LDS each.  In place
// is safe: with two or more passes every load of a tile precedes the barrier
// that ends its first pass, and a one-pass line (a single radix) is one
// butterfly of one thread.
fft_status_t plan_mixed_2d(dpfft_plan_s *P) {
  const int64_t NY = P->ny, NX = P->nx, B = P->batch, D = P->dist;
  const int CR = mixed_lines(NX, ELEM_FAST, ELEM_FAST, 256, 1);
  const int CC = mixed_lines(NY, LINE_FAST, LINE_FAST, 1024, 1);
  auto r = CR ? make_mixed(P, "mixed_rows", NX, ELEM_FAST, ELEM_FAST, false, CR) : nullptr;
  auto c = CC ? make_mixed(P, "mixed_columns", NY, LINE_FAST, LINE_FAST, false, std::min(CC, 16))
              : nullptr;
  if (!r || !c) return fail(FFT_E_UNSUPPORTED, "no runtime-radix 2D kernels for this shape");
  r->a.in_b = r->a.out_b = D;
  r->a.in_l = r->a.out_l = NX;
  r->a.in_e = r->a.out_e = 1;
  r->a.lines = NY;
  r->a.tiles_per_batch = (NY + r->a.mp.C - 1) / r->a.mp.C;
  r->grid = dim3((unsigned)(B * r->a.tiles_per_batch));
  r->first = true;
  r->src = BUF_IN;
  r->dst = BUF_OUT;
  c->a.in_b = c->a.out_b = D;
  c->a.in_l = c->a.out_l = 1;
  c->a.in_e = c->a.out_e = NX;
  c->a.lines = NX;
  c->a.tiles_per_batch = (NX + c->a.mp.C - 1) / c->a.mp.C;
  c->a.flags = F_REMAP;
  c->grid = dim3((unsigned)(B * c->a.tiles_per_batch));
  c->last = true;
  c->inv_scale = (float)(1.0 / ((double)NX * (double)NY));
  c->src = BUF_OUT;
  c->dst = BUF_OUT;
  P->steps.push_back(std::move(r));
  P->steps.push_back(std::move(c));
  P->variant = "mixed 2d rows+columns";
  return FFT_OK;
}

fft_status_t plan_mixed_1d(dpfft_plan_s *P) {
  const int64_t N = P->n, B = P->batch, D = P->dist;
  const Override ov = read_override();
  if (N <= kSinglePassMax) {
    int C = mixed_lines(N, ELEM_FAST, ELEM_FAST, 256, 1);
    if (ov.c[0] > 0) {
      const int cmax = mixed_lines(N, ELEM_FAST, ELEM_FAST, 1024, 1);
      if (ov.c[0] > cmax) return fail(FFT_E_UNSUPPORTED, "override c0 too large for N");
      C = ov.c[0];
    }
    auto s = C ? make_mixed(P, "mixed_rows", N, ELEM_FAST, ELEM_FAST, false, C) : nullptr;
    if (!s) return fail(FFT_E_UNSUPPORTED, "no mixed-radix plan for N=" + std::to_string(N));
    s->a.in_b = s->a.out_b = 0;
    s->a.in_l = s->a.out_l = D;
    s->a.in_e = s->a.out_e = 1;
    s->a.lines = B;
    s->a.tiles_per_batch = (B + C - 1) / C;
    s->grid = dim3((unsigned)s->a.tiles_per_batch);
    s->first = s->last = true;
    s->inv_scale = (float)(1.0 / (double)N);
    P->steps.push_back(std::move(s));
    P->variant = "mixed single-pass";
    return FFT_OK;
  }
  std::unique_ptr<MixedStep> a, b;
  if (!mixed_fourstep_steps(P, N, B, D, D, a, b))
    return fail(FFT_E_UNSUPPORTED, "no mixed four-step plan for N=" + std::to_string(N));
  const int64_t N1 = a->a.mp.L, N2 = b->a.mp.L;
  P->steps.push_back(std::move(a));
  P->steps.push_back(std::move(b));
  P->ws_bytes = (size_t)B * (size_t)N * sizeof(float2);
  P->variant = "mixed four-step " + std::to_string(N1) + "x" + std::to_string(N2);
  return FFT_OK;
}

std::unique_ptr<MfmaStep> make_mfma(dpfft_plan_s *P, const char *name, int prec, int map,
                                    int omap, bool tw4) {
  auto s = std::make_unique<MfmaStep>();
  s->prec = prec;
  s->name = name;
  s->tw4 = tw4;
  for (int sw = 0; sw < 4; ++sw) s->fn_sw[sw] = mfma_kernel(prec, map, omap, tw4, sw);
  const std::vector<uint16_t> am = mfma_dft16_operands(prec);
  s->amat_off = P->tables.add_bytes(am.data(), am.size() * sizeof(uint16_t));
  std::vector<std::complex<double>> t16(256);
  for (int k1 = 0; k1 < 16; ++k1)
    for (int n2 = 0; n2 < 16; ++n2) t16[k1 * 16 + n2] = omega(256, (int64_t)n2 * k1);
  s->tw16_off = P->tables.add(t16);
  s->a.scale = 1.0f;
  return s;
}

// Matrix-core plans: N = 256 (one pass), N = 65536 (four-step 256 x 256 with
// both passes on the matrix cores), and N = 256 N2 for N2 = 64 .. 4096 (the
// 256-point column pass on the matrix cores, the N2-point transposed-row pass
// with the FP32 line kernels).
fft_status_t plan_mfma_1d(dpfft_plan_s *P) {
  const int64_t N = P->n, B = P->batch, D = P->dist;
  const int prec = P->precision;
  const int C = kMfmaLines;
  if (N == 256) {
    auto s = make_mfma(P, "mfma_rows", prec, ELEM_FAST, ELEM_FAST, false);
    s->a.in_b = s->a.out_b = 0;
    s->a.in_l = s->a.out_l = D;
    s->a.in_e = s->a.out_e = 1;
    s->a.lines = B;
    s->a.tiles_per_batch = (B + C - 1) / C;
    s->grid = dim3((unsigned)s->a.tiles_per_batch);
    s->first = s->last = true;
    s->inv_scale = 1.0f / 256.0f;
    P->steps.push_back(std::move(s));
    P->variant = "mfma single-pass";
    return FFT_OK;
  }
  const int64_t N2 = N / 256;
  if (N % 256 != 0 || N2 < 64 || N2 > 4096 || (N2 & (N2 - 1)) != 0)
    return fail(FFT_E_UNSUPPORTED, "MFMA precision forms support N = 256 and N = 256 N2 with N2 "
                                   "a power of two from 64 to 4096");
  if (N2 != 256) {
    const Override ov = read_override();
    const int lg = ilog2(N);
    auto a = make_mfma(P, "mfma_fourstep_columns", prec, LINE_FAST, LINE_FAST, true);
    auto b = make_line(P, "fourstep_rows_transposed", (int)N2, ELEM_FAST, LINE_FAST, false, 16, 1,
                       B * 256, ov);
    if (!b) return fail(FFT_E_UNSUPPORTED, "no transposed-row kernel for N2=" + std::to_string(N2));
    std::vector<std::complex<double>> lo, hi;
    const int shift = (lg + 1) / 2;
    fourstep_tables(N, shift, lo, hi);
    a->tw4_lo_off = P->tables.add(lo);
    a->tw4_hi_off = P->tables.add(hi);
    a->a.tw4_shift = shift;
    a->a.in_b = D;
    a->a.in_l = 1;
    a->a.in_e = N2;
    a->a.out_b = N;
    a->a.out_l = 1;
    a->a.out_e = N2;
    a->a.lines = N2;
    a->a.tiles_per_batch = (N2 + C - 1) / C;
    a->a.flags = F_REMAP | F_ROUNDS;
    a->grid = dim3((unsigned)(B * a->a.tiles_per_batch));
    a->first = true;
    a->src = BUF_IN;
    a->dst = BUF_WS;
    const int CB = b->k.lines;
    b->a.in_b = N;
    b->a.in_l = N2;
    b->a.in_e = 1;
    b->a.out_b = D;
    b->a.out_l = 1;
    b->a.out_e = 256;
    b->a.lines = 256;
    b->a.tiles_per_batch = 256 / CB;
    b->a.flags = F_REMAP | F_ROUNDS;
    b->grid = dim3((unsigned)(B * b->a.tiles_per_batch));
    b->a.ntiles = b->grid.x;
    b->last = true;
    b->inv_scale = (float)(1.0 / (double)N);
    b->src = BUF_WS;
    b->dst = BUF_OUT;
    P->steps.push_back(std::move(a));
    P->steps.push_back(std::move(b));
    P->ws_bytes = (size_t)B * (size_t)N * sizeof(float2);
    P->variant = "mfma four-step 256x" + std::to_string(N2) + " (matrix-core columns, FP32 rows)";
    return FFT_OK;
  }
  auto a = make_mfma(P, "mfma_fourstep_columns", prec, LINE_FAST, LINE_FAST, true);
  auto b = make_mfma(P, "mfma_fourstep_rows_transposed", prec, ELEM_FAST, LINE_FAST, false);
  std::vector<std::complex<double>> lo, hi;
  fourstep_tables(N, 8, lo, hi);
  a->tw4_lo_off = P->tables.add(lo);
  a->tw4_hi_off = P->tables.add(hi);
  a->a.tw4_shift = 8;
  a->a.in_b = D;
  a->a.in_l = 1;
  a->a.in_e = 256;
  a->a.out_b = N;
  a->a.out_l = 1;
  a->a.out_e = 256;
  a->a.lines = 256;
  a->a.tiles_per_batch = 256 / C;
  a->a.flags = F_REMAP | F_ROUNDS;
  a->grid = dim3((unsigned)(B * a->a.tiles_per_batch));
  a->first = true;
  a->src = BUF_IN;
  a->dst = BUF_WS;
  b->a.in_b = N;
  b->a.in_l = 256;
  b->a.in_e = 1;
  b->a.out_b = D;
  b->a.out_l = 1;
  b->a.out_e = 256;
  b->a.lines = 256;
  b->a.tiles_per_batch = 256 / C;
  b->a.flags = F_REMAP | F_ROUNDS;
  b->grid = dim3((unsigned)(B * b->a.tiles_per_batch));
  b->last = true;
  b->inv_scale = (float)(1.0 / (double)N);
  b->src = BUF_WS;
  b->dst = BUF_OUT;
  P->steps.push_back(std::move(a));
  P->steps.push_back(std::move(b));
  P->ws_bytes = (size_t)B * (size_t)N * sizeof(float2);
  P->variant = "mfma four-step 256x256";
  return FFT_OK;
}

// Real-input row step: lines of N = 2L reals <-> L + 1 bins.  `rows` lines per
// batch item, items `real_b` float pairs apart on the real side and `cplx_b`
// complex elements apart on the spectrum side.
std::unique_ptr<RealStep> make_real(dpfft_plan_s *P, const char *name, int64_t N, bool inv,
                                    int64_t rows, int64_t real_b, int64_t cplx_b) {
  auto s = std::make_unique<RealStep>();
  const int L = (int)(N / 2);
  if (!real_kernel(L, &s->k)) return nullptr;
  s->L = L;
  s->inv = inv;
  s->name = name;
  s->tw_off = P->tables.add(stockham_table_pow2(L, 16));
  {
    std::vector<std::complex<double>> lo, hi;
    fourstep_tables(L, tw2_shift(ilog2(L)), lo, hi);
    lo.insert(lo.end(), hi.begin(), hi.end());
    s->tw2_off = P->tables.add(lo);
  }
  std::vector<std::complex<double>> wn((size_t)L);
  for (int k = 0; k < L; ++k) wn[(size_t)k] = omega(N, k);
  s->wn_off = P->tables.add(wn);
  const int C = s->k.lines;
  if (!inv) {
    s->a.in_b = real_b;
    s->a.in_l = L;
    s->a.out_b = cplx_b;
    s->a.out_l = L + 1;
  } else {
    s->a.in_b = cplx_b;
    s->a.in_l = L + 1;
    s->a.out_b = real_b;
    s->a.out_l = L;
  }
  s->a.in_e = s->a.out_e = 1;
  s->a.lines = rows;
  s->a.tiles_per_batch = (rows + C - 1) / C;
  s->grid = dim3((unsigned)(P->batch * s->a.tiles_per_batch));
  s->a.ntiles = s->grid.x;
  s->a.scale = inv ? (float)(1.0 / (double)N) : 1.0f;
  return s;
}

// Real-input batch of 1D signals: one launch per direction while the
// N/2-point complex core fits one workgroup; above, the core is the
// four-step pair of launches and the pairing of k with N/2 - k a launch of its
// own.  Forward: the core from the input through the output (used as scratch
// at N/2 elements per signal, so every tile stays on 128-byte boundaries)
// into the workspace, then the pairing from the workspace into the output's
// N/2 + 1 bins per signal, whose rows start at any 8-byte offset but which
// the pairing writes as contiguous runs.  Inverse: the pairing from the input
// into the output, then the core from the output through the workspace back
// into it, scaled by 1/N.
fft_status_t plan_real_1d(dpfft_plan_s *P) {
  const int64_t N = P->n, B = P->batch;
  if (!is_pow2(N) || N / 2 > kSinglePassMax) {
    const int64_t L = N / 2;
    const Override ov = read_override();
    std::vector<std::complex<double>> lo, hi;
    const int shift = (ilog2(N) + 1) / 2;
    fourstep_tables(N, shift, lo, hi);
    const size_t lo_off = P->tables.add(lo), hi_off = P->tables.add(hi);
    auto pair = [&](bool inv, int src, int dst) {
      auto r = std::make_unique<RealPairStep>();
      r->inv = inv;
      r->name = inv ? "real_pairs_inverse" : "real_pairs";
      r->a.L = L;
      r->a.batch = B;
      r->a.in_b = inv ? L + 1 : L;  // inverse: the bins; forward: Z at L per signal
      r->a.out_b = inv ? L : L + 1;
      r->a.shift = shift;
      r->lo_off = lo_off;
      r->hi_off = hi_off;
      r->src = src;
      r->dst = dst;
      return r;
    };
    std::string core;
    if (L <= kSinglePassMax && !is_pow2(L)) {
      // single-pass runtime-radix core: input -> workspace (forward), and
      // workspace -> output after the pairing (inverse), never in place
      int C = mixed_lines(L, ELEM_FAST, ELEM_FAST, 256, 1);
      if (ov.c[0] > 0 && ov.c[0] <= mixed_lines(L, ELEM_FAST, ELEM_FAST, 1024, 1)) C = ov.c[0];
      std::unique_ptr<MixedStep> c[2];
      for (int i = 0; i < 2; ++i) {
        c[i] = C ? make_mixed(P, i ? "real_core_rows_inverse" : "real_core_rows", L, ELEM_FAST,
                              ELEM_FAST, false, C)
                 : nullptr;
        if (!c[i]) return fail(FFT_E_UNSUPPORTED, "no runtime-radix core for real N=" + std::to_string(N));
        c[i]->a.in_b = c[i]->a.out_b = 0;
        c[i]->a.in_l = c[i]->a.out_l = L;
        c[i]->a.in_e = c[i]->a.out_e = 1;
        c[i]->a.lines = B;
        c[i]->a.tiles_per_batch = (B + C - 1) / C;
        c[i]->grid = dim3((unsigned)c[i]->a.tiles_per_batch);
        c[i]->first = c[i]->last = true;
        c[i]->inv_scale = (float)(1.0 / (double)N);
      }
      c[0]->src = BUF_IN;
      c[0]->dst = BUF_WS;
      c[1]->src = BUF_WS;
      c[1]->dst = BUF_OUT;
      P->steps.push_back(std::move(c[0]));
      P->steps.push_back(pair(false, BUF_WS, BUF_OUT));
      P->isteps.push_back(pair(true, BUF_IN, BUF_WS));
      P->isteps.push_back(std::move(c[1]));
      core = "runtime-radix single-pass";
    } else {
      // four-step core (powers of two: the line kernels; else runtime radix)
      std::unique_ptr<Step> a, b, ai, bi;
      std::string split;
      if (is_pow2(L)) {
        std::unique_ptr<LineStep> x[4];
        if (!fourstep_steps(P, L, B, L, L, ov, x[0], x[1]) || !fourstep_steps(P, L, B, L, L, ov, x[2], x[3]))
          return fail(FFT_E_UNSUPPORTED, "no four-step kernels for the real-input core L=" + std::to_string(L));
        const char *nm[4] = {"real_core_columns", "real_core_rows_transposed",
                             "real_core_columns_inverse", "real_core_rows_transposed_inverse"};
        for (int i = 0; i < 4; ++i) x[i]->name = nm[i];
        split = std::to_string(x[0]->L) + "x" + std::to_string(x[1]->L);
        // forward: Y in the output as scratch (L per signal, whole 128-byte
        // lines), Z into the workspace; inverse: output -> workspace -> output
        x[0]->dst = BUF_OUT;
        x[1]->src = BUF_OUT;
        x[1]->dst = BUF_WS;
        x[2]->src = BUF_OUT;
        x[3]->inv_scale = (float)(1.0 / (double)N);
        a = std::move(x[0]), b = std::move(x[1]), ai = std::move(x[2]), bi = std::move(x[3]);
      } else {
        std::unique_ptr<MixedStep> x[4];
        if (!mixed_fourstep_steps(P, L, B, L, L, x[0], x[1]) || !mixed_fourstep_steps(P, L, B, L, L, x[2], x[3]))
          return fail(FFT_E_UNSUPPORTED, "no four-step core for real N=" + std::to_string(N));
        const char *nm[4] = {"real_core_columns", "real_core_rows_transposed",
                             "real_core_columns_inverse", "real_core_rows_transposed_inverse"};
        for (int i = 0; i < 4; ++i) x[i]->name = nm[i];
        split = std::to_string(x[0]->a.mp.L) + "x" + std::to_string(x[1]->a.mp.L);
        x[0]->dst = BUF_OUT;
        x[1]->src = BUF_OUT;
        x[1]->dst = BUF_WS;
        x[2]->src = BUF_OUT;
        x[3]->inv_scale = (float)(1.0 / (double)N);
        a = std::move(x[0]), b = std::move(x[1]), ai = std::move(x[2]), bi = std::move(x[3]);
      }
      P->steps.push_back(std::move(a));
      P->steps.push_back(std::move(b));
      P->steps.push_back(pair(false, BUF_WS, BUF_OUT));
      P->isteps.push_back(pair(true, BUF_IN, BUF_OUT));
      P->isteps.push_back(std::move(ai));
      P->isteps.push_back(std::move(bi));
      core = "four-step " + split;
    }
    P->ws_bytes = (size_t)B * (size_t)L * sizeof(float2);
    P->variant = "real " + core + " + pairing";
    return FFT_OK;
  }
  auto f = make_real(P, "real_forward", N, false, B, 0, 0);
  auto i = make_real(P, "real_inverse", N, true, B, 0, 0);
  if (!f || !i) return fail(FFT_E_UNSUPPORTED, "no real-input kernel for N=" + std::to_string(N));
  P->steps.push_back(std::move(f));
  P->isteps.push_back(std::move(i));
  P->variant = "real single-pass";
  return FFT_OK;
}

// Real-input images: forward = real rows -> ny x (nx/2 + 1) bins in `out`,
// then the column transforms in place on `out`; inverse = column transforms
// of `in` into the workspace (scale 1/ny), then the complex-to-real rows from
// the workspace into `out` (scale 1/nx).
// Real-input images whose sides are not both powers of two: the rows of
// nx/2 complex pairs through the runtime-radix single pass, the pairing of
// bin k with nx/2 - k per row, then the runtime-radix column tiles over the
// nx/2 + 1 columns.  Forward: rows input -> workspace, pairing workspace ->
// output, columns in place on the output.  Inverse: columns input ->
// workspace (scale 1/ny), pairing workspace -> output (rows of nx/2), rows in
// place on the output (scale 1/nx).
fft_status_t plan_real_2d_mixed(dpfft_plan_s *P) {
  const int64_t NY = P->ny, NX = P->nx, B = P->batch;
  const int64_t L = NX / 2, W = L + 1, R = B * NY;
  const int CR = mixed_lines(L, ELEM_FAST, ELEM_FAST, 256, 1);
  const int CC = mixed_lines(NY, LINE_FAST, LINE_FAST, 1024, 1);
  std::unique_ptr<MixedStep> row[2], col[2];
  for (int i = 0; i < 2; ++i) {
    row[i] = CR ? make_mixed(P, i ? "real_core_rows_inverse" : "real_core_rows", L, ELEM_FAST,
                             ELEM_FAST, false, CR)
                : nullptr;
    col[i] = CC ? make_mixed(P, i ? "columns_inverse" : "columns", NY, LINE_FAST, LINE_FAST, false,
                             std::min(CC, 16))
                : nullptr;
    if (!row[i] || !col[i])
      return fail(FFT_E_UNSUPPORTED, "no runtime-radix kernels for this real-input image");
    MixedStep &r = *row[i];
    r.a.in_b = r.a.out_b = 0;
    r.a.in_l = r.a.out_l = L;
    r.a.in_e = r.a.out_e = 1;
    r.a.lines = R;
    r.a.tiles_per_batch = (R + r.a.mp.C - 1) / r.a.mp.C;
    r.grid = dim3((unsigned)r.a.tiles_per_batch);
    r.first = r.last = true;
    r.inv_scale = (float)(1.0 / (double)NX);
    MixedStep &c = *col[i];
    c.a.in_b = c.a.out_b = NY * W;
    c.a.in_l = c.a.out_l = 1;
    c.a.in_e = c.a.out_e = W;
    c.a.lines = W;
    c.a.tiles_per_batch = (W + c.a.mp.C - 1) / c.a.mp.C;
    c.a.flags = F_REMAP;
    c.grid = dim3((unsigned)(B * c.a.tiles_per_batch));
    c.first = c.last = true;
    c.inv_scale = (float)(1.0 / (double)NY);
  }
  std::vector<std::complex<double>> lo, hi;
  const int shift = (ilog2(NX) + 1) / 2;
  fourstep_tables(NX, shift, lo, hi);
  const size_t lo_off = P->tables.add(lo), hi_off = P->tables.add(hi);
  auto pair = [&](bool inv) {
    auto r = std::make_unique<RealPairStep>();
    r->inv = inv;
    r->name = inv ? "real_pairs_inverse" : "real_pairs";
    r->a.L = L;
    r->a.batch = R;
    r->a.in_b = inv ? W : L;
    r->a.out_b = inv ? L : W;
    r->a.shift = shift;
    r->lo_off = lo_off;
    r->hi_off = hi_off;
    r->src = BUF_WS;
    r->dst = BUF_OUT;
    return r;
  };
  row[0]->src = BUF_IN;
  row[0]->dst = BUF_WS;
  col[0]->src = col[0]->dst = BUF_OUT;
  col[1]->src = BUF_IN;
  col[1]->dst = BUF_WS;
  row[1]->src = row[1]->dst = BUF_OUT;
  P->steps.push_back(std::move(row[0]));
  P->steps.push_back(pair(false));
  P->steps.push_back(std::move(col[0]));
  P->isteps.push_back(std::move(col[1]));
  P->isteps.push_back(pair(true));
  P->isteps.push_back(std::move(row[1]));
  P->ws_bytes = (size_t)B * (size_t)NY * (size_t)W * sizeof(float2);
  P->variant = "real 2d runtime-radix rows + pairing + columns";
  return FFT_OK;
}

fft_status_t plan_real_2d(dpfft_plan_s *P) {
  const int64_t NY = P->ny, NX = P->nx, B = P->batch;
  if (!is_pow2(NY) || !is_pow2(NX)) return plan_real_2d_mixed(P);
  const int64_t W = NX / 2 + 1;  // bins per row
  const Override ov = read_override();
  auto rf = make_real(P, "real_rows", NX, false, NY, NY * NX / 2, NY * W);
  auto ri = make_real(P, "real_rows_inverse", NX, true, NY, NY * NX / 2, NY * W);
  if (!rf || !ri) return fail(FFT_E_UNSUPPORTED, "no real-input row kernel for nx=" + std::to_string(NX));
  std::unique_ptr<LineStep> cf, ci;
  if (NY > 1) {
    cf = make_line(P, "columns", (int)NY, LINE_FAST, LINE_FAST, false, 64, 1, B * W, ov);
    ci = make_line(P, "columns_inverse", (int)NY, LINE_FAST, LINE_FAST, false, 64, 0, B * W, ov);
    if (!cf || !ci) return fail(FFT_E_UNSUPPORTED, "no column kernel for ny=" + std::to_string(NY));
    for (LineStep *c : {cf.get(), ci.get()}) {
      const int CC = c->k.lines;
      c->a.in_b = c->a.out_b = NY * W;
      c->a.in_l = c->a.out_l = 1;
      c->a.in_e = c->a.out_e = W;
      c->a.lines = W;
      c->a.tiles_per_batch = (W + CC - 1) / CC;
      c->a.flags = F_REMAP | F_ROUNDS;
      c->grid = dim3((unsigned)(B * c->a.tiles_per_batch));
      c->a.ntiles = c->grid.x;
    }
    cf->src = cf->dst = BUF_OUT;
    ci->src = BUF_IN;
    ci->dst = BUF_WS;
    ci->first = ci->last = true;
    ci->inv_scale = (float)(1.0 / (double)NY);
    ri->src = BUF_WS;
    ri->a.scale = (float)(1.0 / (double)NX);
  }
  P->steps.push_back(std::move(rf));
  if (cf) P->steps.push_back(std::move(cf));
  if (ci) P->isteps.push_back(std::move(ci));
  P->isteps.push_back(std::move(ri));
  P->ws_bytes = NY > 1 ? (size_t)B * (size_t)NY * (size_t)W * sizeof(float2) : 0;
  P->variant = "real 2d rows+columns";
  return FFT_OK;
}

fft_status_t validate_desc(const fft_desc_t *d) {
  if (!d) return fail(FFT_E_INVALID, "desc is NULL");
  if (d->rank != 1 && d->rank != 2) return fail(FFT_E_INVALID, "rank must be 1 or 2");
  if (d->batch < 0) return fail(FFT_E_INVALID, "batch must be >= 0");
  if (d->dist < 0) return fail(FFT_E_INVALID, "dist must be >= 0");
  if (d->precision < FFT_FP32 || d->precision > FFT_BF16_SPLIT3)
    return fail(FFT_E_INVALID, "unknown precision");
  if (d->flags &
      ~(FFT_F_INPLACE | FFT_F_NO_AUTOTUNE | FFT_F_GRAPH | FFT_F_PER_SIZE | FFT_F_REAL | FFT_F_CONV))
    return fail(FFT_E_INVALID, "unknown flag bits");
  if (d->flags & FFT_F_CONV) {
    if (d->rank != 1 || d->ragged_sizes || (d->flags & FFT_F_REAL) || d->precision != FFT_FP32)
      return fail(FFT_E_UNSUPPORTED, "convolution plans are rank 1, complex, FFT_FP32, not ragged");
    if (!is_pow2(d->n[0]) || d->n[0] > kMaxN)
      return fail(FFT_E_UNSUPPORTED, "convolution lengths are powers of two <= 2^24");
  }
  if (d->flags & FFT_F_REAL) {
    if (d->ragged_sizes) return fail(FFT_E_UNSUPPORTED, "real-input plans are not ragged");
    if (d->precision != FFT_FP32) return fail(FFT_E_UNSUPPORTED, "real-input plans are FFT_FP32");
    if (d->flags & FFT_F_INPLACE) return fail(FFT_E_UNSUPPORTED, "real-input plans are out of place");
    if (d->dist != 0) return fail(FFT_E_INVALID, "real-input plans are dense (dist must be 0)");
    const int64_t nr = d->rank == 1 ? d->n[0] : d->n[1];
    if (nr <= 0 || (d->rank == 2 && d->n[0] <= 0)) return fail(FFT_E_INVALID, "sizes must be >= 1");
    if (d->rank == 1) {
      if (nr < 2 || nr % 2 || nr > kMaxN || largest_prime_factor(nr) > 7)
        return fail(FFT_E_UNSUPPORTED, "real-input lengths are even 7-smooth numbers in [2, 2^24]");
    } else if (nr < 2 || nr % 2 || nr > 2 * kSinglePassMax || largest_prime_factor(nr) > 7) {
      return fail(FFT_E_UNSUPPORTED, "real-input rows are even 7-smooth numbers in [2, 32768]");
    }
    if (d->rank == 2 && (largest_prime_factor(d->n[0]) > 7 || d->n[0] > kSinglePassMax))
      return fail(FFT_E_UNSUPPORTED, "real-input images need ny <= 16384 with prime factors <= 7");
  }
  if (d->ragged_offsets && !d->ragged_sizes)
    return fail(FFT_E_INVALID, "ragged_offsets given without ragged_sizes");
  if (d->rank == 1) {
    if (d->ragged_sizes) {
      for (int64_t i = 0; i < d->batch; ++i) {
        int64_t n = d->ragged_sizes[i];
        if (n <= 0) return fail(FFT_E_INVALID, "ragged size must be >= 1");
        if (n > kMaxN) return fail(FFT_E_UNSUPPORTED, "ragged size above 2^24");
        if (largest_prime_factor(n) > 7)
          return fail(FFT_E_UNSUPPORTED, "ragged size has a prime factor above 7");
        if (d->ragged_offsets && d->ragged_offsets[i] < 0)
          return fail(FFT_E_INVALID, "ragged offset must be >= 0");
      }
      return FFT_OK;
    }
    const int64_t n = d->n[0];
    if (n <= 0) return fail(FFT_E_INVALID, "N must be >= 1");
    if (d->flags & FFT_F_REAL) return FFT_OK;
    if (n > kMaxN) return fail(FFT_E_UNSUPPORTED, "N above 2^24");
    if (largest_prime_factor(n) > 7) return fail(FFT_E_UNSUPPORTED, "N has a prime factor above 7");
    if (d->dist != 0 && d->dist < n) return fail(FFT_E_INVALID, "dist must be 0 or >= N");
  } else {
    if (d->ragged_sizes) return fail(FFT_E_INVALID, "ragged batches are rank 1 only");
    if (d->n[0] <= 0 || d->n[1] <= 0) return fail(FFT_E_INVALID, "image sides must be >= 1");
    if (d->flags & FFT_F_REAL) return FFT_OK;
    if (largest_prime_factor(d->n[0]) > 7 || largest_prime_factor(d->n[1]) > 7 ||
        d->n[0] > kSinglePassMax || d->n[1] > kSinglePassMax)
      return fail(FFT_E_UNSUPPORTED, "rank 2 needs sides <= 16384 with prime factors <= 7");
    if (d->dist != 0 && d->dist < d->n[0] * d->n[1])
      return fail(FFT_E_INVALID, "dist must be 0 or >= ny*nx");
  }
  return FFT_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *fft_status_str(fft_status_t s) {
  switch (s) {
    case FFT_OK: return "FFT_OK";
    case FFT_E_INVALID: return "FFT_E_INVALID";
    case FFT_E_UNSUPPORTED: return "FFT_E_UNSUPPORTED";
    case FFT_E_NOMEM: return "FFT_E_NOMEM";
    case FFT_E_DEVICE: return "FFT_E_DEVICE";
    case FFT_E_INTERNAL: return "FFT_E_INTERNAL";
  }
  return "FFT_E_UNKNOWN";
}

const char *fft_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

// Host part of fft_plan: validation, kernel choice, tables, bounds checks.
static fft_status_t build_plan_once(const fft_desc_t *desc, std::unique_ptr<dpfft_plan_s> &out) {
  fft_status_t st = validate_desc(desc);
  if (st != FFT_OK) return st;
  auto P = std::make_unique<dpfft_plan_s>();
  P->rank = desc->rank;
  P->batch = desc->batch;
  P->precision = desc->precision;
  P->flags = desc->flags;
  if (desc->rank == 1) {
    P->n = desc->n[0];
    P->dist = desc->dist ? desc->dist : desc->n[0];
  } else {
    P->ny = desc->n[0];
    P->nx = desc->n[1];
    P->dist = desc->dist ? desc->dist : desc->n[0] * desc->n[1];
  }
  if (desc->precision != FFT_FP32 && desc->rank != 1)
    return fail(FFT_E_UNSUPPORTED, "MFMA precision forms are rank 1 only");
  if (desc->rank == 1 && desc->ragged_sizes && desc->precision != FFT_FP32)
    return fail(FFT_E_UNSUPPORTED, "ragged batches are FFT_FP32 only");

  struct Guard {
    Guard(const fft_desc_t *d) { g_building = d; }
    ~Guard() { g_building = nullptr; }
  } guard(desc);
  const Override ov = read_override();
  P->real = (desc->flags & FFT_F_REAL) != 0;
  if (P->real) {
    st = desc->rank == 1 ? plan_real_1d(P.get()) : plan_real_2d(P.get());
  } else if (desc->rank == 1 && desc->ragged_sizes) {
    st = plan_ragged(P.get(), desc->ragged_sizes, desc->ragged_offsets);
  } else if (desc->rank == 1) {
    if (desc->precision != FFT_FP32)
      st = plan_mfma_1d(P.get());
    else
      st = is_pow2(P->n) ? plan_pow2_1d(P.get()) : plan_mixed_1d(P.get());
  } else {
    st = is_pow2(P->ny) && is_pow2(P->nx) ? plan_pow2_2d(P.get()) : plan_mixed_2d(P.get());
  }
  if (st != FFT_OK) return st;
  if (desc->flags & FFT_F_CONV) {
    st = plan_conv(P.get());
    if (st != FFT_OK) return st;
  }

  // every index a kernel forms must stay inside its buffer
  if (P->rsizes.empty())
    P->io_elems = P->batch == 0 ? 0
                  : P->rank == 1 ? (P->batch - 1) * P->dist + P->n
                                 : (P->batch - 1) * P->dist + P->ny * P->nx;
  if (P->real) {
    const int64_t per_real = P->rank == 1 ? P->n / 2 : P->ny * (P->nx / 2);
    const int64_t per_cplx = P->rank == 1 ? P->n / 2 + 1 : P->ny * (P->nx / 2 + 1);
    P->real_elems = P->batch * per_real;
    P->cplx_elems = P->batch * per_cplx;
    if (P->steps.size() != P->isteps.size())
      return fail(FFT_E_INTERNAL, "real-input plan with unequal launch counts");
  }
  if (P->batch > 0) {
    // both step lists; a real plan's buffers differ in size by direction
    for (int dir = 0; dir < 3; ++dir) {
      const auto &list = dir == 0 ? P->steps : dir == 1 ? P->isteps : P->csteps;
      for (auto &s : list) {
        int64_t mi, mo;
        int si, di;
        s->extent(mi, mo, si, di);
        auto cap = [&](int id) -> int64_t {
          if (id == BUF_WS) return (int64_t)(P->ws_bytes / sizeof(float2));
          if (!P->real) return P->io_elems;
          const bool real_side = (id == BUF_IN) == (dir != 1);
          return real_side ? P->real_elems : P->cplx_elems;
        };
        if (mi >= cap(si) || mo >= cap(di))
          return fail(FFT_E_INTERNAL, "plan bounds check failed in " + s->describe());
        if (!s->valid())
          return fail(FFT_E_INTERNAL, "plan layout check failed in " + s->describe());
      }
    }
  }

  std::ostringstream o;
  if (!P->rsizes.empty())
    o << "rank=1 ragged count=" << P->batch;
  else if (P->rank == 1)
    o << "rank=1 N=" << P->n << " batch=" << P->batch << " dist=" << P->dist;
  else
    o << "rank=2 ny=" << P->ny << " nx=" << P->nx << " batch=" << P->batch << " dist=" << P->dist;
  o << " variant=" << P->variant << " launches=" << P->steps.size()
    << " workspace=" << P->ws_bytes << "B tables=" << P->tables.host.size() * sizeof(float2) << "B";
  if (!ov.empty()) o << " override=\"" << ov.text << "\"";
  {
    const std::string key = tune_key(desc);
    if (!key.empty()) o << " tune_key=" << key;
  }
  if (P->real) o << " real-input";
  for (auto &s : P->steps) o << "\n  " << s->describe();
  if (!P->isteps.empty()) {
    o << "\n  inverse:";
    for (auto &s : P->isteps) o << "\n  " << s->describe();
  }
  if (!P->csteps.empty()) {
    o << "\n  convolution:";
    for (auto &s : P->csteps) o << "\n  " << s->describe();
  }
  P->text = o.str();
  out = std::move(P);
  return FFT_OK;
}

// A tuning-cache entry names kernel choices of the build that wrote it; if the
// plan they lead to cannot be built (an instance since removed, a shape that
// no longer fits), the plan is built again with the heuristic choices.
static fft_status_t build_plan(const fft_desc_t *desc, std::unique_ptr<dpfft_plan_s> &out,
                               int cus) {
  set_plan_cus(cus);
  g_cache_used = false;
  g_skip_cache = false;
  fft_status_t st = build_plan_once(desc, out);
  if (st != FFT_OK && g_cache_used) {
    const std::string why = fft_last_error();
    if (getenv("DPFFT_LOG"))
      fprintf(stderr, "[dpfft] cached plan choice failed (%s); using the default plan\n",
              why.c_str());
    g_skip_cache = true;
    st = build_plan_once(desc, out);
    g_skip_cache = false;
  }
  g_cache_used = false;
  set_plan_cus(kDefaultCus);
  return st;
}

extern "C" {

fft_status_t fft_plan_dry(const fft_desc_t *desc, char *buf, size_t len) {
  std::unique_ptr<dpfft_plan_s> P;
  fft_status_t st = build_plan(desc, P, kDefaultCus);
  if (st != FFT_OK) return st;
  if (buf && len) {
    const size_t n = std::min(P->text.size(), len - 1);
    memcpy(buf, P->text.data(), n);
    buf[n] = 0;
  }
  return FFT_OK;
}

fft_status_t fft_plan(fft_plan_t *out, const fft_desc_t *desc, void *hip_stream) {
  if (!out) return fail(FFT_E_INVALID, "out is NULL");
  *out = nullptr;
  std::unique_ptr<dpfft_plan_s> P;
  fft_status_t st = build_plan(desc, P, device_cus());
  if (st != FFT_OK) return st;

  // per-function launch attributes (dynamic LDS opt-in)
  for (const auto *list : {&P->steps, &P->isteps, &P->csteps}) {
    for (auto &s : *list) {
      const hipError_t e = s->prepare();
      if (e != hipSuccess)
        return fail(FFT_E_DEVICE, std::string("kernel attributes: ") + hipGetErrorString(e));
    }
  }

  // upload every table in one allocation
  hipStream_t stream = (hipStream_t)hip_stream;
  size_t bytes = P->tables.host.size() * sizeof(float2);
  if (bytes) {
    hipError_t e = hipMalloc((void **)&P->tables.dev, bytes);
    if (e != hipSuccess) {
      P->tables.dev = nullptr;
      return fail(e == hipErrorOutOfMemory ? FFT_E_NOMEM : FFT_E_DEVICE,
                  std::string("hipMalloc(tables): ") + hipGetErrorString(e));
    }
    e = hipMemcpyAsync(P->tables.dev, P->tables.host.data(), bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess)
      return fail(FFT_E_DEVICE, std::string("table upload: ") + hipGetErrorString(e));
  }
  for (auto &s : P->steps) s->bind(P->tables.dev);
  for (auto &s : P->isteps) s->bind(P->tables.dev);
  for (auto &s : P->csteps) s->bind(P->tables.dev);
  if (getenv("DPFFT_LOG")) fprintf(stderr, "[dpfft] plan %s\n", P->text.c_str());
  *out = P.release();
  return FFT_OK;
}

static fft_status_t exec_range(fft_plan_t plan, const void *in, void *out, int direction,
                               void *workspace, void *hip_stream, int first, int count,
                               bool graphs = true) {
  if (!plan) return fail(FFT_E_INVALID, "plan is NULL");
  if (direction != FFT_FORWARD && direction != FFT_INVERSE)
    return fail(FFT_E_INVALID, "direction must be FFT_FORWARD or FFT_INVERSE");
  const int nsteps = (int)plan->steps.size();
  if (first < 0 || count < 0 || first + count > nsteps)
    return fail(FFT_E_INVALID, "step range outside the plan");
  if (plan->batch == 0) return FFT_OK;
  if (!in || !out) return fail(FFT_E_INVALID, "in/out is NULL");
  if (((uintptr_t)in | (uintptr_t)out) & 7u) return fail(FFT_E_INVALID, "in/out not 8-byte aligned");
  if (in == out && !(plan->flags & FFT_F_INPLACE))
    return fail(FFT_E_INVALID, "in == out needs FFT_F_INPLACE");
  if (plan->ws_bytes && !workspace) return fail(FFT_E_INVALID, "plan needs a workspace");
  ExecCtx ctx{in, out, workspace, (hipStream_t)hip_stream, direction == FFT_INVERSE};
  ctx.graphs = graphs;
  const auto &list = ctx.inverse && !plan->isteps.empty() ? plan->isteps : plan->steps;
  for (int i = first; i < first + count; ++i) {
    hipError_t e = list[i]->launch(ctx);
    if (e != hipSuccess) return fail(FFT_E_DEVICE, std::string("launch: ") + hipGetErrorString(e));
  }
  return FFT_OK;
}

}  // extern "C"

fft_status_t dpfft::exec_plan(fft_plan_t plan, const void *in, void *out, int direction,
                              void *workspace, void *hip_stream, bool graphs) {
  if (!plan) return fail(FFT_E_INVALID, "plan is NULL");
  return exec_range(plan, in, out, direction, workspace, hip_stream, 0, (int)plan->steps.size(),
                    graphs);
}

extern "C" {

fft_status_t fft_exec(fft_plan_t plan, const void *in, void *out, int direction, void *workspace,
                      void *hip_stream) {
  if (!plan) return fail(FFT_E_INVALID, "plan is NULL");
  return exec_range(plan, in, out, direction, workspace, hip_stream, 0, (int)plan->steps.size());
}

fft_status_t fft_exec_steps(fft_plan_t plan, const void *in, void *out, int direction,
                            void *workspace, void *hip_stream, int first, int count) {
  return exec_range(plan, in, out, direction, workspace, hip_stream, first, count);
}

int fft_plan_num_steps(fft_plan_t plan) { return plan ? (int)plan->steps.size() : 0; }

fft_status_t fft_conv_exec(fft_plan_t plan, const void *in, const void *filter,
                           int64_t filter_dist, void *out, void *workspace, void *hip_stream) {
  if (!plan) return fail(FFT_E_INVALID, "plan is NULL");
  if (!(plan->flags & FFT_F_CONV)) return fail(FFT_E_INVALID, "plan was made without FFT_F_CONV");
  if (filter_dist < 0 || (filter_dist > 0 && filter_dist < plan->n))
    return fail(FFT_E_INVALID, "filter_dist must be 0 or >= N");
  if (plan->batch == 0) return FFT_OK;
  if (!in || !out || !filter) return fail(FFT_E_INVALID, "in/out/filter is NULL");
  if (((uintptr_t)in | (uintptr_t)out | (uintptr_t)filter) & 7u)
    return fail(FFT_E_INVALID, "in/out/filter not 8-byte aligned");
  if (in == out && !(plan->flags & FFT_F_INPLACE))
    return fail(FFT_E_INVALID, "in == out needs FFT_F_INPLACE");
  if (plan->ws_bytes && !workspace) return fail(FFT_E_INVALID, "plan needs a workspace");
  ExecCtx ctx{in, out, workspace, (hipStream_t)hip_stream, false};
  ctx.filt = (const float2 *)filter;
  ctx.filt_dist = filter_dist;
  for (size_t i = 0; i < plan->csteps.size(); ++i) {
    ctx.inverse = plan->cinv[i];
    hipError_t e = plan->csteps[i]->launch(ctx);
    if (e != hipSuccess) return fail(FFT_E_DEVICE, std::string("launch: ") + hipGetErrorString(e));
  }
  return FFT_OK;
}


fft_status_t fft_destroy(fft_plan_t plan) {
  delete plan;
  return FFT_OK;
}

size_t fft_workspace_bytes(fft_plan_t plan) { return plan ? plan->ws_bytes : 0; }

size_t fft_plan_describe(fft_plan_t plan, char *buf, size_t len) {
  if (!plan) return 0;
  const std::string &t = plan->text;
  if (buf && len) {
    size_t n = t.size() < len - 1 ? t.size() : len - 1;
    memcpy(buf, t.data(), n);
    buf[n] = 0;
  }
  return t.size();
}

}  // extern "C"
