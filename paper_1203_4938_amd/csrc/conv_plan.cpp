// Plans of the fused circular convolution (FFT_F_CONV): the launches of
// fft_conv_exec and their tables.
#include <sstream>
#include <string>

#include "internal.h"
#include "plan.h"
#include "twiddle.h"

namespace dpfft {

void ConvStep::bind(const float2 *tables) {
  a.tw = tables + tw_off;
  a.tw2 = tables + tw2_off;
  if (k.rows4) {
    a.tw4_lo = tables + tw4_lo_off;
    a.tw4_hi = tables + tw4_hi_off;
  }
}

hipError_t ConvStep::launch(const ExecCtx &ctx) const {
  const float2 *s = buf_c(ctx, src, 0);
  float2 *d = buf_m(ctx, dst, 0);
  LineArgs args = a;
  // single pass: one line per signal, spectra filt_dist apart per line;
  // four-step rows: N1 rows per signal, spectra filt_dist apart per signal
  ConvArgs f{ctx.filt, k.rows4 ? ctx.filt_dist : 0, k.rows4 ? 0 : ctx.filt_dist};
  void *kargs[] = {(void *)&s, (void *)&d, (void *)&args, (void *)&f};
  return hipLaunchKernel(k.fn, grid, dim3(k.threads), kargs, 0, ctx.stream);
}

void ConvStep::extent(int64_t &max_in, int64_t &max_out, int &src_id, int &dst_id) const {
  const int64_t nb = (int64_t)grid.x / a.tiles_per_batch;
  const int64_t last_line = std::min<int64_t>(a.lines, a.tiles_per_batch * k.lines) - 1;
  max_in = (nb - 1) * a.in_b + last_line * a.in_l + (L - 1);
  max_out = (nb - 1) * a.out_b + last_line * a.out_l + (L - 1);
  src_id = src;
  dst_id = dst;
}

bool ConvStep::valid() const {
  if (!k.fn || a.in_e != 1 || a.out_e != 1) return false;
  if (k.rows4) {
    // whole row tiles, and every batch item a whole number of tiles
    return a.lines % k.lines == 0 && (int64_t)grid.x % a.tiles_per_batch == 0;
  }
  return true;
}

std::string ConvStep::describe() const {
  std::ostringstream o;
  o << name << ": L=" << L << " C=" << k.lines << " threads=" << k.threads << " grid=" << grid.x
    << " lds=" << k.lds_bytes << "B" << (k.rows4 ? " (four-step rows, filter tile via LDS)" : "");
  return o.str();
}

namespace {

bool pick_conv(int L, bool rows4, ConvKernel *out) {
  ConvKernel cand[8];
  const int n = std::min(8, list_conv_kernels(L, rows4, cand, 8));
  const char *env = getenv("DPFFT_CONV_THREADS");  // opt-in instance (tests, timing)
  const int want = env ? atoi(env) : 0;
  for (int i = 0; i < n; ++i)
    if (want > 0 ? cand[i].threads == want : cand[i].preferred) {
      *out = cand[i];
      return true;
    }
  for (int i = 0; i < n; ++i)
    if (cand[i].preferred) {
      *out = cand[i];
      return true;
    }
  return false;
}

std::unique_ptr<ConvStep> make_conv(dpfft_plan_s *P, const char *name, int L, bool rows4) {
  auto s = std::make_unique<ConvStep>();
  if (!pick_conv(L, rows4, &s->k)) return nullptr;
  s->L = L;
  s->name = name;
  s->tw_off = P->tables.add(stockham_table_pow2(L, s->k.ept));
  std::vector<std::complex<double>> lo, hi;
  int lg = 0;
  while ((1 << lg) < L) ++lg;
  fourstep_tables(L, tw2_shift(lg), lo, hi);
  lo.insert(lo.end(), hi.begin(), hi.end());
  s->tw2_off = P->tables.add(lo);
  s->a.in_e = s->a.out_e = 1;
  return s;
}

}  // namespace

// Single pass for N <= 16384: one launch.  Longer power-of-two N = N1 N2 (the
// split of the plan's four-step): forward column pass (in -> workspace), the
// fused row launch (workspace in place), inverse column pass (workspace ->
// out).
fft_status_t plan_conv(dpfft_plan_s *P) {
  const int64_t N = P->n, B = P->batch, D = P->dist;
  const double invn = 1.0 / (double)N;
  if (N <= kSinglePassMax) {
    auto s = make_conv(P, "conv_single_pass", (int)N, false);
    if (!s) return fail(FFT_E_UNSUPPORTED, "no convolution kernel for N=" + std::to_string(N));
    const int C = s->k.lines;
    s->a.in_b = s->a.out_b = 0;
    s->a.in_l = s->a.out_l = D;
    s->a.lines = B;
    s->a.tiles_per_batch = (B + C - 1) / C;
    s->a.ntiles = s->a.tiles_per_batch;
    s->a.scale = (float)invn;
    s->grid = dim3((unsigned)s->a.tiles_per_batch);
    P->csteps.push_back(std::move(s));
    P->cinv.push_back(false);
    return FFT_OK;
  }
  int lg = 0;
  while ((int64_t(1) << lg) < N) ++lg;
  const int lg1 = lg / 2;
  const int N1 = 1 << lg1, N2 = 1 << (lg - lg1);
  Override none;
  auto a = make_line_step(P, "conv_fourstep_columns", N1, LINE_FAST, LINE_FAST, true,
                          16, 0, B * N2, none);
  auto r = make_conv(P, "conv_fourstep_rows", N2, true);
  auto c = make_line_step(P, "conv_columns_inverse", N1, LINE_FAST, LINE_FAST, false, 16, 2,
                          B * N2, none);
  if (!a || !r || !c)
    return fail(FFT_E_UNSUPPORTED, "no four-step convolution kernels for N=" + std::to_string(N));
  const int shift = (lg + 1) / 2;
  std::vector<std::complex<double>> lo, hi;
  fourstep_tables(N, shift, lo, hi);
  const size_t lo_off = P->tables.add(lo), hi_off = P->tables.add(hi);

  // forward column pass: x[n1 N2 + n2] -> Y[k1][n2] (the four-step's pass A)
  a->has_tw4 = true;
  a->tw4_lo_off = lo_off;
  a->tw4_hi_off = hi_off;
  a->a.tw4_shift = shift;
  a->a.in_b = D;
  a->a.in_l = 1;
  a->a.in_e = N2;
  a->a.out_b = N;
  a->a.out_l = 1;
  a->a.out_e = N2;
  a->a.lines = N2;
  a->a.tiles_per_batch = N2 / a->k.lines;
  a->a.flags = F_REMAP | (a->k.lines >= 8 ? F_ROUNDS : 0u);
  a->grid = dim3((unsigned)(B * a->a.tiles_per_batch));
  a->a.ntiles = a->grid.x;
  a->src = BUF_IN;
  a->dst = BUF_WS;

  // rows of Y in place: forward, product with H / N, inverse, w_N^{-k1 n2}
  r->tw4_lo_off = lo_off;
  r->tw4_hi_off = hi_off;
  r->a.tw4_shift = shift;
  r->a.in_b = r->a.out_b = N;
  r->a.in_l = r->a.out_l = N2;
  r->a.lines = N1;
  r->a.tiles_per_batch = N1 / r->k.lines;
  r->a.ntiles = B * r->a.tiles_per_batch;
  r->a.scale = (float)invn;
  r->grid = dim3((unsigned)r->a.ntiles);
  r->src = BUF_WS;
  r->dst = BUF_WS;

  // inverse column pass over k1 (swap in and out, no further scale), stored
  // in natural order
  c->a.in_b = N;
  c->a.in_l = 1;
  c->a.in_e = N2;
  c->a.out_b = D;
  c->a.out_l = 1;
  c->a.out_e = N2;
  c->a.lines = N2;
  c->a.tiles_per_batch = N2 / c->k.lines;
  c->a.flags = F_REMAP | (c->k.lines >= 8 ? F_ROUNDS : 0u);
  c->grid = dim3((unsigned)(B * c->a.tiles_per_batch));
  c->a.ntiles = c->grid.x;
  c->first = c->last = true;
  c->inv_scale = 1.0f;
  c->src = BUF_WS;
  c->dst = BUF_OUT;

  P->csteps.push_back(std::move(a));
  P->cinv.push_back(false);
  P->csteps.push_back(std::move(r));
  P->cinv.push_back(false);
  P->csteps.push_back(std::move(c));
  P->cinv.push_back(true);
  P->ws_bytes = std::max(P->ws_bytes, (size_t)B * (size_t)N * sizeof(float2));
  return FFT_OK;
}

}  // namespace dpfft
