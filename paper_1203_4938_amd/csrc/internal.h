// Helpers shared by the plan builders of the library (host only).
#pragma once
#include <stdint.h>

#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "../../include/dpfft.h"

struct dpfft_plan_s;

namespace dpfft {

constexpr int64_t kMaxN = int64_t(1) << 24;
constexpr int kSinglePassMax = 16384;  // longest line one workgroup transforms
constexpr int kLdsBytes = 160 * 1024;  // LDS of one CU

// Record `msg` as this thread's last error and return `s`.
fft_status_t fail(fft_status_t s, const std::string &msg);

// Largest divisor of n that is <= sqrt(n).
int64_t split_factor(int64_t n);

// Compute units of an MI355X; the CU count dry plans assume.
constexpr int kDefaultCus = 256;

// Compute units of the current device (kDefaultCus if it cannot be queried).
int device_cus();

// CU count the plan builders on this thread size persistent grids for.
void set_plan_cus(int cus);

// Workgroups that fit on the device at once for `lds_bytes` and `threads`
// (host arithmetic only, for the CU count set by set_plan_cus).
int resident_for(int lds_bytes, int threads);

// Kernel-choice overrides for the plan builders, per launch step i:
//   c<i>=<C>   lines (rows or columns) per workgroup
//   p<i>=0|1   persistent variant off / on
//   t<i>=<T>   threads per workgroup (instances differing in elements per thread)
//   h<i>=1|2   sub-lines per line: plain tiles / split-first tiles
//   o=0|1      radix order of runtime-radix lengths: powers of two first / odd first
//   k=<n>      two-pass plans: transforms per chunk (0 = the whole batch at once)
//   s=<n>      power-of-two four-step: log2 of the column length N1; ragged
//              lengths: the column length n1 itself
//   f=<n>      ragged lengths: 0 single pass in a 256-thread workgroup, 1
//              four-step, 2 single pass in a 1024-thread workgroup (a form
//              that does not fit a length leaves that length to the heuristic)
//   b=0|1      ragged lengths: the heuristic may not / may choose the
//              1024-thread single pass
//   x=0|1      ragged four-step lines: runtime-radix passes only / also the
//              compile-time instances of common lengths
// Sources, first match wins: the autotuner while it times candidates, the
// DPFFT_FORCE_PLAN environment variable, the tuning cache entry of the plan.
struct Override {
  int c[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
  int p[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
  int t[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
  int h[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
  int order = -1;
  int chunk = -1;
  int split = -1;
  int form = -1;
  int big = -1;
  int ct = -1;
  std::string text;
  bool empty() const { return text.empty(); }
};
Override parse_override(const std::string &text);

// The override in force for length L of the ragged batch being planned.
Override read_ragged_override(int64_t L);

// Tuning-cache key of one length of ragged batches.
std::string ragged_tune_key(int64_t L);

// Override strings the autotuner times for one ragged length.
std::vector<std::string> ragged_candidates(int64_t L);

// Autotune every distinct length of a ragged descriptor (see fft_autotune).
fft_status_t autotune_ragged(const fft_desc_t *desc, void *hip_stream, int reps,
                             std::string *report);

// Store several tuning-cache entries (one write of the cache file).
void tune_cache_store_all(const std::vector<std::pair<std::string, std::string>> &kv);

// Thread-local override installed by the autotuner around candidate plans.
void set_tuner_override(const Override *o);
const Override *tuner_override();

// Tuning cache: in-process map, loaded on first use from the JSON file named by
// DPFFT_TUNE_CACHE (a missing or corrupt file leaves it empty).
bool tune_cache_lookup(const std::string &key, std::string *value);
void tune_cache_store(const std::string &key, const std::string &value);

struct LineStep;
// A power-of-two line launch for (L, map, omap, tw4): the kernel choice (at
// most `cmax` lines per tile unless an instance is the measured default of its
// shape; `step` indexes the override), its Stockham and two-level pass tables
// added to the plan; layout, grid and buffers are left to the caller.
std::unique_ptr<LineStep> make_line_step(dpfft_plan_s *P, const char *name, int L, int map,
                                         int omap, bool tw4, int cmax, int step,
                                         int64_t lines_total, const Override &ov);

// fft_exec with `workspace` as given; graphs = false launches the kernels of
// graph plans directly instead of instantiating or replaying a HIP graph.
fft_status_t exec_plan(dpfft_plan_s *plan, const void *in, void *out, int direction,
                       void *workspace, void *hip_stream, bool graphs);

// The launches of fft_conv_exec for a power-of-two FFT_F_CONV plan.
fft_status_t plan_conv(dpfft_plan_s *P);

}  // namespace dpfft

// key of a plan in the tuning cache ("" = not tunable)
std::string tune_key(const fft_desc_t *d);
fft_status_t plan_ragged(dpfft_plan_s *P, const int64_t *sizes, const int64_t *offsets);
