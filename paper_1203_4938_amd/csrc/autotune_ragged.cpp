// Autotuner of ragged batches: a choice per distinct length.
//
// For every length L of the descriptor, each candidate choice (radix order,
// single pass in a 256- or 1024-thread workgroup, four-step and its split) is
// built as a ragged plan of L-point signals only -- as many as the batch has,
// and at least 2^21 points so that the launches fill the device -- and its
// persistent launches are timed forward with HIP events.  The fastest choice
// of each length goes into the tuning cache under that length's key; the
// ragged planner reads it for every batch that contains the length.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"
#include "plan.h"

namespace dpfft {

namespace {

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  bool reserve(size_t need) {
    if (need <= bytes) return true;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    if (hipMalloc(&p, need) != hipSuccess) return false;
    bytes = need;
    return hipMemset(p, 0, need) == hipSuccess;
  }
};

}  // namespace

fft_status_t autotune_ragged(const fft_desc_t *desc, void *hip_stream, int reps,
                             std::string *report) {
  constexpr int64_t kMinPoints = int64_t(1) << 21;
  std::map<int64_t, int64_t> count;
  for (int64_t i = 0; i < desc->batch; ++i) ++count[desc->ragged_sizes[i]];
  hipStream_t stream = (hipStream_t)hip_stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(FFT_E_DEVICE, "hipEventCreate failed");
  DevBuf in, out, ws;
  std::vector<std::pair<std::string, std::string>> chosen;
  std::map<std::string, int> tally;  // chosen form -> lengths
  std::ostringstream rep;
  fft_status_t status = FFT_OK;
  double total_ms = 0;
  for (const auto &kv : count) {
    const int64_t L = kv.first;
    const std::vector<std::string> cands = ragged_candidates(L);
    if (cands.empty()) continue;
    const int64_t k = std::max(kv.second, (kMinPoints + L - 1) / L);
    std::vector<int64_t> sizes((size_t)k, L);
    fft_desc_t d{};
    d.rank = 1;
    d.batch = k;
    d.ragged_sizes = sizes.data();
    d.precision = FFT_FP32;
    d.flags = FFT_F_NO_AUTOTUNE;
    std::string best = cands[0];
    float best_ms = 1e30f;
    std::ostringstream line;
    line << "L=" << L << " (" << kv.second << " signals, timed on " << k << "):";
    for (const auto &c : cands) {
      if (cands.size() == 1) break;  // nothing to compare
      const Override ov = parse_override(c);
      set_tuner_override(&ov);
      fft_plan_t plan = nullptr;
      fft_status_t st = fft_plan(&plan, &d, hip_stream);
      set_tuner_override(nullptr);
      if (st != FFT_OK) {
        line << " [" << c << ": " << fft_status_str(st) << "]";
        continue;
      }
      if (!in.reserve((size_t)plan->io_elems * sizeof(float2)) ||
          !out.reserve((size_t)plan->io_elems * sizeof(float2)) ||
          !ws.reserve(std::max<size_t>(fft_workspace_bytes(plan), 8))) {
        fft_destroy(plan);
        status = fail(FFT_E_NOMEM, "autotune buffers");
        break;
      }
      float ms = 0;
      for (int w = 0; w < 2 && st == FFT_OK; ++w)
        st = fft_exec(plan, in.p, out.p, FFT_FORWARD, ws.p, hip_stream);
      if (st == FFT_OK && hipEventRecord(e0, stream) == hipSuccess) {
        for (int r = 0; r < reps && st == FFT_OK; ++r)
          st = fft_exec(plan, in.p, out.p, FFT_FORWARD, ws.p, hip_stream);
        if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
          st = FFT_E_DEVICE;
      }
      fft_destroy(plan);
      if (st != FFT_OK) {
        line << " [" << c << ": " << fft_status_str(st) << "]";
        continue;
      }
      ms /= (float)reps;
      line << " [" << c << ": " << ms << " ms]";
      if (ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
    if (status != FFT_OK) break;
    if (best_ms < 1e30f) total_ms += best_ms * (double)kv.second / (double)k;
    line << " -> " << best;
    chosen.push_back({ragged_tune_key(L), best});
    const Override b = parse_override(best);
    ++tally[b.form == 1 ? "four-step" : b.form == 2 ? "1024-thread single pass" : "single pass"];
    if (getenv("DPFFT_LOG")) fprintf(stderr, "[dpfft] %s\n", line.str().c_str());
  }
  // The per-length timings see one length at a time; the batch shares its
  // launches between lengths.  Keep the tuned choices only if the whole batch
  // runs faster with them than with the heuristic ones ("h" entries: the
  // heuristic, recorded as tuned).
  float t_tuned = 0, t_heur = 0;
  if (status == FFT_OK) {
    tune_cache_store_all(chosen);
    fft_desc_t d = *desc;
    d.flags &= ~(uint32_t)(FFT_F_PER_SIZE | FFT_F_GRAPH | FFT_F_NO_AUTOTUNE);
    for (int pass = 0; pass < 2 && status == FFT_OK; ++pass) {
      if (pass == 1) d.flags |= FFT_F_NO_AUTOTUNE;
      fft_plan_t plan = nullptr;
      fft_status_t st = fft_plan(&plan, &d, hip_stream);
      if (st != FFT_OK) {
        status = st;
        break;
      }
      float ms = 0;
      if (!in.reserve((size_t)plan->io_elems * sizeof(float2)) ||
          !out.reserve((size_t)plan->io_elems * sizeof(float2)) ||
          !ws.reserve(std::max<size_t>(fft_workspace_bytes(plan), 8)))
        st = fail(FFT_E_NOMEM, "autotune buffers");
      for (int w = 0; w < 2 && st == FFT_OK; ++w)
        st = fft_exec(plan, in.p, out.p, FFT_FORWARD, ws.p, hip_stream);
      if (st == FFT_OK && hipEventRecord(e0, stream) == hipSuccess) {
        for (int r = 0; r < reps && st == FFT_OK; ++r)
          st = fft_exec(plan, in.p, out.p, FFT_FORWARD, ws.p, hip_stream);
        if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
          st = FFT_E_DEVICE;
      }
      fft_destroy(plan);
      if (st != FFT_OK) {
        status = st;
        break;
      }
      (pass == 0 ? t_tuned : t_heur) = ms / (float)reps;
    }
    if (status == FFT_OK && t_heur < t_tuned) {
      for (auto &e : chosen) e.second = "h";
      tune_cache_store_all(chosen);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status != FFT_OK) return status;
  rep << "ragged: tuned " << chosen.size() << " lengths (";
  bool first = true;
  for (const auto &t : tally) {
    rep << (first ? "" : ", ") << t.second << " " << t.first;
    first = false;
  }
  rep << "); estimated batch time from the per-length timings " << total_ms
      << " ms; whole batch " << t_tuned << " ms tuned, " << t_heur << " ms heuristic: "
      << (t_heur < t_tuned ? "heuristic kept" : "tuned choices kept") << "\n";
  *report = rep.str();
  return FFT_OK;
}

}  // namespace dpfft
