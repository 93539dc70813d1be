// Autotuner: times the compiled kernel variants of a plan on the device and
// remembers the fastest per (architecture, shape, batch bucket, precision).
//
// Candidates are expressed as overrides of the planner's choices (tile width
// per launch, persistent variant, radix order of runtime-radix lengths, chunk
// size of two-pass plans); each
// is built by the normal plan builder, so every candidate passes the same
// validation and bounds checks as a default plan.  Results live in an
// in-process map, optionally persisted as JSON in the file named by
// DPFFT_TUNE_CACHE; a missing or unreadable file simply means "no entries".
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"
#include "kernels.h"
#include "mixed.h"
#include "plan.h"

namespace dpfft {

Override parse_override(const std::string &text) {
  Override o;
  std::istringstream in(text);
  std::string tok;
  while (in >> tok) {
    char kind = 0;
    int idx = -1, val = -1;
    if (sscanf(tok.c_str(), "o=%d", &val) == 1) {
      o.order = val;
    } else if (sscanf(tok.c_str(), "k=%d", &val) == 1) {
      o.chunk = val;
    } else if (sscanf(tok.c_str(), "s=%d", &val) == 1) {
      o.split = val;
    } else if (sscanf(tok.c_str(), "f=%d", &val) == 1) {
      o.form = val;
    } else if (sscanf(tok.c_str(), "b=%d", &val) == 1) {
      o.big = val;
    } else if (sscanf(tok.c_str(), "x=%d", &val) == 1) {
      o.ct = val;
    } else if (sscanf(tok.c_str(), "%c%d=%d", &kind, &idx, &val) == 3 && idx >= 0 && idx < 8) {
      if (kind == 'c') o.c[idx] = val;
      if (kind == 'p') o.p[idx] = val;
      if (kind == 't') o.t[idx] = val;
      if (kind == 'h') o.h[idx] = val;
    }
  }
  o.text = text;
  return o;
}

namespace {
thread_local const Override *t_tuner = nullptr;

std::mutex g_cache_mu;
std::map<std::string, std::string> g_cache;
bool g_cache_loaded = false;

// Minimal reader of the cache file: {"dpfft_tune_cache": 1, "entries": {"k": "v", ...}}
void load_cache_locked() {
  g_cache_loaded = true;
  const char *path = getenv("DPFFT_TUNE_CACHE");
  if (!path) return;
  std::ifstream f(path);
  if (!f) return;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  const size_t e = s.find("\"entries\"");
  if (s.find("\"dpfft_tune_cache\"") == std::string::npos || e == std::string::npos) {
    if (getenv("DPFFT_LOG")) fprintf(stderr, "[dpfft] ignoring unreadable tune cache %s\n", path);
    return;
  }
  std::map<std::string, std::string> got;
  size_t pos = s.find('{', e);
  if (pos == std::string::npos) return;
  ++pos;
  auto read_str = [&](std::string &out) -> bool {
    pos = s.find_first_not_of(" \t\r\n,", pos);
    if (pos == std::string::npos || s[pos] != '"') return false;
    const size_t q = s.find('"', pos + 1);
    if (q == std::string::npos) return false;
    out = s.substr(pos + 1, q - pos - 1);
    pos = q + 1;
    return true;
  };
  while (true) {
    pos = s.find_first_not_of(" \t\r\n,", pos);
    if (pos == std::string::npos) return;  // truncated: keep nothing
    if (s[pos] == '}') break;
    std::string k, v;
    if (!read_str(k)) return;
    pos = s.find_first_not_of(" \t\r\n", pos);
    if (pos == std::string::npos || s[pos] != ':') return;
    ++pos;
    if (!read_str(v)) return;
    got[k] = v;
  }
  g_cache.insert(got.begin(), got.end());
}

void save_cache_locked() {
  const char *path = getenv("DPFFT_TUNE_CACHE");
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  std::ofstream f(tmp);
  if (!f) return;
  f << "{\"dpfft_tune_cache\": 1, \"entries\": {";
  bool first = true;
  for (const auto &kv : g_cache) {
    f << (first ? "\n  " : ",\n  ") << '"' << kv.first << "\": \"" << kv.second << '"';
    first = false;
  }
  f << "\n}}\n";
  f.close();
  rename(tmp.c_str(), path);
}
}  // namespace

void set_tuner_override(const Override *o) { t_tuner = o; }
const Override *tuner_override() { return t_tuner; }

bool tune_cache_lookup(const std::string &key, std::string *value) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  if (!g_cache_loaded) load_cache_locked();
  auto it = g_cache.find(key);
  if (it == g_cache.end()) return false;
  *value = it->second;
  return true;
}

void tune_cache_store(const std::string &key, const std::string &value) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  if (!g_cache_loaded) load_cache_locked();
  g_cache[key] = value;
  save_cache_locked();
}

void tune_cache_store_all(const std::vector<std::pair<std::string, std::string>> &kv) {
  std::lock_guard<std::mutex> lk(g_cache_mu);
  if (!g_cache_loaded) load_cache_locked();
  for (const auto &e : kv) g_cache[e.first] = e.second;
  save_cache_locked();
}

}  // namespace dpfft

using namespace dpfft;

std::string tune_key(const fft_desc_t *d) {
  if (!d || d->ragged_sizes || d->precision != FFT_FP32 || d->batch <= 0 || (d->flags & FFT_F_REAL))
    return "";
  int bucket = 0;
  while ((int64_t(1) << (bucket + 1)) <= d->batch) ++bucket;
  std::ostringstream o;
  char reg[20];
  snprintf(reg, sizeof reg, "%016llx", (unsigned long long)line_registry_digest());
  o << "gfx950|k=" << reg << "|r" << d->rank << "|n=" << d->n[0];
  if (d->rank == 2) o << "x" << d->n[1];
  o << "|b=2^" << bucket << "|fp32";
  return o.str();
}

namespace {

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// Override strings worth timing for this descriptor.
std::vector<std::string> candidates(const fft_desc_t *d) {
  std::vector<std::string> out;
  KernelInfo ks[32], kb[32];
  auto cs = [&](int L, int map, int omap, bool tw4, KernelInfo *k) {
    int n = std::min(32, list_line_kernels(L, map, omap, tw4, k, 32));
    std::vector<std::string> v;
    for (int i = 0; i < n; ++i)
      if (k[i].threads <= 1024)
        v.push_back(std::to_string(k[i].lines) + " " + std::to_string((int)k[i].persistent) + " " +
                    std::to_string(k[i].threads) + " " + std::to_string(k[i].sub));
    return v;
  };
  auto enc = [](int step, const std::string &cpt) {
    std::istringstream in(cpt);
    int c, p, t, h;
    in >> c >> p >> t >> h;
    const std::string i = std::to_string(step);
    return "c" + i + "=" + std::to_string(c) + " p" + i + "=" + std::to_string(p) + " t" + i + "=" +
           std::to_string(t) + " h" + i + "=" + std::to_string(h);
  };
  // two-pass plans: chunk sizes keeping one chunk's intermediate within 64,
  // 128 or 256 MiB (the memory-side cache holds 256 MB)
  auto chunks = [&](int64_t per_bytes) {
    for (int64_t mib : {64, 128, 256}) {
      const int64_t k = std::max<int64_t>(1, (mib << 20) / per_bytes);
      if (k < d->batch) out.push_back("k=" + std::to_string(k));
    }
  };
  if (d->rank == 2) {
    for (const auto &r : cs((int)d->n[1], ELEM_FAST, ELEM_FAST, false, ks))
      for (const auto &c : cs((int)d->n[0], LINE_FAST, LINE_FAST, false, kb))
        out.push_back(enc(0, r) + " " + enc(1, c));
    chunks(d->n[0] * d->n[1] * 8);
    return out;
  }
  const int64_t N = d->n[0];
  if (is_pow2(N)) {
    if (N <= 16384) {
      for (const auto &r : cs((int)N, ELEM_FAST, ELEM_FAST, false, ks)) out.push_back(enc(0, r));
    } else {
      int lg = 0;
      while ((int64_t(1) << lg) < N) ++lg;
      // the balanced split N1 = 2^(lg/2) and its two neighbours, each named
      // explicitly (the planner's default split is not always the balanced one)
      for (int lg1 : {lg / 2, lg / 2 - 1, lg / 2 + 1}) {
        if (lg1 < 1 || lg1 >= lg) continue;
        const int N1 = 1 << lg1, N2 = 1 << (lg - lg1);
        const std::string sp = "s=" + std::to_string(lg1) + " ";
        for (const auto &a : cs(N1, LINE_FAST, LINE_FAST, true, ks))
          for (const auto &b : cs(N2, ELEM_FAST, LINE_FAST, false, kb))
            out.push_back(sp + enc(0, a) + " " + enc(1, b));
      }
      chunks(N * 8);
    }
    return out;
  }
  for (int order : {0, 1}) {
    if (N <= 16384) {
      MixedPlan mp{};
      if (!mixed_radices(N, &mp, order)) continue;
      for (int C = 1; C * mp.T <= 1024; C *= 2)
        out.push_back("o=" + std::to_string(order) + " c0=" + std::to_string(C));
    } else {
      out.push_back("o=" + std::to_string(order));
    }
  }
  return out;
}

}  // namespace

extern "C" fft_status_t fft_autotune(const fft_desc_t *desc, void *hip_stream, int reps,
                                     char *report, size_t len) {
  if (!desc) return fail(FFT_E_INVALID, "desc is NULL");
  if (reps <= 0) reps = 10;
  const std::string key = tune_key(desc);
  std::ostringstream rep;
  auto finish = [&](fft_status_t st) {
    const std::string r = rep.str();
    if (report && len) {
      const size_t n = std::min(r.size(), len - 1);
      memcpy(report, r.data(), n);
      report[n] = 0;
    }
    return st;
  };
  if (desc->ragged_sizes && desc->precision == FFT_FP32 && desc->batch > 0) {
    std::string r;
    const fft_status_t st = autotune_ragged(desc, hip_stream, reps, &r);
    rep << r;
    return finish(st);
  }
  if (key.empty()) {
    rep << "nothing to tune (precision form, real-input or empty batch)";
    return finish(FFT_OK);
  }
  const std::vector<std::string> cands = candidates(desc);
  hipStream_t stream = (hipStream_t)hip_stream;
  void *in = nullptr, *out = nullptr, *ws = nullptr;
  size_t io_bytes = 0, ws_bytes = 0;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return finish(fail(FFT_E_DEVICE, "hipEventCreate failed"));
  std::string best;
  float best_ms = 1e30f;
  fft_status_t status = FFT_OK;
  for (const auto &c : cands) {
    const Override ov = parse_override(c);
    set_tuner_override(&ov);
    fft_plan_t plan = nullptr;
    fft_status_t st = fft_plan(&plan, desc, hip_stream);
    set_tuner_override(nullptr);
    if (st != FFT_OK) {
      rep << c << ": skipped (" << fft_status_str(st) << ")\n";
      continue;
    }
    const size_t need_io = (size_t)plan->io_elems * sizeof(float2), need_ws = fft_workspace_bytes(plan);
    bool ok = true;
    if (need_io > io_bytes) {
      if (in) (void)hipFree(in);
      if (out) (void)hipFree(out);
      in = out = nullptr;
      ok = hipMalloc(&in, need_io) == hipSuccess && hipMalloc(&out, need_io) == hipSuccess;
      if (ok) ok = hipMemsetAsync(in, 0, need_io, stream) == hipSuccess;
      io_bytes = ok ? need_io : 0;
    }
    if (ok && need_ws > ws_bytes) {
      if (ws) (void)hipFree(ws);
      ws = nullptr;
      ok = hipMalloc(&ws, need_ws) == hipSuccess;
      ws_bytes = ok ? need_ws : 0;
    }
    if (!ok) {
      fft_destroy(plan);
      status = fail(FFT_E_NOMEM, "autotune buffers");
      break;
    }
    float ms = 0;
    for (int w = 0; w < 2 && st == FFT_OK; ++w) st = fft_exec(plan, in, out, FFT_FORWARD, ws, hip_stream);
    if (st == FFT_OK && hipEventRecord(e0, stream) == hipSuccess) {
      for (int r = 0; r < reps && st == FFT_OK; ++r) st = fft_exec(plan, in, out, FFT_FORWARD, ws, hip_stream);
      if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
        st = FFT_E_DEVICE;
    }
    fft_destroy(plan);
    if (st != FFT_OK) {
      rep << c << ": failed (" << fft_status_str(st) << ")\n";
      continue;
    }
    ms /= (float)reps;
    rep << c << ": " << ms << " ms\n";
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  }
  if (in) (void)hipFree(in);
  if (out) (void)hipFree(out);
  if (ws) (void)hipFree(ws);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status != FFT_OK) return finish(status);
  if (best.empty()) return finish(fail(FFT_E_INTERNAL, "no autotune candidate ran"));
  tune_cache_store(key, best);
  rep << "best: " << best << " (" << best_ms << " ms) for " << key << "\n";
  return finish(FFT_OK);
}
