// Plan object: an ordered list of kernel launches plus the device tables they
// read.  Built once by fft_plan, replayed by fft_exec.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <complex>
#include <memory>
#include <string>
#include <vector>

#include "../../include/dpfft.h"
#include "conv.h"
#include "kernels.h"
#include "mixed.h"
#include "mfma.h"
#include "real.h"

namespace dpfft {

enum BufId : int { BUF_IN = 0, BUF_OUT = 1, BUF_WS = 2 };

struct ExecCtx {
  const void *in;
  void *out;
  void *ws;
  hipStream_t stream;
  bool inverse;
  const float2 *filt = nullptr;  // convolution launches: filter spectra
  int64_t filt_dist = 0;         // elements between consecutive spectra (0 = shared)
  bool graphs = true;            // graph plans may instantiate and replay HIP graphs
};

inline const float2 *buf_c(const ExecCtx &c, int id, int64_t off) {
  const float2 *p = id == BUF_IN ? (const float2 *)c.in
                    : id == BUF_OUT ? (const float2 *)c.out
                                    : (const float2 *)c.ws;
  return p + off;
}
inline float2 *buf_m(const ExecCtx &c, int id, int64_t off) {
  float2 *p = id == BUF_IN ? (float2 *)c.in : id == BUF_OUT ? (float2 *)c.out : (float2 *)c.ws;
  return p + off;
}

// Host staging for all device tables of a plan: one allocation per plan.
struct TableSet {
  std::vector<float2> host;
  size_t add(const std::vector<std::complex<double>> &t);  // returns element offset
  size_t add_raw(const std::vector<float2> &t);
  size_t add_bytes(const void *p, size_t bytes);           // 8-byte units
  float2 *dev = nullptr;
};

struct Step {
  virtual ~Step() = default;
  // resolve table offsets against the uploaded device tables
  virtual void bind(const float2 *tables) = 0;
  virtual hipError_t launch(const ExecCtx &ctx) const = 0;
  virtual std::string describe() const = 0;
  // largest element index read from `src` / written to `dst` (-1 = none)
  virtual void extent(int64_t &max_in, int64_t &max_out, int &src_id, int &dst_id) const = 0;
  // layout assumptions of the kernel hold and every needed instance exists
  virtual bool valid() const = 0;
  // device-side set-up at fft_plan time (function attributes); never called
  // for dry plans
  virtual hipError_t prepare() const { return hipSuccess; }
};

struct LineStep : Step {
  KernelInfo k;
  int L = 0;
  dim3 grid;
  int src = BUF_IN, dst = BUF_OUT;
  int64_t src_off = 0, dst_off = 0;  // element offsets into the buffers (chunked plans)
  LineArgs a{};
  size_t tw_off = 0, tw4_lo_off = 0, tw4_hi_off = 0, tw2_off = 0;
  int resident = 0;  // persistent instances: workgroups resident on the device
  bool has_tw4 = false;
  bool first = false, last = false;  // receive the inverse swap / scale
  float inv_scale = 1.0f;
  std::string name;
  void bind(const float2 *tables) override;
  hipError_t launch(const ExecCtx &ctx) const override;
  std::string describe() const override;
  void extent(int64_t &max_in, int64_t &max_out, int &src_id, int &dst_id) const override;
  bool valid() const override;
  int inverse_sw() const;
};

struct MixedStep : Step {
  MixedArgs a{};
  const void *fn_sw[4] = {};
  int map = ELEM_FAST, omap = ELEM_FAST;
  bool tw4 = false;
  dim3 grid;
  int threads = 0;
  int lds_bytes = 0;
  int src = BUF_IN, dst = BUF_OUT;
  size_t tw2_off = 0, tw4_lo_off = 0, tw4_hi_off = 0;
  bool first = false, last = false;
  float inv_scale = 1.0f;
  std::string name;
  int inverse_sw() const { return (first ? 1 : 0) | (last ? 2 : 0); }
  void bind(const float2 *tables) override;
  hipError_t launch(const ExecCtx &ctx) const override;
  std::string describe() const override;
  void extent(int64_t &max_in, int64_t &max_out, int &src_id, int &dst_id) const override;
  bool valid() const override;
  hipError_t prepare() const override;
};

struct MfmaStep : Step {
  MfmaArgs a{};
  int prec = 0;
  const void *fn_sw[4] = {};
  dim3 grid;
  int src = BUF_IN, dst = BUF_OUT;
  size_t amat_off = 0, tw16_off = 0, tw4_lo_off = 0, tw4_hi_off = 0;
  bool tw4 = false;
  bool first = false, last = false;
  float inv_scale = 1.0f;
  std::string name;
  int inverse_sw() const { return (first ? 1 : 0) | (last ? 2 : 0); }
  void bind(const float2 *tables) override;
  hipError_t launch(const ExecCtx &ctx) const override;
  std::string describe() const override;
  void extent(int64_t &max_in, int64_t &max_out, int &src_id, int &dst_id) const override;
  bool valid() const override;
};

// Real-input line kernel: N = 2L reals <-> L + 1 bins per line, one launch.
// Forward plans run the R2C kernel, inverse plans the C2R kernel (each step
// list is used for one direction only).
struct RealStep : Step {
  RealKernel k;
  int L = 0;
  bool inv = false;
  dim3 grid;
  int src = BUF_IN, dst = BUF_OUT;
  LineArgs a{};
  size_t tw_off = 0, tw2_off = 0, wn_off = 0;
  std::string name;
  void bind(const float2 *tables) override;
  hipError_t launch(const ExecCtx &ctx) const override;
  std::string describe() const override;
  void extent(int64_t &max_in, int64_t &max_out, int &src_id, int &dst_id) const override;
  bool valid() const override;
};

// Pairing pass of a real transform whose complex core is a four-step pair
// of launches (forward: after them, from the workspace into the output;
// inverse: before them, from the input into the output).
struct RealPairStep : Step {
  bool inv = false;
  RealPairArgs a{};
  size_t lo_off = 0, hi_off = 0;
  int src = BUF_OUT, dst = BUF_OUT;
  std::string name;
  void bind(const float2 *tables) override;
  hipError_t launch(const ExecCtx &ctx) const override;
  std::string describe() const override;
  void extent(int64_t &max_in, int64_t &max_out, int &src_id, int &dst_id) const override;
  bool valid() const override;
};

// Fused convolution launch: a single-pass line (forward, product with the
// filter spectrum, inverse) or the row launch of the four-step form.
struct ConvStep : Step {
  ConvKernel k;
  int L = 0;
  dim3 grid;
  int src = BUF_IN, dst = BUF_OUT;
  LineArgs a{};
  size_t tw_off = 0, tw2_off = 0, tw4_lo_off = 0, tw4_hi_off = 0;
  std::string name;
  void bind(const float2 *tables) override;
  hipError_t launch(const ExecCtx &ctx) const override;
  std::string describe() const override;
  void extent(int64_t &max_in, int64_t &max_out, int &src_id, int &dst_id) const override;
  bool valid() const override;
};

}  // namespace dpfft

struct dpfft_plan_s {
  int32_t rank = 1;
  int64_t n = 0;              // rank 1 length
  int64_t ny = 0, nx = 0;     // rank 2
  int64_t batch = 0;
  int64_t dist = 0;
  int32_t precision = FFT_FP32;
  uint32_t flags = 0;
  std::vector<int64_t> rsizes, roffsets;  // ragged
  std::vector<std::unique_ptr<dpfft::Step>> steps;   // forward (and inverse, if isteps is empty)
  std::vector<std::unique_ptr<dpfft::Step>> isteps;  // inverse launches where they differ
  bool real = false;          // FFT_F_REAL: real samples <-> N/2 + 1 bins
  int64_t real_elems = 0;     // real plans: float pairs of the real-side buffer
  int64_t cplx_elems = 0;     // real plans: complex elements of the spectrum buffer
  // FFT_F_CONV: the launches of fft_conv_exec, each with its direction
  std::vector<std::unique_ptr<dpfft::Step>> csteps;
  std::vector<bool> cinv;
  dpfft::TableSet tables;
  size_t ws_bytes = 0;
  int64_t io_elems = 0;       // complex elements of `in` / `out` the plan touches
  std::string variant;
  std::string text;  // fft_plan_describe output
  ~dpfft_plan_s();
};
