// Execution without a caller-provided workspace, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).
//
// The four-step intermediates (and every other workspace a plan needs) live in
// `scratch`, a file-scope device array of kScratchBytes that each GPU the
// library runs on holds until the process ends.  Host code never passes the
// array's name to a kernel: in host code it is a stand-in, not a device
// address.  The first call on a device looks the array's address up with
// hipGetSymbolAddress (with that device current) and keeps it per device;
// kernels receive that address as their workspace argument, exactly as they
// receive a caller's workspace through fft_exec.
//
// Every call on one GPU shares that GPU's array and leaves its contents behind;
// no kernel reads workspace it has not written in the same call, so nothing
// needs clearing.  Calls whose executions overlap on one GPU (two streams, or
// two threads) race on the array.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.h"
#include "plan.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB: 8 Mi complex64 points
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// the array's device address on the current device (nullptr + status on failure)
fft_status_t scratch_ptr(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess)
    return dpfft::fail(FFT_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return dpfft::fail(FFT_E_UNSUPPORTED, "device index above the scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return dpfft::fail(FFT_E_DEVICE,
                         std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return FFT_OK;
}

}  // namespace

extern "C" fft_status_t fft_exec_noalloc(fft_plan_t plan, const void *in, void *out, int direction,
                                         void *hip_stream) {
  if (!plan) return dpfft::fail(FFT_E_INVALID, "plan is NULL");
  if (plan->ws_bytes > kScratchBytes)
    return dpfft::fail(FFT_E_UNSUPPORTED,
                       "plan needs " + std::to_string(plan->ws_bytes) +
                           " bytes of workspace, above the library's scratch of " +
                           std::to_string(kScratchBytes) + " bytes; use fft_exec");
  void *ws = nullptr;
  if (plan->ws_bytes) {
    const fft_status_t st = scratch_ptr(&ws);
    if (st != FFT_OK) return st;
  }
  return dpfft::exec_plan(plan, in, out, direction, ws, hip_stream, /*graphs=*/false);
}
