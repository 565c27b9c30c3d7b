// hts_denoise for callers that cannot allocate device memory: the
// workspace is a fixed scratch array in the library's device code object
// instead of a caller buffer.  Same stages and kernels as hts_denoise.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hts_internal.h"

namespace {

constexpr size_t kScratchBytes = HTS_NOALLOC_SCRATCH_BYTES;   // per device
constexpr int kMaxDevices = 64;

}  // namespace

// One copy per device, resident from the load of the code object until the
// process ends.  In host code this name is only a stand-in for the symbol:
// its device address comes from hipGetSymbolAddress (scratch_ptr below).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {nullptr};

// Device address of the current device's scratch array, looked up once per
// device with that device current.
hts_status scratch_ptr(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return HTS_ERR_HIP;
  if (dev < 0 || dev >= kMaxDevices) return HTS_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return HTS_ERR_HIP;
    }
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return HTS_OK;
}

}  // namespace

extern "C" {

hts_status hts_denoise_noalloc(const hts_params* p, const float* noisy, int32_t C, int32_t H,
                               int32_t W, float sigma, float* out, void* stream) {
  size_t need = 0;
  const hts_status st = hts_workspace_size(p, C, H, W, &need);
  if (st != HTS_OK) return st;
  if (need > kScratchBytes) return HTS_ERR_WORKSPACE;   // beyond the fixed scratch
  void* ws = nullptr;
  const hts_status sp = scratch_ptr(&ws);
  if (sp != HTS_OK) return sp;
  // every region hts_denoise reads is written or cleared by its own stages
  // first (counters, histogram, accumulators), so the previous call's
  // contents do not matter
  return hts_denoise(p, noisy, C, H, W, sigma, out, nullptr, nullptr, nullptr, nullptr, nullptr,
                     ws, kScratchBytes, stream);
}

}  // extern "C"
