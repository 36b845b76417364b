// tnc_sample_noalloc: tnc_sample for callers that cannot allocate device memory.
//
// Every device buffer the draws need (closed bits and open qubit ids of the targets,
// running sums of one group, the draws before they are copied out) is carved from
// `scratch`, a file-scope device array of kScratchBytes.  Each GPU the library runs on
// holds its own copy until the process ends.  In host code the name `scratch` only stands
// for the device symbol: its device address is taken once per device with
// hipGetSymbolAddress (with that device current) and only that address is ever handed to
// copies and kernels.  Every call on one GPU reuses the same array (the previous call's
// contents stay there and are overwritten), so calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "tnc.h"
#include "tnc_internal.h"

namespace {

constexpr uint64_t kScratchBytes = uint64_t(16) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_mu;
uint8_t* g_scratch[kMaxDevices] = {};

// Device address of this device's scratch array (the device must be current).
tnc_status scratch_of(int dev, uint8_t** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return tnc::report_error(TNC_E_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return tnc::report_error(TNC_E_HIP, (std::string("hipGetSymbolAddress(scratch): ") +
                                           hipGetErrorString(e)).c_str());
    g_scratch[dev] = static_cast<uint8_t*>(ptr);
  }
  *out = g_scratch[dev];
  return TNC_OK;
}

}  // namespace

extern "C" tnc_status tnc_sample_noalloc(tnc_plan plan, const double* d_amps, uint64_t seed,
                                         int64_t n_samples, uint64_t* h_bitstrings,
                                         void* hip_stream) {
  int dev = 0;
  tnc_status st = tnc::plan_device(plan, &dev);
  if (st != TNC_OK) return st;
  int prev = -1;
  hipError_t e = hipGetDevice(&prev);
  if (e == hipSuccess && prev != dev) e = hipSetDevice(dev);
  if (e != hipSuccess)
    return tnc::report_error(TNC_E_HIP, (std::string("hipSetDevice: ") + hipGetErrorString(e)).c_str());
  uint8_t* ptr = nullptr;
  st = scratch_of(dev, &ptr);
  if (st == TNC_OK)
    st = tnc::sample_in_scratch(plan, ptr, kScratchBytes, d_amps, seed, n_samples, h_bitstrings,
                                hip_stream);
  if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
  return st;
}
