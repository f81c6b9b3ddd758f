// Allocation-free state check (rtcc_check_state_noalloc): the non-finite count of rtcc_check_state and
// |T2|, for callers that cannot allocate device memory (code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc). Its only scratch, the per-block partial sums of the
// reduction, lives in the file-scope device array `scratch` below; every GPU the library runs on holds
// one copy of it (8 KB) until the process ends.
#include <mutex>

#include "../../include/rtcc.h"
#include "elementwise.h"

using namespace rtcc;

namespace {

constexpr int64_t kMaxEntries = (int64_t)1 << 40;

// two partial doubles per reduction block of state_guard
__device__ __align__(256) double scratch[2 * kGuardBlocks];

constexpr int kMaxDevices = 64;
double* g_scratch_dev[kMaxDevices] = {nullptr};  // device address of `scratch`, per device
std::mutex g_scratch_mu;

// Device address of this device's copy of `scratch` (looked up once per device, with it current).
double* scratch_ptr(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    RTCC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    RTCC_CHECK(p != nullptr, kEHip, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  return g_scratch_dev[dev];
}

}  // namespace

extern "C" int rtcc_check_state_noalloc(int o, int v, const void* y, double* out_dev, void* hip_stream) {
  if (o < 1 || v < 1 || !y || !out_dev) {
    set_noctx_error("rtcc_check_state_noalloc: invalid arguments");
    return RTCC_EINVAL;
  }
  const int64_t n1 = (int64_t)o * v;
  if (n1 > ((int64_t)1 << 20) || 2 * (n1 + n1 * n1) > kMaxEntries) {
    set_noctx_error("rtcc_check_state_noalloc: state larger than 2^40 entries");
    return RTCC_EINVAL;
  }
  try {
    int dev = 0;
    RTCC_HIP(hipGetDevice(&dev));
    RTCC_CHECK(dev >= 0 && dev < kMaxDevices, kEInval, "rtcc_check_state_noalloc: device index out of range");
    double* part = scratch_ptr(dev);
    const int64_t n2 = n1 * n1, nst = 2 * (n1 + n2);
    // state_guard uses at most kGuardBlocks blocks, each writing its two partials before the final sum
    // reads them, so nothing in `scratch` has to start at zero
    state_guard((hipStream_t)hip_stream, nst, n1, n1 + n2, y, part, out_dev);
    return RTCC_OK;
  } catch (const Error& e) {
    set_noctx_error(e.what());
    return e.code;
  } catch (const std::exception& e) {
    set_noctx_error(e.what());
    return RTCC_EHIP;
  }
}
