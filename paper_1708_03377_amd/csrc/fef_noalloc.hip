// Pair energies without a caller workspace and without any allocation: the
// scratch the pair kernels need (partial-sum slots, queue counters, gap
// pool, stage sums of the total) lives in a fixed device array of this
// library, one copy per GPU, kept until the process ends.
#include <atomic>
#include <mutex>

#include "fef_internal.h"

namespace fef {

constexpr size_t kScratchBytes = FEF_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

// The device array.  In host code `scratch` names a host-side stand-in, not
// device memory: host code only ever uses the address looked up per device.
static __device__ __align__(256) char scratch[kScratchBytes];

static std::atomic<void*> g_scratch[kMaxDevices];
static std::mutex g_setup;

// Looks up this device's copy of the scratch array (once per device, with
// `device` current).  Returns hipSuccess when the address is known.
hipError_t noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (g_scratch[device].load(std::memory_order_acquire)) return hipSuccess;
  std::lock_guard<std::mutex> lock(g_setup);
  if (g_scratch[device].load(std::memory_order_relaxed)) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return e != hipSuccess ? e : hipErrorInvalidSymbol;
  g_scratch[device].store(ptr, std::memory_order_release);
  return hipSuccess;
}

}  // namespace fef

using namespace fef;

extern "C" {

fef_status fef_pair_energies_noalloc(fef_plan p, const void* ops, const double* eps,
                                     fef_prec prec, double* E2_pair, double* E2_total,
                                     int32_t* flags, void* stream) {
  if (!p) return FEF_E_ARG;
  if (prec < 0 || prec >= FEF_NPREC) return FEF_E_PREC;
  if (!E2_total || !flags) return FEF_E_ARG;
  if (p->npair > 0 && (!ops || !eps || !E2_pair)) return FEF_E_ARG;
  if (pair_ws_bytes(*p, prec) > (int64_t)kScratchBytes) return FEF_E_WORKSPACE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return FEF_E_HIP;
  if (dev != p->device) return FEF_E_ARG;
  // normally done when the plan was created; the first call on a device
  // otherwise (an address lookup, no allocation)
  if (noalloc_setup(dev) != hipSuccess) return FEF_E_HIP;
  void* ws = g_scratch[dev].load(std::memory_order_acquire);
  return launch_pair_energies(*p, ops, eps, prec, nullptr, E2_pair, E2_total, flags, ws,
                              static_cast<hipStream_t>(stream)) == hipSuccess
             ? FEF_OK
             : FEF_E_HIP;
}

}  // extern "C"
