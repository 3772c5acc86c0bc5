// Workspace of the no-allocation entry point (pxd_evaluate_flips_device_noalloc).
//
// A file-scope device array: every GPU the library runs on holds one copy of
// kScratchBytes from the moment the code object is loaded on it until the
// process ends.  Its name is a host-side stand-in in host code, so the device
// address of each GPU's copy is looked up once per device with
// hipGetSymbolAddress (that device current) and only that address is handed
// to kernels.  Every call on one GPU shares its copy; calls that overlap on
// one GPU race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.hpp"

namespace pxd {

static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_region(int device, char** ptr, size_t* bytes) {
  if (device < 0 || device >= kMaxDevices || !ptr || !bytes) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if ((e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    const hipError_t e2 = hipSetDevice(cur);
    if (e != hipSuccess) return e;
    if (e2 != hipSuccess) return e2;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[device] = static_cast<char*>(p);
  }
  *ptr = g_ptr[device];
  *bytes = kScratchBytes;
  return hipSuccess;
}

}  // namespace pxd
