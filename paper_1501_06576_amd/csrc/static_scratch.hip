// The library's one statically allocated device buffer: the scratch of
// xs21_power_spectrum_static, for callers that cannot allocate device memory.
//
// `scratch` is a file-scope device array; host code never passes its name to
// a kernel or a copy (in host code the name is only a host-side stand-in).
// static_scratch_init(), called by xs21_create with the context's device
// current, looks up the array's device address once per device; every use
// goes through that address.  Each device keeps its own copy of the array
// until the process ends, and every call on a device shares it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.hpp"

namespace xs21 {

namespace {

constexpr size_t kStaticScratchBytes = size_t(20) << 20;   // 20 MiB
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

size_t static_scratch_bytes() { return kStaticScratchBytes; }

hipError_t static_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_ptr[device] = p;
  return hipSuccess;
}

void* static_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_mu);
  return g_ptr[device];
}

}  // namespace xs21
