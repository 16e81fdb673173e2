// The library's fixed scratch array: device memory that every GPU the library
// runs on holds from the loading of its code object to the end of the
// process, for entry points that may not allocate (the caller-free product).
// Host code reaches it only through the address hipGetSymbolAddress returns
// for the current device, taken once per device at context creation; the
// array's name itself is not a device address in host code.
#include <mutex>

#include "common.hpp"

namespace ffk {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
}  // namespace

void scratch_init(int device) {
  require(device >= 0 && device < kMaxDevices, "scratch: device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return;
  void* p = nullptr;
  HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  require(p != nullptr, "scratch: no device address for the scratch array");
  g_ptr[device] = p;
}

void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_ptr[device];
}

}  // namespace ffk
