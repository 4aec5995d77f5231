// Device scratch of the entry points that allocate nothing (et_synthesize_noalloc): a
// file-scope device array that every GPU holds from the library's first context on it until the
// process ends.  Host code never uses the array's name as an address: each device's address
// comes from hipGetSymbolAddress, taken once per device with that device current (at context
// creation), and kernels receive that pointer.
#include "internal.hpp"

#include <mutex>

namespace et {

namespace {

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};

}  // namespace

void noalloc_init(int device) {
  ET_CHECK(device >= 0 && device < MAX_DEVICES, ET_E_DEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_ptr[device]) return;
  void* p = nullptr;
  ET_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  ET_CHECK(p != nullptr, ET_E_DEVICE, "no address for the device scratch");
  g_ptr[device] = p;
}

void* noalloc_scratch(int device) {
  ET_CHECK(device >= 0 && device < MAX_DEVICES, ET_E_DEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_mu);
  void* p = g_ptr[device];
  ET_CHECK(p != nullptr, ET_E_INTERNAL, "device scratch not set up (no context was created on this device)");
  return p;
}

}  // namespace et
