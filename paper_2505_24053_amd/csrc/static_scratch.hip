// Fixed device memory of the allocation-free forward (geer_render_static).
//
// Every buffer of that forward is carved from one file-scope device array of
// GEER_STATIC_SCRATCH_BYTES.  Each device the library runs on holds its own
// copy of the array from the first look-up until the process ends.  In host
// code the array's name is only a host-side stand-in: host code uses the
// device address that static_scratch_init() looked up, once per device, with
// that device current.
#include <hip/hip_runtime.h>

#include <mutex>

#include "geer.h"
#include "tables.h"

static __device__ __align__(256) unsigned char scratch[GEER_STATIC_SCRATCH_BYTES];

namespace geer {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_lookup;
void* g_addr[kMaxDevices] = {};
std::mutex g_device_lock[kMaxDevices];
}  // namespace

hipError_t static_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_lookup);
  if (g_addr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_addr[device] = p;
  return hipSuccess;
}

void* static_scratch_addr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_lookup);
  return g_addr[device];
}

std::mutex& static_scratch_lock(int device) { return g_device_lock[device]; }

}  // namespace geer
