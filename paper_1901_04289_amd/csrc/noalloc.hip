// Allocation-free matrix product: the workspace of arbgpu_mat_mul cut from
// one static device array instead of buffers the context allocates, for
// callers that cannot allocate device memory.
//
// The array, `scratch`, is a file-scope device variable, so every device
// the library runs on holds its own copy from module load until the process
// ends.  Its name is a host-side stand-in in host code: the device address
// comes from hipGetSymbolAddress, taken once per device with that device
// current (at context creation, noalloc_setup) and kept per device.  All
// calls on one device share that device's copy and leave their contents in
// it: calls that overlap on one device race.
#include <hip/hip_runtime.h>
#include <string.h>

#include <mutex>

#include "internal.hpp"

namespace arbgpu_impl {

namespace {

constexpr size_t kScratchBytes = (size_t)256 << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
char *g_ptr[kMaxDevices] = {nullptr};

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

int noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return ARBGPU_EDEVICE;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return ARBGPU_OK;
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ARBGPU_EDEVICE;
  g_ptr[device] = static_cast<char *>(p);
  return ARBGPU_OK;
}

char *noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_ptr[device];
}

}  // namespace arbgpu_impl
