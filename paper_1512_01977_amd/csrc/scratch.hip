// The library's static device scratch: a file-scope array that every GPU the library runs on
// holds for the lifetime of the process, so that entry points meant for callers that cannot
// allocate (code under stream capture, serving loops) need no hipMalloc.  Host code never uses
// the array's name as an address: each device's copy is looked up with hipGetSymbolAddress
// while that device is current, and that address is what kernels receive.
#include "scratch.h"

#include <mutex>

namespace lbm {

namespace {
constexpr size_t kScratchBytes = size_t(1) << 20;  // 1 MiB
constexpr int kMaxDevices = 64;
std::mutex g_lock;
void* g_ptr[kMaxDevices] = {};
}  // namespace

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

size_t scratch_bytes() { return kScratchBytes; }

hipError_t scratch_attach() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_lock);
  if (g_ptr[dev]) return hipSuccess;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_ptr[dev] = p;
  return hipSuccess;
}

void* scratch_ptr(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_lock);
  return g_ptr[dev];
}

}  // namespace lbm
