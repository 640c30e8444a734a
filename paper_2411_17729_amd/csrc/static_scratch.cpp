// The library's one block of device memory of its own: the state buffers of
// the allocation-free forward apply (ssm_cascade_apply_noalloc). It is a
// file-scope device array, so the code object reserves it on every device the
// library's kernels are loaded on, for the life of the process; no HIP
// allocation call is made for it. Host code never passes the array's name to
// a kernel (on the host that name is only a stand-in symbol): the device
// address is looked up once per device with hipGetSymbolAddress, with that
// device current, and kept.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "ssm_internal.h"

namespace ssmc {

namespace {

constexpr size_t kStaticScratchBytes = size_t(64) << 20;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mutex;
std::map<int, void*> g_scratch_ptr;  // device ordinal -> address of its copy

}  // namespace

size_t static_scratch_bytes() { return kStaticScratchBytes; }

hipError_t static_scratch(void** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    it = g_scratch_ptr.emplace(dev, p).first;
  }
  *out = it->second;
  return hipSuccess;
}

}  // namespace ssmc
