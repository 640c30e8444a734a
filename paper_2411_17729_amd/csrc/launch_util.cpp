// Launch-time helpers shared by the kernel launchers.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <utility>

#include "ssm_internal.h"

namespace ssmc {

namespace {
std::mutex g_lds_mutex;
// (kernel, device) -> dynamic LDS limit already set
std::map<std::pair<const void*, int>, size_t> g_lds_limit;
}  // namespace

hipError_t ensure_dynamic_lds(const void* kernel, size_t bytes) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_lds_mutex);
  size_t& have = g_lds_limit[std::make_pair(kernel, dev)];
  if (have >= bytes) return hipSuccess;
  e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) have = bytes;
  return e;
}

}  // namespace ssmc
