// Host helper: raise a kernel's dynamic-LDS limit on the current device.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <utility>

namespace gkb {

// HIP keeps hipFuncAttributeMaxDynamicSharedMemorySize per device, so the
// attribute is set once for every (device, kernel) pair a launch meets; the
// result of that first call is returned to every later launch of the pair.
inline hipError_t allow_dynamic_lds(const void* kernel, int bytes) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, hipError_t> done;
  int dev = 0;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_pair(dev, kernel);
  const auto it = done.find(key);
  if (it != done.end()) return it->second;
  const hipError_t r = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  done.emplace(key, r);
  return r;
}

}  // namespace gkb
