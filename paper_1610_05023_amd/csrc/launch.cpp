// Per-device launch set-up of the kernels (see launch.hpp).
#include "launch.hpp"

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

namespace dgh {

namespace {

std::mutex g_mu;
std::map<std::pair<int, const void*>, size_t> g_lds;          // limit set so far
std::map<std::tuple<int, const void*, int, size_t>, int> g_res;  // resident workgroups
std::map<int, int> g_cus;

hipError_t cus_locked(int dev, int* cus) {
  auto it = g_cus.find(dev);
  if (it != g_cus.end()) {
    *cus = it->second;
    return hipSuccess;
  }
  hipDeviceProp_t prop;
  const hipError_t e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return e;
  *cus = g_cus[dev] = prop.multiProcessorCount;
  return hipSuccess;
}

}  // namespace

hipError_t kernel_setup(const void* fn, int threads, size_t lds, int* resident) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_mu);
  size_t& have = g_lds[{dev, fn}];
  if (lds > have) {
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    have = lds;
  }
  if (!resident) return hipSuccess;
  const auto key = std::make_tuple(dev, fn, threads, lds);
  auto it = g_res.find(key);
  if (it != g_res.end()) {
    *resident = it->second;
    return hipSuccess;
  }
  int cus = 0, per_cu = 0;
  e = cus_locked(dev, &cus);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds);
  if (e != hipSuccess) return e;
  *resident = g_res[key] = std::max(1, per_cu) * cus;
  return hipSuccess;
}

hipError_t device_cus(int* cus) {
  int dev = 0;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_mu);
  return cus_locked(dev, cus);
}

}  // namespace dgh
