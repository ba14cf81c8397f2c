// Finiteness scan of the state arrays (the failure check that accompanies
// the energy of Section 4.1): one flag per block and array, no atomics.
#include <hip/hip_runtime.h>

#include "levels.hpp"

namespace dgh {

namespace {

__global__ void __launch_bounds__(256) k_nonfinite(ScanList s, int* __restrict__ flags) {
  const int a = blockIdx.y;
  const size_t n = s.n[a];
  int bad = 0;
  if (s.f32[a]) {
    const float* __restrict__ p = static_cast<const float*>(s.ptr[a]);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
      bad |= !isfinite(p[i]);
  } else {
    const double* __restrict__ p = static_cast<const double*>(s.ptr[a]);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
      bad |= !isfinite(p[i]);
  }
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) flags[a * gridDim.x + blockIdx.x] = bad;
}

// Device clock of replayed stepping (one lane; plain vector stores).
__global__ void k_clock_set(double* clk, double t0) {
  if (threadIdx.x == 0) {
    clk[0] = t0;
    clk[1] = 0.0;
  }
}
__global__ void k_clock_tick(double* clk) {
  if (threadIdx.x == 0) clk[1] = clk[1] + 1.0;
}

}  // namespace

hipError_t launch_clock_set(double* clk, double t0, hipStream_t st) {
  hipLaunchKernelGGL(k_clock_set, dim3(1), dim3(64), 0, st, clk, t0);
  return hipGetLastError();
}

hipError_t launch_clock_tick(double* clk, hipStream_t st) {
  hipLaunchKernelGGL(k_clock_tick, dim3(1), dim3(64), 0, st, clk);
  return hipGetLastError();
}

hipError_t launch_nonfinite(const ScanList& s, int* flags, hipStream_t st) {
  if (s.count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_nonfinite, dim3(kScanBlocks, s.count), dim3(256), 0, st, s, flags);
  return hipGetLastError();
}

}  // namespace dgh
