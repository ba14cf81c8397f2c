// Device helpers shared by the HIP kernels (included by .hip files only).
#pragma once
#include <hip/hip_runtime.h>

namespace dgh {

// Stage time of a launch: given by value, or (replayed stepping) from the
// device clock as (t0 + k dt) + cs dt, rounded exactly as the host computes
// the eager value (no fused multiply-add), so both modes agree bitwise.
template <class S>
__device__ __forceinline__ double stage_time(const S& sh) {
  if (!sh.clk) return sh.tau;
  const double t = __dadd_rn(sh.clk[0], __dmul_rn(sh.clk[1], sh.dt));
  return __dadd_rn(t, __dmul_rn(sh.cs, sh.dt));
}

// FP64 4x4x4 MFMA, four 4x4x4 blocks per instruction.
__device__ __forceinline__ double mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// Copies COUNT elements of a small constant table into LDS with NT threads,
// every global load of a thread issued before its first LDS store (one
// memory round trip instead of one per element a thread copies).
template <int NT, int COUNT, class T>
__device__ __forceinline__ void fill_lds(T* __restrict__ dst, const T* __restrict__ src,
                                         int tid) {
  constexpr int IT = (COUNT + NT - 1) / NT;
  T v[IT];
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int x = tid + k * NT;
    v[k] = x < COUNT ? src[x] : T(0);
  }
#pragma unroll
  for (int k = 0; k < IT; ++k) {
    const int x = tid + k * NT;
    if (x < COUNT) dst[x] = v[k];
  }
}

// Work items [0, n) of a persistent launch: the blocks of XCD x (hardware
// block ids are dealt round-robin over the 8 XCDs) walk the contiguous
// range [n x / 8, n (x + 1) / 8), so neighbouring items share an L2.
struct XcdRange {
  long long lo, hi, step;
  // plain != 0: round-robin over all blocks instead (item b, b + grid, ...)
  __device__ XcdRange(long long n, int plain = 0) {
    if (plain) {
      lo = blockIdx.x;
      hi = n;
      step = gridDim.x;
      return;
    }
    const int x = blockIdx.x & 7;
    const int per = (gridDim.x + 7 - x) >> 3;   // blocks on XCD x
    lo = n * x / 8 + (blockIdx.x >> 3);
    hi = n * (x + 1) / 8;
    step = per;
  }
};

}  // namespace dgh
