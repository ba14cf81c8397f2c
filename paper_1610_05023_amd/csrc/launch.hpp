// Launch set-up shared by the kernel launchers: per device and kernel, the
// dynamic LDS limit and the number of resident workgroups, computed once
// and kept in a process-wide table behind a mutex (contexts on several
// devices or host threads may launch at the same time).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>

namespace dgh {

// Makes `lds` bytes of dynamic LDS available to kernel `fn` on the current
// device (raising the limit when a launch needs more than any before it) and,
// if `resident` is not null, stores the number of workgroups of `threads`
// threads with that much dynamic LDS that fit on the device at once (at
// least the number of compute units).
hipError_t kernel_setup(const void* fn, int threads, size_t lds, int* resident);

// Number of compute units of the current device.
hipError_t device_cus(int* cus);

}  // namespace dgh
