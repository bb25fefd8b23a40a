// Properties of the current HIP device that launch configurations depend on,
// looked up once per device.
#pragma once
#include <atomic>

#include <hip/hip_runtime.h>

namespace snx {

// Compute units of the current device.
inline hipError_t device_cus(int *cus)
{
    constexpr int kMaxDev = 64;
    static std::atomic<int> cached[kMaxDev];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
    int n = cached[dev].load(std::memory_order_relaxed);
    if (n <= 0) {
        if ((e = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev)) !=
            hipSuccess)
            return e;
        cached[dev].store(n, std::memory_order_relaxed);
    }
    *cus = n;
    return hipSuccess;
}

}  // namespace snx
