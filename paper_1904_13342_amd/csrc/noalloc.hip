// The library's static device scratch: one fixed-size array per GPU, held
// until the process ends, for the FDK entry point that allocates nothing
// (ph_fdk_cone3d_static).  Host code never passes the array's name to a
// kernel or a copy (on the host it is only a stand-in for the device
// symbol): the device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and kept.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/pyrohip.h"
#include "common.h"

namespace ph {
namespace {

static __device__ __align__(256) unsigned char scratch[PH_FDK_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices];   // device address of `scratch` on each device, once looked up

}  // namespace

hipError_t static_scratch(void **ptr, size_t *bytes)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    if (dev < 0 || dev >= kMaxDevices)
        return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return e;
        if (!p)
            return hipErrorInvalidSymbol;
        g_scratch[dev] = p;
    }
    *ptr = g_scratch[dev];
    *bytes = (size_t)PH_FDK_STATIC_SCRATCH_BYTES;
    return hipSuccess;
}

}  // namespace ph
