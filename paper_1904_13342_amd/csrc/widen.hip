// Exact widening of half-precision storage to FP32 (FP16 and BF16 are both
// subsets of FP32), used where a kernel reads a half-precision operand as an
// FP32 copy.
#include "device_util.h"

namespace ph {
namespace {

template <typename T>
__global__ void widen_kernel(const T *__restrict__ in, float *__restrict__ out, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = load_f32(in + i);
}

}  // namespace

hipError_t launch_cast_to_f32(int dtype, const void *in, float *out, size_t n, hipStream_t s)
{
    const size_t blocks = (n + 255) / 256;
    const dim3 grid((unsigned)(blocks < 4096 ? blocks : 4096));
    switch (dtype) {
    case 1: hipLaunchKernelGGL(widen_kernel<f16_t>, grid, dim3(256), 0, s, (const f16_t *)in, out, n); break;
    case 2: hipLaunchKernelGGL(widen_kernel<bf16_t>, grid, dim3(256), 0, s, (const bf16_t *)in, out, n); break;
    default: hipLaunchKernelGGL(widen_kernel<float>, grid, dim3(256), 0, s, (const float *)in, out, n); break;
    }
    return hipGetLastError();
}

}  // namespace ph
