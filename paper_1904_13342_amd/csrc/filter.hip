// Projection-domain weighting and row-wise filtering, q = F^H K F (W p)
// (Eq. 4 / Eq. 5; the filter is a diagonal multiply in the Fourier domain,
// Sec. II.C.4; the weights are Sec. II.C.5's cosine and redundancy weights).
//
// A workgroup transforms two detector rows at once: row a goes into the real
// part and row b into the imaginary part of one complex M-point sequence.
// The response is real and even (it is symmetrised first), so the inverse
// transform of K . DFT(a + i b) is (K * a) + i (K * b): both filtered rows come
// out of one forward / inverse pair.  The transforms are in-place Stockham
// radix-8 passes (radix 4 or 2 for the last one) in LDS with the butterflies
// in registers, natural order in and out.  Workgroups loop over row pairs
// (grid sized to the machine) with the twiddle half-table held in LDS.
#include "fft.h"

namespace ph {
namespace {

using namespace lds_fft;

template <typename T>
__device__ __forceinline__ float weighted(const FilterArgs &a, const T *in, long row, int j)
{
    const int i = (int)(row % a.nv);
    const int k = (int)((row / a.nv) % a.n_proj);
    float w = 1.0f;
    if (a.W_red)
        w *= a.W_red[(size_t)k * a.nu + j];
    if (a.W)
        w *= a.W[(size_t)i * a.nu + j];
    w *= cosine_weight(a, i, j);
    return w * load_f32(in + (size_t)row * a.nu + j);
}

template <typename T, int M>
__global__ void __launch_bounds__(WF_THREADS) weight_filter_kernel(FilterArgs a, const T *__restrict__ in,
                                                                   float *__restrict__ out, long rows)
{
    extern __shared__ float2 lds[];
    constexpr int half = M >> 1;
    float2 *buf = lds, *tw = lds + M;
    const int tid = threadIdx.x;
    const long pairs = (rows + 1) / 2;
    const float inv = 1.0f / (float)M;
    for (int n = tid; n < half; n += WF_THREADS)
        tw[n] = a.tw[n];
    for (long pr = blockIdx.x; pr < pairs; pr += gridDim.x) {
        const long ra = 2 * pr, rb = ra + 1;
        const bool has_b = rb < rows;
        for (int n = tid; n < M; n += WF_THREADS) {
            float2 z = make_float2(0.0f, 0.0f);
            if (n < a.nu) {
                z.x = weighted(a, in, ra, n);
                if (has_b)
                    z.y = weighted(a, in, rb, n);
            }
            buf[n] = z;
        }
        __syncthreads();
        transform_c<-1, M>(buf, tw);
        // multiply by the symmetrised real response
#pragma unroll
        for (int t = 0; t < (M + WF_THREADS - 1) / WF_THREADS; ++t) {
            const int n = tid + t * WF_THREADS;
            if (n < M) {
                const float kf = 0.5f * (a.K[n] + a.K[(M - n) & (M - 1)]);
                buf[n].x *= kf;
                buf[n].y *= kf;
            }
        }
        __syncthreads();
        transform_c<1, M>(buf, tw);
        for (int n = tid; n < a.nu; n += WF_THREADS) {
            const float2 z = buf[n];
            out[(size_t)ra * a.nu + n] = z.x * inv;
            if (has_b)
                out[(size_t)rb * a.nu + n] = z.y * inv;
        }
        __syncthreads();   // buf is overwritten by the next pair's load
    }
}

template <typename T, int M>
hipError_t wf_m(const FilterArgs &a, const void *in, float *out, hipStream_t s)
{
    const long rows = (long)a.batch * a.n_proj * a.nv;
    const long pairs = (rows + 1) / 2;
    const size_t lds = ((size_t)M + M / 2) * sizeof(float2);
    const long max_groups = 256L * 8;   // enough resident workgroups for 256 CUs
    const unsigned grid = (unsigned)(pairs < max_groups ? pairs : max_groups);
    hipLaunchKernelGGL((weight_filter_kernel<T, M>), dim3(grid), dim3(WF_THREADS), lds, s, a, (const T *)in, out,
                       rows);
    return hipGetLastError();
}

template <typename T>
hipError_t wf(const FilterArgs &a, const void *in, float *out, hipStream_t s)
{
    switch (a.log2M) {
    case 4: return wf_m<T, 16>(a, in, out, s);
    case 5: return wf_m<T, 32>(a, in, out, s);
    case 6: return wf_m<T, 64>(a, in, out, s);
    case 7: return wf_m<T, 128>(a, in, out, s);
    case 8: return wf_m<T, 256>(a, in, out, s);
    case 9: return wf_m<T, 512>(a, in, out, s);
    case 10: return wf_m<T, 1024>(a, in, out, s);
    case 11: return wf_m<T, 2048>(a, in, out, s);
    case 12: return wf_m<T, 4096>(a, in, out, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_weight_filter(int dtype, const FilterArgs &a, const void *in, float *out, hipStream_t stream)
{
    switch (dtype) {
    case 0: return wf<float>(a, in, out, stream);
    case 1: return wf<f16_t>(a, in, out, stream);
    default: return wf<bf16_t>(a, in, out, stream);
    }
}

}  // namespace ph
