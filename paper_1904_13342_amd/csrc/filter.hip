// Projection-domain weighting and row-wise filtering, q = F^H K F (W p)
// (Eq. 4 / Eq. 5; the filter is a diagonal multiply in the Fourier domain,
// Sec. II.C.4; the weights are Sec. II.C.5's cosine and redundancy weights).
//
// One workgroup transforms two detector rows at once: row a goes into the
// real part and row b into the imaginary part of one complex M-point
// sequence.  Because the response is real and even (it is symmetrised
// first), the inverse transform of K . DFT(a + i b) is (K * a) + i (K * b), so
// both filtered rows come out of one forward / inverse pair.  The transform
// runs in LDS: decimation in frequency forward (natural order in, bit-reversed
// out), the multiply by K in bit-reversed order, decimation in time inverse
// (bit-reversed in, natural out), so no permutation pass is needed.
#include "common.h"

namespace ph {
namespace {

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

__device__ __forceinline__ float2 cmul_conj(float2 a, float2 b)  // a * conj(b)
{
    return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -a.x * b.y));
}

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
    if (a.cos_sdd > 0.0f) {
        const float u = ((float)j - a.cu) * a.du, v = ((float)i - a.cv) * a.dv;
        w *= a.cos_sdd / sqrtf(fmaf(a.cos_sdd, a.cos_sdd, fmaf(u, u, v * v)));
    }
    return w * load_f32(in + (size_t)row * a.nu + j);
}

template <typename T>
__global__ void __launch_bounds__(256) weight_filter_kernel(FilterArgs a, const T *__restrict__ in,
                                                            float *__restrict__ out, long rows)
{
    extern __shared__ float2 buf[];
    const int tid = threadIdx.x;
    const int M = a.M, half = M >> 1;
    const long ra = 2 * (long)blockIdx.x, rb = ra + 1;
    const bool has_b = rb < rows;

    for (int n = tid; n < M; n += 256) {
        float2 z = make_float2(0.0f, 0.0f);
        if (n < a.nu) {
            z.x = weighted(a, in, ra, n);
            if (has_b)
                z.y = weighted(a, in, rb, n);
        }
        buf[n] = z;
    }
    __syncthreads();

    // forward DIF, half-size h = M/2 ... 1
    for (int lh = a.log2M - 1; lh >= 0; --lh) {
        const int h = 1 << lh, sh = a.log2M - 1 - lh;
        for (int bf = tid; bf < half; bf += 256) {
            const int t = bf & (h - 1);
            const int i0 = ((bf >> lh) << (lh + 1)) + t, i1 = i0 + h;
            const float2 x = buf[i0], y = buf[i1];
            buf[i0] = make_float2(x.x + y.x, x.y + y.y);
            buf[i1] = cmul(make_float2(x.x - y.x, x.y - y.y), a.tw[t << sh]);
        }
        __syncthreads();
    }
    // multiply by the symmetrised real response; position n holds frequency bitrev(n)
    for (int n = tid; n < M; n += 256) {
        const int f = (int)(__brev((unsigned)n) >> (32 - a.log2M));
        const float kf = 0.5f * (a.K[f] + a.K[(M - f) & (M - 1)]);
        buf[n].x *= kf;
        buf[n].y *= kf;
    }
    __syncthreads();
    // inverse DIT, half-size h = 1 ... M/2
    for (int lh = 0; lh < a.log2M; ++lh) {
        const int h = 1 << lh, sh = a.log2M - 1 - lh;
        for (int bf = tid; bf < half; bf += 256) {
            const int t = bf & (h - 1);
            const int i0 = ((bf >> lh) << (lh + 1)) + t, i1 = i0 + h;
            const float2 x = buf[i0];
            const float2 y = cmul_conj(buf[i1], a.tw[t << sh]);
            buf[i0] = make_float2(x.x + y.x, x.y + y.y);
            buf[i1] = make_float2(x.x - y.x, x.y - y.y);
        }
        __syncthreads();
    }
    const float inv = 1.0f / (float)M;
    for (int n = tid; n < a.nu; n += 256) {
        const float2 z = buf[n];
        out[(size_t)ra * a.nu + n] = z.x * inv;
        if (has_b)
            out[(size_t)rb * a.nu + n] = z.y * inv;
    }
}

template <typename T>
hipError_t wf(const FilterArgs &a, const void *in, float *out, hipStream_t s)
{
    const long rows = (long)a.batch * a.n_proj * a.nv;
    const long pairs = (rows + 1) / 2;
    const size_t lds = (size_t)a.M * sizeof(float2);
    hipLaunchKernelGGL((weight_filter_kernel<T>), dim3((unsigned)pairs), dim3(256), lds, s, a, (const T *)in, out,
                       rows);
    return hipGetLastError();
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
