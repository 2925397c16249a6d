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
#include "common.h"

namespace ph {
namespace {

constexpr int WF_THREADS = 256;

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(fmaf(a.x, b.x, -a.y * b.y), fmaf(a.x, b.y, a.y * b.x));
}

// a * exp(DIR * 2 pi i * k / R) for a compile-time k (DIR = -1 forward, +1 inverse)
template <int R, int K, int DIR>
__device__ __forceinline__ float2 rot(float2 a)
{
    constexpr int k = ((K % R) + R) % R;
    if constexpr (k == 0) {
        return a;
    } else if constexpr (4 * k == R) {   // exp(DIR i pi/2) = DIR * i
        return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
    } else if constexpr (2 * k == R) {   // -1
        return make_float2(-a.x, -a.y);
    } else if constexpr (4 * k == 3 * R) {   // exp(DIR i 3pi/2) = -DIR * i
        return DIR < 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
    } else {
        static_assert(R == 8 && (k == 1 || k == 3), "odd multiples of pi/4 only");
        constexpr float h = 0.70710678118654752440f;   // cos(pi/4) = sin(pi/4)
        return cmul(a, make_float2(k == 1 ? h : -h, DIR * h));
    }
}

// In-register DFT of size R (2, 4 or 8): decimation in frequency, then the
// bit-reversal permutation, so v[k] = sum_n v[n] exp(DIR 2 pi i n k / R).
template <int R, int DIR>
__device__ __forceinline__ void dft(float2 *v)
{
#pragma unroll
    for (int h = R / 2; h >= 1; h >>= 1) {
#pragma unroll
        for (int g0 = 0; g0 < R; g0 += 2 * h) {
#pragma unroll
            for (int t = 0; t < h; ++t) {
                const float2 a = v[g0 + t], b = v[g0 + t + h];
                v[g0 + t] = cadd(a, b);
                const float2 d = csub(a, b);
                // twiddle exp(DIR 2 pi i t / (2h)) = exp(DIR 2 pi i t (R / 2h) / R)
                switch (t * (R / (2 * h))) {
                case 0: v[g0 + t + h] = d; break;
                case 1: v[g0 + t + h] = rot<R, 1, DIR>(d); break;
                case 2: v[g0 + t + h] = rot<R, 2, DIR>(d); break;
                case 3: v[g0 + t + h] = rot<R, 3, DIR>(d); break;
                default: break;
                }
            }
        }
    }
    if constexpr (R == 4) {
        const float2 t1 = v[1];
        v[1] = v[2];
        v[2] = t1;
    } else if constexpr (R == 8) {
        float2 t1 = v[1];
        v[1] = v[4];
        v[4] = t1;
        t1 = v[3];
        v[3] = v[6];
        v[6] = t1;
    }
}

// One in-place Stockham pass of radix R over M points with span Ns (the
// product of the radices of the previous passes): every item's inputs are
// read into registers, then all outputs are written.  At most MAXIT items per
// thread (M <= 4096).  Twiddles come from the LDS half table
// tw[t] = exp(-2 pi i t / M), t < M/2, with exp(-2 pi i (t + M/2) / M) = -tw[t].
template <int R, int DIR>
__device__ __forceinline__ void stockham_pass(float2 *buf, const float2 *tw, int M, int Ns)
{
    constexpr int MAXIT = 4096 / R / WF_THREADS;
    const int items = M / R;
    const int twscale = M / (Ns * R);
    const int half = M >> 1;
    float2 v[MAXIT][R];
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
        const int j = threadIdx.x + it * WF_THREADS;
        if (j < items) {
            const int jm = j & (Ns - 1);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float2 x = buf[j + r * items];
                if (r > 0 && jm > 0) {
                    const int t = (jm * r * twscale) & (M - 1);
                    float2 w = tw[t & (half - 1)];
                    if (t >= half)
                        w = make_float2(-w.x, -w.y);
                    if (DIR > 0)
                        w.y = -w.y;
                    x = cmul(x, w);
                }
                v[it][r] = x;
            }
            dft<R, DIR>(v[it]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
        const int j = threadIdx.x + it * WF_THREADS;
        if (j < items) {
            const int jm = j & (Ns - 1);
            const int base = (j - jm) * R + jm;
#pragma unroll
            for (int r = 0; r < R; ++r)
                buf[base + r * Ns] = v[it][r];
        }
    }
    __syncthreads();
}

// Full in-place transform of buf (natural order in and out).
template <int DIR>
__device__ __forceinline__ void fft(float2 *buf, const float2 *tw, int M, int log2M)
{
    int Ns = 1;
    int left = log2M;
    while (left >= 3) {
        stockham_pass<8, DIR>(buf, tw, M, Ns);
        Ns *= 8;
        left -= 3;
    }
    if (left == 2)
        stockham_pass<4, DIR>(buf, tw, M, Ns);
    else if (left == 1)
        stockham_pass<2, DIR>(buf, tw, M, Ns);
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
__global__ void __launch_bounds__(WF_THREADS) weight_filter_kernel(FilterArgs a, const T *__restrict__ in,
                                                                   float *__restrict__ out, long rows)
{
    extern __shared__ float2 lds[];
    const int M = a.M, half = M >> 1;
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
        fft<-1>(buf, tw, M, a.log2M);
        // multiply by the symmetrised real response
        for (int n = tid; n < M; n += WF_THREADS) {
            const float kf = 0.5f * (a.K[n] + a.K[(M - n) & (M - 1)]);
            buf[n].x *= kf;
            buf[n].y *= kf;
        }
        __syncthreads();
        fft<1>(buf, tw, M, a.log2M);
        for (int n = tid; n < a.nu; n += WF_THREADS) {
            const float2 z = buf[n];
            out[(size_t)ra * a.nu + n] = z.x * inv;
            if (has_b)
                out[(size_t)rb * a.nu + n] = z.y * inv;
        }
        __syncthreads();   // buf is overwritten by the next pair's load
    }
}

template <typename T>
hipError_t wf(const FilterArgs &a, const void *in, float *out, hipStream_t s)
{
    const long rows = (long)a.batch * a.n_proj * a.nv;
    const long pairs = (rows + 1) / 2;
    const size_t lds = ((size_t)a.M + a.M / 2) * sizeof(float2);
    const long max_groups = 256L * 8;   // enough resident workgroups for 256 CUs
    const unsigned grid = (unsigned)(pairs < max_groups ? pairs : max_groups);
    hipLaunchKernelGGL((weight_filter_kernel<T>), dim3(grid), dim3(WF_THREADS), lds, s, a, (const T *)in, out, rows);
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
