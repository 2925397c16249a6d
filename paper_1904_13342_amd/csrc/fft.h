// In-LDS complex FFT of power-of-two length M (16 ... 4096) for one
// 256-thread workgroup: in-place Stockham passes of radix 8 (radix 4 or 2 for
// the last one) with the butterflies in registers, natural order in and out,
// twiddles from an LDS half table tw[t] = exp(-2 pi i t / M), t < M/2.
#pragma once

#include "common.h"

namespace ph {
namespace lds_fft {

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
__device__ __forceinline__ void transform(float2 *buf, const float2 *tw, int M, int log2M)
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

// The same passes with the transform length fixed at compile time: index
// arithmetic folds to constants and the per-thread item loop unrolls exactly.
template <int R, int DIR, int M, int NS>
__device__ __forceinline__ void stockham_pass_c(float2 *buf, const float2 *tw)
{
    constexpr int items = M / R;
    constexpr int ITER = (items + WF_THREADS - 1) / WF_THREADS;
    constexpr int twscale = M / (NS * R);
    constexpr int half = M / 2;
    float2 v[ITER][R];
#pragma unroll
    for (int it = 0; it < ITER; ++it) {
        const int j = threadIdx.x + it * WF_THREADS;
        if (items % WF_THREADS == 0 || j < items) {
            const int jm = j & (NS - 1);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float2 x = buf[j + r * items];
                if (NS > 1 && r > 0) {
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
    for (int it = 0; it < ITER; ++it) {
        const int j = threadIdx.x + it * WF_THREADS;
        if (items % WF_THREADS == 0 || j < items) {
            const int jm = j & (NS - 1);
            const int base = (j - jm) * R + jm;
#pragma unroll
            for (int r = 0; r < R; ++r)
                buf[base + r * NS] = v[it][r];
        }
    }
    __syncthreads();
}

template <int DIR, int M, int NS = 1>
__device__ __forceinline__ void transform_c(float2 *buf, const float2 *tw)
{
    if constexpr (NS * 8 <= M) {
        stockham_pass_c<8, DIR, M, NS>(buf, tw);
        transform_c<DIR, M, NS * 8>(buf, tw);
    } else if constexpr (NS * 4 == M) {
        stockham_pass_c<4, DIR, M, NS>(buf, tw);
    } else if constexpr (NS * 2 == M) {
        stockham_pass_c<2, DIR, M, NS>(buf, tw);
    }
}

}  // namespace lds_fft
}  // namespace ph
