// Projection-domain weighting and row-wise filtering, q = F^H K F (W p)
// (Eq. 4 / Eq. 5; the filter is a diagonal multiply in the Fourier domain,
// Sec. II.C.4; the weights are Sec. II.C.5's cosine and redundancy weights).
//
// Two detector rows are transformed at once: row a goes into the real part
// and row b into the imaginary part of one complex M-point sequence.  The
// response is real and even (it is symmetrised first), so the inverse
// transform of K . DFT(a + i b) is (K * a) + i (K * b): both filtered rows come
// out of one forward / inverse pair.
//
// M = 2048 and M = 1024 (the lengths of every workload here) take one wave, or
// half a wave, per pair: a four-step transform with 32-point DFTs in registers
// and wave-private LDS transposes (weight_filter_2048_kernel,
// weight_filter_1024_kernel below).  Other lengths take a workgroup per pair:
// in-place Stockham radix-8 passes (radix 4 or 2 for the last one) in LDS with
// the butterflies in registers, natural order in and out, the twiddle
// half-table held in LDS.  Both loop over pairs on a grid sized to the machine.
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

// ----------------------------------------------------------------- M = 2048
// One wave per pair of rows (a + i b as above), no workgroup barriers after
// set-up.  The 2048-point transform is taken as 32 x 64 (four-step):
//   n = 64 a + b, k = c + 32 d:  X[c + 32 d] = sum_b w64^(b d) w2048^(b c) sum_a x[64 a + b] w32^(a c).
// Lane b holds x[64 a + b] (a = 0..31) and takes the 32-point DFT over a in
// registers, multiplies by w2048^(b c) and writes row c of a wave-private LDS
// transpose; lane (c, p) then reads the even (p = 0) or odd (p = 1) b of
// row c, takes the 32-point DFT over them and one xor-1 exchange forms
// X[c + 32 (d' + 32 p)].  After the multiply by K the inverse runs the same
// steps backwards, and lane b ends with y[64 a + b], of which n < nu is kept.
namespace w2k {

constexpr int WAVES = 8;         // at most: one workgroup per CU (LDS-bound), two waves per SIMD
// Row strides (float2) chosen against LDS bank conflicts: lanes (c, p) read
// [c][2 m + p] of the forward transpose and [c][2 be + p] of the twiddle
// table, which an even stride of 2 mod 32 spreads over all banks.
constexpr int TS = 66;          // forward transpose [c][b] and twiddle table [k][b]
constexpr int US = 33;          // inverse transpose [b][c]
constexpr int BUF = 64 * US;    // float2 per wave
static_assert(BUF >= 32 * TS, "the forward transpose fits in the wave's buffer");
constexpr int MID = 2 * 32;     // middle-step twiddles [d][p] (float2)

__device__ constexpr int rev5(int k)
{
    return ((k & 1) << 4) | ((k & 2) << 2) | (k & 4) | ((k & 8) >> 2) | ((k & 16) >> 4);
}

// d * exp(DIR * 2 pi i t / 32) for t resolved at compile time after unrolling
template <int DIR>
__device__ __forceinline__ float2 tw32(float2 d, int t)
{
    constexpr float C[16] = {1.000000000e+00f, 9.807852507e-01f, 9.238795042e-01f, 8.314695954e-01f,
                             7.071067691e-01f, 5.555702448e-01f, 3.826834261e-01f, 1.950903237e-01f,
                             0.0f,             -1.950903237e-01f, -3.826834261e-01f, -5.555702448e-01f,
                             -7.071067691e-01f, -8.314695954e-01f, -9.238795042e-01f, -9.807852507e-01f};
    constexpr float S[16] = {0.000000000e+00f, 1.950903237e-01f, 3.826834261e-01f, 5.555702448e-01f,
                             7.071067691e-01f, 8.314695954e-01f, 9.238795042e-01f, 9.807852507e-01f,
                             1.000000000e+00f, 9.807852507e-01f, 9.238795042e-01f, 8.314695954e-01f,
                             7.071067691e-01f, 5.555702448e-01f, 3.826834261e-01f, 1.950903237e-01f};
    if (t == 0)
        return d;
    if (t == 8)   // exp(DIR i pi/2) = DIR * i
        return DIR < 0 ? make_float2(d.y, -d.x) : make_float2(-d.y, d.x);
    return cmul(d, make_float2(C[t], DIR * S[t]));
}

// In-register 32-point DFT (radix-2 decimation in frequency): natural order
// in, bit-reversed order out (X[k] = v[rev5(k)]).  With ZERO_TOP the inputs
// v[16..31] are known to be zero and the first stage only twiddles.
template <int DIR, bool ZERO_TOP = false>
__device__ __forceinline__ void dft32(float2 (&v)[32])
{
#pragma unroll
    for (int s = 16; s >= 1; s >>= 1) {
#pragma unroll
        for (int j = 0; j < 32; j += 2 * s) {
#pragma unroll
            for (int k = 0; k < s; ++k) {
                if (ZERO_TOP && s == 16) {
                    v[j + k + s] = tw32<DIR>(v[j + k], k);
                } else {
                    const float2 x = v[j + k], y = v[j + k + s];
                    v[j + k] = cadd(x, y);
                    v[j + k + s] = tw32<DIR>(csub(x, y), k * (16 / s));
                }
            }
        }
    }
}

// the value of lane (lane xor 1): DPP quad permutation [1, 0, 3, 2]
__device__ __forceinline__ float xor1f(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ float2 xor1(float2 x) { return make_float2(xor1f(x.x), xor1f(x.y)); }

// One detector row as a buffer resource: loads past its end (or from an
// absent row, bytes = 0) return 0 without a branch.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void *base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
template <typename T> __device__ __forceinline__ float row_load(__amdgpu_buffer_rsrc_t r, int j);
template <> __device__ __forceinline__ float row_load<float>(__amdgpu_buffer_rsrc_t r, int j)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, j * 4, 0, 0));
}
template <> __device__ __forceinline__ float row_load<f16_t>(__amdgpu_buffer_rsrc_t r, int j)
{
    return (float)__builtin_bit_cast(f16_t, (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, j * 2, 0, 0));
}
template <> __device__ __forceinline__ float row_load<bf16_t>(__amdgpu_buffer_rsrc_t r, int j)
{
    return __uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, j * 2, 0, 0) << 16);
}

// orders the wave's LDS writes before its lanes read each other's values
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace w2k

// The two rows of pair pr: their index ra = 2 pr (rows < 2^30, so 32 bits
// hold it and the next pair's), whether row b exists, and each row's detector
// row i and view k in the (batch, view, row) order.
struct PairRows {
    unsigned ra;
    bool has, has_b;
    int ia, ka, ib, kb;
};

__device__ __forceinline__ PairRows pair_rows(long pr, long rows, int nv, int n_proj)
{
    PairRows r;
    r.ra = (unsigned)(2 * pr);
    r.has = (long)r.ra < rows;
    r.has_b = (long)r.ra + 1 < rows;
    const unsigned q = r.ra / (unsigned)nv;
    r.ia = (int)(r.ra - q * (unsigned)nv);
    r.ka = (int)(q % (unsigned)n_proj);
    r.ib = r.ia + 1;
    r.kb = r.ka;
    if (r.ib == nv) {
        r.ib = 0;
        r.kb = r.ka + 1 == n_proj ? 0 : r.ka + 1;
    }
    return r;
}

// ZERO_TOP: the rows are at most 1024 samples long, so the upper half of the
// zero-padded sequence (and of the output) is never touched, and the registers
// this frees hold the next pair's samples and redundancy weights, loaded while
// the current pair is transformed.
template <typename T, bool ZERO_TOP>
__global__ void __launch_bounds__(w2k::WAVES * 64) __attribute__((amdgpu_waves_per_eu(2))) weight_filter_2048_kernel(FilterArgs a, const T *__restrict__ in,
                                                                             float *__restrict__ out, long rows)
{
    using namespace w2k;
    constexpr int NA = ZERO_TOP ? 16 : 32;   // input and output rows a that can hold samples
    // twt[k TS + b] = w2048^(k b) for k < 32, b < 64: every twiddle of the
    // pair is read at an offset fixed at compile time from a per-lane base;
    // wmid[2 d + p] = w64^d for p = 0 and its conjugate for p = 1
    __shared__ float2 lds[32 * TS + MID + WAVES * BUF];
    float2 *twt = lds;
    float2 *wmid = lds + 32 * TS;
    float2 *buf = lds + 32 * TS + MID + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) * BUF;
    for (int n = threadIdx.x; n < 32 * 64; n += blockDim.x)
        twt[(n >> 6) * TS + (n & 63)] = a.tw[(n >> 6) * (n & 63)];   // k b < 2048
    for (int n = threadIdx.x; n < MID; n += blockDim.x) {
        const float2 w = a.tw[32 * (n >> 1)];
        wmid[n] = make_float2(w.x, (n & 1) ? -w.y : w.y);
    }
    __syncthreads();
    const long pairs = (rows + 1) / 2;
    // The output scale: 1/2048 for the inverse transform, times SDD for the
    // flat detector's cosine weight (applied to the rows below without it).
    const float oscale = (a.cos_sdd > 0.0f && !a.curved) ? a.cos_sdd / 2048.0f : 1.0f / 2048.0f;
    // The symmetrised response at the two outputs k0 = c + 32 d and
    // k1 = k0 + 1024 that meet in this lane's middle step, as their sum and
    // difference, with the output scale (fixed across pairs, kept in registers).
    float ks[32], kd[32];
    {
        const int lc = (threadIdx.x & 63) >> 1;
#pragma unroll
        for (int d = 0; d < 32; ++d) {
            const int k0 = lc + 32 * d, k1 = k0 + 1024;
            const float K0 = 0.5f * (a.K[k0] + a.K[(2048 - k0) & 2047]);
            const float K1 = 0.5f * (a.K[k1] + a.K[2048 - k1]);
            ks[d] = (K0 + K1) * oscale;
            kd[d] = (K0 - K1) * oscale;
        }
    }
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: row bases stay scalar
    const int nw = blockDim.x >> 6;   // waves in this workgroup (1 .. WAVES)
    const long stride = (long)gridDim.x * nw;
    const unsigned row_bytes = (unsigned)a.nu * (unsigned)sizeof(T);
    // the samples of a pair's rows packed as one complex sequence, lane b
    // holding x[64 a + b], and (ZERO_TOP) their redundancy weights: all loads
    // in flight at once, zero past nu and for absent rows
    auto fetch = [&](const PairRows &q, int lane, float2 (&x)[32], float2 (&wr)[32]) {
        const __amdgpu_buffer_rsrc_t sa = row_rsrc(in + (size_t)q.ra * a.nu, q.has ? row_bytes : 0u);
        const __amdgpu_buffer_rsrc_t sb = row_rsrc(in + ((size_t)q.ra + 1) * a.nu * q.has_b, q.has_b ? row_bytes : 0u);
#pragma unroll
        for (int i = 0; i < NA; ++i)
            x[i] = make_float2(row_load<T>(sa, 64 * i + lane), row_load<T>(sb, 64 * i + lane));
        if (ZERO_TOP && a.W_red) {
            const __amdgpu_buffer_rsrc_t wa = row_rsrc(a.W_red + (size_t)q.ka * a.nu, q.has ? 4u * a.nu : 0u);
            const __amdgpu_buffer_rsrc_t wb = row_rsrc(a.W_red + (size_t)q.kb * a.nu, q.has_b ? 4u * a.nu : 0u);
#pragma unroll
            for (int i = 0; i < NA; ++i)
                wr[i] = make_float2(row_load<float>(wa, 64 * i + lane), row_load<float>(wb, 64 * i + lane));
        }
    };
    long pr = (long)blockIdx.x * nw + wave;
    PairRows nxt = pair_rows(pr, rows, a.nv, a.n_proj);
    float2 px[32], pw[32];   // the prefetched pair (ZERO_TOP)
    if constexpr (ZERO_TOP)
        fetch(nxt, threadIdx.x & 63, px, pw);
    for (; pr < pairs; pr += stride) {
        const PairRows cur = nxt;
        // The lane index is made opaque per pair so that per-column terms
        // are recomputed rather than hoisted out of the loop and spilled.
        int lane = threadIdx.x & 63;
        asm volatile("" : "+v"(lane));
        const int c = lane >> 1, p = lane & 1;          // roles in the middle steps
        float2 v[32], wr[32];
        if constexpr (ZERO_TOP) {
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                v[i] = px[i];
                wr[i] = pw[i];
            }
        } else {
            fetch(cur, lane, v, wr);
        }
        // the weights, one wave-uniform pass per factor present
        const int ia = cur.ia, ib = cur.ib;
        // Cosine weights (Kak & Slaney) with u_j = (j - cu) du: on the arc
        // cos(u_j / SDD), the same for both rows (the hardware cosine takes
        // revolutions); on a flat detector SDD / sqrt(SDD^2 + u_j^2 + v_i^2),
        // whose factor SDD is applied with the output scale.
        if (a.cos_sdd > 0.0f && a.curved) {
            const float rev = 1.0f / (a.cos_sdd * 6.283185307f);
            const float g0 = ((float)lane - a.cu) * a.du * rev, gs = 64.0f * a.du * rev;
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                const float w = __builtin_amdgcn_cosf(fmaf((float)i, gs, g0));
                v[i].x *= w;
                v[i].y *= w;
            }
        } else if (a.cos_sdd > 0.0f) {
            const float va = ((float)ia - a.cv) * a.dv, vb = ((float)ib - a.cv) * a.dv;
            const float s2 = a.cos_sdd * a.cos_sdd;
            const float ca = fmaf(va, va, s2), cb = fmaf(vb, vb, s2);
            const float u0 = ((float)lane - a.cu) * a.du, us = 64.0f * a.du;
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                const float u = fmaf((float)i, us, u0), uu = u * u;
                v[i].x *= __builtin_amdgcn_rsqf(uu + ca);
                v[i].y *= __builtin_amdgcn_rsqf(uu + cb);
            }
        }
        if (a.W_red) {
            if constexpr (!ZERO_TOP) {
                const __amdgpu_buffer_rsrc_t wa = row_rsrc(a.W_red + (size_t)cur.ka * a.nu, 4u * a.nu);
                const __amdgpu_buffer_rsrc_t wb = row_rsrc(a.W_red + (size_t)cur.kb * a.nu, 4u * a.nu);
#pragma unroll
                for (int i = 0; i < NA; ++i)
                    wr[i] = make_float2(row_load<float>(wa, 64 * i + lane), row_load<float>(wb, 64 * i + lane));
            }
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                v[i].x *= wr[i].x;
                v[i].y *= wr[i].y;
            }
        }
        if (a.W) {
            const __amdgpu_buffer_rsrc_t wa = row_rsrc(a.W + (size_t)ia * a.nu, 4u * a.nu);
            const __amdgpu_buffer_rsrc_t wb = row_rsrc(a.W + (size_t)ib * a.nu, 4u * a.nu);
#pragma unroll
            for (int i = 0; i < NA; ++i) {
                v[i].x *= row_load<float>(wa, 64 * i + lane);
                v[i].y *= row_load<float>(wb, 64 * i + lane);
            }
        }
        nxt = pair_rows(pr + stride, rows, a.nv, a.n_proj);
        if constexpr (ZERO_TOP)
            fetch(nxt, lane, px, pw);
        dft32<-1, ZERO_TOP>(v);
#pragma unroll
        for (int k = 0; k < 32; ++k)
            buf[k * TS + lane] = k == 0 ? v[rev5(0)] : cmul(v[rev5(k)], twt[k * TS + lane]);
        wave_sync();
#pragma unroll
        for (int m = 0; m < 32; ++m)
            v[m] = buf[c * TS + 2 * m + p];
        dft32<-1>(v);
        // Per output d (held bit-reversed at v[rev5(d)]) lane p = 0 holds the
        // even half's E[d] and lane p = 1 the odd half's O[d].  The last forward
        // step gives X0 = E + w O and X1 = E - w O (w = w64^d, at outputs
        // c + 32 d and c + 32 d + 1024), the response scales them by K0 and K1,
        // and the inverse's first step forms X0 K0 + X1 K1 and
        // (X0 K0 - X1 K1) conj(w).  Written out, lane p = 0 needs
        // (K0 + K1) E + (K0 - K1) w O and lane p = 1 (K0 + K1) O +
        // (K0 - K1) conj(w) E: its own value, the partner's value times its
        // wmid entry, and the two response sums.  The result is stored in
        // natural order at v[d]; bit reversal pairs d with rev5(d), so both
        // entries of a pair are read before either is written.
        auto mid = [&](int d, float2 g) {
            const float2 t = cmul(xor1(g), wmid[2 * d + p]);
            return make_float2(fmaf(ks[d], g.x, kd[d] * t.x), fmaf(ks[d], g.y, kd[d] * t.y));
        };
#pragma unroll
        for (int d = 0; d < 32; ++d) {
            const int r = rev5(d);
            if (r > d) {
                const float2 gd = v[r], gr = v[d];
                v[d] = mid(d, gd);
                v[r] = mid(r, gr);
            } else if (r == d) {
                v[d] = mid(d, v[d]);
            }
        }
        dft32<1>(v);
        wave_sync();   // the forward transpose has been read
#pragma unroll
        for (int be = 0; be < 32; ++be) {
            const int b = 2 * be + p;
            const float2 w = twt[c * TS + b];
            buf[b * US + c] = cmul(v[rev5(be)], make_float2(w.x, -w.y));
        }
        wave_sync();
#pragma unroll
        for (int k = 0; k < 32; ++k)
            v[k] = buf[lane * US + k];
        dft32<1>(v);
        // n < nu is kept (stores past the row's end, or to an absent row b,
        // are dropped by the buffer range check)
        const __amdgpu_buffer_rsrc_t oa = row_rsrc(out + (size_t)cur.ra * a.nu, 4u * a.nu);
        const __amdgpu_buffer_rsrc_t ob = row_rsrc(out + ((size_t)cur.ra + 1) * a.nu * cur.has_b,
                                                   cur.has_b ? 4u * a.nu : 0u);
#pragma unroll
        for (int i = 0; i < NA; ++i) {
            const float2 y = v[rev5(i)];
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(y.x), oa, (64 * i + lane) * 4, 0, 0);
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(y.y), ob, (64 * i + lane) * 4, 0, 0);
        }
        wave_sync();   // the inverse transpose has been read before the next pair writes
    }
}

// ----------------------------------------------------------------- M = 1024
// The same scheme at 1024 = 32 x 32 (n = 32 a + b, k = c + 32 d): each half
// of a wave transforms one pair of rows, lane b of the half holding
// x[32 a + b], and the second step is a plain 32-point DFT per lane c, so no
// lane exchange is needed.  A wave takes four consecutive rows; one buffer
// resource covers them, and a lane's offset for a column past nu (or a row
// past the end) lies beyond the resource, so its loads read 0 and its stores
// are dropped.
namespace w1k {

constexpr int WAVES = 8;        // at most: one workgroup per CU (LDS-bound)
constexpr int S = 33;           // transposes [32][33] per half-wave, twiddle table [32][33] (float2)
constexpr int BUF = 2 * 32 * S; // float2 per wave
constexpr int FAR = 1 << 28;    // element offset past four rows and past any weight table under 1 GiB

}  // namespace w1k

template <typename T>
__global__ void __launch_bounds__(w1k::WAVES * 64) __attribute__((amdgpu_waves_per_eu(2))) weight_filter_1024_kernel(
    FilterArgs a, const T *__restrict__ in, float *__restrict__ out, long rows)
{
    using namespace w1k;
    using w2k::dft32;
    using w2k::rev5;
    using w2k::row_load;
    using w2k::row_rsrc;
    using w2k::wave_sync;
    // twt[k S + b] = w1024^(k b) for k, b < 32; ks: the symmetrised response
    __shared__ float2 lds[32 * S + WAVES * BUF + 512];
    float2 *twt = lds;
    float *ks = (float *)(lds + 32 * S + WAVES * BUF);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: row bases stay scalar
    for (int n = threadIdx.x; n < 32 * 32; n += blockDim.x) {
        twt[(n >> 5) * S + (n & 31)] = a.tw[(n >> 5) * (n & 31)];   // k b < 1024
        ks[n] = 0.5f * (a.K[n] + a.K[(1024 - n) & 1023]);
    }
    __syncthreads();
    const long quads = (rows + 3) / 4;
    const int nw = blockDim.x >> 6;   // waves in this workgroup (1 .. WAVES)
    for (long qd = (long)blockIdx.x * nw + wave; qd < quads; qd += (long)gridDim.x * nw) {
        int lane = threadIdx.x & 63;
        asm volatile("" : "+v"(lane));   // per-column terms recomputed, not hoisted and spilled
        const int h = lane >> 5, l = lane & 31;
        float2 *buf = lds + 32 * S + wave * BUF + h * 32 * S;
        const long r0 = 4 * qd;
        const int nrows = (int)(rows - r0 < 4 ? rows - r0 : 4);
        // this half's rows r0 + 2h (real part) and r0 + 2h + 1 (imaginary part):
        // detector row i and view k of each, from those of r0
        const int i0 = (int)(r0 % a.nv), k0 = (int)((r0 / a.nv) % a.n_proj);
        int ia = i0 + 2 * h, ka = k0;
        while (ia >= a.nv) {
            ia -= a.nv;
            ka = ka + 1 == a.n_proj ? 0 : ka + 1;
        }
        int ib = ia + 1, kb = ka;
        if (ib == a.nv) {
            ib = 0;
            kb = kb + 1 == a.n_proj ? 0 : kb + 1;
        }
        const __amdgpu_buffer_rsrc_t rin = row_rsrc(in + (size_t)r0 * a.nu, (unsigned)nrows * a.nu * (unsigned)sizeof(T));
        const int ea = 2 * h * a.nu, eb = ea + a.nu;   // element offsets of the two rows
        float2 v[32];
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            const int n = 32 * i + l;
            const bool in_row = n < a.nu;
            v[i] = make_float2(row_load<T>(rin, in_row ? ea + n : FAR), row_load<T>(rin, in_row ? eb + n : FAR));
        }
        float oscale = 1.0f / 1024.0f;
        if (a.cos_sdd > 0.0f && a.curved) {
            const float rev = 1.0f / (a.cos_sdd * 6.283185307f);
            const float g0 = ((float)l - a.cu) * a.du * rev, gs = 32.0f * a.du * rev;
#pragma unroll
            for (int i = 0; i < 32; ++i) {
                const float w = __builtin_amdgcn_cosf(fmaf((float)i, gs, g0));
                v[i].x *= w;
                v[i].y *= w;
            }
        } else if (a.cos_sdd > 0.0f) {
            const float va = ((float)ia - a.cv) * a.dv, vb = ((float)ib - a.cv) * a.dv;
            const float s2 = a.cos_sdd * a.cos_sdd;
            const float ca = fmaf(va, va, s2), cb = fmaf(vb, vb, s2);
            const float u0 = ((float)l - a.cu) * a.du, us = 32.0f * a.du;
            oscale *= a.cos_sdd;
#pragma unroll
            for (int i = 0; i < 32; ++i) {
                const float u = fmaf((float)i, us, u0), uu = u * u;
                v[i].x *= __builtin_amdgcn_rsqf(uu + ca);
                v[i].y *= __builtin_amdgcn_rsqf(uu + cb);
            }
        }
        if (a.W_red) {
            const __amdgpu_buffer_rsrc_t wr = row_rsrc(a.W_red, 4u * (unsigned)a.n_proj * a.nu);
            const int wa = ka * a.nu, wb = kb * a.nu;
#pragma unroll
            for (int i = 0; i < 32; ++i) {
                const int n = 32 * i + l;
                const bool in_row = n < a.nu;
                v[i].x *= row_load<float>(wr, in_row ? wa + n : FAR);
                v[i].y *= row_load<float>(wr, in_row ? wb + n : FAR);
            }
        }
        if (a.W) {
            const __amdgpu_buffer_rsrc_t wl = row_rsrc(a.W, 4u * (unsigned)a.nv * a.nu);
            const int wa = ia * a.nu, wb = ib * a.nu;
#pragma unroll
            for (int i = 0; i < 32; ++i) {
                const int n = 32 * i + l;
                const bool in_row = n < a.nu;
                v[i].x *= row_load<float>(wl, in_row ? wa + n : FAR);
                v[i].y *= row_load<float>(wl, in_row ? wb + n : FAR);
            }
        }
        // forward: 32-point DFTs over a (lane b), twiddles w1024^(b c), transpose,
        // 32-point DFTs over b (lane c): X[c + 32 d] at v[rev5(d)]
        dft32<-1>(v);
#pragma unroll
        for (int k = 0; k < 32; ++k)
            buf[k * S + l] = k == 0 ? v[rev5(0)] : cmul(v[rev5(k)], twt[k * S + l]);
        wave_sync();
#pragma unroll
        for (int m = 0; m < 32; ++m)
            v[m] = buf[l * S + m];
        dft32<-1>(v);
        // times the symmetrised response, put in natural order over d in
        // place (bit reversal pairs d with rev5(d))
        const float *kc = ks + l;   // K_s[c + 32 d] = kc[32 d]
#pragma unroll
        for (int d = 0; d < 32; ++d) {
            const int r = rev5(d);
            if (r > d) {
                const float2 gd = v[r], gr = v[d];
                const float kd = kc[32 * d], kq = kc[32 * r];
                v[d] = make_float2(gd.x * kd, gd.y * kd);
                v[r] = make_float2(gr.x * kq, gr.y * kq);
            } else if (r == d) {
                const float kd = kc[32 * d];
                v[d] = make_float2(v[d].x * kd, v[d].y * kd);
            }
        }
        // inverse: 32-point DFTs over d (lane c), twiddles w1024^(-b c),
        // transpose, 32-point DFTs over c (lane b): y[32 a + b] at v[rev5(a)]
        dft32<1>(v);
        wave_sync();   // the forward transpose has been read
#pragma unroll
        for (int b = 0; b < 32; ++b) {
            const float2 w = twt[l * S + b];
            buf[b * S + l] = cmul(v[rev5(b)], make_float2(w.x, -w.y));
        }
        wave_sync();
#pragma unroll
        for (int c = 0; c < 32; ++c)
            v[c] = buf[l * S + c];
        dft32<1>(v);
        const __amdgpu_buffer_rsrc_t ro = row_rsrc(out + (size_t)r0 * a.nu, (unsigned)nrows * a.nu * 4u);
#pragma unroll
        for (int i = 0; i < 32; ++i) {
            const int n = 32 * i + l;
            const bool in_row = n < a.nu;
            const float2 y = v[rev5(i)];
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(y.x * oscale), ro, (in_row ? ea + n : FAR) * 4, 0, 0);
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(y.y * oscale), ro, (in_row ? eb + n : FAR) * 4, 0, 0);
        }
        wave_sync();   // the inverse transpose has been read before the next rows are written
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
hipError_t wf_2048(const FilterArgs &a, const void *in, float *out, hipStream_t s)
{
    const long rows = (long)a.batch * a.n_proj * a.nv;
    if (rows >= (1L << 30))   // row indices are 32-bit
        return wf_m<T, 2048>(a, in, out, s);
    const long pairs = (rows + 1) / 2;
    // One workgroup per CU. Few pairs spread over the CUs one wave each
    // rather than sharing a few CUs' SIMDs; many fill eight waves per CU.
    const long per_cu = (pairs + 255) / 256;
    const int waves = (int)(per_cu < w2k::WAVES ? per_cu : w2k::WAVES);
    const long groups = (pairs + waves - 1) / waves;
    const unsigned grid = (unsigned)(groups < 256 ? groups : 256);
    if (a.nu <= 1024)
        hipLaunchKernelGGL((weight_filter_2048_kernel<T, true>), dim3(grid), dim3(waves * 64), 0, s, a, (const T *)in,
                           out, rows);
    else
        hipLaunchKernelGGL((weight_filter_2048_kernel<T, false>), dim3(grid), dim3(waves * 64), 0, s, a, (const T *)in,
                           out, rows);
    return hipGetLastError();
}

template <typename T>
hipError_t wf_1024(const FilterArgs &a, const void *in, float *out, hipStream_t s)
{
    // weight tables are addressed by 32-bit offsets from one resource
    if ((size_t)a.n_proj * a.nu * 4 >= ((size_t)w1k::FAR) * 4 || (size_t)a.nv * a.nu * 4 >= ((size_t)w1k::FAR) * 4)
        return wf_m<T, 1024>(a, in, out, s);
    const long rows = (long)a.batch * a.n_proj * a.nv;
    const long quads = (rows + 3) / 4;
    const long per_cu = (quads + 255) / 256;
    const int waves = (int)(per_cu < w1k::WAVES ? per_cu : w1k::WAVES);
    const long groups = (quads + waves - 1) / waves;
    const unsigned grid = (unsigned)(groups < 256 ? groups : 256);
    hipLaunchKernelGGL((weight_filter_1024_kernel<T>), dim3(grid), dim3(waves * 64), 0, s, a, (const T *)in, out,
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
    case 10: return wf_1024<T>(a, in, out, s);
    case 11: return wf_2048<T>(a, in, out, s);
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
