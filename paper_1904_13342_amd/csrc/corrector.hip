// Training kernels of the learned sinogram-domain corrector
//     x = B F^H diag(K) F (W . W_red . W_cos . p)
// (Sec. III.A: the FDK network of Eq. 5 with trainable projection-domain
// weights, after Wurfl et al.; Sec. III.B / Eq. 6: the trainable filter K):
// the MSE loss and its gradient in the volume, the gradients with respect to
// K and W given the gradient with respect to the filtered projections, and
// the Adam update.
//
// With r = W . W_red . W_cos . p and q = Re IDFT_M(K_s . DFT_M(r)) row by row
// (K_s the symmetrised response), for the row gradient g = dL/dq:
//   dL/dr = Re IDFT_M(K_s . DFT_M(g))      (the filter is its own transpose)
//   dL/dW[i][j] = sum over batch and views of dL/dr . W_red . W_cos . p
//   dL/dK[f] = (1/M) sum over rows of Re(R_f conj(G_f)), symmetrised in f.
// Two rows share each complex transform; the cross terms of the packed
// spectra cancel in the symmetrisation.  A workgroup owns one detector row
// index i and a share of the (batch, view) rows with that index, keeps its dK
// and dW[i] partial sums (and the spectrum R of the current pair) in
// registers, and adds them to the outputs once.
#include "fft.h"

namespace ph {
namespace {

using namespace lds_fft;

__device__ __forceinline__ float wave_sum(float x)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        x += __shfl_xor(x, o);
    return x;
}

__global__ void __launch_bounds__(256) mse_kernel(const float *__restrict__ x, const float *__restrict__ ref,
                                                  const float *__restrict__ mask, size_t n, float inv_n,
                                                  float *__restrict__ grad, double *__restrict__ loss)
{
    __shared__ float part[4];
    float local = 0.0f;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256) {
        const float mi = mask ? mask[i] : 1.0f;
        const float d = mi * (x[i] - ref[i]);
        grad[i] = 2.0f * inv_n * mi * d;
        local = fmaf(d, d, local);
    }
    if (!loss)
        return;
    local = wave_sum(local);
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x >> 6] = local;
    __syncthreads();
    if (threadIdx.x == 0)   // workgroup partials meet in FP64
        unsafeAtomicAdd(loss, ((double)part[0] + part[1] + part[2] + part[3]) * (double)inv_n);
}

// W_red[k][j] * W_cos(i, j), the fixed part of the weight of pixel (i, j) in
// view k (no cosine weight for parallel beams, cos_sdd = 0)
__device__ __forceinline__ float pixel_weight(const FilterArgs &a, int k, int i, int j)
{
    return a.W_red[(size_t)k * a.nu + j] * cosine_weight(a, i, j);
}

template <int M>
__global__ void __launch_bounds__(256) corrector_grad_kernel(FilterArgs a, int splits, const float *__restrict__ p,
                                                             const float *__restrict__ gq, float *__restrict__ dK,
                                                             float *__restrict__ dW)
{
    constexpr int MAXF = (M + 255) / 256;   // frequencies (and detector pixels) per thread
    extern __shared__ float2 lds[];
    constexpr int half = M >> 1;
    float2 *buf = lds, *tw = lds + M;
    const int tid = threadIdx.x;
    const int i = blockIdx.x % a.nv, split = blockIdx.x / a.nv;
    const int rows = a.batch * a.n_proj;   // (batch, view) rows with detector row index i
    const int pairs = (rows + 1) / 2;
    for (int n = tid; n < half; n += 256)
        tw[n] = a.tw[n];
    float dk[MAXF], dw[MAXF], ks[MAXF];
    float2 R[MAXF];
#pragma unroll
    for (int t = 0; t < MAXF; ++t) {
        const int f = tid + 256 * t;
        dk[t] = 0.0f;
        dw[t] = 0.0f;
        ks[t] = f < M ? 0.5f * (a.K[f] + a.K[(M - f) & (M - 1)]) : 0.0f;
    }
    for (int pr = split; pr < pairs; pr += splits) {
        const int ra = 2 * pr, rb = ra + 1;
        const bool has_b = rb < rows;
        const int ka = ra % a.n_proj, kb = has_b ? rb % a.n_proj : 0;
        const size_t oa = ((size_t)ra * a.nv + i) * a.nu, ob = ((size_t)rb * a.nv + i) * a.nu;
        // R = DFT(r_a + i r_b), kept in registers
        __syncthreads();   // buf free
        for (int n = tid; n < M; n += 256) {
            float2 z = make_float2(0.0f, 0.0f);
            if (n < a.nu) {
                const float w = a.W ? a.W[(size_t)i * a.nu + n] : 1.0f;
                z.x = w * pixel_weight(a, ka, i, n) * p[oa + n];
                if (has_b)
                    z.y = w * pixel_weight(a, kb, i, n) * p[ob + n];
            }
            buf[n] = z;
        }
        __syncthreads();
        transform_c<-1, M>(buf, tw);
#pragma unroll
        for (int t = 0; t < MAXF; ++t) {
            const int f = tid + 256 * t;
            R[t] = f < M ? buf[f] : make_float2(0.0f, 0.0f);
        }
        // G = DFT(g_a + i g_b)
        __syncthreads();
        for (int n = tid; n < M; n += 256) {
            float2 z = make_float2(0.0f, 0.0f);
            if (n < a.nu) {
                z.x = gq[oa + n];
                if (has_b)
                    z.y = gq[ob + n];
            }
            buf[n] = z;
        }
        __syncthreads();
        transform_c<-1, M>(buf, tw);
#pragma unroll
        for (int t = 0; t < MAXF; ++t) {
            const int f = tid + 256 * t;
            if (f < M) {
                const float2 G = buf[f];
                dk[t] = fmaf(R[t].x, G.x, fmaf(R[t].y, G.y, dk[t]));   // Re(R conj G)
                buf[f] = make_float2(ks[t] * G.x, ks[t] * G.y);
            }
        }
        __syncthreads();
        transform_c<1, M>(buf, tw);   // M * (dL/dr_a + i dL/dr_b)
        const float inv = 1.0f / (float)M;
#pragma unroll
        for (int t = 0; t < MAXF; ++t) {
            const int j = tid + 256 * t;
            if (j < a.nu) {
                const float2 dr = buf[j];
                float acc = dr.x * inv * pixel_weight(a, ka, i, j) * p[oa + j];
                if (has_b)
                    acc = fmaf(dr.y * inv, pixel_weight(a, kb, i, j) * p[ob + j], acc);
                dw[t] += acc;
            }
        }
    }
    // dK: symmetrise over f <-> M - f through LDS, then one atomic per
    // frequency; dW[i]: one atomic per pixel
    __syncthreads();
    float *sym = (float *)buf;
#pragma unroll
    for (int t = 0; t < MAXF; ++t) {
        const int f = tid + 256 * t;
        if (f < M)
            sym[f] = dk[t];
    }
    __syncthreads();
    const float invM = 1.0f / (float)M;
#pragma unroll
    for (int t = 0; t < MAXF; ++t) {
        const int f = tid + 256 * t;
        if (f < M)
            unsafeAtomicAdd(dK + f, 0.5f * (sym[f] + sym[(M - f) & (M - 1)]) * invM);
        if (dW && f < a.nu)
            unsafeAtomicAdd(dW + (size_t)i * a.nu + f, dw[t]);
    }
}

__global__ void adam_kernel(float *__restrict__ param, const float *__restrict__ grad, float *__restrict__ m,
                            float *__restrict__ v, size_t n, float lr, float b1, float b2, float eps, float c1,
                            float c2)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float gi = grad[i];
        const float mi = fmaf(b1, m[i], (1.0f - b1) * gi);
        const float vi = fmaf(b2, v[i], (1.0f - b2) * gi * gi);
        m[i] = mi;
        v[i] = vi;
        param[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

}  // namespace

hipError_t launch_mse(const float *x, const float *ref, const float *mask, size_t n, float *grad, double *loss,
                      hipStream_t s)
{
    if (loss) {   // no loss requested: the gradient only
        const hipError_t e = fill_zero((float *)loss, 2, s);
        if (e != hipSuccess)
            return e;
    }
    const size_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(mse_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, s, x, ref, mask, n,
                       1.0f / (float)n, grad, loss);
    return hipGetLastError();
}

hipError_t launch_corrector_grad(const FilterArgs &a, const float *p, const float *gq, float *dK, float *dW,
                                 hipStream_t s)
{
    hipError_t e = fill_zero(dK, (size_t)a.M, s);
    if (e == hipSuccess && dW)
        e = fill_zero(dW, (size_t)a.nv * a.nu, s);
    if (e != hipSuccess)
        return e;
    // one workgroup per (detector row index, share of the rows with that index);
    // about 2048 workgroups in all so that every CU holds several
    const int pairs = (a.batch * a.n_proj + 1) / 2;
    int splits = (2048 + a.nv - 1) / a.nv;
    if (splits > pairs)
        splits = pairs;
    const size_t lds = ((size_t)a.M + a.M / 2) * sizeof(float2);
    const dim3 grid((unsigned)(a.nv * splits));
    switch (a.log2M) {
    case 4: hipLaunchKernelGGL(corrector_grad_kernel<16>, grid, dim3(256), lds, s, a, splits, p, gq, dK, dW); break;
    case 5: hipLaunchKernelGGL(corrector_grad_kernel<32>, grid, dim3(256), lds, s, a, splits, p, gq, dK, dW); break;
    case 6: hipLaunchKernelGGL(corrector_grad_kernel<64>, grid, dim3(256), lds, s, a, splits, p, gq, dK, dW); break;
    case 7: hipLaunchKernelGGL(corrector_grad_kernel<128>, grid, dim3(256), lds, s, a, splits, p, gq, dK, dW); break;
    case 8: hipLaunchKernelGGL(corrector_grad_kernel<256>, grid, dim3(256), lds, s, a, splits, p, gq, dK, dW); break;
    case 9: hipLaunchKernelGGL(corrector_grad_kernel<512>, grid, dim3(256), lds, s, a, splits, p, gq, dK, dW); break;
    case 10: hipLaunchKernelGGL(corrector_grad_kernel<1024>, grid, dim3(256), lds, s, a, splits, p, gq, dK, dW); break;
    case 11: hipLaunchKernelGGL(corrector_grad_kernel<2048>, grid, dim3(256), lds, s, a, splits, p, gq, dK, dW); break;
    case 12: hipLaunchKernelGGL(corrector_grad_kernel<4096>, grid, dim3(256), lds, s, a, splits, p, gq, dK, dW); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_adam(float *param, const float *grad, float *m, float *v, size_t n, float lr, float b1, float b2,
                       float eps, int t, hipStream_t s)
{
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    const size_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, s, param, grad, m,
                       v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace ph
