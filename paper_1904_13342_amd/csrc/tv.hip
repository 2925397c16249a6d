// Total variation and its gradient, the regulariser of the iterative
// reconstruction (Sec. III.B.1, Eq. 7), with forward differences
// D_d(q) = x[q + e_d] - x[q] (zero where q + e_d leaves the grid):
//   isotropic    TV = sum_q phi(q),  phi(q) = sqrt(sum_d D_d(q)^2 + eps^2),
//                dTV/dx[p] = -sum_d D_d(p) / phi(p) + sum_d D_d(p - e_d) / phi(p - e_d);
//   anisotropic  TV = sum_q sum_d psi(D_d(q)),  psi(t) = sqrt(t^2 + eps^2), over
//                the axes of extent > 1
//                (|t| at eps = 0: the sum of absolute differences, the total
//                variation of the framework the paper takes TV from),
//                dTV/dx[p] = -sum_d r(D_d(p)) + sum_d r(D_d(p - e_d)),
//                r(t) = t / psi(t) (sign(t) at eps = 0, and 0 at t = 0).
// One thread per voxel; the 13 neighbours it reads come through the caches
// (the kernel is bound by the 12 bytes per voxel of x and the gradient).
#include "common.h"

namespace ph {
namespace {

struct TvArgs {
    int nx, ny, nz;
    float eps2, weight;
};

// anisotropic summand and its derivative for one difference t
__device__ __forceinline__ float tv_psi(float t, float eps2) { return sqrtf(fmaf(t, t, eps2)); }
__device__ __forceinline__ float tv_r(float t, float eps2)
{
    if (eps2 > 0.0f)
        return t / sqrtf(fmaf(t, t, eps2));
    return t > 0.0f ? 1.0f : t < 0.0f ? -1.0f : 0.0f;
}

// phi(q) for q = (x, y, z) inside the grid
__device__ __forceinline__ float tv_phi(const float *__restrict__ v, const TvArgs &a, int x, int y, int z, size_t q,
                                        size_t sy, size_t sz)
{
    const float c = v[q];
    const float dx = x + 1 < a.nx ? v[q + 1] - c : 0.0f;
    const float dy = y + 1 < a.ny ? v[q + sy] - c : 0.0f;
    const float dz = z + 1 < a.nz ? v[q + sz] - c : 0.0f;
    return sqrtf(fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, a.eps2))));
}

template <bool ANISO>
__global__ void __launch_bounds__(256) tv_kernel(TvArgs a, const float *__restrict__ vol, float *__restrict__ grad,
                                                 double *__restrict__ value, long n_per_item, int batch)
{
    __shared__ double part[4];
    const size_t sy = (size_t)a.nx, sz = (size_t)a.nx * a.ny;
    const long total = n_per_item * batch;
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    // every workgroup lies inside one batch item (n_per_item is a multiple of
    // 256 or the grid is laid out per item)
    const int b = (int)(((long)blockIdx.x * 256) / n_per_item);
    float phi_p = 0.0f;
    if (i < total) {
        const long r = i - (long)b * n_per_item;
        const int x = (int)(r % a.nx), y = (int)((r / a.nx) % a.ny), z = (int)(r / sz);
        const float *v = vol + (size_t)b * n_per_item;
        const size_t p = (size_t)r;
        const float c = v[p];
        const float dx = x + 1 < a.nx ? v[p + 1] - c : 0.0f;
        const float dy = y + 1 < a.ny ? v[p + sy] - c : 0.0f;
        const float dz = z + 1 < a.nz ? v[p + sz] - c : 0.0f;
        if (ANISO) {
            // axes of extent 1 (the z axis of a 2D image) have no differences: no eps term
            phi_p = (a.nx > 1 ? tv_psi(dx, a.eps2) : 0.0f) + (a.ny > 1 ? tv_psi(dy, a.eps2) : 0.0f) +
                    (a.nz > 1 ? tv_psi(dz, a.eps2) : 0.0f);
            if (grad) {
                float g = -(tv_r(dx, a.eps2) + tv_r(dy, a.eps2) + tv_r(dz, a.eps2));
                if (x > 0)
                    g += tv_r(c - v[p - 1], a.eps2);
                if (y > 0)
                    g += tv_r(c - v[p - sy], a.eps2);
                if (z > 0)
                    g += tv_r(c - v[p - sz], a.eps2);
                float *gp = grad + (size_t)b * n_per_item + p;
                *gp = fmaf(a.weight, g, *gp);
            }
        } else {
            phi_p = sqrtf(fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, a.eps2))));
            if (grad) {
                float g = -(dx + dy + dz) / phi_p;
                if (x > 0)
                    g += (c - v[p - 1]) / tv_phi(v, a, x - 1, y, z, p - 1, sy, sz);
                if (y > 0)
                    g += (c - v[p - sy]) / tv_phi(v, a, x, y - 1, z, p - sy, sy, sz);
                if (z > 0)
                    g += (c - v[p - sz]) / tv_phi(v, a, x, y, z - 1, p - sz, sy, sz);
                float *gp = grad + (size_t)b * n_per_item + p;
                *gp = fmaf(a.weight, g, *gp);
            }
        }
    }
    if (value) {
        // workgroup sum in FP64, one atomic per workgroup
        double s = (double)phi_p;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1)
            s += __shfl_xor(s, o);
        if ((threadIdx.x & 63) == 0)
            part[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0)
            unsafeAtomicAdd(value + b, part[0] + part[1] + part[2] + part[3]);
    }
}

}  // namespace

hipError_t launch_tv(const float *vol, int nx, int ny, int nz, int batch, bool aniso, float eps, float weight,
                     float *grad, double *value, hipStream_t s)
{
    const auto kernel = aniso ? tv_kernel<true> : tv_kernel<false>;
    const long n = (long)nx * ny * nz;
    if (value) {
        hipError_t e = fill_zero((float *)value, 2 * (size_t)batch, s);
        if (e != hipSuccess)
            return e;
    }
    TvArgs a;
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.eps2 = eps * eps;
    a.weight = weight;
    if (n % 256 == 0 || batch == 1) {
        const long blocks = (n * batch + 255) / 256;
        hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, vol, grad, value, n, batch);
        return hipGetLastError();
    }
    // items whose size is not a multiple of 256: one launch per item, so no
    // workgroup straddles two items
    for (int b = 0; b < batch; ++b) {
        const long blocks = (n + 255) / 256;
        hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(256), 0, s, a, vol + (size_t)b * n,
                           grad ? grad + (size_t)b * n : nullptr, value ? value + b : nullptr, n, 1);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace ph
