// Ray-driven cone-beam forward projection from projection matrices
// (Sec. II.B.2, after Galigekere et al.): one thread per detector pixel; the
// ray from the source through the pixel is sampled at fixed steps on the
// lattice anchored at its point closest to the isocentre, and the volume is
// interpolated trilinearly with zero outside the grid.
#include "common.h"

namespace ph {
namespace {

template <typename T>
__device__ __forceinline__ float vox(const T *f, int nx, int ny, int nz, int ix, int iy, int iz)
{
    return ((unsigned)ix < (unsigned)nx && (unsigned)iy < (unsigned)ny && (unsigned)iz < (unsigned)nz)
               ? load_f32(f + ((size_t)iz * ny + iy) * nx + ix)
               : 0.0f;
}

__device__ __forceinline__ bool krange(float p, float e, int n, float &lo, float &hi)
{
    if (fabsf(e) < 1e-30f)
        return p > -1.0f && p < (float)n;
    const float t1 = (-1.0f - p) / e, t2 = ((float)n - p) / e;
    lo = fmaxf(lo, fminf(t1, t2));
    hi = fminf(hi, fmaxf(t1, t2));
    return true;
}

template <typename T>
__global__ void __launch_bounds__(256) fp_cone_kernel(Geom3D g, const ConeFPView *__restrict__ views,
                                                      const T *__restrict__ vol, T *__restrict__ proj)
{
    const int j = blockIdx.x * 64 + (threadIdx.x & 63);
    const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int k = blockIdx.z % g.n_proj, b = blockIdx.z / g.n_proj;
    if (j >= g.nu || i >= g.nv)
        return;
    // ray setup in double precision: anchor (point closest to the isocentre)
    // and unit direction, then index coordinates rounded once to FP32
    const ConeFPView &v = views[k];
    const double jc = (double)j - (double)g.cu, ic = (double)i - (double)g.cv;
    double d[3];
#pragma unroll
    for (int t = 0; t < 3; ++t)
        d[t] = fma(jc, v.du[t], fma(ic, v.dv[t], v.d0[t]));
    const double rn = 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
#pragma unroll
    for (int t = 0; t < 3; ++t)
        d[t] *= rn;
    const double t0 = -(v.s[0] * d[0] + v.s[1] * d[1] + v.s[2] * d[2]);
    const float X0 = (float)((fma(t0, d[0], v.s[0]) - (double)g.ox) / (double)g.sx);
    const float Y0 = (float)((fma(t0, d[1], v.s[1]) - (double)g.oy) / (double)g.sy);
    const float Z0 = (float)((fma(t0, d[2], v.s[2]) - (double)g.oz) / (double)g.sz);
    const float eX = (float)((double)g.step * d[0] / (double)g.sx);
    const float eY = (float)((double)g.step * d[1] / (double)g.sy);
    const float eZ = (float)((double)g.step * d[2] / (double)g.sz);
    float lo = -3.0e38f, hi = 3.0e38f;
    float acc = 0.0f;
    const T *f = vol + (size_t)b * g.nx * g.ny * g.nz;
    if (krange(X0, eX, g.nx, lo, hi) && krange(Y0, eY, g.ny, lo, hi) && krange(Z0, eZ, g.nz, lo, hi) && lo < hi) {
        const int k0 = (int)floorf(lo) - 1, k1 = (int)ceilf(hi) + 1;
        for (int m = k0; m <= k1; ++m) {
            const float fm = (float)m;
            const float X = fmaf(fm, eX, X0), Y = fmaf(fm, eY, Y0), Z = fmaf(fm, eZ, Z0);
            const float fx = floorf(X), fy = floorf(Y), fz = floorf(Z);
            const int ix = (int)fx, iy = (int)fy, iz = (int)fz;
            const float tx = X - fx, ty = Y - fy, tz = Z - fz;
            float c[2];
#pragma unroll
            for (int dz = 0; dz < 2; ++dz) {
                const float p00 = vox(f, g.nx, g.ny, g.nz, ix, iy, iz + dz);
                const float p01 = vox(f, g.nx, g.ny, g.nz, ix + 1, iy, iz + dz);
                const float p10 = vox(f, g.nx, g.ny, g.nz, ix, iy + 1, iz + dz);
                const float p11 = vox(f, g.nx, g.ny, g.nz, ix + 1, iy + 1, iz + dz);
                const float a0 = fmaf(tx, p01 - p00, p00), a1 = fmaf(tx, p11 - p10, p10);
                c[dz] = fmaf(ty, a1 - a0, a0);
            }
            acc += fmaf(tz, c[1] - c[0], c[0]);
        }
    }
    store_f32(proj + (((size_t)b * g.n_proj + k) * g.nv + i) * g.nu + j, g.step * acc);
}

template <typename T>
hipError_t fp_cone(const Geom3D &g, const ConeFPView *views, const void *vol, void *proj, int batch, hipStream_t s)
{
    dim3 grid((g.nu + 63) / 64, (g.nv + 3) / 4, g.n_proj * batch);
    hipLaunchKernelGGL((fp_cone_kernel<T>), grid, dim3(256), 0, s, g, views, (const T *)vol, (T *)proj);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_project_cone(int dtype, const Geom3D &g, const ConeFPView *views, const void *vol, void *proj,
                               int batch, hipStream_t stream)
{
    switch (dtype) {
    case 0: return fp_cone<float>(g, views, vol, proj, batch, stream);
    case 1: return fp_cone<f16_t>(g, views, vol, proj, batch, stream);
    default: return fp_cone<bf16_t>(g, views, vol, proj, batch, stream);
    }
}

}  // namespace ph
