// Exact transposes of the two operators (Sec. II.B.2 notes that the
// ray-driven projector and the voxel-driven back-projector are an unmatched
// pair; Eq. 4 and Sec. II.B.1 use A^T as A's gradient operator).
//
// A^T, the transpose of the fixed-step multilinear ray sampler, is computed
// by gather and without atomics: voxel j receives
//     step * sum_r g_r * sum_k Lambda(X_rk - j),
// Lambda the tensor-product hat function, X_rk the same FP32 sample positions
// the forward projector uses.  A thread owns a voxel (2D) or a column segment
// (3D) and walks, per view, the rays that cross its support (j - 1, j + 1)^d.
// In 3D the rays crossing a brick's support are set up once per view into an
// LDS table shared by the block, and every thread accumulates its segment in
// its own LDS slots.
//
// B^T in 2D, the transpose of the voxel-driven distance-weighted
// back-projector, scatters each pixel's value times dbeta * weight into the
// two detector bins of its linear footprint with float atomics (FP32 output);
// the 3D B^T sits beside the back-projector it mirrors.
#include "device_util.h"

namespace ph {
namespace {

// --------------------------------------------------------------- A^T, 2D

// S lanes share one pixel (S a power of two, at most 64, so the lanes of a
// pixel lie in one wave): lane s gathers views s, s + S, ... and the partial
// sums meet in a fixed shuffle tree.
template <typename T, typename TI, bool FAN, int S>
__global__ void __launch_bounds__(256) fpT2d_kernel(Geom2D g, const float2 *__restrict__ views,
                                                    const TI *__restrict__ sino, T *__restrict__ img, long n_pix)
{
    const long t = (long)blockIdx.x * 256 + threadIdx.x;
    const long q = t / S;
    const int s = (int)(t % S);
    if (q >= n_pix)
        return;   // whole pixels only: the S lanes of a pixel leave together
    const int ix = (int)(q % g.nx), iy = (int)((q / g.nx) % g.ny), b = (int)(q / ((long)g.nx * g.ny));
    const TI *sb = sino + (size_t)b * g.n_proj * g.nu;
    const float fx = (float)ix, fy = (float)iy;
    // corners of the support square (ix +- 1, iy +- 1) in world mm
    const float x0 = fmaf(fx - 1.0f, g.sx, g.ox), x1 = fmaf(fx + 1.0f, g.sx, g.ox);
    const float y0 = fmaf(fy - 1.0f, g.sy, g.oy), y1 = fmaf(fy + 1.0f, g.sy, g.oy);
    float acc = 0.0f;
    const float rdu = __builtin_amdgcn_rcpf(g.du);
    for (int k = s; k < g.n_proj; k += S) {
        const float2 c = views[k];
        // detector bins whose rays can cross the support: project its corners
        // (hardware reciprocals: the bin range keeps a margin of one bin below
        // and two above)
        float smin = 3.0e38f, smax = -3.0e38f;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float x = (q & 1) ? x1 : x0, y = (q & 2) ? y1 : y0;
            const float xu = -x * c.y + y * c.x;
            const float w = fmaf(x, c.x, fmaf(y, c.y, g.sid));
            // detector coordinate in mm (arc length on the equiangular detector)
            const float su = !FAN ? xu : g.curved ? g.sdd * atan2f(xu, w) : g.sdd * xu * __builtin_amdgcn_rcpf(w);
            smin = fminf(smin, su);
            smax = fmaxf(smax, su);
        }
        const int j0 = max((int)floorf(fmaf(smin, rdu, g.cu)) - 1, 0);
        const int j1 = min((int)floorf(fmaf(smax, rdu, g.cu)) + 2, g.nu - 1);
        for (int j = j0; j <= j1; ++j) {
            const float gv = load_f32(sb + (size_t)k * g.nu + j);
            if (gv == 0.0f)
                continue;
            float X0, Y0, eX, eY;
            make_ray_2d<FAN>(g, c, j, X0, Y0, eX, eY);
            // the samples that can reach the support: the clip only picks the
            // range to visit (hardware reciprocals, widened by a sample on
            // each side); the exact weights below decide every sample
            float lo = -3.0e38f, hi = 3.0e38f;
            if (!clip_line_rcp(X0, eX, fx - 1.0f, fx + 1.0f, lo, hi) ||
                !clip_line_rcp(Y0, eY, fy - 1.0f, fy + 1.0f, lo, hi) || !(lo < hi + 0.01f))
                continue;
            float w = 0.0f;
            for (int m = (int)floorf(lo) - 1; m <= (int)ceilf(hi) + 1; ++m) {
                const float X = fmaf((float)m, eX, X0), Y = fmaf((float)m, eY, Y0);
                const float wx = 1.0f - fabsf(X - fx), wy = 1.0f - fabsf(Y - fy);
                if (wx > 0.0f && wy > 0.0f)
                    w = fmaf(wx, wy, w);
            }
            acc = fmaf(gv, w, acc);
        }
    }
#pragma unroll
    for (int o = S / 2; o >= 1; o >>= 1)
        acc += __shfl_xor(acc, o);
    if (s == 0)
        store_f32(img + ((size_t)b * g.ny + iy) * g.nx + ix, g.step * acc);
}

// --------------------------------------------------------------- A^T, 3D

constexpr int AT_NZ = 8;          // voxels per column segment
constexpr int AT_RAYS = 1024;     // rays per view held in the block's LDS table

template <typename T, typename TI>
__global__ void __launch_bounds__(256) fpT_cone_kernel(Geom3D g, const ConeFPView *__restrict__ fviews,
                                                       const ConeBPView *__restrict__ bviews,
                                                       const TI *__restrict__ proj, T *__restrict__ vol, int nbx,
                                                       int nby, int nzb)
{
    __shared__ float rtab[7][AT_RAYS];        // X0 Y0 Z0 eX eY eZ, step * g
    __shared__ float accl[AT_NZ][256];        // per-thread segment accumulators
    const int tid = threadIdx.x;
    const int bxi = (int)(blockIdx.x % (unsigned)nbx), byi = (int)((blockIdx.x / (unsigned)nbx) % (unsigned)nby);
    const int bzb = (int)(blockIdx.x / (unsigned)(nbx * nby));
    const int zb = bzb % nzb, b = bzb / nzb;
    const int ix = bxi * 16 + (tid & 15), iy = byi * 16 + (tid >> 4);
    const int z0 = zb * AT_NZ;
    const bool active = ix < g.nx && iy < g.ny;
    const float fx = (float)ix, fy = (float)iy;
#pragma unroll
    for (int z = 0; z < AT_NZ; ++z)
        accl[z][tid] = 0.0f;

    const float hx = 0.5f * (g.nx - 1), hy = 0.5f * (g.ny - 1), hz = 0.5f * (g.nz - 1);
    // support boxes in centred voxel indices: the brick's (for the table) and
    // this column segment's (for its own loop)
    const int corner = tid & 7;
    const float bcx = (float)((corner & 1) ? min(bxi * 16 + 15, g.nx - 1) + 1 : bxi * 16 - 1) - hx;
    const float bcy = (float)((corner & 2) ? min(byi * 16 + 15, g.ny - 1) + 1 : byi * 16 - 1) - hy;
    const float bcz = (float)((corner & 4) ? min(z0 + AT_NZ - 1, g.nz - 1) + 1 : z0 - 1) - hz;
    const TI *pb = proj + (size_t)b * g.n_proj * g.nv * g.nu;

    for (int k = 0; k < g.n_proj; ++k) {
        const ConeBPView bv = bviews[k];
        const ConeFPView &fv = fviews[k];
        const float rw = rcp_nr(dot4(bv.r[2], bcx, bcy, bcz));
        const float cu = dot4(bv.r[0], bcx, bcy, bcz) * rw, cv = dot4(bv.r[1], bcx, bcy, bcz) * rw;
        const int j_lo = max((int)floorf(min8(cu) + g.cu) - 1, 0), j_hi = min((int)floorf(max8(cu) + g.cu) + 2, g.nu - 1);
        const int i_lo = max((int)floorf(min8(cv) + g.cv) - 1, 0), i_hi = min((int)floorf(max8(cv) + g.cv) + 2, g.nv - 1);
        const int W = j_hi - j_lo + 1, H = i_hi - i_lo + 1;
        const bool staged = W > 0 && H > 0 && W * H <= AT_RAYS;
        const TI *qk = pb + (size_t)k * g.nv * g.nu;
        __syncthreads();   // the previous view's table has been consumed
        if (staged) {
            for (int idx = tid; idx < W * H; idx += 256) {
                const int ii = idx / W, jj = idx - ii * W;
                const Ray r = make_cone_ray(g, fv, j_lo + jj, i_lo + ii);
#pragma unroll
                for (int t = 0; t < 3; ++t) {
                    rtab[t][idx] = r.p[t];
                    rtab[3 + t][idx] = r.e[t];
                }
                rtab[6][idx] = g.step * load_f32(qk + (size_t)(i_lo + ii) * g.nu + (j_lo + jj));
            }
        }
        __syncthreads();
        if (!active || W <= 0 || H <= 0)
            continue;
        // rays crossing this column's support: project its 8 corners
        float umin = 3.0e38f, umax = -3.0e38f, vmin = 3.0e38f, vmax = -3.0e38f;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const float cx = fx + ((c & 1) ? 1.0f : -1.0f) - hx, cy = fy + ((c & 2) ? 1.0f : -1.0f) - hy;
            const float cz = (float)((c & 4) ? min(z0 + AT_NZ - 1, g.nz - 1) + 1 : z0 - 1) - hz;
            const float w = rcp_nr(dot4(bv.r[2], cx, cy, cz));
            const float uu = dot4(bv.r[0], cx, cy, cz) * w, vv = dot4(bv.r[1], cx, cy, cz) * w;
            umin = fminf(umin, uu);
            umax = fmaxf(umax, uu);
            vmin = fminf(vmin, vv);
            vmax = fmaxf(vmax, vv);
        }
        const int ja = max((int)floorf(umin + g.cu) - 1, j_lo), jb = min((int)floorf(umax + g.cu) + 2, j_hi);
        const int ia = max((int)floorf(vmin + g.cv) - 1, i_lo), ib = min((int)floorf(vmax + g.cv) + 2, i_hi);
        const float zlo = (float)(z0 - 1), zhi = (float)min(z0 + AT_NZ, g.nz);
        for (int ii = ia; ii <= ib; ++ii) {
            for (int jj = ja; jj <= jb; ++jj) {
                float X0, Y0, Z0, eX, eY, eZ, gv;
                if (staged) {
                    const int idx = (ii - i_lo) * W + (jj - j_lo);
                    X0 = rtab[0][idx];
                    Y0 = rtab[1][idx];
                    Z0 = rtab[2][idx];
                    eX = rtab[3][idx];
                    eY = rtab[4][idx];
                    eZ = rtab[5][idx];
                    gv = rtab[6][idx];
                } else {
                    const Ray r = make_cone_ray(g, fv, jj, ii);
                    X0 = r.p[0];
                    Y0 = r.p[1];
                    Z0 = r.p[2];
                    eX = r.e[0];
                    eY = r.e[1];
                    eZ = r.e[2];
                    gv = g.step * load_f32(qk + (size_t)ii * g.nu + jj);
                }
                if (gv == 0.0f)
                    continue;
                // the samples that can reach the support: the clip only picks
                // the range to visit (hardware reciprocals, widened by a step
                // on each side); the exact test below decides every sample
                float lo = -3.0e38f, hi = 3.0e38f;
                if (!clip_line_rcp(X0, eX, fx - 1.0f, fx + 1.0f, lo, hi) ||
                    !clip_line_rcp(Y0, eY, fy - 1.0f, fy + 1.0f, lo, hi) || !clip_line_rcp(Z0, eZ, zlo, zhi, lo, hi) ||
                    !(lo < hi + 0.01f))   // reciprocal error is below 1e-3 step at these ranges
                    continue;
                // the projector's biased sample positions, un-biased exactly
                const float Xb = X0 + RAY_BIAS, Yb = Y0 + RAY_BIAS, Zb = Z0 + RAY_BIAS;
                for (int m = (int)floorf(lo) - 1; m <= (int)ceilf(hi) + 1; ++m) {
                    const float X = ray_coord_biased(Xb, eX, m) - RAY_BIAS;
                    const float Y = ray_coord_biased(Yb, eY, m) - RAY_BIAS;
                    const float Z = ray_coord_biased(Zb, eZ, m) - RAY_BIAS;
                    const float w = gv * (1.0f - fabsf(X - fx)) * (1.0f - fabsf(Y - fy));
                    if (!(fabsf(X - fx) < 1.0f && fabsf(Y - fy) < 1.0f))
                        continue;
                    const float fz = floorf(Z);
                    const float tz = Z - fz;
                    const int iz = (int)fz - z0;
                    if (iz >= 0 && iz < AT_NZ)
                        accl[iz][tid] = fmaf(w, 1.0f - tz, accl[iz][tid]);
                    if (iz + 1 >= 0 && iz + 1 < AT_NZ)
                        accl[iz + 1][tid] = fmaf(w, tz, accl[iz + 1][tid]);
                }
            }
        }
    }
    if (!active)
        return;
    T *out = vol + (size_t)b * g.nz * g.ny * g.nx + (size_t)iy * g.nx + ix;
    for (int z = 0; z < AT_NZ && z0 + z < g.nz; ++z)
        store_f32(out + (size_t)(z0 + z) * g.ny * g.nx, accl[z][tid]);
}

// --------------------------------------------------------------- B^T, 2D

__global__ void fill_zero_kernel(float *__restrict__ p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

template <typename TI, bool FAN>
__global__ void __launch_bounds__(256) bpT2d_kernel(Geom2D g, const float2 *__restrict__ views,
                                                    const TI *__restrict__ img, float *__restrict__ sino)
{
    const int ix = blockIdx.x * 16 + (threadIdx.x & 15);
    const int iy = blockIdx.y * 16 + (threadIdx.x >> 4);
    const int b = blockIdx.z;
    if (ix >= g.nx || iy >= g.ny)
        return;
    const float val = load_f32(img + ((size_t)b * g.ny + iy) * g.nx + ix);
    if (val == 0.0f)
        return;
    float *sb = sino + (size_t)b * g.n_proj * g.nu;
    const float x = fmaf((float)ix, g.sx, g.ox), y = fmaf((float)iy, g.sy, g.oy);
    const float rdu = 1.0f / g.du;
    for (int k = 0; k < g.n_proj; ++k) {
        const float2 c = views[k];
        int j;
        float t, wt;
        if (!FAN) {
            const float su = fmaf(-x * c.y + y * c.x, rdu, g.cu);
            const float fu = floorf(su);
            j = (int)fu;
            t = su - fu;
            wt = 1.0f;
        } else {
            fan2d_point(g, c, ix, iy, j, t, wt);
        }
        const float v = g.dbeta * wt * val;
        if (j >= 0 && j < g.nu)
            unsafeAtomicAdd(sb + (size_t)k * g.nu + j, v * (1.0f - t));
        if (j + 1 >= 0 && j + 1 < g.nu)
            unsafeAtomicAdd(sb + (size_t)k * g.nu + j + 1, v * t);
    }
}

template <typename T, typename TI, bool FAN, int S>
hipError_t fpT2d_l(const Geom2D &g, const float2 *views, const void *sino, void *img, long n_pix, hipStream_t s)
{
    const long blocks = (n_pix * S + 255) / 256;
    hipLaunchKernelGGL((fpT2d_kernel<T, TI, FAN, S>), dim3((unsigned)blocks), dim3(256), 0, s, g, views,
                       (const TI *)sino, (T *)img, n_pix);
    return hipGetLastError();
}

template <typename T, typename TI, bool FAN>
hipError_t fpT2d_f(const Geom2D &g, const float2 *views, const void *sino, void *img, long n_pix, hipStream_t s)
{
    // lanes per pixel: about 2^20 threads in all, at most one lane per view
    int S = 1;
    while (S < 64 && 2 * S <= g.n_proj && n_pix * S * 2 <= (1L << 20))
        S *= 2;
    switch (S) {
    case 1: return fpT2d_l<T, TI, FAN, 1>(g, views, sino, img, n_pix, s);
    case 2: return fpT2d_l<T, TI, FAN, 2>(g, views, sino, img, n_pix, s);
    case 4: return fpT2d_l<T, TI, FAN, 4>(g, views, sino, img, n_pix, s);
    case 8: return fpT2d_l<T, TI, FAN, 8>(g, views, sino, img, n_pix, s);
    case 16: return fpT2d_l<T, TI, FAN, 16>(g, views, sino, img, n_pix, s);
    case 32: return fpT2d_l<T, TI, FAN, 32>(g, views, sino, img, n_pix, s);
    default: return fpT2d_l<T, TI, FAN, 64>(g, views, sino, img, n_pix, s);
    }
}

template <typename T, typename TI>
hipError_t fpT2d(bool fan, const Geom2D &g, const float2 *views, const void *sino, void *img, int batch,
                 hipStream_t s)
{
    const long n_pix = (long)g.nx * g.ny * batch;
    return fan ? fpT2d_f<T, TI, true>(g, views, sino, img, n_pix, s)
               : fpT2d_f<T, TI, false>(g, views, sino, img, n_pix, s);
}

template <typename T>
hipError_t fpT_cone(const Geom3D &g, const ConeFPView *fviews, const ConeBPView *bviews, const void *proj, void *vol,
                    int batch, hipStream_t s)
{
    const int nbx = (g.nx + 15) / 16, nby = (g.ny + 15) / 16, nzb = (g.nz + AT_NZ - 1) / AT_NZ;
    hipLaunchKernelGGL((fpT_cone_kernel<T, T>), dim3((unsigned)(nbx * nby * nzb * batch)), dim3(256), 0, s, g, fviews,
                       bviews, (const T *)proj, (T *)vol, nbx, nby, nzb);
    return hipGetLastError();
}

}  // namespace

template <typename T>
__global__ void cast_kernel(const float *__restrict__ in, T *__restrict__ out, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        store_f32(out + i, in[i]);
}

hipError_t launch_cast_from_f32(int dtype, const float *in, void *out, size_t n, hipStream_t s)
{
    const size_t blocks = (n + 255) / 256;
    const dim3 grid((unsigned)(blocks < 4096 ? blocks : 4096));
    switch (dtype) {
    case 1: hipLaunchKernelGGL(cast_kernel<f16_t>, grid, dim3(256), 0, s, in, (f16_t *)out, n); break;
    case 2: hipLaunchKernelGGL(cast_kernel<bf16_t>, grid, dim3(256), 0, s, in, (bf16_t *)out, n); break;
    default: hipLaunchKernelGGL(cast_kernel<float>, grid, dim3(256), 0, s, in, (float *)out, n); break;
    }
    return hipGetLastError();
}

hipError_t fill_zero(float *p, size_t n, hipStream_t s)
{
    const size_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_project_adjoint_2d(int dtype, bool fan, const Geom2D &g, const float2 *views, const void *sino,
                                     void *img, int batch, hipStream_t stream)
{
    switch (dtype) {
    case 0: return fpT2d<float, float>(fan, g, views, sino, img, batch, stream);
    case 1: return fpT2d<f16_t, f16_t>(fan, g, views, sino, img, batch, stream);
    default: return fpT2d<bf16_t, bf16_t>(fan, g, views, sino, img, batch, stream);
    }
}

hipError_t launch_project_adjoint_cone(int dtype, const Geom3D &g, const ConeFPView *fviews,
                                       const ConeBPView *bviews, const void *proj, void *vol, int batch,
                                       hipStream_t stream)
{
    switch (dtype) {
    case 0: return fpT_cone<float>(g, fviews, bviews, proj, vol, batch, stream);
    case 1: return fpT_cone<f16_t>(g, fviews, bviews, proj, vol, batch, stream);
    default: return fpT_cone<bf16_t>(g, fviews, bviews, proj, vol, batch, stream);
    }
}

template <typename TI>
hipError_t bpT2d(bool fan, const Geom2D &g, const float2 *views, const void *img, float *sino, int batch,
                 hipStream_t stream)
{
    dim3 grid((g.nx + 15) / 16, (g.ny + 15) / 16, batch);
    if (fan)
        hipLaunchKernelGGL((bpT2d_kernel<TI, true>), grid, dim3(256), 0, stream, g, views, (const TI *)img, sino);
    else
        hipLaunchKernelGGL((bpT2d_kernel<TI, false>), grid, dim3(256), 0, stream, g, views, (const TI *)img, sino);
    return hipGetLastError();
}

hipError_t launch_backproject_adjoint_2d(int in_dtype, bool fan, const Geom2D &g, const float2 *views,
                                         const void *img, float *sino, int batch, hipStream_t stream)
{
    hipError_t e = fill_zero(sino, (size_t)batch * g.n_proj * g.nu, stream);
    if (e != hipSuccess)
        return e;
    switch (in_dtype) {
    case 0: return bpT2d<float>(fan, g, views, img, sino, batch, stream);
    case 1: return bpT2d<f16_t>(fan, g, views, img, sino, batch, stream);
    default: return bpT2d<bf16_t>(fan, g, views, img, sino, batch, stream);
    }
}

}  // namespace ph
