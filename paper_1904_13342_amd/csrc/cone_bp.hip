// Voxel-driven, distance-weighted cone-beam back-projection from projection
// matrices (Sec. II.B.2; Eq. 5's A^T in the FDK network).
//
// Mapping: a workgroup owns a 16 x 16 x NZ brick of voxels; each thread owns
// one (x, y) column segment of NZ voxels and accumulates it in registers over
// all views, so the volume is written exactly once.  Per view, the brick's
// footprint on the detector (bounded by the projections of its 8 corners,
// plus a one-pixel margin) is staged in LDS with zero outside the detector;
// the bilinear fetches then come from LDS instead of texture units.
//
// For a circular trajectory about z (AXIAL: the matrices have no z term in
// the u and w rows) the column coordinate, the depth w and the weight are
// constant along a column, and only the row coordinate moves with z: one FMA
// per voxel.  General matrices take the per-voxel path.
#include "common.h"

namespace ph {
namespace {

constexpr int BP_TW = 64;  // max staged footprint width (detector columns)
constexpr int BP_TH = 64;  // max staged footprint height (detector rows)

template <typename TI>
__device__ __forceinline__ float det_pix(const TI *q, int nu, int nv, int i, int j)
{
    return (i >= 0 && j >= 0 && i < nv && j < nu) ? load_f32(q + (size_t)i * nu + j) : 0.0f;
}

__device__ __forceinline__ float dot4(const float r[4], float x, float y, float z)
{
    return fmaf(r[0], x, fmaf(r[1], y, fmaf(r[2], z, r[3])));
}

template <typename T, typename TI, int NZ, bool AXIAL>
__global__ void __launch_bounds__(256) bp_cone_kernel(Geom3D g, const ConeBPView *__restrict__ views,
                                                      const TI *__restrict__ proj, T *__restrict__ vol, int nzb)
{
    __shared__ float tile[BP_TH * BP_TW];
    const int tid = threadIdx.x;
    const int ix = blockIdx.x * 16 + (tid & 15);
    const int iy = blockIdx.y * 16 + (tid >> 4);
    const int zb = blockIdx.z % nzb, b = blockIdx.z / nzb;
    const int z0 = zb * NZ;
    const int zcount = min(NZ, g.nz - z0);
    const bool active = ix < g.nx && iy < g.ny;

    const float hx = 0.5f * (g.nx - 1), hy = 0.5f * (g.ny - 1), hz = 0.5f * (g.nz - 1);
    const float xc = (float)ix - hx, yc = (float)iy - hy, zc0 = (float)z0 - hz;
    // brick corners (centred voxel indices), clamped to the grid
    const float bx0 = (float)(blockIdx.x * 16) - hx, bx1 = (float)min(blockIdx.x * 16 + 15, g.nx - 1) - hx;
    const float by0 = (float)(blockIdx.y * 16) - hy, by1 = (float)min(blockIdx.y * 16 + 15, g.ny - 1) - hy;
    const float bz0 = zc0, bz1 = zc0 + (float)(zcount - 1);

    const TI *pb = proj + (size_t)b * g.n_proj * g.nv * g.nu;
    float acc[NZ];
#pragma unroll
    for (int z = 0; z < NZ; ++z)
        acc[z] = 0.0f;

    for (int k = 0; k < g.n_proj; ++k) {
        ConeBPView v = views[k];
        // footprint of the brick: extreme detector coordinates over the corners
        float umin = 3.0e38f, umax = -3.0e38f, vmin = 3.0e38f, vmax = -3.0e38f;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const float cx = (c & 1) ? bx1 : bx0, cy = (c & 2) ? by1 : by0, cz = (c & 4) ? bz1 : bz0;
            const float rw = 1.0f / dot4(v.r[2], cx, cy, cz);
            const float uu = dot4(v.r[0], cx, cy, cz) * rw, vv = dot4(v.r[1], cx, cy, cz) * rw;
            umin = fminf(umin, uu);
            umax = fmaxf(umax, uu);
            vmin = fminf(vmin, vv);
            vmax = fmaxf(vmax, vv);
        }
        const int u_lo = (int)floorf(umin + g.cu) - 1, u_hi = (int)floorf(umax + g.cu) + 2;
        const int v_lo = (int)floorf(vmin + g.cv) - 1, v_hi = (int)floorf(vmax + g.cv) + 2;
        const int tw = u_hi - u_lo + 1, th = v_hi - v_lo + 1;
        const bool staged = tw <= BP_TW && th <= BP_TH;
        const TI *qk = pb + (size_t)k * g.nv * g.nu;
        if (staged) {
            __syncthreads();
            for (int idx = tid; idx < tw * th; idx += 256) {
                const int r = idx / tw, c = idx - r * tw;
                tile[r * BP_TW + c] = det_pix(qk, g.nu, g.nv, v_lo + r, u_lo + c);
            }
            __syncthreads();
        }
        if (!active)
            continue;
        if (AXIAL) {
            const float W = dot4(v.r[2], xc, yc, zc0);
            const float rW = 1.0f / W;
            const float sw = g.sid * rW, wt = sw * sw;
            const float uc = dot4(v.r[0], xc, yc, zc0) * rW;
            const float vc0 = dot4(v.r[1], xc, yc, zc0) * rW;
            const float dvz = v.r[1][2] * rW;
            if (staged) {
                const float su = uc + g.cu - (float)u_lo;
                const float sv0 = vc0 + g.cv - (float)v_lo;
                const int iu = (int)su;
                const float fu = su - (float)iu;
                const float *col = tile + iu;
#pragma unroll
                for (int z = 0; z < NZ; ++z) {
                    if (z < zcount) {
                        const float sv = fmaf((float)z, dvz, sv0);
                        const int iv = (int)sv;
                        const float fv = sv - (float)iv;
                        const float *p = col + iv * BP_TW;
                        const float p00 = p[0], p01 = p[1], p10 = p[BP_TW], p11 = p[BP_TW + 1];
                        const float a0 = fmaf(fu, p01 - p00, p00), a1 = fmaf(fu, p11 - p10, p10);
                        acc[z] = fmaf(wt, fmaf(fv, a1 - a0, a0), acc[z]);
                    }
                }
            } else {
                const float su = uc + g.cu;
                const float fsu = floorf(su);
                const int j = (int)fsu;
                const float fu = su - fsu;
                const float sv0 = vc0 + g.cv;
#pragma unroll
                for (int z = 0; z < NZ; ++z) {
                    if (z < zcount) {
                        const float sv = fmaf((float)z, dvz, sv0);
                        const float fsv = floorf(sv);
                        const int i = (int)fsv;
                        const float fv = sv - fsv;
                        const float p00 = det_pix(qk, g.nu, g.nv, i, j), p01 = det_pix(qk, g.nu, g.nv, i, j + 1);
                        const float p10 = det_pix(qk, g.nu, g.nv, i + 1, j);
                        const float p11 = det_pix(qk, g.nu, g.nv, i + 1, j + 1);
                        const float a0 = fmaf(fu, p01 - p00, p00), a1 = fmaf(fu, p11 - p10, p10);
                        acc[z] = fmaf(wt, fmaf(fv, a1 - a0, a0), acc[z]);
                    }
                }
            }
        } else {
#pragma unroll
            for (int z = 0; z < NZ; ++z) {
                if (z < zcount) {
                    const float zc = zc0 + (float)z;
                    const float rW = 1.0f / dot4(v.r[2], xc, yc, zc);
                    const float sw = g.sid * rW, wt = sw * sw;
                    float su = dot4(v.r[0], xc, yc, zc) * rW + g.cu;
                    float sv = dot4(v.r[1], xc, yc, zc) * rW + g.cv;
                    if (staged) {
                        su -= (float)u_lo;
                        sv -= (float)v_lo;
                        const int iu = (int)su, iv = (int)sv;
                        const float fu = su - (float)iu, fv = sv - (float)iv;
                        const float *p = tile + iv * BP_TW + iu;
                        const float p00 = p[0], p01 = p[1], p10 = p[BP_TW], p11 = p[BP_TW + 1];
                        const float a0 = fmaf(fu, p01 - p00, p00), a1 = fmaf(fu, p11 - p10, p10);
                        acc[z] = fmaf(wt, fmaf(fv, a1 - a0, a0), acc[z]);
                    } else {
                        const float fsu = floorf(su), fsv = floorf(sv);
                        const int j = (int)fsu, i = (int)fsv;
                        const float fu = su - fsu, fv = sv - fsv;
                        const float p00 = det_pix(qk, g.nu, g.nv, i, j), p01 = det_pix(qk, g.nu, g.nv, i, j + 1);
                        const float p10 = det_pix(qk, g.nu, g.nv, i + 1, j);
                        const float p11 = det_pix(qk, g.nu, g.nv, i + 1, j + 1);
                        const float a0 = fmaf(fu, p01 - p00, p00), a1 = fmaf(fu, p11 - p10, p10);
                        acc[z] = fmaf(wt, fmaf(fv, a1 - a0, a0), acc[z]);
                    }
                }
            }
        }
    }
    if (!active)
        return;
    T *out = vol + (size_t)b * g.nz * g.ny * g.nx + (size_t)iy * g.nx + ix;
#pragma unroll
    for (int z = 0; z < NZ; ++z)
        if (z < zcount)
            store_f32(out + (size_t)(z0 + z) * g.ny * g.nx, g.dbeta * acc[z]);
}

template <typename T, typename TI>
hipError_t bp_cone(const Geom3D &g, const ConeBPView *views, bool axial, const void *proj, void *vol, int batch,
                   hipStream_t s)
{
    constexpr int NZ = 16;
    const int nzb = (g.nz + NZ - 1) / NZ;
    dim3 grid((g.nx + 15) / 16, (g.ny + 15) / 16, nzb * batch);
    if (axial)
        hipLaunchKernelGGL((bp_cone_kernel<T, TI, NZ, true>), grid, dim3(256), 0, s, g, views, (const TI *)proj,
                           (T *)vol, nzb);
    else
        hipLaunchKernelGGL((bp_cone_kernel<T, TI, NZ, false>), grid, dim3(256), 0, s, g, views, (const TI *)proj,
                           (T *)vol, nzb);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_backproject_cone(int dtype, const Geom3D &g, const ConeBPView *views, bool axial,
                                   const void *proj, bool proj_is_f32, void *vol, int batch, hipStream_t stream)
{
    switch (dtype) {
    case 0: return bp_cone<float, float>(g, views, axial, proj, vol, batch, stream);
    case 1:
        return proj_is_f32 ? bp_cone<f16_t, float>(g, views, axial, proj, vol, batch, stream)
                           : bp_cone<f16_t, f16_t>(g, views, axial, proj, vol, batch, stream);
    default:
        return proj_is_f32 ? bp_cone<bf16_t, float>(g, views, axial, proj, vol, batch, stream)
                           : bp_cone<bf16_t, bf16_t>(g, views, axial, proj, vol, batch, stream);
    }
}

}  // namespace ph
