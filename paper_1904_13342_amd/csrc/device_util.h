// Device helpers shared by the projector, back-projector and adjoint kernels.
#pragma once

#include "common.h"

namespace ph {

// Index coordinates (x, y, z) of a ray's anchor (its point closest to the
// isocentre) and of one sampling step: sample m sits at p + m * e.
struct Ray {
    float p[3], e[3];
};

// Ray of cone-beam detector pixel (j, i), set up in double precision (the
// source is ~SID away, so an FP32 direction would misplace the ray by
// ~SID * 2^-24 at the volume) and rounded once to FP32.  The direction is
// normalised with the hardware reciprocal square root refined by two Newton
// steps, and the per-view reciprocals of the spacing replace divisions, so
// the set-up takes a few dozen double-precision operations.  The forward
// projector and its transpose both use this, so they see the same samples.
__device__ __forceinline__ Ray make_cone_ray(const Geom3D &g, const ConeFPView &v, int j, int i)
{
    const double jc = (double)j - (double)g.cu, ic = (double)i - (double)g.cv;
    double d[3];
#pragma unroll
    for (int t = 0; t < 3; ++t)
        d[t] = fma(jc, v.du[t], fma(ic, v.dv[t], v.d0[t]));
    const double n2 = fma(d[0], d[0], fma(d[1], d[1], d[2] * d[2]));
    const double h = 0.5 * n2;
    double rn = __builtin_amdgcn_rsq(n2);
    rn = rn * fma(-h * rn, rn, 1.5);
    rn = rn * fma(-h * rn, rn, 1.5);
#pragma unroll
    for (int t = 0; t < 3; ++t)
        d[t] *= rn;
    const double t0 = -(v.s[0] * d[0] + v.s[1] * d[1] + v.s[2] * d[2]);
    const double o[3] = {g.ox, g.oy, g.oz};
    Ray r;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        r.p[t] = (float)((fma(t0, d[t], v.s[t]) - o[t]) * v.inv_sp[t]);
        r.e[t] = (float)(d[t] * v.step_sp[t]);
    }
    return r;
}

// Sample positions of cone rays are evaluated around a +4 bias on every axis
// (biased coordinates stay positive, so the slab walk can floor by
// truncation); un-biasing is exact (subtracting 4 from a float in [4, 2^20)).
// Every kernel that visits cone samples uses this one expression, so the
// projector and its transpose see bitwise the same positions.
constexpr float RAY_BIAS = 4.0f;

__device__ __forceinline__ float ray_coord_biased(float p_biased, float e, int m)
{
    return fmaf((float)m, e, p_biased);
}

// Ray of 2D detector bin j in a view with central ray vector c: index
// coordinates (x, y) of its anchor and of one step (fan rays set up in double
// precision for the same reason as cone rays).  On the equiangular detector
// bin j sits at fan angle u / SDD on the arc of radius SDD about the source,
// so its ray is the central ray turned by that angle.
template <bool FAN>
__device__ __forceinline__ void make_ray_2d(const Geom2D &g, float2 c, int j, float &X0, float &Y0, float &eX,
                                            float &eY)
{
    const double cx = c.x, cy = c.y, ex = -cy, ey = cx;
    const double u = ((double)j - (double)g.cu) * (double)g.du;
    double ax, ay, dx, dy;
    if (!FAN) {
        ax = u * ex;
        ay = u * ey;
        dx = cx;
        dy = cy;
    } else if (g.curved) {
        const double gam = u / (double)g.sdd, cg = cos(gam), sg = sin(gam);
        const double sx = -(double)g.sid * cx, sy = -(double)g.sid * cy;
        dx = cg * cx + sg * ex;
        dy = cg * cy + sg * ey;
        const double t0 = -(sx * dx + sy * dy);
        ax = fma(t0, dx, sx);
        ay = fma(t0, dy, sy);
    } else {
        const double sx = -(double)g.sid * cx, sy = -(double)g.sid * cy;
        const double tx = (double)g.sdd * cx + u * ex, ty = (double)g.sdd * cy + u * ey;  // detector - source
        const double rn = 1.0 / sqrt(tx * tx + ty * ty);
        dx = tx * rn;
        dy = ty * rn;
        const double t0 = -(sx * dx + sy * dy);
        ax = fma(t0, dx, sx);
        ay = fma(t0, dy, sy);
    }
    X0 = (float)((ax - (double)g.ox) / (double)g.sx);
    Y0 = (float)((ay - (double)g.oy) / (double)g.sy);
    eX = (float)((double)g.step * dx / (double)g.sx);
    eY = (float)((double)g.step * dy / (double)g.sy);
}

// Detector bin j, fraction t in [0, 1) and distance weight of pixel (ix, iy)
// in a fan view with central ray c: central projection onto the flat detector
// with weight (SID / w)^2, w the depth along the central ray; on the
// equiangular detector the bin of the pixel's fan angle, with weight
// (SID / L)^2, L the distance from the source.  All in FP32: the arctangent
// places a wide fan's samples to a few 1e-6 bin.  The back-projector and its
// transpose both use this, so they see the same coordinates.
__device__ __forceinline__ void fan2d_point(const Geom2D &g, float2 c, int ix, int iy, int &j, float &t, float &wt)
{
    if (g.curved) {
        const float x = fmaf((float)ix, g.sx, g.ox), y = fmaf((float)iy, g.sy, g.oy);
        const float xu = -x * c.y + y * c.x;
        const float w = fmaf(x, c.x, fmaf(y, c.y, g.sid));
        const float s = fmaf(atan2f(xu, w), g.sdd / g.du, g.cu);
        const float fs = floorf(s);
        j = (int)fs;
        t = s - fs;
        wt = g.sid * g.sid / fmaf(w, w, xu * xu);
    } else {
        const float x = fmaf((float)ix, g.sx, g.ox), y = fmaf((float)iy, g.sy, g.oy);
        const float xu = -x * c.y + y * c.x;
        const float w = fmaf(x, c.x, fmaf(y, c.y, g.sid));
        const float rw = 1.0f / w;
        const float su = fmaf(g.sdd * xu * rw, 1.0f / g.du, g.cu);
        const float fu = floorf(su);
        j = (int)fu;
        t = su - fu;
        const float sw = g.sid * rw;
        wt = sw * sw;
    }
}

// Narrow [lo, hi] to the parameters t with p + t e inside the open interval
// (a, b); false if the line never enters it.
__device__ __forceinline__ bool clip_line(float p, float e, float a, float b, float &lo, float &hi)
{
    if (fabsf(e) < 1e-30f)
        return p > a && p < b;
    const float t1 = (a - p) / e, t2 = (b - p) / e;
    lo = fmaxf(lo, fminf(t1, t2));
    hi = fminf(hi, fmaxf(t1, t2));
    return true;
}

// clip_line with the hardware reciprocal in place of the divisions: the
// bounds may be off by a few ulps, so callers widen the range they derive and
// test each sample exactly.
__device__ __forceinline__ bool clip_line_rcp(float p, float e, float a, float b, float &lo, float &hi)
{
    if (fabsf(e) < 1e-30f)
        return p > a && p < b;
    const float r = __builtin_amdgcn_rcpf(e);
    const float t1 = (a - p) * r, t2 = (b - p) * r;
    lo = fmaxf(lo, fminf(t1, t2));
    hi = fminf(hi, fmaxf(t1, t2));
    return true;
}

__device__ __forceinline__ float dot4(const float r[4], float x, float y, float z)
{
    return fmaf(r[0], x, fmaf(r[1], y, fmaf(r[2], z, r[3])));
}

// 1/x from the hardware estimate refined by one Newton step
__device__ __forceinline__ float rcp_nr(float x)
{
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// nearest integer of x (ties toward +inf) in one instruction; the
// fixed-point LDS accumulators of the transposes round every term with it
__device__ __forceinline__ int round_to_int(float x)
{
    int r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

template <int CTRL>
__device__ __forceinline__ float dpp(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// min / max over the 8 corners held by lanes with corner index lane mod 8:
// xor 1 and xor 2 within quads, then rotate each 16-lane row by 4 lanes,
// which pairs a quad holding corners 0-3 with one holding corners 4-7.
__device__ __forceinline__ float min8(float x)
{
    x = fminf(x, dpp<0xB1>(x));
    x = fminf(x, dpp<0x4E>(x));
    return fminf(x, dpp<0x124>(x));
}
__device__ __forceinline__ float max8(float x)
{
    x = fmaxf(x, dpp<0xB1>(x));
    x = fmaxf(x, dpp<0x4E>(x));
    return fmaxf(x, dpp<0x124>(x));
}

// the same over integers (no NaN handling, so each step is one DPP min/max)
template <int CTRL>
__device__ __forceinline__ int dppi(int x)
{
    return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ int imin8(int x)
{
    x = min(x, dppi<0xB1>(x));
    x = min(x, dppi<0x4E>(x));
    return min(x, dppi<0x124>(x));
}
__device__ __forceinline__ int imax8(int x)
{
    x = max(x, dppi<0xB1>(x));
    x = max(x, dppi<0x4E>(x));
    return max(x, dppi<0x124>(x));
}

}  // namespace ph
