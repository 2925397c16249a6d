// Exact transposes of the two operators (Sec. II.B.2 notes that the
// ray-driven projector and the voxel-driven back-projector are an unmatched
// pair; Eq. 4 and Sec. II.B.1 use A^T as A's gradient operator).
//
// A^T, the transpose of the fixed-step multilinear ray sampler: voxel j
// receives
//     step * sum_r g_r * sum_k Lambda(X_rk - j),
// Lambda the tensor-product hat function, X_rk the same FP32 sample positions
// the forward projector uses.  In 2D a thread owns a pixel and gathers, per
// view, over the rays that cross its support (j - 1, j + 1)^2, without
// atomics.  In 3D a workgroup owns a brick and its rays splat into an LDS
// accumulator (below).
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
//
// A workgroup owns a 16 x 16 x 16 brick of voxels; each thread holds the
// FP64 sums of one 16-voxel z-column of it in registers, over every view.
// Per view, the rays that can reach the brick's support box (the detector
// pixels of its footprint: 8 corners projected by eight lanes and reduced with
// DPP) are set up exactly as the forward projector sets them up (FP64 set-up,
// the same biased FP32 sample positions, so the pair is transposed sample for
// sample) and clipped to the support box.  The rays are then counting-sorted
// by their number of samples, so the 64 rays a wave walks together have
// nearly equal lengths, and each lane walks one ray, splatting every sample's
// eight trilinear corner weights into an LDS accumulator.
//
// The accumulator holds 32-bit fixed-point integers (u32 LDS atomics issue
// in about half the time of FP64 ones, and integer sums are exact, so the
// result does not depend on the order of the adds).  The scale of a pass is
// set from its own rays: a sample's weight at one cell is at most 1, and the
// samples of one ray add at most 1 / e_max + 1 at a cell (e_max its largest
// per-step index increment), so no cell's sum exceeds
//     bound = sum over rays of |g_r| (1 / e_max,r + 1),
// and with scale = 2^30 / bound no cell can overflow.  Each corner term is
// rounded to the nearest integer; after the pass every thread adds its own
// cells, divided by the scale, to its FP64 sums and clears them.  The waves
// take the sorted rays in tasks of 64 from a shared counter, longest first.  Cells of
// the two-voxel halo are never read (the neighbouring bricks own those
// voxels), so they need no clearing and may wrap.
//
// Sample ranges come from a clip with hardware reciprocals (relative error
// ~1e-7 of a few thousand steps), widened by 0.01 step: every sample inside
// the support box is visited, and a visited sample lies at most 0.01 step
// outside it, so its cell stays inside the padded accumulator
// (floor coordinates x0 - 2 .. x0 + 17).  Its rows and planes have odd
// pitches: the rays of a wave, sorted by length, often sit at one x at the
// same step, and even pitches would put their cells on a quarter of the
// banks.

constexpr int AT_B = 16;                       // brick edge (voxels)
constexpr int AT_P = AT_B + 4;                 // accumulator edge (cells)
constexpr int AT_PY = AT_P + 1;                // row pitch (words)
constexpr int AT_PZ = AT_P * AT_PY + 1;        // plane pitch (words)
constexpr int AT_CELLS = AT_P * AT_PZ;
constexpr int AT_RAYS = 536;                   // footprint pixels per pass (ray-table capacity; with the
                                               // accumulator, three workgroups fit a CU's LDS)
constexpr int AT_PER_THREAD = (AT_RAYS + 255) / 256;
constexpr int AT_BINS = 256;                   // sample-count bins of the ray sort
constexpr float AT_EPS = 0.01f;                // clip widening (steps)
constexpr float AT_FIX = 1073741824.0f;        // 2^30

template <typename T, typename TI>
__global__ void __launch_bounds__(256) fpT_cone_kernel(Geom3D g, const ConeFPView *__restrict__ fviews,
                                                       const ConeBPView *__restrict__ bviews,
                                                       const TI *__restrict__ proj, T *__restrict__ vol, int nbx,
                                                       int nby, int nbz)
{
    __shared__ int acc[AT_CELLS];
    __shared__ float4 s_ra[AT_RAYS];   // biased anchor X, Y, Z and the ray's value
    __shared__ float4 s_rb[AT_RAYS];   // step e_x, e_y, e_z and the first sample (int bits)
    __shared__ int s_cnt[AT_RAYS];
    __shared__ int hist[AT_BINS];
    __shared__ int s_wsum[4];
    __shared__ float s_wbound[4];
    __shared__ int s_nhit;
    __shared__ int s_next;   // next 64-ray task of the walk
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int bxi = (int)(blockIdx.x % (unsigned)nbx), byi = (int)((blockIdx.x / (unsigned)nbx) % (unsigned)nby);
    const int bzb = (int)(blockIdx.x / (unsigned)(nbx * nby));
    const int bzi = bzb % nbz, b = bzb / nbz;
    const int x0 = bxi * AT_B, y0 = byi * AT_B, z0 = bzi * AT_B;
    for (int n = tid; n < AT_CELLS; n += 256)
        acc[n] = 0;
    hist[tid] = 0;
    if (tid == 0)
        s_next = 0;
    // this thread's voxel column (x0 + lx, y0 + ly, z0 .. z0 + 15) and its cells
    const int lx = tid % AT_B, ly = tid / AT_B;
    const int own = 2 * AT_PZ + (ly + 2) * AT_PY + lx + 2;   // cell of (lx, ly, 0); + AT_PZ per z
    double out[AT_B];
#pragma unroll
    for (int z = 0; z < AT_B; ++z)
        out[z] = 0.0;
    __syncthreads();

    const float hx = 0.5f * (g.nx - 1), hy = 0.5f * (g.ny - 1), hz = 0.5f * (g.nz - 1);
    // support box of the brick's voxels, (x0 - 1, min(x0 + B, N)) per axis:
    // inside the grid's support (-1, N), which the host has checked lies in
    // front of every source
    const int xe = min(x0 + AT_B, g.nx), ye = min(y0 + AT_B, g.ny), ze = min(z0 + AT_B, g.nz);
    // this lane's corner of the support box in centred voxel indices
    const int corner = tid & 7;
    const float bcx = (float)((corner & 1) ? xe : x0 - 1) - hx;
    const float bcy = (float)((corner & 2) ? ye : y0 - 1) - hy;
    const float bcz = (float)((corner & 4) ? ze : z0 - 1) - hz;
    // the same box in (unbiased) index coordinates, for the clip
    const float sx0 = (float)(x0 - 1), sx1 = (float)xe;
    const float sy0 = (float)(y0 - 1), sy1 = (float)ye;
    const float sz0 = (float)(z0 - 1), sz1 = (float)ze;
    // biased floor coordinate -> accumulator cell: floor(X) - (x0 - 2) = (int)(X + 4) - (x0 + 2);
    // the cell's byte address is 4 (iz PZ + iy PY + ix) + base (modulo 2^32)
    const unsigned base = 0u - 4u * (unsigned)((z0 + 2) * AT_PZ + (y0 + 2) * AT_PY + (x0 + 2));
    const TI *pb = proj + (size_t)b * g.n_proj * g.nv * g.nu;

    for (int k = 0; k < g.n_proj; ++k) {
        const ConeBPView bv = bviews[k];
        const float rw = rcp_nr(dot4(bv.r[2], bcx, bcy, bcz));
        const float cu = dot4(bv.r[0], bcx, bcy, bcz) * rw, cv = dot4(bv.r[1], bcx, bcy, bcz) * rw;
        // the corners' floors reduced as integers (floor is monotonic); the
        // sums are rounded on their own, not fused with the products above
        const int ju = (int)floorf(__fadd_rn(cu, g.cu)), iv = (int)floorf(__fadd_rn(cv, g.cv));
        const int j_lo = max(imin8(ju) - 1, 0), j_hi = min(imax8(ju) + 2, g.nu - 1);
        const int i_lo = max(imin8(iv) - 1, 0), i_hi = min(imax8(iv) + 2, g.nv - 1);
        const int W = j_hi - j_lo + 1, H = i_hi - i_lo + 1;
        if (W <= 0 || H <= 0)
            continue;
        const ConeFPView &fv = fviews[k];
        const TI *qk = pb + (size_t)k * g.nv * g.nu;
        const int nfp = W * H;
        for (int c0 = 0; c0 < nfp; c0 += AT_RAYS) {
            const int nc = min(AT_RAYS, nfp - c0);
            // set-up: this thread's footprint pixels of the pass
            float4 ra[AT_PER_THREAD], rb[AT_PER_THREAD];
            int cnt[AT_PER_THREAD];
            float lb = 0.0f;   // this thread's share of the bound
#pragma unroll
            for (int u = 0; u < AT_PER_THREAD; ++u) {
                cnt[u] = 0;
                const int idx = tid + 256 * u;
                if (idx >= nc)
                    continue;
                const int f = c0 + idx, ii = f / W, jj = f - ii * W;
                const int i = i_lo + ii, j = j_lo + jj;
                const float gv = load_f32(qk + (size_t)i * g.nu + j);
                if (gv == 0.0f)
                    continue;
                const Ray r = make_cone_ray(g, fv, j, i);
                float lo = -3.0e38f, hi = 3.0e38f;
                if (!clip_line_rcp(r.p[0], r.e[0], sx0, sx1, lo, hi) ||
                    !clip_line_rcp(r.p[1], r.e[1], sy0, sy1, lo, hi) ||
                    !clip_line_rcp(r.p[2], r.e[2], sz0, sz1, lo, hi) || !(lo < hi + 2.0f * AT_EPS))
                    continue;
                const int m0 = (int)ceilf(lo - AT_EPS), m1 = (int)floorf(hi + AT_EPS);
                if (m1 < m0)
                    continue;
                cnt[u] = m1 - m0 + 1;
                ra[u] = make_float4(r.p[0] + RAY_BIAS, r.p[1] + RAY_BIAS, r.p[2] + RAY_BIAS, gv);
                rb[u] = make_float4(r.e[0], r.e[1], r.e[2], __int_as_float(m0));
                const float emax = fmaxf(fabsf(r.e[0]), fmaxf(fabsf(r.e[1]), fabsf(r.e[2])));
                // 1 / e_max + 1, rounded up by a relative 1e-5 (the hardware reciprocal is within 1 ulp)
                lb = fmaf(fabsf(gv), fmaf(__builtin_amdgcn_rcpf(emax), 1.00001f, 1.00001f), lb);
                atomicAdd(&hist[min(cnt[u], AT_BINS - 1)], 1);
            }
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1)
                lb += __shfl_xor(lb, o);
            if (lane == 0)
                s_wbound[wave] = lb;
            __syncthreads();
            // slots in descending order of sample count: bin AT_BINS - 1 - tid
            // starts after the rays of all longer bins
            {
                const int bin = AT_BINS - 1 - tid;
                const int v = hist[bin];
                int x = v;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const int y = __shfl_up(x, o);
                    if (lane >= o)
                        x += y;
                }
                if (lane == 63)
                    s_wsum[wave] = x;
                __syncthreads();
                int off = 0;
                for (int w = 0; w < wave; ++w)
                    off += s_wsum[w];
                hist[bin] = off + x - v;
                if (tid == 255)
                    s_nhit = off + x;
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < AT_PER_THREAD; ++u) {
                if (cnt[u] > 0) {
                    const int slot = atomicAdd(&hist[min(cnt[u], AT_BINS - 1)], 1);
                    s_ra[slot] = ra[u];
                    s_rb[slot] = rb[u];
                    s_cnt[slot] = cnt[u];
                }
            }
            __syncthreads();
            const int nhit = s_nhit;
            // summed in a fixed order: the result does not depend on the waves' timing
            const float bound = (s_wbound[0] + s_wbound[1]) + (s_wbound[2] + s_wbound[3]);
            if (nhit > 0) {   // uniform
                const float scale = AT_FIX / bound;
                // the waves take 64-ray tasks in order of decreasing ray length
                for (;;) {
                    int t = 0;
                    if (lane == 0)
                        t = atomicAdd(&s_next, 1);
                    const int slot = __builtin_amdgcn_readfirstlane(t) * 64 + lane;
                    if (slot - lane >= nhit)
                        break;
                    if (slot >= nhit)
                        continue;
                    const float4 A = s_ra[slot], E = s_rb[slot];
                    const float gs = A.w * scale;
                    float fm = (float)__float_as_int(E.w);
                    const float fend = fm + (float)s_cnt[slot];
                    for (; fm < fend; fm += 1.0f) {
                        // the projector's biased sample position (positive: near the support box)
                        const float X = fmaf(fm, E.x, A.x), Y = fmaf(fm, E.y, A.y), Z = fmaf(fm, E.z, A.z);
                        const unsigned ix = (unsigned)X, iy = (unsigned)Y, iz = (unsigned)Z;
                        const float tx = __builtin_amdgcn_fractf(X), ty = __builtin_amdgcn_fractf(Y),
                                    tz = __builtin_amdgcn_fractf(Z);
                        unsigned off = 4u * (__umul24(iz, AT_PZ) + __umul24(iy, AT_PY) + ix) + base;
                        // the finished offset goes into one register, so the eight corners take
                        // immediate offsets (otherwise the constant part is split off per corner)
                        asm("" : "+v"(off));
                        int *c = (int *)((char *)acc + off);
                        const float a1 = gs * tz, a0 = gs - a1;
                        const float a01 = a0 * ty, a00 = a0 - a01, a11 = a1 * ty, a10 = a1 - a11;
                        // corner terms in fixed point, rounded to the nearest integer
                        atomicAdd(c, round_to_int(fmaf(-a00, tx, a00)));
                        atomicAdd(c + 1, round_to_int(a00 * tx));
                        atomicAdd(c + AT_PY, round_to_int(fmaf(-a01, tx, a01)));
                        atomicAdd(c + AT_PY + 1, round_to_int(a01 * tx));
                        atomicAdd(c + AT_PZ, round_to_int(fmaf(-a10, tx, a10)));
                        atomicAdd(c + AT_PZ + 1, round_to_int(a10 * tx));
                        atomicAdd(c + AT_PZ + AT_PY, round_to_int(fmaf(-a11, tx, a11)));
                        atomicAdd(c + AT_PZ + AT_PY + 1, round_to_int(a11 * tx));
                    }
                }
                __syncthreads();
                // fold this thread's cells into its FP64 sums and clear them
                const double inv = 1.0 / (double)scale;
#pragma unroll
                for (int z = 0; z < AT_B; ++z) {
                    const int n = own + z * AT_PZ;
                    out[z] = fma((double)acc[n], inv, out[z]);
                    acc[n] = 0;
                }
            }
            hist[tid] = 0;
            if (tid == 0)
                s_next = 0;
            __syncthreads();
        }
    }
    // write the brick's own voxels
    const size_t plane = (size_t)g.nx * g.ny;
    T *vb = vol + (size_t)b * g.nz * plane;
    const int ix = x0 + lx, iy = y0 + ly;
    if (ix < g.nx && iy < g.ny) {
#pragma unroll
        for (int z = 0; z < AT_B; ++z)
            if (z0 + z < g.nz)
                store_f32(vb + (size_t)(z0 + z) * plane + (size_t)iy * g.nx + ix, (float)((double)g.step * out[z]));
    }
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
    const int nbx = (g.nx + AT_B - 1) / AT_B, nby = (g.ny + AT_B - 1) / AT_B, nbz = (g.nz + AT_B - 1) / AT_B;
    const long blocks = (long)nbx * nby * nbz * batch;
    if (blocks > 0x7fffffffL)
        return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((fpT_cone_kernel<T, T>), dim3((unsigned)blocks), dim3(256), 0, s, g, fviews, bviews,
                       (const T *)proj, (T *)vol, nbx, nby, nbz);
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
