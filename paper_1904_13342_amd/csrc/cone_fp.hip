// Ray-driven cone-beam forward projection from projection matrices
// (Sec. II.B.2, after Galigekere et al.): one thread per detector pixel; the
// ray from the source through the pixel is sampled at fixed steps on the
// lattice anchored at its point closest to the isocentre, and the volume is
// interpolated trilinearly with zero outside the grid.
//
// Mapping: a workgroup owns a 16 x 16 detector tile of one view.  Its rays
// form a thin pyramid from the source and all advance along one horizontal
// axis A (x or y, chosen per tile from its corner rays).  The volume is walked
// in slabs of D planes across A; for each slab the cross-section of the
// pyramid (bounded by the tile's four corner rays, plus a one-voxel margin,
// clipped to the grid and a two-voxel zero halo) is staged in LDS, and every
// ray then takes the samples whose floor(A coordinate) falls in the slab,
// with all eight trilinear corners read from LDS.  A sample belongs to
// exactly one slab, decided by the same FP32 coordinate the interpolation
// uses.  Slabs that do not fit in LDS read the volume directly.
#include "device_util.h"

namespace ph {
namespace {

constexpr int FP_TILE = 16;            // detector tile edge (pixels)
constexpr int FP_D = 6;                // slab depth (planes along A; D + 1 odd keeps LDS rows off shared banks)
constexpr int FP_WA = FP_D + 1;        // planes held per slab
constexpr int FP_LDS_FLOATS = 6400;    // 25 KiB slab capacity (with the boxes: six workgroups per CU)
constexpr int FP_HALF = FP_LDS_FLOATS / 2;   // one buffer of the double-buffered pair
constexpr int FP_BIAS = (int)RAY_BIAS;  // biased coordinates stay positive (floor == truncation)
constexpr int FP_VG = 12;              // views of one tile scheduled together (measured: 4-36)
constexpr int FP_XCDS = 8;             // accelerator complex dies, each with its own L2
constexpr int FP_BOXES = 32;           // slab cross-sections computed per batch (ring of two batches)

template <typename T>
__device__ __forceinline__ float vox(const T *f, int nx, int ny, int nz, int ix, int iy, int iz)
{
    return ((unsigned)ix < (unsigned)nx && (unsigned)iy < (unsigned)ny && (unsigned)iz < (unsigned)nz)
               ? load_f32(f + ((size_t)iz * ny + iy) * nx + ix)
               : 0.0f;
}

// Raw buffer reads of the slab staging: the descriptor holds the base of a
// run of z planes (word 3 is the gfx9 raw-buffer format), the lane's byte
// offset within a plane goes in a VGPR and the plane's byte offset in an SGPR,
// so a load costs no vector address arithmetic.  Every offset used stays
// below the descriptor's record count.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_run(const void *base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
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
__device__ __forceinline__ float sample_global(const T *f, const Geom3D &g, float X, float Y, float Z)
{
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
    return fmaf(tz, c[1] - c[0], c[0]);
}

// Whether sample m (biased A coordinate fma(m, eA, PA0)) lies in the slab
// whose first biased plane is offA.
__device__ __forceinline__ bool in_slab(int m, float eA, float PA0, int offA)
{
    return (unsigned)((int)fmaf((float)m, eA, PA0) - offA) < (unsigned)FP_D;
}

// Trilinear sample at (float) index fm from the LDS slab ([c][b][a], a
// fastest).  Biased coordinates are positive, so truncation is floor; the
// cell's byte offset is formed with 24-bit multiplies (every factor is below
// 2^24), and `base` folds the slab's offsets in (bytes, modulo 2^32).
__device__ __forceinline__ float sample_lds(const float *slab, float fm, float PA0, float eA, float PB0, float eB,
                                            float PC0, float eC, unsigned base, unsigned sc)
{
    const float A = fmaf(fm, eA, PA0), B = fmaf(fm, eB, PB0), C = fmaf(fm, eC, PC0);
    const unsigned iA = (unsigned)A, iB = (unsigned)B, iC = (unsigned)C;
    const float tA = __builtin_amdgcn_fractf(A), tB = __builtin_amdgcn_fractf(B), tC = __builtin_amdgcn_fractf(C);
    const unsigned off = __umul24(iC, 4u * sc) + __umul24(iB, 4u * FP_WA) + (iA << 2) + base;   // bytes
    const float *p = (const float *)((const char *)slab + off);
    constexpr int sb = FP_WA;
    const float l00 = fmaf(tA, p[1] - p[0], p[0]);
    const float l10 = fmaf(tA, p[sb + 1] - p[sb], p[sb]);
    const float l01 = fmaf(tA, p[sc + 1] - p[sc], p[sc]);
    const float l11 = fmaf(tA, p[sc + sb + 1] - p[sc + sb], p[sc + sb]);
    const float m0 = fmaf(tB, l10 - l00, l00), m1 = fmaf(tB, l11 - l01, l01);
    return fmaf(tC, m1 - m0, m0);
}

// Stage one slab (cross-section box b_lo.., c_lo.. of HB x HC cells, planes
// a0 .. a0 + D along A) into LDS at buf, layout [c][b][a].  Each thread owns
// fixed (a, b) cells and walks them up through the z planes.  Planes outside
// the grid are zero; the rest are read through buffer descriptors over runs
// of eight planes (plane offsets are uniform, the cell's byte offset is per
// lane) straight into LDS, one word per cell, and are still in flight on
// return (the caller waits).
template <int AX>
__device__ __forceinline__ void stage_slab(const Geom3D &g, const float *f, float *buf, int a0, int b_lo, int c_lo,
                                           int HB, int HC, int tid)
{
    const int plane = FP_WA * HB;   // cells per z plane
    const int z_lo = max(c_lo, 0), z_hi = min(c_lo + HC - 1, g.nz - 1);
    const int n_below = min(z_lo - c_lo, HC), n_in = max(z_hi - z_lo + 1, 0);   // n_below + n_in <= HC
    const size_t zstride = (size_t)g.nx * g.ny;
    const unsigned zbytes = (unsigned)(zstride * sizeof(float));
    const float *fz = f + (size_t)z_lo * zstride;
    // cell q of a plane is LDS word q, so a wave fills 64 consecutive words
    // per plane; columns outside the grid are zeroed
    for (int q = tid; q < plane; q += 256) {
        const int ib = q / FP_WA, ia = q - ib * FP_WA;
        const int ga = a0 + ia, gb = b_lo + ib;
        const int gx = AX == 0 ? ga : gb, gy = AX == 0 ? gb : ga;
        const bool in_xy = (unsigned)gx < (unsigned)g.nx && (unsigned)gy < (unsigned)g.ny;
        float *dst = buf + q;
        for (int ic = 0; ic < n_below; ++ic)
            dst[ic * plane] = 0.0f;
        for (int ic = n_below + n_in; ic < HC; ++ic)
            dst[ic * plane] = 0.0f;
        if (in_xy) {
            const unsigned xy = (unsigned)(gy * g.nx + gx) * (unsigned)sizeof(float);
            // first word of this wave's run of 64 cells
            float *wrun = buf + __builtin_amdgcn_readfirstlane(q & ~63);
            const float *src = fz;
            for (int ic0 = 0; ic0 < n_in; ic0 += 8) {
                const int cnt = min(n_in - ic0, 8);
                const __amdgpu_buffer_rsrc_t rs = plane_run(src, (unsigned)cnt * zbytes);
                float *wd = wrun + (n_below + ic0) * plane;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    if (u < cnt) {   // uniform
                        auto *l = (__attribute__((address_space(3))) void *)(wd + u * plane);
                        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, l, 4, xy, (unsigned)u * zbytes, 0, 0);
                    }
                }
                src += 8 * zstride;
            }
        } else {
            for (int ic = n_below; ic < n_below + n_in; ++ic)
                dst[ic * plane] = 0.0f;
        }
    }
}

// Slab walk of one tile along the dominant axis AX (0: x, 1: y); B is the
// other horizontal axis, C = z.  LDS layout [c][b][a], a fastest.
template <int AX>
__device__ __forceinline__ float slab_walk(const Geom3D &g, const float *f, float *slab, int *s_range, int4 *s_box,
                                           const Ray &r, const Ray cr[4], bool hit, int kb, int ke)
{
    constexpr int BX = 1 - AX;
    const int tid = threadIdx.x;
    const int NB = AX == 0 ? g.ny : g.nx, NC = g.nz;
    const float sgn = cr[0].e[AX] > 0.0f ? 1.0f : -1.0f;
    // biased coordinates of this ray
    const float PA0 = r.p[AX] + RAY_BIAS, eA = r.e[AX];
    const float PB0 = r.p[BX] + RAY_BIAS, eB = r.e[BX];
    const float PC0 = r.p[2] + RAY_BIAS, eC = r.e[2];

    // slabs cover floor(A) in [-2, NA]; slab s holds floor(A) in [-2 + s D, -2 + (s+1) D)
    if (tid == 0) {
        s_range[0] = 1 << 30;
        s_range[1] = -(1 << 30);
    }
    __syncthreads();
    if (hit) {
        const int ia = (int)fmaf((float)kb, eA, PA0) - FP_BIAS, ie = (int)fmaf((float)ke, eA, PA0) - FP_BIAS;
        atomicMin(&s_range[0], (min(ia, ie) + 2) / FP_D);
        atomicMax(&s_range[1], (max(ia, ie) + 2) / FP_D);
    }
    __syncthreads();
    const int s_min = s_range[0], s_max = s_range[1];

    float rA[4];   // 1 / (A step) of the corner rays
#pragma unroll
    for (int c = 0; c < 4; ++c)
        rA[c] = 1.0f / cr[c].e[AX];
    const float rEA = 1.0f / eA;

    float acc = 0.0f;
    int m = kb;   // next sample of this ray
    const int n_slabs = s_max - s_min + 1;
    // cross-sections of the tile's pyramid between planes a0 and a0 + D of
    // slabs n0 .. n0 + FP_BOXES - 1, one slab per thread: the corner rays
    // clipped to the grid plus a two-voxel halo (one more cell below, two
    // above the floor of the extreme coordinates); a ring of two batches, so
    // the next slab's box is known while the current one is sampled
    auto fill_boxes = [&](int n0) {
        for (int u = tid; u < min(FP_BOXES, n_slabs - n0); u += 256) {
            const int su = sgn > 0.0f ? s_min + n0 + u : s_max - n0 - u;
            const int au = -2 + su * FP_D;
            float bmin = 3.0e38f, bmax = -3.0e38f, cmin = 3.0e38f, cmax = -3.0e38f;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const float t = ((float)(au + e * FP_D) - cr[c].p[AX]) * rA[c];
                    const float bb = fmaf(t, cr[c].e[BX], cr[c].p[BX]), cc = fmaf(t, cr[c].e[2], cr[c].p[2]);
                    bmin = fminf(bmin, bb);
                    bmax = fmaxf(bmax, bb);
                    cmin = fminf(cmin, cc);
                    cmax = fmaxf(cmax, cc);
                }
            }
            s_box[(n0 + u) % (2 * FP_BOXES)] =
                make_int4(max((int)floorf(bmin) - 1, -2), min((int)floorf(bmax) + 2, NB + 1),
                          max((int)floorf(cmin) - 1, -2), min((int)floorf(cmax) + 2, NC + 1));
        }
    };
    if (n_slabs > 0) {
        fill_boxes(0);
        __syncthreads();
    }
    bool in_flight = false;   // the current slab was loaded during the previous one (uniform)
    for (int n = 0; n < n_slabs; ++n) {
        const int s = sgn > 0.0f ? s_min + n : s_max - n;
        const int a0 = -2 + s * FP_D;   // first plane of the slab
        const int4 box = s_box[n % (2 * FP_BOXES)];
        const int b_lo = box.x, b_hi = box.y, c_lo = box.z, c_hi = box.w;
        const int HB = b_hi - b_lo + 1, HC = c_hi - c_lo + 1;
        const bool staged = HB > 0 && HC > 0 && FP_WA * HB * HC <= FP_LDS_FLOATS;
        // slabs that fit one half of the buffer are double-buffered: slab
        // n + 1 is loaded into the other half while slab n is sampled
        const bool small = staged && FP_WA * HB * HC <= FP_HALF;
        float *buf = small ? slab + (n & 1) * FP_HALF : slab;
        if (in_flight) {
            __builtin_amdgcn_s_waitcnt(0);   // this slab's loads have landed in LDS
            __syncthreads();
        } else if (staged) {
            __syncthreads();   // the previous slab has been consumed
            stage_slab<AX>(g, f, buf, a0, b_lo, c_lo, HB, HC, tid);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
        }
        in_flight = false;
        if (n + 1 < n_slabs) {
            if ((n + 1) % FP_BOXES == 0) {
                fill_boxes(n + 1);
                __syncthreads();
            }
            const int4 nb = s_box[(n + 1) % (2 * FP_BOXES)];
            const int nHB = nb.y - nb.x + 1, nHC = nb.w - nb.z + 1;
            // every wave has passed this iteration's barrier, so the other
            // half (slab n - 1) is free
            if (small && nHB > 0 && nHC > 0 && FP_WA * nHB * nHC <= FP_HALF) {
                const int ns = sgn > 0.0f ? s + 1 : s - 1;
                stage_slab<AX>(g, f, slab + ((n + 1) & 1) * FP_HALF, -2 + ns * FP_D, nb.x, nb.z, nHB, nHC, tid);
                in_flight = true;
            }
        }
        if (!hit)
            continue;
        // samples of this ray inside the slab: m .. m_end-1, counted exactly
        // with the FP32 coordinate the interpolation uses (A is monotonic in m)
        const int offA = a0 + FP_BIAS, offB = b_lo + FP_BIAS, offC = c_lo + FP_BIAS;
        int m_end = m;
        if (m <= ke && in_slab(m, eA, PA0, offA)) {
            const float bound = sgn > 0.0f ? (float)(offA + FP_D) : (float)offA;
            const float est = (bound - fmaf((float)m, eA, PA0)) * rEA;
            m_end = min(m + max((int)ceilf(est), 1), ke + 1);
            // the estimate is off by at most a step, so the corrections run
            // once or not at all: keep them scalar loops
#pragma clang loop unroll(disable) vectorize(disable) interleave(disable)
            while (m_end > m + 1 && !in_slab(m_end - 1, eA, PA0, offA))
                --m_end;
#pragma clang loop unroll(disable) vectorize(disable) interleave(disable)
            while (m_end <= ke && in_slab(m_end, eA, PA0, offA))
                ++m_end;
        }
        if (staged) {
            // LDS cell of biased coordinates (A, B, C), as a byte offset
            const unsigned base = 4u * (unsigned)(-(offC * HB + offB) * FP_WA - offA);
            const unsigned sc = (unsigned)(FP_WA * HB);
            // two samples per pass (sample indices are exact in FP32); an odd
            // last pass repeats the final sample and drops it, so a wave
            // runs ceil(n / 2) passes for the longest lane's n samples
            const float fend = (float)m_end;
            for (float fm = (float)m; fm < fend; fm += 2.0f) {
                acc += sample_lds(buf, fm, PA0, eA, PB0, eB, PC0, eC, base, sc);
                const float f1 = fm + 1.0f;
                const float s1 = sample_lds(buf, fminf(f1, fend - 1.0f), PA0, eA, PB0, eB, PC0, eC, base, sc);
                acc += f1 < fend ? s1 : 0.0f;
            }
            m = m_end;
        } else {
            for (; m < m_end; ++m) {
                const float fm = (float)m;
                float q[3];
                q[AX] = fmaf(fm, eA, PA0) - (float)FP_BIAS;
                q[BX] = fmaf(fm, eB, PB0) - (float)FP_BIAS;
                q[2] = fmaf(fm, eC, PC0) - (float)FP_BIAS;
                acc += sample_global(f, g, q[0], q[1], q[2]);
            }
        }
    }
    return acc;
}

// Work order.  Consecutive views of one detector tile sample nearly the same
// cells, so they run side by side and share the slabs in L2: work item
// w = ((b * n_groups + group) * n_tiles + tile) * FP_VG + view-in-group.
// Workgroups are dealt to the 8 XCDs round-robin (XCD = blockIdx mod 8),
// each with its own L2, so every XCD is given one contiguous range of work
// items.
struct FpWork {
    int ntu, ntiles, ngroups, total;   // total = batch * ngroups * ntiles * FP_VG
};

// The volume is FP32 (a half-precision volume is widened first, exactly);
// TO is the projections' storage type.
template <typename TO>
__global__ void __launch_bounds__(256) fp_cone_kernel(Geom3D g, const ConeFPView *__restrict__ views,
                                                      const float *__restrict__ vol, TO *__restrict__ proj, FpWork wk)
{
    __shared__ float slab[FP_LDS_FLOATS];
    __shared__ int4 s_box[2 * FP_BOXES];
    __shared__ Ray s_corner[4];
    __shared__ int s_range[2];
    const int tid = threadIdx.x;
    const unsigned per_xcd = gridDim.x / FP_XCDS;
    const int w = (int)((blockIdx.x % FP_XCDS) * per_xcd + blockIdx.x / FP_XCDS);
    if (w >= wk.total)
        return;
    const int kk = w % FP_VG, t = (w / FP_VG) % wk.ntiles, bg = w / (FP_VG * wk.ntiles);
    const int k = (bg % wk.ngroups) * FP_VG + kk, b = bg / wk.ngroups;
    if (k >= g.n_proj)
        return;
    const int j0 = (t % wk.ntu) * FP_TILE, i0 = (t / wk.ntu) * FP_TILE;
    const int j = j0 + (tid % FP_TILE), i = i0 + (tid / FP_TILE);
    const bool valid = j < g.nu && i < g.nv;
    const ConeFPView &v = views[k];
    const float *f = vol + (size_t)b * g.nx * g.ny * g.nz;

    const Ray r = make_cone_ray(g, v, valid ? j : j0, valid ? i : i0);
    float lo = -3.0e38f, hi = 3.0e38f;
    const bool hit = valid && krange(r.p[0], r.e[0], g.nx, lo, hi) && krange(r.p[1], r.e[1], g.ny, lo, hi) &&
                     krange(r.p[2], r.e[2], g.nz, lo, hi) && lo < hi;
    // one sample of margin on each side; samples outside the box add zeros
    const int kb = hit ? (int)floorf(lo) : 0, ke = hit ? (int)ceilf(hi) : -1;

    // the tile's four corner rays bound the pyramid of its rays; they are the
    // rays of the threads owning the corner pixels (always valid pixels), so
    // those threads publish theirs instead of every thread setting up four
    // more rays in double precision
    const int jh = min(j0 + FP_TILE - 1, g.nu - 1), ih = min(i0 + FP_TILE - 1, g.nv - 1);
    {
        const int tj = tid % FP_TILE, ti = tid / FP_TILE;
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (tj == ((c & 1) ? jh - j0 : 0) && ti == ((c & 2) ? ih - i0 : 0))
                s_corner[c] = r;
    }
    __syncthreads();
    Ray cr[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
        cr[c] = s_corner[c];
    // slab axis A of this tile: the horizontal axis along which its slowest
    // corner ray still advances fastest (the rays of a tile span a fraction of
    // a degree, so near 45 degrees one tile walks x and its neighbour y).
    // The walk needs every ray to advance along A in one direction (interior
    // rays are positive combinations of the corner directions) and by at
    // most one voxel per step on every axis (margin samples stay inside the
    // two-voxel halo); the cross-section may grow faster than one voxel per
    // plane, in which case a slab that outgrows LDS reads the volume
    // directly.  A run of eight planes must also fit a buffer descriptor's
    // 32-bit range.
    float mx = 3.0e38f, my = 3.0e38f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        mx = fminf(mx, fabsf(cr[c].e[0]));
        my = fminf(my, fabsf(cr[c].e[1]));
    }
    const int ax = mx >= my ? 0 : 1;
    bool slab_ok = g.step <= fminf(g.sx, fminf(g.sy, g.sz)) && (size_t)g.nx * g.ny * sizeof(float) * 8 <= 0xffffffffu;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const float eA = cr[c].e[ax], eB = cr[c].e[1 - ax];
        slab_ok = slab_ok && eA * cr[0].e[ax] > 0.0f && fabsf(eA) <= 1.0f && fabsf(eB) <= 1.0f &&
                  fabsf(cr[c].e[2]) <= 1.0f;
    }

    float acc = 0.0f;
    if (!slab_ok) {
        const float P0 = r.p[0] + RAY_BIAS, P1 = r.p[1] + RAY_BIAS, P2 = r.p[2] + RAY_BIAS;
        for (int m = kb; m <= ke; ++m)
            acc += sample_global(f, g, ray_coord_biased(P0, r.e[0], m) - RAY_BIAS,
                                 ray_coord_biased(P1, r.e[1], m) - RAY_BIAS, ray_coord_biased(P2, r.e[2], m) - RAY_BIAS);
    } else if (ax == 0) {
        acc = slab_walk<0>(g, f, slab, s_range, s_box, r, cr, hit, kb, ke);
    } else {
        acc = slab_walk<1>(g, f, slab, s_range, s_box, r, cr, hit, kb, ke);
    }
    if (valid)
        store_f32(proj + (((size_t)b * g.n_proj + k) * g.nv + i) * g.nu + j, g.step * acc);
}

template <typename TO>
hipError_t fp_cone(const Geom3D &g, const ConeFPView *views, const float *vol, void *proj, int batch, hipStream_t s)
{
    FpWork wk;
    wk.ntu = (g.nu + FP_TILE - 1) / FP_TILE;
    wk.ntiles = wk.ntu * ((g.nv + FP_TILE - 1) / FP_TILE);
    wk.ngroups = (g.n_proj + FP_VG - 1) / FP_VG;
    const long total = (long)batch * wk.ngroups * wk.ntiles * FP_VG;
    if (total > (1L << 30))
        return hipErrorInvalidConfiguration;
    wk.total = (int)total;
    const unsigned grid = (unsigned)((total + FP_XCDS - 1) / FP_XCDS * FP_XCDS);
    hipLaunchKernelGGL((fp_cone_kernel<TO>), dim3(grid), dim3(256), 0, s, g, views, vol, (TO *)proj, wk);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_project_cone(int dtype, const Geom3D &g, const ConeFPView *views, const float *vol, void *proj,
                               int batch, hipStream_t stream)
{
    switch (dtype) {
    case 0: return fp_cone<float>(g, views, vol, proj, batch, stream);
    case 1: return fp_cone<f16_t>(g, views, vol, proj, batch, stream);
    default: return fp_cone<bf16_t>(g, views, vol, proj, batch, stream);
    }
}

}  // namespace ph
