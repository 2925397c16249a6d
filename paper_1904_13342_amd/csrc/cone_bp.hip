// Voxel-driven, distance-weighted cone-beam back-projection from projection
// matrices (Sec. II.B.2; Eq. 5's A^T in the FDK network).
//
// Mapping: a workgroup owns a 16 x 16 x NZ brick of voxels (NZ = 16 or 32,
// the deeper one when its footprint fits the LDS tile); each thread owns
// one (x, y) column segment of NZ voxels and accumulates it in registers over
// all views, so the volume is written exactly once.  Per view, the brick's
// footprint on the detector (bounded by the projections of its 8 corners,
// plus a one-pixel margin) is staged in LDS with zero outside the detector;
// the bilinear fetches then come from LDS instead of texture units.  The
// corners are projected by eight lanes each and reduced across lanes with DPP
// moves, so every wave gets the footprint without an extra barrier.
//
// The exact transpose B^T (below) mirrors this kernel.
//
// For a circular trajectory about z (AXIAL: the matrices have no z term in
// the u and w rows) the column coordinate, the depth w and the weight are
// constant along a column, and only the row coordinate moves with z: one FMA
// per voxel.  General matrices take the per-voxel path, projected in FP64.
#include "device_util.h"

namespace ph {
namespace {

constexpr int BP_TW = 64;    // max staged footprint width (detector columns)
constexpr int BP_TH = 102;   // max staged footprint height (detector rows)
// Tile row stride: 78 floats measured fastest of 65-68, 70, 74, 78, 82 and 90,
// each with the largest height that keeps five workgroups per CU.
constexpr int BP_TS = 78;

// One detector row as a raw buffer: its first word and its length in bytes.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t det_row(const float *row, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(row), (short)0, (int)bytes, 0x00020000);
}

template <typename TI>
__device__ __forceinline__ float det_pix(const TI *q, int nu, int nv, int i, int j)
{
    return (i >= 0 && j >= 0 && i < nv && j < nu) ? load_f32(q + (size_t)i * nu + j) : 0.0f;
}

// bilinear fetch at tile-local coordinates, unit-stride columns
__device__ __forceinline__ float bilerp_tile(const float *p, float fu, float fv)
{
    const float p00 = p[0], p01 = p[1], p10 = p[BP_TS], p11 = p[BP_TS + 1];
    const float a0 = fmaf(fu, p01 - p00, p00), a1 = fmaf(fu, p11 - p10, p10);
    return fmaf(fv, a1 - a0, a0);
}

template <typename TI>
__device__ __forceinline__ float bilerp_global(const TI *q, const Geom3D &g, float su, float sv)
{
    const float fsu = floorf(su), fsv = floorf(sv);
    const int j = (int)fsu, i = (int)fsv;
    const float fu = su - fsu, fv = sv - fsv;
    const float p00 = det_pix(q, g.nu, g.nv, i, j), p01 = det_pix(q, g.nu, g.nv, i, j + 1);
    const float p10 = det_pix(q, g.nu, g.nv, i + 1, j), p11 = det_pix(q, g.nu, g.nv, i + 1, j + 1);
    const float a0 = fmaf(fu, p01 - p00, p00), a1 = fmaf(fu, p11 - p10, p10);
    return fmaf(fv, a1 - a0, a0);
}

// Footprint of a brick on the detector for one view: the projections of its
// 8 corners (one per lane, lane mod 8) reduced across lanes, widened by one
// pixel.  B and B^T call this with the same corners, so they stage the same
// tile and evaluate the same tile-local coordinates.
struct Footprint {
    int u_lo, v_lo, tw, th;
};

__device__ __forceinline__ Footprint brick_footprint(const ConeBPView &v, const Geom3D &g, float cx, float cy,
                                                     float cz)
{
#pragma clang fp contract(off)
    const float crw = rcp_nr(dot4(v.r[2], cx, cy, cz));
    const float cu = dot4(v.r[0], cx, cy, cz) * crw, cv = dot4(v.r[1], cx, cy, cz) * crw;
    // floor is monotonic, so the floor of the extreme corner is the extreme
    // of the corners' floors
    const int ju = (int)floorf(cu + g.cu), iv = (int)floorf(cv + g.cv);
    Footprint f;
    f.u_lo = imin8(ju) - 1;
    f.v_lo = imin8(iv) - 1;
    f.tw = imax8(ju) + 2 - f.u_lo + 1;
    f.th = imax8(iv) + 2 - f.v_lo + 1;
    return f;
}

// Per-column quantities of a circular view (the matrices have no z term in
// the u and w rows): distance weight (SID/w)^2, centred detector coordinates
// (uc, vc0) of the column's first voxel and the row step per voxel in z.
// Shared by B and B^T (no contraction across these roundings), so the pair
// sees bitwise the same positions.
struct AxialCol {
    float wt, uc, vc0, dvz;
};

__device__ __forceinline__ AxialCol axial_col(const ConeBPView &v, float sid, float xc, float yc, float zc0)
{
#pragma clang fp contract(off)
    AxialCol c;
    const float rW = rcp_nr(dot4(v.r[2], xc, yc, zc0));
    const float sw = sid * rW;
    c.wt = sw * sw;
    c.uc = dot4(v.r[0], xc, yc, zc0) * rW;
    c.vc0 = dot4(v.r[1], xc, yc, zc0) * rW;
    c.dvz = v.r[1][2] * rW;
    return c;
}

// detector coordinate relative to a staged tile (lo) or absolute (lo = 0 form)
__device__ __forceinline__ float tile_coord(float c, float centre, int lo)
{
#pragma clang fp contract(off)
    return c + centre - (float)lo;
}

__device__ __forceinline__ float det_coord(float c, float centre)
{
#pragma clang fp contract(off)
    return c + centre;
}

// Projection of one voxel in a view of a general trajectory, in double
// precision from the FP64 rows: the cell (j, i) of its bilinear footprint
// relative to (u_lo, v_lo) (a staged tile's corner, or 0 for the detector
// itself), the fractions within the cell and the distance weight
// (SID/w)^2.  Shared by B and B^T, so the pair sees bitwise the same
// positions.
struct DetPoint {
    int j, i;
    float fu, fv, wt;
};

__device__ __forceinline__ DetPoint general_point(const ConeBPView64 &v, const Geom3D &g, float xc, float yc,
                                                  float zc, int u_lo, int v_lo)
{
#pragma clang fp contract(off)
    const double x = xc, y = yc, z = zc;
    const double U = fma(v.r[0][0], x, fma(v.r[0][1], y, fma(v.r[0][2], z, v.r[0][3])));
    const double V = fma(v.r[1][0], x, fma(v.r[1][1], y, fma(v.r[1][2], z, v.r[1][3])));
    const double W = fma(v.r[2][0], x, fma(v.r[2][1], y, fma(v.r[2][2], z, v.r[2][3])));
    const double rW = 1.0 / W;
    const double su = fma(U, rW, (double)g.cu - (double)u_lo);
    const double sv = fma(V, rW, (double)g.cv - (double)v_lo);
    const double fsu = floor(su), fsv = floor(sv);
    const double sw = (double)g.sid * rW;
    DetPoint p;
    p.j = (int)fsu;
    p.i = (int)fsv;
    p.fu = (float)(su - fsu);
    p.fv = (float)(sv - fsv);
    p.wt = (float)(sw * sw);
    return p;
}

// bilinear fetch of cell (j, i) of a detector image, zero outside it
template <typename TI>
__device__ __forceinline__ float bilerp_cell(const TI *q, const Geom3D &g, int j, int i, float fu, float fv)
{
    const float p00 = det_pix(q, g.nu, g.nv, i, j), p01 = det_pix(q, g.nu, g.nv, i, j + 1);
    const float p10 = det_pix(q, g.nu, g.nv, i + 1, j), p11 = det_pix(q, g.nu, g.nv, i + 1, j + 1);
    const float a0 = fmaf(fu, p01 - p00, p00), a1 = fmaf(fu, p11 - p10, p10);
    return fmaf(fv, a1 - a0, a0);
}

template <typename T, typename TI, int BP_NZ, bool AXIAL>
__global__ void __launch_bounds__(256) bp_cone_kernel(Geom3D g, const ConeBPView *__restrict__ views,
                                                      const ConeBPView64 *__restrict__ views64,
                                                      const TI *__restrict__ proj, T *__restrict__ vol, int nbx,
                                                      int nby, int nzb, int accumulate)
{
    __shared__ float tile[BP_TH * BP_TS];
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const unsigned lin = blockIdx.x;
    const int bxi = (int)(lin % (unsigned)nbx), byi = (int)((lin / (unsigned)nbx) % (unsigned)nby);
    const int bzb = (int)(lin / (unsigned)(nbx * nby));
    const int ix = bxi * 16 + tx;
    const int iy = byi * 16 + ty;
    const int zb = bzb % nzb, b = bzb / nzb;
    const int z0 = zb * BP_NZ;
    const int zcount = min(BP_NZ, g.nz - z0);
    const bool active = ix < g.nx && iy < g.ny;

    const float hx = 0.5f * (g.nx - 1), hy = 0.5f * (g.ny - 1), hz = 0.5f * (g.nz - 1);
    const float xc = (float)ix - hx, yc = (float)iy - hy, zc0 = (float)z0 - hz;
    // this lane's brick corner (centred voxel indices), clamped to the grid
    const int corner = tid & 7;
    const float cx = (float)((corner & 1) ? min(bxi * 16 + 15, g.nx - 1) : bxi * 16) - hx;
    const float cy = (float)((corner & 2) ? min(byi * 16 + 15, g.ny - 1) : byi * 16) - hy;
    const float cz = zc0 + ((corner & 4) ? (float)(zcount - 1) : 0.0f);

    const TI *pb = proj + (size_t)b * g.n_proj * g.nv * g.nu;
    float acc[BP_NZ];
#pragma unroll
    for (int z = 0; z < BP_NZ; ++z)
        acc[z] = 0.0f;

    for (int k = 0; k < g.n_proj; ++k) {
        const ConeBPView v = views[k];
        const Footprint fp = brick_footprint(v, g, cx, cy, cz);
        const int u_lo = fp.u_lo, v_lo = fp.v_lo, tw = fp.tw, th = fp.th;
        const bool staged = tw <= BP_TW && th <= BP_TH;
        const TI *qk = pb + (size_t)k * g.nv * g.nu;
        if (staged) {
            __syncthreads();
            // FP32 projections whose footprint lies on the detector: each wave
            // loads whole tile rows of BP_TW pixels straight into LDS, one
            // load per row (the pixels past tw are never read; any past the
            // detector's row end fall outside the row's buffer).  Otherwise
            // thread by thread, with zeros off the detector.
            const bool inside = u_lo >= 0 && u_lo + tw <= g.nu && v_lo >= 0 && v_lo + th <= g.nv;
            if (sizeof(TI) == 4 && inside) {
                const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
                const int vs = __builtin_amdgcn_readfirstlane(v_lo), hs = __builtin_amdgcn_readfirstlane(th);
                const unsigned voff = (unsigned)(u_lo + (tid & 63)) * 4u;
                const unsigned row_bytes = (unsigned)g.nu * 4u;
                for (int r = wave; r < hs; r += 4) {
                    const __amdgpu_buffer_rsrc_t rs = det_row((const float *)qk + (size_t)(vs + r) * g.nu, row_bytes);
                    auto *l = (__attribute__((address_space(3))) void *)(tile + r * BP_TS);
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, l, 4, voff, 0, 0, 0);
                }
                __builtin_amdgcn_s_waitcnt(0);   // this wave's rows have landed
            } else {
                for (int r = ty; r < th; r += 16) {
                    const int gi = v_lo + r;
                    const bool row_ok = (unsigned)gi < (unsigned)g.nv;
                    const TI *rowp = qk + (size_t)(row_ok ? gi : 0) * g.nu;
                    for (int c = tx; c < tw; c += 16) {
                        const int gj = u_lo + c;
                        tile[r * BP_TS + c] =
                            (row_ok && (unsigned)gj < (unsigned)g.nu) ? load_f32(rowp + gj) : 0.0f;
                    }
                }
            }
            __syncthreads();
        }
        if (!active)
            continue;
        if (AXIAL) {
            const AxialCol ac = axial_col(v, g.sid, xc, yc, zc0);
            const float wt = ac.wt, dvz = ac.dvz;
            if (staged) {
                // tile-local coordinates are >= 1 (one-pixel margin): floor == truncation
                const float su = tile_coord(ac.uc, g.cu, u_lo);
                const float sv0 = tile_coord(ac.vc0, g.cv, v_lo);
                const int iu = (int)su;
                const float fu = __builtin_amdgcn_fractf(su);
                const float *col = tile + iu;
                if (zcount == BP_NZ) {
#pragma unroll
                    for (int z = 0; z < BP_NZ; ++z) {
                        const float sv = fmaf((float)z, dvz, sv0);
                        const int iv = (int)sv;
                        acc[z] = fmaf(wt, bilerp_tile(col + iv * BP_TS, fu, __builtin_amdgcn_fractf(sv)), acc[z]);
                    }
                } else {
#pragma unroll
                    for (int z = 0; z < BP_NZ; ++z) {
                        if (z < zcount) {
                            const float sv = fmaf((float)z, dvz, sv0);
                            const int iv = (int)sv;
                            acc[z] = fmaf(wt, bilerp_tile(col + iv * BP_TS, fu, __builtin_amdgcn_fractf(sv)),
                                          acc[z]);
                        }
                    }
                }
            } else {
                const float su = det_coord(ac.uc, g.cu), sv0 = det_coord(ac.vc0, g.cv);
#pragma unroll
                for (int z = 0; z < BP_NZ; ++z)
                    if (z < zcount)
                        acc[z] = fmaf(wt, bilerp_global(qk, g, su, fmaf((float)z, dvz, sv0)), acc[z]);
            }
        } else {
            const ConeBPView64 &v64 = views64[k];
#pragma unroll
            for (int z = 0; z < BP_NZ; ++z) {
                if (z < zcount) {
                    const DetPoint d =
                        general_point(v64, g, xc, yc, zc0 + (float)z, staged ? u_lo : 0, staged ? v_lo : 0);
                    const float val = staged ? bilerp_tile(tile + d.i * BP_TS + d.j, d.fu, d.fv)
                                             : bilerp_cell(qk, g, d.j, d.i, d.fu, d.fv);
                    acc[z] = fmaf(d.wt, val, acc[z]);
                }
            }
        }
    }
    if (!active)
        return;
    T *out = vol + (size_t)b * g.nz * g.ny * g.nx + (size_t)iy * g.nx + ix;
#pragma unroll
    for (int z = 0; z < BP_NZ; ++z) {
        if (z < zcount) {
            T *p = out + (size_t)(z0 + z) * g.ny * g.nx;
            // accumulate: add to the volume (a later share of the views)
            store_f32(p, accumulate ? load_f32(p) + g.dbeta * acc[z] : g.dbeta * acc[z]);
        }
    }
}

// ------------------------------------------------------------------- B^T
// Exact transpose of the kernel above: the same bricks, footprints and FP32
// detector coordinates (so the pair is transposed to the last rounding of the
// positions), with each voxel's value times dbeta * (SID/w)^2 splatted into
// the four pixels of its bilinear footprint.  Splats go to an LDS tile of the
// brick's footprint; the tile is then added to the projections with one global
// float atomic per pixel.  FP32 in and out; the output must be zero on entry.
//
// The LDS tile accumulates 32-bit fixed-point integers: on gfx950 u32 LDS
// atomic adds issue in about half the time of FP64 ones, and FP32 LDS atomic
// adds are serialised per lane.  A view's scale is set so that no pixel can
// overflow: each voxel adds at most |x| dbeta (SID/w)^2 to the tile in all
// (its four bilinear weights sum to 1), w is at least the smallest depth of
// the brick's corners in that view (w is affine in the position), so the
// tile's total is bounded by (sum of |x| dbeta over the brick) times
// (SID / w_min)^2.  Every term is rounded to the nearest integer; the flush
// divides by the scale.
// Equal addresses within one instruction still serialise, and columns lined
// up along a ray land on the same detector column, so for circular views the
// lanes of a wave are laid out across the rays: 16 columns on a line along
// the volume axis most perpendicular to the view's central ray times 4 groups
// of z (a quarter of the segment apart), and each thread's voxels (4 columns
// x NZ/4 z) are re-read whenever the views' orientation changes.  One
// instruction then hits 64 distinct pixels whenever neighbouring columns
// project at least a pixel apart.

// tile row stride (words, >= BP_TW + 1): 66, two banks on per row.  At
// 512^3 strides of 2 mod 32 measured fastest (66 and 98: 36.4 ms) of 65-70,
// 72-90 in steps of 4 and 97-100; odd strides took 42-47 ms, 68 and 100 54 ms.
constexpr int BPT_TS = 66;
constexpr float BPT_FIX = 2145386496.0f;   // 2^31 (1 - 2^-10)

__device__ __forceinline__ void splat_tile(int *p, float xs, float fu, float fv, int stride)
{
    const float b = xs * fv, a = xs - b;
    atomicAdd(p, round_to_int(fmaf(-a, fu, a)));
    atomicAdd(p + 1, round_to_int(a * fu));
    atomicAdd(p + stride, round_to_int(fmaf(-b, fu, b)));
    atomicAdd(p + stride + 1, round_to_int(b * fu));
}

__device__ __forceinline__ void splat_global(float *q, const Geom3D &g, float su, float sv, float x)
{
    const float fsu = floorf(su), fsv = floorf(sv);
    const int j = (int)fsu, i = (int)fsv;
    const float fu = su - fsu, fv = sv - fsv;
    const float a = x * (1.0f - fv), b = x * fv;
    const bool r0 = (unsigned)i < (unsigned)g.nv, r1 = (unsigned)(i + 1) < (unsigned)g.nv;
    const bool c0 = (unsigned)j < (unsigned)g.nu, c1 = (unsigned)(j + 1) < (unsigned)g.nu;
    if (r0 && c0)
        unsafeAtomicAdd(q + (size_t)i * g.nu + j, a * (1.0f - fu));
    if (r0 && c1)
        unsafeAtomicAdd(q + (size_t)i * g.nu + j + 1, a * fu);
    if (r1 && c0)
        unsafeAtomicAdd(q + (size_t)(i + 1) * g.nu + j, b * (1.0f - fu));
    if (r1 && c1)
        unsafeAtomicAdd(q + (size_t)(i + 1) * g.nu + j + 1, b * fu);
}

// splat into cell (j, i) of a detector image, skipping pixels outside it
__device__ __forceinline__ void splat_cell(float *q, const Geom3D &g, int j, int i, float fu, float fv, float x)
{
    const float a = x * (1.0f - fv), b = x * fv;
    const bool r0 = (unsigned)i < (unsigned)g.nv, r1 = (unsigned)(i + 1) < (unsigned)g.nv;
    const bool c0 = (unsigned)j < (unsigned)g.nu, c1 = (unsigned)(j + 1) < (unsigned)g.nu;
    if (r0 && c0)
        unsafeAtomicAdd(q + (size_t)i * g.nu + j, a * (1.0f - fu));
    if (r0 && c1)
        unsafeAtomicAdd(q + (size_t)i * g.nu + j + 1, a * fu);
    if (r1 && c0)
        unsafeAtomicAdd(q + (size_t)(i + 1) * g.nu + j, b * (1.0f - fu));
    if (r1 && c1)
        unsafeAtomicAdd(q + (size_t)(i + 1) * g.nu + j + 1, b * fu);
}

// The tile is cleared once per workgroup; each flush then reads and clears
// the footprint it adds to the projections (splats never leave the
// footprint), so the tile is zero again whenever the next view starts.
__device__ __forceinline__ void clear_tile(int *tile, int tid)
{
    for (int n = tid; n < BP_TH * BPT_TS; n += 256)
        tile[n] = 0;
}

__device__ __forceinline__ void flush_tile(int *tile, const Footprint &fp, const Geom3D &g, float *qk, float inv,
                                           int tid)
{
    // Whole footprint rows per wave instruction: a row takes 16, 32 or 64
    // lanes (the least power of two not below tw), lane c of it column c, so
    // each row's atomics fall on consecutive pixels of one detector row, and
    // the row and column need no division.
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int tw = __builtin_amdgcn_readfirstlane(fp.tw), th = __builtin_amdgcn_readfirstlane(fp.th);
    const int v_lo = __builtin_amdgcn_readfirstlane(fp.v_lo);
    const int lc = tw <= 16 ? 4 : (tw <= 32 ? 5 : 6);   // log2 of the lanes per row
    const int c = lane & ((1 << lc) - 1), rows = 64 >> lc;
    const int gj = fp.u_lo + c;
    const bool in_tile = c < tw, col_ok = (unsigned)gj < (unsigned)g.nu;
    for (int r = wave * rows + (lane >> lc); r < th; r += 4 * rows) {
        if (in_tile) {
            int *cell = tile + r * BPT_TS + c;
            const int t = *cell;
            *cell = 0;
            const int gi = v_lo + r;
            if (t != 0 && col_ok && (unsigned)gi < (unsigned)g.nv)
                unsafeAtomicAdd(qk + (size_t)gi * g.nu + gj, (float)t * inv);
        }
    }
}

// Sum of |x| dbeta over the brick's voxels, reduced over the workgroup in a
// fixed order (the same on every run).
__device__ __forceinline__ float brick_abs_sum(float s, float *red, int tid)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
        s += __shfl_xor(s, o);
    if ((tid & 63) == 0)
        red[tid >> 6] = s;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// Fixed-point scale of one view: BPT_FIX / (S (SID / w_min)^2), w_min the
// smallest depth of the brick's corners (8 lanes, one corner each), widened
// by a relative 1e-3 for the reciprocal's rounding.
__device__ __forceinline__ float view_scale(const ConeBPView &v, const Geom3D &g, float cx, float cy, float cz,
                                            float S)
{
    const float wmin = min8(dot4(v.r[2], cx, cy, cz));
    const float sw = g.sid * __builtin_amdgcn_rcpf(wmin);
    return BPT_FIX / (S * (sw * sw * 1.001f));
}

template <typename TI, int BP_NZ>
__global__ void __launch_bounds__(256) bpT_axial_kernel(Geom3D g, const ConeBPView *__restrict__ views,
                                                        const TI *__restrict__ vol, float *__restrict__ proj,
                                                        int nbx, int nby, int nzb)
{
    constexpr int ZQ = BP_NZ / 4;   // voxels in z per lane group
    __shared__ int tile[BP_TH * BPT_TS];
    __shared__ float red[4];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int a = lane & 15, zq = lane >> 4;
    const unsigned lin = blockIdx.x;
    const int bxi = (int)(lin % (unsigned)nbx), byi = (int)((lin / (unsigned)nbx) % (unsigned)nby);
    const int bzb = (int)(lin / (unsigned)(nbx * nby));
    const int zb = bzb % nzb, b = bzb / nzb;
    const int z0 = zb * BP_NZ;
    const int zcount = min(BP_NZ, g.nz - z0);

    const float hx = 0.5f * (g.nx - 1), hy = 0.5f * (g.ny - 1), hz = 0.5f * (g.nz - 1);
    const float zc0 = (float)z0 - hz;
    const int corner = tid & 7;
    const float cx = (float)((corner & 1) ? min(bxi * 16 + 15, g.nx - 1) : bxi * 16) - hx;
    const float cy = (float)((corner & 2) ? min(byi * 16 + 15, g.ny - 1) : byi * 16) - hy;
    const float cz = zc0 + ((corner & 4) ? (float)(zcount - 1) : 0.0f);

    const TI *vb = vol + (size_t)b * g.nz * g.ny * g.nx + (size_t)z0 * g.ny * g.nx;
    float *pb = proj + (size_t)b * g.n_proj * g.nv * g.nu;
    float val[4][ZQ];
    int cur = -1;   // lane layout of val: 0 = lanes along y, 1 = lanes along x
    float S = 0.0f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int ix = bxi * 16 + 4 * wave + c, iy = byi * 16 + a;
        if (ix < g.nx && iy < g.ny)
#pragma unroll
            for (int m = 0; m < ZQ; ++m) {
                const int z = zq * ZQ + m;
                if (z < zcount)
                    S += fabsf(g.dbeta * load_f32(vb + ((size_t)z * g.ny + iy) * g.nx + ix));
            }
    }
    S = brick_abs_sum(S, red, tid);
    if (S == 0.0f)
        return;   // the brick adds nothing (uniform)
    clear_tile(tile, tid);   // ordered before the first splat by the view loop's barrier

    for (int k = 0; k < g.n_proj; ++k) {
        const ConeBPView v = views[k];
        // rays mostly along x (depth row dominated by x): put the lanes along y
        const int orient = fabsf(v.r[2][0]) >= fabsf(v.r[2][1]) ? 0 : 1;
        if (orient != cur) {
            cur = orient;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int ix = bxi * 16 + (orient == 0 ? 4 * wave + c : a);
                const int iy = byi * 16 + (orient == 0 ? a : 4 * wave + c);
                const bool act = ix < g.nx && iy < g.ny;
                const TI *src = vb + (size_t)(act ? iy : 0) * g.nx + (act ? ix : 0);
#pragma unroll
                for (int m = 0; m < ZQ; ++m) {
                    const int z = zq * ZQ + m;
                    val[c][m] = (act && z < zcount) ? g.dbeta * load_f32(src + (size_t)z * g.ny * g.nx) : 0.0f;
                }
            }
        }
        const Footprint fp = brick_footprint(v, g, cx, cy, cz);
        const bool staged = fp.tw <= BP_TW && fp.th <= BP_TH;
        const float scale = view_scale(v, g, cx, cy, cz, S);
        float *qk = pb + (size_t)k * g.nv * g.nu;
        if (staged)
            __syncthreads();   // the previous tile has been flushed and cleared
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int ix = bxi * 16 + (orient == 0 ? 4 * wave + c : a);
            const int iy = byi * 16 + (orient == 0 ? a : 4 * wave + c);
            if (ix >= g.nx || iy >= g.ny)
                continue;
            const AxialCol ac = axial_col(v, g.sid, (float)ix - hx, (float)iy - hy, zc0);
            const float wt = ac.wt, dvz = ac.dvz;
            if (staged) {
                const float su = tile_coord(ac.uc, g.cu, fp.u_lo);
                const float sv0 = tile_coord(ac.vc0, g.cv, fp.v_lo);
                const int iu = (int)su;
                const float fu = __builtin_amdgcn_fractf(su);
                const float ws = wt * scale;
                int *col = tile + iu;
#pragma unroll
                for (int m = 0; m < ZQ; ++m) {
                    const int z = zq * ZQ + m;
                    if (z < zcount) {
                        const float sv = fmaf((float)z, dvz, sv0);
                        const int iv = (int)sv;
                        splat_tile(col + iv * BPT_TS, ws * val[c][m], fu, __builtin_amdgcn_fractf(sv), BPT_TS);
                    }
                }
            } else {
                const float su = det_coord(ac.uc, g.cu), sv0 = det_coord(ac.vc0, g.cv);
#pragma unroll
                for (int m = 0; m < ZQ; ++m) {
                    const int z = zq * ZQ + m;
                    if (z < zcount)
                        splat_global(qk, g, su, fmaf((float)z, dvz, sv0), wt * val[c][m]);
                }
            }
        }
        if (staged) {
            __syncthreads();
            flush_tile(tile, fp, g, qk, 1.0f / scale, tid);
        }
    }
}

// General projection matrices: one thread per column segment, as in B.
template <typename TI, int BP_NZ>
__global__ void __launch_bounds__(256) bpT_general_kernel(Geom3D g, const ConeBPView *__restrict__ views,
                                                          const ConeBPView64 *__restrict__ views64,
                                                          const TI *__restrict__ vol, float *__restrict__ proj,
                                                          int nbx, int nby, int nzb)
{
    __shared__ int tile[BP_TH * BPT_TS];
    __shared__ float red[4];
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const unsigned lin = blockIdx.x;
    const int bxi = (int)(lin % (unsigned)nbx), byi = (int)((lin / (unsigned)nbx) % (unsigned)nby);
    const int bzb = (int)(lin / (unsigned)(nbx * nby));
    const int ix = bxi * 16 + tx;
    const int iy = byi * 16 + ty;
    const int zb = bzb % nzb, b = bzb / nzb;
    const int z0 = zb * BP_NZ;
    const int zcount = min(BP_NZ, g.nz - z0);
    const bool active = ix < g.nx && iy < g.ny;

    const float hx = 0.5f * (g.nx - 1), hy = 0.5f * (g.ny - 1), hz = 0.5f * (g.nz - 1);
    const float xc = (float)ix - hx, yc = (float)iy - hy, zc0 = (float)z0 - hz;
    const int corner = tid & 7;
    const float cx = (float)((corner & 1) ? min(bxi * 16 + 15, g.nx - 1) : bxi * 16) - hx;
    const float cy = (float)((corner & 2) ? min(byi * 16 + 15, g.ny - 1) : byi * 16) - hy;
    const float cz = zc0 + ((corner & 4) ? (float)(zcount - 1) : 0.0f);

    float val[BP_NZ];
    const TI *src = vol + (size_t)b * g.nz * g.ny * g.nx + (size_t)(active ? iy : 0) * g.nx + (active ? ix : 0);
#pragma unroll
    for (int z = 0; z < BP_NZ; ++z)
        val[z] = (active && z < zcount) ? g.dbeta * load_f32(src + (size_t)(z0 + z) * g.ny * g.nx) : 0.0f;
    float S = 0.0f;
#pragma unroll
    for (int z = 0; z < BP_NZ; ++z)
        S += fabsf(val[z]);
    S = brick_abs_sum(S, red, tid);
    if (S == 0.0f)
        return;   // the brick adds nothing (uniform)
    float *pb = proj + (size_t)b * g.n_proj * g.nv * g.nu;
    clear_tile(tile, tid);   // ordered before the first splat by the view loop's barrier

    for (int k = 0; k < g.n_proj; ++k) {
        const ConeBPView v = views[k];
        const Footprint fp = brick_footprint(v, g, cx, cy, cz);
        const bool staged = fp.tw <= BP_TW && fp.th <= BP_TH;
        const float scale = view_scale(v, g, cx, cy, cz, S);
        float *qk = pb + (size_t)k * g.nv * g.nu;
        if (staged)
            __syncthreads();   // the previous tile has been flushed and cleared
        if (active) {
            const ConeBPView64 &v64 = views64[k];
#pragma unroll
            for (int z = 0; z < BP_NZ; ++z) {
                if (z < zcount) {
                    const DetPoint d = general_point(v64, g, xc, yc, zc0 + (float)z, staged ? fp.u_lo : 0,
                                                     staged ? fp.v_lo : 0);
                    if (staged)
                        splat_tile(tile + d.i * BPT_TS + d.j, d.wt * scale * val[z], d.fu, d.fv, BPT_TS);
                    else
                        splat_cell(qk, g, d.j, d.i, d.fu, d.fv, d.wt * val[z]);
                }
            }
        }
        if (staged) {
            __syncthreads();
            flush_tile(tile, fp, g, qk, 1.0f / scale, tid);
        }
    }
}

template <typename T, typename TI, int NZ>
hipError_t bp_cone_nz(const Geom3D &g, const ConeBPView *views, const ConeBPView64 *views64, bool axial,
                      const void *proj, void *vol, int batch, int acc, hipStream_t s)
{
    const int nbx = (g.nx + 15) / 16, nby = (g.ny + 15) / 16, nzb = (g.nz + NZ - 1) / NZ;
    const unsigned blocks = (unsigned)(nbx * nby * nzb * batch);
    if (axial)
        hipLaunchKernelGGL((bp_cone_kernel<T, TI, NZ, true>), dim3(blocks), dim3(256), 0, s, g, views,
                           (const ConeBPView64 *)nullptr, (const TI *)proj, (T *)vol, nbx, nby, nzb, acc);
    else
        hipLaunchKernelGGL((bp_cone_kernel<T, TI, NZ, false>), dim3(blocks), dim3(256), 0, s, g, views, views64,
                           (const TI *)proj, (T *)vol, nbx, nby, nzb, acc);
    return hipGetLastError();
}

template <typename T, typename TI>
hipError_t bp_cone(const Geom3D &g, const ConeBPView *views, const ConeBPView64 *views64, bool axial, int nz_seg,
                   const void *proj, void *vol, int batch, int acc, hipStream_t s)
{
    if (!axial && !views64)
        return hipErrorInvalidValue;
    if (nz_seg >= 32)
        return bp_cone_nz<T, TI, 32>(g, views, views64, axial, proj, vol, batch, acc, s);
    return bp_cone_nz<T, TI, 16>(g, views, views64, axial, proj, vol, batch, acc, s);
}

}  // namespace

hipError_t launch_backproject_cone(int dtype, const Geom3D &g, const ConeBPView *views, const ConeBPView64 *views64,
                                   bool axial, int nz_seg, const void *proj, bool proj_is_f32, void *vol, int batch,
                                   hipStream_t stream, bool accumulate)
{
    const int a = accumulate ? 1 : 0;
    switch (dtype) {
    case 0: return bp_cone<float, float>(g, views, views64, axial, nz_seg, proj, vol, batch, a, stream);
    case 1:
        return proj_is_f32 ? bp_cone<f16_t, float>(g, views, views64, axial, nz_seg, proj, vol, batch, a, stream)
                           : bp_cone<f16_t, f16_t>(g, views, views64, axial, nz_seg, proj, vol, batch, a, stream);
    default:
        return proj_is_f32 ? bp_cone<bf16_t, float>(g, views, views64, axial, nz_seg, proj, vol, batch, a, stream)
                           : bp_cone<bf16_t, bf16_t>(g, views, views64, axial, nz_seg, proj, vol, batch, a, stream);
    }
}

template <typename TI>
hipError_t bpT_cone(const Geom3D &g, const ConeBPView *views, const ConeBPView64 *v64, bool axial, int nz_seg,
                    const void *vol, float *proj, int batch, hipStream_t stream)
{
    if (!axial && !v64)
        return hipErrorInvalidValue;
    const int NZ = nz_seg >= 32 ? 32 : 16;
    const int nbx = (g.nx + 15) / 16, nby = (g.ny + 15) / 16, nzb = (g.nz + NZ - 1) / NZ;
    const dim3 grid((unsigned)(nbx * nby * nzb * batch));
    const TI *v = (const TI *)vol;
    if (NZ == 32) {
        if (axial)
            hipLaunchKernelGGL((bpT_axial_kernel<TI, 32>), grid, dim3(256), 0, stream, g, views, v, proj, nbx, nby,
                               nzb);
        else
            hipLaunchKernelGGL((bpT_general_kernel<TI, 32>), grid, dim3(256), 0, stream, g, views, v64, v, proj, nbx,
                               nby, nzb);
    } else {
        if (axial)
            hipLaunchKernelGGL((bpT_axial_kernel<TI, 16>), grid, dim3(256), 0, stream, g, views, v, proj, nbx, nby,
                               nzb);
        else
            hipLaunchKernelGGL((bpT_general_kernel<TI, 16>), grid, dim3(256), 0, stream, g, views, v64, v, proj, nbx,
                               nby, nzb);
    }
    return hipGetLastError();
}

hipError_t launch_backproject_adjoint_cone(int in_dtype, const Geom3D &g, const ConeBPView *views,
                                           const ConeBPView64 *views64, bool axial, int nz_seg, const void *vol,
                                           float *proj, int batch, hipStream_t stream)
{
    hipError_t e = fill_zero(proj, (size_t)batch * g.n_proj * g.nv * g.nu, stream);
    if (e != hipSuccess)
        return e;
    switch (in_dtype) {
    case 0: return bpT_cone<float>(g, views, views64, axial, nz_seg, vol, proj, batch, stream);
    case 1: return bpT_cone<f16_t>(g, views, views64, axial, nz_seg, vol, proj, batch, stream);
    default: return bpT_cone<bf16_t>(g, views, views64, axial, nz_seg, vol, proj, batch, stream);
    }
}

}  // namespace ph
