// Internal definitions shared by the HIP kernels and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ph {

// ------------------------------------------------------------- storage types
// FP32 math everywhere; volumes and projections may be stored as FP16 or BF16
// (round to nearest even on store).

typedef _Float16 f16_t;
struct bf16_t {
    uint16_t bits;
};

__device__ __forceinline__ float load_f32(const float *p) { return *p; }
__device__ __forceinline__ float load_f32(const f16_t *p) { return (float)(*p); }
__device__ __forceinline__ float load_f32(const bf16_t *p) { return __uint_as_float((uint32_t)p->bits << 16); }

__device__ __forceinline__ void store_f32(float *p, float v) { *p = v; }
__device__ __forceinline__ void store_f32(f16_t *p, float v) { *p = (f16_t)v; }
__device__ __forceinline__ void store_f32(bf16_t *p, float v)
{
    uint32_t u = __float_as_uint(v);
    uint16_t r;
    if ((u & 0x7fffffffu) > 0x7f800000u)
        r = (uint16_t)((u >> 16) | 0x40u);  // NaN stays a (quiet) NaN
    else
        r = (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
    p->bits = r;
}

// ----------------------------------------------------------- device geometry

struct Geom2D {
    int nx, ny, nu, n_proj;
    int curved;            // fan beams: 1 for the equiangular (arc) detector, 0 for the flat one
    float ox, oy;          // world mm of pixel (0,0)
    float inv_sx, inv_sy;  // 1 / spacing
    float sx, sy;
    float du, cu;          // detector spacing, (nu-1)/2
    float sid, sdd;
    float step;            // ray sampling step (mm)
    float dbeta;           // range / n_proj
};

struct Geom3D {
    int nx, ny, nz, nu, nv, n_proj;
    float ox, oy, oz;
    float sx, sy, sz;
    float inv_sx, inv_sy, inv_sz;
    float du, dv, cu, cv;
    float sid, sdd;
    float step;
    float dbeta;
};

// Per-view parameters of the cone back-projector: rows mapping the centred
// voxel index (x - (nx-1)/2, y - (ny-1)/2, z - (nz-1)/2, 1) to
// (Uc, Vc, W) with Uc = (j - cu) W, Vc = (i - cv) W, W the depth in mm.
struct ConeBPView {
    float r[3][4];
};

// The same rows in double precision, for trajectories that are not a rotation
// about z.  There every voxel is projected on its own (no per-column
// shortcut), and FP32 rows and positions would place it only to ~ulp(|u|)
// ~ 3e-5 pixel on a detector a thousand pixels wide; the transpose of the
// back-projector at high magnification (a voxel projecting onto several
// pixels) is sensitive to exactly that.  Full-rate FP64 VALU on gfx950 makes
// the FP64 projection cost about what the FP32 one does per instruction.
// The library's cached back-projector table of such a trajectory holds
// n_proj ConeBPView followed by n_proj ConeBPView64.
struct ConeBPView64 {
    double r[3][4];
};

// Per-view parameters of the cone forward projector (world mm, isocentre at
// the origin): source s; the ray of centred pixel (jc, ic) has direction
// d0 + jc*du + ic*dv (not normalised, pointing away from the source).
// Double precision: the source sits ~SID from the volume, so an FP32 ray
// direction would misplace the ray by ~SID * 2^-24 at the volume.
struct ConeFPView {
    double s[3];
    double d0[3];
    double du[3];
    double dv[3];
    double inv_sp[3];    // 1 / voxel spacing (x, y, z)
    double step_sp[3];   // sampling step / voxel spacing (x, y, z)
};

// ------------------------------------------------------------------ launchers
// Each returns hipSuccess or the launch error.  `dtype`: 0 f32, 1 f16, 2 bf16.

hipError_t launch_project_2d(int dtype, bool fan, const Geom2D &g, const float2 *views, const void *img, void *sino,
                             int batch, hipStream_t stream);
hipError_t launch_backproject_2d(int dtype, bool fan, const Geom2D &g, const float2 *views, const void *sino,
                                 bool sino_is_f32, void *img, int batch, hipStream_t stream);
// FP32 volume in; projections stored as dtype (FP32, FP16 or BF16)
hipError_t launch_project_cone(int dtype, const Geom3D &g, const ConeFPView *views, const float *vol, void *proj,
                               int batch, hipStream_t stream);
// nz_seg: voxels per thread column segment (16 or 32), chosen by the host
// so that a brick's detector footprint fits the LDS tile (64 x 128 pixels).
// views64: the FP64 rows of a trajectory that is not a rotation about z
// (axial = false), NULL otherwise.  accumulate: add to the volume instead of
// overwriting it (back-projection of the views in shares).
hipError_t launch_backproject_cone(int dtype, const Geom3D &g, const ConeBPView *views, const ConeBPView64 *views64,
                                   bool axial, int nz_seg, const void *proj, bool proj_is_f32, void *vol, int batch,
                                   hipStream_t stream, bool accumulate = false);

// The library's static scratch array on the current device (set up on first
// use per device); PH_ERR_HIP-style failure returns a HIP error.
hipError_t static_scratch(void **ptr, size_t *bytes);

// Exact transposes.  A^T: any storage type (gather, written once).  B^T:
// FP32 in and out (scatter with float atomics into a zero-filled output).
hipError_t launch_project_adjoint_2d(int dtype, bool fan, const Geom2D &g, const float2 *views, const void *sino,
                                     void *img, int batch, hipStream_t stream);
hipError_t launch_project_adjoint_cone(int dtype, const Geom3D &g, const ConeFPView *fviews,
                                       const ConeBPView *bviews, const void *proj, void *vol, int batch,
                                       hipStream_t stream);
hipError_t launch_backproject_adjoint_2d(int in_dtype, bool fan, const Geom2D &g, const float2 *views,
                                         const void *img, float *sino, int batch, hipStream_t stream);
// The output is zero-filled first.
hipError_t launch_backproject_adjoint_cone(int in_dtype, const Geom3D &g, const ConeBPView *views,
                                           const ConeBPView64 *views64, bool axial, int nz_seg, const void *vol,
                                           float *proj, int batch, hipStream_t stream);
// out[i] = in[i] rounded to the storage type (nearest even)
hipError_t launch_cast_from_f32(int dtype, const float *in, void *out, size_t n, hipStream_t stream);
// widens n values of storage type dtype to FP32 (exactly)
hipError_t launch_cast_to_f32(int dtype, const void *in, float *out, size_t n, hipStream_t stream);
// zero-fill kernel (used in place of a memset, which would not replay
// correctly inside a captured graph)
hipError_t fill_zero(float *p, size_t n, hipStream_t stream);

// Row filter: rows of length nu (count = batch * n_proj * nv) are weighted by
// W_red[view][u] * W_cos[v][u] * W[v][u] (any of the three may be NULL; the
// cosine weight is computed from sdd when cos_sdd > 0), filtered with the
// real response K[M] (symmetrised) and written as FP32.
struct FilterArgs {
    int nu, nv, n_proj, batch, M, log2M;
    float du, dv, cu, cv;
    float cos_sdd;       // > 0: apply SDD / sqrt(SDD^2 + u^2 + v^2), or cos(u / SDD) if curved
    int curved;          // 2D fan beam on the equiangular (arc) detector
    const float *K;      // device [M]
    const float2 *tw;    // device [M] exp(-2 pi i t / M)
    const float *W_red;  // device [n_proj][nu] or NULL
    const float *W;      // device [nv][nu] or NULL
};
hipError_t launch_weight_filter(int dtype, const FilterArgs &a, const void *in, float *out, hipStream_t stream);

// Cosine weight of detector pixel (i, j) (Kak & Slaney): SDD / sqrt(SDD^2 +
// u^2 + v^2) on a flat detector, cos(gamma_j) with gamma_j = u / SDD on the
// equiangular arc, 1 for parallel beams (cos_sdd = 0).
__device__ __forceinline__ float cosine_weight(const FilterArgs &a, int i, int j)
{
    if (a.cos_sdd <= 0.0f)
        return 1.0f;
    const float u = ((float)j - a.cu) * a.du;
    if (a.curved)   // |gamma| < pi / 2: the hardware cosine is accurate to a few ulp here
        return __cosf(u * (1.0f / a.cos_sdd));
    const float v = ((float)i - a.cv) * a.dv;
    return a.cos_sdd * __builtin_amdgcn_rsqf(fmaf(a.cos_sdd, a.cos_sdd, fmaf(u, u, v * v)));
}

// Learned-corrector training (FP32)
hipError_t launch_mse(const float *x, const float *ref, const float *mask, size_t n, float *grad, double *loss,
                      hipStream_t stream);
hipError_t launch_corrector_grad(const FilterArgs &a, const float *proj, const float *grad_q, float *dK, float *dW,
                                 hipStream_t stream);
hipError_t launch_adam(float *param, const float *grad, float *m, float *v, size_t n, float lr, float b1, float b2,
                       float eps, int t, hipStream_t stream);

// Total variation (value and / or accumulated gradient)
// aniso: the sum of absolute differences per axis instead of the gradient magnitude
hipError_t launch_tv(const float *vol, int nx, int ny, int nz, int batch, bool aniso, float eps, float weight,
                     float *grad, double *value, hipStream_t stream);

}  // namespace ph
