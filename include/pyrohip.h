/*
 * pyrohip.h -- C ABI of the MI355X-native known-operator CT library
 * (ray-driven forward projection, voxel-driven back-projection, ramp-filtered
 * FBP / FDK) following PYRO-NN, arXiv 1904.13342.
 *
 * All entry points are plain C: geometry records, host or device pointers,
 * sizes and a HIP stream handle passed as void*.  No entry point throws,
 * exits or prints; every one returns a ph_status.
 *
 * Geometry (Sec. II.C.1 lists the attributes: volume shape and spacing,
 * detector shape and spacing, number of projections, angular range, SID and
 * SDD; Sec. II.C.3 adds the trajectory as central ray vectors in 2D and
 * projection matrices in 3D).  Conventions:
 *   - voxel (ix,iy,iz) centre at world (ox+ix*sx, oy+iy*sy, oz+iz*sz) mm,
 *     arrays are C-contiguous with x fastest: 2D image [batch][ny][nx],
 *     3D volume [batch][nz][ny][nx];
 *   - detector pixel (i,j): row i (v, along +z), column j (u); pixel centre
 *     u_j = (j-(nu-1)/2)*du, v_i = (i-(nv-1)/2)*dv; arrays [batch][n_proj][nu]
 *     in 2D and [batch][n_proj][nv][nu] in 3D, u fastest;
 *   - 2D view k has central ray vector c_k = ray_vecs[k] (unit, world x,y);
 *     detector axis e_u = (-c_y, c_x); parallel rays pass through u*e_u with
 *     direction c_k; fan rays leave the source -SID*c_k for the flat detector
 *     centred at (SDD-SID)*c_k;
 *   - 3D view k has projection matrix mats[k] (row-major 3x4) mapping
 *     homogeneous world mm to (j*w, i*w, w); the library rescales each matrix
 *     so that w is the depth in mm along the central ray (positive in front
 *     of the source).
 *
 * Memory: every array argument named img/vol/sino/proj/K/W_red/W/ws is a
 * DEVICE pointer owned by the caller; ray_vecs and mats are HOST pointers,
 * read during the call.  Outputs are overwritten, never accumulated.  Work is
 * enqueued on `stream` (a hipStream_t; NULL = the default stream) and is
 * asynchronous.  The library keeps a small per-device cache of derived
 * per-view parameters (uploaded once per distinct geometry with a blocking
 * copy); besides that it allocates no device memory: FBP/FDK scratch comes
 * from the caller's workspace `ws` sized by ph_workspace_bytes_*.
 *
 * Storage type (ph_dtype) applies to img/vol/sino/proj; arithmetic is FP32
 * and geometry is always FP32.  FP16 and BF16 are rounded to nearest-even on
 * store.
 */
#ifndef PYROHIP_H
#define PYROHIP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PH_OK = 0,
    PH_ERR_NULL = -1,        /* a required pointer is NULL */
    PH_ERR_SHAPE = -2,       /* non-positive size, batch < 1, bad filter length */
    PH_ERR_GEOMETRY = -3,    /* non-positive or non-finite spacing/step, SDD <= SID,
                                source inside the volume, singular or non-finite matrix */
    PH_ERR_DTYPE = -4,       /* unknown storage type */
    PH_ERR_WORKSPACE = -5,   /* workspace NULL or smaller than required */
    PH_ERR_HIP = -6,         /* a HIP call or kernel launch failed */
    PH_ERR_UNSUPPORTED = -7, /* valid request this build does not implement */
    PH_ERR_VALUE = -8        /* scalar argument non-finite or out of range */
} ph_status;

typedef enum { PH_F32 = 0, PH_F16 = 1, PH_BF16 = 2 } ph_dtype;

typedef struct {
    int vol_shape[2];       /* (ny, nx) */
    float vol_spacing[2];   /* (sy, sx) mm */
    float vol_origin[2];    /* (oy, ox): world mm of the centre of pixel (0,0) */
    int det_shape;          /* nu */
    float det_spacing;      /* du mm */
    int n_proj;
    float angular_range;    /* rad; view k nominally at k*range/n_proj */
    float sid, sdd;         /* mm; ignored by the parallel-beam calls */
    float step_mm;          /* ray sampling step of the forward projector; <= 0 -> half the smallest spacing */
    int fan_detector;       /* fan calls: 0 flat, equispaced detector (bin u_j = (j-(nu-1)/2)*du on the line
                               SDD from the source); 1 equiangular arc of radius SDD about the source, bin j
                               at fan angle gamma_j = (j-(nu-1)/2)*du/SDD (du the arc length between bins;
                               requires nu*du/SDD < pi).  Ignored by the parallel-beam calls. */
} ph_geom2d;

typedef struct {
    int vol_shape[3];       /* (nz, ny, nx) */
    float vol_spacing[3];   /* (sz, sy, sx) mm */
    float vol_origin[3];    /* (oz, oy, ox): world mm of the centre of voxel (0,0,0) */
    int det_shape[2];       /* (nv, nu) */
    float det_spacing[2];   /* (dv, du) mm */
    int n_proj;
    float angular_range;    /* rad */
    float sid, sdd;         /* mm */
    float step_mm;          /* <= 0 -> half the smallest spacing */
} ph_geom3d;

/* Human-readable name of a status code (static string). */
const char *ph_status_string(int status);

/* Library version and the GPU architecture it was built for. */
const char *ph_version(void);

/* ------------------------------------------------------------------ trajectories
 * Sec. II.C.3: basic helpers that compute the trajectory of a circular scan
 * from the geometry.  Host only, no GPU needed.  View k at angle
 * beta_k = k*range/n_proj, counter-clockwise about +z. */

/* ray_vecs: host float[n_proj][2] <- (cos beta_k, sin beta_k). */
int ph_ray_vectors_2d(const ph_geom2d *g, float *ray_vecs);

/* mats: host float[n_proj][3][4] <- Kint [R | -R S] with R rows (e_u; e_v; c),
 * S = -SID*c, Kint = [[SDD/du, 0, (nu-1)/2], [0, SDD/dv, (nv-1)/2], [0,0,1]]. */
int ph_projection_matrices_3d(const ph_geom3d *g, float *mats);

/* --------------------------------------------------- forward projection A
 * Sec. II.B.2 (ray-driven forward projection, one ray per detector pixel,
 * absorption accumulated along it; Eq. 1 A x = p).  Every ray r is sampled on
 * the lattice a_r + k*step*d_r, k in Z, with a_r the point of the ray closest
 * to the isocentre and d_r its unit direction; the volume is interpolated
 * bi-/trilinearly with zero outside the grid; p_r = step * sum_k.
 *   img  : device [batch][ny][nx]        (dtype)      input
 *   sino : device [batch][n_proj][nu]    (dtype)      output
 *   vol  : device [batch][nz][ny][nx]    (dtype)      input
 *   proj : device [batch][n_proj][nv][nu](dtype)      output
 * ph_project_cone3d with FP16/BF16 storage widens the volume into an FP32 copy
 * (4 bytes per voxel, taken and freed in stream order on `stream` with
 * hipMallocAsync / hipFreeAsync) and projects that: results equal FP32
 * arithmetic on the stored values, rounded to dtype on store.  If the copy
 * cannot be allocated the call returns PH_ERR_HIP and writes nothing. */
int ph_project_par2d(const ph_geom2d *g, const float *ray_vecs, const void *img, void *sino, int batch,
                     ph_dtype dtype, void *stream);
int ph_project_fan2d(const ph_geom2d *g, const float *ray_vecs, const void *img, void *sino, int batch,
                     ph_dtype dtype, void *stream);
int ph_project_cone3d(const ph_geom3d *g, const float *mats, const void *vol, void *proj, int batch,
                      ph_dtype dtype, void *stream);

/* ------------------------------------------------- back-projection B
 * Sec. II.B.2 (voxel-driven back-projection: every voxel accumulates the
 * interpolated value at its projection in every view).  Detector values are
 * interpolated linearly (2D) / bilinearly (3D) with zero outside the
 * detector; the sum is multiplied by dbeta = range/n_proj and, for fan and
 * cone beams, each term by the distance weight (SID/w)^2, w the depth of the
 * voxel along the central ray.  On the equiangular fan detector
 * (fan_detector = 1) the pixel is read at the bin of its fan angle and
 * weighted by (SID/L)^2, L its distance from the source (Kak & Slaney's
 * equiangular reconstruction).  Same arrays as the forward calls with the
 * roles of input and output exchanged. */
int ph_backproject_par2d(const ph_geom2d *g, const float *ray_vecs, const void *sino, void *img, int batch,
                         ph_dtype dtype, void *stream);
int ph_backproject_fan2d(const ph_geom2d *g, const float *ray_vecs, const void *sino, void *img, int batch,
                         ph_dtype dtype, void *stream);
int ph_backproject_cone3d(const ph_geom3d *g, const float *mats, const void *proj, void *vol, int batch,
                          ph_dtype dtype, void *stream);

/* ------------------------------------------------- exact transposes
 * Sec. II.B.2: the ray-driven projector and the voxel-driven back-projector
 * are an unmatched pair; Sec. II.B.1 (after Eq. 4) uses each operator's
 * adjoint for the gradient.  These are the exact transposes of the two
 * operators above, for matched gradients.
 *
 * ph_project_adjoint_*: A^T, volume_x = step * sum_r g_r sum_k Lambda(X_rk - x)
 * over the same sample positions X_rk as ph_project_* (Lambda the bi/trilinear
 * hat function).  Gather, no atomics; any storage dtype.
 *   sino/proj : device input, same layout as the projector's output
 *   img/vol   : device output, same layout as the projector's input
 * ph_backproject_adjoint_*: B^T, projection_(k,i,j) = dbeta * sum_x f(x)
 * w_k(x) Lambda(j - su_k(x)) Lambda(i - sv_k(x)) with w_k = 1 (parallel) or
 * (SID/w)^2.  Scatter with float atomics: FP32 storage here (other dtypes ->
 * PH_ERR_UNSUPPORTED; the _ws variants below take them); summation order,
 * hence the last bits, may vary from run to run.
 *   img/vol   : device FP32 input; sino/proj : device FP32 output */
int ph_project_adjoint_par2d(const ph_geom2d *g, const float *ray_vecs, const void *sino, void *img, int batch,
                             ph_dtype dtype, void *stream);
int ph_project_adjoint_fan2d(const ph_geom2d *g, const float *ray_vecs, const void *sino, void *img, int batch,
                             ph_dtype dtype, void *stream);
int ph_project_adjoint_cone3d(const ph_geom3d *g, const float *mats, const void *proj, void *vol, int batch,
                              ph_dtype dtype, void *stream);
int ph_backproject_adjoint_par2d(const ph_geom2d *g, const float *ray_vecs, const void *img, void *sino, int batch,
                                 ph_dtype dtype, void *stream);
int ph_backproject_adjoint_fan2d(const ph_geom2d *g, const float *ray_vecs, const void *img, void *sino, int batch,
                                 ph_dtype dtype, void *stream);
int ph_backproject_adjoint_cone3d(const ph_geom3d *g, const float *mats, const void *vol, void *proj, int batch,
                                  ph_dtype dtype, void *stream);

/* B^T with any storage type (extension 1): the scatter accumulates in FP32,
 * in the output itself for FP32 and otherwise in the workspace `ws` of
 * ph_backproject_adjoint_workspace_bytes_*() bytes (0 for FP32, where ws may
 * be NULL), which is then rounded to the storage type (nearest even). */
size_t ph_backproject_adjoint_workspace_bytes_2d(const ph_geom2d *g, int batch, ph_dtype dtype);
size_t ph_backproject_adjoint_workspace_bytes_3d(const ph_geom3d *g, int batch, ph_dtype dtype);
int ph_backproject_adjoint_ws_par2d(const ph_geom2d *g, const float *ray_vecs, const void *img, void *sino, void *ws,
                                    size_t ws_bytes, int batch, ph_dtype dtype, void *stream);
int ph_backproject_adjoint_ws_fan2d(const ph_geom2d *g, const float *ray_vecs, const void *img, void *sino, void *ws,
                                    size_t ws_bytes, int batch, ph_dtype dtype, void *stream);
int ph_backproject_adjoint_ws_cone3d(const ph_geom3d *g, const float *mats, const void *vol, void *proj, void *ws,
                                     size_t ws_bytes, int batch, ph_dtype dtype, void *stream);

/* --------------------------------------------- weighting + ramp filtering
 * Eq. 4 / Eq. 5 without the back-projection: q = F^H K F (W_red * W_cos * W * p),
 * row by row (detector rows along u).  Sec. II.C.4 (Ramp / Ram-Lak filters as
 * a diagonal multiply in the Fourier domain), Sec. II.C.5 (cosine and
 * redundancy weights).
 *   K     : device float[M] real response on the M-point DFT grid, or NULL for
 *           Ram-Lak with sample spacing tau (du for parallel, du*SID/SDD for
 *           fan/cone) and M = smallest power of two >= 2*nu-1 (then the row
 *           filter is an exact linear convolution);  M must be a power of two
 *           in [max(16, nu), 4096];  with K given the output is
 *           Re IDFT_M(K . DFT_M(zero-padded row)), first nu samples;
 *   W_red : device float[n_proj][nu] or NULL -> parallel: pi/range;
 *           fan/cone: 1/2 for a full turn, Parker for a short scan;
 *   W     : device float[nv][nu] extra per-pixel weight or NULL (3D only);
 *   out   : device float[batch][n_proj](nv)[nu], FP32 regardless of dtype.
 * M = 0 with K = NULL selects the default length. */
int ph_weight_filter_2d(const ph_geom2d *g, int fan, const void *sino, float *out, const float *K, int M,
                        const float *W_red, int batch, ph_dtype dtype, void *stream);

/* Filter responses on the M-point DFT grid for the K argument above
 * (Sec. II.C.4; Sec. III.B initialises the learned filter with the ramp).
 * Host only.  kind 0: Ram-Lak, the DFT of the taps h(0) = 1/(4 tau^2),
 * h(n odd) = -1/(n pi tau)^2, h(n even) = 0 for |n| <= M/2, times tau;
 * kind 1: the ramp |f| sampled on the grid, K[k] = min(k, M-k) / (M tau).
 * tau is the iso-centre sample spacing (du for parallel beams, du*SID/SDD
 * for fan and cone beams).  K: host float[M]; M a power of two in [2, 4096],
 * tau > 0 and finite. */
int ph_filter_response(int kind, int M, double tau, float *K);
/* Equiangular Ram-Lak response for the curved fan detector (Kak & Slaney,
 * equiangular rays): the DFT on the M-point grid of the taps t(0) =
 * 1/(4 alpha SID), t(n odd) = -alpha / (pi^2 SID sin^2(n alpha)), t(n even)
 * = 0 for |n| <= M/2 (the ramp kernel of the fan angle times
 * (gamma/sin gamma)^2, with the pre-weight's SID and the step alpha folded
 * in).  alpha = du/SDD is the angular pitch of the bins.  Host only.
 * K: host float[M]; M a power of two in [2, 4096]; alpha in (0, pi/M] and
 * SID > 0, finite. */
int ph_filter_response_equiangular(int M, double alpha, double sid, float *K);
int ph_weight_filter_3d(const ph_geom3d *g, const void *proj, float *out, const float *K, int M,
                        const float *W_red, const float *W, int batch, ph_dtype dtype, void *stream);

/* ------------------------------------------------------- FBP / FDK
 * Eq. 4 (FBP) and Eq. 5 (FDK network): x = B F^H K F W_red W_cos p.
 * Defaults: Ram-Lak K; W_cos the cosine weight SDD / sqrt(SDD^2 + u^2 + v^2)
 * (cos(gamma_j) and the equiangular Ram-Lak response on the equiangular fan
 * detector); W_red 1/2 for a full turn of a fan or cone scan, Parker for a
 * short scan (at the bins' fan angles), pi/range for parallel beams.
 * Workspace: ws of ws_bytes >= ph_workspace_bytes_*() device bytes holds the
 * filtered projections. */
size_t ph_workspace_bytes_2d(const ph_geom2d *g, int batch);
size_t ph_workspace_bytes_3d(const ph_geom3d *g, int batch);
/* Workspace of ph_fdk_cone3d for filter length M (0 = the default Ram-Lak
 * length) and storage type dtype, in bytes: the filtered projections are
 * held in FP32 whatever M and dtype, so this equals ph_workspace_bytes_3d.
 * Returns 0 for an invalid geometry, batch, M or dtype. */
size_t ph_fdk_workspace_bytes(const ph_geom3d *g, int M, int batch, ph_dtype dtype);

int ph_fbp_par2d(const ph_geom2d *g, const float *ray_vecs, const void *sino, void *img, const float *K, int M,
                 const float *W_red, void *ws, size_t ws_bytes, int batch, ph_dtype dtype, void *stream);
int ph_fbp_fan2d(const ph_geom2d *g, const float *ray_vecs, const void *sino, void *img, const float *K, int M,
                 const float *W_red, void *ws, size_t ws_bytes, int batch, ph_dtype dtype, void *stream);
int ph_fdk_cone3d(const ph_geom3d *g, const float *mats, const void *proj, void *vol, const float *K, int M,
                  const float *W_red, const float *W, void *ws, size_t ws_bytes, int batch, ph_dtype dtype,
                  void *stream);

/* ph_fdk_cone3d for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments without ws / ws_bytes and the same result, to the
 * rounding of the sums, with no hipMalloc, hipFree or allocating library
 * call.  Its scratch is a static device array of PH_FDK_STATIC_SCRATCH_BYTES
 * per GPU, held from the first call on that GPU until the process ends: the
 * per-view tables (back-projector rows, the default Ram-Lak response and
 * redundancy weights, FFT twiddles), then the filtered projections of as
 * many views as fit, which are back-projected in shares (each share adds to
 * vol).  The tables are copied from the host, followed by a synchronisation
 * of `stream`, whenever they differ from the ones the array holds.  Errors:
 * PH_ERR_WORKSPACE when the tables and one view's filtered projections
 * (batch * nv * nu * 4 bytes) do not fit, or when an FP16 / BF16 volume
 * would need more than one share (a share adds to the stored volume, which
 * half precision would round each time); the other errors as ph_fdk_cone3d.
 * Every call on a GPU uses that GPU's one array: calls whose work overlaps
 * on one GPU (other streams, other host threads) race. */
#define PH_FDK_STATIC_SCRATCH_BYTES (64u << 20)
int ph_fdk_cone3d_static(const ph_geom3d *g, const float *mats, const void *proj, void *vol, const float *K, int M,
                         const float *W_red, const float *W, int batch, ph_dtype dtype, void *stream);

/* ------------------------------------------- learned corrector training
 * The FDK network of Eq. 5 with trainable projection-domain parameters:
 * Sec. III.A lets the redundancy weights be learned from a loss computed in
 * the volume (the update follows Wurfl et al.), Sec. III.B / Eq. 6 trains the
 * filter K, initialised with the ramp.  The corrected reconstruction is
 *     x = B q,   q = F^H K F r,   r = W * W_red * W_cos * p
 * (ph_weight_filter_3d then ph_backproject_cone3d, or ph_fdk_cone3d).  Its
 * gradient runs backwards through the same operators: dL/dx from
 * ph_mse_grad, dL/dq = B^T dL/dx from ph_backproject_adjoint_cone3d, then
 * ph_corrector_grad_3d gives dL/dK and dL/dW, and ph_adam_step updates
 * them.  All FP32. */

/* L = (1/n) sum_i (m_i (x_i - ref_i))^2 and dL/dx_i = 2 m_i^2 (x_i - ref_i) / n
 * (m_i = mask[i], or 1 when mask is NULL).
 *   x, ref, grad : device float[n]; mask: device float[n] or NULL;
 *   loss         : device double[1], overwritten: FP32 partial sums per
 *                  workgroup, added in FP64 with atomics (the last bits may
 *                  vary from run to run);
 * n >= 1 (else PH_ERR_SHAPE).  grad may alias x, not ref. */
int ph_mse_grad(const float *x, const float *ref, const float *mask, size_t n, float *grad, double *loss,
                void *stream);

/* Gradients of L with respect to the filter K and the pixel weights W, given
 * grad_q = dL/dq for q = Re IDFT_M(K_s . DFT_M(r)) row by row, with
 * r = W * W_red * W_cos * proj and K_s[f] = (K[f] + K[(M - f) mod M]) / 2
 * (the symmetrised response every filter call applies):
 *   dL/dK[f]    = (1/2M) sum_rows Re(R_f conj(G_f) + R_{M-f} conj(G_{M-f})),
 *   dL/dW[i][j] = sum_{b,k} (dL/dr)[b][k][i][j] * W_red[k][j] * W_cos(i,j) * proj[b][k][i][j],
 *   dL/dr       = Re IDFT_M(K_s . DFT_M(grad_q))  (the filter's transpose),
 * with R = DFT_M(r), G = DFT_M(grad_q) over zero-padded rows.
 *   proj, grad_q : device float[batch][n_proj][nv][nu];
 *   K            : device float[M] (required), M a power of two in
 *                  [max(16, nu), 4096];
 *   W_red        : device float[n_proj][nu] or NULL (the default of
 *                  ph_weight_filter_3d); W: device float[nv][nu] or NULL (ones);
 *   dK           : device float[M] output; dW: device float[nv][nu] output or
 *                  NULL to skip it.
 * Partial sums are combined with float atomics: the last bits may vary from
 * run to run. */
int ph_corrector_grad_3d(const ph_geom3d *g, const float *proj, const float *grad_q, const float *K, int M,
                         const float *W_red, const float *W, float *dK, float *dW, int batch, void *stream);

/* The filter gradient of the 2D FBP network (Sec. III.B, Eq. 6: K is the
 * only trainable layer): dL/dK as above for q = F^H K F (W_red W_cos sino),
 * W_cos = 1 for parallel beams (fan = 0), SDD / sqrt(SDD^2 + u^2) for fan
 * beams.  sino, grad_q: device float[batch][n_proj][nu]; K, dK: device
 * float[M]; W_red: device float[n_proj][nu] or NULL (the default of
 * ph_weight_filter_2d). */
int ph_corrector_grad_2d(const ph_geom2d *g, int fan, const float *sino, const float *grad_q, const float *K, int M,
                         const float *W_red, float *dK, int batch, void *stream);

/* One Adam step (Kingma & Ba) on n parameters, in place:
 *   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
 *   param -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
 *   param, m, v : device float[n], updated; grad : device float[n];
 * t >= 1 is the step count (bias correction); lr > 0, b1 and b2 in [0, 1),
 * eps > 0, all finite (else PH_ERR_VALUE); n >= 1 (else PH_ERR_SHAPE). */
int ph_adam_step(float *param, const float *grad, float *m, float *v, size_t n, float lr, float beta1,
                 float beta2, float eps, int t, void *stream);

/* ---------------------------------------- TV-regularised iterative recon
 * Sec. III.B.1, Eq. 7: the image is the weight of an additive layer,
 * forward-projected and trained on the l2 data term plus lambda * TV(x).  One
 * iteration is ph_project_* (A x), ph_mse_grad (residual gradient),
 * ph_project_adjoint_* (A^T), ph_tv_3d (regulariser) and ph_adam_step.
 *
 * Total variation with forward differences D_d(q) = x[q + e_d] - x[q] (none
 * across the last row / column / plane) and smoothing eps:
 *   anisotropic = 0: TV(x) = sum_q sqrt(sum_d D_d(q)^2 + eps^2)  (eps > 0);
 *   anisotropic = 1: TV(x) = sum_q sum_d sqrt(D_d(q)^2 + eps^2) over the axes
 *     of extent > 1, the sum of absolute differences at eps = 0 (eps >= 0;
 *     the gradient takes sign(D), 0 at D = 0) -- the total variation of the
 *     framework Sec. III.B.1 computes TV with.
 *   vol   : device float[batch][nz][ny][nx] (nz = 1 for an image [ny][nx]);
 *   grad  : device float, same shape, or NULL: grad += weight * dTV/dx;
 *   value : device double[batch] or NULL: TV of each item (FP32 terms summed
 *           in FP64 with atomics, so the last bits may vary).
 * anisotropic 0 or 1, eps as above and weight finite (else PH_ERR_VALUE);
 * sizes and batch >= 1 (else PH_ERR_SHAPE).  grad must not alias vol. */
int ph_tv_3d(const float *vol, int nz, int ny, int nx, int batch, int anisotropic, float eps, float weight,
             float *grad, double *value, void *stream);

/* n_iter iterations of the TV-regularised reconstruction in one call (the
 * five steps above, issued from the library without a host round trip):
 *   L(x) = mean((A x - p)^2) + lam * TV_eps(x), Adam with steps t0+1 .. t0+n_iter.
 *   proj     : device float projections [batch][n_proj](nv)[nu] (measured p);
 *   x, m, v  : device float [batch] image / volume, Adam moments; updated;
 *   ws       : device workspace of ph_tv_workspace_bytes_*() bytes;
 *   data_tv  : device double[1 + batch] or NULL: the data term and the TV of
 *              each item at the iterate before the last update.
 * The operator is the matched pair (A, A^T) of the geometry.  Validation as
 * for the operators; t0 >= 0, n_iter >= 1 (else PH_ERR_SHAPE); lam >= 0,
 * eps as for ph_tv_3d, lr > 0, betas in [0, 1), adam_eps > 0, all finite,
 * anisotropic 0 or 1 (else PH_ERR_VALUE). */
typedef struct {
    float lam, eps;                      /* TV weight and smoothing */
    float lr, beta1, beta2, adam_eps;    /* Adam */
    int anisotropic;                     /* 0: isotropic TV, 1: sum of absolute differences (as ph_tv_3d) */
} ph_tv_params;

size_t ph_tv_workspace_bytes_2d(const ph_geom2d *g, int batch);
size_t ph_tv_workspace_bytes_3d(const ph_geom3d *g, int batch);
int ph_tv_iterate_par2d(const ph_geom2d *g, const float *ray_vecs, const float *proj, float *x, float *m, float *v,
                        int t0, int n_iter, const ph_tv_params *prm, void *ws, size_t ws_bytes, double *data_tv,
                        int batch, void *stream);
int ph_tv_iterate_fan2d(const ph_geom2d *g, const float *ray_vecs, const float *proj, float *x, float *m, float *v,
                        int t0, int n_iter, const ph_tv_params *prm, void *ws, size_t ws_bytes, double *data_tv,
                        int batch, void *stream);
int ph_tv_iterate_cone3d(const ph_geom3d *g, const float *mats, const float *proj, float *x, float *m, float *v,
                         int t0, int n_iter, const ph_tv_params *prm, void *ws, size_t ws_bytes, double *data_tv,
                         int batch, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PYROHIP_H */
