/*
 * oracle.c -- plain, slow FP64 CPU reference of the known-operator CT path of
 * PYRO-NN (arXiv 1904.13342): ray-driven forward projection, its exact
 * transpose, voxel-driven distance-weighted back-projection, its exact
 * transpose, the ramp filters and the geometric weights.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the HIP library.
 *
 * Geometry (the paper names the attributes in Sec. II.C.1 and the trajectory
 * description in Sec. II.C.3; it gives no formulas, so these are the readings
 * used throughout):
 *   - voxel (ix,iy,iz) centre at world (ox+ix*sx, oy+iy*sy, oz+iz*sz) mm;
 *   - view k at angle beta_k = k*range/n_proj, counter-clockwise about +z;
 *     central ray vector c = (cos b, sin b, 0), detector axis e_u = (-sin b,
 *     cos b, 0), e_v = +z;
 *   - detector pixel (i,j) (row i, column j) centre u_j = (j-(nu-1)/2)*du,
 *     v_i = (i-(nv-1)/2)*dv;
 *   - parallel: ray through u_j*e_u with direction c;
 *   - fan / cone: source S = -SID*c, flat detector centred at (SDD-SID)*c;
 *   - curved fan (equiangular detector, Kak & Slaney's equiangular rays): the
 *     detector is the arc of radius SDD about the source, column j at fan
 *     angle gamma_j = (j-(nu-1)/2)*du/SDD from the central ray (du is the
 *     arc length between columns), direction cos(g)*c + sin(g)*e_u.
 * 2D geometries are the nz = 1, z = 0 special case of the same code: with
 * z = 0 the trilinear interpolation below reduces exactly to bilinear.
 *
 * Trajectories given as projection matrices (Sec. II.C.3: a trajectory is
 * a set of projection matrices, as calibrated on real scanners): view k's
 * 3x4 matrix P maps homogeneous world mm to (j*w, i*w, w), detector column j
 * and row i.  It is first rescaled so that the 3-vector of its third row has
 * unit length and w > 0 at the centre of the volume grid: w is then the
 * depth in mm of a point in front of the source along the principal ray.
 * The source is the point P sends to zero, S = -M^-1 p4 (M the left 3x3
 * block, p4 the last column); the ray of pixel (i,j) runs along M^-1 (j,i,1);
 * its anchor is its point closest to the world origin (the isocentre); the
 * distance weight of the back-projector is (SID/w)^2 with the nominal SID.
 *
 * Parity unpinned: none.  Every function is pinned by the CPU test-suite
 * against closed forms, brute force or exact invariants.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int kind;          /* 0 parallel 2D, 1 fan 2D (flat detector), 2 circular cone 3D,
                          3 fan 2D (curved equiangular detector) */
    int nx, ny, nz;    /* grid size; nz = 1 in 2D */
    double sx, sy, sz; /* voxel spacing, mm */
    double ox, oy, oz; /* world position of the centre of voxel (0,0,0), mm */
    int nu, nv;        /* detector columns and rows; nv = 1 in 2D */
    double du, dv;     /* detector pixel spacing, mm */
    int n_proj;        /* number of views */
    double range;      /* angular range, rad */
    double sid, sdd;   /* source-isocentre and source-detector distance, mm */
    double step;       /* ray sampling step (mm) of the forward projector */
    const double *mats; /* kind 2 only: NULL for the circular trajectory, else [n_proj][3][4]
                           projection matrices taken as data (any non-zero scale) */
} ora_geom;

int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---------------------------------------------------------------- geometry */

static void view_frame(const ora_geom *g, int k, double c[3], double eu[3])
{
    double beta = g->range * (double)k / (double)g->n_proj;
    c[0] = cos(beta);
    c[1] = sin(beta);
    c[2] = 0.0;
    eu[0] = -c[1];
    eu[1] = c[0];
    eu[2] = 0.0;
}

/* Determinant of the 3x3 block of a row-major 3x4 matrix. */
static double det3(const double *m)
{
    return m[0] * (m[5] * m[10] - m[6] * m[9]) - m[1] * (m[4] * m[10] - m[6] * m[8]) +
           m[2] * (m[4] * m[9] - m[5] * m[8]);
}

/* View k's projection matrix taken as data, rescaled: third row of the 3x3
 * block of unit length, w > 0 at the centre of the volume grid. */
static void view_matrix(const ora_geom *g, int k, double P[12])
{
    const double *m = g->mats + (size_t)k * 12;
    const double cx = g->ox + 0.5 * (g->nx - 1) * g->sx, cy = g->oy + 0.5 * (g->ny - 1) * g->sy,
                 cz = g->oz + 0.5 * (g->nz - 1) * g->sz;
    double s = 1.0 / sqrt(m[8] * m[8] + m[9] * m[9] + m[10] * m[10]);
    if (m[8] * cx + m[9] * cy + m[10] * cz + m[11] < 0.0)
        s = -s;
    for (int t = 0; t < 12; ++t)
        P[t] = s * m[t];
}

/* Solution x of M x = b, M the 3x3 block of P, by Cramer's rule. */
static void solve3(const double P[12], const double b[3], double x[3])
{
    double D = det3(P);
    for (int c = 0; c < 3; ++c) {
        double Q[12];
        memcpy(Q, P, sizeof(Q));
        for (int r = 0; r < 3; ++r)
            Q[r * 4 + c] = b[r];
        x[c] = det3(Q) / D;
    }
}

/* Ray of detector pixel (i,j) in view k: anchor a (the point of the line
 * closest to the isocentre) and unit direction d.  Sec. II.B.2: one ray per
 * detector pixel, cast through the scene. */
static void ray_of(const ora_geom *g, int k, int i, int j, double a[3], double d[3])
{
    if (g->kind == 2 && g->mats) {
        /* source S = -M^-1 p4, direction M^-1 (j, i, 1), anchor closest to
         * the world origin */
        double P[12], s[3], n = 0.0, sd = 0.0;
        view_matrix(g, k, P);
        const double p4[3] = {-P[3], -P[7], -P[11]}, pix[3] = {(double)j, (double)i, 1.0};
        solve3(P, p4, s);
        solve3(P, pix, d);
        for (int t = 0; t < 3; ++t)
            n += d[t] * d[t];
        n = sqrt(n);
        for (int t = 0; t < 3; ++t) {
            d[t] /= n;
            sd += s[t] * d[t];
        }
        for (int t = 0; t < 3; ++t)
            a[t] = s[t] - sd * d[t];
        return;
    }
    double c[3], eu[3];
    view_frame(g, k, c, eu);
    double u = ((double)j - 0.5 * (g->nu - 1)) * g->du;
    double v = ((double)i - 0.5 * (g->nv - 1)) * g->dv;
    if (g->kind == 0) {
        for (int t = 0; t < 3; ++t) {
            a[t] = u * eu[t];
            d[t] = c[t];
        }
        return;
    }
    double s[3], p[3];
    for (int t = 0; t < 3; ++t) {
        s[t] = -g->sid * c[t];
        p[t] = (g->sdd - g->sid) * c[t] + u * eu[t];
    }
    p[2] += v;
    if (g->kind == 3) {
        /* the column's point on the arc of radius SDD about the source */
        double gam = u / g->sdd;
        for (int t = 0; t < 3; ++t)
            p[t] = s[t] + g->sdd * (cos(gam) * c[t] + sin(gam) * eu[t]);
    }
    double n = 0.0;
    for (int t = 0; t < 3; ++t) {
        d[t] = p[t] - s[t];
        n += d[t] * d[t];
    }
    n = sqrt(n);
    double sd = 0.0;
    for (int t = 0; t < 3; ++t) {
        d[t] /= n;
        sd += s[t] * d[t];
    }
    for (int t = 0; t < 3; ++t)
        a[t] = s[t] - sd * d[t];
}

/* Index coordinates of the k-th sample a + k*step*d: X(k) = p0 + k*e per axis. */
static void sample_line(const ora_geom *g, const double a[3], const double d[3], double p0[3], double e[3])
{
    const double o[3] = {g->ox, g->oy, g->oz};
    const double s[3] = {g->sx, g->sy, g->sz};
    for (int t = 0; t < 3; ++t) {
        p0[t] = (a[t] - o[t]) / s[t];
        e[t] = g->step * d[t] / s[t];
    }
}

/* Range of k whose sample lies in the open box (-1, N) on every axis, widened
 * to integers: [k0, k1].  Outside that box the interpolated volume is exactly
 * zero, so a wider k range adds exact zeros.  Returns 0 if the ray misses. */
static int k_range(const ora_geom *g, const double p0[3], const double e[3], long *k0, long *k1)
{
    const int n[3] = {g->nx, g->ny, g->nz};
    double lo = -INFINITY, hi = INFINITY;
    for (int t = 0; t < 3; ++t) {
        if (e[t] == 0.0) {
            if (!(p0[t] > -1.0 && p0[t] < (double)n[t]))
                return 0;
            continue;
        }
        double t1 = (-1.0 - p0[t]) / e[t], t2 = ((double)n[t] - p0[t]) / e[t];
        if (t1 > t2) {
            double tmp = t1;
            t1 = t2;
            t2 = tmp;
        }
        if (t1 > lo)
            lo = t1;
        if (t2 < hi)
            hi = t2;
    }
    if (!(lo < hi))
        return 0;
    *k0 = (long)floor(lo);
    *k1 = (long)ceil(hi);
    return 1;
}

/* -------------------------------------------------------- interpolation */

static double voxel(const ora_geom *g, const double *f, long ix, long iy, long iz)
{
    if (ix < 0 || iy < 0 || iz < 0 || ix >= g->nx || iy >= g->ny || iz >= g->nz)
        return 0.0;
    return f[((size_t)iz * g->ny + (size_t)iy) * g->nx + (size_t)ix];
}

/* Trilinear interpolation of the zero-padded grid at index coordinates (X,Y,Z). */
static double interp3(const ora_geom *g, const double *f, double X, double Y, double Z)
{
    double fx = floor(X), fy = floor(Y), fz = floor(Z);
    long ix = (long)fx, iy = (long)fy, iz = (long)fz;
    double tx = X - fx, ty = Y - fy, tz = Z - fz;
    double acc = 0.0;
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                double w = (cx ? tx : 1.0 - tx) * (cy ? ty : 1.0 - ty) * (cz ? tz : 1.0 - tz);
                acc += w * voxel(g, f, ix + cx, iy + cy, iz + cz);
            }
    return acc;
}

/* Transpose of interp3: add val * (trilinear weight) into each in-range corner. */
static void scatter3(const ora_geom *g, double *f, double X, double Y, double Z, double val)
{
    double fx = floor(X), fy = floor(Y), fz = floor(Z);
    long ix = (long)fx, iy = (long)fy, iz = (long)fz;
    double tx = X - fx, ty = Y - fy, tz = Z - fz;
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                long jx = ix + cx, jy = iy + cy, jz = iz + cz;
                if (jx < 0 || jy < 0 || jz < 0 || jx >= g->nx || jy >= g->ny || jz >= g->nz)
                    continue;
                double w = (cx ? tx : 1.0 - tx) * (cy ? ty : 1.0 - ty) * (cz ? tz : 1.0 - tz);
                f[((size_t)jz * g->ny + (size_t)jy) * g->nx + (size_t)jx] += w * val;
            }
}

static double pixel(const ora_geom *g, const double *q, long i, long j)
{
    if (i < 0 || j < 0 || i >= g->nv || j >= g->nu)
        return 0.0;
    return q[(size_t)i * g->nu + (size_t)j];
}

/* Bilinear interpolation of one zero-padded detector image at column
 * coordinate su and row coordinate sv (row 0 with sv = 0 is linear in 2D). */
static double interp_det(const ora_geom *g, const double *q, double su, double sv)
{
    double fu = floor(su), fv = floor(sv);
    long j = (long)fu, i = (long)fv;
    double tu = su - fu, tv = sv - fv;
    return (1.0 - tv) * ((1.0 - tu) * pixel(g, q, i, j) + tu * pixel(g, q, i, j + 1)) +
           tv * ((1.0 - tu) * pixel(g, q, i + 1, j) + tu * pixel(g, q, i + 1, j + 1));
}

static void scatter_det(const ora_geom *g, double *q, double su, double sv, double val)
{
    double fu = floor(su), fv = floor(sv);
    long j = (long)fu, i = (long)fv;
    double tu = su - fu, tv = sv - fv;
    for (int ci = 0; ci < 2; ++ci)
        for (int cj = 0; cj < 2; ++cj) {
            long ii = i + ci, jj = j + cj;
            if (ii < 0 || jj < 0 || ii >= g->nv || jj >= g->nu)
                continue;
            q[(size_t)ii * g->nu + (size_t)jj] += (ci ? tv : 1.0 - tv) * (cj ? tu : 1.0 - tu) * val;
        }
}

/* ------------------------------------------------ forward projection  A */

/* (A f)_r = step * sum_k f~(a_r + k*step*d_r), Sec. II.B.2 (ray-driven
 * forward projection: per detector pixel, absorption accumulated along the
 * ray).  p is [n_proj][nv][nu]; only the listed views are written (all if
 * views == NULL). */
void ora_project(const ora_geom *g, const double *f, double *p, const int *views, int nviews)
{
    int nsel = views ? nviews : g->n_proj;
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int s = 0; s < nsel; ++s)
        for (int i = 0; i < g->nv; ++i) {
            int k = views ? views[s] : s;
            for (int j = 0; j < g->nu; ++j) {
                double a[3], d[3], p0[3], e[3];
                long k0, k1;
                double acc = 0.0;
                ray_of(g, k, i, j, a, d);
                sample_line(g, a, d, p0, e);
                if (k_range(g, p0, e, &k0, &k1))
                    for (long m = k0; m <= k1; ++m)
                        acc += interp3(g, f, p0[0] + m * e[0], p0[1] + m * e[1], p0[2] + m * e[2]);
                p[((size_t)k * g->nv + i) * g->nu + j] = g->step * acc;
            }
        }
}

/* Exact transpose A^T, by scatter: (A^T q)_x = step * sum_r q_r sum_k
 * Lambda(X_rk - x).  Each thread scatters into a private volume. */
void ora_project_adjoint(const ora_geom *g, const double *p, double *f)
{
    size_t nvox = (size_t)g->nx * g->ny * g->nz;
    memset(f, 0, nvox * sizeof(double));
#pragma omp parallel
    {
        double *loc = (double *)calloc(nvox, sizeof(double));
#pragma omp for collapse(2) schedule(dynamic)
        for (int k = 0; k < g->n_proj; ++k)
            for (int i = 0; i < g->nv; ++i)
                for (int j = 0; j < g->nu; ++j) {
                    double a[3], d[3], p0[3], e[3];
                    long k0, k1;
                    double val = g->step * p[((size_t)k * g->nv + i) * g->nu + j];
                    if (val == 0.0)
                        continue;
                    ray_of(g, k, i, j, a, d);
                    sample_line(g, a, d, p0, e);
                    if (k_range(g, p0, e, &k0, &k1))
                        for (long m = k0; m <= k1; ++m)
                            scatter3(g, loc, p0[0] + m * e[0], p0[1] + m * e[1], p0[2] + m * e[2], val);
                }
#pragma omp critical
        for (size_t n = 0; n < nvox; ++n)
            f[n] += loc[n];
        free(loc);
    }
}

/* Number of samples with every index coordinate strictly inside (-1, N):
 * the implementation-independent work count of the forward projector. */
long long ora_count_samples(const ora_geom *g, const int *views, int nviews)
{
    int nsel = views ? nviews : g->n_proj;
    long long total = 0;
    const int n[3] = {g->nx, g->ny, g->nz};
#pragma omp parallel for collapse(2) reduction(+ : total) schedule(dynamic)
    for (int s = 0; s < nsel; ++s)
        for (int i = 0; i < g->nv; ++i) {
            int k = views ? views[s] : s;
            for (int j = 0; j < g->nu; ++j) {
                double a[3], d[3], p0[3], e[3];
                long k0, k1;
                ray_of(g, k, i, j, a, d);
                sample_line(g, a, d, p0, e);
                if (!k_range(g, p0, e, &k0, &k1))
                    continue;
                for (long m = k0; m <= k1; ++m) {
                    int in = 1;
                    for (int t = 0; t < 3; ++t) {
                        double X = p0[t] + m * e[t];
                        if (!(X > -1.0 && X < (double)n[t]))
                            in = 0;
                    }
                    total += in;
                }
            }
        }
    return total;
}

/* ---------------------------------------------- back-projection  B */

/* Detector coordinates of world point x in view k: column coordinate su, row
 * coordinate sv, and the distance weight.  Parallel: orthogonal projection,
 * weight 1.  Fan / cone: central projection from the source, weight
 * (SID / w)^2 with w = depth of x along the central ray from the source.
 * Curved fan: the column of the fan angle of x, weight (SID / L)^2 with L the
 * distance of x from the source (Kak & Slaney's equiangular back-projection). */
static void project_point(const ora_geom *g, int k, const double x[3], double *su, double *sv, double *wt)
{
    if (g->kind == 2 && g->mats) {
        /* (j w, i w, w) = P [x; 1] with the rescaled matrix: w in mm */
        double P[12], h[3];
        view_matrix(g, k, P);
        for (int r = 0; r < 3; ++r)
            h[r] = P[r * 4] * x[0] + P[r * 4 + 1] * x[1] + P[r * 4 + 2] * x[2] + P[r * 4 + 3];
        *su = h[0] / h[2];
        *sv = h[1] / h[2];
        *wt = (g->sid / h[2]) * (g->sid / h[2]);
        return;
    }
    double c[3], eu[3];
    view_frame(g, k, c, eu);
    double xu = x[0] * eu[0] + x[1] * eu[1];
    if (g->kind == 0) {
        *su = xu / g->du + 0.5 * (g->nu - 1);
        *sv = 0.0;
        *wt = 1.0;
        return;
    }
    double w = x[0] * c[0] + x[1] * c[1] + g->sid;
    if (g->kind == 3) {
        /* fan angle of the ray through x, and 1/L^2 weighting (L = distance
         * from the source) written as (SID/L)^2 */
        *su = atan2(xu, w) * g->sdd / g->du + 0.5 * (g->nu - 1);
        *sv = 0.0;
        *wt = g->sid * g->sid / (w * w + xu * xu);
        return;
    }
    *su = g->sdd * xu / w / g->du + 0.5 * (g->nu - 1);
    *sv = (g->kind == 2) ? g->sdd * x[2] / w / g->dv + 0.5 * (g->nv - 1) : 0.0;
    *wt = (g->sid / w) * (g->sid / w);
}

/* Voxel-driven back-projection, Sec. II.B.2: for every voxel, the projection
 * of its centre on each view is interpolated and accumulated, times
 * dbeta = range / n_proj.  q is [n_proj][nv][nu], f is [nz][ny][nx]; only the
 * listed z slices are written (all if slices == NULL). */
void ora_backproject(const ora_geom *g, const double *q, double *f, const int *slices, int nslices)
{
    int nsel = slices ? nslices : g->nz;
    double dbeta = g->range / (double)g->n_proj;
#pragma omp parallel for collapse(2) schedule(dynamic)
    for (int s = 0; s < nsel; ++s)
        for (int iy = 0; iy < g->ny; ++iy) {
            int iz = slices ? slices[s] : s;
            for (int ix = 0; ix < g->nx; ++ix) {
                double x[3] = {g->ox + ix * g->sx, g->oy + iy * g->sy, g->oz + iz * g->sz};
                if (g->kind != 2)
                    x[2] = 0.0;
                double acc = 0.0;
                for (int k = 0; k < g->n_proj; ++k) {
                    double su, sv, wt;
                    project_point(g, k, x, &su, &sv, &wt);
                    acc += wt * interp_det(g, q + (size_t)k * g->nv * g->nu, su, sv);
                }
                f[((size_t)iz * g->ny + iy) * g->nx + ix] = dbeta * acc;
            }
        }
}

/* Exact transpose B^T, by scatter; views are independent, so each thread owns
 * whole views of the output. */
void ora_backproject_adjoint(const ora_geom *g, const double *f, double *q)
{
    double dbeta = g->range / (double)g->n_proj;
    size_t per_view = (size_t)g->nv * g->nu;
#pragma omp parallel for schedule(dynamic)
    for (int k = 0; k < g->n_proj; ++k) {
        double *qk = q + (size_t)k * per_view;
        memset(qk, 0, per_view * sizeof(double));
        for (int iz = 0; iz < g->nz; ++iz)
            for (int iy = 0; iy < g->ny; ++iy)
                for (int ix = 0; ix < g->nx; ++ix) {
                    double val = f[((size_t)iz * g->ny + iy) * g->nx + ix];
                    if (val == 0.0)
                        continue;
                    double x[3] = {g->ox + ix * g->sx, g->oy + iy * g->sy, g->oz + iz * g->sz};
                    if (g->kind != 2)
                        x[2] = 0.0;
                    double su, sv, wt;
                    project_point(g, k, x, &su, &sv, &wt);
                    scatter_det(g, qk, su, sv, dbeta * wt * val);
                }
    }
}

/* ---------------------------------------------------------------- filters */

/* Ram-Lak impulse response (Kak & Slaney), sample spacing tau. */
static double ramlak_tap(long n, double tau)
{
    if (n == 0)
        return 1.0 / (4.0 * tau * tau);
    if (n % 2 == 0)
        return 0.0;
    return -1.0 / ((double)n * (double)n * M_PI * M_PI * tau * tau);
}

/* Row-wise Ram-Lak filtering as a direct linear convolution (Sec. II.C.4; the
 * F^H K F of Eq. 4 with K the Ram-Lak response and enough zero padding):
 * out(j) = tau * sum_m h(j - m) in(m). */
void ora_ramlak_filter(int rows, int nu, double tau, const double *in, double *out)
{
#pragma omp parallel for schedule(static)
    for (int r = 0; r < rows; ++r) {
        const double *x = in + (size_t)r * nu;
        double *y = out + (size_t)r * nu;
        for (int j = 0; j < nu; ++j) {
            double acc = 0.0;
            for (int m = 0; m < nu; ++m)
                acc += ramlak_tap((long)j - m, tau) * x[m];
            y[j] = tau * acc;
        }
    }
}

/* Row-wise filtering with an arbitrary real frequency response K[0..M-1]
 * on the M-point DFT grid: out = Re IDFT_M(K . DFT_M(zero-padded row)),
 * first nu outputs, computed directly as the circular convolution of the
 * zero-padded row with hK[n] = (1/M) sum_k K[k] cos(2 pi k n / M). */
void ora_circular_filter(int rows, int nu, int M, const double *K, const double *in, double *out)
{
    double *hk = (double *)malloc((size_t)M * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int n = 0; n < M; ++n) {
        double acc = 0.0;
        for (int k = 0; k < M; ++k) {
            long kn = ((long)k * n) % M;
            acc += K[k] * cos(2.0 * M_PI * (double)kn / (double)M);
        }
        hk[n] = acc / (double)M;
    }
#pragma omp parallel for schedule(static)
    for (int r = 0; r < rows; ++r) {
        const double *x = in + (size_t)r * nu;
        double *y = out + (size_t)r * nu;
        for (int j = 0; j < nu; ++j) {
            double acc = 0.0;
            for (int m = 0; m < nu; ++m) {
                long n = ((long)j - m) % M;
                if (n < 0)
                    n += M;
                acc += hk[n] * x[m];
            }
            y[j] = acc;
        }
    }
    free(hk);
}

/* Frequency response of the Ram-Lak filter on the M-point grid:
 * K[k] = tau * sum_n h_w[n] e^{-2 pi i k n / M}, h_w the M-periodic
 * wrap of the taps (h_w[n] = h(min(n, M-n))), real because h is even. */
void ora_ramlak_response(int M, double tau, double *K)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < M; ++k) {
        double acc = 0.0;
        for (int n = 0; n < M; ++n) {
            long nn = n <= M / 2 ? n : n - M;
            long kn = ((long)k * n) % M;
            acc += ramlak_tap(nn, tau) * cos(2.0 * M_PI * (double)kn / (double)M);
        }
        K[k] = tau * acc;
    }
}

/* Naive ramp |w| sampled on the M-point grid (learned-filter initialisation,
 * Sec. III.B): K[k] = |k'| / (M tau), k' = k for k <= M/2 else M - k. */
void ora_ramp_response(int M, double tau, double *K)
{
    for (int k = 0; k < M; ++k) {
        int kk = k <= M / 2 ? k : M - k;
        K[k] = (double)kk / ((double)M * tau);
    }
}

/* Equiangular Ram-Lak taps (Kak & Slaney, equiangular rays): the ramp kernel
 * h of the fan angle times (gamma / sin gamma)^2, sampled at gamma = n*alpha,
 * with the equiangular pre-weight's SID and the quadrature step alpha folded
 * in (the 1/2 of a full turn is the redundancy weight):
 *   t(0) = 1 / (4 alpha SID),  t(n even) = 0,
 *   t(n odd) = -alpha / (pi^2 SID sin^2(n alpha)).
 * For small alpha these tend to the flat taps tau * h_tau(n), tau = alpha SID. */
static double equiangular_tap(long n, double alpha, double sid)
{
    if (n == 0)
        return 1.0 / (4.0 * alpha * sid);
    if (n % 2 == 0)
        return 0.0;
    double sn = sin((double)n * alpha);
    return -alpha / (M_PI * M_PI * sid * sn * sn);
}

/* Row-wise equiangular filtering as a direct linear convolution:
 * out(j) = sum_m t(j - m) in(m). */
void ora_equiangular_filter(int rows, int nu, double alpha, double sid, const double *in, double *out)
{
#pragma omp parallel for schedule(static)
    for (int r = 0; r < rows; ++r) {
        const double *x = in + (size_t)r * nu;
        double *y = out + (size_t)r * nu;
        for (int j = 0; j < nu; ++j) {
            double acc = 0.0;
            for (int m = 0; m < nu; ++m)
                acc += equiangular_tap((long)j - m, alpha, sid) * x[m];
            y[j] = acc;
        }
    }
}

/* Frequency response of the equiangular taps on the M-point grid (taps
 * wrapped M-periodically, as for the Ram-Lak response). */
void ora_equiangular_response(int M, double alpha, double sid, double *K)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < M; ++k) {
        double acc = 0.0;
        for (int n = 0; n < M; ++n) {
            long nn = n <= M / 2 ? n : n - M;
            long kn = ((long)k * n) % M;
            acc += equiangular_tap(nn, alpha, sid) * cos(2.0 * M_PI * (double)kn / (double)M);
        }
        K[k] = acc;
    }
}

/* ---------------------------------------------------------------- weights */

/* Cosine weights (Kak & Slaney), Sec. II.C.5 / Eq. 5 W_cos:
 * SDD / sqrt(SDD^2 + u^2 + v^2); cos(gamma_j) on the curved detector (the
 * factor SID of the equiangular pre-weight sits in the filter taps);
 * identically 1 for parallel beams. */
void ora_cosine_weights(const ora_geom *g, double *wc)
{
    for (int i = 0; i < g->nv; ++i)
        for (int j = 0; j < g->nu; ++j) {
            double u = ((double)j - 0.5 * (g->nu - 1)) * g->du;
            double v = ((double)i - 0.5 * (g->nv - 1)) * g->dv;
            if (g->kind == 3) {
                wc[(size_t)i * g->nu + j] = cos(u / g->sdd);
            } else if (g->kind == 2 || g->kind == 1) {
                if (g->kind == 1)
                    v = 0.0;
                wc[(size_t)i * g->nu + j] = g->sdd / sqrt(g->sdd * g->sdd + u * u + v * v);
            } else {
                wc[(size_t)i * g->nu + j] = 1.0;
            }
        }
}

/* Parker redundancy weight for a short scan of range pi + 2*delta at view
 * angle beta and fan angle gamma (Sec. II.C.5, Eq. 5 W_red). */
double ora_parker(double beta, double gamma, double delta)
{
    double a = delta - gamma, b = delta + gamma;
    if (a > 0.0 && beta < 2.0 * a) {
        double s = sin(0.25 * M_PI * beta / a);
        return s * s;
    }
    if (beta < M_PI - 2.0 * gamma)
        return 1.0;
    if (b > 0.0 && beta <= M_PI + 2.0 * delta) {
        double s = sin(0.25 * M_PI * (M_PI + 2.0 * delta - beta) / b);
        return s * s;
    }
    return 0.0;
}

/* Redundancy weights per (view, column), [n_proj][nu].  Parallel beams:
 * pi / range (1 for a half turn).  Fan / cone: 1/2 for a full turn, Parker
 * with delta = (range - pi)/2 for a short scan. */
void ora_redundancy_weights(const ora_geom *g, double *wr)
{
    int full = fabs(g->range - 2.0 * M_PI) <= 1e-6 * 2.0 * M_PI;
    double delta = 0.5 * (g->range - M_PI);
    for (int k = 0; k < g->n_proj; ++k) {
        double beta = g->range * (double)k / (double)g->n_proj;
        for (int j = 0; j < g->nu; ++j) {
            double w;
            if (g->kind == 0)
                w = M_PI / g->range;
            else if (full)
                w = 0.5;
            else {
                double u = ((double)j - 0.5 * (g->nu - 1)) * g->du;
                w = ora_parker(beta, g->kind == 3 ? u / g->sdd : atan(u / g->sdd), delta);
            }
            wr[(size_t)k * g->nu + j] = w;
        }
    }
}

/* Projection matrices of the circular trajectory, [n_proj][3][4], mapping
 * homogeneous world mm to (j*w, i*w, w) with w the depth along the central
 * ray: P = Kint [R | -R S], R rows (e_u; e_v; c). */
void ora_projection_matrices(const ora_geom *g, double *P)
{
    for (int k = 0; k < g->n_proj; ++k) {
        double c[3], eu[3], ev[3] = {0.0, 0.0, 1.0};
        view_frame(g, k, c, eu);
        double s[3] = {-g->sid * c[0], -g->sid * c[1], 0.0};
        double R[3][3], t[3];
        for (int a = 0; a < 3; ++a) {
            R[0][a] = eu[a];
            R[1][a] = ev[a];
            R[2][a] = c[a];
        }
        for (int r = 0; r < 3; ++r)
            t[r] = -(R[r][0] * s[0] + R[r][1] * s[1] + R[r][2] * s[2]);
        double Kint[3][3] = {{g->sdd / g->du, 0.0, 0.5 * (g->nu - 1)},
                             {0.0, g->sdd / g->dv, 0.5 * (g->nv - 1)},
                             {0.0, 0.0, 1.0}};
        double *Pk = P + (size_t)k * 12;
        for (int r = 0; r < 3; ++r) {
            for (int col = 0; col < 3; ++col)
                Pk[r * 4 + col] = Kint[r][0] * R[0][col] + Kint[r][1] * R[1][col] + Kint[r][2] * R[2][col];
            Pk[r * 4 + 3] = Kint[r][0] * t[0] + Kint[r][1] * t[1] + Kint[r][2] * t[2];
        }
    }
}
