// C-ABI entry points of libpyrohip: argument validation (on the host, before
// any HIP call), derivation of per-view kernel parameters in FP64, a small
// per-device cache of those parameters, and kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pyrohip.h"
#include "common.h"

using namespace ph;

namespace {

constexpr double kPi = 3.14159265358979323846;

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

// ------------------------------------------------------------------ caching
// Derived per-view tables are uploaded once per (device, content) and kept
// until the process ends (or evicted past kMaxEntries).  The key is the exact
// bytes of everything the table depends on.
//
// Several host threads may call the library at once.  A table handed out by
// cached() stays pinned by the calling thread until its entry point returns
// (CallScope), by which time the kernels that read it are enqueued; eviction
// only frees tables no thread has pinned, and hipFree waits for the device,
// so a table is never freed between its lookup and the launch that uses it.

struct Entry {
    int device;
    std::string key;
    void *ptr;
};
std::mutex g_mu;
std::vector<std::shared_ptr<Entry>> g_cache;
constexpr size_t kMaxEntries = 64;
thread_local std::vector<std::shared_ptr<Entry>> t_pins;

// Declared first in every entry point: releases the tables the call pinned.
struct CallScope {
    size_t mark;
    CallScope() : mark(t_pins.size()) {}
    ~CallScope()
    {
        std::lock_guard<std::mutex> lock(g_mu);
        t_pins.resize(mark);
    }
};

template <typename Build>
const void *cached(const std::string &key, Build build, int *status)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        *status = PH_ERR_HIP;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    for (size_t n = 0; n < g_cache.size(); ++n) {
        if (g_cache[n]->device == dev && g_cache[n]->key == key) {
            std::shared_ptr<Entry> e = g_cache[n];
            g_cache.erase(g_cache.begin() + (long)n);
            g_cache.push_back(e);
            t_pins.push_back(e);
            return e->ptr;
        }
    }
    std::vector<unsigned char> host = build();
    void *p = nullptr;
    if (hipMalloc(&p, host.size()) != hipSuccess) {
        *status = PH_ERR_HIP;
        return nullptr;
    }
    if (hipMemcpy(p, host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(p);
        *status = PH_ERR_HIP;
        return nullptr;
    }
    if (g_cache.size() >= kMaxEntries) {
        // the least recently used table that no thread has pinned (hipFree
        // waits for outstanding work that may still read it)
        for (size_t n = 0; n < g_cache.size(); ++n) {
            if (g_cache[n].use_count() == 1) {
                (void)hipFree(g_cache[n]->ptr);
                g_cache.erase(g_cache.begin() + (long)n);
                break;
            }
        }
    }
    auto e = std::make_shared<Entry>(Entry{dev, key, p});
    g_cache.push_back(e);
    t_pins.push_back(e);
    return p;
}

template <typename T>
std::vector<unsigned char> as_bytes(const std::vector<T> &v)
{
    std::vector<unsigned char> out(v.size() * sizeof(T));
    std::memcpy(out.data(), v.data(), out.size());
    return out;
}

template <typename T>
void append(std::string &key, const T *p, size_t n)
{
    key.append(reinterpret_cast<const char *>(p), n * sizeof(T));
}

// ------------------------------------------------------------- validation

int check_dtype(int dtype) { return (dtype == PH_F32 || dtype == PH_F16 || dtype == PH_BF16) ? PH_OK : PH_ERR_DTYPE; }

double default_step(double step, double smin) { return step > 0.0 ? step : 0.5 * smin; }

int make_geom2d(const ph_geom2d *g, bool fan, Geom2D *o)
{
    if (!g)
        return PH_ERR_NULL;
    if (g->vol_shape[0] < 1 || g->vol_shape[1] < 1 || g->det_shape < 1 || g->n_proj < 1)
        return PH_ERR_SHAPE;
    if (!finite_pos(g->vol_spacing[0]) || !finite_pos(g->vol_spacing[1]) || !finite_pos(g->det_spacing) ||
        !finite_pos(g->angular_range) || !std::isfinite(g->vol_origin[0]) || !std::isfinite(g->vol_origin[1]) ||
        !std::isfinite(g->step_mm))
        return PH_ERR_GEOMETRY;
    if (fan && !(finite_pos(g->sid) && std::isfinite(g->sdd) && g->sdd > g->sid))
        return PH_ERR_GEOMETRY;
    // equiangular detector: an arc of less than a half turn about the source
    if (fan && g->fan_detector != 0 &&
        (g->fan_detector != 1 || !((double)g->det_shape * g->det_spacing / g->sdd < kPi)))
        return PH_ERR_GEOMETRY;
    o->ny = g->vol_shape[0];
    o->nx = g->vol_shape[1];
    o->sy = g->vol_spacing[0];
    o->sx = g->vol_spacing[1];
    o->oy = g->vol_origin[0];
    o->ox = g->vol_origin[1];
    o->inv_sx = (float)(1.0 / g->vol_spacing[1]);
    o->inv_sy = (float)(1.0 / g->vol_spacing[0]);
    o->nu = g->det_shape;
    o->du = g->det_spacing;
    o->cu = 0.5f * (float)(g->det_shape - 1);
    o->n_proj = g->n_proj;
    o->sid = fan ? g->sid : 0.0f;
    o->sdd = fan ? g->sdd : 0.0f;
    o->curved = fan && g->fan_detector == 1 ? 1 : 0;
    o->step = (float)default_step(g->step_mm, std::fmin(g->vol_spacing[0], g->vol_spacing[1]));
    o->dbeta = (float)((double)g->angular_range / g->n_proj);
    return PH_OK;
}

int make_geom3d(const ph_geom3d *g, Geom3D *o)
{
    if (!g)
        return PH_ERR_NULL;
    for (int a = 0; a < 3; ++a)
        if (g->vol_shape[a] < 1)
            return PH_ERR_SHAPE;
    if (g->det_shape[0] < 1 || g->det_shape[1] < 1 || g->n_proj < 1)
        return PH_ERR_SHAPE;
    for (int a = 0; a < 3; ++a)
        if (!finite_pos(g->vol_spacing[a]) || !std::isfinite(g->vol_origin[a]))
            return PH_ERR_GEOMETRY;
    if (!finite_pos(g->det_spacing[0]) || !finite_pos(g->det_spacing[1]) || !finite_pos(g->angular_range) ||
        !std::isfinite(g->step_mm) || !finite_pos(g->sid) || !std::isfinite(g->sdd) || !(g->sdd > g->sid))
        return PH_ERR_GEOMETRY;
    o->nz = g->vol_shape[0];
    o->ny = g->vol_shape[1];
    o->nx = g->vol_shape[2];
    o->oz = g->vol_origin[0];
    o->oy = g->vol_origin[1];
    o->ox = g->vol_origin[2];
    o->sz = g->vol_spacing[0];
    o->sy = g->vol_spacing[1];
    o->sx = g->vol_spacing[2];
    o->inv_sz = (float)(1.0 / g->vol_spacing[0]);
    o->inv_sy = (float)(1.0 / g->vol_spacing[1]);
    o->inv_sx = (float)(1.0 / g->vol_spacing[2]);
    o->nv = g->det_shape[0];
    o->nu = g->det_shape[1];
    o->dv = g->det_spacing[0];
    o->du = g->det_spacing[1];
    o->cv = 0.5f * (float)(g->det_shape[0] - 1);
    o->cu = 0.5f * (float)(g->det_shape[1] - 1);
    o->n_proj = g->n_proj;
    o->sid = g->sid;
    o->sdd = g->sdd;
    o->step = (float)default_step(
        g->step_mm, std::fmin(g->vol_spacing[0], std::fmin(g->vol_spacing[1], g->vol_spacing[2])));
    o->dbeta = (float)((double)g->angular_range / g->n_proj);
    return PH_OK;
}

// Unit central-ray vectors of a 2D trajectory; for fan beams every view must
// see the whole image support (index box [-1, N]) in front of the source.
int views2d(const ph_geom2d *g, bool fan, const float *rv, std::vector<float2> *out)
{
    out->resize((size_t)g->n_proj);
    const double y0 = g->vol_origin[0] - g->vol_spacing[0], y1 = g->vol_origin[0] + g->vol_shape[0] * (double)g->vol_spacing[0];
    const double x0 = g->vol_origin[1] - g->vol_spacing[1], x1 = g->vol_origin[1] + g->vol_shape[1] * (double)g->vol_spacing[1];
    for (int k = 0; k < g->n_proj; ++k) {
        const double cx = rv[2 * k], cy = rv[2 * k + 1];
        const double n = std::sqrt(cx * cx + cy * cy);
        if (!std::isfinite(n) || n <= 0.0)
            return PH_ERR_GEOMETRY;
        (*out)[(size_t)k] = make_float2((float)(cx / n), (float)(cy / n));
        if (fan) {
            for (int c = 0; c < 4; ++c) {
                const double x = (c & 1) ? x1 : x0, y = (c & 2) ? y1 : y0;
                if (!(g->sid + (x * cx + y * cy) / n > 0.0))
                    return PH_ERR_GEOMETRY;
            }
        }
    }
    return PH_OK;
}

// Normalised projection matrices (w = depth in mm, positive in front of the
// source), checked to be finite and non-singular, with the whole volume
// support (index box [-1, N] per axis) in front of every source.
int normalised_mats(const ph_geom3d *g, const float *mats, std::vector<double> *P)
{
    P->assign((size_t)g->n_proj * 12, 0.0);
    double lo[3], hi[3], ctr[3];
    for (int a = 0; a < 3; ++a) {  // world x, y, z
        const int ai = 2 - a;
        lo[a] = g->vol_origin[ai] - g->vol_spacing[ai];
        hi[a] = g->vol_origin[ai] + g->vol_shape[ai] * (double)g->vol_spacing[ai];
        ctr[a] = g->vol_origin[ai] + 0.5 * (g->vol_shape[ai] - 1) * (double)g->vol_spacing[ai];
    }
    for (int k = 0; k < g->n_proj; ++k) {
        double m[12];
        for (int t = 0; t < 12; ++t) {
            m[t] = mats[12 * k + t];
            if (!std::isfinite(m[t]))
                return PH_ERR_GEOMETRY;
        }
        const double det = m[0] * (m[5] * m[10] - m[6] * m[9]) - m[1] * (m[4] * m[10] - m[6] * m[8]) +
                           m[2] * (m[4] * m[9] - m[5] * m[8]);
        const double n0 = std::sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
        const double n1 = std::sqrt(m[4] * m[4] + m[5] * m[5] + m[6] * m[6]);
        const double n2 = std::sqrt(m[8] * m[8] + m[9] * m[9] + m[10] * m[10]);
        if (!(n2 > 0.0) || !(std::fabs(det) > 1e-9 * n0 * n1 * n2))
            return PH_ERR_GEOMETRY;
        double s = 1.0 / n2;
        if (m[8] * ctr[0] + m[9] * ctr[1] + m[10] * ctr[2] + m[11] < 0.0)
            s = -s;
        for (int t = 0; t < 12; ++t)
            (*P)[12 * (size_t)k + t] = s * m[t];
        const double *r2 = &(*P)[12 * (size_t)k + 8];
        for (int c = 0; c < 8; ++c) {
            const double x = (c & 1) ? hi[0] : lo[0], y = (c & 2) ? hi[1] : lo[1], z = (c & 4) ? hi[2] : lo[2];
            if (!(r2[0] * x + r2[1] * y + r2[2] * z + r2[3] > 0.0))
                return PH_ERR_GEOMETRY;
        }
    }
    return PH_OK;
}

// Back-projector rows over centred voxel indices, and whether the trajectory
// is a rotation about z (no z term in the u and w rows); out64 receives the
// same rows in double precision.
void bp_views(const ph_geom3d *g, const std::vector<double> &P, std::vector<ConeBPView> *out, bool *axial,
              std::vector<ConeBPView64> *out64)
{
    const double cu = 0.5 * (g->det_shape[1] - 1), cv = 0.5 * (g->det_shape[0] - 1);
    const double s[3] = {g->vol_spacing[2], g->vol_spacing[1], g->vol_spacing[0]};
    double oc[3];
    for (int a = 0; a < 3; ++a)
        oc[a] = g->vol_origin[2 - a] + 0.5 * (g->vol_shape[2 - a] - 1) * (double)g->vol_spacing[2 - a];
    out->resize((size_t)g->n_proj);
    out64->resize((size_t)g->n_proj);
    *axial = true;
    for (int k = 0; k < g->n_proj; ++k) {
        const double *m = &P[12 * (size_t)k];
        double r[3][4];
        for (int t = 0; t < 4; ++t) {
            r[0][t] = m[t] - cu * m[8 + t];
            r[1][t] = m[4 + t] - cv * m[8 + t];
            r[2][t] = m[8 + t];
        }
        ConeBPView &v = (*out)[(size_t)k];
        ConeBPView64 &v64 = (*out64)[(size_t)k];
        for (int row = 0; row < 3; ++row) {
            for (int a = 0; a < 3; ++a)
                v64.r[row][a] = r[row][a] * s[a];
            v64.r[row][3] = r[row][0] * oc[0] + r[row][1] * oc[1] + r[row][2] * oc[2] + r[row][3];
            for (int a = 0; a < 4; ++a)
                v.r[row][a] = (float)v64.r[row][a];
        }
        if (v.r[0][2] != 0.0f || v.r[2][2] != 0.0f)
            *axial = false;
    }
}

// Deeper column segment (32 or 16 voxels) whose 16 x 16 x NZ brick
// footprint fits the back-projector's 64 x 102 pixel LDS tile, from a bound on
// the magnification (nearest approach of a voxel to the source) and on the
// row slope across a brick at the top and bottom of the volume.
int bp_segment(const ph_geom3d *g)
{
    const double sz = g->vol_spacing[0], sy = g->vol_spacing[1], sx = g->vol_spacing[2];
    const double R = 0.5 * std::sqrt(std::pow((g->vol_shape[2] + 1) * sx, 2) + std::pow((g->vol_shape[1] + 1) * sy, 2));
    double zmax = 0.0;
    for (int e = -1; e <= g->vol_shape[0]; e += g->vol_shape[0] + 1)
        zmax = std::fmax(zmax, std::fabs(g->vol_origin[0] + e * sz));
    const double wmin = g->sid - R;
    if (!(wmin > 0.0))
        return 16;
    const double mag = g->sdd / wmin;
    const double brick = 16.0 * std::sqrt(2.0) * std::fmax(sx, sy);
    const double tw = brick * mag / g->det_spacing[1] + 4.0;
    const double slope = zmax * g->sdd / g->det_spacing[0] * brick / (wmin * wmin);
    for (int nz = 32; nz >= 32; nz /= 2) {
        const double th = nz * sz * mag / g->det_spacing[0] + slope + 4.0;
        if (tw <= 64.0 && th <= 102.0)   // the back-projector's LDS tile: 64 x 102 pixels
            return nz;
    }
    return 16;
}

// Forward-projector rays: source S = -M^-1 p4 and the direction
// M^-1 (j, i, 1) written around the detector centre.
void fp_views(const ph_geom3d *g, const std::vector<double> &P, std::vector<ConeFPView> *out)
{
    const double cu = 0.5 * (g->det_shape[1] - 1), cv = 0.5 * (g->det_shape[0] - 1);
    const float step = (float)default_step(
        g->step_mm, std::fmin(g->vol_spacing[0], std::fmin(g->vol_spacing[1], g->vol_spacing[2])));
    out->resize((size_t)g->n_proj);
    for (int k = 0; k < g->n_proj; ++k) {
        const double *m = &P[12 * (size_t)k];
        const double a = m[0], b = m[1], c = m[2], d = m[4], e = m[5], f = m[6], gg = m[8], h = m[9], i = m[10];
        const double det = a * (e * i - f * h) - b * (d * i - f * gg) + c * (d * h - e * gg);
        const double inv[3][3] = {{(e * i - f * h) / det, (c * h - b * i) / det, (b * f - c * e) / det},
                                  {(f * gg - d * i) / det, (a * i - c * gg) / det, (c * d - a * f) / det},
                                  {(d * h - e * gg) / det, (b * gg - a * h) / det, (a * e - b * d) / det}};
        double S[3], d0[3], du[3], dv[3];
        for (int r = 0; r < 3; ++r) {
            S[r] = -(inv[r][0] * m[3] + inv[r][1] * m[7] + inv[r][2] * m[11]);
            du[r] = inv[r][0];
            dv[r] = inv[r][1];
            d0[r] = cu * inv[r][0] + cv * inv[r][1] + inv[r][2];
        }
        ConeFPView &v = (*out)[(size_t)k];
        for (int r = 0; r < 3; ++r) {
            v.s[r] = S[r];
            v.d0[r] = d0[r];
            v.du[r] = du[r];
            v.dv[r] = dv[r];
            // the FP32 spacing and step the kernels see; x, y, z order
            const double sp = (double)(float)g->vol_spacing[2 - r];
            v.inv_sp[r] = 1.0 / sp;
            v.step_sp[r] = (double)step / sp;
        }
    }
}

// --------------------------------------------------------- filter tables

bool is_pow2(int m) { return m > 0 && (m & (m - 1)) == 0; }

int default_fft_size(int nu)
{
    int m = 16;
    while (m < 2 * nu - 1)
        m *= 2;
    return m;
}

int ilog2(int m)
{
    int l = 0;
    while ((1 << l) < m)
        ++l;
    return l;
}

double ramlak_tap(long n, double tau)
{
    if (n == 0)
        return 1.0 / (4.0 * tau * tau);
    if (n % 2 == 0)
        return 0.0;
    return -1.0 / ((double)n * (double)n * kPi * kPi * tau * tau);
}

std::vector<float> ramlak_response(int M, double tau)
{
    std::vector<float> K((size_t)M);
    for (int k = 0; k < M; ++k) {
        double acc = ramlak_tap(0, tau);
        for (int n = 1; n < M; n += 2) {  // odd taps only; even taps are zero
            const long nn = n <= M / 2 ? n : n - M;
            acc += ramlak_tap(nn, tau) * std::cos(2.0 * kPi * (double)(((long)k * n) % M) / M);
        }
        K[(size_t)k] = (float)(tau * acc);
    }
    return K;
}

const float *ramlak_table(int M, double tau, int *st)
{
    std::string key = "ramlak";
    append(key, &M, 1);
    append(key, &tau, 1);
    return (const float *)cached(key, [&] { return as_bytes(ramlak_response(M, tau)); }, st);
}

// Equiangular Ram-Lak (curved fan detector, Kak & Slaney's equiangular rays):
// the ramp kernel of the fan angle gamma = n alpha times (gamma / sin gamma)^2,
// with the SID of the equiangular pre-weight and the quadrature step alpha
// folded into the taps, wrapped M-periodically and transformed like the
// Ram-Lak response.
double equiangular_tap(long n, double alpha, double sid)
{
    if (n == 0)
        return 0.25 / (alpha * sid);
    if (n % 2 == 0)
        return 0.0;
    const double sn = std::sin((double)n * alpha);
    return -alpha / (kPi * kPi * sid * sn * sn);
}

// Taps with |n| > nmax are left out (n alpha stays below pi, where sin has no
// zero); a row of nu bins filtered by linear convolution only meets lags
// |n| <= nu - 1, so the default table stops there.
std::vector<float> equiangular_response(int M, double alpha, double sid, long nmax)
{
    std::vector<float> K((size_t)M);
    for (int k = 0; k < M; ++k) {
        double acc = equiangular_tap(0, alpha, sid);
        for (int n = 1; n < M; ++n) {
            const long nn = n <= M / 2 ? n : n - M;
            if (nn > nmax || -nn > nmax)
                continue;
            acc += equiangular_tap(nn, alpha, sid) * std::cos(2.0 * kPi * (double)(((long)k * n) % M) / M);
        }
        K[(size_t)k] = (float)acc;
    }
    return K;
}

const float *equiangular_table(int M, double alpha, double sid, int nu, int *st)
{
    std::string key = "eqang";
    append(key, &M, 1);
    append(key, &alpha, 1);
    append(key, &sid, 1);
    append(key, &nu, 1);
    return (const float *)cached(key, [&] { return as_bytes(equiangular_response(M, alpha, sid, nu - 1)); }, st);
}

std::vector<float2> twiddles(int M)
{
    std::vector<float2> t((size_t)M);
    for (int n = 0; n < M; ++n)
        t[(size_t)n] = make_float2((float)std::cos(2.0 * kPi * n / M), (float)-std::sin(2.0 * kPi * n / M));
    return t;
}

const float2 *twiddle_table(int M, int *st)
{
    std::string key = "twiddle";
    append(key, &M, 1);
    return (const float2 *)cached(key, [&] { return as_bytes(twiddles(M)); }, st);
}

// Default redundancy weights: parallel pi/range; fan/cone 1/2 for a full
// turn, Parker (delta = (range - pi)/2) for a short scan.
double parker(double beta, double gamma, double delta)
{
    const double a = delta - gamma, b = delta + gamma;
    if (a > 0.0 && beta < 2.0 * a) {
        const double s = std::sin(0.25 * kPi * beta / a);
        return s * s;
    }
    if (beta < kPi - 2.0 * gamma)
        return 1.0;
    if (b > 0.0 && beta <= kPi + 2.0 * delta) {
        const double s = std::sin(0.25 * kPi * (kPi + 2.0 * delta - beta) / b);
        return s * s;
    }
    return 0.0;
}

std::vector<float> wred_values(int kind, int n_proj, int nu, double du, double range, double sdd)
{
    std::vector<float> w((size_t)n_proj * nu);
    const bool full = std::fabs(range - 2.0 * kPi) <= 1e-6 * 2.0 * kPi;
    const double delta = 0.5 * (range - kPi);
    for (int k = 0; k < n_proj; ++k) {
        const double beta = range * k / n_proj;
        for (int j = 0; j < nu; ++j) {
            double v;
            if (kind == 0)
                v = kPi / range;
            else if (full)
                v = 0.5;
            else if (kind == 3)   // equiangular bins: the fan angle is linear in j
                v = parker(beta, (j - 0.5 * (nu - 1)) * du / sdd, delta);
            else
                v = parker(beta, std::atan((j - 0.5 * (nu - 1)) * du / sdd), delta);
            w[(size_t)k * nu + j] = (float)v;
        }
    }
    return w;
}

const float *wred_table(int kind, int n_proj, int nu, double du, double range, double sdd, int *st)
{
    std::string key = "wred";
    append(key, &kind, 1);
    append(key, &n_proj, 1);
    append(key, &nu, 1);
    append(key, &du, 1);
    append(key, &range, 1);
    append(key, &sdd, 1);
    return (const float *)cached(key, [&] { return as_bytes(wred_values(kind, n_proj, nu, du, range, sdd)); }, st);
}

// --------------------------------------------------------- shared drivers

int to_status(hipError_t e) { return e == hipSuccess ? PH_OK : PH_ERR_HIP; }

// Host-only validation of a 2D call's geometry and ray vectors.
int validate2d(const ph_geom2d *g, bool fan, const float *rv)
{
    Geom2D G;
    int st = make_geom2d(g, fan, &G);
    if (st != PH_OK)
        return st;
    if (!rv)
        return PH_ERR_NULL;
    std::vector<float2> v;
    return views2d(g, fan, rv, &v);
}

int prep2d(const ph_geom2d *g, bool fan, const float *rv, Geom2D *G, const float2 **views)
{
    int st = make_geom2d(g, fan, G);
    if (st != PH_OK)
        return st;
    if (!rv)
        return PH_ERR_NULL;
    std::vector<float2> v;
    st = views2d(g, fan, rv, &v);
    if (st != PH_OK)
        return st;
    std::string key = fan ? "v2f" : "v2p";
    append(key, g, 1);
    append(key, rv, 2 * (size_t)g->n_proj);
    st = PH_OK;
    *views = (const float2 *)cached(key, [&] { return as_bytes(v); }, &st);
    return st;
}

// Host-only validation of a 3D call's geometry and matrices.
int validate3d(const ph_geom3d *g, const float *mats, Geom3D *G, std::vector<double> *P)
{
    int st = make_geom3d(g, G);
    if (st != PH_OK)
        return st;
    if (!mats)
        return PH_ERR_NULL;
    return normalised_mats(g, mats, P);
}

// Per-view tables of a validated 3D call (uploaded on first use).
int upload3d(const ph_geom3d *g, const float *mats, const std::vector<double> &P, bool for_bp, const void **views,
             bool *axial)
{
    std::string key = for_bp ? "bp3" : "fp3";
    append(key, g, 1);
    append(key, mats, 12 * (size_t)g->n_proj);
    int st = PH_OK;
    if (for_bp) {
        std::vector<ConeBPView> v;
        std::vector<ConeBPView64> v64;
        bp_views(g, P, &v, axial, &v64);
        *views = cached(
            key,
            [&] {
                // the FP64 rows follow the FP32 ones for the general (per-voxel) paths
                std::vector<unsigned char> b = as_bytes(v);
                if (!*axial) {
                    const std::vector<unsigned char> b64 = as_bytes(v64);
                    b.insert(b.end(), b64.begin(), b64.end());
                }
                return b;
            },
            &st);
    } else {
        std::vector<ConeFPView> v;
        fp_views(g, P, &v);
        *views = cached(key, [&] { return as_bytes(v); }, &st);
    }
    return st;
}

// The FP64 rows that follow the FP32 ones in a back-projector table of a
// trajectory that is not a rotation about z; NULL for a circular one.
const ConeBPView64 *views64_of(const void *views, bool axial, int n_proj)
{
    return axial ? nullptr : reinterpret_cast<const ConeBPView64 *>((const ConeBPView *)views + n_proj);
}

int prep3d(const ph_geom3d *g, const float *mats, bool for_bp, Geom3D *G, const void **views, bool *axial)
{
    std::vector<double> P;
    int st = validate3d(g, mats, G, &P);
    if (st != PH_OK)
        return st;
    return upload3d(g, mats, P, for_bp, views, axial);
}

// Host-only check of the filter length; returns the length to use in *Mout.
int filter_len(const float *K, int M, int nu, int *Mout)
{
    if (K) {
        if (!is_pow2(M) || M < 16 || M < nu || M > 4096)
            return PH_ERR_SHAPE;
    } else {
        if (M == 0)
            M = default_fft_size(nu);
        if (!is_pow2(M) || M < 2 * nu - 1 || M > 4096)
            return PH_ERR_SHAPE;
    }
    *Mout = M;
    return PH_OK;
}

// Filter kind of a 2D call: 0 parallel, 1 fan on the flat detector, 3 fan on
// the equiangular detector (2 is the cone beam).
int kind2d(const ph_geom2d *g, bool fan) { return !fan ? 0 : g->fan_detector == 1 ? 3 : 1; }

// Scalar filter arguments of a validated call (M from filter_len); the
// tables K, tw, W_red and W are left for the caller to set.
void filter_scalars(int kind, int nu, int nv, int n_proj, int batch, double du, double dv, double sdd, int M,
                    FilterArgs *a)
{
    a->nu = nu;
    a->nv = nv;
    a->n_proj = n_proj;
    a->batch = batch;
    a->M = M;
    a->log2M = ilog2(M);
    a->du = (float)du;
    a->dv = (float)dv;
    a->cu = 0.5f * (float)(nu - 1);
    a->cv = 0.5f * (float)(nv - 1);
    a->cos_sdd = kind == 0 ? 0.0f : (float)sdd;
    a->curved = kind == 3 ? 1 : 0;
}

// Filter arguments of a validated call (M from filter_len); uploads the
// default tables on first use.
int filter_args(int kind, int nu, int nv, int n_proj, int batch, double du, double dv, double sid, double sdd,
                double range, const float *K, int M, const float *W_red, const float *W, FilterArgs *a)
{
    int st = PH_OK;
    const double tau = kind == 0 ? du : du * sid / sdd;
    filter_scalars(kind, nu, nv, n_proj, batch, du, dv, sdd, M, a);
    a->K = K ? K : kind == 3 ? equiangular_table(M, du / sdd, sid, nu, &st) : ramlak_table(M, tau, &st);
    if (st != PH_OK)
        return st;
    a->tw = twiddle_table(M, &st);
    if (st != PH_OK)
        return st;
    a->W_red = W_red ? W_red : wred_table(kind, n_proj, nu, du, range, sdd, &st);
    if (st != PH_OK)
        return st;
    a->W = W;
    return PH_OK;
}

size_t round_up(size_t n) { return (n + 255) & ~(size_t)255; }

int project2d(const ph_geom2d *g, bool fan, const float *rv, const void *img, void *sino, int batch, int dtype,
              void *stream)
{
    if (!img || !sino)
        return PH_ERR_NULL;
    if (batch < 1)
        return PH_ERR_SHAPE;
    int st = check_dtype(dtype);
    if (st != PH_OK)
        return st;
    Geom2D G;
    const float2 *views = nullptr;
    st = prep2d(g, fan, rv, &G, &views);
    if (st != PH_OK)
        return st;
    return to_status(launch_project_2d(dtype, fan, G, views, img, sino, batch, (hipStream_t)stream));
}

int backproject2d(const ph_geom2d *g, bool fan, const float *rv, const void *sino, void *img, int batch, int dtype,
                  void *stream)
{
    if (!img || !sino)
        return PH_ERR_NULL;
    if (batch < 1)
        return PH_ERR_SHAPE;
    int st = check_dtype(dtype);
    if (st != PH_OK)
        return st;
    Geom2D G;
    const float2 *views = nullptr;
    st = prep2d(g, fan, rv, &G, &views);
    if (st != PH_OK)
        return st;
    return to_status(launch_backproject_2d(dtype, fan, G, views, sino, false, img, batch, (hipStream_t)stream));
}

int weight_filter2d(const ph_geom2d *g, bool fan, const void *sino, float *out, const float *K, int M,
                    const float *W_red, int batch, int dtype, void *stream)
{
    if (!sino || !out)
        return PH_ERR_NULL;
    if (batch < 1)
        return PH_ERR_SHAPE;
    int st = check_dtype(dtype);
    if (st != PH_OK)
        return st;
    Geom2D G;
    st = make_geom2d(g, fan, &G);
    if (st != PH_OK)
        return st;
    st = filter_len(K, M, g->det_shape, &M);
    if (st != PH_OK)
        return st;
    FilterArgs a;
    st = filter_args(kind2d(g, fan), g->det_shape, 1, g->n_proj, batch, g->det_spacing, 1.0, g->sid, g->sdd,
                     g->angular_range, K, M, W_red, nullptr, &a);
    if (st != PH_OK)
        return st;
    return to_status(launch_weight_filter(dtype, a, sino, out, (hipStream_t)stream));
}

int fbp2d(const ph_geom2d *g, bool fan, const float *rv, const void *sino, void *img, const float *K, int M,
          const float *W_red, void *ws, size_t ws_bytes, int batch, int dtype, void *stream)
{
    if (!sino || !img)
        return PH_ERR_NULL;
    if (batch < 1)
        return PH_ERR_SHAPE;
    int st = check_dtype(dtype);
    if (st != PH_OK)
        return st;
    Geom2D G;
    st = make_geom2d(g, fan, &G);
    if (st != PH_OK)
        return st;
    if (!rv)
        return PH_ERR_NULL;
    {
        std::vector<float2> tmp;
        st = views2d(g, fan, rv, &tmp);
        if (st != PH_OK)
            return st;
    }
    if (!ws || ws_bytes < ph_workspace_bytes_2d(g, batch))
        return PH_ERR_WORKSPACE;
    st = filter_len(K, M, g->det_shape, &M);
    if (st != PH_OK)
        return st;
    const float2 *views = nullptr;
    st = prep2d(g, fan, rv, &G, &views);
    if (st != PH_OK)
        return st;
    FilterArgs a;
    st = filter_args(kind2d(g, fan), g->det_shape, 1, g->n_proj, batch, g->det_spacing, 1.0, g->sid, g->sdd,
                     g->angular_range, K, M, W_red, nullptr, &a);
    if (st != PH_OK)
        return st;
    float *q = (float *)ws;
    st = to_status(launch_weight_filter(dtype, a, sino, q, (hipStream_t)stream));
    if (st != PH_OK)
        return st;
    return to_status(launch_backproject_2d(dtype, fan, G, views, q, true, img, batch, (hipStream_t)stream));
}

// B^T accumulates with float atomics: FP32 output directly, half-precision
// output through an FP32 workspace that is then rounded to the storage type.
int adjoint2d(const ph_geom2d *g, bool fan, bool of_projector, const float *rv, const void *in, void *out,
              int batch, int dtype, void *stream, void *ws = nullptr, size_t ws_bytes = 0, bool ws_call = false)
{
    if (!in || !out)
        return PH_ERR_NULL;
    if (batch < 1)
        return PH_ERR_SHAPE;
    int st = check_dtype(dtype);
    if (st != PH_OK)
        return st;
    if (!of_projector && dtype != PH_F32 && !ws_call)
        return PH_ERR_UNSUPPORTED;
    Geom2D G;
    const float2 *views = nullptr;
    st = validate2d(g, fan, rv);
    if (st != PH_OK)
        return st;
    const size_t n_out = (size_t)batch * g->n_proj * g->det_shape;
    const bool via_ws = !of_projector && dtype != PH_F32;
    if (via_ws && (!ws || ws_bytes < round_up(n_out * sizeof(float))))
        return PH_ERR_WORKSPACE;
    st = prep2d(g, fan, rv, &G, &views);
    if (st != PH_OK)
        return st;
    if (of_projector)
        return to_status(launch_project_adjoint_2d(dtype, fan, G, views, in, out, batch, (hipStream_t)stream));
    float *acc = via_ws ? (float *)ws : (float *)out;
    st = to_status(launch_backproject_adjoint_2d(dtype, fan, G, views, in, acc, batch, (hipStream_t)stream));
    if (st != PH_OK || !via_ws)
        return st;
    return to_status(launch_cast_from_f32(dtype, acc, out, n_out, (hipStream_t)stream));
}

// Tables held in the static scratch array of each device, as last copied
// there: a call copies its tables only when they differ.
std::mutex g_static_mu;
std::vector<std::vector<unsigned char>> g_static_tables(64);

int upload_static_tables(void *base, const std::vector<unsigned char> &host, hipStream_t stream)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= (int)g_static_tables.size())
        return PH_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_static_mu);
    std::vector<unsigned char> &held = g_static_tables[(size_t)dev];
    if (held == host)
        return PH_OK;
    held.clear();
    if (hipMemcpyAsync(base, host.data(), host.size(), hipMemcpyHostToDevice, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return PH_ERR_HIP;
    held = host;
    return PH_OK;
}

}  // namespace

extern "C" {

const char *ph_status_string(int s)
{
    switch (s) {
    case PH_OK: return "ok";
    case PH_ERR_NULL: return "null pointer argument";
    case PH_ERR_SHAPE: return "invalid shape, batch or filter length";
    case PH_ERR_GEOMETRY: return "invalid geometry";
    case PH_ERR_DTYPE: return "unknown storage dtype";
    case PH_ERR_WORKSPACE: return "workspace missing or too small";
    case PH_ERR_HIP: return "HIP runtime error";
    case PH_ERR_UNSUPPORTED: return "unsupported request";
    case PH_ERR_VALUE: return "scalar argument non-finite or out of range";
    default: return "unknown status";
    }
}

const char *ph_version(void) { return "pyrohip 0.1 (gfx950)"; }

int ph_ray_vectors_2d(const ph_geom2d *g, float *ray_vecs)
{
    CallScope scope;
    if (!g || !ray_vecs)
        return PH_ERR_NULL;
    if (g->n_proj < 1)
        return PH_ERR_SHAPE;
    if (!finite_pos(g->angular_range))
        return PH_ERR_GEOMETRY;
    for (int k = 0; k < g->n_proj; ++k) {
        const double b = (double)g->angular_range * k / g->n_proj;
        ray_vecs[2 * k] = (float)std::cos(b);
        ray_vecs[2 * k + 1] = (float)std::sin(b);
    }
    return PH_OK;
}

int ph_projection_matrices_3d(const ph_geom3d *g, float *mats)
{
    CallScope scope;
    if (!g || !mats)
        return PH_ERR_NULL;
    if (g->n_proj < 1 || g->det_shape[0] < 1 || g->det_shape[1] < 1)
        return PH_ERR_SHAPE;
    if (!finite_pos(g->angular_range) || !finite_pos(g->det_spacing[0]) || !finite_pos(g->det_spacing[1]) ||
        !finite_pos(g->sid) || !std::isfinite(g->sdd) || !(g->sdd > g->sid))
        return PH_ERR_GEOMETRY;
    const double cu = 0.5 * (g->det_shape[1] - 1), cv = 0.5 * (g->det_shape[0] - 1);
    const double fu = g->sdd / (double)g->det_spacing[1], fv = g->sdd / (double)g->det_spacing[0];
    for (int k = 0; k < g->n_proj; ++k) {
        const double b = (double)g->angular_range * k / g->n_proj;
        const double c[3] = {std::cos(b), std::sin(b), 0.0}, eu[3] = {-std::sin(b), std::cos(b), 0.0};
        const double ev[3] = {0.0, 0.0, 1.0};
        // R rows (e_u; e_v; c); translation -R S with S = -SID c gives (0, 0, SID)
        const double t[3] = {0.0, 0.0, (double)g->sid};
        const double R[3][3] = {{eu[0], eu[1], eu[2]}, {ev[0], ev[1], ev[2]}, {c[0], c[1], c[2]}};
        float *P = mats + 12 * (size_t)k;
        for (int a = 0; a < 3; ++a) {
            P[a] = (float)(fu * R[0][a] + cu * R[2][a]);
            P[4 + a] = (float)(fv * R[1][a] + cv * R[2][a]);
            P[8 + a] = (float)R[2][a];
        }
        P[3] = (float)(fu * t[0] + cu * t[2]);
        P[7] = (float)(fv * t[1] + cv * t[2]);
        P[11] = (float)t[2];
    }
    return PH_OK;
}

int ph_project_par2d(const ph_geom2d *g, const float *rv, const void *img, void *sino, int batch, ph_dtype dtype,
                     void *stream)
{
    CallScope scope;
    return project2d(g, false, rv, img, sino, batch, dtype, stream);
}

int ph_project_fan2d(const ph_geom2d *g, const float *rv, const void *img, void *sino, int batch, ph_dtype dtype,
                     void *stream)
{
    CallScope scope;
    return project2d(g, true, rv, img, sino, batch, dtype, stream);
}

int ph_backproject_par2d(const ph_geom2d *g, const float *rv, const void *sino, void *img, int batch, ph_dtype dtype,
                         void *stream)
{
    CallScope scope;
    return backproject2d(g, false, rv, sino, img, batch, dtype, stream);
}

int ph_backproject_fan2d(const ph_geom2d *g, const float *rv, const void *sino, void *img, int batch, ph_dtype dtype,
                         void *stream)
{
    CallScope scope;
    return backproject2d(g, true, rv, sino, img, batch, dtype, stream);
}

int ph_project_cone3d(const ph_geom3d *g, const float *mats, const void *vol, void *proj, int batch, ph_dtype dtype,
                      void *stream)
{
    CallScope scope;
    if (!vol || !proj)
        return PH_ERR_NULL;
    if (batch < 1)
        return PH_ERR_SHAPE;
    int st = check_dtype(dtype);
    if (st != PH_OK)
        return st;
    Geom3D G;
    const void *views = nullptr;
    bool axial = false;
    st = prep3d(g, mats, false, &G, &views, &axial);
    if (st != PH_OK)
        return st;
    const hipStream_t s = (hipStream_t)stream;
    if (dtype == PH_F32)
        return to_status(launch_project_cone(dtype, G, (const ConeFPView *)views, (const float *)vol, proj, batch, s));
    // A half-precision volume is widened (exactly) into a stream-ordered FP32
    // copy, projected by the FP32 kernel, and the projections are stored in
    // half precision: the values and arithmetic of FP32 staging, without a
    // 16-bit staging path.  The copy is freed in stream order.
    const size_t n_vox = (size_t)batch * G.nx * G.ny * G.nz;
    void *wide = nullptr;
    if (hipMallocAsync(&wide, n_vox * sizeof(float), s) != hipSuccess)
        return PH_ERR_HIP;
    hipError_t e = launch_cast_to_f32(dtype, vol, (float *)wide, n_vox, s);
    if (e == hipSuccess)
        e = launch_project_cone(dtype, G, (const ConeFPView *)views, (const float *)wide, proj, batch, s);
    const hipError_t ef = hipFreeAsync(wide, s);
    return to_status(e != hipSuccess ? e : ef);
}

int ph_backproject_cone3d(const ph_geom3d *g, const float *mats, const void *proj, void *vol, int batch, ph_dtype dtype,
                          void *stream)
{
    CallScope scope;
    if (!vol || !proj)
        return PH_ERR_NULL;
    if (batch < 1)
        return PH_ERR_SHAPE;
    int st = check_dtype(dtype);
    if (st != PH_OK)
        return st;
    Geom3D G;
    const void *views = nullptr;
    bool axial = false;
    st = prep3d(g, mats, true, &G, &views, &axial);
    if (st != PH_OK)
        return st;
    return to_status(launch_backproject_cone(dtype, G, (const ConeBPView *)views, views64_of(views, axial, g->n_proj),
                                             axial, bp_segment(g), proj, false, vol, batch, (hipStream_t)stream));
}

int ph_weight_filter_2d(const ph_geom2d *g, int fan, const void *sino, float *out, const float *K, int M,
                        const float *W_red, int batch, ph_dtype dtype, void *stream)
{
    CallScope scope;
    return weight_filter2d(g, fan != 0, sino, out, K, M, W_red, batch, dtype, stream);
}

int ph_weight_filter_3d(const ph_geom3d *g, const void *proj, float *out, const float *K, int M, const float *W_red,
                        const float *W, int batch, ph_dtype dtype, void *stream)
{
    CallScope scope;
    if (!proj || !out)
        return PH_ERR_NULL;
    if (batch < 1)
        return PH_ERR_SHAPE;
    int st = check_dtype(dtype);
    if (st != PH_OK)
        return st;
    Geom3D G;
    st = make_geom3d(g, &G);
    if (st != PH_OK)
        return st;
    st = filter_len(K, M, g->det_shape[1], &M);
    if (st != PH_OK)
        return st;
    FilterArgs a;
    st = filter_args(2, g->det_shape[1], g->det_shape[0], g->n_proj, batch, g->det_spacing[1], g->det_spacing[0],
                     g->sid, g->sdd, g->angular_range, K, M, W_red, W, &a);
    if (st != PH_OK)
        return st;
    return to_status(launch_weight_filter(dtype, a, proj, out, (hipStream_t)stream));
}

size_t ph_workspace_bytes_2d(const ph_geom2d *g, int batch)
{
    CallScope scope;
    if (!g || batch < 1 || g->n_proj < 1 || g->det_shape < 1)
        return 0;
    return round_up((size_t)batch * g->n_proj * g->det_shape * sizeof(float));
}

size_t ph_workspace_bytes_3d(const ph_geom3d *g, int batch)
{
    CallScope scope;
    if (!g || batch < 1 || g->n_proj < 1 || g->det_shape[0] < 1 || g->det_shape[1] < 1)
        return 0;
    return round_up((size_t)batch * g->n_proj * g->det_shape[0] * g->det_shape[1] * sizeof(float));
}

size_t ph_fdk_workspace_bytes(const ph_geom3d *g, int M, int batch, ph_dtype dtype)
{
    CallScope scope;
    if (check_dtype(dtype) != PH_OK || !g || g->det_shape[1] < 1)
        return 0;
    // M = 0: the default Ram-Lak length; otherwise a length some response K may have
    if (M != 0 && !(is_pow2(M) && M >= 16 && M >= g->det_shape[1] && M <= 4096))
        return 0;
    return ph_workspace_bytes_3d(g, batch);
}

int ph_fbp_par2d(const ph_geom2d *g, const float *rv, const void *sino, void *img, const float *K, int M,
                 const float *W_red, void *ws, size_t ws_bytes, int batch, ph_dtype dtype, void *stream)
{
    CallScope scope;
    return fbp2d(g, false, rv, sino, img, K, M, W_red, ws, ws_bytes, batch, dtype, stream);
}

int ph_fbp_fan2d(const ph_geom2d *g, const float *rv, const void *sino, void *img, const float *K, int M,
                 const float *W_red, void *ws, size_t ws_bytes, int batch, ph_dtype dtype, void *stream)
{
    CallScope scope;
    return fbp2d(g, true, rv, sino, img, K, M, W_red, ws, ws_bytes, batch, dtype, stream);
}

int ph_fdk_cone3d(const ph_geom3d *g, const float *mats, const void *proj, void *vol, const float *K, int M,
                  const float *W_red, const float *W, void *ws, size_t ws_bytes, int batch, ph_dtype dtype, void *stream)
{
    CallScope scope;
    if (!proj || !vol)
        return PH_ERR_NULL;
    if (batch < 1)
        return PH_ERR_SHAPE;
    int st = check_dtype(dtype);
    if (st != PH_OK)
        return st;
    Geom3D G;
    std::vector<double> P;
    st = validate3d(g, mats, &G, &P);
    if (st != PH_OK)
        return st;
    if (!ws || ws_bytes < ph_workspace_bytes_3d(g, batch))
        return PH_ERR_WORKSPACE;
    st = filter_len(K, M, g->det_shape[1], &M);
    if (st != PH_OK)
        return st;
    const void *views = nullptr;
    bool axial = false;
    st = upload3d(g, mats, P, true, &views, &axial);
    if (st != PH_OK)
        return st;
    FilterArgs a;
    st = filter_args(2, g->det_shape[1], g->det_shape[0], g->n_proj, batch, g->det_spacing[1], g->det_spacing[0],
                     g->sid, g->sdd, g->angular_range, K, M, W_red, W, &a);
    if (st != PH_OK)
        return st;
    float *q = (float *)ws;
    st = to_status(launch_weight_filter(dtype, a, proj, q, (hipStream_t)stream));
    if (st != PH_OK)
        return st;
    return to_status(launch_backproject_cone(dtype, G, (const ConeBPView *)views, views64_of(views, axial, g->n_proj),
                                             axial, bp_segment(g), q, true, vol, batch, (hipStream_t)stream));
}

int ph_fdk_cone3d_static(const ph_geom3d *g, const float *mats, const void *proj, void *vol, const float *K, int M,
                         const float *W_red, const float *W, int batch, ph_dtype dtype, void *stream)
{
    CallScope scope;
    if (!proj || !vol)
        return PH_ERR_NULL;
    if (batch < 1)
        return PH_ERR_SHAPE;
    int st = check_dtype(dtype);
    if (st != PH_OK)
        return st;
    Geom3D G;
    std::vector<double> P;
    st = validate3d(g, mats, &G, &P);
    if (st != PH_OK)
        return st;
    st = filter_len(K, M, g->det_shape[1], &M);
    if (st != PH_OK)
        return st;
    const int nu = g->det_shape[1], nv = g->det_shape[0], np = g->n_proj;
    std::vector<ConeBPView> v;
    std::vector<ConeBPView64> v64;
    bool axial = false;
    bp_views(g, P, &v, &axial, &v64);

    // scratch layout: tables, then the filtered projections of a share of the views
    size_t off = 0;
    auto take = [&](size_t n) {
        const size_t o = off;
        off = round_up(off + n);
        return o;
    };
    const size_t o_views = take((size_t)np * sizeof(ConeBPView));
    const size_t o_v64 = axial ? 0 : take((size_t)np * sizeof(ConeBPView64));
    const size_t o_K = K ? 0 : take((size_t)M * sizeof(float));
    const size_t o_tw = take((size_t)M * sizeof(float2));
    const size_t o_wred = W_red ? 0 : take((size_t)np * nu * sizeof(float));
    const size_t tables = off;
    const size_t per_view = (size_t)batch * nv * nu * sizeof(float);
    const size_t cap = (size_t)PH_FDK_STATIC_SCRATCH_BYTES;
    if (tables >= cap || (cap - tables) / per_view < 1)
        return PH_ERR_WORKSPACE;
    const int share = (int)std::min<size_t>((size_t)np, (cap - tables) / per_view);
    if (share < np && dtype != PH_F32)
        return PH_ERR_WORKSPACE;

    void *base = nullptr;
    size_t bytes = 0;
    if (static_scratch(&base, &bytes) != hipSuccess || bytes != cap)
        return PH_ERR_HIP;
    std::vector<unsigned char> host(tables, 0);
    std::memcpy(host.data() + o_views, v.data(), (size_t)np * sizeof(ConeBPView));
    if (!axial)
        std::memcpy(host.data() + o_v64, v64.data(), (size_t)np * sizeof(ConeBPView64));
    if (!K) {
        const std::vector<float> k = ramlak_response(M, (double)g->det_spacing[1] * g->sid / g->sdd);
        std::memcpy(host.data() + o_K, k.data(), k.size() * sizeof(float));
    }
    {
        const std::vector<float2> t = twiddles(M);
        std::memcpy(host.data() + o_tw, t.data(), t.size() * sizeof(float2));
    }
    if (!W_red) {
        const std::vector<float> w = wred_values(2, np, nu, g->det_spacing[1], g->angular_range, g->sdd);
        std::memcpy(host.data() + o_wred, w.data(), w.size() * sizeof(float));
    }
    hipStream_t s = (hipStream_t)stream;
    st = upload_static_tables(base, host, s);
    if (st != PH_OK)
        return st;

    char *sb = (char *)base;
    FilterArgs a;
    filter_scalars(2, nu, nv, share, 1, g->det_spacing[1], g->det_spacing[0], g->sdd, M, &a);
    a.K = K ? K : (const float *)(sb + o_K);
    a.tw = (const float2 *)(sb + o_tw);
    a.W = W;
    const float *wred = W_red ? W_red : (const float *)(sb + o_wred);
    const ConeBPView *views = (const ConeBPView *)(sb + o_views);
    const ConeBPView64 *views64 = axial ? nullptr : (const ConeBPView64 *)(sb + o_v64);
    float *q = (float *)(sb + tables);
    const size_t elem = dtype == PH_F32 ? sizeof(float) : sizeof(uint16_t);
    const int seg = bp_segment(g);
    // views k0 .. k0 + kc - 1: filter each batch item's rows, then back-project
    // the share (the first share overwrites vol, the others add to it)
    for (int k0 = 0; k0 < np; k0 += share) {
        const int kc = std::min(share, np - k0);
        a.n_proj = kc;
        a.W_red = wred + (size_t)k0 * nu;
        for (int b = 0; b < batch; ++b) {
            const char *in = (const char *)proj + ((size_t)b * np + k0) * nv * nu * elem;
            st = to_status(launch_weight_filter(dtype, a, in, q + (size_t)b * kc * nv * nu, s));
            if (st != PH_OK)
                return st;
        }
        Geom3D Gk = G;
        Gk.n_proj = kc;
        st = to_status(launch_backproject_cone(dtype, Gk, views + k0, views64 ? views64 + k0 : nullptr, axial, seg, q,
                                               true, vol, batch, s, k0 > 0));
        if (st != PH_OK)
            return st;
    }
    return PH_OK;
}

int ph_project_adjoint_par2d(const ph_geom2d *g, const float *rv, const void *sino, void *img, int batch, ph_dtype dtype,
                             void *stream)
{
    CallScope scope;
    return adjoint2d(g, false, true, rv, sino, img, batch, dtype, stream);
}

int ph_project_adjoint_fan2d(const ph_geom2d *g, const float *rv, const void *sino, void *img, int batch, ph_dtype dtype,
                             void *stream)
{
    CallScope scope;
    return adjoint2d(g, true, true, rv, sino, img, batch, dtype, stream);
}

int ph_backproject_adjoint_par2d(const ph_geom2d *g, const float *rv, const void *img, void *sino, int batch,
                                 ph_dtype dtype, void *stream)
{
    CallScope scope;
    return adjoint2d(g, false, false, rv, img, sino, batch, dtype, stream);
}

int ph_backproject_adjoint_fan2d(const ph_geom2d *g, const float *rv, const void *img, void *sino, int batch,
                                 ph_dtype dtype, void *stream)
{
    CallScope scope;
    return adjoint2d(g, true, false, rv, img, sino, batch, dtype, stream);
}

int ph_project_adjoint_cone3d(const ph_geom3d *g, const float *mats, const void *proj, void *vol, int batch,
                              ph_dtype dtype, void *stream)
{
    CallScope scope;
    if (!proj || !vol)
        return PH_ERR_NULL;
    if (batch < 1)
        return PH_ERR_SHAPE;
    int st = check_dtype(dtype);
    if (st != PH_OK)
        return st;
    Geom3D G;
    std::vector<double> P;
    st = validate3d(g, mats, &G, &P);
    if (st != PH_OK)
        return st;
    const void *fv = nullptr, *bv = nullptr;
    bool axial = false;
    st = upload3d(g, mats, P, false, &fv, &axial);
    if (st != PH_OK)
        return st;
    st = upload3d(g, mats, P, true, &bv, &axial);
    if (st != PH_OK)
        return st;
    return to_status(launch_project_adjoint_cone(dtype, G, (const ConeFPView *)fv, (const ConeBPView *)bv, proj, vol,
                                                 batch, (hipStream_t)stream));
}

static int bpT3d(const ph_geom3d *g, const float *mats, const void *vol, void *proj, void *ws, size_t ws_bytes,
                 bool ws_call, int batch, ph_dtype dtype, void *stream)
{
    if (!proj || !vol)
        return PH_ERR_NULL;
    if (batch < 1)
        return PH_ERR_SHAPE;
    int st = check_dtype(dtype);
    if (st != PH_OK)
        return st;
    if (dtype != PH_F32 && !ws_call)
        return PH_ERR_UNSUPPORTED;
    Geom3D G;
    std::vector<double> P;
    st = validate3d(g, mats, &G, &P);
    if (st != PH_OK)
        return st;
    const size_t n_out = (size_t)batch * g->n_proj * g->det_shape[0] * g->det_shape[1];
    const bool via_ws = dtype != PH_F32;
    if (via_ws && (!ws || ws_bytes < round_up(n_out * sizeof(float))))
        return PH_ERR_WORKSPACE;
    const void *views = nullptr;
    bool axial = false;
    st = upload3d(g, mats, P, true, &views, &axial);
    if (st != PH_OK)
        return st;
    float *acc = via_ws ? (float *)ws : (float *)proj;
    st = to_status(launch_backproject_adjoint_cone(dtype, G, (const ConeBPView *)views,
                                                   views64_of(views, axial, g->n_proj), axial, bp_segment(g), vol, acc,
                                                   batch, (hipStream_t)stream));
    if (st != PH_OK || !via_ws)
        return st;
    return to_status(launch_cast_from_f32(dtype, acc, proj, n_out, (hipStream_t)stream));
}

int ph_backproject_adjoint_cone3d(const ph_geom3d *g, const float *mats, const void *vol, void *proj, int batch,
                                  ph_dtype dtype, void *stream)
{
    CallScope scope;
    return bpT3d(g, mats, vol, proj, nullptr, 0, false, batch, dtype, stream);
}

size_t ph_backproject_adjoint_workspace_bytes_2d(const ph_geom2d *g, int batch, ph_dtype dtype)
{
    CallScope scope;
    if (!g || batch < 1 || g->n_proj < 1 || g->det_shape < 1 || check_dtype(dtype) != PH_OK || dtype == PH_F32)
        return 0;
    return round_up((size_t)batch * g->n_proj * g->det_shape * sizeof(float));
}

size_t ph_backproject_adjoint_workspace_bytes_3d(const ph_geom3d *g, int batch, ph_dtype dtype)
{
    CallScope scope;
    if (!g || batch < 1 || g->n_proj < 1 || g->det_shape[0] < 1 || g->det_shape[1] < 1 || check_dtype(dtype) != PH_OK ||
        dtype == PH_F32)
        return 0;
    return round_up((size_t)batch * g->n_proj * g->det_shape[0] * g->det_shape[1] * sizeof(float));
}

int ph_backproject_adjoint_ws_par2d(const ph_geom2d *g, const float *rv, const void *img, void *sino, void *ws,
                                    size_t ws_bytes, int batch, ph_dtype dtype, void *stream)
{
    CallScope scope;
    return adjoint2d(g, false, false, rv, img, sino, batch, dtype, stream, ws, ws_bytes, true);
}

int ph_backproject_adjoint_ws_fan2d(const ph_geom2d *g, const float *rv, const void *img, void *sino, void *ws,
                                    size_t ws_bytes, int batch, ph_dtype dtype, void *stream)
{
    CallScope scope;
    return adjoint2d(g, true, false, rv, img, sino, batch, dtype, stream, ws, ws_bytes, true);
}

int ph_backproject_adjoint_ws_cone3d(const ph_geom3d *g, const float *mats, const void *vol, void *proj, void *ws,
                                     size_t ws_bytes, int batch, ph_dtype dtype, void *stream)
{
    CallScope scope;
    return bpT3d(g, mats, vol, proj, ws, ws_bytes, true, batch, dtype, stream);
}

int ph_filter_response_equiangular(int M, double alpha, double sid, float *K)
{
    CallScope scope;
    if (!K)
        return PH_ERR_NULL;
    if (!is_pow2(M) || M < 2 || M > 4096)
        return PH_ERR_SHAPE;
    if (!finite_pos(alpha) || !(alpha * M <= kPi) || !finite_pos(sid))
        return PH_ERR_VALUE;
    const std::vector<float> t = equiangular_response(M, alpha, sid, M / 2);
    std::copy(t.begin(), t.end(), K);
    return PH_OK;
}

int ph_filter_response(int kind, int M, double tau, float *K)
{
    CallScope scope;
    if (!K)
        return PH_ERR_NULL;
    if (!is_pow2(M) || M < 2 || M > 4096)
        return PH_ERR_SHAPE;
    if (!finite_pos(tau) || (kind != 0 && kind != 1))
        return PH_ERR_VALUE;
    if (kind == 1) {
        for (int k = 0; k < M; ++k)
            K[k] = (float)((double)(k <= M / 2 ? k : M - k) / ((double)M * tau));
        return PH_OK;
    }
    const std::vector<float> t = ramlak_response(M, tau);
    std::memcpy(K, t.data(), sizeof(float) * (size_t)M);
    return PH_OK;
}

int ph_mse_grad(const float *x, const float *ref, const float *mask, size_t n, float *grad, double *loss, void *stream)
{
    CallScope scope;
    if (!x || !ref || !grad || !loss)
        return PH_ERR_NULL;
    if (n < 1)
        return PH_ERR_SHAPE;
    return to_status(launch_mse(x, ref, mask, n, grad, loss, (hipStream_t)stream));
}

int ph_corrector_grad_3d(const ph_geom3d *g, const float *proj, const float *grad_q, const float *K, int M,
                         const float *W_red, const float *W, float *dK, float *dW, int batch, void *stream)
{
    CallScope scope;
    if (!proj || !grad_q || !K || !dK)
        return PH_ERR_NULL;
    if (batch < 1)
        return PH_ERR_SHAPE;
    Geom3D G;
    int st = make_geom3d(g, &G);
    if (st != PH_OK)
        return st;
    st = filter_len(K, M, g->det_shape[1], &M);
    if (st != PH_OK)
        return st;
    FilterArgs a;
    st = filter_args(2, g->det_shape[1], g->det_shape[0], g->n_proj, batch, g->det_spacing[1], g->det_spacing[0],
                     g->sid, g->sdd, g->angular_range, K, M, W_red, W, &a);
    if (st != PH_OK)
        return st;
    return to_status(launch_corrector_grad(a, proj, grad_q, dK, dW, (hipStream_t)stream));
}

int ph_corrector_grad_2d(const ph_geom2d *g, int fan, const float *sino, const float *grad_q, const float *K, int M,
                         const float *W_red, float *dK, int batch, void *stream)
{
    CallScope scope;
    if (!sino || !grad_q || !K || !dK)
        return PH_ERR_NULL;
    if (batch < 1)
        return PH_ERR_SHAPE;
    Geom2D G;
    int st = make_geom2d(g, fan != 0, &G);
    if (st != PH_OK)
        return st;
    st = filter_len(K, M, g->det_shape, &M);
    if (st != PH_OK)
        return st;
    FilterArgs a;
    st = filter_args(kind2d(g, fan), g->det_shape, 1, g->n_proj, batch, g->det_spacing, 1.0, g->sid, g->sdd,
                     g->angular_range, K, M, W_red, nullptr, &a);
    if (st != PH_OK)
        return st;
    return to_status(launch_corrector_grad(a, sino, grad_q, dK, nullptr, (hipStream_t)stream));
}

int ph_adam_step(float *param, const float *grad, float *m, float *v, size_t n, float lr, float beta1, float beta2,
                 float eps, int t, void *stream)
{
    CallScope scope;
    if (!param || !grad || !m || !v)
        return PH_ERR_NULL;
    if (n < 1)
        return PH_ERR_SHAPE;
    const bool ok = std::isfinite(lr) && lr > 0.0f && std::isfinite(beta1) && beta1 >= 0.0f && beta1 < 1.0f &&
                    std::isfinite(beta2) && beta2 >= 0.0f && beta2 < 1.0f && std::isfinite(eps) && eps > 0.0f &&
                    t >= 1;
    if (!ok)
        return PH_ERR_VALUE;
    return to_status(launch_adam(param, grad, m, v, n, lr, beta1, beta2, eps, t, (hipStream_t)stream));
}

int ph_tv_3d(const float *vol, int nz, int ny, int nx, int batch, int anisotropic, float eps, float weight,
             float *grad, double *value, void *stream)
{
    CallScope scope;
    if (!vol)
        return PH_ERR_NULL;
    if (nz < 1 || ny < 1 || nx < 1 || batch < 1 || (double)nx * ny * nz * batch > 1e12)
        return PH_ERR_SHAPE;
    if ((anisotropic != 0 && anisotropic != 1) || !std::isfinite(eps) || !(anisotropic ? eps >= 0.0f : eps > 0.0f) ||
        !std::isfinite(weight))
        return PH_ERR_VALUE;
    if (!grad && !value)
        return PH_OK;
    return to_status(
        launch_tv(vol, nx, ny, nz, batch, anisotropic != 0, eps, weight, grad, value, (hipStream_t)stream));
}

size_t ph_tv_workspace_bytes_2d(const ph_geom2d *g, int batch)
{
    CallScope scope;
    if (!g || batch < 1 || g->n_proj < 1 || g->det_shape < 1 || g->vol_shape[0] < 1 || g->vol_shape[1] < 1)
        return 0;
    const size_t np = (size_t)batch * g->n_proj * g->det_shape, nx = (size_t)batch * g->vol_shape[0] * g->vol_shape[1];
    return 2 * round_up(np * sizeof(float)) + round_up(nx * sizeof(float));
}

size_t ph_tv_workspace_bytes_3d(const ph_geom3d *g, int batch)
{
    CallScope scope;
    if (!g || batch < 1 || g->n_proj < 1 || g->det_shape[0] < 1 || g->det_shape[1] < 1 || g->vol_shape[0] < 1 ||
        g->vol_shape[1] < 1 || g->vol_shape[2] < 1)
        return 0;
    const size_t np = (size_t)batch * g->n_proj * g->det_shape[0] * g->det_shape[1];
    const size_t nx = (size_t)batch * g->vol_shape[0] * g->vol_shape[1] * g->vol_shape[2];
    return 2 * round_up(np * sizeof(float)) + round_up(nx * sizeof(float));
}

}  // extern "C"

namespace {

bool tv_params_ok(const ph_tv_params *p)
{
    auto fin = [](float v) { return std::isfinite(v); };
    return (p->anisotropic == 0 || p->anisotropic == 1) && fin(p->lam) && p->lam >= 0.0f && fin(p->eps) &&
           (p->anisotropic ? p->eps >= 0.0f : p->eps > 0.0f) && fin(p->lr) && p->lr > 0.0f &&
           fin(p->beta1) && p->beta1 >= 0.0f && p->beta1 < 1.0f && fin(p->beta2) && p->beta2 >= 0.0f &&
           p->beta2 < 1.0f && fin(p->adam_eps) && p->adam_eps > 0.0f;
}

// The iteration loop shared by the three geometries: fwd / adj are the
// matched operator pair, (nz, ny, nx) the image grid, np / nx_total the
// element counts of the projections and of the images.
template <typename Fwd, typename Adj>
int tv_iterate(Fwd fwd, Adj adj, int nz, int ny, int nxg, size_t np, size_t nimg, const float *proj, float *x,
               float *m, float *v, int t0, int n_iter, const ph_tv_params *prm, void *ws, size_t ws_bytes,
               size_t ws_need, double *data_tv, int batch, void *stream)
{
    if (!proj || !x || !m || !v || !prm)
        return PH_ERR_NULL;
    if (t0 < 0 || n_iter < 1)
        return PH_ERR_SHAPE;
    if (!tv_params_ok(prm))
        return PH_ERR_VALUE;
    if (!ws || ws_need == 0 || ws_bytes < ws_need)
        return PH_ERR_WORKSPACE;
    char *w = (char *)ws;
    float *r = (float *)w;
    float *gr = (float *)(w + round_up(np * sizeof(float)));
    float *gx = (float *)(w + 2 * round_up(np * sizeof(float)));
    hipStream_t s = (hipStream_t)stream;
    for (int it = 0; it < n_iter; ++it) {
        const bool last = it + 1 == n_iter;
        int st = fwd(x, r);
        if (st != PH_OK)
            return st;
        st = to_status(launch_mse(r, proj, nullptr, np, gr, last ? data_tv : nullptr, s));
        if (st != PH_OK)
            return st;
        st = adj(gr, gx);
        if (st != PH_OK)
            return st;
        st = to_status(launch_tv(x, nxg, ny, nz, batch, prm->anisotropic != 0, prm->eps, prm->lam, gx,
                                 last && data_tv ? data_tv + 1 : nullptr, s));
        if (st != PH_OK)
            return st;
        st = to_status(launch_adam(x, gx, m, v, nimg, prm->lr, prm->beta1, prm->beta2, prm->adam_eps, t0 + it + 1, s));
        if (st != PH_OK)
            return st;
    }
    return PH_OK;
}

}  // namespace

extern "C" {

int ph_tv_iterate_par2d(const ph_geom2d *g, const float *rv, const float *proj, float *x, float *m, float *v, int t0,
                        int n_iter, const ph_tv_params *prm, void *ws, size_t ws_bytes, double *data_tv, int batch,
                        void *stream)
{
    CallScope scope;
    if (!g)
        return PH_ERR_NULL;
    if (batch < 1)
        return PH_ERR_SHAPE;
    Geom2D G;
    int st = make_geom2d(g, false, &G);
    if (st != PH_OK)
        return st;
    const size_t np = (size_t)batch * g->n_proj * g->det_shape, nimg = (size_t)batch * g->vol_shape[0] * g->vol_shape[1];
    auto fwd = [&](const float *img, float *sino) { return ph_project_par2d(g, rv, img, sino, batch, PH_F32, stream); };
    auto adj = [&](const float *sino, float *img) {
        return ph_project_adjoint_par2d(g, rv, sino, img, batch, PH_F32, stream);
    };
    return tv_iterate(fwd, adj, 1, g->vol_shape[0], g->vol_shape[1], np, nimg, proj, x, m, v, t0, n_iter, prm, ws,
                      ws_bytes, ph_tv_workspace_bytes_2d(g, batch), data_tv, batch, stream);
}

int ph_tv_iterate_fan2d(const ph_geom2d *g, const float *rv, const float *proj, float *x, float *m, float *v, int t0,
                        int n_iter, const ph_tv_params *prm, void *ws, size_t ws_bytes, double *data_tv, int batch,
                        void *stream)
{
    CallScope scope;
    if (!g)
        return PH_ERR_NULL;
    if (batch < 1)
        return PH_ERR_SHAPE;
    Geom2D G;
    int st = make_geom2d(g, true, &G);
    if (st != PH_OK)
        return st;
    const size_t np = (size_t)batch * g->n_proj * g->det_shape, nimg = (size_t)batch * g->vol_shape[0] * g->vol_shape[1];
    auto fwd = [&](const float *img, float *sino) { return ph_project_fan2d(g, rv, img, sino, batch, PH_F32, stream); };
    auto adj = [&](const float *sino, float *img) {
        return ph_project_adjoint_fan2d(g, rv, sino, img, batch, PH_F32, stream);
    };
    return tv_iterate(fwd, adj, 1, g->vol_shape[0], g->vol_shape[1], np, nimg, proj, x, m, v, t0, n_iter, prm, ws,
                      ws_bytes, ph_tv_workspace_bytes_2d(g, batch), data_tv, batch, stream);
}

int ph_tv_iterate_cone3d(const ph_geom3d *g, const float *mats, const float *proj, float *x, float *m, float *v,
                         int t0, int n_iter, const ph_tv_params *prm, void *ws, size_t ws_bytes, double *data_tv,
                         int batch, void *stream)
{
    CallScope scope;
    if (!g)
        return PH_ERR_NULL;
    if (batch < 1)
        return PH_ERR_SHAPE;
    Geom3D G;
    int st = make_geom3d(g, &G);
    if (st != PH_OK)
        return st;
    const size_t np = (size_t)batch * g->n_proj * g->det_shape[0] * g->det_shape[1];
    const size_t nimg = (size_t)batch * g->vol_shape[0] * g->vol_shape[1] * g->vol_shape[2];
    auto fwd = [&](const float *vol, float *pr) { return ph_project_cone3d(g, mats, vol, pr, batch, PH_F32, stream); };
    auto adj = [&](const float *pr, float *vol) {
        return ph_project_adjoint_cone3d(g, mats, pr, vol, batch, PH_F32, stream);
    };
    return tv_iterate(fwd, adj, g->vol_shape[0], g->vol_shape[1], g->vol_shape[2], np, nimg, proj, x, m, v, t0, n_iter,
                      prm, ws, ws_bytes, ph_tv_workspace_bytes_3d(g, batch), data_tv, batch, stream);
}

}  // extern "C"

