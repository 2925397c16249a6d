"""FP64 CPU oracle of the known-operator CT path (PYRO-NN, arXiv 1904.13342).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check in
``__graft_entry__.py`` and the CPU-baseline leg of ``bench.py`` may import
this package.  It shares no code with the HIP library; both take their
inputs from ``synth``.

The arithmetic lives in ``oracle.c`` (plain C99, double precision, OpenMP over
output elements, no fast-math).  This module builds it with gcc, loads it with
ctypes and composes the FBP / FDK pipeline of Eq. 4 / Eq. 5:
``x = B( filter( W_red * W_cos * p ) )``.

Array conventions (float64, C-contiguous):
  2D image ``[ny, nx]``, sinogram ``[n_proj, nu]``;
  3D volume ``[nz, ny, nx]``, projections ``[n_proj, nv, nu]``.

Parity unpinned: none (see the oracle test-suite for the pin of every entry).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")


def build(force=True):
    """Compile oracle.c with gcc (-O2 -fopenmp, IEEE semantics)."""
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c99", "-D_GNU_SOURCE", "-O2", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
           "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Geom(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("sx", ctypes.c_double), ("sy", ctypes.c_double), ("sz", ctypes.c_double),
        ("ox", ctypes.c_double), ("oy", ctypes.c_double), ("oz", ctypes.c_double),
        ("nu", ctypes.c_int), ("nv", ctypes.c_int),
        ("du", ctypes.c_double), ("dv", ctypes.c_double),
        ("n_proj", ctypes.c_int),
        ("range", ctypes.c_double),
        ("sid", ctypes.c_double), ("sdd", ctypes.c_double),
        ("step", ctypes.c_double),
        ("mats", ctypes.POINTER(ctypes.c_double)),
    ]


_KIND = {"par2d": 0, "fan2d": 1, "cone3d": 2, "fan2d_curved": 3}
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        dp, ip, gp = P(ctypes.c_double), P(ctypes.c_int), P(_Geom)
        sig = {
            "ora_project": (None, [gp, dp, dp, ip, ctypes.c_int]),
            "ora_project_adjoint": (None, [gp, dp, dp]),
            "ora_count_samples": (ctypes.c_longlong, [gp, ip, ctypes.c_int]),
            "ora_backproject": (None, [gp, dp, dp, ip, ctypes.c_int]),
            "ora_backproject_adjoint": (None, [gp, dp, dp]),
            "ora_ramlak_filter": (None, [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp]),
            "ora_circular_filter": (None, [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp, dp]),
            "ora_ramlak_response": (None, [ctypes.c_int, ctypes.c_double, dp]),
            "ora_ramp_response": (None, [ctypes.c_int, ctypes.c_double, dp]),
            "ora_equiangular_filter": (None, [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp]),
            "ora_equiangular_response": (None, [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp]),
            "ora_cosine_weights": (None, [gp, dp]),
            "ora_parker": (ctypes.c_double, [ctypes.c_double, ctypes.c_double, ctypes.c_double]),
            "ora_redundancy_weights": (None, [gp, dp]),
            "ora_projection_matrices": (None, [gp, dp]),
            "ora_num_threads": (ctypes.c_int, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def geom(spec, mats=None):
    """Oracle geometry record from a ``synth.GeometrySpec``.  For a cone
    geometry, ``mats`` ([n_proj, 3, 4], any non-zero scale per view) gives the
    trajectory as projection matrices in place of the circular scan."""
    g = _Geom()
    g.kind = _KIND[spec.kind]
    org = spec.origin
    if spec.ndim == 2:
        (g.ny, g.nx), (g.sy, g.sx), (g.oy, g.ox) = spec.vol_shape, spec.vol_spacing, org
        g.nz, g.sz, g.oz = 1, 1.0, 0.0
        g.nu, g.nv, g.du, g.dv = spec.det_shape[0], 1, spec.det_spacing[0], 1.0
    else:
        (g.nz, g.ny, g.nx), (g.sz, g.sy, g.sx), (g.oz, g.oy, g.ox) = spec.vol_shape, spec.vol_spacing, org
        (g.nv, g.nu), (g.dv, g.du) = spec.det_shape, spec.det_spacing
    g.n_proj = spec.n_proj
    g.range = spec.angular_range
    g.sid, g.sdd = spec.sid, spec.sdd
    g.step = spec.step
    if mats is not None:
        if spec.kind != "cone3d":
            raise ValueError("projection matrices describe cone-beam trajectories only")
        m = np.ascontiguousarray(mats, dtype=np.float64).reshape(spec.n_proj, 12)
        if not np.all(np.isfinite(m)) or np.any(np.abs(np.linalg.det(m.reshape(-1, 3, 4)[:, :, :3])) == 0.0):
            raise ValueError("projection matrices must be finite with a non-singular 3x3 block")
        g._mats = m   # keeps the array alive for as long as the record
        g.mats = _dp(m)
    return g


def num_threads():
    return _load().ora_num_threads()


def _vol3(spec, f):
    f = np.ascontiguousarray(f, dtype=np.float64)
    return f.reshape((1,) + tuple(spec.vol_shape)) if spec.ndim == 2 else f.reshape(spec.vol_shape)


def _proj_shape(spec):
    return (spec.n_proj, 1, spec.det_shape[0]) if spec.ndim == 2 else (spec.n_proj,) + tuple(spec.det_shape)


def _out_proj(spec, p):
    return p.reshape(spec.n_proj, spec.det_shape[0]) if spec.ndim == 2 else p


def _out_vol(spec, f):
    return f.reshape(spec.vol_shape)


def _idx(sel):
    return None if sel is None else np.ascontiguousarray(sel, dtype=np.int32)


# ------------------------------------------------------------------ operators

def project(spec, f, views=None, mats=None):
    """Ray-driven forward projection A f (fixed-step multilinear sampling).
    With ``views`` only those views are computed; the others are zero.
    ``mats``: the trajectory as projection matrices (cone beams)."""
    g = geom(spec, mats)
    f3 = _vol3(spec, f)
    p = np.zeros(_proj_shape(spec))
    v = _idx(views)
    _load().ora_project(ctypes.byref(g), _dp(f3), _dp(p), _ip(v), 0 if v is None else len(v))
    return _out_proj(spec, p)


def project_adjoint(spec, p, mats=None):
    """Exact transpose A^T of ``project`` (scatter)."""
    g = geom(spec, mats)
    p3 = np.ascontiguousarray(p, dtype=np.float64).reshape(_proj_shape(spec))
    f = np.zeros((g.nz, g.ny, g.nx))
    _load().ora_project_adjoint(ctypes.byref(g), _dp(p3), _dp(f))
    return _out_vol(spec, f)


def count_samples(spec, views=None, mats=None):
    g = geom(spec, mats)
    v = _idx(views)
    return int(_load().ora_count_samples(ctypes.byref(g), _ip(v), 0 if v is None else len(v)))


def backproject(spec, q, slices=None, mats=None):
    """Voxel-driven, distance-weighted back-projection B q.  With ``slices``
    only those z slices are computed; the others are zero."""
    g = geom(spec, mats)
    q3 = np.ascontiguousarray(q, dtype=np.float64).reshape(_proj_shape(spec))
    f = np.zeros((g.nz, g.ny, g.nx))
    s = _idx(slices)
    _load().ora_backproject(ctypes.byref(g), _dp(q3), _dp(f), _ip(s), 0 if s is None else len(s))
    return _out_vol(spec, f)


def backproject_adjoint(spec, f, mats=None):
    """Exact transpose B^T of ``backproject`` (scatter)."""
    g = geom(spec, mats)
    f3 = _vol3(spec, f)
    q = np.zeros(_proj_shape(spec))
    _load().ora_backproject_adjoint(ctypes.byref(g), _dp(f3), _dp(q))
    return _out_proj(spec, q)


# -------------------------------------------------------------------- filters

def tau(spec):
    """Iso-scaled detector sample spacing of the ramp filter (for the curved
    fan detector: the angular pitch du/SDD times SID)."""
    du = spec.det_spacing[-1]
    return du if spec.kind == "par2d" else du * spec.sid / spec.sdd


def fan_angle_pitch(spec):
    """Angular pitch alpha = du / SDD of the curved (equiangular) detector."""
    return spec.det_spacing[-1] / spec.sdd


def fft_size(nu):
    """Smallest power of two >= 2*nu - 1 (linear convolution without wrap)."""
    m = 1
    while m < 2 * nu - 1:
        m *= 2
    return m


def ramlak_filter(rows, t):
    rows = np.ascontiguousarray(rows, dtype=np.float64)
    nu = rows.shape[-1]
    out = np.empty_like(rows)
    _load().ora_ramlak_filter(rows.size // nu, nu, float(t), _dp(rows), _dp(out))
    return out


def circular_filter(rows, K):
    rows = np.ascontiguousarray(rows, dtype=np.float64)
    K = np.ascontiguousarray(K, dtype=np.float64)
    nu = rows.shape[-1]
    out = np.empty_like(rows)
    _load().ora_circular_filter(rows.size // nu, nu, len(K), _dp(K), _dp(rows), _dp(out))
    return out


def ramlak_response(M, t):
    K = np.empty(M)
    _load().ora_ramlak_response(M, float(t), _dp(K))
    return K


def ramp_response(M, t):
    K = np.empty(M)
    _load().ora_ramp_response(M, float(t), _dp(K))
    return K


def equiangular_filter(rows, alpha, sid):
    """Equiangular Ram-Lak filtering of rows sampled at fan-angle pitch alpha."""
    rows = np.ascontiguousarray(rows, dtype=np.float64)
    nu = rows.shape[-1]
    out = np.empty_like(rows)
    _load().ora_equiangular_filter(rows.size // nu, nu, float(alpha), float(sid), _dp(rows), _dp(out))
    return out


def equiangular_response(M, alpha, sid):
    K = np.empty(M)
    _load().ora_equiangular_response(M, float(alpha), float(sid), _dp(K))
    return K


# -------------------------------------------------------------------- weights

def cosine_weights(spec):
    g = geom(spec)
    w = np.empty((g.nv, g.nu))
    _load().ora_cosine_weights(ctypes.byref(g), _dp(w))
    return w


def redundancy_weights(spec):
    g = geom(spec)
    w = np.empty((g.n_proj, g.nu))
    _load().ora_redundancy_weights(ctypes.byref(g), _dp(w))
    return w


def parker(beta, gamma, delta):
    return float(_load().ora_parker(float(beta), float(gamma), float(delta)))


def projection_matrices(spec):
    g = geom(spec)
    P = np.empty((g.n_proj, 3, 4))
    _load().ora_projection_matrices(ctypes.byref(g), _dp(P))
    return P


# ------------------------------------------------------------------ pipelines

def weight(spec, p, W_red=None, W=None):
    """W_red * W_cos (* W) * p  (Eq. 5 without the filter)."""
    p3 = np.asarray(p, dtype=np.float64).reshape(_proj_shape(spec))
    wc = cosine_weights(spec)
    wr = redundancy_weights(spec) if W_red is None else np.asarray(W_red, dtype=np.float64)
    out = p3 * wc[None, :, :] * wr[:, None, :]
    if W is not None:
        out = out * np.asarray(W, dtype=np.float64).reshape(wc.shape)[None]
    return out


def filter_projections(spec, p, K=None):
    """Row-wise ramp filtering: Ram-Lak (equiangular Ram-Lak on the curved
    fan detector) as a direct linear convolution when ``K`` is None,
    otherwise the circular filter with response ``K``."""
    p3 = np.asarray(p, dtype=np.float64).reshape(_proj_shape(spec))
    if K is None:
        if spec.kind == "fan2d_curved":
            return equiangular_filter(p3, fan_angle_pitch(spec), spec.sid)
        return ramlak_filter(p3, tau(spec))
    return circular_filter(p3, K)


def fbp(spec, p, W_red=None, K=None, W=None, slices=None, mats=None):
    """FBP / FDK, Eq. 4 / Eq. 5: x = B filter(W_red W_cos p).  With ``mats``
    the weights and the filter are those of the nominal circular geometry and
    the back-projection follows the given projection matrices."""
    q = filter_projections(spec, weight(spec, p, W_red=W_red, W=W), K=K)
    return backproject(spec, q, slices=slices, mats=mats)


# ------------------------------------------------------- learned corrector
#
# Sec. III.A (trainable projection-domain weights in the FDK network of Eq. 5,
# updated from a loss computed in the volume) and Sec. III.B / Eq. 6 (the
# filter K as the trainable layer, initialised with the ramp):
#     x = B q,  q = filter_K(r),  r = W * W_red * W_cos * p,
# trained on the mean squared error to the ground-truth volume with Adam.

def mse(x, ref, mask=None):
    """L = mean((m (x - ref))^2) and dL/dx = 2 m^2 (x - ref) / n."""
    x = np.asarray(x, dtype=np.float64)
    d = x - np.asarray(ref, dtype=np.float64)
    m = np.ones_like(d) if mask is None else np.asarray(mask, dtype=np.float64)
    return float(np.mean((m * d) ** 2)), 2.0 * m * m * d / d.size


def corrector_grad(spec, p, grad_q, K, W_red=None, W=None):
    """(dL/dK, dL/dW) for q = filter_K(W W_red W_cos p), given g = dL/dq;
    ``p`` and ``grad_q`` are [n_proj, nv, nu] or [batch, n_proj, nv, nu].

    The filter output is Re IDFT_M(K . DFT_M(r)) on zero-padded rows, which
    is linear in K:  q_n = (1/M) sum_f K[f] Re(R_f exp(2 pi i f n / M)).
    Hence dL/dK[f] = (1/M) sum over rows and n < nu of g_n Re(R_f exp(...)),
    which is (1/M) sum_rows Re(R_f conj(G_f)) with G = DFT_M(g) (g real) --
    taken here with K's symmetric part, the one the real output depends on:
    dL/dK[f] = (c[f] + c[M - f]) / 2.  The row filter is a circular
    convolution with an even kernel restricted to the first nu samples, so it
    is its own transpose: dL/dr = filter_K(g), and dL/dW[i][j] is the sum
    over batch and views of dL/dr * W_red * W_cos * p."""
    K = np.asarray(K, dtype=np.float64)
    M = len(K)
    shp = _proj_shape(spec)
    p4 = np.asarray(p, dtype=np.float64).reshape((-1,) + shp)
    g4 = np.asarray(grad_q, dtype=np.float64).reshape((-1,) + shp)
    nv, nu = shp[1], shp[2]
    c = np.zeros(M)
    dW = np.zeros((nv, nu))
    for b in range(p4.shape[0]):
        r = weight(spec, p4[b], W_red=W_red, W=W)
        R = np.fft.fft(r, n=M, axis=-1)
        G = np.fft.fft(g4[b], n=M, axis=-1)
        c += np.real(R * np.conj(G)).reshape(-1, M).sum(axis=0) / M
        dr = circular_filter(g4[b], K)
        dW += (dr * weight(spec, p4[b], W_red=W_red)).sum(axis=0)
    mirror = c[(M - np.arange(M)) % M]
    return 0.5 * (c + mirror), dW


def corrector_forward(spec, p, K, W_red=None, W=None):
    """x = B filter_K(W W_red W_cos p) for one set of projections."""
    return fbp(spec, p, W_red=W_red, K=K, W=W)


def adam(param, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba, Algorithm 1) on float64 copies; returns
    (param, m, v)."""
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return np.asarray(param, dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ------------------------------------------------- TV-regularised iteration
#
# Sec. III.B.1 / Eq. 7: an additive layer holding the image, forward
# projected, trained on the l2 data term plus lambda * TV.  Forward
# differences D_d(q) = x[q + e_d] - x[q], zero where q + e_d leaves the grid.
# Two readings: the isotropic total variation (the gradient magnitude per
# voxel, smoothed by eps), and the anisotropic one, the sum of absolute
# differences per axis, which is the total variation of the framework the
# paper computes TV with (eps = 0 gives it exactly; eps > 0 smooths each
# absolute value as sqrt(t^2 + eps^2)).

def _differences(x):
    D = []
    for ax in range(x.ndim):
        d = np.zeros_like(x)
        sl_hi = [slice(None)] * x.ndim
        sl_lo = [slice(None)] * x.ndim
        sl_hi[ax] = slice(1, None)
        sl_lo[ax] = slice(0, -1)
        d[tuple(sl_lo)] = x[tuple(sl_hi)] - x[tuple(sl_lo)]
        D.append(d)
    return D


def tv(x, eps, anisotropic=False):
    """Total variation of a 2D [ny, nx] or 3D [nz, ny, nx] array.
    Isotropic: TV_eps(x) = sum_q sqrt(sum_d D_d(q)^2 + eps^2).
    Anisotropic: sum_q sum_d sqrt(D_d(q)^2 + eps^2) (= sum |D_d(q)| at eps = 0)
    over the axes d of extent > 1."""
    x = np.asarray(x, dtype=np.float64)
    D = _differences(x)
    if anisotropic:
        # axes of extent 1 have no differences and add nothing
        return float(sum(np.sqrt(d * d + eps * eps).sum() for ax, d in enumerate(D) if x.shape[ax] > 1))
    s = np.full(x.shape, eps * eps)
    for d in D:
        s += d * d
    return float(np.sqrt(s).sum())


def tv_grad(x, eps, anisotropic=False):
    """Gradient of ``tv``.  With r_d(q) the derivative of the summand at q by
    D_d(q) -- D_d(q) / phi(q), phi(q) the isotropic summand, or
    D_d(q) / sqrt(D_d(q)^2 + eps^2) anisotropically (sign(D_d(q)) at eps = 0,
    0 where D_d(q) = 0) --
    dTV/dx[p] = -sum_d r_d(p) + sum_d [p - e_d in the grid] r_d(p - e_d)."""
    x = np.asarray(x, dtype=np.float64)
    D = _differences(x)
    if anisotropic:
        R = []
        for d in D:
            if eps > 0:
                R.append(d / np.sqrt(d * d + eps * eps))
            else:
                R.append(np.sign(d))
    else:
        s = np.full(x.shape, eps * eps)
        for d in D:
            s += d * d
        phi = np.sqrt(s)
        R = [d / phi for d in D]
    g = np.zeros_like(x)
    for ax, q in enumerate(R):
        g -= q
        sl_hi = [slice(None)] * x.ndim
        sl_lo = [slice(None)] * x.ndim
        sl_hi[ax] = slice(1, None)
        sl_lo[ax] = slice(0, -1)
        g[tuple(sl_hi)] += q[tuple(sl_lo)]
    return g


__all__ = [
    "build", "geom", "num_threads", "project", "project_adjoint", "count_samples", "backproject",
    "backproject_adjoint", "tau", "fft_size", "ramlak_filter", "circular_filter", "ramlak_response",
    "ramp_response", "fan_angle_pitch", "equiangular_filter", "equiangular_response", "cosine_weights",
    "redundancy_weights", "parker", "projection_matrices", "weight",
    "filter_projections", "fbp", "mse", "corrector_grad", "corrector_forward", "adam", "tv", "tv_grad",
]
