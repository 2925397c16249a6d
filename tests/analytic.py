"""Closed-form references used to pin the oracle.

Written independently of ``oracle/oracle.c``: the rays are constructed here
from the geometry conventions (view angle beta_k = k * range / n_proj counter-
clockwise, central ray c = (cos b, sin b, 0), detector axis e_u = (-sin b,
cos b, 0), e_v = +z, centred detector, source at -SID c, flat detector centred
at (SDD - SID) c; the curved fan detector is the arc of radius SDD about the
source, column u at fan angle u / SDD), and the line integrals of ellipses, ellipsoids and Gaussian
blobs are the textbook chord-length / Gaussian formulas.
"""
import math

import numpy as np


def view_angles(spec):
    return spec.angular_range * np.arange(spec.n_proj) / spec.n_proj


def detector_coords(spec):
    """(u [nu], v [nv]) pixel-centre coordinates in mm; v = [0] in 2D."""
    if spec.ndim == 2:
        nu, du = spec.det_shape[0], spec.det_spacing[0]
        return (np.arange(nu) - (nu - 1) / 2.0) * du, np.zeros(1)
    (nv, nu), (dv, du) = spec.det_shape, spec.det_spacing
    return (np.arange(nu) - (nu - 1) / 2.0) * du, (np.arange(nv) - (nv - 1) / 2.0) * dv


def rays(spec, views=None):
    """Point on each ray and its unit direction, arrays [n_views, nv, nu, 3]."""
    beta = view_angles(spec)
    if views is not None:
        beta = beta[np.asarray(views)]
    u, v = detector_coords(spec)
    B, V, U = np.meshgrid(beta, v, u, indexing="ij")
    c = np.stack([np.cos(B), np.sin(B), np.zeros_like(B)], -1)
    eu = np.stack([-np.sin(B), np.cos(B), np.zeros_like(B)], -1)
    ez = np.zeros_like(c)
    ez[..., 2] = 1.0
    if spec.kind == "par2d":
        return U[..., None] * eu, c
    src = -spec.sid * c
    if spec.kind == "fan2d_curved":
        # equiangular detector: column u sits at fan angle u / SDD on the arc
        # of radius SDD about the source
        gam = U / spec.sdd
        return src, np.cos(gam)[..., None] * c + np.sin(gam)[..., None] * eu
    det = (spec.sdd - spec.sid) * c + U[..., None] * eu + V[..., None] * ez
    d = det - src
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    return src, d


def _quadric_chord(p, d):
    """Length of the chord of the unit ball on the line p + t d (t in the
    units of d): roots of |p + t d|^2 = 1."""
    A = np.sum(d * d, -1)
    Bq = np.sum(p * d, -1)
    C = np.sum(p * p, -1) - 1.0
    disc = Bq * Bq - A * C
    return np.where(disc > 0, 2.0 * np.sqrt(np.maximum(disc, 0.0)) / A, 0.0)


def ellipse_line_integrals(params, a, d):
    """Sum over ellipses (cx, cy, A, B, theta, rho) of rho * chord length."""
    out = np.zeros(a.shape[:-1])
    for cx, cy, ea, eb, th, rho in np.asarray(params):
        ct, st = math.cos(th), math.sin(th)
        px, py = a[..., 0] - cx, a[..., 1] - cy
        # coordinates along the ellipse's own axes, scaled to the unit circle
        p = np.stack([(px * ct + py * st) / ea, (-px * st + py * ct) / eb], -1)
        q = np.stack([(d[..., 0] * ct + d[..., 1] * st) / ea, (-d[..., 0] * st + d[..., 1] * ct) / eb], -1)
        out += rho * _quadric_chord(p, q)
    return out


def ellipsoid_line_integrals(params, a, d):
    """Sum over ellipsoids (centre, semi-axes, R, rho) of rho * chord length."""
    out = np.zeros(a.shape[:-1])
    for row in np.asarray(params):
        c, ax, R, rho = row[0:3], row[3:6], row[6:15].reshape(3, 3), row[15]
        p = ((a - c) @ R) / ax   # R^T (a - c), row-vector form
        q = (d @ R) / ax
        out += rho * _quadric_chord(p, q)
    return out


def gaussian_line_integrals(params, a, d, dim):
    """Sum over isotropic Gaussians amp * exp(-r^2 / (2 s^2)) of the integral
    along the line: amp * sqrt(2 pi) s exp(-rho^2 / (2 s^2)), with rho the
    distance of the centre from the line."""
    out = np.zeros(a.shape[:-1])
    for row in np.asarray(params):
        c = np.zeros(3)
        c[:dim] = row[:dim]
        s, amp = row[dim], row[dim + 1]
        w = c - a
        t = np.sum(w * d, -1, keepdims=True)
        r2 = np.sum((w - t * d) ** 2, -1)
        out += amp * math.sqrt(2.0 * math.pi) * s * np.exp(-r2 / (2.0 * s * s))
    return out


def rel_l2(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm((x - ref).ravel()) / np.linalg.norm(ref.ravel()))
