"""Seeded non-circular cone-beam trajectories, given as scanner poses and as
the projection matrices that describe them.

These stand in for the calibrated projection matrices of real scanners (a
C-arm, say) that the paper's trajectories may be built from, which are not
available here.  Each view is a pinhole camera: a source position S, a
principal ray direction n, detector axes e_u and e_v (with e_u, e_v, n
orthonormal), a source-detector distance D and a principal point (pu, pv)
in pixel units.  The matrix of the view is the usual camera matrix

    P = Kint [R | -R S],  R rows (e_u; e_v; n),
    Kint = [[D/du, 0, pu], [0, D/dv, pv], [0, 0, 1]],

which sends the world point of detector pixel (i, j),
S + D n + (j - pu) du e_u + (i - pv) dv e_v, to D * (j, i, 1).

The perturbations are those of a real orbit: the source distance and the
detector distance wobble from view to view, the orbit plane is tilted
(so the matrices have z terms in every row), the detector rolls about the
principal ray, the principal point is offset from the detector centre, the
angular steps jitter and the rotation centre is shifted off the world
origin.  No arithmetic of the reconstruction method is here: the poses are
inputs to the operators, and the matrices are their standard encoding.
"""
from __future__ import annotations

import math

import numpy as np


def _rot(axis, ang):
    """Rotation matrix about the unit vector ``axis`` by ``ang`` (Rodrigues)."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    return np.eye(3) + math.sin(ang) * K + (1.0 - math.cos(ang)) * (K @ K)


def perturbed_poses(spec, seed, tilt_deg=8.0, tilt_wobble_deg=3.0, roll_deg=4.0, sid_wobble=0.04,
                    sdd_wobble=0.03, offset_px=(3.5, -2.25), jitter_deg=0.3, iso_shift_mm=None):
    """Per-view poses of a perturbed orbit around the nominal circular scan of
    ``spec`` (a cone geometry).  Returns a dict of float64 arrays:
    ``src`` [n, 3], ``n`` [n, 3], ``e_u`` [n, 3], ``e_v`` [n, 3], ``sdd`` [n],
    ``pu`` [n], ``pv`` [n] (pixel units)."""
    rng = np.random.default_rng(seed)
    n_proj = spec.n_proj
    (nv, nu) = spec.det_shape
    beta = spec.angular_range * np.arange(n_proj) / n_proj + np.deg2rad(jitter_deg) * rng.uniform(-1, 1, n_proj)
    phase = rng.uniform(0, 2 * math.pi, 4)
    t = np.arange(n_proj) / max(n_proj, 1)
    if iso_shift_mm is None:
        half = 0.5 * min(n * s for n, s in zip(spec.vol_shape, spec.vol_spacing))
        iso_shift_mm = 0.04 * half
    iso = rng.uniform(-1, 1, 3) * iso_shift_mm
    out = {k: np.zeros((n_proj, 3)) for k in ("src", "n", "e_u", "e_v")}
    out.update(sdd=np.zeros(n_proj), pu=np.zeros(n_proj), pv=np.zeros(n_proj))
    tilt_axis = _rot([0.0, 0.0, 1.0], phase[3]) @ np.array([1.0, 0.0, 0.0])
    tilt0 = _rot(tilt_axis, np.deg2rad(tilt_deg))
    for k in range(n_proj):
        b = beta[k]
        c = np.array([math.cos(b), math.sin(b), 0.0])
        eu = np.array([-math.sin(b), math.cos(b), 0.0])
        ev = np.array([0.0, 0.0, 1.0])
        # a tilted orbit plane, wobbling along the orbit, and a roll of the
        # detector about the principal ray
        wob = _rot(eu, np.deg2rad(tilt_wobble_deg) * math.sin(2 * math.pi * t[k] + phase[0]))
        Rw = tilt0 @ wob
        c, eu, ev = Rw @ c, Rw @ eu, Rw @ ev
        roll = _rot(c, np.deg2rad(roll_deg) * math.sin(4 * math.pi * t[k] + phase[1]))
        eu, ev = roll @ eu, roll @ ev
        sid = spec.sid * (1.0 + sid_wobble * math.sin(2 * math.pi * t[k] + phase[2]))
        sdd = spec.sdd * (1.0 + sdd_wobble * math.cos(2 * math.pi * t[k] + phase[2]))
        out["src"][k] = iso - sid * c
        out["n"][k], out["e_u"][k], out["e_v"][k] = c, eu, ev
        out["sdd"][k] = sdd
        out["pu"][k] = 0.5 * (nu - 1) + offset_px[0] * (1.0 + 0.3 * math.sin(2 * math.pi * t[k]))
        out["pv"][k] = 0.5 * (nv - 1) + offset_px[1] * (1.0 + 0.3 * math.cos(2 * math.pi * t[k]))
    return out


def pose_matrices(spec, poses):
    """Camera matrices [n, 3, 4] (float64) of the poses (module docstring)."""
    (dv, du) = spec.det_spacing
    n_proj = len(poses["sdd"])
    P = np.zeros((n_proj, 3, 4))
    for k in range(n_proj):
        R = np.stack([poses["e_u"][k], poses["e_v"][k], poses["n"][k]])
        t = -R @ poses["src"][k]
        D = poses["sdd"][k]
        Kint = np.array([[D / du, 0.0, poses["pu"][k]], [0.0, D / dv, poses["pv"][k]], [0.0, 0.0, 1.0]])
        P[k, :, :3] = Kint @ R
        P[k, :, 3] = Kint @ t
    return P


def pixel_positions(spec, poses):
    """World positions [n, nv, nu, 3] of the detector pixel centres."""
    (nv, nu), (dv, du) = spec.det_shape, spec.det_spacing
    j = np.arange(nu, dtype=np.float64)
    i = np.arange(nv, dtype=np.float64)
    out = np.zeros((len(poses["sdd"]), nv, nu, 3))
    for k in range(len(poses["sdd"])):
        ctr = poses["src"][k] + poses["sdd"][k] * poses["n"][k]
        out[k] = (ctr[None, None, :] + ((j - poses["pu"][k]) * du)[None, :, None] * poses["e_u"][k][None, None, :]
                  + ((i - poses["pv"][k]) * dv)[:, None, None] * poses["e_v"][k][None, None, :])
    return out
