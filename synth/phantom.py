"""Seeded random ellipse / ellipsoid phantoms and their rasterisation.

The paper's phantom tools offer circles, ellipses, spheres and ellipsoids
(Sec. II.C.2); the workloads here use seeded random sets of them in place of
the Shepp-Logan phantoms, which are not available.

Parameter draws (all in units of the volume half-width ``hw``, which is half of
the smallest physical extent ``N*s`` of the grid):
  centres U[-0.8, 0.8], semi-axes U[0.05, 0.4], densities U[-0.5, 1],
  orientation angles U[0, pi).
Overlapping figures add.  Rasterisation is the mean of the indicator function
over ``sub**d`` regularly spaced sub-samples inside each voxel.

Voxel centres: voxel ``i`` along an axis sits at ``o + i*s`` with ``o`` the
world position of voxel 0 (default ``-(N-1)/2*s``, i.e. the grid is centred on
the rotation axis).
"""
from __future__ import annotations

import math

import numpy as np
import torch


def default_origin(shape, spacing):
    return tuple(-(n - 1) / 2.0 * s for n, s in zip(shape, spacing))


def grid_axes(shape, spacing, origin=None):
    """World coordinates (mm) of the voxel centres along each axis, same axis
    order as ``shape``."""
    if origin is None:
        origin = default_origin(shape, spacing)
    return [o + s * np.arange(n, dtype=np.float64) for n, s, o in zip(shape, spacing, origin)]


def _half_width(shape, spacing):
    return 0.5 * min(n * s for n, s in zip(shape, spacing))


def random_ellipses(seed, n, shape, spacing):
    """``n`` random ellipses for an image of ``shape=(ny, nx)`` and
    ``spacing=(sy, sx)``.  Returns float64 array ``[n, 6]`` with columns
    ``(cx, cy, a, b, theta, rho)``: centre (mm), semi-axes (mm) along the
    ellipse's own axes, rotation of the ``a`` axis from +x (rad), density
    (1/mm)."""
    rng = np.random.default_rng(seed)
    hw = _half_width(shape, spacing)
    out = np.empty((n, 6))
    out[:, 0:2] = rng.uniform(-0.8, 0.8, size=(n, 2)) * hw
    out[:, 2:4] = rng.uniform(0.05, 0.4, size=(n, 2)) * hw
    out[:, 4] = rng.uniform(0.0, math.pi, size=n)
    out[:, 5] = rng.uniform(-0.5, 1.0, size=n)
    return out


def _rot_zyx(a, b, c):
    """Rotation matrix Rz(a) @ Ry(b) @ Rx(c)."""
    ca, sa, cb, sb, cc, sc = map(float, (np.cos(a), np.sin(a), np.cos(b), np.sin(b), np.cos(c), np.sin(c)))
    rz = np.array([[ca, -sa, 0.0], [sa, ca, 0.0], [0.0, 0.0, 1.0]])
    ry = np.array([[cb, 0.0, sb], [0.0, 1.0, 0.0], [-sb, 0.0, cb]])
    rx = np.array([[1.0, 0.0, 0.0], [0.0, cc, -sc], [0.0, sc, cc]])
    return rz @ ry @ rx


def random_ellipsoids(seed, n, shape, spacing):
    """``n`` random ellipsoids for a volume of ``shape=(nz, ny, nx)``.
    Returns float64 array ``[n, 16]``: columns 0-2 centre ``(cx, cy, cz)`` mm,
    3-5 semi-axes mm, 6-14 the row-major rotation matrix ``R`` whose columns
    are the ellipsoid's axes in world coordinates, 15 density (1/mm)."""
    rng = np.random.default_rng(seed)
    hw = _half_width(shape, spacing)
    out = np.empty((n, 16))
    out[:, 0:3] = rng.uniform(-0.8, 0.8, size=(n, 3)) * hw
    out[:, 3:6] = rng.uniform(0.05, 0.4, size=(n, 3)) * hw
    ang = rng.uniform(0.0, math.pi, size=(n, 3))
    for e in range(n):
        out[e, 6:15] = _rot_zyx(*ang[e]).reshape(-1)
    out[:, 15] = rng.uniform(-0.5, 1.0, size=n)
    return out


def disk(radius, rho=1.0, centre=(0.0, 0.0)):
    """A single disk as an ellipse parameter row set."""
    return np.array([[centre[0], centre[1], radius, radius, 0.0, rho]], dtype=np.float64)


def sphere(radius, rho=1.0, centre=(0.0, 0.0, 0.0)):
    """A single sphere as an ellipsoid parameter row set."""
    row = np.zeros((1, 16))
    row[0, 0:3] = centre
    row[0, 3:6] = radius
    row[0, 6:15] = np.eye(3).reshape(-1)
    row[0, 15] = rho
    return row


def random_gaussians(seed, n, shape, spacing):
    """``n`` isotropic Gaussian blobs: centres U[-0.5, 0.5] * hw, widths
    sigma U[0.06, 0.15] * hw, amplitudes U[0.5, 1].  Returns float64
    ``[n, d+2]`` with columns ``(centre..., sigma, amplitude)``; the centre
    columns are in the order x, y[, z]."""
    rng = np.random.default_rng(seed)
    hw = _half_width(shape, spacing)
    d = len(shape)
    out = np.empty((n, d + 2))
    out[:, :d] = rng.uniform(-0.5, 0.5, size=(n, d)) * hw
    out[:, d] = rng.uniform(0.06, 0.15, size=n) * hw
    out[:, d + 1] = rng.uniform(0.5, 1.0, size=n)
    return out


def rasterize_gaussians(params, shape, spacing, origin=None, device="cpu", dtype=torch.float64):
    """Point samples of a sum of isotropic Gaussians at the voxel centres:
    ``amp * exp(-|x - c|^2 / (2 sigma^2))``.  Returns a torch tensor of
    ``shape``."""
    axes = grid_axes(shape, spacing, origin)
    d = len(shape)
    # axes are in array order (z,) y, x; centres are stored x, y(, z)
    coords = [torch.as_tensor(a, dtype=dtype, device=device) for a in axes]
    out = torch.zeros(tuple(shape), dtype=dtype, device=device)
    for row in np.asarray(params, dtype=np.float64):
        c = row[:d]
        sig, amp = float(row[d]), float(row[d + 1])
        r2 = torch.zeros(tuple(shape), dtype=dtype, device=device)
        for ax in range(d):
            world_axis = d - 1 - ax  # array axis 0 is the last world axis
            view = [1] * d
            view[ax] = shape[ax]
            r2 = r2 + ((coords[ax] - c[world_axis]) ** 2).view(view)
        out += amp * torch.exp(-r2 / (2.0 * sig * sig))
    return out


def _sub_offsets(sub, s):
    return [((m + 0.5) / sub - 0.5) * s for m in range(sub)]


def rasterize_ellipses(params, shape, spacing, origin=None, sub=4, device="cpu", dtype=torch.float64):
    """Mean indicator over ``sub*sub`` sub-samples per pixel, summed over the
    ellipses weighted by density.  Returns a torch tensor ``[ny, nx]``."""
    ny, nx = shape
    sy, sx = spacing
    ys, xs = grid_axes(shape, spacing, origin)
    y = torch.as_tensor(ys, dtype=dtype, device=device).view(ny, 1)
    x = torch.as_tensor(xs, dtype=dtype, device=device).view(1, nx)
    img = torch.zeros((ny, nx), dtype=dtype, device=device)
    oy_list, ox_list = _sub_offsets(sub, sy), _sub_offsets(sub, sx)
    for cx, cy, a, b, th, rho in np.asarray(params, dtype=np.float64):
        ct, st = math.cos(th), math.sin(th)
        cnt = torch.zeros((ny, nx), dtype=dtype, device=device)
        for oy in oy_list:
            for ox in ox_list:
                px = x + ox - cx
                py = y + oy - cy
                qa = (px * ct + py * st) / a
                qb = (-px * st + py * ct) / b
                cnt += (qa * qa + qb * qb <= 1.0).to(dtype)
        img += float(rho) * cnt / float(sub * sub)
    return img


def rasterize_ellipsoids(params, shape, spacing, origin=None, sub=2, device="cpu", dtype=torch.float64,
                         slab=16):
    """Mean indicator over ``sub**3`` sub-samples per voxel, summed over the
    ellipsoids weighted by density.  Returns a torch tensor ``[nz, ny, nx]``.
    Works slab by slab in z to bound temporary memory."""
    nz, ny, nx = shape
    sz, sy, sx = spacing
    zs, ys, xs = grid_axes(shape, spacing, origin)
    yv = torch.as_tensor(ys, dtype=dtype, device=device).view(1, ny, 1)
    xv = torch.as_tensor(xs, dtype=dtype, device=device).view(1, 1, nx)
    vol = torch.zeros((nz, ny, nx), dtype=dtype, device=device)
    offs = [(oz, oy, ox) for oz in _sub_offsets(sub, sz) for oy in _sub_offsets(sub, sy)
            for ox in _sub_offsets(sub, sx)]
    prm = np.asarray(params, dtype=np.float64)
    for z0 in range(0, nz, slab):
        z1 = min(nz, z0 + slab)
        zv = torch.as_tensor(zs[z0:z1], dtype=dtype, device=device).view(-1, 1, 1)
        acc = torch.zeros((z1 - z0, ny, nx), dtype=dtype, device=device)
        for row in prm:
            c = row[0:3]
            ax = row[3:6]
            r = row[6:15].reshape(3, 3)
            rho = float(row[15])
            # skip slabs the ellipsoid cannot reach (bounding sphere test)
            rmax = float(ax.max())
            if zs[z0] - 0.5 * sz > c[2] + rmax or zs[z1 - 1] + 0.5 * sz < c[2] - rmax:
                continue
            cnt = torch.zeros_like(acc)
            for oz, oy, ox in offs:
                px = xv + (ox - c[0])
                py = yv + (oy - c[1])
                pz = zv + (oz - c[2])
                # local coordinates q = R^T p (columns of R are the axes)
                q0 = (px * r[0, 0] + py * r[1, 0] + pz * r[2, 0]) / ax[0]
                q1 = (px * r[0, 1] + py * r[1, 1] + pz * r[2, 1]) / ax[1]
                q2 = (px * r[0, 2] + py * r[1, 2] + pz * r[2, 2]) / ax[2]
                cnt += (q0 * q0 + q1 * q1 + q2 * q2 <= 1.0).to(dtype)
            acc += rho * cnt / float(len(offs))
        vol[z0:z1] = acc
    return vol
