"""Pins of the oracle's projection-matrix path (trajectories given as
projection matrices, Sec. II.C.3) against things other than itself:

* on the circular trajectory the matrices reproduce the circular operators,
  which closed forms pin elsewhere, whatever scale each matrix carries;
* on a perturbed orbit (tilted, wobbling, rolled detector, offset principal
  point, shifted rotation centre) the line integrals of Gaussian blobs and of
  a sphere, along rays built here from the scanner poses, converge to the
  closed forms;
* back-projecting linear detector data gives the closed form computed here
  by intersecting the line from the source with the detector plane;
* the transposes equal the dense transposes, and a rotation of the world
  that maps the grid onto itself is a rotation of the volume.

Every test runs on the CPU."""
import math

import numpy as np
import pytest

import analytic as an
import synth


def cone(N, L=96.0, n_proj=8, rng_=2 * math.pi, det_fac=2.2, sid=300.0, sdd=500.0):
    s = L / N
    nd = int(round(det_fac * N))
    dd = L * det_fac / nd
    return synth.config("cone3d_256_short").with_(vol_shape=(N, N, N), vol_spacing=(s, s, s), det_shape=(nd, nd),
                                                  det_spacing=(dd, dd), n_proj=n_proj, angular_range=rng_, sid=sid,
                                                  sdd=sdd)


def _pose_rays(spec, poses):
    src = poses["src"][:, None, None, :]
    pix = synth.pixel_positions(spec, poses)
    d = pix - src
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    return np.broadcast_to(src, d.shape), d


RAGGED = synth.config("cone3d_crop32").with_(vol_shape=(9, 11, 13), vol_spacing=(1.1, 0.9, 1.0),
                                             det_shape=(15, 17), det_spacing=(1.7, 1.5), n_proj=7,
                                             angular_range=200 * math.pi / 180, sid=60.0, sdd=100.0,
                                             vol_origin=(-4.0, -5.5, -6.5))


def test_circular_matrices_reproduce_circular_operators(ora):
    spec = RAGGED
    P = ora.projection_matrices(spec)
    # any non-zero scale, negative included, describes the same view
    P = P * np.array([1.0, -2.5, 0.01, 7.0, -1.0, 3.0, 1e3])[:, None, None]
    f = synth.random_array(spec.vol_shape, 1)
    q = synth.random_array((spec.n_proj,) + tuple(spec.det_shape), 2)
    for name, op, x in (("A", ora.project, f), ("A^T", ora.project_adjoint, q), ("B", ora.backproject, q),
                        ("B^T", ora.backproject_adjoint, f)):
        ref = op(spec, x)
        got = op(spec, x, mats=P)
        assert np.abs(ref).max() > 0, name
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max(), err_msg=name)
    assert ora.count_samples(spec, mats=P) == ora.count_samples(spec)


def test_gaussian_line_integrals_perturbed_orbit(ora):
    """Smooth blobs: second-order convergence of the trilinear sampler along
    rays from the poses (source to pixel centre)."""
    errs = []
    for N in (24, 48):
        spec = cone(N)
        poses = synth.perturbed_poses(spec, 3)
        P = synth.pose_matrices(spec, poses)
        g = synth.random_gaussians(5, 4, spec.vol_shape, spec.vol_spacing)
        f = synth.rasterize_gaussians(g, spec.vol_shape, spec.vol_spacing).numpy()
        a, d = _pose_rays(spec, poses)
        ref = an.gaussian_line_integrals(g, a, d, 3)
        errs.append(an.rel_l2(ora.project(spec, f, mats=P), ref))
    assert errs[1] < 2.5e-2 and errs[0] / errs[1] > 3.3, errs


def test_sphere_chord_perturbed_orbit(ora):
    """An off-centre sphere: the chord 2 sqrt(r^2 - s^2) of each ray from the
    poses, s the distance of the sphere's centre from the ray."""
    errs = []
    for N in (24, 48):
        spec = cone(N)
        poses = synth.perturbed_poses(spec, 4)
        P = synth.pose_matrices(spec, poses)
        r, c = 0.25 * 96.0, np.array([6.0, -4.0, 5.0])
        f = synth.rasterize_ellipsoids(synth.sphere(r, centre=tuple(c)), spec.vol_shape, spec.vol_spacing,
                                       sub=3).numpy()
        a, d = _pose_rays(spec, poses)
        w = c - a
        s = np.linalg.norm(w - np.sum(w * d, -1, keepdims=True) * d, axis=-1)
        ref = 2.0 * np.sqrt(np.maximum(r * r - s * s, 0.0))
        errs.append(an.rel_l2(ora.project(spec, f, mats=P), ref))
    assert errs[1] < 0.05 and errs[0] > 1.3 * errs[1], errs


def test_backprojection_of_linear_detector_data(ora):
    """q_k(i, j) = alpha_k j + beta_k i + gamma_k is reproduced exactly by
    bilinear interpolation inside the detector, so B q at a voxel x is
    dbeta * sum_k (SID / w_k)^2 (alpha_k j_k + beta_k i_k + gamma_k), with
    (j_k, i_k) where the line from the source through x meets the detector
    plane and w_k = n_k . (x - S_k) the depth along the principal ray."""
    spec = cone(10, L=20.0, n_proj=9, rng_=1.4 * math.pi, det_fac=6.0, sid=60.0, sdd=150.0)
    poses = synth.perturbed_poses(spec, 5, tilt_deg=12.0, offset_px=(2.5, -1.75))
    P = synth.pose_matrices(spec, poses)
    (nv, nu), (dv, du) = spec.det_shape, spec.det_spacing
    coef = synth.random_array((spec.n_proj, 3), 6)
    jj, ii = np.meshgrid(np.arange(nu), np.arange(nv))
    q = coef[:, 0, None, None] * jj + coef[:, 1, None, None] * ii + coef[:, 2, None, None]
    zs, ys, xs = synth.grid_axes(spec.vol_shape, spec.vol_spacing)
    X = np.stack(np.meshgrid(xs, ys, zs, indexing="ij"), -1).transpose(2, 1, 0, 3)   # [z, y, x, (x, y, z)]
    dbeta = spec.angular_range / spec.n_proj
    ref = np.zeros(spec.vol_shape)
    inside = np.ones(spec.vol_shape, bool)
    for k in range(spec.n_proj):
        S, n, eu, ev, D = (poses[key][k] for key in ("src", "n", "e_u", "e_v", "sdd"))
        rel = X - S
        w = rel @ n
        hit = rel * (D / w)[..., None]             # from the source to the detector plane
        j = (hit @ eu) / du + poses["pu"][k]
        i = (hit @ ev) / dv + poses["pv"][k]
        inside &= (j > 0) & (j < nu - 1) & (i > 0) & (i < nv - 1)
        ref += dbeta * (spec.sid / w) ** 2 * (coef[k, 0] * j + coef[k, 1] * i + coef[k, 2])
    assert inside.all()
    got = ora.backproject(spec, q, mats=P)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_transposes_equal_dense_transposes(ora):
    spec = cone(6, L=6.0, n_proj=3, det_fac=1.5, sid=20.0, sdd=32.0).with_(vol_shape=(5, 6, 7),
                                                                           vol_spacing=(1.0, 1.1, 0.9),
                                                                           det_shape=(7, 8), det_spacing=(1.6, 1.5))
    P = synth.pose_matrices(spec, synth.perturbed_poses(spec, 7, tilt_deg=15.0))

    def dense(op, shape):
        n = int(np.prod(shape))
        cols = []
        for t in range(n):
            e = np.zeros(n)
            e[t] = 1.0
            cols.append(np.asarray(op(e.reshape(shape))).ravel())
        return np.stack(cols, 1)

    pshape = (spec.n_proj,) + tuple(spec.det_shape)
    A = dense(lambda f: ora.project(spec, f, mats=P), spec.vol_shape)
    At = dense(lambda p: ora.project_adjoint(spec, p, mats=P), pshape)
    assert np.abs(A).max() > 0
    np.testing.assert_allclose(At, A.T, rtol=0, atol=1e-12 * np.abs(A).max())
    B = dense(lambda q: ora.backproject(spec, q, mats=P), pshape)
    Bt = dense(lambda f: ora.backproject_adjoint(spec, f, mats=P), spec.vol_shape)
    assert np.abs(B).max() > 0
    np.testing.assert_allclose(Bt, B.T, rtol=0, atol=1e-12 * np.abs(B).max())


def test_world_rotation_is_volume_rotation(ora):
    """Composing every matrix with a rotation of the world that maps the
    (cubic, centred) grid onto itself equals rotating the volume: exact for
    the sampler (the anchor stays closest to the origin, the lattice turns
    with it) and for the back-projector."""
    spec = cone(12, L=24.0, n_proj=5, det_fac=2.5, sid=60.0, sdd=110.0)
    P = synth.pose_matrices(spec, synth.perturbed_poses(spec, 8, iso_shift_mm=0.0))
    # world point X' = R X with R: (x, y, z) -> (x, -z, y)
    R = np.array([[1, 0, 0, 0], [0, 0, -1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.float64)
    Pr = P @ R
    f = synth.random_array(spec.vol_shape, 9)
    # voxel [iz, iy, ix] at world (x, y, z) is seen at (x, -z, y): voxel [iy, n-1-iz, ix]
    fr = np.ascontiguousarray(np.transpose(f[:, ::-1, :], (1, 0, 2)))
    p, pr = ora.project(spec, f, mats=P), ora.project(spec, fr, mats=Pr)
    np.testing.assert_allclose(pr, p, rtol=0, atol=1e-12 * np.abs(p).max())
    q = synth.random_array((spec.n_proj,) + tuple(spec.det_shape), 10)
    b, br = ora.backproject(spec, q, mats=P), ora.backproject(spec, q, mats=Pr)
    expect = np.ascontiguousarray(np.transpose(b[:, ::-1, :], (1, 0, 2)))
    np.testing.assert_allclose(br, expect, rtol=0, atol=1e-12 * np.abs(b).max())


def test_matrix_path_rejects_bad_input(ora):
    spec = RAGGED
    P = ora.projection_matrices(spec)
    with pytest.raises(ValueError):
        ora.project(spec, np.zeros(spec.vol_shape), mats=P * np.nan)
    bad = P.copy()
    bad[0, :, :3] = 0.0
    with pytest.raises(ValueError):
        ora.project(spec, np.zeros(spec.vol_shape), mats=bad)
    with pytest.raises(ValueError):
        ora.project(synth.config("par2d_64"), np.zeros((64, 64)), mats=P)
