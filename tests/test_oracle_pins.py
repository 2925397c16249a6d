"""Pins of the FP64 oracle against things other than itself: closed-form line
integrals, exact invariants, brute force on tiny grids, textbook filter
identities and the analytic FBP/FDK of uniform objects.

Every test here runs on the CPU (no GPU marker)."""
import math

import numpy as np
import pytest

import analytic as an
import synth


# ----------------------------------------------------------------- geometries

def par2d(N, L=64.0, n_proj=36, rng_=math.pi, nu_fac=1.5):
    s = L / N
    nu = int(round(nu_fac * N))
    return synth.config("par2d_64").with_(vol_shape=(N, N), vol_spacing=(s, s), det_shape=(nu,),
                                          det_spacing=(L * nu_fac / nu,), n_proj=n_proj, angular_range=rng_)


def fan2d(N, L=256.0, n_proj=36, rng_=2 * math.pi):
    s = L / N
    nu = int(round(1.5 * N))
    return synth.config("fan2d_512").with_(vol_shape=(N, N), vol_spacing=(s, s), det_shape=(nu,),
                                           det_spacing=(L * 1.5 * 1.6 * 1.2 / nu,), n_proj=n_proj,
                                           angular_range=rng_)


def cone3d(N, L=96.0, n_proj=8, rng_=2 * math.pi, det_fac=1.6 * 1.3):
    s = L / N
    nd = int(round(det_fac * N))
    dd = L * det_fac / nd
    return synth.config("cone3d_256_short").with_(vol_shape=(N, N, N), vol_spacing=(s, s, s),
                                                  det_shape=(nd, nd), det_spacing=(dd, dd), n_proj=n_proj,
                                                  angular_range=rng_)


def _gauss_err(ora, spec, seed=1, n=4):
    g = synth.random_gaussians(seed, n, spec.vol_shape, spec.vol_spacing)
    f = synth.rasterize_gaussians(g, spec.vol_shape, spec.vol_spacing).numpy()
    p = ora.project(spec, f)
    a, d = an.rays(spec)
    if spec.ndim == 2:
        a, d = a[:, 0], d[:, 0]
    ref = an.gaussian_line_integrals(g, a, d, spec.ndim)
    return an.rel_l2(p, ref)


# --------------------------------------------- P1/P2: closed-form line integrals

@pytest.mark.parametrize("make", [par2d, fan2d], ids=["par2d", "fan2d"])
def test_gaussian_line_integrals_converge_2d(ora, make):
    e64, e128 = _gauss_err(ora, make(64)), _gauss_err(ora, make(128))
    # bilinear sampling of a smooth function: second-order convergence
    assert e128 < 2e-3, (e64, e128)
    assert e64 / e128 > 3.5, (e64, e128)


def test_gaussian_line_integrals_anisotropic_voxels(ora):
    """Unequal spacings per axis: each index coordinate uses its own spacing."""
    spec = par2d(64).with_(vol_shape=(96, 48), vol_spacing=(64.0 / 96, 64.0 / 48))
    assert _gauss_err(ora, spec) < 8e-3
    spec = cone3d(32).with_(vol_shape=(24, 32, 40), vol_spacing=(96.0 / 24, 96.0 / 32, 96.0 / 40))
    spec2 = cone3d(64).with_(vol_shape=(48, 64, 80), vol_spacing=(96.0 / 48, 96.0 / 64, 96.0 / 80))
    e1, e2 = _gauss_err(ora, spec, seed=2), _gauss_err(ora, spec2, seed=2)
    assert e2 < 1.5e-2 and e1 / e2 > 3.3, (e1, e2)


def test_gaussian_line_integrals_converge_cone(ora):
    e24, e48 = _gauss_err(ora, cone3d(24), seed=2), _gauss_err(ora, cone3d(48), seed=2)
    assert e48 < 2.5e-2, (e24, e48)
    assert e24 / e48 > 3.3, (e24, e48)


@pytest.mark.parametrize("make", [par2d, fan2d], ids=["par2d", "fan2d"])
def test_ellipse_line_integrals_converge(ora, make):
    errs = []
    for N in (64, 128, 256):
        spec = make(N)
        e = synth.random_ellipses(0, 10, spec.vol_shape, spec.vol_spacing)
        f = synth.rasterize_ellipses(e, spec.vol_shape, spec.vol_spacing).numpy()
        a, d = an.rays(spec)
        errs.append(an.rel_l2(ora.project(spec, f), an.ellipse_line_integrals(e, a[:, 0], d[:, 0])))
    # edges of indicator functions converge slowly, but steadily
    assert errs[2] < 0.025, errs
    assert errs[0] / errs[1] > 1.25 and errs[1] / errs[2] > 1.25, errs


def test_ellipsoid_line_integrals_converge(ora):
    errs = []
    for N in (24, 48):
        spec = cone3d(N)
        e = synth.random_ellipsoids(0, 12, spec.vol_shape, spec.vol_spacing)
        f = synth.rasterize_ellipsoids(e, spec.vol_shape, spec.vol_spacing).numpy()
        a, d = an.rays(spec)
        errs.append(an.rel_l2(ora.project(spec, f), an.ellipsoid_line_integrals(e, a, d)))
    assert errs[1] < 0.2 and errs[0] / errs[1] > 1.3, errs


@pytest.mark.parametrize("make", [par2d, fan2d], ids=["par2d", "fan2d"])
def test_disk_chord_same_in_every_view(ora, make):
    """A centred disk projects to the chord length 2 sqrt(r^2 - s^2) in every
    view (s = distance of the ray from the centre)."""
    errs = []
    for N in (64, 128, 256):
        spec = make(N)
        r = 0.3 * spec.vol_shape[0] * spec.vol_spacing[0]
        f = synth.rasterize_ellipses(synth.disk(r), spec.vol_shape, spec.vol_spacing).numpy()
        p = ora.project(spec, f)
        a, d = an.rays(spec)
        a, d = a[:, 0], d[:, 0]
        s = np.linalg.norm(a - np.sum(a * d, -1, keepdims=True) * d, axis=-1)
        ref = 2.0 * np.sqrt(np.maximum(r * r - s * s, 0.0))
        errs.append(an.rel_l2(p, ref))
    assert errs[2] < 0.02 and errs[0] > errs[1] > errs[2], errs


def test_sphere_chord(ora):
    errs = []
    for N in (24, 48):
        spec = cone3d(N)
        r = 0.3 * 96.0
        f = synth.rasterize_ellipsoids(synth.sphere(r), spec.vol_shape, spec.vol_spacing, sub=3).numpy()
        p = ora.project(spec, f)
        a, d = an.rays(spec)
        s = np.linalg.norm(a - np.sum(a * d, -1, keepdims=True) * d, axis=-1)
        errs.append(an.rel_l2(p, 2.0 * np.sqrt(np.maximum(r * r - s * s, 0.0))))
    assert errs[1] < 0.05 and errs[0] > 1.3 * errs[1], errs


def test_orientation_of_offcentre_blob(ora):
    """View 0 looks along +x with e_u = +y: a blob at +y lands on the upper
    half of the detector; a quarter turn later (view along +y, e_u = -x) a blob
    at -x lands there.  In 3D a blob at +z lands on rows above the centre."""
    spec = par2d(64, n_proj=4, rng_=2 * math.pi)
    g = np.array([[0.0, 15.0, 2.0, 1.0], [-15.0, 0.0, 2.0, 1.0]])
    for blob, view in ((g[:1], 0), (g[1:], 1)):
        f = synth.rasterize_gaussians(blob, spec.vol_shape, spec.vol_spacing).numpy()
        p = ora.project(spec, f)
        u = (np.arange(spec.det_shape[0]) - (spec.det_shape[0] - 1) / 2.0) * spec.det_spacing[0]
        assert abs(u[np.argmax(p[view])] - 15.0) <= spec.det_spacing[0]
    spec = cone3d(32, n_proj=4)
    blob = np.array([[0.0, 0.0, 20.0, 2.0, 1.0]])
    f = synth.rasterize_gaussians(blob, spec.vol_shape, spec.vol_spacing).numpy()
    p = ora.project(spec, f)
    nv = spec.det_shape[0]
    row = np.unravel_index(np.argmax(p[0]), p[0].shape)[0]
    v = (row - (nv - 1) / 2.0) * spec.det_spacing[0]
    assert abs(v - 20.0 * spec.sdd / spec.sid) <= 1.5 * spec.det_spacing[0]


# ------------------------------------------------------ P4: exact rotation covariance

@pytest.mark.parametrize("case", ["par2d", "fan2d", "cone3d"])
def test_quarter_turn_is_a_view_shift(ora, case):
    """Rotating the object by +90 deg about the axis shifts the sinogram by a
    quarter turn of views.  The anchored sample lattice rotates with the ray,
    so this holds to rounding."""
    if case == "par2d":
        spec, shift = par2d(32, n_proj=40, rng_=math.pi), 20
    elif case == "fan2d":
        spec, shift = fan2d(32, n_proj=36), 9
    else:
        spec, shift = cone3d(16, n_proj=8), 2
    rng = np.random.default_rng(5)
    f = rng.standard_normal(spec.vol_shape)
    # f'(x, y) = f(y, -x) rotates the object counter-clockwise by 90 deg;
    # with array axes (.., y, x) that is np.rot90 over (y, x) axes.
    fr = np.rot90(f, k=1, axes=(-1, -2)).copy()
    p, pr = ora.project(spec, f), ora.project(spec, fr)
    np.testing.assert_allclose(pr[shift:], p[:-shift], rtol=0, atol=1e-11 * np.abs(p).max())


def test_parallel_mass(ora):
    """Each parallel view integrates the whole object: sum_j p_kj du = s^2 sum f."""
    spec = par2d(64, n_proj=24)
    e = synth.random_ellipses(3, 10, spec.vol_shape, spec.vol_spacing)
    e[:, 0:2] *= 0.5
    f = synth.rasterize_ellipses(e, spec.vol_shape, spec.vol_spacing).numpy()
    p = ora.project(spec, f)
    mass = f.sum() * spec.vol_spacing[0] ** 2
    np.testing.assert_allclose(p.sum(1) * spec.det_spacing[0], mass, rtol=1e-3)


# ------------------------------------------------------------- P3: brute force adjoints

def _tiny(case):
    if case == "par2d":
        return synth.config("par2d_64").with_(vol_shape=(8, 8), vol_spacing=(1.0, 1.0), det_shape=(12,),
                                              det_spacing=(1.0,), n_proj=6, angular_range=math.pi)
    if case == "fan2d":
        return synth.config("fan2d_512").with_(vol_shape=(8, 8), vol_spacing=(1.0, 1.0), det_shape=(12,),
                                               det_spacing=(1.6,), n_proj=6, sid=20.0, sdd=32.0)
    return synth.config("cone3d_256_short").with_(vol_shape=(6, 6, 6), vol_spacing=(1.0, 1.0, 1.0),
                                                  det_shape=(8, 8), det_spacing=(1.7, 1.7), n_proj=4,
                                                  sid=20.0, sdd=32.0, angular_range=2 * math.pi)


def _dense(op, in_shape):
    n = int(np.prod(in_shape))
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        cols.append(np.asarray(op(e.reshape(in_shape))).ravel())
    return np.stack(cols, 1)


@pytest.mark.parametrize("case", ["par2d", "fan2d", "cone3d"])
def test_adjoints_equal_dense_transpose(ora, case):
    spec = _tiny(case)
    A = _dense(lambda f: ora.project(spec, f), spec.vol_shape)
    pshape = (spec.n_proj,) + tuple(spec.det_shape)
    At = _dense(lambda p: ora.project_adjoint(spec, p), pshape)
    assert np.abs(A).max() > 0
    np.testing.assert_allclose(At, A.T, rtol=0, atol=1e-12 * np.abs(A).max())
    B = _dense(lambda q: ora.backproject(spec, q), pshape)
    Bt = _dense(lambda f: ora.backproject_adjoint(spec, f), spec.vol_shape)
    assert np.abs(B).max() > 0
    np.testing.assert_allclose(Bt, B.T, rtol=0, atol=1e-12 * np.abs(B).max())
    # the pair is unmatched: B is not proportional to A^T
    scale = np.sum(B * A.T) / np.sum(A.T * A.T)
    assert np.linalg.norm(B - scale * A.T) > 1e-3 * np.linalg.norm(B)


@pytest.mark.parametrize("case", ["par2d", "fan2d", "cone3d"])
def test_adjoint_identity_random(ora, case):
    spec = {"par2d": par2d(48, n_proj=30), "fan2d": fan2d(48, n_proj=30), "cone3d": cone3d(20, n_proj=10)}[case]
    pshape = (spec.n_proj,) + tuple(spec.det_shape)
    x = synth.random_array(spec.vol_shape, 11)
    y = synth.random_array(pshape, 12)
    lhs = np.vdot(ora.project(spec, x), y)
    rhs = np.vdot(x, ora.project_adjoint(spec, y))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0) * 100
    lhs = np.vdot(ora.backproject(spec, y), x)
    rhs = np.vdot(y, ora.backproject_adjoint(spec, x))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0) * 100


# ----------------------------------------------------------------- P6: filters

def test_ramlak_response_identities(ora):
    tau = 0.625
    for M in (256, 1024, 2048):
        K = ora.ramlak_response(M, tau)
        # only the even taps survive in K[0] + K[M/2]: tau * 2 h(0)
        assert abs(K[0] + K[M // 2] - 1.0 / (2.0 * tau)) < 1e-12 / tau
        # DC is positive and close to 2 / (pi^2 tau M) (tail of sum 1/n^2)
        assert K[0] > 0 and abs(K[0] * math.pi ** 2 * tau * M / 2.0 - 1.0) < 0.02
        # mid-band follows the ramp |k| / (M tau)
        k = np.arange(1, M // 4)
        assert np.max(np.abs(K[k] - k / (M * tau))) < 2.0 / (math.pi ** 2 * tau * M) * 1.01
        np.testing.assert_allclose(K[1:], K[1:][::-1], rtol=0, atol=1e-12 / tau)
    R = ora.ramp_response(16, tau)
    assert R[0] == 0.0
    np.testing.assert_allclose(R[:9], np.arange(9) / (16 * tau), rtol=1e-15)
    np.testing.assert_allclose(R[9:], np.arange(7, 0, -1) / (16 * tau), rtol=1e-15)


def test_ramlak_direct_convolution_matches_fft_route(ora):
    """The direct linear convolution equals IFFT(K . FFT(zero-padded row))
    computed with numpy's FFT, for M >= 2 nu - 1."""
    tau, nu = 0.8, 50
    rows = synth.random_array((7, nu), 3)
    M = ora.fft_size(nu)
    K = ora.ramlak_response(M, tau)
    pad = np.zeros((7, M))
    pad[:, :nu] = rows
    ref = np.fft.ifft(np.fft.fft(pad, axis=1) * K, axis=1).real[:, :nu]
    np.testing.assert_allclose(ora.ramlak_filter(rows, tau), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    np.testing.assert_allclose(ora.circular_filter(rows, K), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_circular_filter_arbitrary_response(ora):
    """M < 2 nu - 1 wraps around: the circular sum equals Re IFFT(K . FFT)."""
    nu, M = 40, 64
    rows = synth.random_array((5, nu), 4)
    K = synth.random_array((M,), 5)
    pad = np.zeros((5, M))
    pad[:, :nu] = rows
    ref = np.fft.ifft(np.fft.fft(pad, axis=1) * K, axis=1).real[:, :nu]
    np.testing.assert_allclose(ora.circular_filter(rows, K), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


# ----------------------------------------------------------------- P7: Parker

def test_parker_complementary_rays(ora):
    """Every line measured in a short scan carries total weight 1: for each
    ray (beta, u) find, by intersecting the line with the source circle, the
    other source position beta' on it and the fan angle gamma' there."""
    sid, sdd = 750.0, 1200.0
    rng_ = 200.0 * math.pi / 180.0
    delta = 0.5 * (rng_ - math.pi)
    rng = np.random.default_rng(7)
    worst = 0.0
    for _ in range(3000):
        beta = rng.uniform(0, rng_)
        u = rng.uniform(-310, 310)
        c = np.array([math.cos(beta), math.sin(beta)])
        eu = np.array([-math.sin(beta), math.cos(beta)])
        src = -sid * c
        d = sdd * c + u * eu
        d /= np.linalg.norm(d)
        # second intersection of src + t d with |x| = sid (t != 0)
        t = -2.0 * np.dot(src, d)
        src2 = src + t * d
        beta2 = math.atan2(-src2[1], -src2[0]) % (2 * math.pi)
        c2 = np.array([math.cos(beta2), math.sin(beta2)])
        eu2 = np.array([-math.sin(beta2), math.cos(beta2)])
        d2 = -d  # the same line travelled from the other source
        gamma2 = math.atan2(np.dot(d2, eu2), np.dot(d2, c2))
        gamma = math.atan(u / sdd)
        w = ora.parker(beta, gamma, delta)
        w2 = ora.parker(beta2, gamma2, delta) if beta2 <= rng_ else 0.0
        worst = max(worst, abs(w + w2 - 1.0))
    assert worst < 1e-12, worst


def test_redundancy_weight_kinds(ora):
    assert np.all(ora.redundancy_weights(par2d(16, n_proj=8)) == 1.0)
    assert np.all(ora.redundancy_weights(fan2d(16, n_proj=8)) == 0.5)
    w = ora.redundancy_weights(synth.config("cone3d_256_short"))
    assert w.shape == (248, 620) and w.min() >= 0.0 and w.max() <= 1.0
    # the central column is weighted 1 over the middle of the scan
    assert w[124, 309] == 1.0


def test_cosine_weights(ora):
    spec = synth.config("cone3d_256_short")
    wc = ora.cosine_weights(spec)
    (nv, nu), (dv, du) = spec.det_shape, spec.det_spacing
    u = (np.arange(nu) - (nu - 1) / 2) * du
    v = (np.arange(nv) - (nv - 1) / 2) * dv
    # cosine of the angle between the pixel ray and the central ray
    ref = spec.sdd / np.linalg.norm(np.stack(np.broadcast_arrays(spec.sdd, u[None, :], v[:, None]), -1), axis=-1)
    np.testing.assert_allclose(wc, ref, rtol=1e-14)


# ------------------------------------------------------- P8: FBP / FDK constants

@pytest.mark.parametrize("make", [par2d, fan2d], ids=["par2d", "fan2d"])
def test_fbp_of_disk(ora, make):
    spec = make(128, n_proj=180) if make is par2d else make(128, n_proj=360)
    L = spec.vol_shape[0] * spec.vol_spacing[0]
    r = 0.3 * L
    f = synth.rasterize_ellipses(synth.disk(r, rho=1.0), spec.vol_shape, spec.vol_spacing).numpy()
    x = ora.fbp(spec, ora.project(spec, f))
    ys, xs = synth.grid_axes(spec.vol_shape, spec.vol_spacing)
    rr = np.hypot(ys[:, None], xs[None, :])
    # measured: interior within 3e-5, exterior within 2e-4
    assert abs(x[rr < 0.8 * r].mean() - 1.0) < 1e-3
    assert abs(x[(rr > 1.2 * r) & (rr < 1.5 * r)].mean()) < 1e-3


def test_fbp_fan_short_scan_offcentre_disk(ora):
    """Parker short scan: the distance weight and the redundancy weights no
    longer average out over a full turn."""
    spec = fan2d(128, n_proj=200, rng_=math.pi + 2 * 0.3)
    r, cx, cy = 0.12 * 256.0, 0.25 * 256.0, 0.075 * 256.0
    f = synth.rasterize_ellipses(synth.disk(r, centre=(cx, cy)), spec.vol_shape, spec.vol_spacing).numpy()
    x = ora.fbp(spec, ora.project(spec, f))
    ys, xs = synth.grid_axes(spec.vol_shape, spec.vol_spacing)
    inside = np.hypot(ys[:, None] - cy, xs[None, :] - cx) < 0.7 * r
    assert abs(x[inside].mean() - 1.0) < 1e-3


_SPHERE_C, _SPHERE_R = (15.0, -5.0, 18.0), 12.0


def _fdk_sphere(ora, rng_, n_proj):
    """FDK of a uniform sphere placed off-centre and above the mid-plane."""
    spec = cone3d(48, L=96.0, n_proj=n_proj, rng_=rng_).with_(sid=400.0, sdd=640.0)
    c, r = _SPHERE_C, _SPHERE_R
    f = synth.rasterize_ellipsoids(synth.sphere(r, centre=c), spec.vol_shape, spec.vol_spacing, sub=3).numpy()
    zs, ys, xs = synth.grid_axes(spec.vol_shape, spec.vol_spacing)
    iz = int(np.argmin(np.abs(zs - c[2])))
    sl = [iz - 1, iz, iz + 1]
    x = ora.fbp(spec, ora.project(spec, f), slices=sl)[sl]
    rr = np.hypot(ys[:, None] - c[1], xs[None, :] - c[0])
    return x, np.broadcast_to(rr < 0.6 * r, x.shape), np.broadcast_to((rr > 1.3 * r) & (rr < 1.6 * r), x.shape)


def test_fdk_of_sphere_full_and_short_scan(ora):
    x_full, inside, ring = _fdk_sphere(ora, 2 * math.pi, 120)
    # measured: interior within 1.2e-3 on the three slices through the centre
    assert abs(x_full[inside].mean() - 1.0) < 5e-3
    assert abs(x_full[ring].mean()) < 5e-3
    # Parker short scan over pi + 2 delta reproduces the full scan inside
    x_short, _, _ = _fdk_sphere(ora, math.pi + 2 * 0.2, 80)
    assert abs(x_short[inside].mean() - 1.0) < 5e-3
    assert an.rel_l2(x_short[inside], x_full[inside]) < 0.01


# --------------------------------------------- sample count and matrices

def test_sample_count_brute_force(ora):
    spec = cone3d(6, L=12.0, n_proj=3, det_fac=1.5)
    a, d = an.rays(spec)
    org = np.array(spec.origin[::-1])  # (ox, oy, oz)
    s = np.array(spec.vol_spacing[::-1])
    n = np.array(spec.vol_shape[::-1])
    # anchor at the point of the line closest to the isocentre
    anc = a - np.sum(a * d, -1, keepdims=True) * d
    total = 0
    for k in range(-200, 201):
        X = (anc + k * spec.step * d - org) / s
        total += int(np.sum(np.all((X > -1) & (X < n), -1)))
    assert total == ora.count_samples(spec) and total > 0


def test_projection_matrices_geometry(ora):
    spec = synth.config("cone3d_256_short").with_(n_proj=12)
    P = ora.projection_matrices(spec)
    beta = an.view_angles(spec)
    (nv, nu) = spec.det_shape
    u, v = an.detector_coords(spec)
    for k in range(spec.n_proj):
        c = np.array([math.cos(beta[k]), math.sin(beta[k]), 0.0])
        eu = np.array([-math.sin(beta[k]), math.cos(beta[k]), 0.0])
        src = -spec.sid * c
        np.testing.assert_allclose(P[k] @ np.append(src, 1.0), 0.0, atol=1e-9)
        for (i, j) in ((0, 0), (nv - 1, nu - 1), (17, 400)):
            pix = (spec.sdd - spec.sid) * c + u[j] * eu + np.array([0, 0, v[i]])
            h = P[k] @ np.append(pix, 1.0)
            np.testing.assert_allclose(h[:2] / h[2], (j, i), atol=1e-9)
            np.testing.assert_allclose(h[2], spec.sdd, rtol=1e-12)


@pytest.mark.parametrize("make", [par2d, fan2d], ids=["par2d", "fan2d"])
def test_fbp_of_offcentre_disk(ora, make):
    """Off-centre objects see the distance weight (SID/w)^2 at first order."""
    spec = make(128, n_proj=180) if make is par2d else make(128, n_proj=360)
    L = spec.vol_shape[0] * spec.vol_spacing[0]
    r, cx = 0.12 * L, 0.3 * L
    f = synth.rasterize_ellipses(synth.disk(r, rho=1.0, centre=(cx, 0.0)), spec.vol_shape,
                                 spec.vol_spacing).numpy()
    x = ora.fbp(spec, ora.project(spec, f))
    ys, xs = synth.grid_axes(spec.vol_shape, spec.vol_spacing)
    rr = np.hypot(ys[:, None], xs[None, :] - cx)
    assert abs(x[rr < 0.7 * r].mean() - 1.0) < 0.01
    assert an.rel_l2(x[rr < 0.7 * r], np.ones(int((rr < 0.7 * r).sum()))) < 0.02


def test_sample_lattice_is_centred(ora):
    """Samples sit at a + k*step*d with a the point of the ray closest to the
    isocentre.  Reflecting the object along a ray through that point maps the
    sample set onto itself, so those line integrals are exactly unchanged."""
    rng = np.random.default_rng(9)
    # parallel, view 0 looks along +x: every ray is mapped onto itself by x -> -x
    spec = par2d(24, n_proj=4, rng_=2 * math.pi).with_(step_mm=0.37)
    f = rng.standard_normal(spec.vol_shape)
    p, pf = ora.project(spec, f), ora.project(spec, f[:, ::-1].copy())
    np.testing.assert_allclose(pf[0], p[0], rtol=0, atol=1e-12 * np.abs(p).max())
    # fan / cone: the central ray of view 0 (odd detector), SID not a multiple of the step
    fan = fan2d(24, n_proj=4).with_(det_shape=(37,), sid=300.3, sdd=480.0, step_mm=0.37)
    f = rng.standard_normal(fan.vol_shape)
    p, pf = ora.project(fan, f), ora.project(fan, f[:, ::-1].copy())
    assert abs(pf[0, 18] - p[0, 18]) < 1e-12 * np.abs(p).max()
    cone = cone3d(12, n_proj=4).with_(det_shape=(21, 21), sid=300.3, sdd=480.0, step_mm=0.37)
    f = rng.standard_normal(cone.vol_shape)
    p, pf = ora.project(cone, f), ora.project(cone, f[:, :, ::-1].copy())
    assert abs(pf[0, 10, 10] - p[0, 10, 10]) < 1e-12 * np.abs(p).max()


@pytest.mark.parametrize("case", ["par2d", "fan2d", "cone3d"])
def test_fbp_reproduces_gaussian_blobs(ora, case):
    """FBP / FDK of smooth blobs reproduces them point by point; sensitive to
    detector centring and to the magnification of the back-projection (blobs
    sit well above and below the mid-plane in 3D)."""
    if case == "par2d":
        spec, tol = par2d(128, n_proj=180), 6e-3       # measured 2.9e-3
    elif case == "fan2d":
        spec, tol = fan2d(128, n_proj=360), 7e-3       # measured 3.5e-3
    else:
        spec, tol = cone3d(48, L=96.0, n_proj=120).with_(sid=400.0, sdd=640.0), 0.04  # measured 2.7e-2
    g = synth.random_gaussians(4, 5, spec.vol_shape, spec.vol_spacing)
    if case == "cone3d":
        g[:, 2] = (20.0, -18.0, 15.0, -10.0, 22.0)
    f = synth.rasterize_gaussians(g, spec.vol_shape, spec.vol_spacing).numpy()
    x = ora.fbp(spec, ora.project(spec, f))
    assert an.rel_l2(x, f) < tol


@pytest.mark.parametrize("case", ["par2d", "fan2d", "cone3d"])
def test_backprojection_of_linear_ramps(ora, case):
    """Linear interpolation is exact on linear data, so back-projecting the
    detector coordinates themselves (q = u, q = v in mm, every view) gives, at
    each voxel, dbeta * sum_k weight_k * (coordinate of the voxel's projection)
    -- computed here from the projection geometry: parallel u = x.e_u; fan /
    cone u = SDD x.e_u / w, v = SDD z / w, weight (SID / w)^2, w = SID + x.c."""
    spec = {"par2d": par2d(16, n_proj=12), "fan2d": fan2d(16, n_proj=12),
            "cone3d": cone3d(12, L=24.0, n_proj=10, rng_=1.3 * math.pi, det_fac=3.5).with_(sid=60.0, sdd=150.0)}[case]
    u, v = an.detector_coords(spec)
    beta = an.view_angles(spec)
    dbeta = spec.angular_range / spec.n_proj
    pts = np.stack(np.meshgrid(*synth.grid_axes(spec.vol_shape, spec.vol_spacing), indexing="ij"), -1)
    if spec.ndim == 2:
        y, x, z = pts[..., 0], pts[..., 1], np.zeros(spec.vol_shape)
    else:
        z, y, x = pts[..., 0], pts[..., 1], pts[..., 2]
    ref_u, ref_v = np.zeros(spec.vol_shape), np.zeros(spec.vol_shape)
    inside = np.ones(spec.vol_shape, bool)
    for b in beta:
        xu = -x * math.sin(b) + y * math.cos(b)
        if case == "par2d":
            pu, pv, wt = xu, 0 * xu, 1.0
        else:
            w = spec.sid + x * math.cos(b) + y * math.sin(b)
            pu, pv, wt = spec.sdd * xu / w, spec.sdd * z / w, (spec.sid / w) ** 2
        ref_u += dbeta * wt * pu
        ref_v += dbeta * wt * pv
        inside &= (np.abs(pu) <= u.max()) & (np.abs(pv) <= max(v.max(), 0.0))
    assert inside.sum() > 0.3 * inside.size
    qu = np.broadcast_to(u, (spec.n_proj,) + tuple(spec.det_shape[:-1]) + (len(u),)).copy()
    bu = ora.backproject(spec, qu)
    scale = spec.angular_range * max(u.max(), v.max())  # size of the summed terms
    np.testing.assert_allclose(bu[inside], ref_u[inside], rtol=0, atol=1e-12 * scale)
    if case == "cone3d":
        qv = np.broadcast_to(v[:, None], (spec.n_proj, len(v), len(u))).copy()
        bv = ora.backproject(spec, qv)
        np.testing.assert_allclose(bv[inside], ref_v[inside], rtol=0, atol=1e-12 * scale)
