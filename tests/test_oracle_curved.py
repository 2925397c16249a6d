"""Pins of the oracle's curved (equiangular) fan-beam detector, the variant of
the fan geometry with equal angular spacing of the detector columns (Kak &
Slaney's equiangular rays; the paper names fan beams in Sec. II.B.2 and the
Kak & Slaney weights and filters in Sec. II.C.4-5).

Closed forms and invariants only: analytic line integrals, the chord of a
disk, dense transposes on a tiny grid, the small-angle limit of the
equiangular Ram-Lak taps, and the FBP of uniform and smooth objects (full and
Parker short scans), which fixes every weight and constant of the pipeline."""
import math

import numpy as np
import pytest

import analytic as an
import synth


def curved(N, L=256.0, n_proj=36, rng_=2 * math.pi):
    s = L / N
    nu = int(round(1.5 * N))
    return synth.config("fan2d_512").with_(kind="fan2d_curved", vol_shape=(N, N), vol_spacing=(s, s),
                                           det_shape=(nu,), det_spacing=(L * 1.5 * 1.6 * 1.2 / nu,),
                                           n_proj=n_proj, angular_range=rng_)


def flat(N, **kw):
    return curved(N, **kw).with_(kind="fan2d")


def test_gaussian_line_integrals_converge(ora):
    errs = []
    for N in (64, 128):
        spec = curved(N)
        g = synth.random_gaussians(1, 4, spec.vol_shape, spec.vol_spacing)
        f = synth.rasterize_gaussians(g, spec.vol_shape, spec.vol_spacing).numpy()
        a, d = an.rays(spec)
        errs.append(an.rel_l2(ora.project(spec, f), an.gaussian_line_integrals(g, a[:, 0], d[:, 0], 2)))
    assert errs[1] < 2e-3 and errs[0] / errs[1] > 3.5, errs


def test_disk_chord_same_in_every_view(ora):
    errs = []
    for N in (64, 128, 256):
        spec = curved(N)
        r = 0.3 * spec.vol_shape[0] * spec.vol_spacing[0]
        f = synth.rasterize_ellipses(synth.disk(r), spec.vol_shape, spec.vol_spacing).numpy()
        p = ora.project(spec, f)
        a, d = an.rays(spec)
        a, d = a[:, 0], d[:, 0]
        s = np.linalg.norm(a - np.sum(a * d, -1, keepdims=True) * d, axis=-1)
        errs.append(an.rel_l2(p, 2.0 * np.sqrt(np.maximum(r * r - s * s, 0.0))))
    assert errs[2] < 0.02 and errs[0] > errs[1] > errs[2], errs


def test_columns_are_equiangular(ora):
    """A narrow off-axis blob is seen by the columns around its fan angle: the
    projection is symmetric about column atan2(x.e_u, SID + x.c) / alpha +
    (nu-1)/2 (equal angles per column), several columns away from where a flat
    detector would put it (SDD tan(gamma) / du)."""
    spec = synth.config("fan2d_512").with_(kind="fan2d_curved", vol_shape=(256, 256), vol_spacing=(1.0, 1.0),
                                           det_shape=(512,), det_spacing=(1.0,), n_proj=8, sid=300.0, sdd=480.0)
    cx, cy, sig = 95.0, 20.0, 2.0
    g = np.array([[cx, cy, sig, 1.0]])
    f = synth.rasterize_gaussians(g, spec.vol_shape, spec.vol_spacing).numpy()
    p = ora.project(spec, f)
    alpha = ora.fan_angle_pitch(spec)
    nu = spec.det_shape[0]
    cols = np.arange(nu)
    shifts = []
    for k, b in enumerate(an.view_angles(spec)):
        xu = -cx * math.sin(b) + cy * math.cos(b)
        w = cx * math.cos(b) + cy * math.sin(b) + spec.sid
        j_curved = math.atan2(xu, w) / alpha + (nu - 1) / 2
        j_flat = spec.sdd * xu / w / spec.det_spacing[0] + (nu - 1) / 2
        row = p[k]
        centroid = float(np.sum(row * cols) / np.sum(row))
        assert abs(centroid - j_curved) < 0.02, (k, centroid, j_curved, j_flat)
        shifts.append(abs(j_flat - j_curved))
    assert max(shifts) > 2.0, shifts


@pytest.mark.parametrize("what", ["A", "B"])
def test_adjoints_equal_dense_transpose(ora, what):
    spec = synth.config("fan2d_512").with_(kind="fan2d_curved", vol_shape=(8, 8), vol_spacing=(1.0, 1.0),
                                           det_shape=(12,), det_spacing=(1.6,), n_proj=6, sid=20.0, sdd=32.0)
    pshape = (spec.n_proj,) + tuple(spec.det_shape)

    def dense(op, in_shape):
        n = int(np.prod(in_shape))
        cols = []
        for i in range(n):
            e = np.zeros(n)
            e[i] = 1.0
            cols.append(np.asarray(op(e.reshape(in_shape))).ravel())
        return np.stack(cols, 1)

    if what == "A":
        M = dense(lambda f: ora.project(spec, f), spec.vol_shape)
        Mt = dense(lambda p: ora.project_adjoint(spec, p), pshape)
    else:
        M = dense(lambda q: ora.backproject(spec, q), pshape)
        Mt = dense(lambda f: ora.backproject_adjoint(spec, f), spec.vol_shape)
    assert np.abs(M).max() > 0
    np.testing.assert_allclose(Mt, M.T, rtol=0, atol=1e-12 * np.abs(M).max())


def test_equiangular_taps_small_angle_limit(ora):
    """(gamma / sin gamma)^2 -> 1: at a tiny angular pitch the equiangular
    filter is the flat Ram-Lak filter with tau = alpha * SID."""
    rows = synth.random_array((3, 40), 5)
    alpha, sid = 1e-6, 750.0
    a = ora.equiangular_filter(rows, alpha, sid)
    b = ora.ramlak_filter(rows, alpha * sid)
    assert an.rel_l2(a, b) < 1e-9


def test_equiangular_taps_known_values(ora):
    """Impulse response: t(0) = 1/(4 alpha SID), zero at even lags, and at odd
    lags the ramp kernel 1/(n alpha)^2 stretched to 1/sin^2(n alpha)."""
    alpha, sid, nu = 0.02, 500.0, 41
    e = np.zeros((1, nu))
    e[0, nu // 2] = 1.0
    t = ora.equiangular_filter(e, alpha, sid)[0]
    lag = np.arange(nu) - nu // 2
    assert t[nu // 2] == pytest.approx(1.0 / (4 * alpha * sid), rel=1e-14)
    assert np.all(t[(lag % 2 == 0) & (lag != 0)] == 0.0)
    odd = lag % 2 != 0
    ref = -alpha / (math.pi ** 2 * sid * np.sin(lag[odd] * alpha) ** 2)
    np.testing.assert_allclose(t[odd], ref, rtol=1e-13)
    # and the same taps through the M-point response (circular route)
    M = ora.fft_size(nu)
    K = ora.equiangular_response(M, alpha, sid)
    np.testing.assert_allclose(ora.circular_filter(e, K)[0], t, rtol=0, atol=1e-12 * abs(t).max())


def test_fbp_of_disk(ora):
    spec = curved(128, n_proj=360)
    r = 0.3 * 256.0
    f = synth.rasterize_ellipses(synth.disk(r, rho=1.0), spec.vol_shape, spec.vol_spacing).numpy()
    x = ora.fbp(spec, ora.project(spec, f))
    ys, xs = synth.grid_axes(spec.vol_shape, spec.vol_spacing)
    rr = np.hypot(ys[:, None], xs[None, :])
    assert abs(x[rr < 0.8 * r].mean() - 1.0) < 1e-3
    assert abs(x[(rr > 1.2 * r) & (rr < 1.5 * r)].mean()) < 1e-3


def test_fbp_short_scan_offcentre_disk(ora):
    """Parker weights at the columns' fan angles: a short scan of pi + 2 delta
    reconstructs an off-centre disk (the (SID/L)^2 weight and the redundancy
    weights do not average out over a partial turn)."""
    spec = curved(128, n_proj=200, rng_=math.pi + 2 * 0.3)
    r, cx, cy = 0.12 * 256.0, 0.25 * 256.0, 0.075 * 256.0
    f = synth.rasterize_ellipses(synth.disk(r, centre=(cx, cy)), spec.vol_shape, spec.vol_spacing).numpy()
    x = ora.fbp(spec, ora.project(spec, f))
    ys, xs = synth.grid_axes(spec.vol_shape, spec.vol_spacing)
    inside = np.hypot(ys[:, None] - cy, xs[None, :] - cx) < 0.7 * r
    assert abs(x[inside].mean() - 1.0) < 1e-3


def test_fbp_reproduces_gaussian_blobs_like_flat(ora):
    """Smooth blobs: the curved and the flat detector both reproduce them,
    and agree with each other to the discretisation error."""
    spec_c, spec_f = curved(128, n_proj=360), flat(128, n_proj=360)
    g = synth.random_gaussians(4, 5, spec_c.vol_shape, spec_c.vol_spacing)
    f = synth.rasterize_gaussians(g, spec_c.vol_shape, spec_c.vol_spacing).numpy()
    xc = ora.fbp(spec_c, ora.project(spec_c, f))
    xf = ora.fbp(spec_f, ora.project(spec_f, f))
    assert an.rel_l2(xc, f) < 7e-3
    assert an.rel_l2(xc, xf) < 7e-3
