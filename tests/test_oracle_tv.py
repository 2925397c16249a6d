"""Pins of the oracle's total variation (the regulariser of the iterative
reconstruction, Sec. III.B.1 / Eq. 7): closed forms (a constant image, a
linear ramp, a single step edge), invariance under flips, and the gradient
against central finite differences of the value."""
import math

import numpy as np
import pytest


def test_constant_image(ora):
    x = np.full((7, 9), 3.25)
    assert ora.tv(x, 0.1) == pytest.approx(63 * 0.1, rel=1e-14)
    assert np.abs(ora.tv_grad(x, 0.1)).max() == 0.0


def test_linear_ramp_2d(ora):
    # x = a*i + b*j: interior pixels have |grad| = sqrt(a^2 + b^2); the last
    # row (no i difference) has |b|, the last column |a|, the corner 0
    a, b, eps = 0.3, -0.7, 1e-3
    ny, nx = 6, 8
    i, j = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    x = a * i + b * j
    expect = ((ny - 1) * (nx - 1) * math.sqrt(a * a + b * b + eps * eps) + (nx - 1) * math.sqrt(b * b + eps * eps)
              + (ny - 1) * math.sqrt(a * a + eps * eps) + eps)
    assert ora.tv(x, eps) == pytest.approx(expect, rel=1e-13)


def test_step_edge_3d(ora):
    # a unit step across x in a [nz, ny, nx] volume: every voxel left of the
    # edge has one x difference of 1; all others are flat
    eps = 1e-2
    x = np.zeros((3, 4, 5))
    x[:, :, 3:] = 1.0
    n_edge = 3 * 4
    expect = n_edge * math.sqrt(1 + eps * eps) + (x.size - n_edge) * eps
    assert ora.tv(x, eps) == pytest.approx(expect, rel=1e-13)


def test_flip_invariance(ora):
    rng = np.random.default_rng(1)
    x = rng.standard_normal((5, 6, 7))
    v = ora.tv(x, 0.05)
    # reversing an axis turns forward into backward differences, which
    # changes which voxel carries each difference: the values differ; but a
    # transpose of two axes keeps the summands
    assert ora.tv(np.swapaxes(x, 1, 2).copy(), 0.05) == pytest.approx(v, rel=1e-13)
    assert ora.tv(np.swapaxes(x, 0, 2).copy(), 0.05) == pytest.approx(v, rel=1e-13)


@pytest.mark.parametrize("shape", [(9, 11), (4, 5, 6), (1, 7, 3)])
def test_gradient_finite_differences(ora, shape):
    rng = np.random.default_rng(2)
    x = rng.standard_normal(shape)
    eps = 0.1
    g = ora.tv_grad(x, eps)
    for _ in range(3):
        d = rng.standard_normal(shape)
        h = 1e-5
        fd = (ora.tv(x + h * d, eps) - ora.tv(x - h * d, eps)) / (2 * h)
        assert fd == pytest.approx(float((g * d).sum()), rel=1e-7, abs=1e-9)
    # single coordinates, including border voxels
    for idx in [(0,) * len(shape), tuple(n - 1 for n in shape), tuple(n // 2 for n in shape)]:
        e = np.zeros(shape)
        e[idx] = 1.0
        h = 1e-6
        fd = (ora.tv(x + h * e, eps) - ora.tv(x - h * e, eps)) / (2 * h)
        assert fd == pytest.approx(g[idx], rel=1e-6, abs=1e-8)


# ---------------------------------------------------------- anisotropic TV
# The sum of absolute forward differences per axis (the total variation of
# the framework Sec. III.B.1 takes TV from), smoothed per difference by eps.

def test_aniso_constant_image(ora):
    x = np.full((4, 7, 9), -1.5)
    # every voxel has 3 differences of 0, each contributing eps
    assert ora.tv(x, 0.1, anisotropic=True) == pytest.approx(3 * x.size * 0.1, rel=1e-14)
    assert ora.tv(x, 0.0, anisotropic=True) == 0.0
    assert np.abs(ora.tv_grad(x, 0.1, anisotropic=True)).max() == 0.0
    assert np.abs(ora.tv_grad(x, 0.0, anisotropic=True)).max() == 0.0


def test_aniso_linear_ramp_2d(ora):
    # x = a*i + b*j: (ny-1)*nx differences of a along i, ny*(nx-1) of b along j
    a, b = 0.3, -0.7
    ny, nx = 6, 8
    i, j = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    x = a * i + b * j
    assert ora.tv(x, 0.0, anisotropic=True) == pytest.approx((ny - 1) * nx * abs(a) + ny * (nx - 1) * abs(b),
                                                               rel=1e-13)
    eps = 0.2
    expect = ((ny - 1) * nx * math.sqrt(a * a + eps * eps) + ny * (nx - 1) * math.sqrt(b * b + eps * eps)
              + (nx + ny) * eps)
    assert ora.tv(x, eps, anisotropic=True) == pytest.approx(expect, rel=1e-13)
    # the ramp's gradient: interior voxels see equal differences on both
    # sides and get 0; the first row loses sign(a), the last gains it
    g = ora.tv_grad(x, 0.0, anisotropic=True)
    assert g[2, 3] == 0.0
    assert g[0, 3] == pytest.approx(-np.sign(a)) and g[ny - 1, 3] == pytest.approx(np.sign(a))
    assert g[3, 0] == pytest.approx(-np.sign(b)) and g[3, nx - 1] == pytest.approx(np.sign(b))


def test_aniso_equals_isotropic_for_one_axis_images(ora):
    # an image varying along one axis only has one non-zero difference per
    # voxel, so the two readings differ only by eps for each of the other
    # (zero) differences, and their gradients agree
    rng = np.random.default_rng(3)
    for shape, ax in (((5, 6, 7), 1), ((9, 11), 0)):
        prof = rng.standard_normal(shape[ax])
        x = np.broadcast_to(np.expand_dims(prof, tuple(a for a in range(len(shape)) if a != ax)), shape).copy()
        assert ora.tv(x, 0.0, anisotropic=True) == pytest.approx(ora.tv(x, 0.0), rel=1e-13)
        eps = 1e-3
        assert ora.tv(x, eps, anisotropic=True) == pytest.approx(ora.tv(x, eps) + (len(shape) - 1) * x.size * eps,
                                                                 rel=1e-13)
        assert np.allclose(ora.tv_grad(x, eps, anisotropic=True), ora.tv_grad(x, eps), rtol=1e-13, atol=1e-13)


def test_aniso_axes_of_extent_one_add_nothing(ora):
    rng = np.random.default_rng(6)
    x = rng.standard_normal((7, 5))
    for eps in (0.0, 0.1):
        v = ora.tv(x, eps, anisotropic=True)
        assert ora.tv(x[None], eps, anisotropic=True) == pytest.approx(v, rel=1e-14)
        assert ora.tv(x[:, None, :], eps, anisotropic=True) == pytest.approx(v, rel=1e-14)


def test_aniso_homogeneous_and_translation_invariant(ora):
    rng = np.random.default_rng(4)
    x = rng.standard_normal((5, 6, 7))
    v = ora.tv(x, 0.0, anisotropic=True)
    assert ora.tv(-2.5 * x, 0.0, anisotropic=True) == pytest.approx(2.5 * v, rel=1e-13)
    assert ora.tv(x + 3.0, 0.0, anisotropic=True) == pytest.approx(v, rel=1e-12)
    # the anisotropic sum bounds the isotropic one: |D|_2 <= |D|_1 <= sqrt(3) |D|_2
    iso = ora.tv(x, 0.0)
    assert iso <= v <= math.sqrt(3) * iso


@pytest.mark.parametrize("shape,eps", [((9, 11), 0.1), ((4, 5, 6), 0.05), ((4, 5, 6), 0.0)])
def test_aniso_gradient_finite_differences(ora, shape, eps):
    # at eps = 0 the value is piecewise linear; random data has no zero
    # differences, so it is differentiable there and the differences are exact
    rng = np.random.default_rng(5)
    x = rng.standard_normal(shape)
    g = ora.tv_grad(x, eps, anisotropic=True)
    for _ in range(3):
        d = rng.standard_normal(shape)
        h = 1e-6
        fd = (ora.tv(x + h * d, eps, anisotropic=True) - ora.tv(x - h * d, eps, anisotropic=True)) / (2 * h)
        assert fd == pytest.approx(float((g * d).sum()), rel=1e-6, abs=1e-8)
