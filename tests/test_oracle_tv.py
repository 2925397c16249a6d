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
