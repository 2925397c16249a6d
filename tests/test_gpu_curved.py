"""Parity of the HIP path on the curved (equiangular) fan detector with the
FP64 oracle: A, B, their exact transposes, the weighting/filter stage
(cos(gamma) weights, Parker at the bins' fan angles, the equiangular Ram-Lak
response) and FBP.  FP32 storage: rel-L2 below 1e-5; FP16 storage below 2e-3."""
import math

import numpy as np
import pytest
import torch

import gpu_common as gc
import synth
from gpu_common import FP32_TOL, check, as_f32, rel_l2, say, to_dev, to_np

pytestmark = pytest.mark.gpu

SPECS = {
    # the fan workload's sizes with equiangular bins of 1 mm arc length
    "curved_512": synth.config("fan2d_512").with_(kind="fan2d_curved"),
    # ragged grid, short scan (Parker), anisotropic pixels, off-centre origin
    "curved_ragged": synth.config("fan2d_512").with_(kind="fan2d_curved", vol_shape=(45, 31), vol_spacing=(1.0, 1.2),
                                                     det_shape=(77,), det_spacing=(1.1,), n_proj=11,
                                                     angular_range=250 * math.pi / 180, sid=100.0, sdd=160.0,
                                                     vol_origin=(-20.0, -16.0)),
    # a wide fan (about 100 degrees), where arc and flat bins differ most
    "curved_wide": synth.config("fan2d_512").with_(kind="fan2d_curved", vol_shape=(64, 64), vol_spacing=(2.0, 2.0),
                                                   det_shape=(181,), det_spacing=(2.0,), n_proj=24, sid=150.0,
                                                   sdd=210.0),
}


@pytest.fixture(scope="module")
def ph():
    gc.device()
    import paper_1904_13342_amd as ph
    return ph


def _setup(ph, name):
    spec = SPECS[name]
    g = ph.from_spec(spec)
    assert g.fan_detector == 1
    return spec, g, ph.ray_vectors_2d(g)


@pytest.mark.parametrize("name", list(SPECS))
def test_project(ph, ora, name):
    spec, g, rv = _setup(ph, name)
    say(f"[curved project] {name}")
    f = gc.phantom(spec)
    out = ph.project_fan2d(g, rv, to_dev(f))
    check(to_np(out), ora.project(spec, f), "")


@pytest.mark.parametrize("name", list(SPECS))
def test_backproject(ph, ora, name):
    spec, g, rv = _setup(ph, name)
    say(f"[curved backproject] {name}")
    f = gc.phantom(spec)
    q = as_f32(ora.filter_projections(spec, ora.weight(spec, ora.project(spec, f))).reshape(spec.n_proj, -1))
    out = ph.backproject_fan2d(g, rv, to_dev(q))
    check(to_np(out), ora.backproject(spec, q), "")


@pytest.mark.parametrize("name", list(SPECS))
def test_weight_filter(ph, ora, name):
    """Default weights and filter of the curved detector: W_red (1/2 or
    Parker at gamma_j) * cos(gamma_j), then the equiangular Ram-Lak."""
    spec, g, rv = _setup(ph, name)
    say(f"[curved weight_filter] {name}")
    p = as_f32(ora.project(spec, gc.phantom(spec)))
    out = ph.weight_filter_2d(g, to_dev(p), True)
    ref = ora.filter_projections(spec, ora.weight(spec, p)).reshape(spec.n_proj, -1)
    check(to_np(out), ref, "")


@pytest.mark.parametrize("name", list(SPECS))
def test_fbp(ph, ora, name):
    spec, g, rv = _setup(ph, name)
    say(f"[curved fbp] {name}")
    p = as_f32(ora.project(spec, gc.phantom(spec)))
    out = ph.fbp_fan2d(g, rv, to_dev(p))
    check(to_np(out), ora.fbp(spec, p), "")


@pytest.mark.parametrize("name", ["curved_ragged", "curved_wide"])
def test_transposes(ph, ora, name):
    spec, g, rv = _setup(ph, name)
    say(f"[curved transposes] {name}")
    # parity on the workload's data (as for the flat detector): the phantom
    # and its projections
    f = gc.phantom(spec)
    p = as_f32(ora.project(spec, f))
    check(to_np(ph.project_adjoint_fan2d(g, rv, to_dev(p))), ora.project_adjoint(spec, p), "A^T")
    check(to_np(ph.backproject_adjoint_fan2d(g, rv, to_dev(f))), ora.backproject_adjoint(spec, f), "B^T")
    # the GPU pairs are transposes of each other on signed noise (FP64 inner
    # products of the FP32 outputs)
    y = as_f32(synth.random_array((spec.n_proj, spec.det_shape[0]), 3))
    x = as_f32(synth.random_array(spec.vol_shape, 4))
    at = ph.project_adjoint_fan2d(g, rv, to_dev(y))
    bt = ph.backproject_adjoint_fan2d(g, rv, to_dev(x))
    ax = to_np(ph.project_fan2d(g, rv, to_dev(x)))
    lhs, rhs = np.vdot(ax, y), np.vdot(x, to_np(at))
    assert abs(lhs - rhs) <= 2e-6 * max(abs(lhs), abs(rhs))
    bx = to_np(ph.backproject_fan2d(g, rv, to_dev(y)))
    lhs, rhs = np.vdot(bx, x), np.vdot(y, to_np(bt))
    assert abs(lhs - rhs) <= 2e-6 * max(abs(lhs), abs(rhs))


def test_half_storage(ph, ora):
    spec, g, rv = _setup(ph, "curved_ragged")
    f = gc.phantom(spec)
    fh = torch.tensor(f, dtype=torch.float16)
    out = ph.project_fan2d(g, rv, fh.cuda())
    assert out.dtype == torch.float16
    check(to_np(out), ora.project(spec, fh.double().numpy()), "[curved f16 project]", tol=2e-3,
          elem=gc.ELEM_TOL_HALF["f16"])


def test_fbp_of_disk(ph, ora):
    """Uniform disk at the fan workload's sizes: density 1 inside, 0 outside."""
    spec, g, rv = _setup(ph, "curved_512")
    r = 60.0
    f = as_f32(synth.rasterize_ellipses(synth.disk(r, rho=1.0), spec.vol_shape, spec.vol_spacing, sub=4).numpy())
    p = ph.project_fan2d(g, rv, to_dev(f))
    x = to_np(ph.fbp_fan2d(g, rv, p))
    ys, xs = synth.grid_axes(spec.vol_shape, spec.vol_spacing)
    rr = np.hypot(ys[:, None], xs[None, :])
    inner, ring = x[rr < 0.8 * r].mean(), x[(rr > 1.2 * r) & (rr < 1.5 * r)].mean()
    say(f"[curved disk fbp] inside {inner:.5f} ring {ring:.2e}")
    assert abs(inner - 1.0) < 2e-3 and abs(ring) < 2e-3
