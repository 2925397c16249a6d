"""Degenerate and extreme cases on the GPU, against the oracle: a one-voxel
volume and one-pixel detector, a single view, a one-slice cone volume, views
at exact multiples of 45 degrees (the dominant-axis tie; flat and curved fan
detectors), odd detector sizes
(rays exactly along the grid axes through the centre row and column), and
the longest filter (M = 4096)."""
import math

import numpy as np
import pytest
import torch

import gpu_common as gc
import synth
from gpu_common import FP32_TOL, check, as_f32, rel_l2, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ph():
    gc.device()
    import paper_1904_13342_amd as ph
    return ph


def _all_ops(ph, ora, spec, seed):
    """A, B, A^T, B^T and FBP/FDK of the configuration against the oracle."""
    g = ph.from_spec(spec)
    if spec.kind == "cone3d":
        traj = ph.projection_matrices_3d(g)
        A, B, AT, BT = ph.project_cone3d, ph.backproject_cone3d, ph.project_adjoint_cone3d, \
            ph.backproject_adjoint_cone3d
        rec = lambda p: ph.fdk_cone3d(g, traj, p)
    else:
        traj = ph.ray_vectors_2d(g)
        fan = spec.kind in ("fan2d", "fan2d_curved")
        A = ph.project_fan2d if fan else ph.project_par2d
        B = ph.backproject_fan2d if fan else ph.backproject_par2d
        AT = ph.project_adjoint_fan2d if fan else ph.project_adjoint_par2d
        BT = ph.backproject_adjoint_fan2d if fan else ph.backproject_adjoint_par2d
        rec = lambda p: (ph.fbp_fan2d if fan else ph.fbp_par2d)(g, traj, p)
    proj_shape = (spec.n_proj,) + tuple(spec.det_shape)
    f = as_f32(0.5 + synth.random_array(spec.vol_shape, seed, dist="uniform"))
    p = as_f32(0.5 + synth.random_array(proj_shape, seed + 1, dist="uniform"))
    out = {
        "A": (A(g, traj, to_dev(f)), ora.project(spec, f)),
        "B": (B(g, traj, to_dev(p)), ora.backproject(spec, p)),
        "A^T": (AT(g, traj, to_dev(p)), ora.project_adjoint(spec, p)),
        "B^T": (BT(g, traj, to_dev(f)), ora.backproject_adjoint(spec, f)),
        "FBP": (rec(to_dev(p)), ora.fbp(spec, p)),
    }
    for name, (gpu, ref) in out.items():
        ref = np.asarray(ref).reshape(tuple(gpu.shape))
        if np.linalg.norm(ref) == 0.0:
            err = float(np.abs(to_np(gpu)).max())
            say(f"  {name}: reference is zero, max |gpu| {err:.2e}")
            assert err == 0.0
        else:
            check(to_np(gpu), ref, f"{name}")


CASES = {
    "cone_one_voxel_one_pixel": synth.config("cone3d_crop32").with_(vol_shape=(1, 1, 1), vol_spacing=(1.0, 1.0, 1.0),
                                                                     det_shape=(1, 1), det_spacing=(1.0, 1.0),
                                                                     n_proj=3, sid=100.0, sdd=150.0),
    "cone_single_view": synth.config("cone3d_crop32").with_(vol_shape=(9, 10, 11), det_shape=(13, 15), n_proj=1),
    "cone_one_slice": synth.config("cone3d_crop32").with_(vol_shape=(1, 24, 20), det_shape=(9, 41), n_proj=17),
    "cone_octant_views_odd_detector": synth.config("cone3d_crop32").with_(vol_shape=(17, 19, 21),
                                                                           det_shape=(21, 23), n_proj=8,
                                                                           angular_range=2 * math.pi),
    "par2d_one_pixel": synth.config("par2d_64").with_(vol_shape=(1, 1), det_shape=(1,), n_proj=4),
    "par2d_single_view_odd": synth.config("par2d_64").with_(vol_shape=(15, 17), det_shape=(25,), n_proj=1),
    "fan2d_octant_views": synth.config("fan2d_512").with_(vol_shape=(31, 33), vol_spacing=(1.0, 1.0),
                                                          det_shape=(61,), n_proj=8, sid=120.0, sdd=200.0),
    "fan2d_curved_octant_views": synth.config("fan2d_512").with_(kind="fan2d_curved", vol_shape=(31, 33),
                                                                 vol_spacing=(1.0, 1.0), det_shape=(61,), n_proj=8,
                                                                 sid=120.0, sdd=200.0),
    "fan2d_curved_one_pixel_one_bin": synth.config("fan2d_512").with_(kind="fan2d_curved", vol_shape=(1, 1),
                                                                      vol_spacing=(1.0, 1.0), det_shape=(1,),
                                                                      n_proj=3, sid=50.0, sdd=80.0),
}


@pytest.mark.parametrize("name", list(CASES))
def test_degenerate_geometries(ph, ora, name):
    say(f"[edge] {name}")
    _all_ops(ph, ora, CASES[name], seed=sum(map(ord, name)) % 1000)


def test_longest_filter(ph, ora):
    """2048-bin rows take the longest supported transform (M = 4096), both for
    the default Ram-Lak filter (linear convolution) and a learned response."""
    spec = synth.config("par2d_64").with_(vol_shape=(8, 8), det_shape=(2048,), det_spacing=(0.5,), n_proj=6)
    g = ph.from_spec(spec)
    p = as_f32(synth.random_array((spec.n_proj, 2048), 5))
    out = ph.weight_filter_2d(g, to_dev(p), fan=False)
    ref = ora.filter_projections(spec, ora.weight(spec, p)).reshape(spec.n_proj, 2048)
    check(to_np(out), ref, "[edge] Ram-Lak at M=4096")
    K = as_f32(ora.ramp_response(4096, ora.tau(spec)) + 0.01 * synth.random_array((4096,), 6))
    out = ph.weight_filter_2d(g, to_dev(p), fan=False, K=to_dev(K))
    ref = ora.filter_projections(spec, ora.weight(spec, p), K=K).reshape(spec.n_proj, 2048)
    check(to_np(out), ref, "[edge] learned K at M=4096")
