"""Trajectories given as general projection matrices (Sec. II.C.3: a
trajectory is a set of projection matrices, as calibrated on real scanners):
A, B, A^T, B^T and FDK on the GPU against the oracle's projection-matrix path
(pinned on the CPU against closed forms, dense transposes and the circular
operators), element by element.

The orbits are perturbed circular scans (tilted and wobbling orbit plane,
rolled detector, offset principal point, varying source and detector
distances, jittered angles, shifted rotation centre), so every matrix has z
terms in its u and w rows and the kernels take their per-voxel and per-ray
general paths.  The three cases cover a ragged grid with an off-centre volume
and a negative, non-unit matrix scale; tall detector pixels, which make the
back-projector's bricks 16 voxels deep; and magnification 10, where a brick's
footprint outgrows the LDS tile and the back-projector and its transpose read
and write the detector directly."""
import math

import numpy as np
import pytest

import gpu_common as gc
import synth
from gpu_common import as_f32, check, say, to_dev, to_np

pytestmark = pytest.mark.gpu

CASES = {
    "orbit_ragged": dict(
        spec=synth.config("cone3d_crop32").with_(vol_shape=(23, 29, 35), vol_spacing=(1.1, 0.9, 1.0),
                                                 det_shape=(37, 41), det_spacing=(1.7, 1.5), n_proj=17,
                                                 angular_range=200 * math.pi / 180, sid=300.0, sdd=500.0,
                                                 vol_origin=(-10.0, -14.0, -15.0)),
        seed=11, scale=-3.0, kw={}),
    # tall pixels: 16-voxel bricks, staged
    "orbit_nz16": dict(
        spec=synth.config("cone3d_crop32").with_(det_shape=(140, 72), det_spacing=(0.2, 0.4), n_proj=60),
        seed=12, scale=1.0, kw=dict(offset_px=(4.0, -6.0))),
    # magnification 10: footprints beyond the LDS tile
    "orbit_unstaged": dict(
        spec=synth.config("cone3d_crop32").with_(vol_shape=(40, 40, 40), vol_spacing=(1.0, 1.0, 1.0),
                                                 det_shape=(300, 640), det_spacing=(2.0, 1.6), n_proj=8,
                                                 sid=60.0, sdd=600.0),
        seed=13, scale=1.0, kw=dict(tilt_deg=5.0, sid_wobble=0.03, iso_shift_mm=1.0)),
}


@pytest.fixture(scope="module")
def ph():
    gc.device()
    import paper_1904_13342_amd as ph
    return ph


def _case(name):
    c = CASES[name]
    spec = c["spec"]
    P = synth.pose_matrices(spec, synth.perturbed_poses(spec, c["seed"], **c["kw"]))
    P32 = np.ascontiguousarray((P * c["scale"]).astype(np.float32))
    return spec, P32, P32.astype(np.float64)


@pytest.mark.parametrize("name", list(CASES))
def test_general_project_and_adjoint(ph, ora, name):
    spec, P32, P = _case(name)
    say(f"[general A, A^T] {name}")
    g = ph.from_spec(spec)
    f = gc.phantom(spec)
    p = ph.project_cone3d(g, P32, to_dev(f))
    ref = ora.project(spec, f, mats=P)
    check(to_np(p), ref, "A")
    q = as_f32(ref)
    check(to_np(ph.project_adjoint_cone3d(g, P32, to_dev(q))), ora.project_adjoint(spec, q, mats=P), "A^T")


@pytest.mark.parametrize("name", list(CASES))
def test_general_backproject_and_adjoint(ph, ora, name):
    spec, P32, P = _case(name)
    say(f"[general B, B^T, FDK] {name}")
    g = ph.from_spec(spec)
    f = gc.phantom(spec)
    p = as_f32(ora.project(spec, f, mats=P))
    check(to_np(ph.backproject_cone3d(g, P32, to_dev(p))), ora.backproject(spec, p, mats=P), "B")
    check(to_np(ph.backproject_adjoint_cone3d(g, P32, to_dev(f))), ora.backproject_adjoint(spec, f, mats=P), "B^T")
    check(to_np(ph.fdk_cone3d(g, P32, to_dev(p))), ora.fbp(spec, p, mats=P), "FDK")


def test_general_adjoint_identities(ph):
    """<A x, y> = <x, A^T y> and <B y, x> = <y, B^T x> on random data, FP64
    inner products of the FP32 results."""
    spec, P32, _ = _case("orbit_nz16")
    say("[general adjoint identities] orbit_nz16")
    g = ph.from_spec(spec)
    x = as_f32(synth.random_array(spec.vol_shape, 21))
    y = as_f32(synth.random_array((spec.n_proj,) + tuple(spec.det_shape), 22))
    xd, yd = to_dev(x), to_dev(y)
    Ax, Aty = to_np(ph.project_cone3d(g, P32, xd)), to_np(ph.project_adjoint_cone3d(g, P32, yd))
    By, Btx = to_np(ph.backproject_cone3d(g, P32, yd)), to_np(ph.backproject_adjoint_cone3d(g, P32, xd))
    for what, lhs, rhs in (("A", np.vdot(Ax, y), np.vdot(x, Aty)), ("B", np.vdot(By, x), np.vdot(y, Btx))):
        rel = abs(lhs - rhs) / abs(lhs)
        say(f"  {what}: {lhs:.9e} vs {rhs:.9e}, rel {rel:.1e}")
        assert rel < 1e-5, (what, rel)
