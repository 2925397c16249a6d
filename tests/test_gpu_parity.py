"""Parity of the HIP kernels with the FP64 oracle, element by element, on the
seeded phantoms of the workloads.  FP32 storage: rel-L2 below 1e-5.

Small cases are compared in full (several tiles plus ragged tails); the
large configurations (256^3 and 512^3) are compared on sampled views, slices
and rows that the oracle computes one by one, in the launch configuration the
benchmark times."""
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


# ------------------------------------------------------------------ 2D cases

SPECS_2D = {
    "par2d_64": synth.config("par2d_64"),
    "par2d_ragged": synth.config("par2d_64").with_(vol_shape=(37, 53), vol_spacing=(0.9, 1.1), det_shape=(61,),
                                                   det_spacing=(1.3,), n_proj=7, vol_origin=(-15.0, -30.0)),
    "fan2d_512": synth.config("fan2d_512"),
    "fan2d_ragged": synth.config("fan2d_512").with_(vol_shape=(45, 31), vol_spacing=(1.0, 1.2), det_shape=(77,),
                                                    det_spacing=(1.1,), n_proj=11, angular_range=250 * math.pi / 180,
                                                    sid=100.0, sdd=160.0),
}


def _fns(ph, spec):
    if spec.kind == "par2d":
        return ph.project_par2d, ph.backproject_par2d, ph.fbp_par2d, False
    return ph.project_fan2d, ph.backproject_fan2d, ph.fbp_fan2d, True


@pytest.mark.parametrize("name", list(SPECS_2D))
def test_project_2d(ph, ora, name):
    spec = SPECS_2D[name]
    say(f"[project_2d] {name}")
    f = gc.phantom(spec)
    g = ph.from_spec(spec)
    fp, _, _, _ = _fns(ph, spec)
    out = fp(g, ph.ray_vectors_2d(g), to_dev(f))
    check(to_np(out), ora.project(spec, f), "")


@pytest.mark.parametrize("name", list(SPECS_2D))
def test_backproject_2d(ph, ora, name):
    spec = SPECS_2D[name]
    say(f"[backproject_2d] {name}")
    f = gc.phantom(spec)
    q = as_f32(ora.filter_projections(spec, ora.weight(spec, ora.project(spec, f))).reshape(spec.n_proj, -1))
    g = ph.from_spec(spec)
    _, bp, _, _ = _fns(ph, spec)
    out = bp(g, ph.ray_vectors_2d(g), to_dev(q))
    check(to_np(out), ora.backproject(spec, q), "")


@pytest.mark.parametrize("name", list(SPECS_2D))
def test_fbp_2d(ph, ora, name):
    spec = SPECS_2D[name]
    say(f"[fbp_2d] {name}")
    p = as_f32(ora.project(spec, gc.phantom(spec)))
    g = ph.from_spec(spec)
    _, _, fbp, _ = _fns(ph, spec)
    out = fbp(g, ph.ray_vectors_2d(g), to_dev(p))
    check(to_np(out), ora.fbp(spec, p), "")


@pytest.mark.parametrize("name", ["par2d_64", "fan2d_ragged"])
def test_weight_filter_2d_ramlak_and_learned(ph, ora, name):
    spec = SPECS_2D[name]
    say(f"[weight_filter_2d] {name}")
    p = as_f32(ora.project(spec, gc.phantom(spec)))
    g = ph.from_spec(spec)
    fan = spec.kind == "fan2d"
    out = ph.weight_filter_2d(g, to_dev(p), fan)
    ref = ora.filter_projections(spec, ora.weight(spec, p)).reshape(p.shape)
    check(to_np(out), ref, "Ram-Lak")
    # an arbitrary response K on a grid too short for a linear convolution wraps around
    M = 128 if spec.det_shape[0] <= 128 else 1024
    K = as_f32(np.abs(synth.random_array((M,), 3)) / spec.det_spacing[0])
    W_red = as_f32(synth.random_array((spec.n_proj, spec.det_shape[0]), 4, dist="uniform"))
    out = ph.weight_filter_2d(g, to_dev(p), fan, K=to_dev(K), W_red=to_dev(W_red))
    ref = ora.filter_projections(spec, ora.weight(spec, p, W_red=W_red), K=K).reshape(p.shape)
    check(to_np(out), ref, "learned-K")


def test_batch_2d(ph, ora):
    spec = SPECS_2D["fan2d_ragged"]
    f = np.stack([gc.phantom(spec, seed=s) for s in (0, 1, 2)])
    g = ph.from_spec(spec)
    rv = ph.ray_vectors_2d(g)
    out = to_np(ph.project_fan2d(g, rv, to_dev(f)))
    for b in range(3):
        check(out[b], ora.project(spec, f[b]))
    x = to_np(ph.fbp_fan2d(g, rv, to_dev(as_f32(out))))
    for b in range(3):
        check(x[b], ora.fbp(spec, as_f32(out[b])))


# ------------------------------------------------------------- small 3D cases

SPECS_3D = {
    "crop32": synth.config("cone3d_crop32"),
    "ragged": synth.config("cone3d_crop32").with_(vol_shape=(23, 29, 35), vol_spacing=(1.1, 0.9, 1.0),
                                                  det_shape=(37, 41), det_spacing=(1.7, 1.5), n_proj=17,
                                                  angular_range=200 * math.pi / 180, sid=300.0, sdd=500.0,
                                                  vol_origin=(-10.0, -14.0, -15.0)),
    "short64": synth.config("cone3d_256_short").with_(vol_shape=(64, 64, 64), vol_spacing=(4.0, 4.0, 4.0),
                                                      det_shape=(120, 155), det_spacing=(4.0, 4.0), n_proj=62),
    # tall pixels: a 32-voxel column's footprint outgrows the back-projector's
    # LDS tile, so the bricks are 16 voxels deep, staged
    "tall_pixels": synth.config("cone3d_crop32").with_(det_shape=(140, 72), det_spacing=(0.2, 0.4), n_proj=90),
}


@pytest.mark.parametrize("name", list(SPECS_3D))
def test_project_cone_small(ph, ora, name):
    spec = SPECS_3D[name]
    say(f"[project_cone] {name}")
    f = gc.phantom(spec)
    g = ph.from_spec(spec)
    out = ph.project_cone3d(g, ph.projection_matrices_3d(g), to_dev(f))
    check(to_np(out), ora.project(spec, f), "")


@pytest.mark.parametrize("name", list(SPECS_3D))
def test_backproject_cone_small(ph, ora, name):
    spec = SPECS_3D[name]
    say(f"[backproject_cone] {name}")
    f = gc.phantom(spec)
    q = as_f32(ora.filter_projections(spec, ora.weight(spec, ora.project(spec, f))))
    g = ph.from_spec(spec)
    out = ph.backproject_cone3d(g, ph.projection_matrices_3d(g), to_dev(q))
    check(to_np(out), ora.backproject(spec, q), "")


@pytest.mark.parametrize("name", list(SPECS_3D))
def test_fdk_cone_small(ph, ora, name):
    spec = SPECS_3D[name]
    say(f"[fdk_cone] {name}")
    p = as_f32(ora.project(spec, gc.phantom(spec)))
    g = ph.from_spec(spec)
    out = ph.fdk_cone3d(g, ph.projection_matrices_3d(g), to_dev(p))
    check(to_np(out), ora.fbp(spec, p), "")


def test_weight_filter_3d_learned(ph, ora):
    spec = SPECS_3D["ragged"]
    say("[weight_filter_3d] ragged, learned K and W")
    p = as_f32(ora.project(spec, gc.phantom(spec)))
    g = ph.from_spec(spec)
    M = 64
    K = as_f32(np.abs(synth.random_array((M,), 5)))
    W = as_f32(synth.random_array(spec.det_shape, 6, dist="uniform", low=0.5, high=1.5))
    out = ph.weight_filter_3d(g, to_dev(p), K=to_dev(K), W=to_dev(W))
    ref = ora.filter_projections(spec, ora.weight(spec, p, W=W), K=K)
    check(to_np(out), ref, "")


def test_backproject_cone_unstaged_footprint(ph, ora):
    """Magnification 10: a brick's footprint exceeds the LDS tile and the
    kernel reads the detector from global memory."""
    spec = synth.config("cone3d_crop32").with_(vol_shape=(40, 40, 40), vol_spacing=(1.0, 1.0, 1.0),
                                               det_shape=(300, 640), det_spacing=(2.0, 1.6), n_proj=8,
                                               sid=60.0, sdd=600.0)
    say("[backproject_cone] unstaged footprint")
    f = gc.phantom(spec)
    q = as_f32(ora.project(spec, f))
    g = ph.from_spec(spec)
    out = ph.backproject_cone3d(g, ph.projection_matrices_3d(g), to_dev(q))
    check(to_np(out), ora.backproject(spec, q), "")


def test_cone_general_matrices(ph, ora):
    """A quarter turn of the world about x makes the matrices non-axial (u and
    w depend on z) and maps the cubic grid onto itself: back-projecting with
    P o R equals back-projecting with P and permuting the volume axes;
    projecting the permuted volume with P o R equals projecting with P."""
    spec = synth.config("cone3d_crop32").with_(vol_shape=(24, 24, 24), vol_spacing=(1.0, 1.0, 1.0),
                                               det_shape=(40, 44), det_spacing=(1.0, 1.0), n_proj=9,
                                               sid=120.0, sdd=200.0)
    say("[cone] general matrices")
    g = ph.from_spec(spec)
    P = ph.projection_matrices_3d(g).astype(np.float64)
    # world point X' = R X with R: (x, y, z) -> (x, -z, y)
    R = np.array([[1, 0, 0, 0], [0, 0, -1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.float64)
    Pr = np.ascontiguousarray((P @ R).astype(np.float32))
    f = gc.phantom(spec)
    q = as_f32(ora.project(spec, f))
    vol = to_np(ph.backproject_cone3d(g, Pr, to_dev(q)))
    # voxel [iz, iy, ix] at world (x, y, z) is seen at (x, -z, y), i.e. at
    # voxel [iy, n-1-iz, ix] of the unrotated grid
    ref = ora.backproject(spec, q)
    expect = np.ascontiguousarray(np.transpose(ref[:, ::-1, :], (1, 0, 2)))
    check(vol, expect, "back-projection")
    # forward: the volume seen through P o R is f permuted the same way
    fr = np.ascontiguousarray(np.transpose(f[:, ::-1, :], (1, 0, 2)))
    p = to_np(ph.project_cone3d(g, Pr, to_dev(fr)))
    check(p, ora.project(spec, f), "projection")


def test_batch_3d(ph, ora):
    spec = SPECS_3D["ragged"]
    f = np.stack([gc.phantom(spec, seed=s) for s in (0, 1)])
    g = ph.from_spec(spec)
    mats = ph.projection_matrices_3d(g)
    p = to_np(ph.project_cone3d(g, mats, to_dev(f)))
    x = to_np(ph.fdk_cone3d(g, mats, to_dev(as_f32(p))))
    for b in range(2):
        check(p[b], ora.project(spec, f[b]))
        check(x[b], ora.fbp(spec, as_f32(p[b])))


# --------------------------------------------------------- full-size configs

LARGE = {
    "cone3d_256_short": dict(views=[0, 61, 123, 247], slices=[0, 77, 128, 255], fdk_slices=[101, 128, 150],
                             coarse=4, fp_views=4),
    # views 45 and 225 sit in the band near 45 degrees where neighbouring
    # detector tiles walk different slab axes; 90 walks y; 314 is ragged
    "cone3d_512": dict(views=[0, 45, 90, 135, 225, 314], slices=[3, 256, 500], fdk_slices=[230, 256, 281],
                       coarse=8, fp_views=6),
}


def _large_phantom(spec):
    prm = synth.random_ellipsoids(0, spec.n_figures, spec.vol_shape, spec.vol_spacing)
    f = synth.rasterize_ellipsoids(prm, spec.vol_shape, spec.vol_spacing, sub=1, device=gc.device(),
                                   dtype=torch.float32)
    return f


def _row_band(spec, slices, margin=3):
    """Detector rows that the given z slices project onto in any view: row
    coordinate SDD z / w over the depths w in SID -+ (half-diagonal of the
    xy extent)."""
    zs = synth.grid_axes(spec.vol_shape, spec.vol_spacing)[0][slices]
    R = 0.5 * math.hypot(spec.vol_shape[1] * spec.vol_spacing[1], spec.vol_shape[2] * spec.vol_spacing[2])
    nv, dv = spec.det_shape[0], spec.det_spacing[0]
    rows = set()
    for z in zs:
        vs = [spec.sdd * z / w / dv + (nv - 1) / 2 for w in (spec.sid - R, spec.sid + R)]
        lo, hi = int(math.floor(min(vs))) - margin, int(math.ceil(max(vs))) + margin
        rows.update(range(max(0, lo), min(nv, hi + 1)))
    return sorted(rows)


@pytest.mark.parametrize("name", list(LARGE))
def test_project_cone_large(ph, ora, name):
    spec, cfg = synth.config(name), LARGE[name]
    say(f"[project_cone] {name} full size, oracle on views {cfg['views'][:cfg['fp_views']]}")
    f = _large_phantom(spec)
    g = ph.from_spec(spec)
    out = ph.project_cone3d(g, ph.projection_matrices_3d(g), f)
    torch.cuda.synchronize()
    views = cfg["views"][:cfg["fp_views"]]
    ref = ora.project(spec, to_np(f), views=views)
    check(to_np(out[views]), ref[views], "")


@pytest.mark.parametrize("name", list(LARGE))
def test_backproject_and_fdk_cone_large(ph, ora, name):
    spec, cfg = synth.config(name), LARGE[name]
    say(f"[backproject/fdk_cone] {name} full size, oracle on slices {cfg['slices']}")
    p = gc.coarse_projections(ora, spec, cfg["coarse"])
    g = ph.from_spec(spec)
    mats = ph.projection_matrices_3d(g)
    pd = to_dev(p)
    sl = cfg["slices"]
    # back-projection of the projections as they are
    vol = ph.backproject_cone3d(g, mats, pd)
    torch.cuda.synchronize()
    check(to_np(vol[sl]), ora.backproject(spec, p, slices=sl)[sl], "back-projection")
    del vol
    # weighting + filtering on the rows some slices need, then FDK on those slices
    sl = cfg["fdk_slices"]
    rows = _row_band(spec, sl)
    pw = ora.weight(spec, p)
    qrows = ora.ramlak_filter(pw[:, rows, :], ora.tau(spec))
    q_gpu = to_np(ph.weight_filter_3d(g, pd)[:, rows, :])
    check(q_gpu, qrows, f"weight+filter on {len(rows)} rows/view")
    q = np.zeros_like(p)
    q[:, rows, :] = qrows
    x = to_np(ph.fdk_cone3d(g, mats, pd)[sl])
    check(x, ora.backproject(spec, q, slices=sl)[sl], "FDK")
