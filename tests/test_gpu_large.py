"""Element-wise parity at the full 512^3 size (360 views of 1024 x 768 at
0.8 mm) for the operators whose full-size check would otherwise be a sum: the
transposes A^T and B^T on inputs that are non-zero in a few views or slices
(the oracle's scatters skip zero rays and voxels, so it finishes in seconds
while the GPU runs the whole launch the benchmark times), and FP16 / BF16
storage of A, B and FDK on sampled views and slices.  Every element is
compared."""
import math

import numpy as np
import pytest
import torch

import gpu_common as gc
import synth
from gpu_common import ELEM_TOL_HALF, as_f32, check, say, to_dev, to_np

pytestmark = pytest.mark.gpu

SPEC = synth.config("cone3d_512")


@pytest.fixture(scope="module")
def ph():
    gc.device()
    import paper_1904_13342_amd as ph
    return ph


@pytest.fixture(scope="module")
def coarse(ora):
    """Projections of the workload's phantom with the structure of real data
    (oracle projections at 1/8 resolution, upsampled)."""
    return gc.coarse_projections(ora, SPEC, 8)


def _phantom_dev():
    prm = synth.random_ellipsoids(0, SPEC.n_figures, SPEC.vol_shape, SPEC.vol_spacing)
    return synth.rasterize_ellipsoids(prm, SPEC.vol_shape, SPEC.vol_spacing, sub=1, device=gc.device(),
                                      dtype=torch.float32)


def test_project_adjoint_512_nine_views(ph, ora, coarse):
    """Projections non-zero in nine views.  The sample positions are FP32
    index coordinates up to ~516 (ulp 3e-5 to 6e-5 voxel) reached in up to
    ~700 steps, so each sample sits within ~1e-5 to 6e-5 voxel of the oracle's
    FP64 position; A^T's weights move by as much (the hat's slope is 1), and
    with three views the rel-L2 comes to 1.1e-5.  Nine views average those
    position errors to about 6e-6."""
    views = [10, 50, 100, 140, 190, 230, 251, 300, 340]
    say(f"[A^T 512^3] projections non-zero in views {views}; every voxel compared")
    p = np.zeros_like(coarse)
    p[views] = coarse[views]
    g = ph.from_spec(SPEC)
    out = to_np(ph.project_adjoint_cone3d(g, ph.projection_matrices_3d(g), to_dev(p)))
    check(out, ora.project_adjoint(SPEC, p), "A^T")


def test_backproject_adjoint_512_three_slices(ph, ora):
    slices = [40, 256, 471]
    say(f"[B^T 512^3] volume non-zero in slices {slices}; every pixel of every view compared")
    f = _phantom_dev()
    keep = torch.zeros(SPEC.vol_shape[0], dtype=torch.bool, device=f.device)
    keep[slices] = True
    f[~keep] = 0.0
    g = ph.from_spec(SPEC)
    out = to_np(ph.backproject_adjoint_cone3d(g, ph.projection_matrices_3d(g), f))
    fh = to_np(f)
    del f
    check(out, ora.backproject_adjoint(SPEC, fh), "B^T")


def _quantise(a, dtype):
    return torch.as_tensor(np.asarray(a, dtype=np.float32)).to(dtype).to(torch.float64).numpy()


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16], ids=["f16", "bf16"])
def test_half_storage_512(ph, ora, coarse, dtype):
    tag = "f16" if dtype == torch.float16 else "bf16"
    tol, elem = (2e-3 if dtype == torch.float16 else 1e-2), ELEM_TOL_HALF[tag]
    views, slices, fdk_slices = [0, 45, 135], [3, 256, 500], [230, 256, 281]
    say(f"[{tag} 512^3] A on views {views}, B on slices {slices}, FDK on slices {fdk_slices}")
    g = ph.from_spec(SPEC)
    mats = ph.projection_matrices_3d(g)
    f = _phantom_dev().to(dtype)
    out = ph.project_cone3d(g, mats, f)
    assert out.dtype == dtype
    fq = to_np(f)
    del f
    check(to_np(out[views]), ora.project(SPEC, fq, views=views)[views], f"A {tag}", tol=tol, elem=elem)
    del out, fq
    pq = _quantise(coarse, dtype)
    pd = to_dev(pq, dtype)
    vol = ph.backproject_cone3d(g, mats, pd)
    assert vol.dtype == dtype
    check(to_np(vol[slices]), ora.backproject(SPEC, pq, slices=slices)[slices], f"B {tag}", tol=tol, elem=elem)
    del vol
    # FDK on the slices: weighting and filtering of the detector rows they need
    # (the oracle's direct convolution), then B on those slices
    zs = synth.grid_axes(SPEC.vol_shape, SPEC.vol_spacing)[0][fdk_slices]
    R = 0.5 * math.hypot(SPEC.vol_shape[1] * SPEC.vol_spacing[1], SPEC.vol_shape[2] * SPEC.vol_spacing[2])
    nv, dv = SPEC.det_shape[0], SPEC.det_spacing[0]
    rows = set()
    for z in zs:
        vs = [SPEC.sdd * z / w / dv + (nv - 1) / 2 for w in (SPEC.sid - R, SPEC.sid + R)]
        rows.update(range(max(0, int(math.floor(min(vs))) - 3), min(nv, int(math.ceil(max(vs))) + 4)))
    rows = sorted(rows)
    q = np.zeros_like(pq)
    q[:, rows, :] = ora.ramlak_filter(ora.weight(SPEC, pq)[:, rows, :], ora.tau(SPEC))
    rec = ph.fdk_cone3d(g, mats, pd)
    assert rec.dtype == dtype
    check(to_np(rec[fdk_slices]), ora.backproject(SPEC, q, slices=fdk_slices)[fdk_slices], f"FDK {tag}", tol=tol,
          elem=elem)
