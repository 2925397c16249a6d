"""Reduced-precision storage: volumes and projections stored as FP16 or BF16,
all arithmetic in FP32, geometry in FP32.

The oracle runs in FP64 on the dequantised half-precision input, so the
difference measures the kernel (FP32 arithmetic plus rounding of the output to
the storage type, rel-L2 about u/sqrt(3): 2.8e-4 for FP16, 2.3e-3 for BF16).
Bounds: 2e-3 for FP16; BF16's own rounding already exceeds that, so its bound
is 1e-2 and the value is printed.  The end-to-end error against FP64 on the
unquantised input is printed beside it."""
import math

import numpy as np
import pytest
import torch

import gpu_common as gc
import synth
from gpu_common import ELEM_TOL_HALF, as_f32, check, rel_l2, say, to_dev, to_np

pytestmark = pytest.mark.gpu

BOUND = {torch.float16: 2e-3, torch.bfloat16: 1e-2}
DTYPES = [torch.float16, torch.bfloat16]


def hcheck(out, ref, dtype, what):
    """rel-L2 within the storage type's bound and every element within two
    of its rounding steps of the largest value."""
    assert out.dtype == dtype, (what, out.dtype)
    return check(to_np(out), ref, what, tol=BOUND[dtype],
                 elem=ELEM_TOL_HALF["f16" if dtype == torch.float16 else "bf16"])


@pytest.fixture(scope="module")
def ph():
    gc.device()
    import paper_1904_13342_amd as ph
    return ph


def quantise(a, dtype):
    """Round to the storage type (round to nearest even) and back to float64."""
    return torch.as_tensor(np.asarray(a, dtype=np.float32)).to(dtype).to(torch.float64).numpy()


SPEC_3D = synth.config("cone3d_crop32").with_(vol_shape=(29, 33, 31), n_proj=40,
                                               angular_range=200 * math.pi / 180)
SPEC_2D = synth.config("fan2d_512").with_(vol_shape=(96, 80), vol_spacing=(1.0, 1.0), det_shape=(151,),
                                          det_spacing=(1.2,), n_proj=60, sid=200.0, sdd=320.0)


@pytest.mark.parametrize("dtype", DTYPES, ids=["f16", "bf16"])
def test_project_cone_half(ph, ora, dtype):
    spec = SPEC_3D
    f = gc.phantom(spec)
    fq = quantise(f, dtype)
    g = ph.from_spec(spec)
    out = ph.project_cone3d(g, ph.projection_matrices_3d(g), to_dev(fq, dtype))
    assert out.dtype == dtype
    hcheck(out, ora.project(spec, fq), dtype, f"[project_cone {dtype}] vs FP64 on stored input")
    say(f"  end to end {rel_l2(to_np(out), ora.project(spec, f)):.2e}")


@pytest.mark.parametrize("dtype", DTYPES, ids=["f16", "bf16"])
def test_project_cone_half_is_fp32_rounded_once(ph, dtype):
    """A half-precision volume is projected with FP32 arithmetic on its exact
    FP32 values, and each projection is rounded once to the storage type: bit
    for bit the FP32 projection of the widened volume, rounded to nearest
    even.  Checked at the 29 x 33 x 31 grid and at 128^3 with 64 views."""
    for spec in (SPEC_3D, synth.config("cone3d_256_short").with_(vol_shape=(128, 128, 128), n_proj=64)):
        g = ph.from_spec(spec)
        mats = ph.projection_matrices_3d(g)
        vh = torch.from_numpy(as_f32(synth.random_array(tuple(spec.vol_shape), 21, dist="uniform"))).to(dtype)
        vh = vh.to(gc.device()).contiguous()
        out = ph.project_cone3d(g, mats, vh)
        ref = ph.project_cone3d(g, mats, vh.float()).to(dtype)
        say(f"[project_cone {dtype}] {tuple(spec.vol_shape)}: {int((out != ref).sum())} of {out.numel()} differ")
        assert out.dtype == dtype and torch.equal(out, ref)


@pytest.mark.parametrize("dtype", DTYPES, ids=["f16", "bf16"])
def test_backproject_and_fdk_cone_half(ph, ora, dtype):
    spec = SPEC_3D
    p = as_f32(ora.project(spec, gc.phantom(spec)))
    pq = quantise(p, dtype)
    g = ph.from_spec(spec)
    mats = ph.projection_matrices_3d(g)
    q = as_f32(ora.filter_projections(spec, ora.weight(spec, p)))
    qq = quantise(q, dtype)
    out = ph.backproject_cone3d(g, mats, to_dev(qq, dtype))
    hcheck(out, ora.backproject(spec, qq), dtype, f"[backproject_cone {dtype}]")
    say(f"  end to end {rel_l2(to_np(out), ora.backproject(spec, q)):.2e}")
    rec = ph.fdk_cone3d(g, mats, to_dev(pq, dtype))
    hcheck(rec, ora.fbp(spec, pq), dtype, f"[fdk_cone {dtype}]")
    say(f"  end to end {rel_l2(to_np(rec), ora.fbp(spec, p)):.2e}")


@pytest.mark.parametrize("dtype", DTYPES, ids=["f16", "bf16"])
def test_fan2d_half(ph, ora, dtype):
    spec = SPEC_2D
    f = gc.phantom(spec)
    fq = quantise(f, dtype)
    g = ph.from_spec(spec)
    rv = ph.ray_vectors_2d(g)
    sino = ph.project_fan2d(g, rv, to_dev(fq, dtype))
    hcheck(sino, ora.project(spec, fq), dtype, f"[project_fan2d {dtype}]")
    sq = to_np(sino)
    rec = ph.fbp_fan2d(g, rv, sino)
    hcheck(rec, ora.fbp(spec, sq), dtype, f"[fbp_fan2d {dtype}]")
    say(f"  end to end {rel_l2(to_np(rec), ora.fbp(spec, ora.project(spec, f))):.2e}")


def test_half_rounding_is_nearest_even(ph):
    """Stored values equal torch's round-to-nearest-even conversion of the FP32
    result: back-project an exactly representable input whose FP32 output
    is known (a constant projection gives dbeta * sum_k (SID/w)^2 ...); here
    we check the simplest exact case, the parallel-beam back-projection of a
    constant sinogram, whose FP32 result is n_proj * dbeta * c."""
    spec = synth.config("par2d_64").with_(n_proj=8, det_shape=(200,))
    g = ph.from_spec(spec)
    rv = ph.ray_vectors_2d(g)
    for dtype in DTYPES:
        sino = torch.full((spec.n_proj, spec.det_shape[0]), 0.3, dtype=dtype, device=gc.device())
        img = ph.backproject_par2d(g, rv, sino)
        c32 = float(torch.tensor(0.3, dtype=dtype).float())
        dbeta = np.float32(spec.angular_range) / np.float32(spec.n_proj)
        acc = np.float32(0.0)
        for _ in range(spec.n_proj):
            acc = np.float32(acc + np.float32(c32))
        expect = torch.tensor(float(np.float32(dbeta) * acc), dtype=torch.float32).to(dtype)
        centre = img[32, 32]
        assert centre.item() == expect.item(), (dtype, centre.item(), expect.item())


@pytest.mark.parametrize("dtype", DTYPES, ids=["f16", "bf16"])
@pytest.mark.parametrize("kind", ["cone3d", "fan2d", "par2d"])
def test_adjoints_half(ph, ora, kind, dtype):
    """A^T and B^T with half-precision storage (FP32 accumulation; B^T through
    its workspace entry point) against the oracle's transposes on the stored
    input."""
    spec = {"cone3d": SPEC_3D, "fan2d": SPEC_2D, "par2d": synth.config("par2d_64")}[kind]
    g = ph.from_spec(spec)
    if kind == "cone3d":
        traj, aT, bT = ph.projection_matrices_3d(g), ph.project_adjoint_cone3d, ph.backproject_adjoint_cone3d
    else:
        traj = ph.ray_vectors_2d(g)
        aT = ph.project_adjoint_fan2d if kind == "fan2d" else ph.project_adjoint_par2d
        bT = ph.backproject_adjoint_fan2d if kind == "fan2d" else ph.backproject_adjoint_par2d
    f = gc.phantom(spec)
    p = as_f32(ora.project(spec, f))
    pq, fq = quantise(p, dtype), quantise(f, dtype)
    out = aT(g, traj, to_dev(pq, dtype))
    hcheck(out, ora.project_adjoint(spec, pq), dtype, f"[project_adjoint {kind} {dtype}]")
    out = bT(g, traj, to_dev(fq, dtype))
    hcheck(out, ora.backproject_adjoint(spec, fq), dtype, f"[backproject_adjoint {kind} {dtype}]")
