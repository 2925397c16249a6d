"""Helpers shared by the GPU parity tests: device handles, seeded inputs
(from ``synth`` and the oracle only, never from the HIP path) and error
measures."""
import sys

import numpy as np
import pytest
import torch

import synth

FP32_TOL = 1e-5   # rel-L2 bound of FP32 kernels against the FP64 oracle
# Bound on every single element, as a fraction of the largest reference
# magnitude: FP32 sample positions carry ~3e-5 voxel of rounding (coordinates
# up to a few hundred), which moves a sample across a unit jump of the
# phantom by at most that much, so one element of a line integral or a
# back-projected sum may differ by a few 1e-5 of the largest value; 1e-4
# leaves a factor of three.  A seam error (a tile, slab or brick edge handled
# wrongly) shows up here even where the rel-L2 over a large array hides it.
ELEM_TOL = 1e-4
# Storage rounding of one element (nearest even): 2^-11 (FP16) and 2^-8
# (BF16) of the element, doubled.
ELEM_TOL_HALF = {"f16": 2.0 ** -10, "bf16": 2.0 ** -7}


def device():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    return torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(x, ref):
    x = np.asarray(x, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


def max_rel(x, ref):
    """max |x - ref| / max |ref| over all elements."""
    x = np.asarray(x, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    return float(np.abs(x - ref).max() / np.abs(ref).max())


def check(x, ref, what="", tol=FP32_TOL, elem=ELEM_TOL):
    """Assert rel-L2(x, ref) < tol and every element within elem * max|ref|;
    prints both figures."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert x.shape == ref.shape, (what, x.shape, ref.shape)
    assert np.abs(ref).max() > 0, what
    assert np.all(np.isfinite(x)), what
    err, mx = rel_l2(x, ref), max_rel(x, ref)
    say(f"  {what} rel-L2 {err:.2e}, max elem {mx:.2e}")
    assert err < tol, (what, err, tol)
    assert mx <= elem, (what, mx, elem)
    return err


def to_dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=device(), dtype=dtype).contiguous()


def to_np(t):
    return t.detach().to(torch.float64).cpu().numpy()


def as_f32(a):
    """Round to FP32 and back: the exact values both sides receive."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def phantom(spec, seed=0, sub=None):
    """The configuration's seeded phantom, rounded to FP32."""
    if spec.ndim == 2:
        prm = synth.random_ellipses(seed, spec.n_figures, spec.vol_shape, spec.vol_spacing)
        f = synth.rasterize_ellipses(prm, spec.vol_shape, spec.vol_spacing, sub=sub or 4)
    else:
        prm = synth.random_ellipsoids(seed, spec.n_figures, spec.vol_shape, spec.vol_spacing)
        f = synth.rasterize_ellipsoids(prm, spec.vol_shape, spec.vol_spacing, sub=sub or 2)
    return as_f32(f.numpy())


def coarse_projections(ora, spec, factor, seed=0):
    """Projections of the configuration's phantom with the structure of real
    data at a fraction of the oracle's cost: the oracle projects a phantom
    rasterised ``factor`` times coarser onto a detector ``factor`` times
    coarser, and the result is bilinearly upsampled to the full detector.
    Returns FP32-rounded float64 [n_proj, (nv,) nu]."""
    cs = spec.with_(vol_shape=tuple(max(1, n // factor) for n in spec.vol_shape),
                    vol_spacing=tuple(s * factor for s in spec.vol_spacing),
                    det_shape=tuple(max(2, n // factor) for n in spec.det_shape),
                    det_spacing=tuple(d * factor for d in spec.det_spacing), step_mm=0.0)
    prm = (synth.random_ellipsoids(seed, spec.n_figures, spec.vol_shape, spec.vol_spacing) if spec.ndim == 3 else
           synth.random_ellipses(seed, spec.n_figures, spec.vol_shape, spec.vol_spacing))
    f = (synth.rasterize_ellipsoids(prm, cs.vol_shape, cs.vol_spacing, sub=2) if spec.ndim == 3 else
         synth.rasterize_ellipses(prm, cs.vol_shape, cs.vol_spacing)).numpy()
    p = ora.project(cs, f)
    p = p.reshape((spec.n_proj,) + tuple(cs.det_shape))

    def axis_map(n_full, d_full, n_c, d_c):
        x = (np.arange(n_full) - (n_full - 1) / 2) * d_full
        t = x / d_c + (n_c - 1) / 2
        t = np.clip(t, 0, n_c - 1)
        i0 = np.minimum(np.floor(t).astype(int), n_c - 2)
        return i0, t - i0

    if spec.ndim == 2:
        i0, w = axis_map(spec.det_shape[0], spec.det_spacing[0], cs.det_shape[0], cs.det_spacing[0])
        out = p[:, i0] * (1 - w) + p[:, i0 + 1] * w
    else:
        j0, wu = axis_map(spec.det_shape[1], spec.det_spacing[1], cs.det_shape[1], cs.det_spacing[1])
        i0, wv = axis_map(spec.det_shape[0], spec.det_spacing[0], cs.det_shape[0], cs.det_spacing[0])
        rows = p[:, i0, :] * (1 - wv)[None, :, None] + p[:, i0 + 1, :] * wv[None, :, None]
        out = rows[:, :, j0] * (1 - wu) + rows[:, :, j0 + 1] * wu
    return as_f32(out)
