"""The FDK entry point that allocates nothing (ph_fdk_cone3d_static), called
through the C ABI, against ph_fdk_cone3d with a caller-supplied workspace on
the same inputs: two calls in a row, the second with a smaller input.  The
first needs several shares of the views (the static scratch holds the
filtered projections of only some of them), so the shares' adding into the
volume is exercised; the second fits one share."""
import ctypes
import math

import numpy as np
import pytest
import torch

import gpu_common as gc
import synth
from gpu_common import check, say, to_np

pytestmark = pytest.mark.gpu

SCRATCH = 64 << 20


@pytest.fixture(scope="module")
def ph():
    gc.device()
    import paper_1904_13342_amd as ph
    return ph


def _case(ph, spec, batch, seed, dtype=torch.float32):
    g = ph.from_spec(spec)
    mats = ph.projection_matrices_3d(g)
    gen = torch.Generator(device=gc.device()).manual_seed(seed)
    proj = torch.rand((batch, spec.n_proj) + tuple(spec.det_shape), device=gc.device(), generator=gen)
    proj = proj.to(dtype).contiguous()
    return g, mats, proj


def _call_static(ph, g, mats, proj, out):
    L = ph._lib.lib()
    t = np.ascontiguousarray(mats, dtype=np.float32)
    status = L.ph_fdk_cone3d_static(ctypes.byref(g), t.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                    ctypes.c_void_p(proj.data_ptr()), ctypes.c_void_p(out.data_ptr()), None, 0,
                                    None, None, proj.shape[0], ph.ops._DTYPES[proj.dtype],
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return status


def test_static_fdk_two_calls(ph):
    big = synth.config("cone3d_crop32").with_(vol_shape=(96, 128, 128), vol_spacing=(1.0, 1.0, 1.0),
                                              det_shape=(384, 512), det_spacing=(1.0, 1.0), n_proj=240,
                                              angular_range=200 * math.pi / 180)
    small = synth.config("cone3d_crop32").with_(n_proj=90, det_shape=(96, 128), det_spacing=(1.2, 1.2))
    for name, spec, batch, seed in (("several shares", big, 2, 1), ("one share", small, 1, 2)):
        g, mats, proj = _case(ph, spec, batch, seed)
        per_view = batch * spec.det_shape[0] * spec.det_shape[1] * 4
        say(f"{name}: {spec.vol_shape}, {spec.n_proj} views of {spec.det_shape}, batch {batch}: "
            f"{per_view * spec.n_proj / 2**20:.1f} MiB of filtered projections for a {SCRATCH >> 20} MiB scratch")
        ref = ph.fdk_cone3d(g, mats, proj)
        out = torch.full_like(ref, float("nan"))
        assert _call_static(ph, g, mats, proj, out) == 0
        torch.cuda.synchronize()
        check(to_np(out), to_np(ref), f"{name}: static vs workspace FDK")


def test_static_fdk_half_one_share(ph):
    small = synth.config("cone3d_crop32").with_(n_proj=90, det_shape=(96, 128), det_spacing=(1.2, 1.2))
    for dt, key in ((torch.float16, "f16"), (torch.bfloat16, "bf16")):
        g, mats, proj = _case(ph, small, 1, 3, dt)
        ref = ph.fdk_cone3d(g, mats, proj)
        out = torch.empty_like(ref)
        assert _call_static(ph, g, mats, proj, out) == 0
        torch.cuda.synchronize()
        check(to_np(out), to_np(ref), f"{key}: static vs workspace FDK", tol=gc.FP32_TOL,
              elem=gc.ELEM_TOL_HALF[key])


def test_static_fdk_rejects_half_in_shares(ph):
    big = synth.config("cone3d_crop32").with_(det_shape=(384, 512), det_spacing=(1.0, 1.0), n_proj=240)
    g, mats, proj = _case(ph, big, 1, 4, torch.float16)
    out = torch.empty((1,) + tuple(big.vol_shape), dtype=torch.float16, device=proj.device)
    assert _call_static(ph, g, mats, proj, out) == -5   # PH_ERR_WORKSPACE
