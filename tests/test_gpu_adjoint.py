"""Exact transposes A^T and B^T on the GPU: element-wise parity with the
oracle's scatter transposes (themselves pinned against dense brute force),
the adjoint identity <A x, y> = <x, A^T y> at full size, and finite-difference
gradient checks of the autograd layers on the 32^3 crop of the 512^3
workload (the losses are quadratic, so central differences are exact up to
rounding)."""
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


SPECS = {
    "par2d_64": synth.config("par2d_64"),
    "fan2d_ragged": synth.config("fan2d_512").with_(vol_shape=(45, 31), vol_spacing=(1.0, 1.2), det_shape=(77,),
                                                    det_spacing=(1.1,), n_proj=11, angular_range=250 * math.pi / 180,
                                                    sid=100.0, sdd=160.0),
    "cone_crop32": synth.config("cone3d_crop32").with_(n_proj=60),
    "cone_tall_pixels": synth.config("cone3d_crop32").with_(det_shape=(140, 72), det_spacing=(0.2, 0.4), n_proj=90),
    "cone_ragged": synth.config("cone3d_crop32").with_(vol_shape=(23, 29, 35), vol_spacing=(1.1, 0.9, 1.0),
                                                       det_shape=(37, 41), det_spacing=(1.7, 1.5), n_proj=17,
                                                       angular_range=200 * math.pi / 180, sid=300.0, sdd=500.0),
}


def _ops(ph, spec):
    g = ph.from_spec(spec)
    if spec.kind == "cone3d":
        return g, ph.projection_matrices_3d(g), ph.project_cone3d, ph.project_adjoint_cone3d, \
            ph.backproject_cone3d, ph.backproject_adjoint_cone3d
    rv = ph.ray_vectors_2d(g)
    if spec.kind == "par2d":
        return g, rv, ph.project_par2d, ph.project_adjoint_par2d, ph.backproject_par2d, ph.backproject_adjoint_par2d
    return g, rv, ph.project_fan2d, ph.project_adjoint_fan2d, ph.backproject_fan2d, ph.backproject_adjoint_fan2d


@pytest.mark.parametrize("name", list(SPECS))
def test_project_adjoint_parity(ph, ora, name):
    spec = SPECS[name]
    say(f"[project_adjoint] {name}")
    g, traj, _, fT, _, _ = _ops(ph, spec)
    p = as_f32(ora.project(spec, gc.phantom(spec)))       # realistic projection data
    out = fT(g, traj, to_dev(p))
    check(to_np(out), ora.project_adjoint(spec, p), "")


@pytest.mark.parametrize("name", list(SPECS))
def test_backproject_adjoint_parity(ph, ora, name):
    spec = SPECS[name]
    say(f"[backproject_adjoint] {name}")
    g, traj, _, _, _, bT = _ops(ph, spec)
    f = gc.phantom(spec)
    out = bT(g, traj, to_dev(f))
    check(to_np(out), ora.backproject_adjoint(spec, f), "")


def test_backproject_adjoint_plain_entry_rejects_half(ph):
    """The plain B^T entry point is FP32-only (its scatter accumulates in the
    output); half precision goes through the workspace variant."""
    import ctypes
    from paper_1904_13342_amd._lib import lib
    spec = SPECS["cone_crop32"]
    g, traj, _, _, _, _ = _ops(ph, spec)
    x = torch.zeros(spec.vol_shape, dtype=torch.float16, device=gc.device())
    y = torch.zeros((spec.n_proj,) + tuple(spec.det_shape), dtype=torch.float16, device=gc.device())
    st = lib().ph_backproject_adjoint_cone3d(ctypes.byref(g), traj.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                             ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), 1, 1, None)
    assert st == -7
    st = lib().ph_backproject_adjoint_ws_cone3d(ctypes.byref(g), traj.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), None, 0,
                                                1, 1, None)
    assert st == -5


def _dot(a, b):
    return float((a.double() * b.double()).sum())


@pytest.mark.parametrize("name", ["fan2d_512", "cone3d_256_short", "cone3d_512"])
def test_adjoint_identity_full_size(ph, name):
    """<A x, y> = <x, A^T y> and <B y, x> = <y, B^T x> with random x, y, in the
    launch configuration of the benchmark; FP32 kernels, FP64 inner products."""
    spec = synth.config(name)
    say(f"[adjoint identity] {name}")
    g, traj, f, fT, b, bT = _ops(ph, spec)
    dev = gc.device()
    gen = torch.Generator(device=dev).manual_seed(7)
    x = torch.randn(spec.vol_shape, device=dev, generator=gen)
    y = torch.randn((spec.n_proj,) + tuple(spec.det_shape), device=dev, generator=gen)
    Ax = f(g, traj, x)
    lhs, rhs = _dot(Ax, y), _dot(x, fT(g, traj, y))
    del Ax
    rel = abs(lhs - rhs) / abs(lhs)
    say(f"  A: {lhs:.6e} vs {rhs:.6e}  rel {rel:.2e}")
    assert rel < 1e-5
    By = b(g, traj, y)
    lhs, rhs = _dot(By, x), _dot(y, bT(g, traj, x))
    rel = abs(lhs - rhs) / abs(lhs)
    say(f"  B: {lhs:.6e} vs {rhs:.6e}  rel {rel:.2e}")
    assert rel < 1e-5


@pytest.mark.parametrize("pairing", ["matched", "paper"])
def test_autograd_wiring(ph, pairing):
    """backward of the layers is the selected operator."""
    spec = SPECS["cone_ragged"]
    g, traj, f, fT, b, bT = _ops(ph, spec)
    dev = gc.device()
    x = torch.randn(spec.vol_shape, device=dev, requires_grad=True)
    y = torch.randn((spec.n_proj,) + tuple(spec.det_shape), device=dev)
    (ph.autograd.project(x, g, traj, pairing=pairing) * y).sum().backward()
    expect = fT(g, traj, y) if pairing == "matched" else b(g, traj, y)
    assert torch.equal(x.grad, expect)
    q = torch.randn_like(y, requires_grad=True)
    (ph.autograd.backproject(q, g, traj, pairing=pairing) * x.detach()).sum().backward()
    expect = bT(g, traj, x.detach()) if pairing == "matched" else f(g, traj, x.detach())
    assert rel_l2(to_np(q.grad), to_np(expect)) < 1e-6   # B^T sums with atomics: order may differ


def test_finite_difference_gradient_crop32(ph):
    """L(x) = 1/2 |A x - p|^2 on the 32^3 crop (0.5 mm voxels, 48 x 48 central
    detector window at 0.8 mm, 360 views): the autograd gradient A^T (A x - p)
    matches central differences along random directions (exact for a
    quadratic up to rounding)."""
    spec = synth.config("cone3d_crop32")
    g, traj, f, _, _, _ = _ops(ph, spec)
    dev = gc.device()
    gen = torch.Generator(device=dev).manual_seed(3)
    p = f(g, traj, to_dev(gc.phantom(spec)))
    x = torch.rand(spec.vol_shape, device=dev, generator=gen).requires_grad_(True)

    def loss(v):
        r = f(g, traj, v.contiguous()).double() - p.double()
        return 0.5 * float((r * r).sum())

    r = ph.autograd.project(x, g, traj) - p
    (0.5 * (r * r).sum()).backward()
    grad = x.grad.double()
    for seed in range(3):
        d = torch.randn(spec.vol_shape, device=dev, generator=gen)
        eps = 0.5
        fd = (loss(x.detach() + eps * d) - loss(x.detach() - eps * d)) / (2 * eps)
        an = float((grad * d.double()).sum())
        rel = abs(fd - an) / abs(an)
        say(f"[FD crop32] direction {seed}: FD {fd:.6e} autograd {an:.6e} rel {rel:.2e}")
        assert rel < 1e-3
