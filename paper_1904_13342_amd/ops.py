"""Python binding of the C ABI (include/pyrohip.h), one function per entry
point with the same name minus the ``ph_`` prefix.

Argument marshalling only: tensors must already live on the GPU; shapes are
checked against the geometry here (the C ABI sees plain pointers), outputs
are allocated with torch, and the work is enqueued on torch's current HIP
stream.  Every operator runs in the HIP kernels of libpyrohip.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from ._lib import Geom2D, Geom3D, PH_BF16, PH_F16, PH_F32, TvParams, check, lib

_DTYPES = {torch.float32: PH_F32, torch.float16: PH_F16, torch.bfloat16: PH_BF16}


# ------------------------------------------------------------------ geometry

def geom2d(vol_shape, vol_spacing, det_shape, det_spacing, n_proj, angular_range, sid=0.0, sdd=0.0, step_mm=0.0,
           vol_origin=None, detector="flat"):
    """ph_geom2d record; shapes/spacings in (y, x) order; origin defaults to a
    grid centred on the rotation axis.  ``detector`` (fan beams): "flat" or
    "curved" (equiangular arc of radius SDD about the source, det_spacing the
    arc length between bins)."""
    if detector not in ("flat", "curved"):
        raise ValueError('detector must be "flat" or "curved"')
    g = Geom2D()
    vol_shape = tuple(int(v) for v in vol_shape)
    vol_spacing = tuple(float(v) for v in vol_spacing)
    if vol_origin is None:
        vol_origin = tuple(-(n - 1) / 2.0 * s for n, s in zip(vol_shape, vol_spacing))
    g.vol_shape[:] = vol_shape
    g.vol_spacing[:] = vol_spacing
    g.vol_origin[:] = tuple(float(v) for v in vol_origin)
    g.det_shape = int(det_shape[0] if isinstance(det_shape, (tuple, list)) else det_shape)
    g.det_spacing = float(det_spacing[0] if isinstance(det_spacing, (tuple, list)) else det_spacing)
    g.n_proj = int(n_proj)
    g.angular_range = float(angular_range)
    g.sid, g.sdd, g.step_mm = float(sid), float(sdd), float(step_mm)
    g.fan_detector = 1 if detector == "curved" else 0
    return g


def geom3d(vol_shape, vol_spacing, det_shape, det_spacing, n_proj, angular_range, sid, sdd, step_mm=0.0,
           vol_origin=None):
    """ph_geom3d record; volume in (z, y, x) order, detector in (v, u) order."""
    g = Geom3D()
    vol_shape = tuple(int(v) for v in vol_shape)
    vol_spacing = tuple(float(v) for v in vol_spacing)
    if vol_origin is None:
        vol_origin = tuple(-(n - 1) / 2.0 * s for n, s in zip(vol_shape, vol_spacing))
    g.vol_shape[:] = vol_shape
    g.vol_spacing[:] = vol_spacing
    g.vol_origin[:] = tuple(float(v) for v in vol_origin)
    g.det_shape[:] = tuple(int(v) for v in det_shape)
    g.det_spacing[:] = tuple(float(v) for v in det_spacing)
    g.n_proj = int(n_proj)
    g.angular_range = float(angular_range)
    g.sid, g.sdd, g.step_mm = float(sid), float(sdd), float(step_mm)
    return g


def from_spec(spec):
    """Geometry record from any object with the attributes kind, vol_shape,
    vol_spacing, det_shape, det_spacing, n_proj, angular_range, sid, sdd,
    step_mm (and optionally vol_origin); kind "fan2d_curved" selects the
    equiangular fan detector (use the *_fan2d calls with it)."""
    origin = getattr(spec, "vol_origin", None)
    if spec.kind == "cone3d":
        return geom3d(spec.vol_shape, spec.vol_spacing, spec.det_shape, spec.det_spacing, spec.n_proj,
                      spec.angular_range, spec.sid, spec.sdd, spec.step_mm, origin)
    return geom2d(spec.vol_shape, spec.vol_spacing, spec.det_shape, spec.det_spacing, spec.n_proj,
                  spec.angular_range, spec.sid, spec.sdd, spec.step_mm, origin,
                  detector="curved" if spec.kind == "fan2d_curved" else "flat")


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def ray_vectors_2d(g):
    out = np.empty((g.n_proj, 2), dtype=np.float32)
    check("ph_ray_vectors_2d", lib().ph_ray_vectors_2d(ctypes.byref(g), _fptr(out)))
    return out


def projection_matrices_3d(g):
    out = np.empty((g.n_proj, 3, 4), dtype=np.float32)
    check("ph_projection_matrices_3d", lib().ph_projection_matrices_3d(ctypes.byref(g), _fptr(out)))
    return out


# --------------------------------------------------------------- marshalling

def _host_traj(traj, shape):
    a = np.ascontiguousarray(np.asarray(traj, dtype=np.float32))
    if a.shape != shape:
        raise ValueError(f"trajectory has shape {a.shape}, expected {shape}")
    return a


def _dev(t, name, expect_tail):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor")
    if t.dtype not in _DTYPES:
        raise ValueError(f"{name} has unsupported dtype {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    tail = tuple(t.shape[-len(expect_tail):]) if t.dim() >= len(expect_tail) else None
    if tail != tuple(expect_tail) or t.dim() not in (len(expect_tail), len(expect_tail) + 1):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected [B,] {tuple(expect_tail)}")
    batch = 1 if t.dim() == len(expect_tail) else t.shape[0]
    if batch < 1:
        raise ValueError(f"{name} has an empty batch")
    return batch


def _f32_dev(t, name, n):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float32:
        raise ValueError(f"{name} must be a float32 GPU tensor")
    if not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be contiguous with {n} elements")
    return t.data_ptr()


def _stream(t):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _vol_tail(g):
    return tuple(g.vol_shape)


def _sino_tail(g):
    if isinstance(g, Geom3D):
        return (g.n_proj, g.det_shape[0], g.det_shape[1])
    return (g.n_proj, g.det_shape)


def _traj(g, traj):
    if isinstance(g, Geom3D):
        return _host_traj(traj, (g.n_proj, 3, 4))
    return _host_traj(traj, (g.n_proj, 2))


def _unary(fn, g, traj, x, in_tail, out_tail, out=None):
    batch = _dev(x, "input", in_tail)
    t = _traj(g, traj)
    shape = (tuple(x.shape[:1]) if x.dim() == len(in_tail) + 1 else ()) + tuple(out_tail)
    if out is None:
        out = torch.empty(shape, dtype=x.dtype, device=x.device)
    elif tuple(out.shape) != shape or out.dtype != x.dtype or not out.is_contiguous() or out.device != x.device:
        raise ValueError("out has the wrong shape, dtype, device or layout")
    status = getattr(lib(), fn)(ctypes.byref(g), _fptr(t), ctypes.c_void_p(x.data_ptr()),
                                ctypes.c_void_p(out.data_ptr()), batch, _DTYPES[x.dtype], _stream(x))
    check(fn, status)
    return out


# ----------------------------------------------------------------- operators

def project_par2d(g, ray_vecs, img, out=None):
    return _unary("ph_project_par2d", g, ray_vecs, img, _vol_tail(g), _sino_tail(g), out)


def project_fan2d(g, ray_vecs, img, out=None):
    return _unary("ph_project_fan2d", g, ray_vecs, img, _vol_tail(g), _sino_tail(g), out)


def project_cone3d(g, mats, vol, out=None):
    return _unary("ph_project_cone3d", g, mats, vol, _vol_tail(g), _sino_tail(g), out)


def backproject_par2d(g, ray_vecs, sino, out=None):
    return _unary("ph_backproject_par2d", g, ray_vecs, sino, _sino_tail(g), _vol_tail(g), out)


def backproject_fan2d(g, ray_vecs, sino, out=None):
    return _unary("ph_backproject_fan2d", g, ray_vecs, sino, _sino_tail(g), _vol_tail(g), out)


def backproject_cone3d(g, mats, proj, out=None):
    return _unary("ph_backproject_cone3d", g, mats, proj, _sino_tail(g), _vol_tail(g), out)


def project_adjoint_par2d(g, ray_vecs, sino, out=None):
    """A^T of project_par2d (exact transpose)."""
    return _unary("ph_project_adjoint_par2d", g, ray_vecs, sino, _sino_tail(g), _vol_tail(g), out)


def project_adjoint_fan2d(g, ray_vecs, sino, out=None):
    return _unary("ph_project_adjoint_fan2d", g, ray_vecs, sino, _sino_tail(g), _vol_tail(g), out)


def project_adjoint_cone3d(g, mats, proj, out=None):
    return _unary("ph_project_adjoint_cone3d", g, mats, proj, _sino_tail(g), _vol_tail(g), out)


def _bpT(fn, g, traj, x, out):
    """B^T; half-precision storage goes through the FP32-accumulating _ws entry point."""
    if x.dtype == torch.float32:
        return _unary(fn, g, traj, x, _vol_tail(g), _sino_tail(g), out)
    batch = _dev(x, "input", _vol_tail(g))
    t = _traj(g, traj)
    shape = (tuple(x.shape[:1]) if x.dim() == len(_vol_tail(g)) + 1 else ()) + tuple(_sino_tail(g))
    if out is None:
        out = torch.empty(shape, dtype=x.dtype, device=x.device)
    elif tuple(out.shape) != shape or out.dtype != x.dtype or not out.is_contiguous() or out.device != x.device:
        raise ValueError(f"out must be a contiguous {x.dtype} tensor of shape {shape} on {x.device}")
    q = lib().ph_backproject_adjoint_workspace_bytes_3d if isinstance(g, Geom3D) else \
        lib().ph_backproject_adjoint_workspace_bytes_2d
    nbytes = int(q(ctypes.byref(g), batch, _DTYPES[x.dtype]))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    name = fn.replace("ph_backproject_adjoint_", "ph_backproject_adjoint_ws_")
    status = getattr(lib(), name)(ctypes.byref(g), _fptr(t), ctypes.c_void_p(x.data_ptr()),
                                  ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()), nbytes, batch,
                                  _DTYPES[x.dtype], _stream(x))
    check(name, status)
    return out


def backproject_adjoint_par2d(g, ray_vecs, img, out=None):
    """B^T of backproject_par2d (exact transpose; any storage type, FP32 accumulation)."""
    return _bpT("ph_backproject_adjoint_par2d", g, ray_vecs, img, out)


def backproject_adjoint_fan2d(g, ray_vecs, img, out=None):
    return _bpT("ph_backproject_adjoint_fan2d", g, ray_vecs, img, out)


def backproject_adjoint_cone3d(g, mats, vol, out=None):
    return _bpT("ph_backproject_adjoint_cone3d", g, mats, vol, out)


def _filter_len(K, M):
    if K is not None:
        return K.numel() if M in (None, 0) else M
    return 0 if M is None else M


def weight_filter_2d(g, sino, fan, K=None, M=None, W_red=None, out=None):
    batch = _dev(sino, "sino", _sino_tail(g))
    M = _filter_len(K, M)
    shape = tuple(sino.shape)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=sino.device)
    status = lib().ph_weight_filter_2d(ctypes.byref(g), int(bool(fan)), ctypes.c_void_p(sino.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), _f32_dev(K, "K", M), M,
                                       _f32_dev(W_red, "W_red", g.n_proj * g.det_shape), batch,
                                       _DTYPES[sino.dtype], _stream(sino))
    check("ph_weight_filter_2d", status)
    return out


def weight_filter_3d(g, proj, K=None, M=None, W_red=None, W=None, out=None):
    batch = _dev(proj, "proj", _sino_tail(g))
    M = _filter_len(K, M)
    nv, nu = g.det_shape[0], g.det_shape[1]
    if out is None:
        out = torch.empty(tuple(proj.shape), dtype=torch.float32, device=proj.device)
    status = lib().ph_weight_filter_3d(ctypes.byref(g), ctypes.c_void_p(proj.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), _f32_dev(K, "K", M), M,
                                       _f32_dev(W_red, "W_red", g.n_proj * nu), _f32_dev(W, "W", nv * nu), batch,
                                       _DTYPES[proj.dtype], _stream(proj))
    check("ph_weight_filter_3d", status)
    return out


def filter_response(kind, M, tau):
    """Host float32 [M] response on the M-point grid: kind "ramlak" or "ramp"."""
    kinds = {"ramlak": 0, "ramp": 1}
    if kind not in kinds:
        raise ValueError(f"kind must be one of {sorted(kinds)}")
    K = (ctypes.c_float * int(M))()
    check("ph_filter_response", lib().ph_filter_response(kinds[kind], int(M), float(tau), K))
    return torch.tensor(list(K), dtype=torch.float32)


def filter_response_equiangular(M, alpha, sid):
    """Host float32 [M] equiangular Ram-Lak response (curved fan detector,
    angular bin pitch alpha = du / SDD)."""
    K = (ctypes.c_float * int(M))()
    check("ph_filter_response_equiangular",
          lib().ph_filter_response_equiangular(int(M), float(alpha), float(sid), K))
    return torch.tensor(list(K), dtype=torch.float32)


def _f32_like(t, name, numel=None):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float32:
        raise ValueError(f"{name} must be a float32 GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, has {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def mse_grad(x, ref, mask=None, grad=None, loss=None):
    """(loss, grad): L = mean((mask * (x - ref))^2) as a float64 device scalar, and dL/dx."""
    n = x.numel()
    px = _f32_like(x, "x")
    pr = _f32_like(ref, "ref", n)
    pm = None if mask is None else _f32_like(mask, "mask", n)
    if grad is None:
        grad = torch.empty_like(x)
    if loss is None:
        loss = torch.empty((), dtype=torch.float64, device=x.device)
    if loss.dtype != torch.float64 or loss.numel() != 1 or loss.device != x.device:
        raise ValueError("loss must be a one-element float64 tensor on the device of x")
    status = lib().ph_mse_grad(px, pr, pm, n, _f32_like(grad, "grad", n), ctypes.c_void_p(loss.data_ptr()),
                               _stream(x))
    check("ph_mse_grad", status)
    return loss, grad


def corrector_grad_3d(g, proj, grad_q, K, W_red=None, W=None, dK=None, dW=None, want_dW=True):
    """(dL/dK, dL/dW) of q = F^H K F (W W_red W_cos proj) given dL/dq; dW is
    None when want_dW is false."""
    if proj.dtype != torch.float32 or grad_q.dtype != torch.float32:
        raise ValueError("proj and grad_q must be float32")
    batch = _dev(proj, "proj", _sino_tail(g))
    if _dev(grad_q, "grad_q", _sino_tail(g)) != batch or grad_q.shape != proj.shape:
        raise ValueError("grad_q must have the shape of proj")
    M = K.numel()
    nv, nu = g.det_shape[0], g.det_shape[1]
    if dK is None:
        dK = torch.empty(M, dtype=torch.float32, device=proj.device)
    if want_dW and dW is None:
        dW = torch.empty((nv, nu), dtype=torch.float32, device=proj.device)
    if not want_dW:
        dW = None
    status = lib().ph_corrector_grad_3d(ctypes.byref(g), ctypes.c_void_p(proj.data_ptr()),
                                        ctypes.c_void_p(grad_q.data_ptr()), _f32_like(K, "K"), M,
                                        _f32_dev(W_red, "W_red", g.n_proj * nu), _f32_dev(W, "W", nv * nu),
                                        _f32_like(dK, "dK", M), None if dW is None else _f32_like(dW, "dW", nv * nu),
                                        batch, _stream(proj))
    check("ph_corrector_grad_3d", status)
    return dK, dW


def corrector_grad_2d(g, sino, grad_q, K, fan, W_red=None, dK=None):
    """dL/dK of q = F^H K F (W_red W_cos sino) given dL/dq (2D FBP network)."""
    if sino.dtype != torch.float32 or grad_q.dtype != torch.float32:
        raise ValueError("sino and grad_q must be float32")
    batch = _dev(sino, "sino", _sino_tail(g))
    if grad_q.shape != sino.shape or not grad_q.is_contiguous() or grad_q.device != sino.device:
        raise ValueError("grad_q must be a contiguous tensor of the shape of sino")
    M = K.numel()
    if dK is None:
        dK = torch.empty(M, dtype=torch.float32, device=sino.device)
    status = lib().ph_corrector_grad_2d(ctypes.byref(g), int(bool(fan)), ctypes.c_void_p(sino.data_ptr()),
                                        ctypes.c_void_p(grad_q.data_ptr()), _f32_like(K, "K"), M,
                                        _f32_dev(W_red, "W_red", g.n_proj * g.det_shape), _f32_like(dK, "dK", M),
                                        batch, _stream(sino))
    check("ph_corrector_grad_2d", status)
    return dK


def adam_step(param, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One in-place Adam step (t counts from 1)."""
    n = param.numel()
    status = lib().ph_adam_step(_f32_like(param, "param"), _f32_like(grad, "grad", n), _f32_like(m, "m", n),
                                _f32_like(v, "v", n), n, float(lr), float(beta1), float(beta2), float(eps), int(t),
                                _stream(param))
    check("ph_adam_step", status)
    return param


def tv(x, eps, dims, weight=1.0, grad=None, want_value=True, anisotropic=False):
    """Total variation of x, whose last `dims` (2 or 3) axes are spatial
    ([..., ny, nx] or [..., nz, ny, nx]) and the others a batch, FP32:
    isotropic, or with anisotropic=True the sum of absolute differences per
    axis (eps = 0 allowed).  Returns (value, grad): value is a float64 device
    tensor with the batch shape (a scalar when there is no batch axis); grad,
    when given, is updated in place: grad += weight * dTV/dx."""
    if dims not in (2, 3):
        raise ValueError("dims must be 2 or 3")
    if not isinstance(x, torch.Tensor) or x.device.type != "cuda" or x.dtype != torch.float32:
        raise ValueError("x must be a float32 GPU tensor")
    if not x.is_contiguous() or x.dim() < dims:
        raise ValueError(f"x must be contiguous with at least {dims} dimensions")
    nx, ny = x.shape[-1], x.shape[-2]
    nz = x.shape[-3] if dims == 3 else 1
    lead = tuple(x.shape[:-dims])
    batch = 1
    for n in lead:
        batch *= n
    if grad is not None:
        _f32_like(grad, "grad", x.numel())
        if grad.data_ptr() == x.data_ptr():
            raise ValueError("grad must not alias x")
    value = torch.empty(max(batch, 1), dtype=torch.float64, device=x.device) if want_value else None
    status = lib().ph_tv_3d(ctypes.c_void_p(x.data_ptr()), nz, ny, nx, batch, int(bool(anisotropic)), float(eps),
                            float(weight),
                            None if grad is None else ctypes.c_void_p(grad.data_ptr()),
                            None if value is None else ctypes.c_void_p(value.data_ptr()), _stream(x))
    check("ph_tv_3d", status)
    if value is not None:
        value = value.reshape(lead) if lead else value[0]
    return value, grad


def tv_workspace_bytes(g, batch=1):
    fn = lib().ph_tv_workspace_bytes_3d if isinstance(g, Geom3D) else lib().ph_tv_workspace_bytes_2d
    return int(fn(ctypes.byref(g), int(batch)))


def tv_iterate(kind, g, traj, proj, x, m, v, t0, n_iter, lam, eps, lr=1e-2, beta1=0.9, beta2=0.999, adam_eps=1e-8,
               ws=None, data_tv=None, anisotropic=False):
    """n_iter iterations of the TV-regularised reconstruction in one library
    call (x, m, v updated in place, Adam steps t0+1 .. t0+n_iter).  Returns
    data_tv, a float64 device tensor [1 + batch]: the data term and each
    item's TV at the iterate before the last update."""
    fns = {"par2d": "ph_tv_iterate_par2d", "fan2d": "ph_tv_iterate_fan2d", "cone3d": "ph_tv_iterate_cone3d"}
    if kind not in fns:
        raise ValueError(f"kind must be one of {sorted(fns)}")
    batch = _dev(proj, "proj", _sino_tail(g))
    if proj.dtype != torch.float32:
        raise ValueError("proj must be float32")
    nimg = batch * int(torch.tensor(list(g.vol_shape)).prod())
    for t, name in ((x, "x"), (m, "m"), (v, "v")):
        _f32_like(t, name, nimg)
    t = _traj(g, traj)
    need = tv_workspace_bytes(g, batch)
    if ws is None or ws.numel() * ws.element_size() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=proj.device)
    if data_tv is None:
        data_tv = torch.empty(1 + batch, dtype=torch.float64, device=proj.device)
    prm = TvParams(float(lam), float(eps), float(lr), float(beta1), float(beta2), float(adam_eps),
                   int(bool(anisotropic)))
    status = getattr(lib(), fns[kind])(ctypes.byref(g), _fptr(t), ctypes.c_void_p(proj.data_ptr()),
                                       ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(m.data_ptr()),
                                       ctypes.c_void_p(v.data_ptr()), int(t0), int(n_iter), ctypes.byref(prm),
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                                       ctypes.c_void_p(data_tv.data_ptr()), batch, _stream(proj))
    check(fns[kind], status)
    return data_tv


def workspace_bytes_2d(g, batch=1):
    return int(lib().ph_workspace_bytes_2d(ctypes.byref(g), int(batch)))


def workspace_bytes_3d(g, batch=1):
    return int(lib().ph_workspace_bytes_3d(ctypes.byref(g), int(batch)))


def fdk_workspace_bytes(g, M=0, batch=1, dtype=torch.float32):
    return int(lib().ph_fdk_workspace_bytes(ctypes.byref(g), int(M), int(batch), _DTYPES[dtype]))


def _fbp2d(fn, g, ray_vecs, sino, K, M, W_red, out, ws):
    batch = _dev(sino, "sino", _sino_tail(g))
    t = _traj(g, ray_vecs)
    M = _filter_len(K, M)
    shape = (tuple(sino.shape[:1]) if sino.dim() == 3 else ()) + _vol_tail(g)
    if out is None:
        out = torch.empty(shape, dtype=sino.dtype, device=sino.device)
    nbytes = workspace_bytes_2d(g, batch)
    if ws is None:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=sino.device)
    status = getattr(lib(), fn)(ctypes.byref(g), _fptr(t), ctypes.c_void_p(sino.data_ptr()),
                                ctypes.c_void_p(out.data_ptr()), _f32_dev(K, "K", M), M,
                                _f32_dev(W_red, "W_red", g.n_proj * g.det_shape), ctypes.c_void_p(ws.data_ptr()),
                                ws.numel() * ws.element_size(), batch, _DTYPES[sino.dtype], _stream(sino))
    check(fn, status)
    return out


def fbp_par2d(g, ray_vecs, sino, K=None, M=None, W_red=None, out=None, ws=None):
    return _fbp2d("ph_fbp_par2d", g, ray_vecs, sino, K, M, W_red, out, ws)


def fbp_fan2d(g, ray_vecs, sino, K=None, M=None, W_red=None, out=None, ws=None):
    return _fbp2d("ph_fbp_fan2d", g, ray_vecs, sino, K, M, W_red, out, ws)


def fdk_cone3d(g, mats, proj, K=None, M=None, W_red=None, W=None, out=None, ws=None):
    batch = _dev(proj, "proj", _sino_tail(g))
    t = _traj(g, mats)
    M = _filter_len(K, M)
    nv, nu = g.det_shape[0], g.det_shape[1]
    shape = (tuple(proj.shape[:1]) if proj.dim() == 4 else ()) + _vol_tail(g)
    if out is None:
        out = torch.empty(shape, dtype=proj.dtype, device=proj.device)
    nbytes = fdk_workspace_bytes(g, M, batch, proj.dtype)
    if ws is None:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=proj.device)
    status = lib().ph_fdk_cone3d(ctypes.byref(g), _fptr(t), ctypes.c_void_p(proj.data_ptr()),
                                 ctypes.c_void_p(out.data_ptr()), _f32_dev(K, "K", M), M,
                                 _f32_dev(W_red, "W_red", g.n_proj * nu), _f32_dev(W, "W", nv * nu),
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(), batch,
                                 _DTYPES[proj.dtype], _stream(proj))
    check("ph_fdk_cone3d", status)
    return out


def fdk_cone3d_static(g, mats, proj, out, K=None, M=None, W_red=None, W=None):
    """ph_fdk_cone3d_static: FDK into the caller's ``out`` with the library's
    static scratch (no device allocation in the library or here)."""
    batch = _dev(proj, "proj", _sino_tail(g))
    t = _traj(g, mats)
    M = _filter_len(K, M)
    nv, nu = g.det_shape[0], g.det_shape[1]
    shape = (tuple(proj.shape[:1]) if proj.dim() == 4 else ()) + _vol_tail(g)
    if tuple(out.shape) != shape or out.dtype != proj.dtype or out.device != proj.device or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous {proj.dtype} tensor of shape {shape} on {proj.device}")
    status = lib().ph_fdk_cone3d_static(ctypes.byref(g), _fptr(t), ctypes.c_void_p(proj.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), _f32_dev(K, "K", M), M,
                                        _f32_dev(W_red, "W_red", g.n_proj * nu), _f32_dev(W, "W", nv * nu), batch,
                                        _DTYPES[proj.dtype], _stream(proj))
    check("ph_fdk_cone3d_static", status)
    return out


def version():
    return lib().ph_version().decode()


__all__ = [
    "Geom2D", "Geom3D", "geom2d", "geom3d", "from_spec", "ray_vectors_2d", "projection_matrices_3d", "project_par2d",
    "project_fan2d", "project_cone3d", "backproject_par2d", "backproject_fan2d", "backproject_cone3d",
    "project_adjoint_par2d", "project_adjoint_fan2d", "project_adjoint_cone3d", "backproject_adjoint_par2d",
    "backproject_adjoint_fan2d", "backproject_adjoint_cone3d",
    "weight_filter_2d", "weight_filter_3d", "workspace_bytes_2d", "workspace_bytes_3d", "fdk_workspace_bytes",
    "fbp_par2d",
    "fbp_fan2d", "fdk_cone3d", "fdk_cone3d_static", "filter_response", "filter_response_equiangular", "tv", "tv_workspace_bytes",
    "tv_iterate", "mse_grad",
    "corrector_grad_3d", "corrector_grad_2d", "adam_step", "version",
]
