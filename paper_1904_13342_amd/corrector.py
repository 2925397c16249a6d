"""Learned sinogram-domain corrector for short-scan cone-beam FDK.

The FDK network of Eq. 5 with two trainable projection-domain layers: the
filter K on the M-point DFT grid (Sec. III.B / Eq. 6 trains it from a ramp
initialisation) and per-detector-pixel weights W multiplying the fixed
cosine and redundancy weights (Sec. III.A: the redundancy weights can be
learned, updated by back-propagation from a loss in the volume, as in Wurfl
et al.):

    x = B F^H K F (W * W_red * W_cos * p).

One training step is five library calls on the caller's stream: FDK with the
current K and W, the MSE loss and its gradient, B^T, the K / W gradient
reduction and Adam on both.  This module only owns the parameters and the
buffers (torch tensors used as device memory); every step runs in the HIP
kernels behind the C ABI.
"""
from __future__ import annotations

import torch

from . import ops


class LearnedCorrector:
    """Trainable (K, W) of the corrected FDK of one cone-beam geometry.

    g, mats : the geometry record and host [n_proj, 3, 4] projection matrices;
    M       : filter length (power of two, >= nu);
    K, W    : initial parameters (default: the ramp |f| on the DFT grid and
              ones), copied to FP32 device tensors;
    lr, betas, eps : Adam hyper-parameters;
    k_unit, w_unit : the units K and W are learned in: Adam steps
              theta = K / k_unit and omega = W / w_unit with lr and eps, so
              K moves by about lr * k_unit per step and W by lr * w_unit.
              k_unit defaults to 1 / (M tau), the ramp's step between
              adjacent DFT bins (the ramp initialisation is min(f, M - f) in
              it); w_unit to 1e-2.  1.0 learns a parameter in its own units.
    """

    def __init__(self, g, mats, M=1024, K=None, W=None, lr=1e-3, betas=(0.9, 0.999), eps=1e-8, device="cuda",
                 k_unit=None, w_unit=1e-2):
        self.g, self.mats = g, mats
        nv, nu = g.det_shape[0], g.det_shape[1]
        tau = g.det_spacing[1] * g.sid / g.sdd
        if K is None:
            K = ops.filter_response("ramp", M, tau)
        M = K.numel()
        self.k_unit = 1.0 / (M * tau) if k_unit is None else float(k_unit)
        self.K = K.detach().to(device=device, dtype=torch.float32).contiguous().clone()
        if W is None:
            W = torch.ones((nv, nu))
        self.W = W.detach().to(device=device, dtype=torch.float32).reshape(nv, nu).contiguous().clone()
        self.M = self.K.numel()
        self.lr, self.betas, self.eps = lr, betas, eps
        self.w_unit = float(w_unit)
        self.mK, self.vK = torch.zeros_like(self.K), torch.zeros_like(self.K)
        self.mW, self.vW = torch.zeros_like(self.W), torch.zeros_like(self.W)
        self.t = 0
        self._ws = None
        self._buf = {}

    def _buffer(self, name, shape, like):
        b = self._buf.get(name)
        if b is None or tuple(b.shape) != tuple(shape) or b.device != like.device:
            b = torch.empty(shape, dtype=torch.float32, device=like.device)
            self._buf[name] = b
        return b

    def _workspace(self, proj):
        batch = proj.shape[0] if proj.dim() == 4 else 1
        need = ops.workspace_bytes_3d(self.g, batch)
        if self._ws is None or self._ws.numel() < need or self._ws.device != proj.device:
            self._ws = torch.empty(need, dtype=torch.uint8, device=proj.device)
        return self._ws

    def reconstruct(self, proj, out=None):
        """x = B F^H K F (W W_red W_cos proj) with the current parameters."""
        return ops.fdk_cone3d(self.g, self.mats, proj, K=self.K, W=self.W, out=out, ws=self._workspace(proj))

    def gradients(self, proj, target, mask=None):
        """(loss, dL/dK, dL/dW) of L = mean((mask (x - target))^2) at the
        current parameters; loss is a device scalar."""
        shape = tuple(target.shape)
        x = self.reconstruct(proj, out=self._buffer("x", shape, proj))
        loss, gx = ops.mse_grad(x, target, mask, grad=self._buffer("gx", shape, proj))
        gq = ops.backproject_adjoint_cone3d(self.g, self.mats, gx, out=self._buffer("gq", tuple(proj.shape), proj))
        dK, dW = ops.corrector_grad_3d(self.g, proj, gq, self.K, W=self.W, dK=self._buffer("dK", (self.M,), proj),
                                       dW=self._buffer("dW", tuple(self.W.shape), proj))
        return loss, dK, dW

    def step(self, proj, target, mask=None):
        """One Adam step on K and W; returns the loss (device scalar) before it."""
        loss, dK, dW = self.gradients(proj, target, mask)
        self.t += 1
        b1, b2 = self.betas
        # Adam on theta = K / k_unit, whose gradient is k_unit dK: Adam is
        # invariant to the gradient's scale, so this is Adam on K with the
        # step times k_unit and eps over k_unit (likewise for W)
        ops.adam_step(self.K, dK, self.mK, self.vK, self.t, lr=self.lr * self.k_unit, beta1=b1, beta2=b2,
                      eps=self.eps / self.k_unit)
        ops.adam_step(self.W, dW, self.mW, self.vW, self.t, lr=self.lr * self.w_unit, beta1=b1, beta2=b2,
                      eps=self.eps / self.w_unit)
        return loss.clone()


class LearnedFilter2D:
    """The 2D FBP network of Sec. III.B / Eq. 6, x = B F^H K F W p, with the
    filter K as its only trainable layer (initialised with the ramp).

    g, ray_vecs : a 2D geometry and its central ray vectors; fan selects the
    fan-beam pair (cosine weight, distance-weighted B) over the parallel one.
    M defaults to the linear-convolution length (smallest power of two
    >= 2 nu - 1).
    """

    def __init__(self, g, ray_vecs, fan=False, M=None, K=None, lr=1e-3, betas=(0.9, 0.999), eps=1e-8,
                 device="cuda"):
        self.g, self.rv, self.fan = g, ray_vecs, bool(fan)
        nu = g.det_shape
        if M is None:
            M = 16
            while M < 2 * nu - 1:
                M *= 2
        tau = g.det_spacing * (g.sid / g.sdd if fan else 1.0)
        if K is None:
            K = ops.filter_response("ramp", M, tau)
        self.K = K.detach().to(device=device, dtype=torch.float32).contiguous().clone()
        self.M = self.K.numel()
        self.tau = tau
        self.lr, self.betas, self.eps = lr, betas, eps
        self.mK, self.vK = torch.zeros_like(self.K), torch.zeros_like(self.K)
        self.t = 0

    def reconstruct(self, sino):
        fbp = ops.fbp_fan2d if self.fan else ops.fbp_par2d
        return fbp(self.g, self.rv, sino, K=self.K)

    def gradients(self, sino, target, mask=None):
        """(loss, dL/dK) of L = mean((mask (x - target))^2)."""
        x = self.reconstruct(sino)
        loss, gx = ops.mse_grad(x, target, mask)
        bT = ops.backproject_adjoint_fan2d if self.fan else ops.backproject_adjoint_par2d
        gq = bT(self.g, self.rv, gx)
        dK = ops.corrector_grad_2d(self.g, sino, gq, self.K, self.fan)
        return loss, dK

    def step(self, sino, target, mask=None):
        loss, dK = self.gradients(sino, target, mask)
        self.t += 1
        b1, b2 = self.betas
        ops.adam_step(self.K, dK, self.mK, self.vK, self.t, lr=self.lr, beta1=b1, beta2=b2, eps=self.eps)
        return loss


__all__ = ["LearnedCorrector", "LearnedFilter2D"]
