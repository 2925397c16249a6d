"""TV-regularised iterative reconstruction as a network (Sec. III.B.1, Eq. 7).

The image is the weight of an additive layer fed with zeros, so the network
output is the image itself; it is forward projected and trained on

    L(x) = mean((A x - p)^2) + lam * TV_eps(x)

with Adam, starting from zero.  (Eq. 7 writes the data term as a squared
norm; the mean only rescales lam.)  One iteration is five library calls on
the caller's stream: the forward projection, the residual gradient, the
matched adjoint A^T, the TV gradient added in place and the Adam step;
`run` issues many iterations from the library in one call.  This module
only owns the buffers.
"""
from __future__ import annotations

import torch

from . import ops

_PROJECT = {"par2d": (ops.project_par2d, ops.project_adjoint_par2d, 2),
            "fan2d": (ops.project_fan2d, ops.project_adjoint_fan2d, 2),
            "cone3d": (ops.project_cone3d, ops.project_adjoint_cone3d, 3)}


class TVReconstruction:
    """Iterative reconstruction of the measured projections p.

    kind : "par2d", "fan2d" or "cone3d" (g and traj as for the operators);
    p    : FP32 device projections, [n_proj, nu] / [n_proj, nv, nu] or with a
           leading batch axis;
    lam, eps : TV weight and smoothing; lr, betas, adam_eps : Adam;
    anisotropic : TV as the sum of absolute differences per axis (the
           framework's own total variation the paper uses) instead of the
           isotropic gradient magnitude.
    """

    def __init__(self, kind, g, traj, p, lam=1e-3, eps=1e-3, lr=1e-2, betas=(0.9, 0.999), adam_eps=1e-8,
                 anisotropic=False):
        if kind not in _PROJECT:
            raise ValueError(f"kind must be one of {sorted(_PROJECT)}")
        self.project, self.adjoint, self.dims = _PROJECT[kind]
        self.kind, self.g, self.traj, self.p = kind, g, traj, p
        self.lam, self.eps, self.lr, self.betas, self.adam_eps = lam, eps, lr, betas, adam_eps
        self.anisotropic = bool(anisotropic)
        lead = tuple(p.shape[:-self.dims])   # batch axes (the projection tail has `dims` axes)
        shape = lead + tuple(g.vol_shape)
        self.x = torch.zeros(shape, dtype=torch.float32, device=p.device)
        self.m = torch.zeros_like(self.x)
        self.v = torch.zeros_like(self.x)
        self.t = 0
        self._r = torch.empty_like(p)
        self._gr = torch.empty_like(p)
        self._gx = torch.empty_like(self.x)
        self._ws = None

    def step(self):
        """One Adam step; returns (data term, TV) at the iterate before it,
        as device scalars."""
        self.project(self.g, self.traj, self.x, out=self._r)
        data, _ = ops.mse_grad(self._r, self.p, grad=self._gr)
        self.adjoint(self.g, self.traj, self._gr, out=self._gx)
        tv, _ = ops.tv(self.x, self.eps, self.dims, weight=self.lam, grad=self._gx, anisotropic=self.anisotropic)
        self.t += 1
        b1, b2 = self.betas
        ops.adam_step(self.x, self._gx, self.m, self.v, self.t, lr=self.lr, beta1=b1, beta2=b2, eps=self.adam_eps)
        return data, tv

    def run(self, iters):
        """iters iterations in one library call (the same five steps, issued
        without a host round trip per kernel); returns the float64 device
        tensor [data term, TV per item] at the iterate before the last update."""
        if self._ws is None:
            batch = self.x.numel() // max(1, int(torch.tensor(list(self.g.vol_shape)).prod()))
            self._ws = torch.empty(ops.tv_workspace_bytes(self.g, batch), dtype=torch.uint8, device=self.x.device)
        b1, b2 = self.betas
        out = ops.tv_iterate(self.kind, self.g, self.traj, self.p, self.x, self.m, self.v, self.t, iters, self.lam,
                             self.eps, lr=self.lr, beta1=b1, beta2=b2, adam_eps=self.adam_eps, ws=self._ws,
                             anisotropic=self.anisotropic)
        self.t += iters
        return out


__all__ = ["TVReconstruction"]
