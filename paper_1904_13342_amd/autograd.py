"""torch.autograd.Function wrappers of the projector and back-projector.

Sec. II.A / II.C.1: the layers register their gradients so that networks
built from them train end to end; Sec. II.B.1 (after Eq. 4) takes each
operator's adjoint as its gradient.  ``pairing="matched"`` (default) uses the
exact transposes (A^T for the projector, B^T for the back-projector);
``pairing="paper"`` uses the unmatched pair the paper ships (the
back-projector as the projector's gradient and vice versa, Sec. II.B.2 and
Sec. IV).  Argument marshalling only: every pass runs in libpyrohip.
"""
from __future__ import annotations

import torch

from . import ops

_FWD = {"par2d": ops.project_par2d, "fan2d": ops.project_fan2d, "cone3d": ops.project_cone3d}
_FWD_T = {"par2d": ops.project_adjoint_par2d, "fan2d": ops.project_adjoint_fan2d,
          "cone3d": ops.project_adjoint_cone3d}
_BP = {"par2d": ops.backproject_par2d, "fan2d": ops.backproject_fan2d, "cone3d": ops.backproject_cone3d}
_BP_T = {"par2d": ops.backproject_adjoint_par2d, "fan2d": ops.backproject_adjoint_fan2d,
         "cone3d": ops.backproject_adjoint_cone3d}


def _kind(g, fan):
    if isinstance(g, ops.Geom3D):
        return "cone3d"
    return "fan2d" if fan else "par2d"


class _Project(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, g, traj, kind, pairing):
        ctx.g, ctx.traj, ctx.kind, ctx.pairing = g, traj, kind, pairing
        return _FWD[kind](g, traj, x.contiguous())

    @staticmethod
    def backward(ctx, grad):
        grad = grad.contiguous()
        if ctx.pairing == "matched":
            gx = _FWD_T[ctx.kind](ctx.g, ctx.traj, grad)
        else:
            gx = _BP[ctx.kind](ctx.g, ctx.traj, grad)
        return gx, None, None, None, None


class _Backproject(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, g, traj, kind, pairing):
        ctx.g, ctx.traj, ctx.kind, ctx.pairing = g, traj, kind, pairing
        return _BP[kind](g, traj, q.contiguous())

    @staticmethod
    def backward(ctx, grad):
        grad = grad.contiguous()
        if ctx.pairing == "matched":
            gq = _BP_T[ctx.kind](ctx.g, ctx.traj, grad)
        else:
            gq = _FWD[ctx.kind](ctx.g, ctx.traj, grad)
        return gq, None, None, None, None


def project(x, g, traj, fan=False, pairing="matched"):
    """A x as a differentiable layer (2D: ``fan`` selects the fan beam)."""
    if pairing not in ("matched", "paper"):
        raise ValueError("pairing must be 'matched' or 'paper'")
    return _Project.apply(x, g, traj, _kind(g, fan), pairing)


def backproject(q, g, traj, fan=False, pairing="matched"):
    """B q as a differentiable layer."""
    if pairing not in ("matched", "paper"):
        raise ValueError("pairing must be 'matched' or 'paper'")
    return _Backproject.apply(q, g, traj, _kind(g, fan), pairing)


__all__ = ["project", "backproject"]
