"""Workload presets: geometry scalars only, as the paper's geometry classes
list them (Sec. II.C.1): volume shape and spacing, detector shape and
spacing, number of projections, angular range, SID and SDD, plus the ray
sampling step of the forward projector.

Axis order: 2D volume ``(ny, nx)``, 3D volume ``(nz, ny, nx)``; 2D detector
``(nu,)``, 3D detector ``(nv, nu)``.  Angles in radians, lengths in mm.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace


@dataclass(frozen=True)
class GeometrySpec:
    kind: str                      # "par2d" | "fan2d" | "cone3d"
    vol_shape: tuple
    vol_spacing: tuple
    det_shape: tuple
    det_spacing: tuple
    n_proj: int
    angular_range: float
    sid: float = 0.0
    sdd: float = 0.0
    step_mm: float = 0.0           # 0 -> half the smallest voxel spacing
    vol_origin: tuple = None       # None -> grid centred on the rotation axis
    # phantom recipe
    n_figures: int = 10
    seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def ndim(self):
        return len(self.vol_shape)

    @property
    def origin(self):
        if self.vol_origin is not None:
            return tuple(self.vol_origin)
        return tuple(-(n - 1) / 2.0 * s for n, s in zip(self.vol_shape, self.vol_spacing))

    @property
    def step(self):
        return self.step_mm if self.step_mm > 0 else 0.5 * min(self.vol_spacing)

    def with_(self, **kw):
        return replace(self, **kw)


DEG = math.pi / 180.0

CONFIGS = {
    # 2D parallel-beam FBP, 64x64 image of 10 ellipses, 90 views over 180 deg, 96 bins.
    "par2d_64": GeometrySpec("par2d", (64, 64), (1.0, 1.0), (96,), (1.0,), 90, math.pi,
                             n_figures=10),
    # 2D fan-beam, flat detector, 512x512 at 0.5 mm, 360 views over 360 deg, 725 bins.
    "fan2d_512": GeometrySpec("fan2d", (512, 512), (0.5, 0.5), (725,), (1.0,), 360, 2 * math.pi,
                              sid=750.0, sdd=1200.0, n_figures=10),
    # 3D circular short-scan FDK: 256^3 at 1 mm, 248 views over 200 deg, 620x480 detector.
    "cone3d_256_short": GeometrySpec("cone3d", (256, 256, 256), (1.0, 1.0, 1.0), (480, 620), (1.0, 1.0),
                                     248, 200 * DEG, sid=750.0, sdd=1200.0, n_figures=12),
    # 3D cone-beam 512^3 at 0.5 mm, 360 views over 360 deg, 1024x768 detector at 0.8 mm.
    "cone3d_512": GeometrySpec("cone3d", (512, 512, 512), (0.5, 0.5, 0.5), (768, 1024), (0.8, 0.8),
                               360, 2 * math.pi, sid=750.0, sdd=1200.0, n_figures=12),
    # Centred 32^3 crop of the 512^3 case with a 48x48 central detector window.
    "cone3d_crop32": GeometrySpec("cone3d", (32, 32, 32), (0.5, 0.5, 0.5), (48, 48), (0.8, 0.8),
                                  360, 2 * math.pi, sid=750.0, sdd=1200.0, n_figures=12),
}


def config(name, **overrides):
    spec = CONFIGS[name]
    return spec.with_(**overrides) if overrides else spec
