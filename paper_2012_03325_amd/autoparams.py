"""Automatic rendering parameters (paper Sec. 6): an educated guess of the
camera, the light rig and the SSAO radius from the scene's extent alone, so
that any scene renders sensibly whatever its unit system.

Host logic only (no kernels); the results feed the C-ABI calls like any
hand-set parameters.  The paper states the rules and leaves their constants
open; the readings taken here:

* scene scale: the diameter of the bounding sphere of the scene's objects
  (centre = centre of the axis-aligned bounding box, radius = the farthest
  object extent from it);
* SSAO radius: 5 % of that scale (the paper's default);
* camera: on the given viewing direction, at the distance where the bounding
  sphere just fits the vertical and horizontal fields of view, looking at the
  centre;
* three-point lights: a key light (most of the light), a fill light softening
  its shadows and a rim light behind the object, at camera-relative azimuth /
  elevation (+45, 45), (-60, 15) and (180, 60) degrees, each at 3 bounding
  radii from the centre, with intensity set so that the radiance arriving at
  the centre (colour x intensity / d^2) is the predefined value: 1, 0.35 and
  0.6 of ``radiance``.  Scaling the scene by s scales every distance by s and
  leaves the radiance at the object unchanged.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

from . import synth

SSAO_RADIUS_FRACTION = 0.05
RIG = (  # name, azimuth (deg, from the camera's side of the object), elevation (deg), share of the radiance
    ("key", 45.0, 45.0, 1.0),
    ("fill", -60.0, 15.0, 0.35),
    ("rim", 180.0, 60.0, 0.6),
)
RIG_DISTANCE_RADII = 3.0


@dataclasses.dataclass
class Bounds:
    center: np.ndarray  # (3,)
    radius: float

    @property
    def scale(self) -> float:
        return 2.0 * self.radius


def sphere_bounds(spheres: synth.SphereScene) -> Bounds:
    """Bounding sphere of a sphere field (the ground plane is unbounded and does
    not count)."""
    c = np.asarray(spheres.centers, np.float64).reshape(-1, 3)
    r = np.asarray(spheres.radii, np.float64).reshape(-1)
    if len(r) == 0:
        return Bounds(np.zeros(3), 1.0)
    lo, hi = (c - r[:, None]).min(0), (c + r[:, None]).max(0)
    centre = 0.5 * (lo + hi)
    radius = float((np.linalg.norm(c - centre, axis=1) + r).max())
    return Bounds(centre, radius)


def point_bounds(points) -> Bounds:
    p = np.asarray(points, np.float64).reshape(-1, 3)
    lo, hi = p.min(0), p.max(0)
    centre = 0.5 * (lo + hi)
    return Bounds(centre, float(np.linalg.norm(p - centre, axis=1).max()))


def ssao_radius(b: Bounds) -> float:
    return SSAO_RADIUS_FRACTION * b.scale


def fit_camera(b: Bounds, direction, width: int, height: int, vfov_deg: float = 45.0,
               up=(0.0, 1.0, 0.0)) -> synth.Camera:
    """Camera looking at the bounds' centre from ``direction`` (pointing from
    the centre towards the camera) at the distance where the bounding sphere
    fits both fields of view."""
    d = np.asarray(direction, np.float64)
    d = d / np.linalg.norm(d)
    half_v = math.radians(vfov_deg) / 2.0
    half_h = math.atan(math.tan(half_v) * width / height)
    dist = b.radius / math.sin(min(half_v, half_h))
    return synth.look_at(b.center + dist * d, b.center, up, vfov_deg, width, height)


def three_point_lights(b: Bounds, cam: synth.Camera, radiance: float = 1.0) -> List[synth.Light]:
    """Key, fill and rim lights around the bounds, placed relative to the
    camera's horizontal viewing direction; each delivers its share of
    ``radiance`` at the centre."""
    to_cam = cam.position - b.center
    az0 = math.atan2(to_cam[2], to_cam[0])
    dist = RIG_DISTANCE_RADII * b.radius
    lights = []
    for _name, az, el, share in RIG:
        a = az0 + math.radians(az)
        e = math.radians(el)
        pos = b.center + dist * np.array([math.cos(e) * math.cos(a), math.sin(e), math.cos(e) * math.sin(a)])
        pos = pos.astype(np.float32).astype(np.float64)
        d2 = float(np.sum((pos - b.center) ** 2))
        lights.append(synth.Light(pos, np.array([1.0, 1.0, 1.0]), share * radiance * d2))
    return lights


def rig_names() -> Tuple[str, ...]:
    return tuple(r[0] for r in RIG)
