"""Seeded synthetic inputs for the deferred shading pass.

This module builds *inputs only*: G-buffers and light-space depth maps ray-cast
from seeded sphere scenes, environment cube maps, cameras, lights, and the SSAO
sample kernel and rotation noise.  It contains none of the shading arithmetic
(no BRDF, no SSAO test, no filtering), so it can feed both the FP64 oracle and
the HIP path without coupling them.

The G-buffer stands in for the rasterised geometry pass of the paper (Sec. 4,
Tab. 1): per pixel a linear view depth (``+inf`` for background), a world-space
unit normal, a linear albedo, a roughness and a metalness (Sec. 3).  Shadow maps
are depth renders from each point light "as a normal camera" (Sec. 5.1).  The
paper's scenes (scanned meshes, drone environments) are not available, so seeded
sphere fields stand in for them.

Conventions shared with the shading code are *definitions of the data*:

* pinhole camera, image y down, pixel centres at (x + 0.5, y + 0.5); a view-space
  point at linear depth d of pixel (x, y) is
  ((x + 0.5 - cx) / fx * d, -(y + 0.5 - cy) / fy * d, -d);
* ``world_to_cam`` is a row-major 3x4 rigid transform [R | t];
* cube faces in the order +X, -X, +Y, -Y, +Z, -Z; texel (i, j) of a face of size
  S has s = 2 (i + 0.5) / S - 1, t = 2 (j + 0.5) / S - 1 and points along
  +X (1, -t, -s), -X (-1, -t, s), +Y (s, 1, t), -Y (s, -1, -t), +Z (s, -t, 1),
  -Z (-s, -t, -1); texels are stored as RGBA float (A unused).
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess
from typing import List, Optional

import numpy as np


# ----------------------------------------------------------------------------
# cameras
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Camera:
    world_to_cam: np.ndarray  # (3, 4) float64, rows of [R | t]
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    @property
    def R(self) -> np.ndarray:
        return self.world_to_cam[:, :3]

    @property
    def t(self) -> np.ndarray:
        return self.world_to_cam[:, 3]

    @property
    def position(self) -> np.ndarray:
        return -self.R.T @ self.t

    def as_f32(self) -> "Camera":
        """The same camera with every float rounded to float32 (what the GPU gets)."""
        return Camera(self.world_to_cam.astype(np.float32).astype(np.float64),
                      float(np.float32(self.fx)), float(np.float32(self.fy)),
                      float(np.float32(self.cx)), float(np.float32(self.cy)),
                      self.width, self.height)


def look_at(eye, target, up, vfov_deg: float, width: int, height: int) -> Camera:
    """Camera at ``eye`` looking at ``target``; vertical field of view in degrees."""
    eye = np.asarray(eye, np.float64)
    target = np.asarray(target, np.float64)
    up = np.asarray(up, np.float64)
    f = target - eye
    f /= np.linalg.norm(f)
    x = np.cross(f, up)
    x /= np.linalg.norm(x)
    y = np.cross(x, f)
    R = np.stack([x, y, -f])
    t = -R @ eye
    fy = (height / 2.0) / math.tan(math.radians(vfov_deg) / 2.0)
    # round the intrinsics to float32 once so that every consumer sees the same numbers
    cam = Camera(np.concatenate([R, t[:, None]], axis=1), fy, fy, width / 2.0, height / 2.0,
                 width, height)
    return cam.as_f32()


# ----------------------------------------------------------------------------
# scenes
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class SphereScene:
    centers: np.ndarray      # (n, 3)
    radii: np.ndarray        # (n,)
    albedo: np.ndarray       # (n, 3)
    roughness: np.ndarray    # (n,)
    metalness: np.ndarray    # (n,)
    plane: bool = False      # the plane y = 0
    plane_albedo: tuple = (0.5, 0.5, 0.5)
    plane_roughness: float = 0.6
    plane_metalness: float = 0.0


def make_spheres(rng: np.random.Generator, n: int, plane: bool) -> SphereScene:
    """Spheres drawn in order: centre x, z ~ U[-3, 3] on y = 0, radius ~ U[0.1, 0.5],
    albedo ~ U[0, 1]^3, roughness ~ U[0.05, 1], metalness ~ Bernoulli(0.3)."""
    cx = rng.uniform(-3.0, 3.0, n)
    cz = rng.uniform(-3.0, 3.0, n)
    radii = rng.uniform(0.1, 0.5, n)
    albedo = rng.uniform(0.0, 1.0, (n, 3))
    rough = rng.uniform(0.05, 1.0, n)
    metal = (rng.uniform(0.0, 1.0, n) < 0.3).astype(np.float64)
    centers = np.stack([cx, np.zeros(n), cz], axis=1)
    return SphereScene(centers, radii, albedo, rough, metal, plane)


def _pixel_rays(cam: Camera, xs: np.ndarray, ys: np.ndarray) -> np.ndarray:
    """World-space ray directions scaled so that the view-space z component is -1
    (the ray parameter then equals the linear view depth)."""
    dv = np.stack([(xs + 0.5 - cam.cx) / cam.fx,
                   -(ys + 0.5 - cam.cy) / cam.fy,
                   -np.ones_like(xs, dtype=np.float64)], axis=-1)
    return dv @ cam.R  # == (R^T dv^T)^T


def _sphere_bbox(cam: Camera, c: np.ndarray, r: float):
    """Conservative pixel bounding box of a sphere, or None for the whole image."""
    cv = cam.R @ c + cam.t
    if -(cv[2] + r) <= 1e-3 and -(cv[2] - r) <= 1e-3:
        return (0, 0, 0, 0)  # entirely behind the camera
    if -(cv[2] + r) <= 1e-3:
        return None  # crosses the camera plane
    corners = cv[None, :] + r * np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1)
                                         for sz in (-1, 1)], np.float64)
    z = -corners[:, 2]
    px = cam.cx + cam.fx * corners[:, 0] / z - 0.5
    py = cam.cy - cam.fy * corners[:, 1] / z - 0.5
    x0 = max(int(math.floor(px.min())) - 1, 0)
    x1 = min(int(math.ceil(px.max())) + 2, cam.width)
    y0 = max(int(math.floor(py.min())) - 1, 0)
    y1 = min(int(math.ceil(py.max())) + 2, cam.height)
    return (x0, x1, y0, y1)


def raycast_numpy(scene: SphereScene, cam: Camera, depth_only: bool = False) -> dict:
    """Nearest-hit ray cast of the scene through every pixel of ``cam``.

    Returns float32 planes: ``depth`` (H, W) linear view depth or +inf; unless
    ``depth_only``, also ``normal`` and ``albedo`` (3, H, W) and ``roughness``,
    ``metalness`` (H, W).  Spheres are tested in index order and the plane last;
    an exactly equal hit distance keeps the earlier object.  Slow; the same cast
    as :func:`raycast`, kept as its reference."""
    W, H = cam.width, cam.height
    depth = np.full((H, W), np.inf, np.float64)
    ident = np.full((H, W), -1, np.int32)
    o = cam.position
    n = len(scene.radii)
    for k in range(n):
        c = scene.centers[k]
        r = scene.radii[k]
        bb = _sphere_bbox(cam, c, r)
        if bb is None:
            bb = (0, W, 0, H)
        x0, x1, y0, y1 = bb
        if x1 <= x0 or y1 <= y0:
            continue
        ys, xs = np.meshgrid(np.arange(y0, y1, dtype=np.float64),
                             np.arange(x0, x1, dtype=np.float64), indexing="ij")
        d = _pixel_rays(cam, xs, ys)
        oc = o - c
        a = np.einsum("...i,...i->...", d, d)
        b = d @ oc
        cc = oc @ oc - r * r
        disc = b * b - a * cc
        hit = disc >= 0.0
        tt = np.where(hit, (-b - np.sqrt(np.where(hit, disc, 0.0))) / a, np.inf)
        tt = np.where(tt > 0.0, tt, np.inf)
        sub = depth[y0:y1, x0:x1]
        closer = tt < sub
        sub[closer] = tt[closer]
        ident[y0:y1, x0:x1][closer] = k
    if scene.plane:
        ys, xs = np.meshgrid(np.arange(H, dtype=np.float64), np.arange(W, dtype=np.float64),
                             indexing="ij")
        d = _pixel_rays(cam, xs, ys)
        with np.errstate(divide="ignore", invalid="ignore"):
            tt = np.where(d[..., 1] < 0.0, -o[1] / d[..., 1], np.inf)
        tt = np.where(tt > 0.0, tt, np.inf)
        closer = tt < depth
        depth[closer] = tt[closer]
        ident[closer] = n
    out = {"depth": depth.astype(np.float32)}
    if depth_only:
        return out
    normal = np.zeros((3, H, W), np.float64)
    albedo = np.zeros((3, H, W), np.float64)
    rough = np.zeros((H, W), np.float64)
    metal = np.zeros((H, W), np.float64)
    ys, xs = np.nonzero(ident >= 0)
    ids = ident[ys, xs]
    d = _pixel_rays(cam, xs.astype(np.float64), ys.astype(np.float64))
    p = o[None, :] + depth[ys, xs][:, None] * d
    sph = ids < n
    nrm = np.zeros_like(p)
    nrm[sph] = (p[sph] - scene.centers[ids[sph]]) / scene.radii[ids[sph]][:, None]
    nrm[~sph] = np.array([0.0, 1.0, 0.0])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    alb = np.empty_like(p)
    alb[sph] = scene.albedo[ids[sph]]
    alb[~sph] = np.asarray(scene.plane_albedo)
    rgh = np.where(sph, scene.roughness[np.minimum(ids, n - 1)], scene.plane_roughness)
    mtl = np.where(sph, scene.metalness[np.minimum(ids, n - 1)], scene.plane_metalness)
    normal[:, ys, xs] = nrm.T
    albedo[:, ys, xs] = alb.T
    rough[ys, xs] = rgh
    metal[ys, xs] = mtl
    out.update(normal=normal.astype(np.float32), albedo=albedo.astype(np.float32),
               roughness=rough.astype(np.float32), metalness=metal.astype(np.float32))
    return out


# ----------------------------------------------------------------------------
# the same ray cast in C (OpenMP over rows): fast enough for many large views
# ----------------------------------------------------------------------------
_HERE = os.path.dirname(os.path.abspath(__file__))
_RC_SRC = os.path.join(_HERE, "synth_raycast.c")
_RC_LIB = os.path.join(_HERE, "libsynth.so")
_rc = None


def build_raycaster() -> str:
    subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", _RC_SRC,
                    "-o", _RC_LIB, "-lm"], check=True)
    return _RC_LIB


def _raycaster():
    global _rc
    if _rc is None:
        if not os.path.exists(_RC_LIB) or os.path.getmtime(_RC_LIB) < os.path.getmtime(_RC_SRC):
            build_raycaster()
        lib = ctypes.CDLL(_RC_LIB)
        lib.syn_raycast.restype = None
        _rc = lib
    return _rc


def raycast(scene: SphereScene, cam: Camera, depth_only: bool = False) -> dict:
    """Nearest-hit ray cast of the scene through every pixel of ``cam`` (same
    contract as :func:`raycast_numpy`, computed by the C caster)."""
    W, H = cam.width, cam.height
    n = len(scene.radii)
    bbox = np.zeros((max(n, 1), 4), np.int32)
    for k in range(n):
        bb = _sphere_bbox(cam, scene.centers[k], scene.radii[k])
        bbox[k] = (0, W, 0, H) if bb is None else bb
    f64 = lambda a: np.ascontiguousarray(a, np.float64)
    centers, radii = f64(scene.centers.reshape(-1, 3)), f64(scene.radii)
    alb, rgh, mtl = f64(scene.albedo.reshape(-1, 3)), f64(scene.roughness), f64(scene.metalness)
    R, o = f64(cam.R), f64(cam.position)
    depth = np.empty((H, W), np.float32)
    outs = [None] * 4 if depth_only else [np.empty((3, H, W), np.float32), np.empty((3, H, W), np.float32),
                                          np.empty((H, W), np.float32), np.empty((H, W), np.float32)]
    P = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
    d = ctypes.c_double
    _raycaster().syn_raycast(
        ctypes.c_int(n), P(centers), P(radii), P(alb), P(rgh), P(mtl), ctypes.c_int(1 if scene.plane else 0),
        P(f64(scene.plane_albedo)), d(scene.plane_roughness), d(scene.plane_metalness), P(R), P(o),
        d(cam.fx), d(cam.fy), d(cam.cx), d(cam.cy), ctypes.c_int(W), ctypes.c_int(H), P(bbox), P(depth),
        *[P(a) for a in outs])
    out = {"depth": depth}
    if not depth_only:
        out.update(normal=outs[0], albedo=outs[1], roughness=outs[2], metalness=outs[3])
    return out


# ----------------------------------------------------------------------------
# environment cube maps
# ----------------------------------------------------------------------------
def cube_texel_dirs(S: int) -> np.ndarray:
    """Unnormalised texel-centre directions, shape (6, S, S, 3) indexed [face][j][i]."""
    c = 2.0 * (np.arange(S, dtype=np.float64) + 0.5) / S - 1.0
    t, s = np.meshgrid(c, c, indexing="ij")  # t varies with row j, s with column i
    one = np.ones_like(s)
    faces = [
        np.stack([one, -t, -s], -1),
        np.stack([-one, -t, s], -1),
        np.stack([s, one, t], -1),
        np.stack([s, -one, -t], -1),
        np.stack([s, -t, one], -1),
        np.stack([-s, -t, -one], -1),
    ]
    return np.stack(faces)


def _rgba(rgb: np.ndarray) -> np.ndarray:
    out = np.zeros(rgb.shape[:-1] + (4,), np.float32)
    out[..., :3] = rgb
    return out


def env_sky_gradient(S: int) -> np.ndarray:
    """Procedural sky gradient: zenith (0.25, 0.45, 1.0), horizon white, ground
    (0.3, 0.25, 0.2), blended linearly in the y component of the direction."""
    d = cube_texel_dirs(S)
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    wy = d[..., 1:2]
    cz = np.array([0.25, 0.45, 1.0])
    ch = np.array([1.0, 1.0, 1.0])
    cg = np.array([0.3, 0.25, 0.2])
    rgb = ch + (cz - ch) * np.maximum(wy, 0.0) + (cg - ch) * np.maximum(-wy, 0.0)
    return _rgba(rgb)


def env_sky_sun(S: int, sun_dir=(0.3, 0.8, 0.5), sun_radius_deg: float = 2.0,
                sky_tint=(0.7, 0.85, 1.0), sun_tint=(1.0, 0.95, 0.85)) -> np.ndarray:
    """HDR sky: log10 radiance rising linearly from -2 (nadir) to 2 (zenith), times
    a tint, plus a sun disc of radiance 1e4 (times a tint) around ``sun_dir``."""
    d = cube_texel_dirs(S)
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    wy = d[..., 1:2]
    sky = 10.0 ** (-2.0 + 4.0 * (0.5 + 0.5 * wy)) * np.asarray(sky_tint)
    sd = np.asarray(sun_dir, np.float64)
    sd /= np.linalg.norm(sd)
    in_sun = (d @ sd) >= math.cos(math.radians(sun_radius_deg))
    rgb = np.where(in_sun[..., None], 1e4 * np.asarray(sun_tint), sky)
    return _rgba(rgb)


def env_constant(S: int, value=1.0) -> np.ndarray:
    return _rgba(np.full((6, S, S, 3), value, np.float64))


def env_linear(S: int, c: float, b) -> np.ndarray:
    """Radiance c + b . w (same in all three channels), w the unit texel direction."""
    d = cube_texel_dirs(S)
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    v = c + d @ np.asarray(b, np.float64)
    return _rgba(np.repeat(v[..., None], 3, axis=-1))


# ----------------------------------------------------------------------------
# SSAO sample kernel and rotation noise (random draws of the method, as inputs)
# ----------------------------------------------------------------------------
def ssao_kernel(rng: np.random.Generator, n: int) -> np.ndarray:
    """n tangent-space hemisphere vectors (z > 0), lengths in (0, 1], denser near
    the origin: a uniform length scaled by lerp(0.1, 1, (k / n)^2)."""
    out = np.empty((n, 3), np.float64)
    for k in range(n):
        while True:
            v = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(0, 1)])
            ln = np.linalg.norm(v)
            if 1e-3 < ln <= 1.0 and v[2] > 1e-3:
                break
        v /= ln
        s = k / n
        v *= rng.uniform(0.05, 1.0) * (0.1 + 0.9 * s * s)
        out[k] = v
    return out.astype(np.float32)


def ssao_noise(rng: np.random.Generator) -> np.ndarray:
    """4x4 unit vectors in the view-space xy plane, shape (4, 4, 2) [row][col]."""
    ang = rng.uniform(0.0, 2.0 * math.pi, (4, 4))
    return np.stack([np.cos(ang), np.sin(ang)], -1).astype(np.float32)


# ----------------------------------------------------------------------------
# lights
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Light:
    pos: np.ndarray
    color: np.ndarray
    intensity: float
    shadow_cam: Optional[Camera] = None
    shadow_map: Optional[np.ndarray] = None  # (h, w) float32 linear depth / +inf
    shadow_bias: float = 0.02


# ----------------------------------------------------------------------------
# whole inputs of one view
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class ViewInputs:
    name: str
    cam: Camera
    gbuf: dict
    lights: List[Light]
    env: np.ndarray          # (6, S, S, 4) float32
    ssao_kernel: np.ndarray  # (N, 3) float32
    ssao_noise: np.ndarray   # (4, 4, 2) float32
    ssao_radius: float = 0.5
    ssao_bias: float = 0.025
    blur_tau: float = 0.1
    bloom_threshold: float = 1.0
    bloom_strength: float = 0.04
    exposure: float = 1.0
    gamma: float = 2.2
    tonemap: int = 0         # 0 ACES, 1 Reinhard (Sec. 5.4)
    ibl: dict = dataclasses.field(default_factory=lambda: dict(
        irr_size=32, irr_src_size=64, pref_size=128, pref_levels=5, pref_samples=1024,
        lut_size=256, lut_samples=1024))
    scene: int = -1          # index of the shared scene (many-view workloads)

    @property
    def width(self) -> int:
        return self.cam.width

    @property
    def height(self) -> int:
        return self.cam.height


def _f32(x) -> float:
    return float(np.float32(x))


def make_view(name: str, width: int, height: int, n_spheres: int, plane: bool, seed: int,
              n_lights: int, shadow_size: int, env_size: int, env_kind: str, ssao_n: int,
              ibl: Optional[dict] = None, eye=(0.0, 3.5, 8.5), up=(0.0, 1.0, 0.0)) -> ViewInputs:
    """One seeded view.  ``n_lights == 1`` puts a white light of intensity 40 at
    (3, 5, 4); otherwise the first four lights are white and sit at azimuth
    45 + 90 k degrees, radius 6, height 6, and lights 4 .. 7 (up to the
    C ABI's eight) on a lower ring at azimuth 90 (k - 4) degrees, radius 4.5,
    height 3.5, each with its own tint (so that every colour channel of the
    light radiance differs).  ``shadow_size > 0`` renders a square depth map
    per light with a 90 degree camera looking at the origin.  The view's
    camera looks at the origin from ``eye`` with the given ``up`` direction.

    Under the HDR sky-and-sun environment (sky radiance up to 1e2, sun 1e4) the
    lights get intensity 1500 (about the sky's irradiance at the scene) and the
    exposure is 0.012, which maps the median shaded radiance (about 24) to the
    middle of the ACES curve; with exposure 1 that sky saturates every pixel."""
    rng = np.random.default_rng(seed)
    scene = make_spheres(rng, n_spheres, plane)
    cam = look_at(eye, (0.0, 0.0, 0.0), up, 45.0, width, height)
    gbuf = raycast(scene, cam)
    lights = []
    tints = [(1.0, 0.6, 0.3), (0.3, 0.8, 1.0), (0.9, 1.0, 0.4), (0.6, 0.4, 1.0)]
    if n_lights == 1:
        positions = [np.array([3.0, 5.0, 4.0])]
        colours = [(1.0, 1.0, 1.0)]
    else:
        positions = [np.array([6.0 * math.cos(math.radians(45 + 90 * k)), 6.0,
                               6.0 * math.sin(math.radians(45 + 90 * k))]) if k < 4 else
                     np.array([4.5 * math.cos(math.radians(90 * (k - 4))), 3.5,
                               4.5 * math.sin(math.radians(90 * (k - 4)))])
                     for k in range(n_lights)]
        colours = [(1.0, 1.0, 1.0) if k < 4 else tints[(k - 4) % 4] for k in range(n_lights)]
    for p, col in zip(positions, colours):
        p = p.astype(np.float32).astype(np.float64)
        light = Light(p, np.array(col), 1500.0 if env_kind == "sun" else 40.0)
        if shadow_size > 0:
            lc = look_at(p, (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 90.0, shadow_size, shadow_size)
            light.shadow_cam = lc
            light.shadow_map = raycast(scene, lc, depth_only=True)["depth"]
        lights.append(light)
    if env_kind == "gradient":
        env = env_sky_gradient(env_size)
    elif env_kind == "sun":
        env = env_sky_sun(env_size)
    elif env_kind == "white":
        env = env_constant(env_size, 1.0)
    else:
        raise ValueError(env_kind)
    krng = np.random.default_rng(seed + 10000)
    kern = ssao_kernel(krng, ssao_n)
    noise = ssao_noise(krng)
    v = ViewInputs(name, cam, gbuf, lights, env, kern, noise)
    if env_kind == "sun":
        v.exposure = 0.012
    if ibl is not None:
        v.ibl = dict(v.ibl, **ibl)
    return v


def config_small(seed: int = 1) -> ViewInputs:
    """256x256 single view: 64 spheres, no plane, one light without shadows, a
    6x64x64 sky-gradient cube, SSAO with 16 samples of radius 0.5."""
    return make_view("plain-256x256", 256, 256, 64, False, seed, 1, 0, 64, "gradient", 16)


def config_1080p(seed: int = 2) -> ViewInputs:
    """1920x1080 single view: 512 spheres plus the plane, four lights each with a
    2048x2048 depth map, SSAO with 64 samples, a 6x512x512 HDR sky-and-sun cube."""
    return make_view("plain-1920x1080", 1920, 1080, 512, True, seed, 4, 2048, 512, "sun", 64)


def config_reduced(width: int, height: int, seed: int = 5, shadow_size: int = 256,
                   env_size: int = 32, ssao_n: int = 16, n_spheres: int = 48,
                   n_lights: int = 4, eye=(0.0, 3.5, 8.5), up=(0.0, 1.0, 0.0)) -> ViewInputs:
    """A reduced copy of the 1080p workload (plane, shadowed lights, sun sky) at a
    size the FP64 oracle finishes in seconds; used for parity tests."""
    base = min(128, env_size)
    ibl = dict(irr_src_size=min(64, env_size), pref_size=base, pref_samples=256,
               pref_levels=min(5, base.bit_length() - 1), lut_size=32, lut_samples=256)
    return make_view(f"reduced-{width}x{height}", width, height, n_spheres, True, seed, n_lights,
                     shadow_size, env_size, "sun", ssao_n, ibl, eye, up)


# ----------------------------------------------------------------------------
# many views of many scenes (the batched and serving workloads)
# ----------------------------------------------------------------------------
BATCH_RESOLUTIONS = ((320, 240), (640, 480), (1280, 720), (1920, 1080))
SERVING_RESOLUTIONS = ((256, 256), (640, 480), (1920, 1080), (3840, 2160))


@dataclasses.dataclass
class SceneInputs:
    """A scene shared by many views: spheres on the plane, one white light at
    (3, 5, 4) without a depth map, its own HDR sky-and-sun cube (seeded sun
    direction and tints), and the SSAO kernel and noise of its views."""
    seed: int
    spheres: SphereScene
    env: np.ndarray
    light: Light
    ssao_kernel: np.ndarray
    ssao_noise: np.ndarray
    ibl: dict


@dataclasses.dataclass
class ViewSpec:
    scene: int
    cam: Camera


def make_scene(seed: int, env_size: int = 256, ssao_n: int = 16, sphere_range=(64, 1024),
               ibl: Optional[dict] = None) -> SceneInputs:
    """Sphere count ~ U{lo..hi}; sun azimuth ~ U[0, 360), elevation ~ U[20, 70]
    degrees; sky tint ~ U[0.6, 1]^3, sun tint ~ U[0.85, 1]^3."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(sphere_range[0], sphere_range[1] + 1))
    spheres = make_spheres(rng, n, True)
    az = rng.uniform(0.0, 2.0 * math.pi)
    el = math.radians(rng.uniform(20.0, 70.0))
    sun = (math.cos(el) * math.cos(az), math.sin(el), math.cos(el) * math.sin(az))
    env = env_sky_sun(env_size, sun_dir=sun, sky_tint=tuple(rng.uniform(0.6, 1.0, 3)),
                      sun_tint=tuple(rng.uniform(0.85, 1.0, 3)))
    light = Light(np.array([3.0, 5.0, 4.0]), np.array([1.0, 1.0, 1.0]), 1500.0)
    krng = np.random.default_rng(seed + 10000)
    kern = ssao_kernel(krng, ssao_n)
    noise = ssao_noise(krng)
    base = min(128, env_size)
    p = dict(irr_size=32, irr_src_size=min(64, env_size), pref_size=base,
             pref_levels=min(5, base.bit_length() - 1), pref_samples=1024, lut_size=256, lut_samples=1024)
    if ibl is not None:
        p.update(ibl)
    return SceneInputs(seed, spheres, env, light, kern, noise, p)


def orbit_camera(rng: np.random.Generator, width: int, height: int) -> Camera:
    """Camera looking at the origin from azimuth ~ U[0, 360), elevation ~
    U[15, 45] degrees and distance ~ U[7, 10], vertical field of view 45."""
    az = rng.uniform(0.0, 2.0 * math.pi)
    el = math.radians(rng.uniform(15.0, 45.0))
    dist = rng.uniform(7.0, 10.0)
    eye = (dist * math.cos(el) * math.cos(az), dist * math.sin(el), dist * math.cos(el) * math.sin(az))
    return look_at(eye, (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 45.0, width, height)


def view_specs(n_scenes: int, n_views: int, seed: int, resolutions=BATCH_RESOLUTIONS) -> List[ViewSpec]:
    """View k draws its scene ~ U{n_scenes}, its resolution ~ U(resolutions) and an
    orbit camera, in that order."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_views):
        s = int(rng.integers(0, n_scenes))
        w, h = resolutions[int(rng.integers(0, len(resolutions)))]
        out.append(ViewSpec(s, orbit_camera(rng, w, h)))
    return out


def scene_view(scene: SceneInputs, cam: Camera, name: str, gbuf: Optional[dict] = None,
               index: int = -1) -> ViewInputs:
    """The inputs of one view of a shared scene (the cube map is shared, not copied)."""
    if gbuf is None:
        gbuf = raycast(scene.spheres, cam)
    v = ViewInputs(name, cam, gbuf, [scene.light], scene.env, scene.ssao_kernel, scene.ssao_noise,
                   scene=index)
    v.exposure = 0.012
    v.ibl = dict(scene.ibl)
    return v


def config_batch(n_scenes: int = 16, n_views: int = 256, scene_seed: int = 100, view_seed: int = 200,
                 resolutions=BATCH_RESOLUTIONS, env_size: int = 256, ssao_n: int = 16,
                 sphere_range=(64, 1024), ibl: Optional[dict] = None):
    """Many views of uneven resolution over shared scenes: scenes from seeds
    scene_seed + i, views from view_seed.  Returns (scenes, views)."""
    scenes = [make_scene(scene_seed + i, env_size, ssao_n, sphere_range, ibl) for i in range(n_scenes)]
    specs = view_specs(n_scenes, n_views, view_seed, resolutions)
    gbufs = [raycast(scenes[s.scene].spheres, s.cam) for s in specs]
    views = [scene_view(scenes[s.scene], s.cam, f"view{k}-scene{s.scene}-{s.cam.width}x{s.cam.height}", g,
                        s.scene) for k, (s, g) in enumerate(zip(specs, gbufs))]
    return scenes, views


def config_batch_small(seed: int = 40):
    """A reduced batch for parity tests: 3 scenes with 16 - 48 spheres and 16^2
    cubes, 12 views of ragged sizes."""
    return config_batch(3, 12, scene_seed=seed, view_seed=seed + 1,
                        resolutions=((64, 48), (33, 17), (130, 70), (5, 3)), env_size=16,
                        sphere_range=(16, 48), ibl=dict(pref_samples=128, lut_size=32, lut_samples=128))


# ----------------------------------------------------------------------------
# surfel-splatted G-buffers (accumulated attributes and weights)
# ----------------------------------------------------------------------------
def surfel_accumulate(view: ViewInputs, seed: int, max_surfels: int = 4, jitter: float = 0.05) -> ViewInputs:
    """The view's G-buffer as surfel splatting would leave it: on every surface
    pixel k ~ U{1..max_surfels} overlapping surfels with splat weights u ~
    U[0.25, 1] each add u times their own attributes (the pixel's albedo,
    roughness and metalness scaled by U[1 - jitter, 1 + jitter] and clamped to
    their ranges, the normal tilted by the same amount) to the accumulated
    planes, and u to the weight plane.  Background pixels keep weight 0 and zero
    attributes; depth is unchanged."""
    import copy
    rng = np.random.default_rng(seed)
    g = view.gbuf
    H, W = g["depth"].shape
    fg = np.isfinite(g["depth"])
    k = rng.integers(1, max_surfels + 1, (H, W))
    wsum = np.zeros((H, W))
    nsum = np.zeros((3, H, W))
    asum = np.zeros((3, H, W))
    rsum = np.zeros((H, W))
    msum = np.zeros((H, W))
    for s in range(max_surfels):
        on = fg & (k > s)
        u = rng.uniform(0.25, 1.0, (H, W)) * on
        jit = lambda shape: rng.uniform(1.0 - jitter, 1.0 + jitter, shape)
        nsum += u * (g["normal"] + rng.uniform(-jitter, jitter, (3, H, W)))
        asum += u * np.clip(g["albedo"] * jit((3, H, W)), 0.0, 1.0)
        rsum += u * np.clip(g["roughness"] * jit((H, W)), 0.05, 1.0)
        msum += u * np.clip(g["metalness"] * jit((H, W)), 0.0, 1.0)
        wsum += u
    out = copy.copy(view)
    out.name = view.name + "-surfels"
    f32 = lambda a: np.where(fg, a, 0.0).astype(np.float32)
    out.gbuf = dict(depth=g["depth"], normal=f32(nsum), albedo=f32(asum), roughness=f32(rsum),
                    metalness=f32(msum), weight=f32(wsum))
    return out


# ----------------------------------------------------------------------------
# point clouds (the depth-only renders eye-dome lighting composes)
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class PointCloudView:
    name: str
    cam: Camera
    depth: np.ndarray   # (H, W) float32 linear view depth of the nearest point, +inf = none
    color: np.ndarray   # (3, H, W) float32 colour of that point (0 where none)
    env: np.ndarray     # background cube (6, S, S, 4)
    ao: np.ndarray      # (Hh, Wh) float32 ambient occlusion in [0.3, 1] (smooth noise)
    edl_radius: int = 2
    edl_dirs: int = 8
    edl_strength: float = 8.0
    edl_far: float = 1000.0


def point_cloud_view(width: int, height: int, n_points: int, seed: int, n_spheres: int = 512,
                     env_size: int = 64, ground: float = 8.0) -> PointCloudView:
    """A seeded point cloud sampled from a sphere field and its ground patch,
    rendered as one-pixel points with a depth test (the nearest point of a pixel
    wins, an equal depth the lower index): points uniform by area over the sphere
    surfaces and the square [-ground, ground]^2 of the plane y = 0, coloured by their
    object's albedo, seen by the 1080p workload's camera.  Sparse clouds leave
    holes (background) and let far surfaces show through, which is what the
    eye-dome shading has to make legible."""
    rng = np.random.default_rng(seed)
    scene = make_spheres(rng, n_spheres, True)
    cam = look_at((0.0, 3.5, 8.5), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 45.0, width, height)
    areas = np.concatenate([4.0 * math.pi * scene.radii ** 2, [(2.0 * ground) ** 2]])
    obj = rng.choice(len(areas), size=n_points, p=areas / areas.sum())
    on_plane = obj == n_spheres
    u = rng.normal(size=(n_points, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    sph = np.minimum(obj, n_spheres - 1)
    pts = scene.centers[sph] + scene.radii[sph, None] * u
    pts[on_plane] = np.stack([rng.uniform(-ground, ground, on_plane.sum()), np.zeros(on_plane.sum()),
                              rng.uniform(-ground, ground, on_plane.sum())], 1)
    col = np.where(on_plane[:, None], np.asarray(scene.plane_albedo)[None, :], scene.albedo[sph])
    pv = pts @ cam.R.T + cam.t
    d = -pv[:, 2]
    ok = d > 1e-6
    px = np.floor(cam.cx + cam.fx * pv[:, 0] / np.where(ok, d, 1.0)).astype(np.int64)
    py = np.floor(cam.cy - cam.fy * pv[:, 1] / np.where(ok, d, 1.0)).astype(np.int64)
    ok &= (px >= 0) & (px < width) & (py >= 0) & (py < height)
    idx = np.nonzero(ok)[0]
    pix = py[idx] * width + px[idx]
    d32 = d[idx].astype(np.float32)
    # depth test: positive float32 bit patterns order like the values, so the
    # smallest (depth bits, point index) key of a pixel is its nearest point
    key = (d32.view(np.uint32).astype(np.uint64) << np.uint64(32)) | idx.astype(np.uint64)
    zbuf = np.full(width * height, np.iinfo(np.uint64).max, np.uint64)
    np.minimum.at(zbuf, pix, key)
    hit = zbuf != np.iinfo(np.uint64).max
    win = (zbuf[hit] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    depth = np.full(width * height, np.inf, np.float32)
    color = np.zeros((3, width * height), np.float32)
    depth[hit] = d[win].astype(np.float32)
    color[:, hit] = col[win].T.astype(np.float32)
    Wh, Hh = (width + 1) // 2, (height + 1) // 2
    yy, xx = np.mgrid[0:Hh, 0:Wh]
    ao = (0.65 + 0.35 * np.sin(0.21 * xx + 0.5 * rng.uniform()) * np.cos(0.17 * yy)).astype(np.float32)
    return PointCloudView(f"points-{width}x{height}-{n_points}", cam, depth.reshape(height, width),
                          color.reshape(3, height, width), env_sky_gradient(env_size), ao)
