"""ctypes front-end of the FP64 CPU oracle (``epb_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline of the benchmark.  The product package never imports this module.

Every function takes the same float32 arrays the GPU path receives (or float64
intermediates), widens them to float64 and calls the C oracle.  Functions that
involve floating-point decisions return a pair ``(lo, hi)``: the smallest and
largest result over the outcomes of every decision within the tie margin.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import List, NamedTuple, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "epb_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

class Tie(NamedTuple):
    """Half-widths of the ambiguous bands of the float decisions, each as a
    fraction of its decision's magnitude scale S (defined in epb_oracle.h): an
    operand within ``field * S`` of its threshold counts as a tie."""
    ssao_coord: float
    ssao_depth: float
    pcf_coord: float
    pcf_depth: float
    face: float


ULP32 = 2.0 ** -24  # unit roundoff of float32
# A float32 implementation's operand error is a few units of 2^-24 S (one per
# rounding on the operand's chain, S the decision's magnitude scale of
# epb_oracle.h).  Bands: 16 units for the SSAO coordinate (its S carries the
# final rounding of the sum twice), 8 for the SSAO depth test, 4 for the
# light-map coordinate and depth, and 1e-5 of the largest component for
# cube-face choices (directions of GPU sine and cosine evaluations).
DEFAULT_TIE = Tie(16 * ULP32, 8 * ULP32, 4 * ULP32, 4 * ULP32, 1e-5)
EXACT = Tie(0.0, 0.0, 0.0, 0.0, 0.0)  # every decision taken once, in float64


def build(src: str = _SRC, out: str = _LIB_PATH) -> str:
    """Compile the oracle with gcc (IEEE double, no fast-math, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas", "-I", _HERE, "-o", out + ".tmp", src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


_lib = None


class OrcCamera(C.Structure):
    _fields_ = [("world_to_cam", C.c_double * 12), ("fx", C.c_double), ("fy", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("width", C.c_int32),
                ("height", C.c_int32)]


class OrcTie(C.Structure):
    _fields_ = [(k, C.c_double) for k in Tie._fields]


class OrcLight(C.Structure):
    _fields_ = [("pos", C.c_double * 3), ("color", C.c_double * 3), ("intensity", C.c_double),
                ("shadow_map", C.POINTER(C.c_double)), ("shadow_cam", OrcCamera),
                ("shadow_bias", C.c_double)]


_D = C.POINTER(C.c_double)


class OrcScene(C.Structure):
    _fields_ = [("n", C.c_int32), ("center", _D), ("radius", _D), ("albedo", _D), ("rough", _D),
                ("metal", _D), ("plane", C.c_int32), ("plane_albedo", C.c_double * 3),
                ("plane_rough", C.c_double), ("plane_metal", C.c_double)]



def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        _lib = load(_LIB_PATH)
    return _lib


def load(path: str):
    """Load a build of the oracle's C source and declare its signatures."""
    L = C.CDLL(path)
    L.orc_cube_texel_dir.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _D]
    L.orc_texel_solid_angle.argtypes = [C.c_int, C.c_int, C.c_int]
    L.orc_texel_solid_angle.restype = C.c_double
    L.orc_ggx_D.argtypes = [C.c_double, C.c_double]
    L.orc_ggx_D.restype = C.c_double
    L.orc_brdf_lut_point.argtypes = [C.c_double, C.c_double, C.c_int, _D]
    L.orc_aces.argtypes = [C.c_double]
    L.orc_aces.restype = C.c_double
    L.orc_encode_u8.argtypes = [C.c_double, C.c_double, C.c_double]
    L.orc_encode_u8.restype = C.c_int
    L.orc_reinhard.argtypes = [C.c_double]
    L.orc_reinhard.restype = C.c_double
    L.orc_encode_u8_op.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int]
    L.orc_encode_u8_op.restype = C.c_int
    L.orc_env_downsample.argtypes = [_D, C.c_int, _D]
    L.orc_irradiance.argtypes = [_D, C.c_int, _D, C.c_int]
    L.orc_prefilter.argtypes = [_D, C.c_int, _D, _D, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int]
    L.orc_brdf_lut.argtypes = [_D, C.c_int, C.c_int]
    L.orc_ssao_raw.argtypes = [_D, _D, C.POINTER(OrcCamera), _D, C.c_int, _D, C.c_double,
                               C.c_double, C.POINTER(OrcTie), _D, _D]
    L.orc_ssao_blur.argtypes = [_D, _D, _D, C.c_int, C.c_int, C.c_double, _D, _D]
    L.orc_shade.argtypes = [_D, _D, _D, _D, _D, C.POINTER(OrcCamera), _D, _D,
                            C.POINTER(OrcLight), C.c_int, _D, C.c_int, _D, _D, C.c_int, C.c_int,
                            _D, C.c_int, _D, C.c_int, C.POINTER(OrcTie), _D, _D]
    L.orc_normalize_gbuffer.argtypes = [_D, C.c_int, C.c_int, _D, _D, _D, _D]
    L.orc_raycast.argtypes = [C.POINTER(OrcScene), C.POINTER(OrcCamera), C.c_double, _D,
                              C.POINTER(C.c_int32), _D, _D, _D, _D, C.POINTER(C.c_uint8)]
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_edl_offsets.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.orc_edl.argtypes = [_D, _D, C.POINTER(OrcCamera), _D, _D, C.c_int, C.c_int, C.c_double,
                          C.c_double, _D, C.c_int, C.c_double, _D, _D]
    L.orc_bloom_tonemap.argtypes = [_D, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                    C.c_double, C.c_double, C.c_int, C.POINTER(C.c_uint8), _D, _D]
    return L


def _d(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _cam(cam) -> OrcCamera:
    c = OrcCamera()
    for k, v in enumerate(np.asarray(cam.world_to_cam, np.float64).reshape(-1)):
        c.world_to_cam[k] = float(v)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height = int(cam.width), int(cam.height)
    return c


def _tie(tie) -> OrcTie:
    return OrcTie(*Tie(*tie))


# ---------------------------------------------------------------------------
# building blocks
# ---------------------------------------------------------------------------
def cube_texel_dir(face: int, i: int, j: int, S: int) -> np.ndarray:
    d = np.zeros(3)
    lib().orc_cube_texel_dir(face, i, j, S, _p(d))
    return d


def texel_solid_angle(i: int, j: int, S: int) -> float:
    return lib().orc_texel_solid_angle(i, j, S)


def ggx_D(NoH: float, alpha: float) -> float:
    return lib().orc_ggx_D(NoH, alpha)


def brdf_lut_point(NoV: float, rough: float, samples: int = 1024) -> Tuple[float, float]:
    ab = np.zeros(2)
    lib().orc_brdf_lut_point(NoV, rough, samples, _p(ab))
    return float(ab[0]), float(ab[1])


def aces(x: float) -> float:
    return lib().orc_aces(x)


def encode_u8(x: float, exposure: float = 1.0, gamma: float = 2.2, tonemap: int = 0) -> int:
    if tonemap:
        return lib().orc_encode_u8_op(x, exposure, gamma, tonemap)
    return lib().orc_encode_u8(x, exposure, gamma)


def reinhard(x: float) -> float:
    return lib().orc_reinhard(x)


# ---------------------------------------------------------------------------
# a1: image-based-lighting precompute
# ---------------------------------------------------------------------------
def env_downsample(src) -> np.ndarray:
    src = _d(src)
    S = src.shape[1]
    out = np.zeros((6, S // 2, S // 2, 4))
    lib().orc_env_downsample(_p(src), S, _p(out))
    return out


def irradiance_source(env, size: int) -> np.ndarray:
    """Repeated solid-angle-weighted 2x2 means down to ``min(S, size)``."""
    src = _d(env)
    while src.shape[1] > size:
        src = env_downsample(src)
    return src


def irradiance(src, out_size: int) -> np.ndarray:
    src = _d(src)
    out = np.zeros((6, out_size, out_size, 4))
    lib().orc_irradiance(_p(src), src.shape[1], _p(out), out_size)
    return out


def prefilter(env, base: int, levels: int, samples: int, tie=DEFAULT_TIE,
              with_hi: bool = False, fis: bool = False):
    """Prefiltered chain as a list of (6, s, s, 4) levels; with ``with_hi`` also
    the upper ends of the face-tie intervals; ``fis`` reads each sample from the
    environment's mip chain at the level its pdf asks for."""
    env = _d(env)
    assert not fis or (env.shape[1] & (env.shape[1] - 1)) == 0, "filtered importance sampling needs a power-of-two size"
    total = sum(6 * (base >> m) ** 2 * 4 for m in range(levels))
    lo = np.zeros(total)
    hi = np.zeros(total)
    lib().orc_prefilter(_p(env), env.shape[1], _p(lo), _p(hi), base, levels, samples, Tie(*tie).face,
                       1 if fis else 0)

    def split(out):
        res, off = [], 0
        for m in range(levels):
            s = base >> m
            n = 6 * s * s * 4
            res.append(out[off:off + n].reshape(6, s, s, 4))
            off += n
        return res

    return (split(lo), split(hi)) if with_hi else split(lo)


def brdf_lut(size: int, samples: int) -> np.ndarray:
    out = np.zeros((size, size, 2))
    lib().orc_brdf_lut(_p(out), size, samples)
    return out


def precompute_ibl(env, irr_size=32, irr_src_size=64, pref_size=128, pref_levels=5,
                   pref_samples=1024, lut_size=256, lut_samples=1024, pref_fis=0, **_unused) -> dict:
    """The whole per-environment precompute (Sec. 3.1)."""
    env = _d(env)
    S = env.shape[1]
    src = irradiance_source(env, min(S, irr_src_size))
    base = min(S, pref_size)
    plo, phi = prefilter(env, base, pref_levels, pref_samples, with_hi=True, fis=bool(pref_fis))
    return dict(irradiance=irradiance(src, irr_size), prefiltered=plo, prefiltered_hi=phi,
                lut=brdf_lut(lut_size, lut_samples))


# ---------------------------------------------------------------------------
# a2 / a3: SSAO
# ---------------------------------------------------------------------------
def ssao_raw(depth, normal, cam, kernel, noise, radius=0.5, bias=0.025,
             tie=DEFAULT_TIE) -> Tuple[np.ndarray, np.ndarray]:
    depth, normal, kernel, noise = _d(depth), _d(normal), _d(kernel), _d(noise)
    H, W = depth.shape
    Wh, Hh = (W + 1) // 2, (H + 1) // 2
    lo = np.zeros((Hh, Wh))
    hi = np.zeros((Hh, Wh))
    c, t = _cam(cam), _tie(tie)
    lib().orc_ssao_raw(_p(depth), _p(normal), C.byref(c), _p(kernel), kernel.shape[0], _p(noise),
                       radius, bias, C.byref(t), _p(lo), _p(hi))
    return lo, hi


def ssao_blur(raw_lo, raw_hi, depth, tau=0.1) -> Tuple[np.ndarray, np.ndarray]:
    raw_lo, raw_hi, depth = _d(raw_lo), _d(raw_hi), _d(depth)
    H, W = depth.shape
    lo = np.zeros_like(raw_lo)
    hi = np.zeros_like(raw_hi)
    lib().orc_ssao_blur(_p(raw_lo), _p(raw_hi), _p(depth), W, H, tau, _p(lo), _p(hi))
    return lo, hi


# ---------------------------------------------------------------------------
# a4: shading
# ---------------------------------------------------------------------------
RAY_TIE_REL = 1e-9


def raycast(scene, cam, attributes: bool = True, rel: float = RAY_TIE_REL) -> dict:
    """Nearest-hit ray cast of a sphere field (and the plane y = 0) through every
    pixel of ``cam`` in float64 (the step the GPU ray caster performs).  ``scene``
    has centers (n, 3), radii, albedo (n, 3), roughness, metalness, plane and the
    plane material.  Returns depth, id, ambiguous and, with ``attributes``, the
    normal, albedo, roughness and metalness planes."""
    n = len(scene.radii)
    cen, rad = _d(np.asarray(scene.centers).reshape(-1, 3)), _d(scene.radii)
    alb, rgh, mtl = _d(np.asarray(scene.albedo).reshape(-1, 3)), _d(scene.roughness), _d(scene.metalness)
    sc = OrcScene()
    sc.n = n
    sc.center, sc.radius, sc.albedo, sc.rough, sc.metal = _p(cen), _p(rad), _p(alb), _p(rgh), _p(mtl)
    sc.plane = 1 if scene.plane else 0
    for c in range(3):
        sc.plane_albedo[c] = float(scene.plane_albedo[c])
    sc.plane_rough, sc.plane_metal = float(scene.plane_roughness), float(scene.plane_metalness)
    W, H = cam.width, cam.height
    depth = np.empty((H, W))
    ids = np.empty((H, W), np.int32)
    amb = np.empty((H, W), np.uint8)
    out = dict(depth=depth, id=ids, ambiguous=amb)
    if attributes:
        out.update(normal=np.empty((3, H, W)), albedo=np.empty((3, H, W)), roughness=np.empty((H, W)),
                   metalness=np.empty((H, W)))
    P = lambda k: _p(out[k]) if attributes else C.cast(None, _D)
    lib().orc_raycast(C.byref(sc), C.byref(_cam(cam)), rel, _p(depth), ids.ctypes.data_as(C.POINTER(C.c_int32)),
                      P("normal"), P("albedo"), P("roughness"), P("metalness"),
                      amb.ctypes.data_as(C.POINTER(C.c_uint8)))
    return out


def normalize_gbuffer(weight, normal, albedo, rough, metal) -> None:
    """Surfel G-buffer normalisation (Sec. 4.4), in place on float64 arrays."""
    w = _d(weight)
    H, W = w.shape
    for a in (normal, albedo, rough, metal):
        assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    lib().orc_normalize_gbuffer(_p(w), W, H, _p(normal), _p(albedo), _p(rough), _p(metal))


def shade(gbuf: dict, cam, ao_lo, ao_hi, lights: Sequence, ibl: dict, env,
          tie=DEFAULT_TIE) -> Tuple[np.ndarray, np.ndarray]:
    depth, normal, albedo = _d(gbuf["depth"]), _d(gbuf["normal"]), _d(gbuf["albedo"])
    rough, metal = _d(gbuf["roughness"]), _d(gbuf["metalness"])
    ao_lo, ao_hi = _d(ao_lo), _d(ao_hi)
    H, W = depth.shape
    if gbuf.get("weight") is not None:  # surfel G-buffer: normalise first (copies: in place)
        normal, albedo, rough, metal = (np.array(a, np.float64) for a in (normal, albedo, rough, metal))
        normalize_gbuffer(gbuf["weight"], normal, albedo, rough, metal)
    keep = []
    arr = (OrcLight * max(1, len(lights)))()
    for k, L in enumerate(lights):
        o = arr[k]
        for c in range(3):
            o.pos[c] = float(L.pos[c])
            o.color[c] = float(L.color[c])
        o.intensity = float(L.intensity)
        if L.shadow_map is not None:
            sm = _d(L.shadow_map)
            keep.append(sm)
            o.shadow_map = _p(sm)
            o.shadow_cam = _cam(L.shadow_cam)
            o.shadow_bias = float(L.shadow_bias)
        else:
            o.shadow_map = C.cast(None, _D)
    irr = _d(ibl["irradiance"])
    pref = _d(np.concatenate([np.asarray(m, np.float64).reshape(-1) for m in ibl["prefiltered"]]))
    pref_hi = _d(np.concatenate([np.asarray(m, np.float64).reshape(-1)
                                 for m in ibl.get("prefiltered_hi", ibl["prefiltered"])]))
    lut = _d(ibl["lut"])
    env = _d(env)
    lo = np.zeros((3, H, W))
    hi = np.zeros((3, H, W))
    c, t = _cam(cam), _tie(tie)
    lib().orc_shade(_p(depth), _p(normal), _p(albedo), _p(rough), _p(metal), C.byref(c),
                    _p(ao_lo), _p(ao_hi), arr, len(lights), _p(irr), irr.shape[1], _p(pref),
                    _p(pref_hi), ibl["prefiltered"][0].shape[1], len(ibl["prefiltered"]), _p(lut), lut.shape[0],
                    _p(env), env.shape[1], C.byref(t), _p(lo), _p(hi))
    return lo, hi


# ---------------------------------------------------------------------------
# eye-dome lighting (Sec. 4.3)
# ---------------------------------------------------------------------------
def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops."""
    lib().orc_set_threads(int(n))


def edl_offsets(radius: int, n_dirs: int) -> List[Tuple[int, int]]:
    dx = (C.c_int * n_dirs)()
    dy = (C.c_int * n_dirs)()
    lib().orc_edl_offsets(radius, n_dirs, dx, dy)
    return list(zip(dx, dy))


def edl(depth, color, cam, ao_lo=None, ao_hi=None, radius=1, n_dirs=8, strength=8.0,
        far_depth=1000.0, env=None, tie=DEFAULT_TIE) -> Tuple[np.ndarray, np.ndarray]:
    """Eye-dome lighting of a depth map with per-pixel colour; ``(lo, hi)`` differ
    only through the AO interval and cube-face ties of the background."""
    assert 1 <= n_dirs <= 64
    depth, color = _d(depth), _d(color)
    H, W = depth.shape
    null = C.cast(None, _D)
    aol = _d(ao_lo) if ao_lo is not None else None
    aoh = _d(ao_hi) if ao_hi is not None else aol
    envd = _d(env) if env is not None else None
    lo = np.zeros((3, H, W))
    hi = np.zeros((3, H, W))
    c = _cam(cam)
    lib().orc_edl(_p(depth), _p(color), C.byref(c), _p(aol) if aol is not None else null,
                  _p(aoh) if aoh is not None else null, radius, n_dirs, strength, far_depth,
                  _p(envd) if envd is not None else null, envd.shape[1] if envd is not None else 0,
                  Tie(*tie).face, _p(lo), _p(hi))
    return lo, hi


# ---------------------------------------------------------------------------
# a5 / a6: bloom + tonemap (monotone, so an interval maps end to end)
# ---------------------------------------------------------------------------
def bloom_tonemap(hdr, levels=6, threshold=1.0, strength=0.04, exposure=1.0, gamma=2.2,
                  want_composite=False, want_pyramid=False, tonemap=0):
    hdr = _d(hdr)
    _, H, W = hdr.shape
    ldr = np.zeros((H, W, 4), np.uint8)
    comp = np.zeros((3, H, W)) if want_composite else None
    sizes = []
    w, h = W, H
    for _ in range(1, levels):
        w, h = (w + 1) // 2, (h + 1) // 2
        sizes.append((h, w))
    pyr = np.zeros(sum(3 * a * b for a, b in sizes)) if want_pyramid else None
    lib().orc_bloom_tonemap(_p(hdr), W, H, levels, threshold, strength, exposure, gamma, tonemap,
                            ldr.ctypes.data_as(C.POINTER(C.c_uint8)),
                            _p(comp) if comp is not None else C.cast(None, _D),
                            _p(pyr) if pyr is not None else C.cast(None, _D))
    out = {"ldr": ldr}
    if comp is not None:
        out["composite"] = comp
    if pyr is not None:
        lv, off = [], 0
        for (h, w) in sizes:
            lv.append(pyr[off:off + 3 * h * w].reshape(3, h, w))
            off += 3 * h * w
        out["pyramid"] = lv
    return out


# ---------------------------------------------------------------------------
# the whole pass on one view
# ---------------------------------------------------------------------------
def render(view, tie=DEFAULT_TIE, ibl: Optional[dict] = None) -> dict:
    """Oracle of the full per-frame path on a :class:`synth.ViewInputs`:
    SSAO (raw + blur), shading, bloom and tonemap, with intervals."""
    g = view.gbuf
    if ibl is None:
        ibl = precompute_ibl(view.env, **view.ibl)
    raw_lo, raw_hi = ssao_raw(g["depth"], g["normal"], view.cam, view.ssao_kernel,
                              view.ssao_noise, view.ssao_radius, view.ssao_bias, tie)
    ao_lo, ao_hi = ssao_blur(raw_lo, raw_hi, g["depth"], view.blur_tau)
    hdr_lo, hdr_hi = shade(g, view.cam, ao_lo, ao_hi, view.lights, ibl, view.env, tie)
    post = dict(threshold=view.bloom_threshold, strength=view.bloom_strength,
                exposure=view.exposure, gamma=view.gamma, tonemap=getattr(view, "tonemap", 0))
    lo = bloom_tonemap(hdr_lo, **post)["ldr"]
    hi = bloom_tonemap(hdr_hi, **post)["ldr"]
    return dict(ibl=ibl, ao_raw=(raw_lo, raw_hi), ao=(ao_lo, ao_hi), hdr=(hdr_lo, hdr_hi),
                ldr=(lo, hi))
