"""Python binding of ``libepb.so`` (include/epb.h): ctypes structures and the
C-ABI entry points under the same names.

Marshalling only: every step of the shading pass runs in the HIP kernels of the
library.  Device memory and streams come from PyTorch; tensors are passed by
their data pointers.  Importing this module loads the library and fails loudly
if it has not been built (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libepb.so")

EPB_OK = 0
EPB_ERR_NULL = -1
EPB_ERR_SIZE = -2
EPB_ERR_DTYPE = -3
EPB_ERR_ALIGN = -4
EPB_ERR_SCRATCH = -5
EPB_ERR_PARAM = -6
EPB_ERR_HIP = -7
EPB_ERR_TIMEOUT = -8

EPB_F32 = 0
EPB_F16 = 1

EPB_MAX_LIGHTS = 8
EPB_MAX_SSAO_SAMPLES = 256
EPB_MAX_BLOOM_LEVELS = 6
EPB_MAX_BATCH_VIEWS = 4096
EPB_MAX_PERSISTENT_CHUNK = 4096

EPB_OP_PRECOMPUTE_IBL = 0
EPB_OP_SSAO = 1
EPB_OP_BLOOM_TONEMAP = 2
EPB_OP_RAYCAST = 3
EPB_MAX_SPHERES = 65536
EPB_TONEMAP_ACES = 0
EPB_TONEMAP_REINHARD = 1
EPB_MAX_EDL_RADIUS = 16
EPB_MAX_EDL_DIRS = 32
EPB_MAP_ROWS = 0
EPB_MAP_TILES = 1
EPB_SSAO_STATIC_SCRATCH_BYTES = 16 << 20

ENTRY_POINTS = ("epb_precompute_ibl", "epb_ssao", "epb_ssao_static", "epb_shade", "epb_bloom_tonemap",
                "epb_shade_post",
                "epb_scratch_bytes", "epb_status_str", "epb_last_hip_error",
                "epb_batch_table_bytes", "epb_view_scratch_bytes", "epb_batch_scratch_bytes",
                "epb_batch_build",
                "epb_render_batch", "epb_batch_status", "epb_raycast", "epb_edl", "epb_shadow_tiles_bytes", "epb_shadow_tiles")


class EpbError(RuntimeError):
    def __init__(self, fn: str, status: int):
        msg = f"{fn} returned {status}: {epb_status_str(status)}"
        if status == EPB_ERR_HIP:
            msg += f" (HIP error {epb_last_hip_error()})"
        super().__init__(msg)
        self.status = status


class epb_camera(C.Structure):
    _fields_ = [("world_to_cam", C.c_float * 12), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class epb_gbuffer(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("dtype", C.c_int),
                ("depth", C.c_void_p), ("normal", C.c_void_p), ("albedo", C.c_void_p),
                ("roughness", C.c_void_p), ("metalness", C.c_void_p), ("weight", C.c_void_p)]


class epb_cube(C.Structure):
    _fields_ = [("size", C.c_int32), ("levels", C.c_int32), ("data", C.c_void_p)]


class epb_ibl_params(C.Structure):
    _fields_ = [("irr_size", C.c_int32), ("irr_src_size", C.c_int32), ("pref_size", C.c_int32),
                ("pref_levels", C.c_int32), ("pref_samples", C.c_int32), ("lut_size", C.c_int32),
                ("lut_samples", C.c_int32), ("pref_fis", C.c_int32)]


class epb_ibl_maps(C.Structure):
    _fields_ = [("irradiance", epb_cube), ("prefiltered", epb_cube), ("brdf_lut", C.c_void_p),
                ("lut_size", C.c_int32)]


class epb_ssao_params(C.Structure):
    _fields_ = [("n_samples", C.c_int32), ("kernel", C.c_void_p), ("noise", C.c_void_p),
                ("radius", C.c_float), ("bias", C.c_float), ("blur_tau", C.c_float),
                ("blur", C.c_int32), ("out_dtype", C.c_int)]


class epb_light(C.Structure):
    _fields_ = [("pos", C.c_float * 3), ("color", C.c_float * 3), ("intensity", C.c_float),
                ("shadow_map", C.c_void_p), ("shadow_cam", epb_camera), ("shadow_bias", C.c_float),
                ("shadow_layout", C.c_int32)]


class epb_post_params(C.Structure):
    _fields_ = [("bloom_levels", C.c_int32), ("threshold", C.c_float), ("strength", C.c_float),
                ("exposure", C.c_float), ("gamma", C.c_float), ("pyr_dtype", C.c_int),
                ("tonemap", C.c_int32)]


class epb_sphere_scene(C.Structure):
    _fields_ = [("n", C.c_int32), ("center", C.c_void_p), ("radius", C.c_void_p), ("albedo", C.c_void_p),
                ("rough", C.c_void_p), ("metal", C.c_void_p), ("plane", C.c_int32),
                ("plane_albedo", C.c_float * 3), ("plane_rough", C.c_float), ("plane_metal", C.c_float)]


class epb_view(C.Structure):
    _fields_ = [("gbuf", epb_gbuffer), ("cam", epb_camera), ("lights", C.c_void_p),
                ("n_lights", C.c_int32), ("ibl", C.c_void_p), ("env", C.c_void_p),
                ("ssao", C.c_void_p), ("post", C.c_void_p), ("hdr_dtype", C.c_int),
                ("ao", C.c_void_p), ("hdr", C.c_void_p), ("ldr", C.c_void_p),
                ("scratch", C.c_void_p)]


class epb_edl_params(C.Structure):
    _fields_ = [("radius", C.c_int32), ("n_dirs", C.c_int32), ("strength", C.c_float),
                ("far_depth", C.c_float)]


class epb_schedule(C.Structure):
    _fields_ = [("shade_tile", C.c_int32), ("ssao_tile", C.c_int32), ("ssao_batch", C.c_int32),
                ("blocks_per_cu", C.c_int32), ("persistent", C.c_int32), ("wait_limit", C.c_int32),
                ("fuse_bloom", C.c_int32)]


STRUCTS = dict(epb_camera=epb_camera, epb_gbuffer=epb_gbuffer, epb_cube=epb_cube,
               epb_ibl_params=epb_ibl_params, epb_ibl_maps=epb_ibl_maps,
               epb_ssao_params=epb_ssao_params, epb_light=epb_light,
               epb_post_params=epb_post_params, epb_view=epb_view, epb_schedule=epb_schedule,
               epb_sphere_scene=epb_sphere_scene, epb_edl_params=epb_edl_params)


def _load() -> C.CDLL:
    # PyTorch-ROCm carries its own HIP runtime under the same soname; import it
    # first so that libepb.so binds to that runtime and shares torch's device
    # memory and streams (a second runtime loaded first would see no device).
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2012_03325_amd.build` "
                          "(the shading pass has no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    lib.epb_precompute_ibl.argtypes = [C.POINTER(epb_cube), C.POINTER(epb_ibl_params),
                                       C.POINTER(epb_ibl_maps), P, C.c_size_t, P]
    lib.epb_ssao.argtypes = [C.POINTER(epb_gbuffer), C.POINTER(epb_camera),
                             C.POINTER(epb_ssao_params), P, P, C.c_size_t, P]
    lib.epb_ssao_static.argtypes = [C.POINTER(epb_gbuffer), C.POINTER(epb_camera),
                                    C.POINTER(epb_ssao_params), P, P]
    lib.epb_shade.argtypes = [C.POINTER(epb_gbuffer), C.POINTER(epb_camera), P, C.c_int,
                              C.POINTER(epb_light), C.c_int32, C.POINTER(epb_ibl_maps),
                              C.POINTER(epb_cube), P, C.c_int, P]
    lib.epb_bloom_tonemap.argtypes = [P, C.c_int, C.c_int32, C.c_int32, C.POINTER(epb_post_params),
                                      P, P, C.c_size_t, P]
    lib.epb_shade_post.argtypes = [C.POINTER(epb_gbuffer), C.POINTER(epb_camera), P, C.c_int,
                                   C.POINTER(epb_light), C.c_int32, C.POINTER(epb_ibl_maps),
                                   C.POINTER(epb_cube), P, C.c_int, C.POINTER(epb_post_params), P, P,
                                   C.c_size_t, P]
    lib.epb_scratch_bytes.argtypes = [C.c_int32, C.c_int32, C.c_int32, P]
    lib.epb_scratch_bytes.restype = C.c_size_t
    lib.epb_status_str.argtypes = [C.c_int]
    lib.epb_status_str.restype = C.c_char_p
    lib.epb_last_hip_error.argtypes = []
    lib.epb_batch_table_bytes.argtypes = [C.c_int32]
    lib.epb_batch_table_bytes.restype = C.c_size_t
    lib.epb_view_scratch_bytes.argtypes = [P]
    lib.epb_view_scratch_bytes.restype = C.c_size_t
    lib.epb_batch_scratch_bytes.argtypes = [P, C.c_int32]
    lib.epb_batch_scratch_bytes.restype = C.c_size_t
    lib.epb_batch_build.argtypes = [P, C.c_int32, P, P, C.c_size_t, P, C.c_size_t]
    lib.epb_render_batch.argtypes = [P, P, P]
    lib.epb_batch_status.argtypes = [P, P, P]
    lib.epb_raycast.argtypes = [C.POINTER(epb_sphere_scene), C.POINTER(epb_camera), C.POINTER(epb_gbuffer), P,
                                C.c_size_t, P]
    lib.epb_edl.argtypes = [P, P, C.c_int, C.POINTER(epb_camera), P, C.c_int, C.POINTER(epb_edl_params),
                            C.POINTER(epb_cube), P, C.c_int, P]
    lib.epb_shadow_tiles_bytes.argtypes = [C.c_int32, C.c_int32]
    lib.epb_shadow_tiles_bytes.restype = C.c_size_t
    lib.epb_shadow_tiles.argtypes = [P, C.c_int32, C.c_int32, P, C.c_size_t, P]
    for fn in ("epb_precompute_ibl", "epb_ssao", "epb_ssao_static", "epb_shade", "epb_bloom_tonemap",
               "epb_shade_post", "epb_last_hip_error", "epb_batch_build", "epb_render_batch", "epb_batch_status",
               "epb_raycast", "epb_edl",
               "epb_shadow_tiles"):
        getattr(lib, fn).restype = C.c_int
    return lib


lib = _load()


def _ptr(x) -> Optional[int]:
    """Device pointer of a torch tensor (or an int / None passed through)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(fn: str, status: int, check: bool) -> int:
    if check and status != EPB_OK:
        raise EpbError(fn, status)
    return status


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ---------------------------------------------------------------------------
def epb_status_str(status: int) -> str:
    return lib.epb_status_str(status).decode()


def epb_last_hip_error() -> int:
    return lib.epb_last_hip_error()


def epb_scratch_bytes(op: int, width: int, height: int, params=None) -> int:
    return lib.epb_scratch_bytes(op, width, height, C.byref(params) if params is not None else None)


def epb_precompute_ibl(env: epb_cube, params: epb_ibl_params, out: epb_ibl_maps, scratch,
                       scratch_bytes: int, stream=None, check: bool = True) -> int:
    st = lib.epb_precompute_ibl(C.byref(env), C.byref(params), C.byref(out), _ptr(scratch),
                                scratch_bytes, _stream(stream))
    return _check("epb_precompute_ibl", st, check)


def epb_ssao(gbuf: epb_gbuffer, cam: epb_camera, params: epb_ssao_params, ao_out, scratch,
             scratch_bytes: int, stream=None, check: bool = True) -> int:
    st = lib.epb_ssao(C.byref(gbuf), C.byref(cam), C.byref(params), _ptr(ao_out), _ptr(scratch),
                      scratch_bytes, _stream(stream))
    return _check("epb_ssao", st, check)


def epb_ssao_static(gbuf: epb_gbuffer, cam: epb_camera, params: epb_ssao_params, ao_out, stream=None,
                    check: bool = True) -> int:
    st = lib.epb_ssao_static(C.byref(gbuf), C.byref(cam), C.byref(params), _ptr(ao_out), _stream(stream))
    return _check("epb_ssao_static", st, check)


def epb_shade(gbuf: epb_gbuffer, cam: epb_camera, ao, ao_dtype: int, lights: Sequence[epb_light],
              ibl: epb_ibl_maps, env: epb_cube, hdr_out, hdr_dtype: int, stream=None,
              check: bool = True) -> int:
    n = len(lights)
    arr = (epb_light * max(1, n))(*lights)
    st = lib.epb_shade(C.byref(gbuf), C.byref(cam), _ptr(ao), ao_dtype, arr if n else None, n,
                       C.byref(ibl), C.byref(env), _ptr(hdr_out), hdr_dtype, _stream(stream))
    return _check("epb_shade", st, check)


def epb_bloom_tonemap(hdr, hdr_dtype: int, width: int, height: int, params: epb_post_params,
                      ldr_out, scratch, scratch_bytes: int, stream=None, check: bool = True) -> int:
    st = lib.epb_bloom_tonemap(_ptr(hdr), hdr_dtype, width, height, C.byref(params), _ptr(ldr_out),
                               _ptr(scratch), scratch_bytes, _stream(stream))
    return _check("epb_bloom_tonemap", st, check)


def epb_shade_post(gbuf: epb_gbuffer, cam: epb_camera, ao, ao_dtype: int, lights: Sequence[epb_light],
                   ibl: epb_ibl_maps, env: epb_cube, hdr_out, hdr_dtype: int, params: epb_post_params,
                   ldr_out, scratch, scratch_bytes: int, stream=None, check: bool = True) -> int:
    n = len(lights)
    arr = (epb_light * max(1, n))(*lights)
    st = lib.epb_shade_post(C.byref(gbuf), C.byref(cam), _ptr(ao), ao_dtype, arr if n else None, n,
                            C.byref(ibl), C.byref(env), _ptr(hdr_out), hdr_dtype, C.byref(params),
                            _ptr(ldr_out), _ptr(scratch), scratch_bytes, _stream(stream))
    return _check("epb_shade_post", st, check)


def epb_batch_table_bytes(n_views: int) -> int:
    return lib.epb_batch_table_bytes(n_views)


def _views(views) -> C.Array:
    return (epb_view * len(views))(*views)


def epb_view_scratch_bytes(view: epb_view) -> int:
    return lib.epb_view_scratch_bytes(C.addressof(view))


def epb_batch_scratch_bytes(views: Sequence[epb_view]) -> int:
    arr = _views(views)
    return lib.epb_batch_scratch_bytes(C.addressof(arr), len(views))


def epb_batch_build(views: Sequence[epb_view], schedule: Optional[epb_schedule], scratch,
                    scratch_bytes: int, table, table_bytes: int, check: bool = True) -> int:
    """`table` is a host buffer (a ctypes buffer, a pinned CPU tensor or an int address)."""
    arr = _views(views)
    tab = C.addressof(table) if isinstance(table, C.Array) else _ptr(table)
    st = lib.epb_batch_build(C.addressof(arr), len(views),
                             C.addressof(schedule) if schedule is not None else None,
                             _ptr(scratch), scratch_bytes, tab, table_bytes)
    return _check("epb_batch_build", st, check)


def epb_render_batch(table, table_dev, stream=None, check: bool = True) -> int:
    tab = C.addressof(table) if isinstance(table, C.Array) else _ptr(table)
    st = lib.epb_render_batch(tab, _ptr(table_dev), _stream(stream))
    return _check("epb_render_batch", st, check)


def epb_batch_status(table, table_dev, stream=None, check: bool = True) -> int:
    tab = C.addressof(table) if isinstance(table, C.Array) else _ptr(table)
    st = lib.epb_batch_status(tab, _ptr(table_dev), _stream(stream))
    return _check("epb_batch_status", st, check)


def epb_raycast(scene: epb_sphere_scene, cam: epb_camera, out: epb_gbuffer, scratch, scratch_bytes: int,
                stream=None, check: bool = True) -> int:
    st = lib.epb_raycast(C.byref(scene), C.byref(cam), C.byref(out), _ptr(scratch), scratch_bytes, _stream(stream))
    return _check("epb_raycast", st, check)


def epb_edl(depth, color, color_dtype: int, cam: epb_camera, ao, ao_dtype: int, params: epb_edl_params,
            env: Optional[epb_cube], hdr_out, hdr_dtype: int, stream=None, check: bool = True) -> int:
    st = lib.epb_edl(_ptr(depth), _ptr(color), color_dtype, C.byref(cam), _ptr(ao), ao_dtype, C.byref(params),
                     C.byref(env) if env is not None else None, _ptr(hdr_out), hdr_dtype, _stream(stream))
    return _check("epb_edl", st, check)


def epb_shadow_tiles_bytes(width: int, height: int) -> int:
    return lib.epb_shadow_tiles_bytes(width, height)


def epb_shadow_tiles(shadow_map, width: int, height: int, tiles, tiles_bytes: int, stream=None,
                     check: bool = True) -> int:
    st = lib.epb_shadow_tiles(_ptr(shadow_map), width, height, _ptr(tiles), tiles_bytes, _stream(stream))
    return _check("epb_shadow_tiles", st, check)


# ---------------------------------------------------------------------------
# struct constructors
# ---------------------------------------------------------------------------
def make_camera(world_to_cam, fx, fy, cx, cy, width, height) -> epb_camera:
    c = epb_camera()
    flat = [float(v) for row in world_to_cam for v in row] if hasattr(world_to_cam[0], "__len__") \
        else [float(v) for v in world_to_cam]
    for k, v in enumerate(flat):
        c.world_to_cam[k] = v
    c.fx, c.fy, c.cx, c.cy = float(fx), float(fy), float(cx), float(cy)
    c.width, c.height = int(width), int(height)
    return c
