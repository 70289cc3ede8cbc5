"""Device-resident frames: upload a seeded view to HBM once, allocate its
outputs and scratch with PyTorch, and run the C-ABI calls on a stream.

This is plumbing around :mod:`paper_2012_03325_amd.epb` (allocation and
argument marshalling); the shading itself runs in the library's kernels.
"""
from __future__ import annotations

from typing import List, Optional

import ctypes as C

import numpy as np
import torch

from . import epb as E

_TORCH_DT = {E.EPB_F32: torch.float32, E.EPB_F16: torch.float16}


def _cam_struct(cam) -> E.epb_camera:
    return E.make_camera(np.asarray(cam.world_to_cam, np.float32).reshape(-1), cam.fx, cam.fy,
                         cam.cx, cam.cy, cam.width, cam.height)


def tile_shadow_map(m: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Tiled form (EPB_MAP_TILES) of the row-major [h][w] float32 depth map ``m``."""
    h, w = m.shape
    n = E.epb_shadow_tiles_bytes(w, h)
    if out is None or out.numel() * 4 < n:
        out = torch.empty(n // 4, dtype=torch.float32, device=m.device)
    E.epb_shadow_tiles(m, w, h, out, out.numel() * 4, stream)
    return out


class DeviceIBL:
    """Environment cube and its image-based-lighting tables on the device."""

    def __init__(self, env: np.ndarray, irr_size=32, irr_src_size=64, pref_size=128,
                 pref_levels=5, pref_samples=1024, lut_size=256, lut_samples=1024,
                 device="cuda", pref_fis=0, **_unused):
        self.device = device
        self.env = torch.from_numpy(np.ascontiguousarray(env, np.float32)).to(device)
        S = env.shape[1]
        self.S = S
        p = E.epb_ibl_params(irr_size, irr_src_size, pref_size, pref_levels, pref_samples,
                             lut_size, lut_samples, pref_fis)
        self.params = p
        self.base = min(S, pref_size)
        self.levels = pref_levels
        n_pref = sum(6 * (self.base >> m) ** 2 * 4 for m in range(pref_levels))
        self.irr = torch.empty((6, irr_size, irr_size, 4), dtype=torch.float32, device=device)
        self.pref = torch.empty(n_pref, dtype=torch.float32, device=device)
        self.lut = torch.empty((lut_size, lut_size, 2), dtype=torch.float32, device=device)
        self.scratch_bytes = E.epb_scratch_bytes(E.EPB_OP_PRECOMPUTE_IBL, S, S, p)
        if self.scratch_bytes == 0:
            raise ValueError("invalid image-based-lighting sizes for this environment")
        self.scratch = torch.empty(self.scratch_bytes, dtype=torch.uint8, device=device)
        self._structs()

    def _structs(self):
        self.env_c = E.epb_cube(self.S, 1, self.env.data_ptr())
        self.maps = E.epb_ibl_maps(E.epb_cube(self.irr.shape[1], 1, self.irr.data_ptr()),
                                   E.epb_cube(self.base, self.levels, self.pref.data_ptr()),
                                   self.lut.data_ptr(), self.lut.shape[0])

    def precompute(self, stream=None):
        E.epb_precompute_ibl(self.env_c, self.params, self.maps, self.scratch, self.scratch_bytes,
                             stream)

    def pref_levels(self) -> List[torch.Tensor]:
        out, off = [], 0
        for m in range(self.levels):
            s = self.base >> m
            n = 6 * s * s * 4
            out.append(self.pref[off:off + n].view(6, s, s, 4))
            off += n
        return out

    def load_tables(self, irradiance, prefiltered, lut):
        """Replace the tables with given (host) values, e.g. to test shading alone."""
        self.irr.copy_(torch.from_numpy(np.asarray(irradiance, np.float32)))
        flat = np.concatenate([np.asarray(m, np.float32).reshape(-1) for m in prefiltered])
        self.pref.copy_(torch.from_numpy(flat))
        self.lut.copy_(torch.from_numpy(np.asarray(lut, np.float32)))


class DevicePost:
    """Bloom and tone-mapping outputs and scratch for a W x H frame."""

    def __init__(self, W: int, H: int, bloom_levels=6, threshold=1.0, strength=0.04,
                 exposure=1.0, gamma=2.2, device="cuda", pyr_dtype=E.EPB_F32, scratch=True,
                 outputs=True, tonemap=E.EPB_TONEMAP_ACES):
        self.W, self.H = W, H
        self.post = E.epb_post_params(bloom_levels, threshold, strength, exposure, gamma, pyr_dtype, tonemap)
        self.ldr = torch.empty((H, W, 4), dtype=torch.uint8, device=device) if outputs else None
        self.scratch_bytes = E.epb_scratch_bytes(E.EPB_OP_BLOOM_TONEMAP, W, H, self.post)
        self.scratch = (torch.empty(self.scratch_bytes, dtype=torch.uint8, device=device)
                        if scratch else None)

    def run(self, hdr: torch.Tensor, stream=None):
        hdt = E.EPB_F16 if hdr.dtype == torch.float16 else E.EPB_F32
        E.epb_bloom_tonemap(hdr, hdt, self.W, self.H, self.post, self.ldr, self.scratch,
                            self.scratch_bytes, stream)

    def pyramid(self) -> List[torch.Tensor]:
        """Blurred bloom levels 1.. from the head of the scratch buffer."""
        out, off = [], 0
        w, h = self.W, self.H
        f = self.scratch.view(_TORCH_DT[self.post.pyr_dtype])
        for _ in range(1, self.post.bloom_levels):
            w, h = (w + 1) // 2, (h + 1) // 2
            out.append(f[off:off + h * w * 4].view(h, w, 4))
            off += h * w * 4
        return out


class DeviceView:
    """One view (G-buffer, camera, lights, SSAO kernel) resident on the device
    with its AO, HDR and LDR outputs and the scratch of each call.

    ``solo_scratch=False`` skips the scratch of the single-view calls (views
    that are only rendered in batches, or that share one scratch buffer:
    assign ``ssao_scratch`` and ``postp.scratch`` before calling them).
    ``src`` takes the G-buffer from another device view (converted to
    ``gdtype`` on the device) instead of uploading it again.  ``outputs=False``
    allocates no AO, HDR or LDR image (views that only serve as templates).
    ``shadow_layout`` is the storage of the lights' depth maps on the device:
    EPB_MAP_TILES (the default, faster to fetch) or EPB_MAP_ROWS."""

    def __init__(self, view, ibl: DeviceIBL, gdtype=E.EPB_F32, ao_dtype=E.EPB_F32,
                 hdr_dtype=E.EPB_F32, device="cuda", bloom_levels=6, solo_scratch=True,
                 src: Optional["DeviceView"] = None, outputs: bool = True, shadow_layout=E.EPB_MAP_TILES):
        self.view = view
        self.ibl = ibl
        self.device = device
        W, H = view.width, view.height
        self.W, self.H = W, H
        self.Wh, self.Hh = (W + 1) // 2, (H + 1) // 2
        self.gdtype, self.ao_dtype, self.hdr_dtype = gdtype, ao_dtype, hdr_dtype
        g = view.gbuf
        gt = _TORCH_DT[gdtype]
        dev = lambda a, dt=torch.float32: torch.from_numpy(np.ascontiguousarray(a)).to(device).to(dt)
        if src is None:
            self.depth = dev(g["depth"])
            self.normal = dev(g["normal"], gt)
            self.albedo = dev(g["albedo"], gt)
            self.rough = dev(g["roughness"], gt)
            self.metal = dev(g["metalness"], gt)
        else:
            self.depth = src.depth
            self.normal, self.albedo = src.normal.to(gt), src.albedo.to(gt)
            self.rough, self.metal = src.rough.to(gt), src.metal.to(gt)
        self.kernel = dev(view.ssao_kernel)
        self.noise = dev(view.ssao_noise)
        self.cam = _cam_struct(view.cam)
        self.weight = None
        if g.get("weight") is not None:  # surfel-splatted G-buffer
            self.weight = dev(g["weight"], gt) if src is None else src.weight.to(gt)
        self.gbuf = E.epb_gbuffer(W, H, gdtype, self.depth.data_ptr(), self.normal.data_ptr(),
                                  self.albedo.data_ptr(), self.rough.data_ptr(), self.metal.data_ptr(),
                                  self.weight.data_ptr() if self.weight is not None else None)
        self.ssao_params = E.epb_ssao_params(self.kernel.shape[0], self.kernel.data_ptr(),
                                             self.noise.data_ptr(), view.ssao_radius, view.ssao_bias,
                                             view.blur_tau, 1, ao_dtype)
        self.shadow_maps = []
        self.lights = []
        for L in view.lights:
            s = E.epb_light()
            for c in range(3):
                s.pos[c] = float(L.pos[c])
                s.color[c] = float(L.color[c])
            s.intensity = float(L.intensity)
            if L.shadow_map is not None:
                m = dev(L.shadow_map)
                if shadow_layout == E.EPB_MAP_TILES:
                    m = tile_shadow_map(m)
                self.shadow_maps.append(m)
                s.shadow_map = m.data_ptr()
                s.shadow_cam = _cam_struct(L.shadow_cam)
                s.shadow_bias = float(L.shadow_bias)
                s.shadow_layout = shadow_layout
            self.lights.append(s)
        self.postp = DevicePost(W, H, bloom_levels, view.bloom_threshold, view.bloom_strength,
                                view.exposure, view.gamma, device, pyr_dtype=hdr_dtype,
                                scratch=solo_scratch, outputs=outputs, tonemap=view.tonemap)
        self.post = self.postp.post
        self.ldr = self.postp.ldr
        self.ao = torch.empty((self.Hh, self.Wh), dtype=_TORCH_DT[ao_dtype], device=device) if outputs else None
        self.hdr = torch.empty((3, H, W), dtype=_TORCH_DT[hdr_dtype], device=device) if outputs else None
        self.ssao_scratch_bytes = E.epb_scratch_bytes(E.EPB_OP_SSAO, W, H, self.ssao_params)
        self.ssao_scratch = (torch.empty(self.ssao_scratch_bytes, dtype=torch.uint8, device=device)
                             if solo_scratch else None)

    # -- the three per-frame calls ------------------------------------------
    def ssao(self, stream=None, blur: bool = True):
        self.ssao_params.blur = 1 if blur else 0
        E.epb_ssao(self.gbuf, self.cam, self.ssao_params, self.ao, self.ssao_scratch,
                   self.ssao_scratch_bytes, stream)

    def shade(self, stream=None, ao: Optional[torch.Tensor] = None, use_ao: bool = True):
        a = (ao if ao is not None else self.ao) if use_ao else None
        adt = E.EPB_F16 if (a is not None and a.dtype == torch.float16) else E.EPB_F32
        E.epb_shade(self.gbuf, self.cam, a, adt, self.lights, self.ibl.maps, self.ibl.env_c, self.hdr,
                    self.hdr_dtype, stream)

    def bloom_tonemap(self, stream=None, hdr: Optional[torch.Tensor] = None):
        self.postp.run(hdr if hdr is not None else self.hdr, stream)

    def shade_post(self, stream=None, ao: Optional[torch.Tensor] = None, use_ao: bool = True):
        """shade() then bloom_tonemap() in one call, bloom level 1 formed while shading."""
        a = (ao if ao is not None else self.ao) if use_ao else None
        adt = E.EPB_F16 if (a is not None and a.dtype == torch.float16) else E.EPB_F32
        pp = self.postp
        E.epb_shade_post(self.gbuf, self.cam, a, adt, self.lights, self.ibl.maps, self.ibl.env_c, self.hdr,
                         self.hdr_dtype, pp.post, pp.ldr, pp.scratch, pp.scratch_bytes, stream)

    def render(self, stream=None, fused: bool = False):
        self.ssao(stream)
        if fused:
            self.shade_post(stream)
        else:
            self.shade(stream)
            self.bloom_tonemap(stream)

    def pyramid(self) -> List[torch.Tensor]:
        return self.postp.pyramid()

    # -- batched form ---------------------------------------------------------
    def batch_view(self, blur: bool = True, keep_ao: bool = True, keep_hdr: bool = True) -> E.epb_view:
        """This view as an entry of a batch (outputs into this view's AO, HDR and
        LDR images; AO or HDR left to batch scratch when not kept)."""
        self.ssao_params.blur = 1 if blur else 0
        self._light_arr = (E.epb_light * max(1, len(self.lights)))(*self.lights)
        v = E.epb_view()
        v.gbuf = self.gbuf
        v.cam = self.cam
        v.lights = C.addressof(self._light_arr) if self.lights else None
        v.n_lights = len(self.lights)
        v.ibl = C.addressof(self.ibl.maps)
        v.env = C.addressof(self.ibl.env_c)
        v.ssao = C.addressof(self.ssao_params)
        v.post = C.addressof(self.post)
        v.hdr_dtype = self.hdr_dtype
        v.ao = self.ao.data_ptr() if keep_ao and self.ao is not None else None
        v.hdr = self.hdr.data_ptr() if keep_hdr and self.hdr is not None else None
        v.ldr = self.ldr.data_ptr() if self.ldr is not None else None
        return v


def make_schedule(shade_tile=0, ssao_tile=0, ssao_batch=0, blocks_per_cu=0, persistent=0,
                  wait_limit=0, fuse_bloom=0) -> E.epb_schedule:
    return E.epb_schedule(shade_tile, ssao_tile, ssao_batch, blocks_per_cu, persistent, wait_limit, fuse_bloom)


class DeviceBatch:
    """Many device views rendered together: one launch per stage for the whole
    batch.  The batch table is written on the host into pinned memory and
    copied to the device once; `render` then only enqueues kernels (and can be
    captured into a HIP graph)."""

    def __init__(self, dviews, schedule: Optional[E.epb_schedule] = None, blur: bool = True,
                 keep_ao: bool = True, keep_hdr: bool = True, device="cuda"):
        self.dviews = list(dviews)
        self.views = [dv.batch_view(blur, keep_ao, keep_hdr) for dv in self.dviews]
        n = len(self.views)
        self.scratch_bytes = E.epb_batch_scratch_bytes(self.views)
        if self.scratch_bytes == 0:
            raise ValueError("invalid batch")
        self.scratch = torch.empty(self.scratch_bytes, dtype=torch.uint8, device=device)
        self.table_bytes = E.epb_batch_table_bytes(n)
        self.table_host = torch.empty(self.table_bytes, dtype=torch.uint8, pin_memory=True)
        self.table_dev = torch.empty(self.table_bytes, dtype=torch.uint8, device=device)
        self.schedule = schedule if schedule is not None else make_schedule()
        self.build(self.schedule)

    def build(self, schedule: E.epb_schedule):
        """(Re)write the table for a schedule and upload it (synchronously)."""
        self.schedule = schedule
        E.epb_batch_build(self.views, schedule, self.scratch, self.scratch_bytes,
                          self.table_host.data_ptr(), self.table_bytes)
        self.table_dev.copy_(self.table_host)
        torch.cuda.synchronize()

    def render(self, stream=None):
        E.epb_render_batch(self.table_host.data_ptr(), self.table_dev, stream)

    def status(self, stream=None, check: bool = False) -> int:
        """EPB_OK, or EPB_ERR_TIMEOUT when a wait of the last persistent render
        gave up (waits for the stream)."""
        return E.epb_batch_status(self.table_host.data_ptr(), self.table_dev, stream, check=check)


class DeviceScene:
    """A sphere field resident on the device (geometry in double, materials in
    float) and the ray-cast pass that turns it into G-buffers and depth maps."""

    def __init__(self, spheres, device="cuda"):
        n = len(spheres.radii)
        self.n = n
        f64 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float64)).to(device)
        f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
        self.center = f64(np.asarray(spheres.centers).reshape(n, 3))
        self.radius = f64(spheres.radii)
        self.albedo = f32(np.asarray(spheres.albedo).reshape(n, 3))
        self.rough = f32(spheres.roughness)
        self.metal = f32(spheres.metalness)
        pa = (C.c_float * 3)(*[float(v) for v in spheres.plane_albedo])
        ptr = lambda t: t.data_ptr() if n > 0 else None
        self.struct = E.epb_sphere_scene(n, ptr(self.center), ptr(self.radius), ptr(self.albedo), ptr(self.rough),
                                         ptr(self.metal), 1 if spheres.plane else 0, pa,
                                         float(spheres.plane_roughness), float(spheres.plane_metalness))
        self.scratch_bytes = E.epb_scratch_bytes(E.EPB_OP_RAYCAST, 1, 1, self.struct)
        self.scratch = torch.empty(self.scratch_bytes, dtype=torch.uint8, device=device)
        self.device = device
        self.version = 0  # bumped whenever the geometry changes (shadow maps go stale)

    def move(self, centers=None, radii=None):
        """Replace sphere centres and/or radii in place (same count); every depth
        map rendered before is stale afterwards."""
        if centers is not None:
            self.center.copy_(torch.from_numpy(np.ascontiguousarray(centers, np.float64).reshape(self.n, 3)))
        if radii is not None:
            self.radius.copy_(torch.from_numpy(np.ascontiguousarray(radii, np.float64).reshape(self.n)))
        self.version += 1

    def render_gbuffer(self, cam, dtype=E.EPB_F32, stream=None) -> dict:
        """G-buffer planes (torch tensors) of the scene seen by ``cam``."""
        W, H = cam.width, cam.height
        dt = _TORCH_DT[dtype]
        g = dict(depth=torch.empty((H, W), device=self.device),
                 normal=torch.empty((3, H, W), dtype=dt, device=self.device),
                 albedo=torch.empty((3, H, W), dtype=dt, device=self.device),
                 roughness=torch.empty((H, W), dtype=dt, device=self.device),
                 metalness=torch.empty((H, W), dtype=dt, device=self.device))
        out = E.epb_gbuffer(W, H, dtype, g["depth"].data_ptr(), g["normal"].data_ptr(), g["albedo"].data_ptr(),
                            g["roughness"].data_ptr(), g["metalness"].data_ptr(), None)
        E.epb_raycast(self.struct, _cam_struct(cam), out, self.scratch, self.scratch_bytes, stream)
        return g

    def render_depth(self, cam, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """Depth map of the scene seen by ``cam`` (a light's shadow map)."""
        W, H = cam.width, cam.height
        d = out if out is not None else torch.empty((H, W), device=self.device)
        g = E.epb_gbuffer(W, H, E.EPB_F32, d.data_ptr(), None, None, None, None, None)
        E.epb_raycast(self.struct, _cam_struct(cam), g, self.scratch, self.scratch_bytes, stream)
        return d


class DeviceEDL:
    """A point-cloud render (depth + colour) on the device and the eye-dome
    lighting call that composes it."""

    def __init__(self, pc, color_dtype=E.EPB_F32, ao_dtype=E.EPB_F32, hdr_dtype=E.EPB_F32, device="cuda",
                 use_ao: bool = True, use_env: bool = True):
        H, W = pc.depth.shape
        self.W, self.H = W, H
        dev = lambda a, dt=torch.float32: torch.from_numpy(np.ascontiguousarray(a)).to(device).to(dt)
        self.color_dtype, self.ao_dtype, self.hdr_dtype = color_dtype, ao_dtype, hdr_dtype
        self.depth = dev(pc.depth)
        self.color = dev(pc.color, _TORCH_DT[color_dtype])
        self.ao = dev(pc.ao, _TORCH_DT[ao_dtype]) if use_ao else None
        self.env = dev(pc.env) if use_env else None
        self.env_c = E.epb_cube(pc.env.shape[1], 1, self.env.data_ptr()) if use_env else None
        self.cam = _cam_struct(pc.cam)
        self.params = E.epb_edl_params(pc.edl_radius, pc.edl_dirs, pc.edl_strength, pc.edl_far)
        self.hdr = torch.empty((3, H, W), dtype=_TORCH_DT[hdr_dtype], device=device)

    def run(self, stream=None, hdr: Optional[torch.Tensor] = None):
        E.epb_edl(self.depth, self.color, self.color_dtype, self.cam, self.ao, self.ao_dtype, self.params,
                  self.env_c, hdr if hdr is not None else self.hdr, self.hdr_dtype, stream)


class ShadowCache:
    """Depth maps of the lights of one scene, kept between frames and rendered
    again only when the scene's geometry or the light's camera changed (the
    paper's shadow maps are updated only when objects or lights move, Sec. 5.1).

    ``scene`` provides ``version`` (bumped on every geometry change) and
    ``render_depth(cam, out=None, stream=None)``; ``maps(cams)`` returns one
    depth map per light camera, reusing the stored map of a light whose camera
    and scene version are those it was rendered with.  With ``tiles=True`` the
    maps are returned in the tiled form (EPB_MAP_TILES), converted once per
    render.  ``renders`` counts the depth renders issued."""

    def __init__(self, scene, tiles: bool = False):
        self.scene = scene
        self.tiles = tiles
        self._entries = {}  # light index -> (camera key, scene version, map, tiled map or None)
        self.renders = 0

    @staticmethod
    def _key(cam) -> tuple:
        return (tuple(np.asarray(cam.world_to_cam, np.float64).reshape(-1).tolist()), float(cam.fx), float(cam.fy),
                float(cam.cx), float(cam.cy), int(cam.width), int(cam.height))

    def maps(self, cams, stream=None) -> list:
        out = []
        for i, cam in enumerate(cams):
            key = self._key(cam)
            ent = self._entries.get(i)
            if ent is not None and ent[0] == key and ent[1] == self.scene.version:
                out.append(ent[3] if self.tiles else ent[2])
                continue
            reuse = ent[2] if ent is not None and tuple(ent[2].shape) == (cam.height, cam.width) else None
            m = self.scene.render_depth(cam, out=reuse, stream=stream)
            self.renders += 1
            t = tile_shadow_map(m, out=ent[3] if ent is not None else None, stream=stream) if self.tiles else None
            self._entries[i] = (key, self.scene.version, m, t)
            out.append(t if self.tiles else m)
        return out

    def invalidate(self):
        """Forget every stored map (the next call renders all of them)."""
        self._entries.clear()
