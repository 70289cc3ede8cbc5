"""Serving loop: continuous batching of render requests against scenes kept
resident in HBM.

A request asks for one frame of a resident scene at one resolution.  The
server keeps three queues -- waiting (arrived, not admitted), ready (admitted:
it holds a memory slot) and in flight (launched batches) -- and on every
step:

1. polls the in-flight batches; a finished batch stamps its requests with the
   completion time of its HIP event, hands them to the ``on_done`` hook and
   returns their slots to the pool;
2. admits waiting requests in arrival order while their slot fits the HBM
   budget (a slot holds a request's output image and the scratch of its
   pass; idle slots of a resolution are reused, idle slots of other
   resolutions are released when memory is short);
3. launches the ready requests as one batch (one launch per stage of the
   shading pass for all of them) on the next of several streams, as long as
   fewer than ``max_inflight`` batches are running -- so requests that arrive
   while others are on the GPU join the next batch, and consecutive batches
   overlap on the device.

The scheduling logic (Server, SlotPool, clocks) is host code and is tested on
the CPU with a mock executor and a simulated clock; GpuExecutor runs the
batches through the C ABI (epb_batch_build + epb_render_batch).
"""
from __future__ import annotations

import collections
import ctypes as C
import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

Res = Tuple[int, int]


@dataclasses.dataclass
class Request:
    rid: int
    scene: int
    width: int
    height: int
    arrival: float                # seconds on the server clock
    admitted: float = math.nan
    launched: float = math.nan
    done: float = math.nan
    batch: int = -1
    slot: object = None
    rejected: bool = False
    cam: object = None            # a camera of its own (synth.Camera of the request's size): the
                                  # G-buffer is ray-cast for it on the device before shading

    @property
    def res(self) -> Res:
        return (self.width, self.height)

    @property
    def px(self) -> int:
        return self.width * self.height

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def poisson_arrivals(rate: float, seed: int, n_scenes: int, resolutions: Sequence[Res],
                     duration: Optional[float] = None, count: Optional[int] = None) -> List[Request]:
    """Requests with exponential inter-arrival gaps of mean 1 / rate, each
    drawing its scene ~ U{n_scenes} and its resolution ~ U(resolutions), until
    ``duration`` seconds or ``count`` requests (whichever is given / first)."""
    rng = np.random.default_rng(seed)
    out, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if duration is not None and t > duration:
            break
        if count is not None and len(out) >= count:
            break
        s = int(rng.integers(0, n_scenes))
        w, h = resolutions[int(rng.integers(0, len(resolutions)))]
        out.append(Request(len(out), s, w, h, t))
    return out


# ---------------------------------------------------------------------------
# clocks
# ---------------------------------------------------------------------------
class RealClock:
    """Wall time since start(); waiting polls every ``poll`` seconds."""

    def __init__(self, poll: float = 50e-6):
        self.poll = poll
        self.t0 = time.perf_counter()

    def start(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def wait(self, until: Optional[float], hint: Optional[float]):
        del hint
        dt = self.poll if until is None else min(self.poll, until - self.now())
        if dt > 0:
            time.sleep(dt)


class SimClock:
    """Simulated time: waiting jumps to the next arrival or completion."""

    def __init__(self):
        self.t = 0.0

    def start(self):
        self.t = 0.0

    def now(self) -> float:
        return self.t

    def wait(self, until: Optional[float], hint: Optional[float]):
        cands = [x for x in (until, hint) if x is not None and x > self.t]
        if not cands:
            raise RuntimeError("simulated server has nothing to wait for")
        self.t = min(cands)


# ---------------------------------------------------------------------------
# HBM-footprint admission
# ---------------------------------------------------------------------------
class SlotPool:
    """Memory slots per resolution under a byte budget.

    ``reserved`` counts every allocated slot, idle or busy; a request is
    admitted only if its class has an idle slot or a new one fits the budget
    (after releasing idle slots of other classes)."""

    def __init__(self, budget: int, footprint: Callable[[Res], int], alloc: Callable[[Res], object],
                 free: Callable[[object], None]):
        self.budget = int(budget)
        self.footprint = footprint
        self._alloc, self._free = alloc, free
        self.idle: Dict[Res, List[object]] = collections.defaultdict(list)
        self.reserved = 0
        self.peak = 0
        self.allocs = 0

    def fits_ever(self, res: Res) -> bool:
        return self.footprint(res) <= self.budget

    def acquire(self, res: Res):
        if self.idle[res]:
            return self.idle[res].pop()
        need = self.footprint(res)
        if self.reserved + need > self.budget:
            for other, slots in self.idle.items():
                while slots and other != res and self.reserved + need > self.budget:
                    self._free(slots.pop())
                    self.reserved -= self.footprint(other)
        if self.reserved + need > self.budget:
            return None
        self.reserved += need
        self.peak = max(self.peak, self.reserved)
        self.allocs += 1
        return self._alloc(res)

    def release(self, res: Res, slot):
        self.idle[res].append(slot)

    def clear(self):
        for res, slots in self.idle.items():
            while slots:
                self._free(slots.pop())
                self.reserved -= self.footprint(res)


# ---------------------------------------------------------------------------
# the server
# ---------------------------------------------------------------------------
class Server:
    def __init__(self, executor, budget_bytes: int, max_batch_views: int = 64,
                 max_batch_px: int = 64 << 20, max_inflight: int = 2,
                 on_done: Optional[Callable[[Request], None]] = None):
        self.ex = executor
        self.pool = SlotPool(budget_bytes, executor.footprint, executor.alloc, executor.free)
        self.max_views = max_batch_views
        self.max_px = max_batch_px
        self.max_inflight = max_inflight
        self.on_done = on_done
        self.waiting: collections.deque = collections.deque()
        self.ready: List[Request] = []
        self.inflight: List[Tuple[object, List[Request]]] = []
        self.finished: List[Request] = []
        self.rejected: List[Request] = []
        self.n_batches = 0
        self.batch_views: List[int] = []

    def submit(self, req: Request):
        if not self.pool.fits_ever(req.res):
            req.rejected = True
            self.rejected.append(req)
            return
        self.waiting.append(req)

    def _poll(self, now: float) -> bool:
        progressed = False
        still = []
        for handle, reqs in self.inflight:
            t = self.ex.done(handle)
            if t is None:
                still.append((handle, reqs))
                continue
            progressed = True
            for r in reqs:
                r.done = t
                if self.on_done is not None:
                    self.on_done(r)
                self.pool.release(r.res, r.slot)
                r.slot = None
                self.finished.append(r)
            self.ex.retire(handle)
        self.inflight = still
        return progressed

    def _admit(self, now: float) -> bool:
        progressed = False
        while self.waiting:
            r = self.waiting[0]
            slot = self.pool.acquire(r.res)
            if slot is None:
                break  # arrival order: later requests wait behind the head
            self.waiting.popleft()
            r.slot, r.admitted = slot, now
            self.ready.append(r)
            progressed = True
        return progressed

    def _launch(self, now: float) -> bool:
        if not self.ready or len(self.inflight) >= self.max_inflight:
            return False
        batch, px = [], 0
        while self.ready and len(batch) < self.max_views:
            r = self.ready[0]
            if batch and px + r.px > self.max_px:
                break
            batch.append(self.ready.pop(0))
            px += r.px
        for r in batch:
            r.launched, r.batch = now, self.n_batches
        self.inflight.append((self.ex.launch(batch), batch))
        self.n_batches += 1
        self.batch_views.append(len(batch))
        return True

    def step(self, now: float) -> bool:
        a = self._poll(now)
        b = self._admit(now)
        c = self._launch(now)
        return a or b or c

    def busy(self) -> bool:
        return bool(self.waiting or self.ready or self.inflight)

    def run(self, arrivals: Sequence[Request], clock) -> dict:
        """Serve ``arrivals`` (sorted by arrival time) in clock time; returns stats."""
        pending = collections.deque(sorted(arrivals, key=lambda r: r.arrival))
        clock.start()
        self.ex.start(clock)
        while pending or self.busy():
            now = clock.now()
            while pending and pending[0].arrival <= now:
                self.submit(pending.popleft())
            if not self.step(now):
                clock.wait(pending[0].arrival if pending else None, self.ex.next_event())
        return self.stats()

    def reset_stats(self):
        """Forget finished requests and batch counts (after an untimed warm-up
        pass); idle slots stay in the pool for the requests that follow."""
        self.finished, self.rejected, self.batch_views = [], [], []
        self.n_batches = 0

    def stats(self) -> dict:
        done = self.finished
        if not done:
            return dict(requests=0, rejected=len(self.rejected))
        lat = np.array([r.latency for r in done])
        px = sum(r.px for r in done)
        t0 = min(r.arrival for r in done)
        t1 = max(r.done for r in done)
        return dict(requests=len(done), rejected=len(self.rejected),
                    p50_ms=1e3 * float(np.percentile(lat, 50)), p99_ms=1e3 * float(np.percentile(lat, 99)),
                    mean_ms=1e3 * float(lat.mean()), max_ms=1e3 * float(lat.max()),
                    Mpix_s=px / max(t1 - t0, 1e-12) / 1e6, span_s=t1 - t0, batches=self.n_batches,
                    mean_batch_views=float(np.mean(self.batch_views)),
                    peak_reserved_bytes=self.pool.peak, slot_allocs=self.pool.allocs)


# ---------------------------------------------------------------------------
# executors
# ---------------------------------------------------------------------------
class MockExecutor:
    """A device model for host tests: batches run one after another, each
    taking ``launch_s + px * s_per_px`` seconds of simulated time."""

    def __init__(self, clock: SimClock, s_per_px: float = 1e-10, launch_s: float = 20e-6,
                 bytes_per_px: int = 40):
        self.clock = clock
        self.s_per_px, self.launch_s, self.bytes_per_px = s_per_px, launch_s, bytes_per_px
        self.busy_until = 0.0
        self.live_slots = 0
        self.log: List[Tuple[float, float, int]] = []

    def start(self, clock):
        self.busy_until = clock.now()

    def footprint(self, res: Res) -> int:
        return res[0] * res[1] * self.bytes_per_px

    def alloc(self, res: Res):
        self.live_slots += 1
        return ("slot", res, self.live_slots)

    def free(self, slot):
        self.live_slots -= 1

    def launch(self, reqs: List[Request]):
        start = max(self.clock.now(), self.busy_until)
        end = start + self.launch_s + self.s_per_px * sum(r.px for r in reqs)
        self.busy_until = end
        self.log.append((start, end, len(reqs)))
        return end

    def done(self, handle) -> Optional[float]:
        return handle if self.clock.now() >= handle else None

    def retire(self, handle):
        pass

    def next_event(self) -> Optional[float]:
        return self.busy_until if self.busy_until > self.clock.now() else None


class GpuExecutor:
    """Batches of requests through the C ABI on a few HIP streams.

    ``templates[(scene, (w, h))]`` is an epb_view of a resident G-buffer with
    its camera, lights, IBL tables, SSAO and post parameters (AO, HDR, LDR and
    scratch unset); a slot gives a request its LDR image and its view scratch
    (which also holds AO and HDR).  The batch table is written into a pinned
    host buffer, copied to the device on the batch's stream and rendered with
    epb_render_batch; a HIP event marks completion.

    With ``geometry`` (scene index -> frame.DeviceScene, the resident sphere
    field of each scene) every slot also holds G-buffer planes and ray-cast
    scratch, and a request that carries its own camera gets its G-buffer
    ray-cast on the batch's stream (epb_raycast) before the batch renders it;
    the scene's lights, IBL tables and parameters come from the template."""

    def __init__(self, templates: Dict[Tuple[int, Res], "object"], schedule=None, n_streams: int = 2,
                 max_inflight: int = 2, max_batch_views: int = 64, geometry: Optional[Dict[int, object]] = None):
        import torch

        from . import epb as E
        self.torch, self.E = torch, E
        self.templates = templates
        self.schedule = schedule if schedule is not None else E.epb_schedule(0, 0, 0, 0)
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]
        self.k = 0
        self.max_views = max_batch_views
        tb = E.epb_batch_table_bytes(max_batch_views)
        self.tb = tb
        self.free_tables = [(torch.empty(tb, dtype=torch.uint8, pin_memory=True),
                             torch.empty(tb, dtype=torch.uint8, device="cuda"))
                            for _ in range(max_inflight)]
        self._fp: Dict[Res, int] = {}
        self.ref = None
        self.t_ref = 0.0
        self.geometry = geometry
        self.ray_scratch = 0
        if geometry:
            self.ray_scratch = max(E.epb_scratch_bytes(E.EPB_OP_RAYCAST, 1, 1, g.struct) for g in geometry.values())

    def start(self, clock):
        torch = self.torch
        torch.cuda.synchronize()
        self.ref = torch.cuda.Event(enable_timing=True)
        self.ref.record()
        torch.cuda.synchronize()
        self.t_ref = clock.now()

    def _template(self, res: Res):
        for (s, r), v in self.templates.items():
            if r == res:
                return v
        raise KeyError(res)

    def _gbuf_bytes(self, res: Res) -> int:
        if not self.geometry:
            return 0
        vb = 2 if self._template(res).gbuf.dtype == self.E.EPB_F16 else 4
        return res[0] * res[1] * (4 + 8 * vb) + self.ray_scratch

    def footprint(self, res: Res) -> int:
        if res not in self._fp:
            v = self._template(res)
            self._fp[res] = (self.E.epb_view_scratch_bytes(v) + 4 * res[0] * res[1] + self._gbuf_bytes(res)
                             + 255) & ~255
        return self._fp[res]

    def alloc(self, res: Res):
        torch = self.torch
        v = self._template(res)
        ldr = torch.empty((res[1], res[0], 4), dtype=torch.uint8, device="cuda")
        scratch = torch.empty(self.E.epb_view_scratch_bytes(v), dtype=torch.uint8, device="cuda")
        slot = dict(ldr=ldr, scratch=scratch)
        if self.geometry:
            w, h = res
            dt = torch.float16 if v.gbuf.dtype == self.E.EPB_F16 else torch.float32
            slot.update(depth=torch.empty((h, w), device="cuda"), normal=torch.empty((3, h, w), dtype=dt, device="cuda"),
                        albedo=torch.empty((3, h, w), dtype=dt, device="cuda"),
                        rough=torch.empty((h, w), dtype=dt, device="cuda"),
                        metal=torch.empty((h, w), dtype=dt, device="cuda"),
                        ray_scratch=torch.empty(max(self.ray_scratch, 16), dtype=torch.uint8, device="cuda"))
        return slot

    def free(self, slot):
        slot.clear()

    def launch(self, reqs: List[Request]):
        torch, E = self.torch, self.E
        n = len(reqs)
        assert n <= self.max_views
        from .frame import _cam_struct
        arr = (E.epb_view * n)()
        casts = []
        for i, r in enumerate(reqs):
            v = E.epb_view.from_buffer_copy(self.templates[(r.scene, r.res)])
            v.ao, v.hdr = None, None
            v.ldr = r.slot["ldr"].data_ptr()
            v.scratch = r.slot["scratch"].data_ptr()
            if r.cam is not None:
                if not self.geometry or r.scene not in self.geometry:
                    raise ValueError("a request with its own camera needs the scene's geometry")
                sl = r.slot
                g = E.epb_gbuffer(r.width, r.height, v.gbuf.dtype, sl["depth"].data_ptr(), sl["normal"].data_ptr(),
                                  sl["albedo"].data_ptr(), sl["rough"].data_ptr(), sl["metal"].data_ptr(), None)
                cam = _cam_struct(r.cam)
                v.gbuf, v.cam = g, cam
                casts.append((self.geometry[r.scene], cam, g, sl["ray_scratch"]))
            arr[i] = v
        host, dev = self.free_tables.pop()
        st = E.lib.epb_batch_build(C.addressof(arr), n, C.addressof(self.schedule), None, 0,
                                   host.data_ptr(), self.tb)
        if st != E.EPB_OK:
            self.free_tables.append((host, dev))
            raise E.EpbError("epb_batch_build", st)
        s = self.streams[self.k % len(self.streams)]
        self.k += 1
        with torch.cuda.stream(s):
            for scene, cam, g, rs in casts:  # G-buffers of requests with their own camera
                E.epb_raycast(scene.struct, cam, g, rs, rs.numel(), s)
            dev.copy_(host, non_blocking=True)
            E.epb_render_batch(host.data_ptr(), dev, s)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(s)
        return dict(ev=ev, tables=(host, dev))

    def done(self, handle) -> Optional[float]:
        ev = handle["ev"]
        if not ev.query():
            return None
        return self.t_ref + self.ref.elapsed_time(ev) / 1e3

    def retire(self, handle):
        self.free_tables.append(handle["tables"])

    def next_event(self):
        return None


# ---------------------------------------------------------------------------
# resident scenes
# ---------------------------------------------------------------------------
class ResidentScenes:
    """Scenes kept in HBM for serving: per scene its IBL tables and, for every
    resolution, the G-buffer of one pose (``views[(scene, (w, h))]``, a
    ViewInputs), uploaded once; ``templates`` are the matching epb_view
    entries for GpuExecutor.  ``outputs`` / ``solo_scratch`` also give every
    resident view its own output images and single-view scratch (to render a
    request alone)."""

    def __init__(self, scene_inputs, views: Dict[Tuple[int, Res], object], gdtype, ao_dtype=None,
                 hdr_dtype=None, outputs: bool = False, solo_scratch: bool = False,
                 fp32_too: bool = False):
        from . import epb as E
        from . import frame
        ao_dtype = gdtype if ao_dtype is None else ao_dtype
        hdr_dtype = gdtype if hdr_dtype is None else hdr_dtype
        self.ibls = [frame.DeviceIBL(sc.env, **sc.ibl) for sc in scene_inputs]
        for ibl in self.ibls:
            ibl.precompute()
        self.dviews: Dict[Tuple[int, Res], object] = {}
        self.dviews32: Dict[Tuple[int, Res], object] = {}
        self.templates: Dict[Tuple[int, Res], object] = {}
        for key, v in views.items():
            src = None
            if fp32_too:
                src = frame.DeviceView(v, self.ibls[key[0]], outputs=outputs, solo_scratch=solo_scratch)
                self.dviews32[key] = src
            dv = frame.DeviceView(v, self.ibls[key[0]], gdtype=gdtype, ao_dtype=ao_dtype, hdr_dtype=hdr_dtype,
                                  outputs=outputs, solo_scratch=solo_scratch, src=src)
            self.dviews[key] = dv
            t = dv.batch_view(blur=True, keep_ao=False, keep_hdr=False)
            t.ldr = None
            self.templates[key] = t
        self.E = E

    def gbuffer_bytes(self) -> int:
        total = 0
        for dv in self.dviews.values():
            total += sum(t.numel() * t.element_size() for t in (dv.depth, dv.normal, dv.albedo, dv.rough, dv.metal))
        return total
