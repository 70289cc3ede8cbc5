"""The serving loop on the GPU: requests of mixed resolutions arriving as a
Poisson stream are served by continuous batching, and every result equals the
same request rendered alone with the single-view calls, bitwise."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2012_03325_amd import synth
from tests.parity_util import log

pytestmark = pytest.mark.gpu

RES = ((64, 48), (130, 70), (33, 17), (256, 144))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_03325_amd import frame  # noqa: F401  (loads libepb.so, fails loudly)
    yield
    torch.cuda.synchronize()


def _resident(gdtype):
    from paper_2012_03325_amd import serve as S
    scenes = [synth.make_scene(500 + i, env_size=16, sphere_range=(16, 48),
                               ibl=dict(pref_samples=128, lut_size=32, lut_samples=128)) for i in range(3)]
    rng = np.random.default_rng(510)
    views = {}
    for i, sc in enumerate(scenes):
        pose = synth.orbit_camera(rng, 8, 8)
        for w, h in RES:
            cam = synth.look_at(pose.position, (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 45.0, w, h)
            views[(i, (w, h))] = synth.scene_view(sc, cam, f"scene{i}-{w}x{h}", index=i)
    return S.ResidentScenes(scenes, views, gdtype, outputs=True, solo_scratch=True)


@pytest.mark.parametrize("dtype,budget_slots", [("f16", 64), ("f32", 64), ("f16", 2)])
def test_each_result_same_alone_and_in_the_mix(dtype, budget_slots):
    from paper_2012_03325_amd import epb as E
    from paper_2012_03325_amd import serve as S
    gdt = E.EPB_F16 if dtype == "f16" else E.EPB_F32
    rs = _resident(gdt)
    ex = S.GpuExecutor(rs.templates, schedule=E.epb_schedule(2, 1, 1, 0), n_streams=2, max_inflight=3,
                       max_batch_views=16)
    budget = budget_slots * ex.footprint((256, 144))
    results = {}

    def on_done(r):  # copy the image out before its slot is reused
        results[r.rid] = r.slot["ldr"].cpu()

    srv = S.Server(ex, budget, max_batch_views=16, max_inflight=3, on_done=on_done)
    reqs = S.poisson_arrivals(4000.0, 520, 3, RES, count=150)
    log(f"[serve] {dtype}, budget {budget / 1e6:.1f} MB: {len(reqs)} requests")
    st = srv.run(reqs, S.RealClock())
    log(f"[serve] {st}")
    assert st["requests"] == len(reqs) and st["rejected"] == 0
    assert st["peak_reserved_bytes"] <= budget
    assert st["batches"] < len(reqs)  # requests were served in mixed batches
    alone = {}
    for key, dv in rs.dviews.items():
        dv.render()
        torch.cuda.synchronize()
        alone[key] = dv.ldr.cpu()
    for r in reqs:
        assert torch.equal(results[r.rid], alone[(r.scene, r.res)]), (r.rid, r.scene, r.res, r.batch)
    # a request served on its own through the server gives the same image too
    one = S.Server(ex, budget, on_done=on_done)
    r0 = S.Request(10_000, 1, 130, 70, 0.0)
    one.run([r0], S.RealClock())
    assert torch.equal(results[10_000], alone[(1, (130, 70))])


@pytest.mark.parametrize("dtype", ["f16", "f32"])
def test_requests_with_their_own_cameras(dtype):
    """Requests that carry a camera of their own: the server ray-casts their
    G-buffer on the device inside the request's slot, then shades it in the
    batch; each image equals that camera's G-buffer (same device ray cast)
    rendered alone with the single-view calls, bitwise."""
    from paper_2012_03325_amd import epb as E
    from paper_2012_03325_amd import frame
    from paper_2012_03325_amd import serve as S
    gdt = E.EPB_F16 if dtype == "f16" else E.EPB_F32
    rs = _resident(gdt)
    scenes = [synth.make_scene(500 + i, env_size=16, sphere_range=(16, 48),
                               ibl=dict(pref_samples=128, lut_size=32, lut_samples=128)) for i in range(3)]
    geometry = {i: frame.DeviceScene(sc.spheres) for i, sc in enumerate(scenes)}
    ex = S.GpuExecutor(rs.templates, schedule=E.epb_schedule(0, 0, 0, 0), n_streams=2, max_inflight=3,
                       max_batch_views=16, geometry=geometry)
    budget = 24 * ex.footprint((256, 144))
    results = {}

    def on_done(r):
        results[r.rid] = r.slot["ldr"].cpu()

    srv = S.Server(ex, budget, max_batch_views=16, max_inflight=3, on_done=on_done)
    reqs = S.poisson_arrivals(3000.0, 530, 3, RES, count=60)
    rng = np.random.default_rng(531)
    for r in reqs[::2]:  # every other request brings its own camera
        r.cam = synth.orbit_camera(rng, r.width, r.height)
    log(f"[serve-cam] {dtype}: {len(reqs)} requests, {len(reqs[::2])} with their own camera")
    st = srv.run(reqs, S.RealClock())
    log(f"[serve-cam] {st}")
    assert st["requests"] == len(reqs) and st["rejected"] == 0
    for r in reqs:
        if r.cam is None:
            dv = rs.dviews[(r.scene, r.res)]
        else:
            g = geometry[r.scene].render_gbuffer(r.cam, dtype=gdt)
            torch.cuda.synchronize()
            gb = {k: t.float().cpu().numpy() for k, t in g.items()}
            v = synth.scene_view(scenes[r.scene], r.cam, f"cam-{r.rid}", gbuf=gb, index=r.scene)
            dv = frame.DeviceView(v, rs.ibls[r.scene], gdtype=gdt, ao_dtype=gdt, hdr_dtype=gdt)
        dv.render()
        torch.cuda.synchronize()
        assert torch.equal(results[r.rid], dv.ldr.cpu()), (r.rid, r.scene, r.res, r.cam is not None)
