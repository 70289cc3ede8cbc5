"""GPU ray-cast G-buffers and depth maps against the FP64 oracle's cast.

The GPU intersects in double precision and stores float32 (or half): on every
pixel whose nearest surface is decided outside the oracle's tie margin, the
hit set, depth and attributes equal the oracle's values rounded to the stored
type (one ulp allowed for the normal, whose division order may differ)."""
import zlib

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2012_03325_amd import synth
from tests.parity_util import assert_interval, assert_ldr, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_03325_amd import frame  # noqa: F401  (loads libepb.so, fails loudly)
    yield
    torch.cuda.synchronize()


def _case(name):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    if name == "64-spheres-201x137":
        return synth.make_spheres(rng, 64, True), synth.look_at((0, 3.5, 8.5), (0, 0, 0), (0, 1, 0), 45, 201, 137)
    if name == "512-spheres-1080p":
        return synth.make_spheres(rng, 512, True), synth.look_at((0, 3.5, 8.5), (0, 0, 0), (0, 1, 0), 45, 1920, 1080)
    if name == "orbit-300-97x61":
        return synth.make_spheres(rng, 300, True), synth.orbit_camera(rng, 97, 61)
    if name == "inside-and-behind":  # the camera sits inside a sphere; others lie behind it
        sc = synth.make_spheres(rng, 40, True)
        sc.centers[0] = (0.0, 3.5, 8.5)
        sc.radii[0] = 0.3
        sc.centers[1] = (0.0, 3.5, 11.0)
        return sc, synth.look_at((0, 3.5, 8.5), (0, 0, 0), (0, 1, 0), 45, 64, 48)
    if name == "no-spheres-plane":
        return synth.make_spheres(rng, 0, True), synth.look_at((0, 2, 6), (0, 0, 0), (0, 1, 0), 60, 33, 17)
    if name == "65536-spheres-256x192":  # the largest scene the C ABI takes: 256 chunks of 256 spheres per tile
        return synth.make_spheres(rng, 65536, True), synth.orbit_camera(rng, 256, 192)
    if name == "1-sphere-no-plane-3x2":
        return synth.make_spheres(rng, 1, False), synth.look_at((0, 0.5, 3), (0, 0, 0), (0, 1, 0), 60, 3, 2)
    raise KeyError(name)


CASES = ["64-spheres-201x137", "512-spheres-1080p", "orbit-300-97x61", "inside-and-behind", "no-spheres-plane",
         "1-sphere-no-plane-3x2", "65536-spheres-256x192"]


def _ulps(a, b):
    a, b = np.asarray(a, np.float32), np.asarray(b, np.float32)
    ia = a.view(np.int32).astype(np.int64)
    ib = b.view(np.int32).astype(np.int64)
    ia = np.where(ia < 0, -(ia & 0x7FFFFFFF), ia)
    ib = np.where(ib < 0, -(ib & 0x7FFFFFFF), ib)
    return np.abs(ia - ib)


@pytest.mark.parametrize("name", CASES)
def test_raycast_gbuffer_parity(name):
    from paper_2012_03325_amd import frame as fr
    sc, cam = _case(name)
    ref = O.raycast(sc, cam)
    ok = ref["ambiguous"] == 0
    log(f"[raycast] {name}: {cam.width}x{cam.height}, {len(sc.radii)} spheres, {int((~ok).sum())} ambiguous px")
    ds = fr.DeviceScene(sc)
    g = {k: v.cpu().numpy() for k, v in ds.render_gbuffer(cam).items()}
    torch.cuda.synchronize()
    ref_depth = ref["depth"].astype(np.float32)
    hit = np.isfinite(ref_depth)
    assert np.array_equal(np.isfinite(g["depth"])[ok], hit[ok])
    both = ok & hit
    du = _ulps(g["depth"][both], ref_depth[both]) if both.any() else np.zeros(1)
    log(f"[raycast] {name}: depth max {int(du.max())} ulp, equal on {100 * (du == 0).mean():.3f}% of hits")
    assert du.max() <= 1
    for k in ("albedo", "roughness", "metalness"):
        assert np.array_equal(g[k][..., ok], ref[k].astype(np.float32)[..., ok]), k
    assert _ulps(g["normal"][:, ok], ref["normal"].astype(np.float32)[:, ok]).max() <= 1
    assert (g["normal"][:, ~hit & ok] == 0).all() and (g["albedo"][:, ~hit & ok] == 0).all()


def test_raycast_half_gbuffer_and_depth_maps():
    from paper_2012_03325_amd import epb as E
    from paper_2012_03325_amd import frame as fr
    sc, cam = _case("orbit-300-97x61")
    ref = O.raycast(sc, cam)
    ok = ref["ambiguous"] == 0
    ds = fr.DeviceScene(sc)
    g = {k: v.float().cpu().numpy() for k, v in ds.render_gbuffer(cam, dtype=E.EPB_F16).items()}
    fin = ok & np.isfinite(ref["depth"])
    assert np.array_equal(np.isfinite(g["depth"])[ok], np.isfinite(ref["depth"])[ok])
    assert _ulps(g["depth"][fin], ref["depth"].astype(np.float32)[fin]).max() <= 1
    for k in ("albedo", "roughness", "metalness"):
        assert np.array_equal(g[k][..., ok], ref[k].astype(np.float16).astype(np.float32)[..., ok]), k
    assert np.abs(g["normal"][:, ok] - ref["normal"][:, ok]).max() <= 2.0 ** -11
    # a light's depth map (2048^2, a 90 degree camera at the light)
    lc = synth.look_at((6 * np.cos(0.8), 6.0, 6 * np.sin(0.8)), (0, 0, 0), (0, 1, 0), 90.0, 2048, 2048)
    refd = O.raycast(sc, lc, attributes=False)
    okd = refd["ambiguous"] == 0
    d = ds.render_depth(lc).cpu().numpy()
    log(f"[raycast] depth map 2048^2: {int((~okd).sum())} ambiguous px")
    find = okd & np.isfinite(refd["depth"])
    assert np.array_equal(np.isfinite(d)[okd], np.isfinite(refd["depth"])[okd])
    assert _ulps(d[find], refd["depth"].astype(np.float32)[find]).max() <= 1
    assert (~okd).mean() < 1e-3


def test_raycast_then_render_matches_the_oracle_pipeline():
    """G-buffer and shadow maps cast on the GPU, then the whole pass on the GPU:
    the casts equal the oracle's away from its tie pixels (within one float32
    ulp), and the pass on the GPU-cast inputs matches the oracle's pass on those
    same inputs on every pixel."""
    import copy
    from paper_2012_03325_amd import frame as fr
    v = synth.config_reduced(160, 96, seed=21, shadow_size=256, env_size=16, ssao_n=16, n_spheres=40)
    rng = np.random.default_rng(21)
    scene = synth.make_spheres(rng, 40, True)  # the same draw config_reduced used
    rg = O.raycast(scene, v.cam)
    ds = fr.DeviceScene(scene)
    g = ds.render_gbuffer(v.cam)
    gpu_view = copy.deepcopy(v)
    gpu_view.gbuf = {k: t.cpu().numpy() for k, t in g.items()}
    for L in gpu_view.lights:
        L.shadow_map = ds.render_depth(L.shadow_cam).cpu().numpy()
    ok = rg["ambiguous"] == 0
    fin = ok & np.isfinite(rg["depth"])
    assert np.array_equal(np.isfinite(gpu_view.gbuf["depth"])[ok], np.isfinite(rg["depth"])[ok])
    assert _ulps(gpu_view.gbuf["depth"][fin], rg["depth"].astype(np.float32)[fin]).max() <= 1
    ref = O.render(gpu_view)
    ibl = fr.DeviceIBL(v.env, **v.ibl)
    ibl.precompute()
    dv = fr.DeviceView(gpu_view, ibl)
    dv.render()
    torch.cuda.synchronize()
    log("[raycast] cast + render 160x96")
    assert_interval("cast+render HDR", dv.hdr.cpu().numpy(), *ref["hdr"])
    assert_ldr("cast+render LDR", dv.ldr.cpu().numpy(), *ref["ldr"])


def test_shadow_cache_on_device():
    """Cached depth maps equal fresh renders; a moved sphere re-renders every
    map, a moved light only its own, an unchanged frame none."""
    from paper_2012_03325_amd import frame
    rng = np.random.default_rng(5)
    spheres = synth.make_spheres(rng, 64, True)
    scene = frame.DeviceScene(spheres)
    cams = [synth.look_at((6.0 * np.cos(a), 6.0, 6.0 * np.sin(a)), (0, 0, 0), (0, 1, 0), 90.0, 96, 96)
            for a in (0.8, 2.4, 3.9, 5.5)]
    cache = frame.ShadowCache(scene)
    log("[shadow-cache] first frame")
    m0 = [m.clone() for m in cache.maps(cams)]
    torch.cuda.synchronize()
    for m, c in zip(m0, cams):
        assert torch.equal(m, scene.render_depth(c))
    cache.maps(cams)
    assert cache.renders == 4
    cams[1] = synth.look_at((2.0, 7.0, -5.0), (0, 0, 0), (0, 1, 0), 90.0, 96, 96)
    m1 = cache.maps(cams)
    assert cache.renders == 5
    torch.cuda.synchronize()
    assert torch.equal(m1[1], scene.render_depth(cams[1]))
    centers = spheres.centers.copy()
    centers[:, 1] += 0.25  # lift every sphere
    scene.move(centers=centers)
    m2 = [m.clone() for m in cache.maps(cams)]
    assert cache.renders == 9
    torch.cuda.synchronize()
    for m, c, old in zip(m2, cams, m0):
        assert torch.equal(m, scene.render_depth(c))
    assert not torch.equal(m2[0], m0[0])
