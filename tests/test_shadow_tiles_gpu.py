"""The tiled shadow-map form (EPB_MAP_TILES) on the device.

The tiling copy is checked element by element against the layout's
definition (built here with numpy index arithmetic), and shading with tiled
maps against shading with the same maps row-major: both read the same nine
texels per light, so the HDR images must be bitwise equal -- through the
single-view call and the batched form, with maps of odd, non-square and
minimal (3x3) sizes whose patches cross tile and map borders, and on the
1080p workload at full size.  Parity of the tiled path with the FP64 oracle
is covered by the parity tests, which upload maps in the tiled form."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2012_03325_amd import synth
from tests.parity_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_03325_amd import frame  # noqa: F401  (loads libepb.so, fails loudly)
    yield
    torch.cuda.synchronize()


def _tiles_by_definition(m: np.ndarray) -> np.ndarray:
    """Tile (p, q) element (j, i) at (p nx + q) 64 + 8 j + i holds
    m[6 p + j - 1, 6 q + i - 1], +inf outside the map; then 64 floats of +inf."""
    h, w = m.shape
    nx, ny = -(-w // 6), -(-h // 6)
    pad = np.full((6 * ny + 2, 6 * nx + 2), np.inf, np.float32)
    pad[1:h + 1, 1:w + 1] = m
    p = np.arange(ny)[:, None, None, None]
    q = np.arange(nx)[None, :, None, None]
    j = np.arange(8)[None, None, :, None]
    i = np.arange(8)[None, None, None, :]
    return np.concatenate([pad[6 * p + j, 6 * q + i].reshape(-1), np.full(64, np.inf, np.float32)])


@pytest.mark.parametrize("w,h", [(3, 3), (8, 8), (9, 9), (7, 5), (13, 11), (64, 48), (1000, 3), (2048, 2048)])
def test_tiling_matches_definition(w, h):
    from paper_2012_03325_amd import epb as E, frame
    log(f"[tiles] {w}x{h}")
    rng = np.random.default_rng(w * 100003 + h)
    m = rng.uniform(0.5, 30.0, (h, w)).astype(np.float32)
    m[rng.uniform(size=(h, w)) < 0.1] = np.inf
    n = E.epb_shadow_tiles_bytes(w, h)
    out = torch.full((n // 4 + 64,), -7.0, device="cuda")  # 64 guard floats after the form
    got = frame.tile_shadow_map(torch.from_numpy(m).cuda(), out=out)
    torch.cuda.synchronize()
    g = got.cpu().numpy()
    np.testing.assert_array_equal(g[: n // 4], _tiles_by_definition(m))
    assert (g[n // 4:] == -7.0).all()  # nothing written past the form


def _odd_map_view():
    """The 201x137 view with four lights whose depth maps are 3x3, 13x11,
    37x29 and 130x97 texels."""
    v = synth.config_reduced(201, 137, seed=7, shadow_size=0, env_size=16, ssao_n=16)
    scene = synth.make_spheres(np.random.default_rng(7), 48, True)
    for L, (w, h) in zip(v.lights, [(3, 3), (13, 11), (37, 29), (130, 97)]):
        L.shadow_cam = synth.look_at(L.pos, (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 90.0, w, h)
        L.shadow_map = synth.raycast(scene, L.shadow_cam, depth_only=True)["depth"]
    return v


def _ibl(view):
    from paper_2012_03325_amd import frame
    S = view.env.shape[1]
    ibl = frame.DeviceIBL(view.env, irr_size=8, irr_src_size=min(16, S), pref_size=min(32, S), pref_levels=4,
                          pref_samples=64, lut_size=32, lut_samples=64)
    ibl.precompute()
    return ibl


def _shade_both(view, ibl, **kw):
    from paper_2012_03325_amd import epb as E, frame
    dvs = [frame.DeviceView(view, ibl, shadow_layout=lay, **kw) for lay in (E.EPB_MAP_ROWS, E.EPB_MAP_TILES)]
    for dv in dvs:
        dv.ssao()
        dv.shade()
    torch.cuda.synchronize()
    return dvs


def test_tiled_shading_equals_row_major_odd_maps():
    from paper_2012_03325_amd import epb as E
    v = _odd_map_view()
    ibl = _ibl(v)
    for gdt in (E.EPB_F32, E.EPB_F16):
        log(f"[tiles] shade 201x137, odd maps, gdtype {gdt}")
        rows, tiles = _shade_both(v, ibl, gdtype=gdt, ao_dtype=gdt, hdr_dtype=gdt)
        assert tiles.lights[0].shadow_layout == E.EPB_MAP_TILES and rows.lights[0].shadow_layout == E.EPB_MAP_ROWS
        assert torch.equal(rows.hdr, tiles.hdr)
    # the maps matter: without them the image changes
    rows.lights = [type(L).from_buffer_copy(L) for L in rows.lights]
    for L in rows.lights:
        L.shadow_map = None
    rows.shade()
    torch.cuda.synchronize()
    assert not torch.equal(rows.hdr, tiles.hdr)


def test_tiled_shading_equals_row_major_batched():
    from paper_2012_03325_amd import epb as E, frame
    v = _odd_map_view()
    ibl = _ibl(v)
    log("[tiles] batched 201x137, odd maps")
    dvs = [frame.DeviceView(v, ibl, shadow_layout=lay, solo_scratch=False)
           for lay in (E.EPB_MAP_ROWS, E.EPB_MAP_TILES, E.EPB_MAP_ROWS, E.EPB_MAP_TILES)]
    b = frame.DeviceBatch(dvs, frame.make_schedule(2, 1, 1, 2))
    b.render()
    torch.cuda.synchronize()
    for dv in dvs[1:]:
        assert torch.equal(dvs[0].hdr, dv.hdr)
        assert torch.equal(dvs[0].ldr, dv.ldr)


def test_tiled_shading_equals_row_major_1080p():
    v = synth.config_1080p()
    from paper_2012_03325_amd import frame
    ibl = frame.DeviceIBL(v.env, **v.ibl)
    ibl.precompute()
    log("[tiles] shade 1920x1080, four 2048x2048 maps")
    rows, tiles = _shade_both(v, ibl)
    assert torch.equal(rows.hdr, tiles.hdr)


def test_shadow_cache_tiled_on_device():
    """The cache's tiled maps are the tiling of its row-major renders, refreshed
    when the scene moves."""
    from paper_2012_03325_amd import frame
    rng = np.random.default_rng(5)
    spheres = synth.make_spheres(rng, 64, True)
    scene = frame.DeviceScene(spheres)
    cams = [synth.look_at((6.0 * np.cos(a), 6.0, 6.0 * np.sin(a)), (0, 0, 0), (0, 1, 0), 90.0, 97, 83)
            for a in (0.8, 2.4)]
    cache = frame.ShadowCache(scene, tiles=True)
    log("[tiles] shadow cache")
    t0 = [t.clone() for t in cache.maps(cams)]
    torch.cuda.synchronize()
    for t, c in zip(t0, cams):
        ref = _tiles_by_definition(scene.render_depth(c).cpu().numpy())
        np.testing.assert_array_equal(t.cpu().numpy(), ref)
    cache.maps(cams)
    assert cache.renders == 2
    centers = spheres.centers.copy()
    centers[:, 1] += 0.25
    scene.move(centers=centers)
    t1 = cache.maps(cams)
    assert cache.renders == 4
    torch.cuda.synchronize()
    for t, c, old in zip(t1, cams, t0):
        np.testing.assert_array_equal(t.cpu().numpy(), _tiles_by_definition(scene.render_depth(c).cpu().numpy()))
        assert not torch.equal(t, old)
