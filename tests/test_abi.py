"""The C ABI on the CPU: the library loads, exports every entry point the
header declares, its structs have the header's layout, and argument
validation returns the documented status before anything is enqueued (no
compute call is made here: every case fails validation)."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2012_03325_amd import epb as E

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "epb.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(epb_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_entry_point():
    names = _declared_functions()
    assert set(E.ENTRY_POINTS) <= set(names)
    lib = C.CDLL(E.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert {"epb_precompute_ibl", "epb_ssao", "epb_shade", "epb_bloom_tonemap"} <= set(names)


def test_struct_layout_matches_header(tmp_path):
    """Compile a probe against the header with gcc and compare sizes and field
    offsets with the ctypes mirrors of the binding."""
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "epb.h"', "int main(void){"]
    for sname, st in E.STRUCTS.items():
        lines.append(f'printf("{sname} __sizeof__ %zu\\n", sizeof({sname}));')
        for fname, _ in st._fields_:
            lines.append(f'printf("{sname} {fname} %zu\\n", offsetof({sname}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    seen = {}
    for line in out.splitlines():
        a, b, v = line.split()
        seen[(a, b)] = int(v)
    for sname, st in E.STRUCTS.items():
        assert seen[(sname, "__sizeof__")] == C.sizeof(st), sname
        for fname, _ in st._fields_:
            assert seen[(sname, fname)] == getattr(st, fname).offset, (sname, fname)


def test_status_strings():
    for code in range(0, -8, -1):
        s = E.epb_status_str(code)
        assert s and s != "unknown status"
    assert E.epb_status_str(-99) == "unknown status"


def test_scratch_sizes():
    post = E.epb_post_params(6, 1.0, 0.04, 1.0, 2.2)
    prev = 0
    for n in (8, 64, 256, 1080, 2160):
        b = E.epb_scratch_bytes(E.EPB_OP_BLOOM_TONEMAP, n, n, post)
        s = E.epb_scratch_bytes(E.EPB_OP_SSAO, n, n, None)
        assert b > 0 and s >= 2 * ((n + 1) // 2) ** 2 * 4
        assert b >= prev
        prev = b
    assert E.epb_scratch_bytes(E.EPB_OP_SSAO, 0, 10, None) == 0
    assert E.epb_scratch_bytes(99, 10, 10, None) == 0
    bad = E.epb_post_params(7, 1.0, 0.04, 1.0, 2.2)
    assert E.epb_scratch_bytes(E.EPB_OP_BLOOM_TONEMAP, 10, 10, bad) == 0
    ip = E.epb_ibl_params(32, 64, 128, 5, 1024, 256, 1024)
    assert E.epb_scratch_bytes(E.EPB_OP_PRECOMPUTE_IBL, 512, 512, ip) > 0
    assert E.epb_scratch_bytes(E.EPB_OP_PRECOMPUTE_IBL, 96, 96, ip) == 0  # 96 / 64 not a power of 2


# A fake but 16-byte-aligned device address: only ever seen by validation,
# since every call below fails before launching.
FAKE = 0x7F0000001000


def _cam(w=64, h=48):
    return E.make_camera([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], 50, 50, w / 2, h / 2, w, h)


def _gbuf(w=64, h=48, dt=E.EPB_F32, base=FAKE):
    return E.epb_gbuffer(w, h, dt, base, base, base, base, base)


def test_ssao_validation():
    cam = _cam()
    p = E.epb_ssao_params(16, FAKE, FAKE, 0.5, 0.025, 0.1, 1, E.EPB_F32)
    call = lambda g=_gbuf(), c=cam, pp=p, out=FAKE, sc=FAKE, n=1 << 30: \
        E.lib.epb_ssao(C.byref(g), C.byref(c), C.byref(pp), out, sc, n, None)
    assert E.lib.epb_ssao(None, C.byref(cam), C.byref(p), FAKE, FAKE, 1 << 30, None) == E.EPB_ERR_NULL
    assert call(out=None) == E.EPB_ERR_NULL
    assert call(g=_gbuf(w=63)) == E.EPB_ERR_SIZE
    assert call(c=_cam(0, 48), g=_gbuf(0, 48)) == E.EPB_ERR_SIZE
    assert call(g=_gbuf(dt=7)) == E.EPB_ERR_DTYPE
    assert call(g=_gbuf(base=FAKE + 4)) == E.EPB_ERR_ALIGN
    assert call(out=FAKE + 8) == E.EPB_ERR_ALIGN
    # 16-byte alignment is the rule (not 256): such planes pass on to the next check
    assert call(g=_gbuf(base=FAKE + 16), out=FAKE + 48, sc=None) == E.EPB_ERR_SCRATCH
    assert call(sc=None) == E.EPB_ERR_SCRATCH
    assert call(n=16) == E.EPB_ERR_SCRATCH
    for bad in (dict(n_samples=0), dict(n_samples=257), dict(radius=0.0), dict(radius=float("nan")),
                dict(blur_tau=0.0)):
        q = E.epb_ssao_params(16, FAKE, FAKE, 0.5, 0.025, 0.1, 1, E.EPB_F32)
        for k, v in bad.items():
            setattr(q, k, v)
        assert call(pp=q) == E.EPB_ERR_PARAM, bad
    q = E.epb_ssao_params(16, None, FAKE, 0.5, 0.025, 0.1, 1, E.EPB_F32)
    assert call(pp=q) == E.EPB_ERR_NULL
    c2 = _cam()
    c2.fx = -1.0
    assert call(c=c2) == E.EPB_ERR_PARAM


def test_ssao_static_validation():
    """The allocation-free SSAO call: missing pointers and images whose scratch
    exceeds the library's own array fail before any device query; 3840x2160
    fits."""
    p = E.epb_ssao_params(16, FAKE, FAKE, 0.5, 0.025, 0.1, 1, E.EPB_F32)
    call = lambda g, c, out=FAKE: E.lib.epb_ssao_static(C.byref(g), C.byref(c), C.byref(p), out, None)
    assert E.lib.epb_ssao_static(None, C.byref(_cam()), C.byref(p), FAKE, None) == E.EPB_ERR_NULL
    assert call(_gbuf(), _cam(), out=None) == E.EPB_ERR_NULL
    assert call(_gbuf(0, 48), _cam(0, 48)) == E.EPB_ERR_SIZE
    assert call(_gbuf(4096, 4096), _cam(4096, 4096)) == E.EPB_ERR_SIZE
    cap = E.EPB_SSAO_STATIC_SCRATCH_BYTES
    assert E.epb_scratch_bytes(E.EPB_OP_SSAO, 3840, 2160, None) <= cap
    w = 3840
    while E.epb_scratch_bytes(E.EPB_OP_SSAO, w, 2160, None) <= cap:
        w += 2
    assert call(_gbuf(w, 2160), _cam(w, 2160)) == E.EPB_ERR_SIZE


def test_shade_validation():
    cam = _cam()
    cube = E.epb_cube(8, 1, FAKE)
    maps = E.epb_ibl_maps(E.epb_cube(4, 1, FAKE), E.epb_cube(8, 3, FAKE), FAKE, 16)
    lights = (E.epb_light * 9)()

    def call(g=None, c=cam, n=0, mp=maps, env=cube, hdr=FAKE, hdt=E.EPB_F32, ao=FAKE):
        g = g or _gbuf()
        return E.lib.epb_shade(C.byref(g), C.byref(c), ao, E.EPB_F32, lights, n, C.byref(mp),
                               C.byref(env), hdr, hdt, None)

    assert call(hdr=None) == E.EPB_ERR_NULL
    assert call(n=9) == E.EPB_ERR_PARAM
    assert call(n=-1) == E.EPB_ERR_PARAM
    assert call(hdt=5) == E.EPB_ERR_DTYPE
    assert call(ao=FAKE + 2) == E.EPB_ERR_ALIGN
    assert call(env=E.epb_cube(8, 1, None)) == E.EPB_ERR_NULL
    assert call(env=E.epb_cube(0, 1, FAKE)) == E.EPB_ERR_SIZE
    assert call(mp=E.epb_ibl_maps(E.epb_cube(4, 1, FAKE), E.epb_cube(4, 4, FAKE), FAKE, 16)) \
        == E.EPB_ERR_SIZE  # 4 >> 3 == 0
    assert call(mp=E.epb_ibl_maps(E.epb_cube(4, 1, FAKE), E.epb_cube(8, 3, FAKE), None, 16)) \
        == E.EPB_ERR_NULL
    bad_light = (E.epb_light * 1)()
    bad_light[0].intensity = float("inf")
    g = _gbuf()
    assert E.lib.epb_shade(C.byref(g), C.byref(cam), FAKE, E.EPB_F32, bad_light, 1, C.byref(maps),
                           C.byref(cube), FAKE, E.EPB_F32, None) == E.EPB_ERR_PARAM
    unaligned_map = (E.epb_light * 1)()
    unaligned_map[0].intensity = 1.0
    unaligned_map[0].shadow_map = FAKE + 4
    assert E.lib.epb_shade(C.byref(g), C.byref(cam), FAKE, E.EPB_F32, unaligned_map, 1,
                           C.byref(maps), C.byref(cube), FAKE, E.EPB_F32, None) == E.EPB_ERR_ALIGN
    bad_layout = (E.epb_light * 1)()
    bad_layout[0].intensity = 1.0
    bad_layout[0].shadow_map = FAKE
    bad_layout[0].shadow_cam = _cam()
    bad_layout[0].shadow_layout = 2
    assert E.lib.epb_shade(C.byref(g), C.byref(cam), FAKE, E.EPB_F32, bad_layout, 1,
                           C.byref(maps), C.byref(cube), FAKE, E.EPB_F32, None) == E.EPB_ERR_PARAM


def test_shadow_tiles_sizes_and_validation():
    """Tiles of 6x6 texels of the map padded by one texel of +inf, stored as
    8x8 floats: ceil(w / 6) x ceil(h / 6) tiles of 256 bytes and one more."""
    nb = E.epb_shadow_tiles_bytes
    assert nb(2048, 2048) == (342 * 342 + 1) * 256
    assert nb(3, 3) == nb(6, 6) == 2 * 256
    assert nb(7, 6) == 3 * 256 and nb(7, 7) == 5 * 256
    assert nb(1920, 1080) == (320 * 180 + 1) * 256
    assert nb(16384, 16384) == (2731 * 2731 + 1) * 256 < 2 ** 32
    assert nb(2, 9) == nb(9, 2) == nb(16385, 9) == nb(-1, 9) == 0
    need = nb(64, 48)

    def call(m=FAKE, w=64, h=48, t=FAKE + (1 << 20), n=need):
        return E.lib.epb_shadow_tiles(m, w, h, t, n, None)

    assert call(m=None) == E.EPB_ERR_NULL
    assert call(t=None) == E.EPB_ERR_NULL
    assert call(w=2) == E.EPB_ERR_SIZE
    assert call(h=16385) == E.EPB_ERR_SIZE
    assert call(n=need - 1) == E.EPB_ERR_SIZE
    assert call(m=FAKE + 4) == E.EPB_ERR_ALIGN
    assert call(t=FAKE + 8 + (1 << 20)) == E.EPB_ERR_ALIGN
    assert call(t=FAKE + 64 * 48 * 4 - 16) == E.EPB_ERR_PARAM  # tiles start inside the map
    assert call(t=FAKE - need + 16) == E.EPB_ERR_PARAM  # tiles end inside the map


def test_bloom_tonemap_validation():
    p = E.epb_post_params(6, 1.0, 0.04, 1.0, 2.2)
    need = E.epb_scratch_bytes(E.EPB_OP_BLOOM_TONEMAP, 64, 48, p)

    def call(hdr=FAKE, dt=E.EPB_F32, w=64, h=48, pp=p, out=FAKE, sc=FAKE, n=need):
        return E.lib.epb_bloom_tonemap(hdr, dt, w, h, C.byref(pp), out, sc, n, None)

    assert call(hdr=None) == E.EPB_ERR_NULL
    assert call(w=0) == E.EPB_ERR_SIZE
    assert call(h=20000) == E.EPB_ERR_SIZE
    assert call(dt=3) == E.EPB_ERR_DTYPE
    assert call(pp=E.epb_post_params(0, 1.0, 0.04, 1.0, 2.2)) == E.EPB_ERR_PARAM
    assert call(pp=E.epb_post_params(6, 1.0, 0.04, 0.0, 2.2)) == E.EPB_ERR_PARAM
    assert call(pp=E.epb_post_params(6, 1.0, 0.04, 1.0, float("nan"))) == E.EPB_ERR_PARAM
    assert call(pp=E.epb_post_params(6, 1.0, 0.04, 1.0, 2.2, E.EPB_F32, 2)) == E.EPB_ERR_PARAM
    assert call(pp=E.epb_post_params(6, 1.0, 0.04, 1.0, 2.2, E.EPB_F32, -1)) == E.EPB_ERR_PARAM
    assert call(out=FAKE + 1) == E.EPB_ERR_ALIGN
    assert call(n=need - 1) == E.EPB_ERR_SCRATCH


def test_shade_post_validation():
    """The fused call validates both halves (shading, then bloom and tone
    mapping) before it enqueues anything."""
    cam = _cam()
    cube = E.epb_cube(8, 1, FAKE)
    maps = E.epb_ibl_maps(E.epb_cube(4, 1, FAKE), E.epb_cube(8, 3, FAKE), FAKE, 16)
    lights = (E.epb_light * 1)()
    p = E.epb_post_params(6, 1.0, 0.04, 1.0, 2.2)
    need = E.epb_scratch_bytes(E.EPB_OP_BLOOM_TONEMAP, 64, 48, p)

    def call(hdr=FAKE, hdt=E.EPB_F32, pp=p, out=FAKE, sc=FAKE, n=need, env=cube):
        g = _gbuf()
        return E.lib.epb_shade_post(C.byref(g), C.byref(cam), FAKE, E.EPB_F32, lights, 0, C.byref(maps),
                                    C.byref(env), hdr, hdt, C.byref(pp), out, sc, n, None)

    assert call(hdr=None) == E.EPB_ERR_NULL
    assert call(hdt=5) == E.EPB_ERR_DTYPE
    assert call(env=E.epb_cube(0, 1, FAKE)) == E.EPB_ERR_SIZE
    assert call(out=None) == E.EPB_ERR_NULL
    assert call(sc=None) == E.EPB_ERR_SCRATCH
    assert call(n=need - 1) == E.EPB_ERR_SCRATCH
    assert call(out=FAKE + 1) == E.EPB_ERR_ALIGN
    assert call(pp=E.epb_post_params(0, 1.0, 0.04, 1.0, 2.2)) == E.EPB_ERR_PARAM
    assert call(pp=E.epb_post_params(6, 1.0, 0.04, 1.0, 2.2, 7)) == E.EPB_ERR_DTYPE
    assert E.lib.epb_shade_post(None, C.byref(cam), FAKE, E.EPB_F32, lights, 0, C.byref(maps), C.byref(cube),
                                FAKE, E.EPB_F32, C.byref(p), FAKE, FAKE, need, None) == E.EPB_ERR_NULL


def test_precompute_ibl_validation():
    ip = E.epb_ibl_params(8, 16, 16, 3, 64, 16, 64)
    need = E.epb_scratch_bytes(E.EPB_OP_PRECOMPUTE_IBL, 32, 32, ip)
    env = E.epb_cube(32, 1, FAKE)
    maps = E.epb_ibl_maps(E.epb_cube(8, 1, FAKE), E.epb_cube(16, 3, FAKE), FAKE, 16)

    def call(e=env, p=ip, m=maps, sc=FAKE, n=need):
        return E.lib.epb_precompute_ibl(C.byref(e), C.byref(p), C.byref(m), sc, n, None)

    assert call(e=E.epb_cube(32, 1, None)) == E.EPB_ERR_NULL
    assert call(e=E.epb_cube(48, 1, FAKE)) == E.EPB_ERR_SIZE  # 48 / 16 not a power of 2
    assert call(m=E.epb_ibl_maps(E.epb_cube(8, 1, FAKE), E.epb_cube(32, 3, FAKE), FAKE, 16)) \
        == E.EPB_ERR_SIZE  # prefiltered base must be min(32, 16)
    assert call(p=E.epb_ibl_params(8, 16, 16, 3, 0, 16, 64)) == E.EPB_ERR_PARAM
    assert call(n=need - 1) == E.EPB_ERR_SCRATCH
    assert call(sc=FAKE + 8) == E.EPB_ERR_ALIGN


# ---------------------------------------------------------------------------
# batched form: building the table is host work, checked here with fake
# device addresses (nothing is launched)
# ---------------------------------------------------------------------------
def _cdiv(a, b):
    return -(-a // b)


class _Batch:
    """Host structs of a batch of fake-address views, kept alive together."""

    def __init__(self, sizes, gdtypes=None, blurs=None, levels=6, keep=True):
        self.env = E.epb_cube(8, 1, FAKE)
        self.maps = E.epb_ibl_maps(E.epb_cube(4, 1, FAKE), E.epb_cube(8, 3, FAKE), FAKE, 16)
        self.post = E.epb_post_params(levels, 1.0, 0.04, 1.0, 2.2, E.EPB_F32)
        self.ssao = []
        self.lights = (E.epb_light * 1)()
        self.lights[0].intensity = 1.0
        self.views = []
        for k, (w, h) in enumerate(sizes):
            p = E.epb_ssao_params(16, FAKE, FAKE, 0.5, 0.025, 0.1,
                                  blurs[k] if blurs else 1, E.EPB_F32)
            self.ssao.append(p)
            v = E.epb_view()
            v.gbuf = _gbuf(w, h, gdtypes[k] if gdtypes else E.EPB_F32)
            v.cam = _cam(w, h)
            v.lights = C.addressof(self.lights)
            v.n_lights = 1
            v.ibl = C.addressof(self.maps)
            v.env = C.addressof(self.env)
            v.ssao = C.addressof(p)
            v.post = C.addressof(self.post)
            v.hdr_dtype = E.EPB_F32
            v.ao = FAKE if keep else None
            v.hdr = FAKE if keep else None
            v.ldr = FAKE
            self.views.append(v)
        self.arr = (E.epb_view * len(self.views))(*self.views)

    def build(self, n=None, sched=None, sc=FAKE, sc_bytes=None, table_bytes=None):
        n = len(self.views) if n is None else n
        tb = E.lib.epb_batch_table_bytes(max(n, 1)) if table_bytes is None else table_bytes
        self.table = (C.c_uint8 * max(tb, 16))()
        need = E.lib.epb_batch_scratch_bytes(C.addressof(self.arr), len(self.views))
        return E.lib.epb_batch_build(C.addressof(self.arr), n, C.addressof(sched) if sched else None,
                                     sc, need if sc_bytes is None else sc_bytes,
                                     C.addressof(self.table), tb)


def _expected_items(w, h, levels=6):
    wh, hh = (w + 1) // 2, (h + 1) // 2
    lw, lh, blur_items = w, h, 0
    dims = []
    for _ in range(1, levels):
        lw, lh = (lw + 1) // 2, (lh + 1) // 2
        dims.append((lw, lh))
        blur_items += _cdiv(lw, 32) * _cdiv(lh, 16)
    down = _cdiv(dims[0][0], 16) * _cdiv(dims[0][1], 16) if dims else 0
    return [hh * _cdiv(wh, 256), _cdiv(wh, 16) * _cdiv(hh, 8), _cdiv(wh, 16) * _cdiv(hh, 8),
            _cdiv(w, 32) * _cdiv(h, 8), down, blur_items, _cdiv(w, 64) * _cdiv(h, 8)]


def test_batch_sizes():
    assert E.epb_batch_table_bytes(0) == 0
    assert E.epb_batch_table_bytes(E.EPB_MAX_BATCH_VIEWS + 1) == 0
    assert 0 < E.epb_batch_table_bytes(1) < E.epb_batch_table_bytes(256)
    kept = _Batch([(64, 48), (33, 17)])
    free = _Batch([(64, 48), (33, 17)], keep=False)
    a = E.lib.epb_batch_scratch_bytes(C.addressof(kept.arr), 2)
    b = E.lib.epb_batch_scratch_bytes(C.addressof(free.arr), 2)
    ssao = sum(E.epb_scratch_bytes(E.EPB_OP_SSAO, w, h) for w, h in ((64, 48), (33, 17)))
    post = sum(E.epb_scratch_bytes(E.EPB_OP_BLOOM_TONEMAP, w, h, kept.post) for w, h in ((64, 48), (33, 17)))
    assert a >= ssao + post
    # AO and HDR images kept in scratch when the view leaves them NULL
    assert b >= a + 3 * 4 * (64 * 48 + 33 * 17) + 4 * (32 * 24 + 17 * 9)
    assert E.lib.epb_batch_scratch_bytes(None, 2) == 0
    assert E.lib.epb_batch_scratch_bytes(C.addressof(kept.arr), 0) == 0


def test_batch_build_table():
    sizes = [(64, 48), (33, 17), (3, 2), (1920, 1080)]
    b = _Batch(sizes)
    assert b.build() == E.EPB_OK
    words = list(C.cast(b.table, C.POINTER(C.c_int32 * 33)).contents)
    assert words[0] == 0x45504232 and words[1] == len(sizes)
    totals = words[13:20]
    exp = [sum(col) for col in zip(*[_expected_items(w, h) for w, h in sizes])]
    assert totals == exp
    assert words[12] == 0 and words[20] == 0  # no fused bloom, stage launches
    assert b.build(sched=E.epb_schedule(0, 1, 1, 2, 0, 0, 1)) == E.EPB_OK
    words = list(C.cast(b.table, C.POINTER(C.c_int32 * 33)).contents)
    assert words[12] == 1 and words[13:20] != [0] * 7


def _persistent_items(w, h, levels=6):
    """Tiles of the persistent launch: SSAO raw and blur on 16x16 texels, the
    composite as groups of four 64x8 tiles; the other stages as above."""
    it = _expected_items(w, h, levels)
    wh, hh = (w + 1) // 2, (h + 1) // 2
    it[1] = it[2] = _cdiv(wh, 16) * _cdiv(hh, 16)
    it[6] = _cdiv(it[6], 4)
    return it


@pytest.mark.parametrize("chunk", [1, 7, 64])
def test_batch_build_persistent_table(chunk):
    """Header of a persistent table: work items per stage, chunks of `chunk`
    tiles per view and stage, the first chunk of each stage, the wait limit."""
    sizes = [(64, 48), (33, 17), (3, 2), (1920, 1080)]
    b = _Batch(sizes)
    assert b.build(sched=E.epb_schedule(0, 0, 0, 0, chunk, 0)) == E.EPB_OK
    words = list(C.cast(b.table, C.POINTER(C.c_int32 * 33)).contents)
    items = [_persistent_items(w, h) for w, h in sizes]
    assert words[13:20] == [sum(col) for col in zip(*items)]
    persistent, k, limit, gate, total = words[20:25]
    assert (persistent, k, limit, gate) == (1, chunk, 1 << 22, 1)
    per_stage = [sum(_cdiv(n, chunk) for n in col) for col in zip(*items)]
    first = [sum(per_stage[:s]) for s in range(8)]
    assert words[25:33] == first and total == sum(per_stage)
    assert b.build(sched=E.epb_schedule(0, 0, 0, 0, chunk, -50)) == E.EPB_OK  # error-path test mode
    words = list(C.cast(b.table, C.POINTER(C.c_int32 * 33)).contents)
    assert words[22:24] == [50, 0]


def test_batch_status_validation():
    junk = (C.c_uint8 * 4096)()
    assert E.lib.epb_batch_status(C.addressof(junk), FAKE, None) == E.EPB_ERR_PARAM
    assert E.lib.epb_batch_status(None, FAKE, None) == E.EPB_ERR_NULL
    b = _Batch([(64, 48)])
    assert b.build() == E.EPB_OK
    assert E.lib.epb_batch_status(C.addressof(b.table), None, None) == E.EPB_ERR_NULL
    assert E.lib.epb_batch_status(C.addressof(b.table), FAKE + 8, None) == E.EPB_ERR_ALIGN
    # stage launches never wait: nothing to read back
    assert E.lib.epb_batch_status(C.addressof(b.table), FAKE, None) == E.EPB_OK
    assert E.epb_status_str(E.EPB_ERR_TIMEOUT).startswith("a dependency wait")


def test_batch_build_validation():
    b = _Batch([(64, 48), (33, 17)])
    assert b.build(n=0) == E.EPB_ERR_SIZE
    assert b.build(sc=None) == E.EPB_ERR_SCRATCH
    assert b.build(sc_bytes=16) == E.EPB_ERR_SCRATCH
    assert b.build(sc=FAKE + 4) == E.EPB_ERR_ALIGN
    assert b.build(table_bytes=64) == E.EPB_ERR_SIZE
    for bad in (E.epb_schedule(3, 0, 0, 0), E.epb_schedule(0, 3, 0, 0), E.epb_schedule(0, 0, 2, 0),
                E.epb_schedule(0, 0, 0, 65), E.epb_schedule(-1, 0, 0, 0), E.epb_schedule(0, 0, 0, 0, -1),
                E.epb_schedule(0, 0, 0, 0, E.EPB_MAX_PERSISTENT_CHUNK + 1),
                E.epb_schedule(0, 0, 0, 0, 0, 0, 2), E.epb_schedule(1, 0, 0, 0, 0, 0, 1),
                E.epb_schedule(2, 0, 0, 0, 0, 0, 1), E.epb_schedule(0, 0, 0, 0, 16, 0, 1)):
        assert b.build(sched=bad) == E.EPB_ERR_PARAM
    assert b.build(sched=E.epb_schedule(2, 1, 1, 4)) == E.EPB_OK
    assert _Batch([(64, 48), (33, 17)], gdtypes=[E.EPB_F32, E.EPB_F16]).build() == E.EPB_ERR_DTYPE
    # the persistent launch takes one storage type throughout (these views: FP16 G-buffer, FP32 rest)
    mixed = _Batch([(64, 48), (33, 17)], gdtypes=[E.EPB_F16, E.EPB_F16])
    assert mixed.build() == E.EPB_OK
    assert mixed.build(sched=E.epb_schedule(0, 0, 0, 0, 16)) == E.EPB_ERR_DTYPE
    assert _Batch([(64, 48), (33, 17)], blurs=[1, 0]).build() == E.EPB_ERR_PARAM
    # a view failing the single-view checks fails the batch with the same status
    bad = _Batch([(64, 48), (33, 17)])
    bad.arr[1].gbuf.width = 32
    assert bad.build() == E.EPB_ERR_SIZE
    bad = _Batch([(64, 48), (33, 17)])
    bad.arr[0].ldr = None
    assert bad.build() == E.EPB_ERR_NULL


def test_views_with_their_own_scratch():
    b = _Batch([(64, 48), (33, 17)])
    per = [E.lib.epb_view_scratch_bytes(C.addressof(b.arr[k])) for k in range(2)]
    assert all(p > 0 for p in per)
    assert E.lib.epb_batch_scratch_bytes(C.addressof(b.arr), 2) == sum(per)
    b.arr[0].scratch = FAKE
    assert E.lib.epb_batch_scratch_bytes(C.addressof(b.arr), 2) == per[1]
    b.arr[1].scratch = FAKE + 4096
    assert E.lib.epb_batch_scratch_bytes(C.addressof(b.arr), 2) == 0
    assert b.build(sc=None, sc_bytes=0) == E.EPB_OK  # no batch scratch needed
    b.arr[1].scratch = FAKE + 8
    assert b.build(sc=None, sc_bytes=0) == E.EPB_ERR_ALIGN
    assert E.lib.epb_view_scratch_bytes(None) == 0


def test_render_batch_rejects_foreign_tables():
    junk = (C.c_uint8 * 4096)()
    assert E.lib.epb_render_batch(C.addressof(junk), FAKE, None) == E.EPB_ERR_PARAM
    assert E.lib.epb_render_batch(None, FAKE, None) == E.EPB_ERR_NULL
    b = _Batch([(64, 48)])
    assert b.build() == E.EPB_OK
    assert E.lib.epb_render_batch(C.addressof(b.table), None, None) == E.EPB_ERR_NULL
    assert E.lib.epb_render_batch(C.addressof(b.table), FAKE + 8, None) == E.EPB_ERR_ALIGN


def test_raycast_validation():
    pa = (C.c_float * 3)(0.5, 0.5, 0.5)
    sc = E.epb_sphere_scene(4, FAKE, FAKE, FAKE, FAKE, FAKE, 1, pa, 0.6, 0.0)
    cam = _cam(64, 48)
    need = E.epb_scratch_bytes(E.EPB_OP_RAYCAST, 64, 48, sc)
    assert need >= 4 * 16

    def call(s=sc, c=cam, g=None, scr=FAKE, n=need):
        g = g or _gbuf(64, 48)
        return E.lib.epb_raycast(C.byref(s), C.byref(c), C.byref(g), scr, n, None)

    assert E.lib.epb_raycast(None, C.byref(cam), C.byref(_gbuf()), FAKE, need, None) == E.EPB_ERR_NULL
    assert call(g=_gbuf(32, 48)) == E.EPB_ERR_SIZE
    assert call(s=E.epb_sphere_scene(-1, FAKE, FAKE, FAKE, FAKE, FAKE, 0, pa, 0.6, 0.0)) == E.EPB_ERR_SIZE
    assert call(s=E.epb_sphere_scene(E.EPB_MAX_SPHERES + 1, FAKE, FAKE, FAKE, FAKE, FAKE, 0, pa, 0.6, 0.0)) \
        == E.EPB_ERR_SIZE
    assert call(s=E.epb_sphere_scene(4, None, FAKE, FAKE, FAKE, FAKE, 0, pa, 0.6, 0.0)) == E.EPB_ERR_NULL
    assert call(s=E.epb_sphere_scene(4, FAKE + 8, FAKE, FAKE, FAKE, FAKE, 0, pa, 0.6, 0.0)) == E.EPB_ERR_ALIGN
    assert call(s=E.epb_sphere_scene(4, FAKE, FAKE, FAKE, FAKE, FAKE, 0, pa, float("nan"), 0.0)) == E.EPB_ERR_PARAM
    w = _gbuf(64, 48)
    w.weight = FAKE
    assert call(g=w) == E.EPB_ERR_PARAM
    half = _gbuf(64, 48)
    half.albedo = None
    assert call(g=half) == E.EPB_ERR_NULL
    assert call(n=need - 1) == E.EPB_ERR_SCRATCH
    assert call(scr=None) == E.EPB_ERR_SCRATCH
    assert call(scr=FAKE + 4) == E.EPB_ERR_ALIGN
    # no spheres: no sphere arrays needed
    empty = E.epb_sphere_scene(0, None, None, None, None, None, 1, pa, 0.6, 0.0)
    assert E.epb_scratch_bytes(E.EPB_OP_RAYCAST, 64, 48, empty) > 0


def test_edl_validation():
    cam = _cam(64, 48)
    ok = E.epb_edl_params(2, 8, 6.0, 1000.0)
    env = E.epb_cube(8, 1, FAKE)

    def call(depth=FAKE, color=FAKE, cd=E.EPB_F32, c=cam, ao=None, ad=E.EPB_F32, p=ok, e=env, hdr=FAKE,
             hd=E.EPB_F32):
        return E.lib.epb_edl(depth, color, cd, C.byref(c) if c is not None else None, ao, ad,
                             C.byref(p) if p is not None else None, C.byref(e) if e is not None else None,
                             hdr, hd, None)

    assert call(depth=None) == E.EPB_ERR_NULL
    assert call(color=None) == E.EPB_ERR_NULL
    assert call(c=None) == E.EPB_ERR_NULL
    assert call(p=None) == E.EPB_ERR_NULL
    assert call(hdr=None) == E.EPB_ERR_NULL
    assert call(c=_cam(0, 48)) == E.EPB_ERR_SIZE
    assert call(cd=7) == E.EPB_ERR_DTYPE
    assert call(hd=2) == E.EPB_ERR_DTYPE
    for bad in (E.epb_edl_params(0, 8, 6.0, 1000.0), E.epb_edl_params(E.EPB_MAX_EDL_RADIUS + 1, 8, 6.0, 1000.0),
                E.epb_edl_params(2, 0, 6.0, 1000.0), E.epb_edl_params(2, E.EPB_MAX_EDL_DIRS + 1, 6.0, 1000.0),
                E.epb_edl_params(2, 8, -1.0, 1000.0), E.epb_edl_params(2, 8, float("inf"), 1000.0),
                E.epb_edl_params(2, 8, 6.0, 0.0), E.epb_edl_params(2, 8, 6.0, float("nan"))):
        assert call(p=bad) == E.EPB_ERR_PARAM
    assert call(e=E.epb_cube(8, 1, None)) == E.EPB_ERR_NULL
    assert call(e=E.epb_cube(1, 1, FAKE)) == E.EPB_ERR_SIZE
    assert call(depth=FAKE + 4) == E.EPB_ERR_ALIGN
    assert call(ao=FAKE + 8) == E.EPB_ERR_ALIGN
    assert call(hdr=FAKE + 2) == E.EPB_ERR_ALIGN


def test_precompute_ibl_fis_validation():
    ok = E.epb_ibl_params(32, 64, 128, 5, 64, 64, 64, 1)
    assert E.epb_scratch_bytes(E.EPB_OP_PRECOMPUTE_IBL, 512, 512, ok) > \
        E.epb_scratch_bytes(E.EPB_OP_PRECOMPUTE_IBL, 512, 512, E.epb_ibl_params(32, 64, 128, 5, 64, 64, 64, 0))
    # the mip chain halves exactly: a power-of-two size is required
    assert E.epb_scratch_bytes(E.EPB_OP_PRECOMPUTE_IBL, 96, 96, E.epb_ibl_params(8, 48, 32, 3, 64, 16, 16, 1)) == 0
    assert E.epb_scratch_bytes(E.EPB_OP_PRECOMPUTE_IBL, 96, 96, E.epb_ibl_params(8, 48, 32, 3, 64, 16, 16, 0)) > 0
    assert E.epb_scratch_bytes(E.EPB_OP_PRECOMPUTE_IBL, 64, 64, E.epb_ibl_params(8, 16, 32, 3, 64, 16, 16, 2)) == 0
