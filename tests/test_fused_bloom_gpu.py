"""The fused form epb_shade_post: the shading pass also writes level 1 of the
bloom pyramid (Sec. 5.3) from its 2x2 pixel blocks, then levels 2.., the blur
and the composite run as in epb_bloom_tonemap.  Its HDR image, 8-bit image and
the whole bloom scratch (unblurred and blurred levels) equal those of
epb_shade followed by epb_bloom_tonemap bit for bit: both storage precisions
and mixed ones, odd sizes (2x2 blocks cut by the right and bottom edges),
images smaller than one block, every pyramid depth, thresholds 0 and 1.  The
fused pyramid also matches the FP64 oracle at rtol 1e-5 and its image the
oracle within +-1 LSB on every pixel.
"""
import copy

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


_cache = {}


def _view(kind):
    if kind not in _cache:
        if kind == "ragged-201x137":
            v = synth.config_reduced(201, 137, seed=7, shadow_size=256, env_size=32, ssao_n=16)
        elif kind == "ragged-97x61":
            v = synth.config_reduced(97, 61, seed=8, shadow_size=128, env_size=16, ssao_n=16, n_spheres=24)
        elif kind == "tiny-3x2":
            v = synth.config_reduced(3, 2, seed=9, shadow_size=16, env_size=8, ssao_n=8, n_spheres=4)
        elif kind == "strip-1x37":
            v = synth.config_reduced(1, 37, seed=12, shadow_size=16, env_size=8, ssao_n=8, n_spheres=4)
        elif kind == "full-1080p":
            v = synth.config_1080p()
        else:
            raise KeyError(kind)
        _cache[kind] = v
    return copy.deepcopy(_cache[kind])


def _device_view(v, gdt, hdt, pdt, levels):
    from paper_2012_03325_amd import frame as fr
    ibl = fr.DeviceIBL(v.env, **v.ibl)
    ibl.precompute()
    dv = fr.DeviceView(v, ibl, gdtype=gdt, ao_dtype=hdt, hdr_dtype=hdt, bloom_levels=levels)
    if pdt != hdt:  # a pyramid stored in the other precision
        dv.postp = fr.DevicePost(v.width, v.height, levels, v.bloom_threshold, v.bloom_strength, v.exposure,
                                 v.gamma, pyr_dtype=pdt, tonemap=v.tonemap)
        dv.post, dv.ldr = dv.postp.post, dv.postp.ldr
    return dv


def _fill(dv):
    # a pattern every output byte must overwrite (0x3f3f3f3f is 0.747 as a float)
    for t in (dv.hdr, dv.ldr, dv.postp.scratch):
        t.view(torch.uint8).fill_(0x3F)


F32, F16 = 0, 1
CASES = [
    ("ragged-201x137", F32, F32, F32, 6, 1.0),
    ("ragged-201x137", F16, F16, F16, 6, 1.0),
    ("ragged-97x61", F32, F32, F16, 3, 0.0),
    ("ragged-97x61", F32, F16, F32, 2, 1.0),
    ("ragged-97x61", F16, F16, F16, 1, 1.0),
    ("tiny-3x2", F32, F32, F32, 6, 0.5),
    ("strip-1x37", F16, F16, F16, 4, 1.0),
    ("full-1080p", F32, F32, F32, 6, 1.0),
    ("full-1080p", F16, F16, F16, 6, 1.0),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-g{c[1]}h{c[2]}p{c[3]}-L{c[4]}-t{c[5]}")
def test_fused_equals_separate_calls(case):
    kind, gdt, hdt, pdt, levels, thr = case
    v = _view(kind)
    v.bloom_threshold = thr
    dv = _device_view(v, gdt, hdt, pdt, levels)
    log(f"[fused] {case}: separate calls")
    dv.ssao()
    _fill(dv)
    dv.shade()
    dv.bloom_tonemap()
    torch.cuda.synchronize()
    ref = [t.clone() for t in (dv.hdr, dv.ldr, dv.postp.scratch)]
    log(f"[fused] {case}: epb_shade_post")
    _fill(dv)
    dv.shade_post()
    torch.cuda.synchronize()
    for name, a, b in zip(("HDR", "LDR", "bloom scratch"), (dv.hdr, dv.ldr, dv.postp.scratch), ref):
        same = torch.equal(a.view(torch.uint8), b.view(torch.uint8))
        if not same:
            d = (a.view(torch.uint8) != b.view(torch.uint8)).nonzero()
            pytest.fail(f"{case}: {name} differs at {d.shape[0]} bytes, first {d[:4].tolist()}")


@pytest.mark.parametrize("kind", ["ragged-201x137", "full-1080p"])
def test_fused_pyramid_and_image_match_oracle(kind):
    """The fused path against the oracle's bloom and tone mapping of the same
    HDR image: every pyramid level at rtol 1e-5, the 8-bit image within +-1."""
    v = _view(kind)
    dv = _device_view(v, F32, F32, F32, 6)
    log(f"[fused-oracle] {kind}")
    dv.ssao()
    dv.shade_post()
    torch.cuda.synchronize()
    hdr = dv.hdr.cpu().numpy().astype(np.float64)
    ref = O.bloom_tonemap(hdr, levels=6, threshold=v.bloom_threshold, strength=v.bloom_strength,
                          exposure=v.exposure, gamma=v.gamma, tonemap=v.tonemap, want_pyramid=True)
    for l, (g, r) in enumerate(zip(dv.pyramid(), ref["pyramid"])):
        gg = g.cpu().numpy()[..., :3].transpose(2, 0, 1)
        assert_interval(f"fused bloom level {l + 1}", gg, r, r, rtol=1e-5)
    frac, exact = assert_ldr(f"fused {kind}", dv.ldr.cpu().numpy(), ref["ldr"], ref["ldr"], min_frac=1.0)
    log(f"[fused-oracle] {kind}: LDR exact {100 * exact:.3f}%")


def test_fused_frame_in_a_graph_replays_equal_eager():
    """A whole frame with the fused call (SSAO, epb_shade_post) captured in a
    HIP graph, as the benchmark times it: every replay, with eager work in
    between, equals the eager frame bit for bit."""
    v = _view("ragged-201x137")
    dv = _device_view(v, F32, F32, F32, 6)
    dv.render(fused=True)
    torch.cuda.synchronize()
    eager = [t.clone() for t in (dv.ao, dv.hdr, dv.ldr)]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        dv.render(fused=True)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    log("[fused-graph] capture")
    with torch.cuda.graph(g):
        dv.render(fused=True)
    for rep in range(3):
        dv.ao.fill_(-1.0)
        dv.hdr.fill_(float(rep))
        dv.ldr.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for name, a, b in zip(("AO", "HDR", "LDR"), (dv.ao, dv.hdr, dv.ldr), eager):
            assert torch.equal(a, b), f"replay {rep}: {name} differs"
