"""Eye-dome lighting (Sec. 4.3) on the GPU against the FP64 oracle.

The path has no floating-point decision (the response is a sum of max(0, .)
terms, continuous in the depths, and the neighbourhood is integer), so every
pixel must match.  Tolerance: relative 1e-4 (float32 log2 of depths up to the
far cap, about 1e-6 absolute per term, times the strength, inside exp2) plus an
absolute floor of 1e-7 of the image maximum (float32 underflow of the darkest
outline shades); half storage adds one half rounding (2^-11 relative) on the
output, the oracle taking the same half-rounded colour and AO as input."""
import zlib

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from paper_2012_03325_amd import synth
from tests.parity_util import assert_interval, log

pytestmark = pytest.mark.gpu

RTOL = 1e-4
ATOL_REL_MAX = 1e-7


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_03325_amd import frame  # noqa: F401  (loads libepb.so, fails loudly)
    yield
    torch.cuda.synchronize()


# name: (W, H, points, radius, dirs, strength, half storage, with AO, with environment)
CASES = {
    "201x137-r2-n8": (201, 137, 150_000, 2, 8, 8.0, False, True, True),
    "97x61-r5-n12-half": (97, 61, 40_000, 5, 12, 4.0, True, True, False),
    "3x2-r1-n4": (3, 2, 200, 1, 4, 8.0, False, False, True),
    "33x17-r16-n32": (33, 17, 8_000, 16, 32, 20.0, False, True, True),
    "130x70-strength0": (130, 70, 30_000, 3, 8, 0.0, False, True, True),
    "64x48-empty": (64, 48, 0, 2, 8, 8.0, False, True, True),
    "1920x1080-r2-n8": (1920, 1080, 4_000_000, 2, 8, 8.0, False, True, True),
}


def _cloud(name):
    W, H, n, r, k, s, half, use_ao, use_env = CASES[name]
    pc = synth.point_cloud_view(W, H, n, seed=zlib.crc32(name.encode()) % 100_000, n_spheres=64 if n < 1e6 else 512)
    pc.edl_radius, pc.edl_dirs, pc.edl_strength = r, k, s
    if half:  # the oracle sees exactly what the half-storage kernel reads
        pc.color = pc.color.astype(np.float16).astype(np.float32)
        pc.ao = pc.ao.astype(np.float16).astype(np.float32)
    return pc, half, use_ao, use_env


@pytest.mark.parametrize("name", list(CASES))
def test_edl_matches_oracle(name):
    from paper_2012_03325_amd import epb as E, frame
    log(f"[edl] {name}")
    pc, half, use_ao, use_env = _cloud(name)
    dt = E.EPB_F16 if half else E.EPB_F32
    dev = frame.DeviceEDL(pc, color_dtype=dt, ao_dtype=dt, hdr_dtype=dt, use_ao=use_ao, use_env=use_env)
    dev.run()
    torch.cuda.synchronize()
    g = dev.hdr.float().cpu().numpy()
    lo, hi = O.edl(pc.depth, pc.color, pc.cam, pc.ao if use_ao else None, pc.ao if use_ao else None,
                   pc.edl_radius, pc.edl_dirs, pc.edl_strength, pc.edl_far, pc.env if use_env else None)
    assert np.isfinite(g).all()
    rtol = RTOL + (2.0 ** -11 if half else 0.0)
    atol = ATOL_REL_MAX * max(1e-30, float(np.abs(hi).max()))
    assert_interval(f"edl {name}", g, lo, hi, rtol=rtol, atol=atol)
    fg = np.isfinite(pc.depth)
    if pc.edl_strength == 0.0:  # no darkening: colour times AO, background the sky
        assert np.all(np.abs(g[:, fg] - lo[:, fg]) <= rtol * lo[:, fg] + atol)
    log(f"[edl] {name}: {fg.mean() * 100:.1f}% points, mean shade-weighted HDR {g.mean():.4f}")


def test_edl_repeatable_and_stream_ordered():
    """Two launches on a side stream write the same bits (no atomics, no races)."""
    from paper_2012_03325_amd import frame
    pc, _, _, _ = _cloud("201x137-r2-n8")
    dev = frame.DeviceEDL(pc)
    s = torch.cuda.Stream()
    other = torch.empty_like(dev.hdr)
    with torch.cuda.stream(s):
        dev.run(stream=s)
        dev.run(stream=s, hdr=other)
    s.synchronize()
    assert torch.equal(dev.hdr, other)
