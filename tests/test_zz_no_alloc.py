"""The allocation-free SSAO entry point (epb_ssao_static, scratch held by the
library) against epb_ssao with caller scratch, through the C ABI: bit-for-bit
equal AO on two calls in a row, the second on a smaller image, blurred and
raw, float32 and half storage."""
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


def _views():
    return [synth.config_reduced(201, 137, seed=7, shadow_size=64, env_size=16, ssao_n=16),
            synth.config_reduced(97, 61, seed=8, shadow_size=64, env_size=16, ssao_n=13, n_spheres=24)]


@pytest.mark.parametrize("gdtype,blur", [(0, 1), (0, 0), (1, 1)])
def test_static_scratch_ssao_matches_caller_scratch(gdtype, blur):
    from paper_2012_03325_amd import epb as E
    from paper_2012_03325_amd import frame
    ibl_p = dict(irr_size=4, irr_src_size=16, pref_size=16, pref_levels=4, pref_samples=16, lut_size=8,
                 lut_samples=16)
    for k, v in enumerate(_views()):  # the second call is on a smaller image
        ibl = frame.DeviceIBL(v.env, **ibl_p)
        dv = frame.DeviceView(v, ibl, gdtype=gdtype, ao_dtype=gdtype)
        dv.ssao_params.blur = blur
        log(f"[no-alloc] call {k}: {v.width}x{v.height} gdtype={gdtype} blur={blur}: caller scratch")
        dv.ao.fill_(-1.0)
        E.epb_ssao(dv.gbuf, dv.cam, dv.ssao_params, dv.ao, dv.ssao_scratch, dv.ssao_scratch_bytes)
        torch.cuda.synchronize()
        ref = dv.ao.clone()
        log(f"[no-alloc] call {k}: library scratch")
        dv.ao.fill_(-2.0)
        E.epb_ssao_static(dv.gbuf, dv.cam, dv.ssao_params, dv.ao)
        torch.cuda.synchronize()
        assert torch.equal(ref, dv.ao), k
        assert (ref.float() >= 0).all() and (ref.float() <= 1).all()
    log("[no-alloc] two calls bitwise equal to the caller-scratch call")
