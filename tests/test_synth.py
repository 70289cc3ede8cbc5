"""The seeded input generator: the C ray caster against its slow numpy
reference, and the shape of the many-view workloads."""
import collections

import numpy as np
import pytest

from paper_2012_03325_amd import synth


@pytest.mark.parametrize("w,h,n,plane,eye", [(97, 61, 24, True, (0.0, 3.5, 8.5)),
                                             (256, 256, 64, False, (0.0, 3.5, 8.5)),
                                             (200, 120, 300, True, (1.0, 0.6, 2.0)),
                                             (31, 7, 5, True, (0.0, 9.0, 0.1))])
def test_c_raycaster_matches_numpy(w, h, n, plane, eye):
    rng = np.random.default_rng(w * h + n)
    sc = synth.make_spheres(rng, n, plane)
    cam = synth.look_at(eye, (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0, w, h)
    a = synth.raycast_numpy(sc, cam)
    b = synth.raycast(sc, cam)
    assert np.array_equal(np.isinf(a["depth"]), np.isinf(b["depth"]))
    assert np.isfinite(a["depth"]).any()
    for k in a:
        x, y = a[k], b[k]
        fin = np.isfinite(x)
        # the two casts differ only in rounding order: one float32 ulp at most
        np.testing.assert_allclose(np.where(fin, y, 0), np.where(fin, x, 0), rtol=2e-7, atol=2e-8, err_msg=k)
    d = synth.raycast(sc, cam, depth_only=True)
    assert set(d) == {"depth"} and np.array_equal(d["depth"], b["depth"])


def test_batch_workload_shape():
    specs = synth.view_specs(16, 256, 200)
    counts = collections.Counter((s.cam.width, s.cam.height) for s in specs)
    assert set(counts) == set(synth.BATCH_RESOLUTIONS)
    assert set(s.scene for s in specs) == set(range(16))
    # uniform draws: each resolution holds about a quarter of the views
    assert all(30 <= c <= 100 for c in counts.values())
    for s in specs[:8]:
        pos = s.cam.position
        dist = np.linalg.norm(pos)
        el = np.degrees(np.arcsin(pos[1] / dist))
        assert 7.0 - 1e-3 <= dist <= 10.0 + 1e-3 and 15.0 - 1e-3 <= el <= 45.0 + 1e-3
    sc = synth.make_scene(100, env_size=64)
    assert 64 <= len(sc.spheres.radii) <= 1024 and sc.env.shape == (6, 64, 64, 4)
    assert sc.env[..., :3].max() >= 1e4 * 0.85  # the sun disc is present
