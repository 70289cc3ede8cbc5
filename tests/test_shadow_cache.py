"""Shadow-map caching (Sec. 5.1: depth maps are rendered again only when the
objects or the lights move), as host logic on the CPU with a stand-in scene
whose depth render is a counter."""
import numpy as np

from paper_2012_03325_amd import frame, synth


class _FakeScene:
    def __init__(self):
        self.version = 0
        self.calls = []

    def render_depth(self, cam, out=None, stream=None):
        self.calls.append((cam.width, out is not None))
        return out if out is not None else np.zeros((cam.height, cam.width))


def _cams(shift=0.0, size=64):
    return [synth.look_at((6.0 * np.cos(a) + shift, 6.0, 6.0 * np.sin(a)), (0, 0, 0), (0, 1, 0), 90.0, size, size)
            for a in (0.3, 1.9, 3.5, 5.1)]


def test_static_scene_renders_each_map_once():
    sc = _FakeScene()
    cache = frame.ShadowCache(sc)
    first = cache.maps(_cams())
    assert cache.renders == 4
    for _ in range(5):
        again = cache.maps(_cams())
        assert all(a is b for a, b in zip(first, again))
    assert cache.renders == 4


def test_moving_one_light_renders_only_its_map_into_the_same_buffer():
    sc = _FakeScene()
    cache = frame.ShadowCache(sc)
    first = cache.maps(_cams())
    cams = _cams()
    cams[2] = synth.look_at((1.0, 7.0, 2.0), (0, 0, 0), (0, 1, 0), 90.0, 64, 64)
    second = cache.maps(cams)
    assert cache.renders == 5
    assert sc.calls[-1] == (64, True)  # re-rendered in place
    assert second[2] is first[2] and all(second[k] is first[k] for k in (0, 1, 3))


def test_geometry_change_invalidates_every_map():
    sc = _FakeScene()
    cache = frame.ShadowCache(sc)
    cache.maps(_cams())
    sc.version += 1
    cache.maps(_cams())
    assert cache.renders == 8
    cache.maps(_cams())
    assert cache.renders == 8


def test_resized_map_gets_a_new_buffer_and_invalidate_forgets():
    sc = _FakeScene()
    cache = frame.ShadowCache(sc)
    cache.maps(_cams(size=64))
    cache.maps(_cams(size=32))
    assert cache.renders == 8 and sc.calls[-1] == (32, False)
    cache.invalidate()
    cache.maps(_cams(size=32))
    assert cache.renders == 12
