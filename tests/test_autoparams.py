"""Automatic parameters (Sec. 6) on the CPU: the SSAO radius is 5 % of the
scene scale, the camera frames the whole scene, the three lights deliver their
predefined radiance at the object, and everything scales with the scene."""
import math

import numpy as np
import pytest

from paper_2012_03325_amd import autoparams as A
from paper_2012_03325_amd import synth


def _scene(scale=1.0, seed=3):
    sc = synth.make_spheres(np.random.default_rng(seed), 40, False)
    sc.centers = sc.centers * scale + np.array([5.0, 1.0, -2.0]) * scale
    sc.radii = sc.radii * scale
    return sc


def test_bounds_enclose_every_sphere_and_touch_one():
    sc = _scene()
    b = A.sphere_bounds(sc)
    far = np.linalg.norm(sc.centers - b.center, axis=1) + sc.radii
    assert np.all(far <= b.radius + 1e-12) and abs(far.max() - b.radius) < 1e-12
    assert A.ssao_radius(b) == pytest.approx(0.05 * 2 * b.radius)


@pytest.mark.parametrize("W,H", [(1920, 1080), (480, 640), (256, 256)])
def test_fitted_camera_sees_the_whole_bounding_sphere(W, H):
    sc = _scene()
    b = A.sphere_bounds(sc)
    cam = A.fit_camera(b, (0.3, 0.5, 1.0), W, H)
    # sample the bounding sphere's surface: every point projects inside the image
    rng = np.random.default_rng(1)
    u = rng.normal(size=(4000, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    p = b.center + b.radius * u
    pv = p @ cam.R.T + cam.t
    d = -pv[:, 2]
    assert np.all(d > 0)
    x = cam.cx + cam.fx * pv[:, 0] / d
    y = cam.cy - cam.fy * pv[:, 1] / d
    assert np.all((x >= -1e-6) & (x <= W + 1e-6) & (y >= -1e-6) & (y <= H + 1e-6))
    # and it is tight: the sphere touches the limiting edge (within 1 %)
    span = max((x.max() - x.min()) / W, (y.max() - y.min()) / H)
    assert span > 0.95


def test_three_point_lights_deliver_the_predefined_radiance():
    sc = _scene()
    b = A.sphere_bounds(sc)
    cam = A.fit_camera(b, (0.0, 0.4, 1.0), 640, 480)
    lights = A.three_point_lights(b, cam, radiance=2.5)
    assert A.rig_names() == ("key", "fill", "rim")
    shares = [r[3] for r in A.RIG]
    for L, share in zip(lights, shares):
        d2 = float(np.sum((L.pos - b.center) ** 2))
        assert L.color[0] * L.intensity / d2 == pytest.approx(2.5 * share, rel=1e-12)
        assert math.sqrt(d2) == pytest.approx(A.RIG_DISTANCE_RADII * b.radius, rel=1e-6)
    key, fill, rim = lights
    to_cam = cam.position - b.center
    # key and fill on the camera's side, the rim light behind the object
    assert np.dot(key.pos - b.center, to_cam) > 0 and np.dot(fill.pos - b.center, to_cam) > 0
    assert np.dot(rim.pos - b.center, to_cam) < 0
    assert key.intensity > fill.intensity  # the key light gives most of the light


def test_everything_scales_with_the_scene():
    b1, b2 = A.sphere_bounds(_scene(1.0)), A.sphere_bounds(_scene(1000.0))
    assert b2.radius == pytest.approx(1000.0 * b1.radius, rel=1e-12)
    assert A.ssao_radius(b2) == pytest.approx(1000.0 * A.ssao_radius(b1), rel=1e-12)
    c1 = A.fit_camera(b1, (0, 0.5, 1), 320, 240)
    c2 = A.fit_camera(b2, (0, 0.5, 1), 320, 240)
    assert np.linalg.norm(c2.position - b2.center) == pytest.approx(
        1000.0 * np.linalg.norm(c1.position - b1.center), rel=1e-5)
    l1, l2 = A.three_point_lights(b1, c1), A.three_point_lights(b2, c2)
    for a, b in zip(l1, l2):
        ra = a.intensity / np.sum((a.pos - b1.center) ** 2)
        rb = b.intensity / np.sum((b.pos - b2.center) ** 2)
        assert ra == pytest.approx(rb, rel=1e-9)  # same radiance at the object at any scale
