"""Hand-worked values that pin the parts of the FP64 oracle that invariants
cannot fail: each case is arranged so that a plausible slip (a swapped table
axis, the wrong lookup vector, a different Smith k, a fourth power for the
fifth, a shifted blur window or upsample position, a reversed view ray)
changes the result by far more than the tolerance.  The expected numbers were
worked out with exact fractions from the method's definitions (the steps are
given in each docstring); pi is the only irrational factor.
"""
import math

import numpy as np

from oracle import oracle as O
from paper_2012_03325_amd import synth

PI = math.pi


def _look_at(eye, target, up, W=1, H=1, f=1.0):
    """Pinhole camera in float64 (no float32 rounding of the pose): view -z
    along target - eye, pixel (x + 1/2, y + 1/2) on the optical axis at the
    image centre."""
    eye, target, up = (np.asarray(v, np.float64) for v in (eye, target, up))
    fw = (target - eye) / np.linalg.norm(target - eye)
    x = np.cross(fw, up)
    x /= np.linalg.norm(x)
    y = np.cross(x, fw)
    R = np.stack([x, y, -fw])
    return synth.Camera(np.concatenate([R, (-R @ eye)[:, None]], 1), f, f, W / 2.0, H / 2.0, W, H)


def _gbuf(depth, normal, albedo, rough, metal):
    H, W = depth.shape
    return dict(depth=np.asarray(depth, np.float64),
                normal=np.broadcast_to(np.asarray(normal, np.float64).reshape(3, 1, 1), (3, H, W)).copy(),
                albedo=np.broadcast_to(np.asarray(albedo, np.float64).reshape(3, 1, 1), (3, H, W)).copy(),
                roughness=np.full((H, W), rough, np.float64), metalness=np.full((H, W), metal, np.float64))


def _black_ibl():
    # no ambient light; a plausible constant BRDF table (A + B > 0 keeps the
    # multiple-scattering term 1 / (1 - Ems F_avg) finite for F0 = 1)
    tab = np.zeros((8, 8, 2))
    tab[..., 0], tab[..., 1] = 0.6, 0.1
    return dict(irradiance=np.zeros((6, 4, 4, 4)), prefiltered=[np.zeros((6, 4 >> m, 4 >> m, 4)) for m in range(3)],
                lut=tab)


# ---------------------------------------------------------------------------
# direct light off the normal (Sec. 3, Eq. 1 with the UE4 Cook-Torrance BRDF)
# ---------------------------------------------------------------------------
def test_direct_light_off_the_normal_by_hand():
    """n = +z; camera and light 60 degrees either side of n at distance 2, so
    n.v = n.l = 1/2, h = n, n.h = 1, v.h = 1/2; roughness 1/2 (alpha = 1/4);
    the light (intensity 4) delivers radiance 4 / 2^2 = 1.
      D(1) = 1 / (pi alpha^2) = 16 / pi
      k = (r + 1)^2 / 8 = 9/32,  G1(1/2) = (1/2) / ((1/2)(23/32) + 9/32) = 32/41,
      G = 1024/1681
      F = F0 + (1 - F0) (1/2)^5 = F0 + (1 - F0) / 32
      spec = D G F / (4 n.l n.v) = (16384 / 1681) F / pi
      L = (c_diff / pi + spec) x 1 x n.l
    dielectric (F0 = 0.04, F = 0.07): spec = 28672 / (42025 pi) = 0.2171702809;
    albedo 0.2 / 0.6 / 1 -> L = (a + 28672/42025) / (2 pi) = 0.1404161291,
    0.2040781063, 0.2677400836.  Metal (F0 = albedo, no diffuse): F = 9/40,
    49/80, 1 -> L = (16384/1681) F / (2 pi) = 0.3490236658, 0.9501199791,
    1.5512162925.  Smith k = alpha/2 instead would give G1 = 8/9 (+46 %),
    a fourth power F = 0.1 (+43 %), alpha = r gives D / 4."""
    s3 = math.sqrt(3.0)
    cam = _look_at((s3, 0.0, 1.0), (0, 0, 0), (0, 1, 0))
    light = synth.Light(np.array([-s3, 0.0, 1.0]), np.ones(3), 4.0)
    ao = np.ones((1, 1))
    env = np.zeros((6, 2, 2, 4))
    cases = [(0.0, [0.14041612909026066, 0.20407810632701878, 0.26774008356377693]),
             (1.0, [0.3490236658024765, 0.9501199791289637, 1.5512162924554511])]
    for metal, expect in cases:
        g = _gbuf(np.full((1, 1), 2.0), (0, 0, 1), (0.2, 0.6, 1.0), 0.5, metal)
        lo, hi = O.shade(g, cam, ao, ao, [light], _black_ibl(), env, tie=O.EXACT)
        assert np.allclose(lo[:, 0, 0], expect, rtol=1e-12, atol=0), (metal, lo[:, 0, 0])
        assert np.array_equal(lo, hi)
        # ambient occlusion darkens the ambient term only, never the direct light
        half = np.full((1, 1), 0.5)
        lo2, _ = O.shade(g, cam, half, half, [light], _black_ibl(), env, tie=O.EXACT)
        assert np.array_equal(lo2, lo)


# ---------------------------------------------------------------------------
# ambient light: split-sum IBL with multiple scattering (Sec. 3.1)
# ---------------------------------------------------------------------------
def _face_constant_cube(size, values, other):
    c = np.zeros((6, size, size, 4))
    for f in range(6):
        c[f, ..., :3] = values.get(f, other)
    return c


def test_ambient_by_hand_with_asymmetric_tables():
    """n = +y, camera 60 degrees from n in the xy plane: n.v = 1/2, reflection
    R = 2 (n.v) n - v = (-sqrt(3)/2, 1/2, 0), on the -X face; roughness 0.55,
    metalness 1/2, albedo (0.2, 0.6, 1), AO 1/2, no lights.
    Tables: irradiance +Y face = E = (0.3, 0.5, 0.7), other faces 5; prefiltered
    level m of the -X face = (m + 1)/10 (1, 2, 4), other faces 7, so at
    lod = 0.55 x 4 = 2.2: P = 0.8 P_2 + 0.2 P_3 = (0.32, 0.64, 1.28); BRDF
    table with A = 0.2 + 0.5 N.V along columns and B = 0.05 + 0.1 r along rows
    (linear, so bilinear lookups are exact): A = 9/20, B = 21/200.
      F0 = 0.04 (1 - m) + a m = (3/25, 8/25, 13/25), c_diff = (1/10, 3/10, 1/2)
      k_S = F0 + (max(1 - r, F0) - F0)(1 - N.V)^5 = (417/3200, 1037/3200, 13/25)
            (the blue channel takes F0 = 0.52 > 1 - r = 0.45 in the max)
      FssEss = k_S A + B = (10473/64000, 16053/64000, 339/1000); Ems = 1 - A - B = 89/200
      F_avg = F0 + (1 - F0)/21; Fms = FssEss F_avg / (1 - Ems F_avg)
      k_D = c_diff (1 - FssEss - Fms Ems)
      ambient = FssEss P + (Fms Ems + k_D) E = (0.0808862134, 0.2892322033, 0.7030618911)
    HDR = AO x ambient = (0.0404431067, 0.1446161017, 0.3515309456).
    Swapped table axes give A = 0.475, B = 0.1; E looked up at R reads 5,
    P at n reads 7; lod = r M reads 2.75; a missing max() changes blue."""
    s3 = math.sqrt(3.0)
    cam = _look_at((s3, 1.0, 0.0), (0, 0, 0), (0, 0, 1))
    irr = _face_constant_cube(4, {2: (0.3, 0.5, 0.7)}, (5.0, 5.0, 5.0))
    pref = [_face_constant_cube(32 >> m, {1: tuple((m + 1) / 10 * np.array([1, 2, 4]))}, (7.0, 7.0, 7.0))
            for m in range(5)]
    n = 16
    lut = np.zeros((n, n, 2))
    u = (np.arange(n) + 0.5) / n
    lut[..., 0] = 0.2 + 0.5 * u[None, :]   # columns: N.V
    lut[..., 1] = 0.05 + 0.1 * u[:, None]  # rows: roughness
    ibl = dict(irradiance=irr, prefiltered=pref, lut=lut)
    g = _gbuf(np.full((1, 1), 2.0), (0, 1, 0), (0.2, 0.6, 1.0), 0.55, 0.5)
    ao = np.full((1, 1), 0.5)
    lo, hi = O.shade(g, cam, ao, ao, [], ibl, np.zeros((6, 2, 2, 4)), tie=O.EXACT)
    expect = [0.040443106710563455, 0.14461610165647767, 0.3515309455641364]
    assert np.allclose(lo[:, 0, 0], expect, rtol=1e-12, atol=0), lo[:, 0, 0]
    assert np.array_equal(lo, hi)


# ---------------------------------------------------------------------------
# SSAO blur (Sec. 5.2: bilateral 4x4)
# ---------------------------------------------------------------------------
def test_ssao_blur_by_hand_with_partial_weights():
    """Half-resolution 6x5 field, raw AO (i + 6 j) / 64, depth 1 except
    d(0,0) = 1.05, d(3,1) = 1.2, d(1,3) = 0.97 and d(3,0) = background.
    Texel (2, 2): window i, j in {0..3} (offsets -2..1); tent weights
    1 - |dq - dp| / (0.1 dp): 0.5 at (0,0), 0 at (3,1), 0.7 at (1,3), 0 at the
    background texel, 1 elsewhere: sum w = 66/5, sum w raw = 1503/640, AO =
    501/2816 = 0.1779119318.  Texel (0, 0) (dp = 1.05, window clipped to
    {0,1}^2): neighbours at depth 1 weigh 1 - 0.05/0.105 = 11/21: AO = (11/21)
    (1 + 6 + 7)/64 / (1 + 3 x 11/21) = 77/1728.  A window of -1..2 or
    -2..2, a box weight or tau d_q in the denominator all miss both."""
    Wh, Hh = 6, 5
    W, H = 2 * Wh, 2 * Hh
    depth = np.ones((H, W))
    for (i, j), d in {(0, 0): 1.05, (3, 1): 1.2, (1, 3): 0.97, (3, 0): np.inf}.items():
        depth[2 * j, 2 * i] = d
    raw = (np.arange(Wh)[None, :] + 6 * np.arange(Hh)[:, None]) / 64.0
    lo, hi = O.ssao_blur(raw, raw, depth, 0.1)
    assert abs(lo[2, 2] - 501 / 2816) < 1e-15
    assert abs(lo[0, 0] - 77 / 1728) < 1e-15
    assert np.array_equal(lo, hi)


# ---------------------------------------------------------------------------
# composite: bilinear upsampling of the blurred levels (Sec. 5.3)
# ---------------------------------------------------------------------------
def test_composite_upsample_position_by_hand():
    """A 4x2 grey image of 3 (columns 0, 1) and 7 (columns 2, 3), threshold 1:
    bright map c max(Y - 1, 0) / Y = 2 and 6; level 1 (2x1) = (2, 6); its
    binomial blur with clamp to edge: (11 x 2 + 5 x 6)/16 = 3.25 and
    (5 x 2 + 11 x 6)/16 = 4.75 (one row: the vertical pass is the identity).
    Upsampled at (x + 1/2)/2 - 1/2 = -0.25, 0.25, 0.75, 1.25 (clamped):
    3.25, 3.625, 4.375, 4.75; composite = HDR + 0.04 x that =
    3.13, 3.145, 7.175, 7.19.  Sampling at (x + 1/2)/2 or x/2 gives
    other values at every pixel; the same along y for the transposed image."""
    hdr = np.zeros((3, 2, 4))
    hdr[:, :, :2], hdr[:, :, 2:] = 3.0, 7.0
    expect = np.array([3.13, 3.145, 7.175, 7.19])
    c = O.bloom_tonemap(hdr, levels=2, threshold=1.0, strength=0.04, want_composite=True)["composite"]
    assert np.allclose(c, np.broadcast_to(expect, (3, 2, 4)), rtol=0, atol=1e-14), c[0]
    ct = O.bloom_tonemap(np.ascontiguousarray(hdr.transpose(0, 2, 1)), levels=2, threshold=1.0, strength=0.04,
                         want_composite=True)["composite"]
    assert np.allclose(ct, np.broadcast_to(expect[:, None], (3, 4, 2)), rtol=0, atol=1e-14), ct[0]


# ---------------------------------------------------------------------------
# background: the environment along the view ray
# ---------------------------------------------------------------------------
def test_background_follows_the_view_ray():
    """A camera at the origin looking down +x (up +y): its view +x axis is world
    +z.  In a 3x1 image with f = 0.8 the rays of pixels 0, 1, 2 are
    (1, 0, -1.25), (1, 0, 0) and (1, 0, 1.25) in the world: faces -Z, +X and
    +Z of an environment whose faces are constants 10^k (k = face index).
    A reversed ray would read -X and swap the z faces."""
    cam = _look_at((0, 0, 0), (1, 0, 0), (0, 1, 0), W=3, H=1, f=0.8)
    env = np.zeros((6, 2, 2, 4))
    for f in range(6):
        env[f, ..., :3] = 10.0 ** f
    g = _gbuf(np.full((1, 3), np.inf), (0, 0, 1), (0.5, 0.5, 0.5), 0.5, 0.0)
    ao = np.ones((1, 2))
    lo, hi = O.shade(g, cam, ao, ao, [], _black_ibl(), env, tie=O.EXACT)
    assert np.array_equal(lo[:, 0, :], np.broadcast_to(np.array([1e5, 1.0, 1e4]), (3, 3)))
    assert np.array_equal(lo, hi)


# ---------------------------------------------------------------------------
# SSAO: the nearest half-resolution texel of a sample (Sec. 5.2)
# ---------------------------------------------------------------------------
def test_ssao_nearest_half_resolution_texel_by_hand():
    """8x2 image, camera at the origin looking down -z (f = 2, c = (4, 1)),
    normal +z, noise (1, 0) (so t = x, b = y), radius 1, one kernel sample.
    Half-resolution texels 0..3 (full-resolution columns 0, 2, 4, 6) at depths
    10, 20, 5, 10.  Texel 0: P = (-17.5, 2.5, -10); the sample (16.075, 0, 0.5)
    lands at Q = (-1.425, 2.5, -9.5), u = 4 + 2 (-1.425) / 9.5 = 3.7, so
    h = (u - 1/2)/2 + 1/2 = 2.1: texel 2 (depth 5 <= 9.5 - bias) occludes it
    with smoothstep(1 / |10 - 5|) = 0.2^2 (3 - 0.4) = 0.104: AO = 0.896.
    Texel 3: P = (12.5, 2.5, -10); the sample (-16.775, 0, 0.5) lands at
    u = 4 + 2 (-4.275) / 9.5 = 3.1, h = 1.8: texel 1 (depth 20) does not
    occlude: AO = 1.  floor(u/2) would pick texel 1 for the first (AO 1),
    floor(u/2 + 3/4) texel 2 for the second (AO 0.896)."""
    W, H = 8, 2
    cam = synth.Camera(np.concatenate([np.eye(3), np.zeros((3, 1))], 1), 2.0, 2.0, 4.0, 1.0, W, H)
    depth = np.full((H, W), 10.0)
    for i, d in enumerate((10.0, 20.0, 5.0, 10.0)):
        depth[:, 2 * i] = d
    normal = np.zeros((3, H, W))
    normal[2] = 1.0
    noise = np.zeros((4, 4, 2))
    noise[..., 0] = 1.0
    lo, hi = O.ssao_raw(depth, normal, cam, np.array([[16.075, 0.0, 0.5]]), noise, 1.0, 0.025, O.EXACT)
    assert abs(lo[0, 0] - 0.896) < 1e-12 and hi[0, 0] == lo[0, 0]
    lo, hi = O.ssao_raw(depth, normal, cam, np.array([[-16.775, 0.0, 0.5]]), noise, 1.0, 0.025, O.EXACT)
    assert lo[0, 3] == 1.0 and hi[0, 3] == 1.0
