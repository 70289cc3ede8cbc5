"""Whole-pipeline Monte Carlo pin of the FP64 oracle's shading (Sec. 3 Eq. 1,
Sec. 3.1): an 8x8 view of a sphere under a smooth analytic environment, each
image-based-lighting lookup recomputed per pixel at the pixel's exact
(n, R, N.V, r) by random-sampling integration of its definition, in float64:

  E(n)        = (1/pi) integral of L(w) max(0, n.w) dw   (cosine-weighted mean)
  P(R, r)     = the N.L-weighted mean of L over GGX samples with N = V = R
  (A, B)(v, r) = the Karis scale and bias of the split sum (k = alpha / 2)

The radiance is the analytic function the environment's texels sample, so
the comparison also spans the tables' discretisation and interpolation.  The
composition (Fdez-Aguera multiple scattering) and the direct light are the
closed forms of the cited methods, written out here; both are pinned
separately by hand-worked values (test_oracle_worked_values.py).  A wrong
lookup vector, table axis, level or frame moves a pixel by 10 % or more;
the tolerance is 3 sigma of the sampling plus 0.5 % for discretisation.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2012_03325_amd import synth

C0 = np.array([1.0, 0.8, 0.6])
B1 = np.array([[0.5, 0.3, -0.2], [-0.2, 0.4, 0.3], [0.3, -0.3, 0.4]])  # per channel, times w
Q = np.array([0.4, -0.3, 0.2])  # per channel, times w_x w_y


def radiance(w):
    """Smooth, asymmetric environment: (..., 3) unit directions -> (..., 3)."""
    return C0 + w @ B1.T + Q * (w[..., 0] * w[..., 1])[..., None]


def env_cube(S):
    env = np.zeros((6, S, S, 4))
    for f in range(6):
        for j in range(S):
            for i in range(S):
                d = O.cube_texel_dir(f, i, j, S)
                env[f, j, i, :3] = radiance(d / np.linalg.norm(d))
    return env


def _frame(n):
    """An orthonormal frame around n (Frisvad's construction)."""
    if n[2] < -0.9999999:
        return np.array([0.0, -1.0, 0.0]), np.array([-1.0, 0.0, 0.0])
    a = 1.0 / (1.0 + n[2])
    b = -n[0] * n[1] * a
    return np.array([1.0 - n[0] ** 2 * a, b, -n[0]]), np.array([b, 1.0 - n[1] ** 2 * a, -n[1]])


def _ggx_h(rng, m, alpha, n):
    u1, u2 = rng.random(m), rng.random(m)
    phi = 2 * math.pi * u1
    ct = np.sqrt((1 - u2) / (1 + (alpha * alpha - 1) * u2))
    st = np.sqrt(np.maximum(0.0, 1 - ct * ct))
    t, b = _frame(n)
    return (st * np.cos(phi))[:, None] * t + (st * np.sin(phi))[:, None] * b + ct[:, None] * n


def _mean_and_sigma(x, batches=16):
    """Mean of a sample and the standard error estimated from batch means."""
    parts = np.array_split(x, batches)
    means = np.array([p.mean(0) for p in parts])
    return x.mean(0), means.std(0, ddof=1) / math.sqrt(batches)


def mc_irradiance(rng, n, m):
    u1, u2 = rng.random(m), rng.random(m)
    r, phi = np.sqrt(u1), 2 * math.pi * u2
    t, b = _frame(n)
    w = (r * np.cos(phi))[:, None] * t + (r * np.sin(phi))[:, None] * b + np.sqrt(1 - u1)[:, None] * n
    return _mean_and_sigma(radiance(w))


def mc_prefiltered(rng, R, rough, m):
    alpha = rough * rough
    h = _ggx_h(rng, m, alpha, R)
    vh = h @ R
    l = 2 * vh[:, None] * h - R
    nl = l @ R
    keep = nl > 0
    w = np.where(keep, nl, 0.0)
    L = np.where(keep[:, None], radiance(l / np.linalg.norm(l, axis=1)[:, None]), 0.0)
    parts_L, parts_w = np.array_split(L * w[:, None], 16), np.array_split(w, 16)
    est = np.array([pl.sum(0) / pw.sum() for pl, pw in zip(parts_L, parts_w)])
    return (L * w[:, None]).sum(0) / w.sum(), est.std(0, ddof=1) / 4.0


def mc_split_sum(rng, NoV, rough, m):
    alpha = rough * rough
    k = alpha / 2
    v = np.array([math.sqrt(max(0.0, 1 - NoV * NoV)), 0.0, NoV])
    h = _ggx_h(rng, m, alpha, np.array([0.0, 0.0, 1.0]))
    vh = h @ v
    l = 2 * vh[:, None] * h - v
    nl, nh = l[:, 2], h[:, 2]
    g1 = lambda x: x / (x * (1 - k) + k)
    gvis = np.where(nl > 0, g1(np.maximum(nl, 0)) * g1(NoV) * vh / (nh * NoV), 0.0)
    fc = (1 - vh) ** 5
    return _mean_and_sigma(np.stack([(1 - fc) * gvis, fc * gvis], 1))


@pytest.mark.slow
def test_shading_matches_monte_carlo_lookups():
    rng = np.random.default_rng(2012)
    S = 64
    env = env_cube(S)
    ibl = O.precompute_ibl(env, irr_size=16, irr_src_size=64, pref_size=64, pref_levels=5, pref_samples=1024,
                           lut_size=64, lut_samples=1024)
    W = H = 8
    cam = synth.look_at((0.3, 0.8, 3.2), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 30.0, W, H)
    scene = synth.SphereScene(np.zeros((1, 3)), np.array([1.0]), np.array([[0.7, 0.5, 0.3]]), np.array([0.5]),
                              np.array([0.0]))
    g = synth.raycast(scene, cam)
    yy, xx = np.mgrid[0:H, 0:W]
    g["roughness"] = np.array([0.0, 0.25, 0.5])[(xx + 2 * yy) % 3].astype(np.float64)
    g["metalness"] = ((xx // 2 + yy) % 2).astype(np.float64)
    light = synth.Light(np.array([2.0, 3.0, 2.5]), np.array([1.0, 0.9, 0.8]), 6.0)
    ao = np.ones(((H + 1) // 2, (W + 1) // 2))
    # (lo and hi differ only where a prefilter sample sat on a cube edge: both checked)
    lo, hi = O.shade(g, cam, ao, ao, [light], ibl, env, tie=O.EXACT)

    M = np.asarray(cam.world_to_cam, np.float64)
    R_, t_ = M[:, :3], M[:, 3]
    cpos = -R_.T @ t_
    m = 1 << 17
    checked = worst = 0.0
    fg = 0
    for y in range(H):
        for x in range(W):
            d = g["depth"][y, x]
            ray = R_.T @ np.array([(x + 0.5 - cam.cx) / cam.fx, -(y + 0.5 - cam.cy) / cam.fy, -1.0])
            if not np.isfinite(d):
                # background: the radiance along the view ray (bilinear texels of a smooth field)
                expect = radiance(ray / np.linalg.norm(ray))
                tol = 5e-3 * np.abs(expect)
            else:
                fg += 1
                Pw = cpos + d * ray
                V = (cpos - Pw) / np.linalg.norm(cpos - Pw)
                n = g["normal"][:, y, x] / np.linalg.norm(g["normal"][:, y, x])
                r, mt = g["roughness"][y, x], g["metalness"][y, x]
                alb = g["albedo"][:, y, x]
                nv_raw = n @ V
                NoV = min(max(nv_raw, 1e-4), 1.0)
                Rv = 2 * nv_raw * n - V
                E, sE = mc_irradiance(rng, n, m)
                if r == 0.0:
                    P, sP = radiance(Rv / np.linalg.norm(Rv)), np.zeros(3)
                else:
                    P, sP = mc_prefiltered(rng, Rv / np.linalg.norm(Rv), r, m)
                AB, sAB = mc_split_sum(rng, NoV, r if r > 0 else 1e-3, m)
                F0 = 0.04 * (1 - mt) + alb * mt
                cd = alb * (1 - mt)
                # ambient: split sum with multiple scattering (Fdez-Aguera 2019)
                kS = F0 + (np.maximum(1 - r, F0) - F0) * (1 - NoV) ** 5
                FssEss = kS * AB[0] + AB[1]
                Ems = 1 - AB[0] - AB[1]
                Favg = F0 + (1 - F0) / 21
                Fms = FssEss * Favg / (1 - Ems * Favg)
                kD = cd * (1 - FssEss - Fms * Ems)
                amb = FssEss * P + (Fms * Ems + kD) * E
                # direct light: Cook-Torrance, GGX / Smith-Schlick (k = (r+1)^2/8) / Schlick
                lv = light.pos - Pw
                dist2 = lv @ lv
                l = lv / math.sqrt(dist2)
                NoL = n @ l
                direct = np.zeros(3)
                if NoL > 0:
                    hh = (V + l) / np.linalg.norm(V + l)
                    a2 = (r * r) ** 2
                    D = a2 / (math.pi * ((n @ hh) ** 2 * (a2 - 1) + 1) ** 2)
                    kd = (r + 1) ** 2 / 8
                    G = NoL / (NoL * (1 - kd) + kd) * NoV / (NoV * (1 - kd) + kd)
                    F = F0 + (1 - F0) * (1 - max(0.0, V @ hh)) ** 5
                    f = cd / math.pi + D * G * F / (4 * NoL * NoV)
                    direct = f * light.color * light.intensity / dist2 * NoL
                expect = direct + amb
                # sampling error propagated to first order, plus 0.5 % for the tables'
                # discretisation and interpolation
                sig = (FssEss * sP + (Fms * Ems + kD) * sE + np.abs(P * kS + E) * (sAB[0] + sAB[1]))
                tol = 3 * sig + 5e-3 * np.abs(amb) + 1e-9
            err = np.maximum(np.abs(lo[:, y, x] - expect), np.abs(hi[:, y, x] - expect))
            assert (err <= tol).all(), (x, y, lo[:, y, x], expect, tol)
            worst = max(worst, float((err / np.maximum(np.abs(expect), 1e-12)).max()))
            checked += 1
    assert fg >= 40
    print(f"8x8 view: {int(checked)} pixels ({fg} shaded), worst relative error {worst:.2e}")
