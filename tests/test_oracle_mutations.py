"""Planted mistakes in the FP64 oracle, on the CPU: each case copies the
oracle's C source, makes one plausible slip in it (a dropped term, a wrong
sign, exponent or index, a transposed operand, a shifted window), builds the
copy, runs the pins that guard that part against it, and requires at least
one of them to fail.  The unmodified oracle passes every one of these pins
(they are ordinary tests of this suite), so a pin that fails here is failing
because of the planted mistake.
"""
import functools
import os

import pytest

from oracle import oracle as O
from tests import test_oracle_monte_carlo as MC
from tests import test_oracle_pins as P
from tests import test_oracle_worked_values as WV


def _pin(fn, *args):
    f = functools.partial(fn, *args)
    f.__name__ = fn.__name__ + (str(args) if args else "")
    return f


# name: (original text, mistaken text, pins expected to catch it)
MUTANTS = {
    # direct light (Sec. 3, Eq. 1)
    "smith k = alpha/2 for direct light": (
        "double kd = (r + 1.0) * (r + 1.0) / 8.0;", "double kd = r * r / 2.0;",
        [WV.test_direct_light_off_the_normal_by_hand]),
    "schlick fourth power": (
        "double fc = pow5(1.0 - VoH);", "double fc = pow(1.0 - VoH, 4.0);",
        [WV.test_direct_light_off_the_normal_by_hand]),
    "ggx alpha = roughness": (
        "double alpha = r * r;", "double alpha = r;",
        [P.test_direct_light_hand_value_at_normal_incidence, WV.test_direct_light_off_the_normal_by_hand]),
    "specular without N.L in the denominator": (
        "D * G * F / (4.0 * NoL * NoV)", "D * G * F / (4.0 * NoV)",
        [WV.test_direct_light_off_the_normal_by_hand]),
    "irradiance without the cosine": (
        "double e = f * rad * NoL;", "double e = f * rad;",
        [WV.test_direct_light_off_the_normal_by_hand]),
    "ambient occlusion on the direct light too": (
        "lo[c] = Llo[c] + aol * amb_lo;", "lo[c] = aol * (Llo[c] + amb_lo);",
        [WV.test_direct_light_off_the_normal_by_hand]),
    # ambient light (Sec. 3.1)
    "brdf table axes swapped": (
        "lut_bilinear(lut, lut_size, NoV, r, AB);", "lut_bilinear(lut, lut_size, r, NoV, AB);",
        [WV.test_ambient_by_hand_with_asymmetric_tables, MC.test_shading_matches_monte_carlo_lookups]),
    "irradiance looked up along the view vector": (
        "cube_bilinear_iv(irradiance, irr_size, n,", "cube_bilinear_iv(irradiance, irr_size, V,",
        [WV.test_ambient_by_hand_with_asymmetric_tables, MC.test_shading_matches_monte_carlo_lookups]),
    "prefiltered looked up at the normal": (
        "chain_trilinear_iv(pref_lo, pref_base, pref_levels, R, r * (pref_levels - 1),",
        "chain_trilinear_iv(pref_lo, pref_base, pref_levels, n, r * (pref_levels - 1),",
        [WV.test_ambient_by_hand_with_asymmetric_tables, MC.test_shading_matches_monte_carlo_lookups]),
    "prefiltered lod = r M": (
        "chain_trilinear_iv(pref_lo, pref_base, pref_levels, R, r * (pref_levels - 1),",
        "chain_trilinear_iv(pref_lo, pref_base, pref_levels, R, r * pref_levels,",
        [WV.test_ambient_by_hand_with_asymmetric_tables, MC.test_shading_matches_monte_carlo_lookups]),
    "k_S without the max": (
        "maxd(1.0 - r, F0[c])", "(1.0 - r)",
        [WV.test_ambient_by_hand_with_asymmetric_tables]),
    "F_avg with 1/20": (
        "(1.0 - F0[c]) / 21.0", "(1.0 - F0[c]) / 20.0",
        [WV.test_ambient_by_hand_with_asymmetric_tables]),
    "multiple scattering Ems = 1 - A": (
        "double Ems = 1.0 - Ess;", "double Ems = 1.0 - AB[0];",
        [WV.test_ambient_by_hand_with_asymmetric_tables, _pin(P.test_ambient_white_furnace, 1.0)]),
    "background along the reversed ray": (
        "cube_bilinear_iv(env, env_size, dw, tie->face, lo, hi);",
        "dw[0] = -dw[0]; dw[1] = -dw[1]; dw[2] = -dw[2];\n"
        "                cube_bilinear_iv(env, env_size, dw, tie->face, lo, hi);",
        [WV.test_background_follows_the_view_ray]),
    # conventions and the per-environment tables (Sec. 3.1)
    "texel solid angle without the square root": (
        "atan2(x * y, sqrt(x * x + y * y + 1.0))", "atan2(x * y, x * x + y * y + 1.0)",
        [_pin(P.test_texel_solid_angles_cover_the_sphere, 7), P.test_texel_solid_angle_single_face_and_symmetry]),
    "+X face with s mirrored": (
        "case 0: d[0] = 1;  d[1] = -t; d[2] = -s; break;", "case 0: d[0] = 1;  d[1] = -t; d[2] = s; break;",
        [P.test_cube_face_orientation_is_consistent]),
    "irradiance texels weighted equally": (
        "double c = maxd(0.0, dot3(n, q)) * q[3];", "double c = maxd(0.0, dot3(n, q));",
        [P.test_irradiance_matches_brute_force_monte_carlo]),
    "downsample weighted equally": (
        "acc[c] += p[c] * dw;", "acc[c] += p[c] * 1.0; dw = 1.0;",
        [P.test_downsample_conserves_radiant_integral_and_constants]),
    "prefilter without the N.L weight": (
        "alo[c] += Llo[c] * nl; ahi[c] += Lhi[c] * nl; }", "alo[c] += Llo[c]; ahi[c] += Lhi[c]; }",
        [P.test_prefilter_matches_quadrature_of_the_ggx_lobe]),
    "ggx sampling with alpha for alpha^2": (
        "sqrt((1.0 - u2) / (1.0 + (a2 - 1.0) * u2))", "sqrt((1.0 - u2) / (1.0 + (alpha - 1.0) * u2))",
        [P.test_prefilter_matches_quadrature_of_the_ggx_lobe, _pin(P.test_brdf_lut_matches_direct_quadrature, 0.5, 0.7)]),
    "brdf table with the direct-light k": (
        "k = alpha / 2.0;", "k = (rough + 1.0) * (rough + 1.0) / 8.0;",
        [_pin(P.test_brdf_lut_matches_direct_quadrature, 0.5, 0.7)]),
    # SSAO (Sec. 5.2)
    "ssao range term inverted": (
        "smoothstep01(radius / fabs(d - ds))", "smoothstep01(fabs(d - ds) / radius)",
        [P.test_ssao_step_by_hand]),
    "ssao bias with the wrong sign": (
        "double m = (zq - bias) - ds;", "double m = (zq + bias) - ds;",
        [P.test_ssao_unoccluded_fronto_parallel_plane, P.test_ssao_step_by_hand]),
    "ssao half-resolution index as floor(u / 2)": (
        "double hx = (u - 0.5) * 0.5 + 0.5", "double hx = u * 0.5",
        [WV.test_ssao_nearest_half_resolution_texel_by_hand]),
    "ssao half-resolution index half a texel late": (
        "double hx = (u - 0.5) * 0.5 + 0.5", "double hx = (u + 0.5) * 0.5 + 0.5",
        [WV.test_ssao_nearest_half_resolution_texel_by_hand]),
    "ssao blur window -1..2": (
        "for (int dy = -2; dy <= 1; ++dy)", "for (int dy = -1; dy <= 2; ++dy)",
        [WV.test_ssao_blur_by_hand_with_partial_weights]),
    "ssao blur relative to the neighbour's depth": (
        "(tau * dp)", "(tau * dq)",
        [WV.test_ssao_blur_by_hand_with_partial_weights]),
    "ao upsampled at pixel centres": (
        "double fx = x * 0.5, fy = y * 0.5;", "double fx = (x + 0.5) * 0.5 - 0.5, fy = (y + 0.5) * 0.5 - 0.5;",
        [P.test_edl_flat_depth_is_unshaded]),
    # shadows (Sec. 5.1)
    "pcf patch one texel right": (
        "int i0 = cu[a], j0 = cv[b];", "int i0 = cu[a] + 1, j0 = cv[b];",
        [P.test_pcf_lit_fraction_by_hand]),
    "pcf comparison reversed": (
        "double m = sd - ref;", "double m = ref - sd;",
        [P.test_pcf_lit_fraction_by_hand]),
    # bloom, composite, tone mapping (Sec. 5.3, 5.4)
    "bright map without the division by Y": (
        "maxd(Y - threshold, 0.0) / Y", "maxd(Y - threshold, 0.0)",
        [P.test_bloom_constant_field, WV.test_composite_upsample_position_by_hand]),
    "box blur instead of the binomial": (
        "static const double k[5] = {1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16};",
        "static const double k[5] = {0.2, 0.2, 0.2, 0.2, 0.2};",
        [P.test_bloom_impulse_by_hand, WV.test_composite_upsample_position_by_hand]),
    "pyramid texel as a sum": (
        "lvl[l][c * cp + (size_t)y * w + x] = s / n;", "lvl[l][c * cp + (size_t)y * w + x] = s / 4.0;",
        [P.test_bloom_ragged_levels_average_in_range_children]),
    "composite sampled without the half-texel shift": (
        "double fx = (x + 0.5) / sc - 0.5", "double fx = (x + 0.5) / sc",
        [WV.test_composite_upsample_position_by_hand]),
    "aces coefficient 0.3": (
        "(2.51 * x + 0.03)", "(2.51 * x + 0.3)",
        [P.test_aces_and_u8_table]),
    "gamma applied the wrong way": (
        "double g = pow(y, 1.0 / gamma);", "double g = pow(y, gamma);",
        [P.test_aces_and_u8_table, P.test_reinhard_curve_by_hand]),
    # surfel G-buffer (Sec. 4.4), eye-dome lighting (Sec. 4.3), ray cast
    "surfel albedo multiplied by the weight": (
        "albedo[c * n + p] /= w;", "albedo[c * n + p] *= w;",
        [P.test_normalize_gbuffer_divides_by_the_weight]),
    "edl response symmetric": (
        "response += maxd(0.0, zp -", "response += fabs(zp -",
        [P.test_edl_depth_step_by_hand]),
    "ray cast takes the far root": (
        "double t = (-b - sqrt(disc)) / aa;", "double t = (-b + sqrt(disc)) / aa;",
        [P.test_raycast_single_sphere_closed_forms]),
}


@pytest.fixture(scope="module")
def source():
    with open(O._SRC) as f:
        return f.read()


@pytest.mark.slow
@pytest.mark.parametrize("name", list(MUTANTS))
def test_pins_catch_planted_mistake(name, source, tmp_path):
    old, new, pins = MUTANTS[name]
    assert source.count(old) >= 1, f"{name}: text not found in the oracle source"
    src = tmp_path / "mutant.c"
    src.write_text(source.replace(old, new))
    path = O.build(str(src), str(tmp_path / "libmutant.so"))
    saved = O._lib
    O._lib = O.load(path)
    caught = []
    try:
        for pin in pins:
            try:
                pin()
            except AssertionError:
                caught.append(pin.__name__)
    finally:
        O._lib = saved
        os.remove(path)
    assert caught, f"{name}: none of {[p.__name__ for p in pins]} failed"
    print(f"{name}: caught by {caught}")
