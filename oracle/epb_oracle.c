/*
 * FP64 CPU oracle of the EasyPBR deferred screen-space shading pass.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark, never by the product library.  It shares no code
 * with the HIP implementation.  See epb_oracle.h for layouts and for the
 * interval ("lo"/"hi") treatment of floating-point decisions.
 *
 * Sources.  The paper fixes the structure: the reflectance equation (Sec. 3,
 * Eq. 1), a Cook-Torrance BRDF with metalness and roughness in the Unreal
 * Engine 4 variant (Sec. 3), image-based lighting from precomputed blurred cube
 * maps and the split-sum specular approximation (Sec. 3.1), multiple-scattering
 * compensation after Fdez-Aguera 2019 (Sec. 3.1), a depth-only G-buffer with
 * position reconstruction (Sec. 4, Tab. 1), shadow mapping with 3x3 PCF
 * (Sec. 5.1), normal-oriented hemisphere SSAO at half resolution with a
 * bilateral blur (Sec. 5.2), a bright-map pyramid bloom of up to six levels
 * blurred from the second level (Sec. 5.3), and ACES tone mapping with gamma
 * correction (Sec. 5.4).  The formulas are those of the methods the paper
 * cites (Karis 2013; Fdez-Aguera 2019; Bavoil and Sainz 2008; Williams 1978;
 * Reeves et al. 1987) and the Narkowicz fit of the ACES curve.
 */
#include "epb_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* small vector helpers                                                      */
/* ------------------------------------------------------------------------ */
static double dot3(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(const double a[3], const double b[3], double o[3]) {
    double x = a[1] * b[2] - a[2] * b[1];
    double y = a[2] * b[0] - a[0] * b[2];
    double z = a[0] * b[1] - a[1] * b[0];
    o[0] = x; o[1] = y; o[2] = z;
}
static void normalize3(double v[3]) {
    double n = sqrt(dot3(v, v));
    v[0] /= n; v[1] /= n; v[2] /= n;
}
static double clampd(double x, double a, double b) { return x < a ? a : (x > b ? b : x); }
static double mind(double a, double b) { return a < b ? a : b; }
static double maxd(double a, double b) { return a > b ? a : b; }
static double pow5(double x) { return x * x * x * x * x; }

/* R * v and R^T * v for a row-major 3x4 [R | t] */
static void rot(const double *m, const double v[3], double o[3]) {
    for (int r = 0; r < 3; ++r) o[r] = m[4 * r] * v[0] + m[4 * r + 1] * v[1] + m[4 * r + 2] * v[2];
}
static void rot_t(const double *m, const double v[3], double o[3]) {
    for (int c = 0; c < 3; ++c) o[c] = m[c] * v[0] + m[4 + c] * v[1] + m[8 + c] * v[2];
}

/* ------------------------------------------------------------------------ */
/* conventions                                                               */
/* ------------------------------------------------------------------------ */

/* Texel-centre direction of cube texel (i, j) on a face of size S (not unit). */
void orc_cube_texel_dir(int face, int i, int j, int S, double d[3]) {
    double s = 2.0 * (i + 0.5) / S - 1.0;
    double t = 2.0 * (j + 0.5) / S - 1.0;
    switch (face) {
    case 0: d[0] = 1;  d[1] = -t; d[2] = -s; break;
    case 1: d[0] = -1; d[1] = -t; d[2] = s;  break;
    case 2: d[0] = s;  d[1] = 1;  d[2] = t;  break;
    case 3: d[0] = s;  d[1] = -1; d[2] = -t; break;
    case 4: d[0] = s;  d[1] = -t; d[2] = 1;  break;
    default: d[0] = -s; d[1] = -t; d[2] = -1; break;
    }
}

/* Solid angle of a face texel: the solid angle of the rectangle from the face
 * centre to (x, y) on the plane at unit distance is atan2(x y, sqrt(x^2+y^2+1));
 * a texel is the inclusion-exclusion of its four corners. */
static double corner_area(double x, double y) { return atan2(x * y, sqrt(x * x + y * y + 1.0)); }
double orc_texel_solid_angle(int i, int j, int S) {
    double x0 = 2.0 * i / S - 1.0, x1 = 2.0 * (i + 1) / S - 1.0;
    double y0 = 2.0 * j / S - 1.0, y1 = 2.0 * (j + 1) / S - 1.0;
    return corner_area(x1, y1) - corner_area(x0, y1) - corner_area(x1, y0) + corner_area(x0, y0);
}

/* Direction -> (face, s, t) for one chosen major axis (0 = x, 1 = y, 2 = z). */
static void face_coords(const double d[3], int axis, int *face, double *s, double *t) {
    double ma;
    if (axis == 0) {
        ma = fabs(d[0]);
        if (d[0] >= 0) { *face = 0; *s = -d[2] / ma; *t = -d[1] / ma; }
        else           { *face = 1; *s = d[2] / ma;  *t = -d[1] / ma; }
    } else if (axis == 1) {
        ma = fabs(d[1]);
        if (d[1] >= 0) { *face = 2; *s = d[0] / ma; *t = d[2] / ma; }
        else           { *face = 3; *s = d[0] / ma; *t = -d[2] / ma; }
    } else {
        ma = fabs(d[2]);
        if (d[2] >= 0) { *face = 4; *s = d[0] / ma;  *t = -d[1] / ma; }
        else           { *face = 5; *s = -d[0] / ma; *t = -d[1] / ma; }
    }
}

/* Bilinear lookup with clamp-to-edge inside one face of a cube level. */
static void face_bilinear(const double *tex, int S, int face, double s, double t, double out[3]) {
    double x = (s + 1.0) * 0.5 * S - 0.5;
    double y = (t + 1.0) * 0.5 * S - 0.5;
    double fx0 = floor(x), fy0 = floor(y);
    double wx = x - fx0, wy = y - fy0;
    int x0 = (int)fx0, y0 = (int)fy0;
    int xa = x0 < 0 ? 0 : (x0 > S - 1 ? S - 1 : x0);
    int xb = x0 + 1 < 0 ? 0 : (x0 + 1 > S - 1 ? S - 1 : x0 + 1);
    int ya = y0 < 0 ? 0 : (y0 > S - 1 ? S - 1 : y0);
    int yb = y0 + 1 < 0 ? 0 : (y0 + 1 > S - 1 ? S - 1 : y0 + 1);
    const double *f = tex + (size_t)face * S * S * 4;
    for (int c = 0; c < 3; ++c) {
        double v00 = f[((size_t)ya * S + xa) * 4 + c], v10 = f[((size_t)ya * S + xb) * 4 + c];
        double v01 = f[((size_t)yb * S + xa) * 4 + c], v11 = f[((size_t)yb * S + xb) * 4 + c];
        out[c] = (1 - wy) * ((1 - wx) * v00 + wx * v10) + wy * ((1 - wx) * v01 + wx * v11);
    }
}

/* Candidate major axes: every axis whose magnitude is within the relative tie
 * margin of the largest one.  Returns the count, axes in x, y, z order. */
static int candidate_axes(const double d[3], double rel, int axes[3]) {
    double a[3] = {fabs(d[0]), fabs(d[1]), fabs(d[2])};
    double m = maxd(a[0], maxd(a[1], a[2]));
    int n = 0;
    for (int k = 0; k < 3; ++k)
        if (a[k] >= m * (1.0 - rel)) axes[n++] = k;
    return n;
}

/* Trilinear lookup in a mip chain at fractional lod, for one chosen axis. */
static void chain_trilinear(const double *chain, int base, int levels, const double d[3], int axis,
                            double lod, double out[3]) {
    int face; double s, t;
    face_coords(d, axis, &face, &s, &t);
    lod = clampd(lod, 0.0, (double)(levels - 1));
    int l0 = (int)floor(lod);
    int l1 = l0 + 1 < levels ? l0 + 1 : levels - 1;
    double f = lod - l0;
    size_t off = 0;
    const double *p0 = NULL, *p1 = NULL;
    for (int m = 0; m < levels; ++m) {
        int sm = base >> m;
        if (m == l0) p0 = chain + off;
        if (m == l1) p1 = chain + off;
        off += (size_t)6 * sm * sm * 4;
    }
    double a[3], b[3];
    face_bilinear(p0, base >> l0, face, s, t, a);
    face_bilinear(p1, base >> l1, face, s, t, b);
    for (int c = 0; c < 3; ++c) out[c] = (1 - f) * a[c] + f * b[c];
}

/* Bilinear lookup of one cube level, min and max over the ambiguous faces. */
static void cube_bilinear_iv(const double *tex, int S, const double d[3], double rel,
                             double lo[3], double hi[3]) {
    int axes[3];
    int n = candidate_axes(d, rel, axes);
    for (int c = 0; c < 3; ++c) { lo[c] = INFINITY; hi[c] = -INFINITY; }
    for (int k = 0; k < n; ++k) {
        int face; double s, t, v[3];
        face_coords(d, axes[k], &face, &s, &t);
        face_bilinear(tex, S, face, s, t, v);
        for (int c = 0; c < 3; ++c) { lo[c] = mind(lo[c], v[c]); hi[c] = maxd(hi[c], v[c]); }
    }
}

static void chain_trilinear_iv(const double *chain, int base, int levels, const double d[3],
                               double lod, double rel, double lo[3], double hi[3]) {
    int axes[3];
    int n = candidate_axes(d, rel, axes);
    for (int c = 0; c < 3; ++c) { lo[c] = INFINITY; hi[c] = -INFINITY; }
    for (int k = 0; k < n; ++k) {
        double v[3];
        chain_trilinear(chain, base, levels, d, axes[k], lod, v);
        for (int c = 0; c < 3; ++c) { lo[c] = mind(lo[c], v[c]); hi[c] = maxd(hi[c], v[c]); }
    }
}

/* Hammersley point k of n: (k / n, base-2 radical inverse of k). */
static double radical_inverse2(uint32_t k) {
    double r = 0.0, f = 0.5;
    while (k) {
        if (k & 1u) r += f;
        f *= 0.5;
        k >>= 1;
    }
    return r;
}

/* Tangent frame around n: up = +z unless n is within 0.999 of it, then +x. */
static void tangent_frame(const double n[3], double T[3], double B[3]) {
    double up[3] = {0, 0, 1};
    if (fabs(n[2]) >= 0.999) { up[0] = 1; up[2] = 0; }
    cross3(up, n, T);
    normalize3(T);
    cross3(n, T, B);
}

/* GGX distribution of half vectors (Karis 2013), alpha = roughness^2. */
double orc_ggx_D(double NoH, double alpha) {
    double a2 = alpha * alpha;
    double q = NoH * NoH * (a2 - 1.0) + 1.0;
    return a2 / (PI * q * q);
}

/* Importance-sampled half vector of GGX for the uniform point (u1, u2):
 * phi = 2 pi u1, cos(theta) = sqrt((1 - u2) / (1 + (alpha^2 - 1) u2)). */
static void ggx_half_vector(double u1, double u2, double alpha, const double n[3],
                            const double T[3], const double B[3], double h[3]) {
    double a2 = alpha * alpha;
    double phi = 2.0 * PI * u1;
    double ct = sqrt((1.0 - u2) / (1.0 + (a2 - 1.0) * u2));
    double st = sqrt(maxd(0.0, 1.0 - ct * ct));
    double hx = st * cos(phi), hy = st * sin(phi);
    for (int c = 0; c < 3; ++c) h[c] = T[c] * hx + B[c] * hy + n[c] * ct;
}

/* Smith-Schlick visibility factor G1(x) = x / (x (1 - k) + k). */
static double smith_g1(double x, double k) { return x / (x * (1.0 - k) + k); }

/* ------------------------------------------------------------------------ */
/* a1: image-based-lighting precompute (Sec. 3.1)                            */
/* ------------------------------------------------------------------------ */

/* One level of the solid-angle-weighted 2x2 mean: dst has size S/2. */
void orc_env_downsample(const double *src, int S, double *dst) {
    int Sd = S / 2;
    for (int f = 0; f < 6; ++f)
        for (int j = 0; j < Sd; ++j)
            for (int i = 0; i < Sd; ++i) {
                double acc[3] = {0, 0, 0}, w = 0;
                for (int b = 0; b < 2; ++b)
                    for (int a = 0; a < 2; ++a) {
                        int ci = 2 * i + a, cj = 2 * j + b;
                        double dw = orc_texel_solid_angle(ci, cj, S);
                        const double *p = src + (((size_t)f * S + cj) * S + ci) * 4;
                        for (int c = 0; c < 3; ++c) acc[c] += p[c] * dw;
                        w += dw;
                    }
                double *o = dst + (((size_t)f * Sd + j) * Sd + i) * 4;
                for (int c = 0; c < 3; ++c) o[c] = acc[c] / w;
                o[3] = 0.0;
            }
}

/* Diffuse irradiance map: cosine-weighted mean radiance around each output
 * texel direction, E(n) = sum L max(0, n.w) dW / sum max(0, n.w) dW over all
 * source texels (irradiance / pi, so that diffuse = c_diff * E). */
void orc_irradiance(const double *src, int S_src, double *out, int S_out) {
    int nsrc = 6 * S_src * S_src;
    double *dirs = malloc(sizeof(double) * 4 * nsrc);
    for (int f = 0; f < 6; ++f)
        for (int j = 0; j < S_src; ++j)
            for (int i = 0; i < S_src; ++i) {
                double *q = dirs + 4 * (((size_t)f * S_src + j) * S_src + i);
                orc_cube_texel_dir(f, i, j, S_src, q);
                normalize3(q);
                q[3] = orc_texel_solid_angle(i, j, S_src);
            }
#pragma omp parallel for schedule(dynamic)
    for (int o = 0; o < 6 * S_out * S_out; ++o) {
        int f = o / (S_out * S_out), j = (o / S_out) % S_out, i = o % S_out;
        double n[3];
        orc_cube_texel_dir(f, i, j, S_out, n);
        normalize3(n);
        double acc[3] = {0, 0, 0}, w = 0;
        for (int t = 0; t < nsrc; ++t) {
            const double *q = dirs + 4 * (size_t)t;
            double c = maxd(0.0, dot3(n, q)) * q[3];
            const double *L = src + 4 * (size_t)t;
            acc[0] += L[0] * c; acc[1] += L[1] * c; acc[2] += L[2] * c;
            w += c;
        }
        double *p = out + 4 * (size_t)o;
        p[0] = acc[0] / w; p[1] = acc[1] / w; p[2] = acc[2] / w; p[3] = 0.0;
    }
    free(dirs);
}

/* Split-sum prefiltered specular chain (Karis 2013): level m has size base >> m
 * and roughness m / (levels - 1); with N = V = R the texel direction, the value
 * is the N.L-weighted mean of the environment over GGX-sampled reflection
 * directions from a Hammersley sequence, looked up bilinearly in level 0.  A
 * sample whose cube-face choice is within the tie margin contributes the
 * smaller face value to lo and the larger to hi. */
/* Prefiltered chain.  With fis == 0 every GGX sample reads the environment
 * itself (level 0).  With fis != 0 (filtered importance sampling, Krivanek and
 * Colbert 2008) a sample reads a pre-blurred copy instead: the environment
 * chain (level m = solid-angle-weighted 2x2 means of level m - 1, down to 2x2
 * faces) at the level whose texels subtend the solid angle the sample stands
 * for, lod = 1/2 log2(omega_s / omega_p) + 1 with omega_s = 1 / (N pdf),
 * omega_p = 4 pi / (6 S^2) the base texel's mean solid angle and pdf the density
 * of the reflected direction, D(n.h) (n.h) / (4 v.h) = D / 4 for v = n; clamped
 * to the chain and read trilinearly. */
void orc_prefilter(const double *env, int S, double *out_lo, double *out_hi, int base, int levels,
                   int samples, double tie_rel, int fis) {
    int M = 0; /* last level of the environment chain (faces of at least 2x2) */
    while ((S >> (M + 1)) >= 2) ++M;
    double *chain = NULL;
    if (fis) {
        size_t tot = 0;
        for (int m = 0; m <= M; ++m) tot += (size_t)6 * (S >> m) * (S >> m) * 4;
        chain = malloc(sizeof(double) * tot);
        memcpy(chain, env, sizeof(double) * 6 * (size_t)S * S * 4);
        size_t o = 0;
        for (int m = 1; m <= M; ++m) {
            size_t prev = (size_t)6 * (S >> (m - 1)) * (S >> (m - 1)) * 4;
            orc_env_downsample(chain + o, S >> (m - 1), chain + o + prev);
            o += prev;
        }
    }
    double omega_p = 4.0 * PI / (6.0 * S * S);
    size_t off = 0;
    for (int m = 0; m < levels; ++m) {
        int sm = base >> m;
        double rough = levels > 1 ? (double)m / (levels - 1) : 0.0;
        double alpha = rough * rough;
#pragma omp parallel for schedule(dynamic)
        for (int o = 0; o < 6 * sm * sm; ++o) {
            int f = o / (sm * sm), j = (o / sm) % sm, i = o % sm;
            double n[3], T[3], B[3];
            orc_cube_texel_dir(f, i, j, sm, n);
            normalize3(n);
            tangent_frame(n, T, B);
            double alo[3] = {0, 0, 0}, ahi[3] = {0, 0, 0}, w = 0;
            for (int k = 0; k < samples; ++k) {
                double h[3], l[3], Llo[3], Lhi[3];
                ggx_half_vector((double)k / samples, radical_inverse2((uint32_t)k), alpha, n, T,
                                B, h);
                double vh = dot3(n, h);
                for (int c = 0; c < 3; ++c) l[c] = 2.0 * vh * h[c] - n[c];
                double nl = dot3(n, l);
                if (nl > 0.0) {
                    if (fis && alpha > 0.0) {
                        double pdf = orc_ggx_D(vh, alpha) * vh / (4.0 * vh);
                        double omega_s = 1.0 / (samples * pdf);
                        double lod = clampd(0.5 * log2(omega_s / omega_p) + 1.0, 0.0, (double)M);
                        chain_trilinear_iv(chain, S, M + 1, l, lod, tie_rel, Llo, Lhi);
                    } else {
                        cube_bilinear_iv(env, S, l, tie_rel, Llo, Lhi);
                    }
                    for (int c = 0; c < 3; ++c) { alo[c] += Llo[c] * nl; ahi[c] += Lhi[c] * nl; }
                    w += nl;
                }
            }
            double *pl = out_lo + off + 4 * (size_t)o, *ph = out_hi + off + 4 * (size_t)o;
            for (int c = 0; c < 3; ++c) { pl[c] = alo[c] / w; ph[c] = ahi[c] / w; }
            pl[3] = ph[3] = 0.0;
        }
        off += (size_t)6 * sm * sm * 4;
    }
    free(chain);
}

/* Split-sum environment BRDF (Karis 2013): with N = +z and V in the xz plane at
 * N.V, average over GGX half vectors of (1 - Fc) G_vis and Fc G_vis, where
 * G_vis = G VoH / (NoH NoV), G uses k = alpha / 2 and Fc = (1 - VoH)^5. */
void orc_brdf_lut_point(double NoV, double rough, int samples, double AB[2]) {
    double alpha = rough * rough, k = alpha / 2.0;
    double V[3] = {sqrt(maxd(0.0, 1.0 - NoV * NoV)), 0.0, NoV};
    double n[3] = {0, 0, 1}, T[3], B[3];
    tangent_frame(n, T, B);
    double A = 0, Bs = 0;
    for (int s = 0; s < samples; ++s) {
        double h[3], l[3];
        ggx_half_vector((double)s / samples, radical_inverse2((uint32_t)s), alpha, n, T, B, h);
        double vh = dot3(V, h);
        for (int c = 0; c < 3; ++c) l[c] = 2.0 * vh * h[c] - V[c];
        double nl = l[2], nh = h[2];
        if (nl > 0.0) {
            double G = smith_g1(nl, k) * smith_g1(NoV, k);
            double Gv = G * vh / (nh * NoV);
            double Fc = pow5(1.0 - vh);
            A += (1.0 - Fc) * Gv;
            Bs += Fc * Gv;
        }
    }
    AB[0] = A / samples;
    AB[1] = Bs / samples;
}

void orc_brdf_lut(double *out, int size, int samples) {
#pragma omp parallel for schedule(dynamic)
    for (int o = 0; o < size * size; ++o) {
        int j = o / size, i = o % size;
        orc_brdf_lut_point((i + 0.5) / size, (j + 0.5) / size, samples, out + 2 * (size_t)o);
    }
}

/* ------------------------------------------------------------------------ */
/* a2 / a3: normal-oriented hemisphere SSAO at half resolution (Sec. 5.2)    */
/* ------------------------------------------------------------------------ */

static double smoothstep01(double x) {
    double t = clampd(x, 0.0, 1.0);
    return t * t * (3.0 - 2.0 * t);
}

/* Candidate integer parts of a coordinate: floor(x) and, inside the tie band,
 * the neighbouring integer.  Returns the count (1 or 2). */
static int floor_candidates(double x, double tie, int out[2]) {
    int a = (int)floor(x - tie), b = (int)floor(x + tie);
    out[0] = a;
    if (b != a) { out[1] = b; return 2; }
    return 1;
}

void orc_ssao_raw(const double *depth, const double *normal, const orc_camera *cam,
                  const double *kernel, int n_samples, const double *noise, double radius,
                  double bias, const orc_tie *tie, double *lo, double *hi) {
    int W = cam->width, H = cam->height;
    int Wh = (W + 1) / 2, Hh = (H + 1) / 2;
    size_t plane = (size_t)W * H;
#pragma omp parallel for schedule(dynamic)
    for (int hj = 0; hj < Hh; ++hj)
        for (int hi_ = 0; hi_ < Wh; ++hi_) {
            size_t o = (size_t)hj * Wh + hi_;
            int x = 2 * hi_, y = 2 * hj;
            double d = depth[(size_t)y * W + x];
            if (isinf(d)) { lo[o] = 1.0; hi[o] = 1.0; continue; }
            /* view-space position and normal of the half-resolution point */
            double P[3] = {(x + 0.5 - cam->cx) / cam->fx * d, -(y + 0.5 - cam->cy) / cam->fy * d, -d};
            double nw[3] = {normal[(size_t)y * W + x], normal[plane + (size_t)y * W + x],
                            normal[2 * plane + (size_t)y * W + x]};
            double nv[3];
            rot(cam->world_to_cam, nw, nv);
            normalize3(nv);
            /* rotation noise tiled every 4x4 half-resolution texels, Gram-Schmidt */
            const double *rn = noise + 2 * ((size_t)(hj % 4) * 4 + (hi_ % 4));
            double r[3] = {rn[0], rn[1], 0.0};
            double rn_d = dot3(nv, r);
            double t[3] = {r[0] - nv[0] * rn_d, r[1] - nv[1] * rn_d, r[2] - nv[2] * rn_d};
            double r_perp = sqrt(dot3(t, t)); /* conditioning of the Gram-Schmidt step */
            normalize3(t);
            double b[3];
            cross3(nv, t, b);
            double occ_min_sum = 0.0, occ_max_sum = 0.0;
            double ax = P[0] / d, ay = P[1] / d; /* view-ray slopes of the pixel */
            for (int k = 0; k < n_samples; ++k) {
                const double *s = kernel + 3 * (size_t)k;
                double w[3], Q[3];
                for (int c = 0; c < 3; ++c) {
                    w[c] = t[c] * s[0] + b[c] * s[1] + nv[c] * s[2];
                    Q[c] = P[c] + radius * w[c];
                }
                double zq = -Q[2];
                double omin = INFINITY, omax = -INFINITY;
                /* magnitude scales of the decisions (epb_oracle.h): the sample
                 * offset's tangent part is amplified by the Gram-Schmidt step */
                double cond = (fabs(s[0]) + fabs(s[1])) / r_perp;
                double wn = sqrt(dot3(w, w));
                double ztie = tie->ssao_depth * (d + radius * (1.0 + cond) + fabs(bias));
                if (zq <= ztie) { omin = mind(omin, 0.0); omax = maxd(omax, 0.0); }
                if (zq > 0.0) {
                    double u = cam->cx + cam->fx * Q[0] / zq;
                    double v = cam->cy - cam->fy * Q[1] / zq;
                    double hx = (u - 0.5) * 0.5 + 0.5, hy = (v - 0.5) * 0.5 + 0.5;
                    double Dx = 0.5 * cam->fx * radius / zq, Dy = 0.5 * cam->fy * radius / zq;
                    double bx = tie->ssao_coord *
                                (1.0 + Dx * (fabs(w[0]) + fabs(ax * w[2]) + wn + cond) + fabs(hx) / 8.0);
                    double by = tie->ssao_coord *
                                (1.0 + Dy * (fabs(w[1]) + fabs(ay * w[2]) + wn + cond) + fabs(hy) / 8.0);
                    int cx[2], cy[2];
                    int ncx = floor_candidates(hx, bx, cx);
                    int ncy = floor_candidates(hy, by, cy);
                    for (int a = 0; a < ncx; ++a)
                        for (int bb = 0; bb < ncy; ++bb) {
                            int ix = cx[a], iy = cy[bb];
                            if (ix < 0 || ix >= Wh || iy < 0 || iy >= Hh) {
                                omin = mind(omin, 0.0); omax = maxd(omax, 0.0);
                                continue;
                            }
                            double ds = depth[(size_t)(2 * iy) * W + 2 * ix];
                            if (isinf(ds)) { omin = mind(omin, 0.0); omax = maxd(omax, 0.0); continue; }
                            double val = smoothstep01(radius / fabs(d - ds));
                            double m = (zq - bias) - ds; /* occluded iff m >= 0 */
                            double ctie = tie->ssao_depth * (fabs(ds - d) + radius * (1.0 + cond) + fabs(bias));
                            if (m >= ctie) { omin = mind(omin, val); omax = maxd(omax, val); }
                            else if (m <= -ctie) { omin = mind(omin, 0.0); omax = maxd(omax, 0.0); }
                            else {
                                omin = mind(omin, mind(0.0, val));
                                omax = maxd(omax, maxd(0.0, val));
                            }
                        }
                }
                occ_min_sum += omin;
                occ_max_sum += omax;
            }
            lo[o] = 1.0 - occ_max_sum / n_samples;
            hi[o] = 1.0 - occ_min_sum / n_samples;
        }
}

/* Depth-aware 4x4 mean at half resolution: offsets -2..1 in both axes, weight
 * max(0, 1 - |d_q - d_p| / (tau d_p)), zero for empty texels.  W, H are the
 * full-resolution sizes; half-resolution depth is the depth at (2i, 2j). */
void orc_ssao_blur(const double *raw_lo, const double *raw_hi, const double *depth, int W,
                   int H, double tau, double *lo, double *hi) {
    int Wh = (W + 1) / 2, Hh = (H + 1) / 2;
#pragma omp parallel for schedule(dynamic)
    for (int j = 0; j < Hh; ++j)
        for (int i = 0; i < Wh; ++i) {
            size_t o = (size_t)j * Wh + i;
            double dp = depth[(size_t)(2 * j) * W + 2 * i];
            if (isinf(dp)) { lo[o] = 1.0; hi[o] = 1.0; continue; }
            double sl = 0, sh = 0, sw = 0;
            for (int dy = -2; dy <= 1; ++dy)
                for (int dx = -2; dx <= 1; ++dx) {
                    int qi = i + dx, qj = j + dy;
                    if (qi < 0 || qi >= Wh || qj < 0 || qj >= Hh) continue;
                    double dq = depth[(size_t)(2 * qj) * W + 2 * qi];
                    double w = isinf(dq) ? 0.0 : maxd(0.0, 1.0 - fabs(dq - dp) / (tau * dp));
                    size_t q = (size_t)qj * Wh + qi;
                    sl += w * raw_lo[q];
                    sh += w * raw_hi[q];
                    sw += w;
                }
            lo[o] = sl / sw;
            hi[o] = sh / sw;
        }
}

/* ------------------------------------------------------------------------ */
/* G-buffer and shadow-map pass: nearest-hit ray cast of a sphere field      */
/* ------------------------------------------------------------------------ */

void orc_raycast(const orc_scene *s, const orc_camera *cam, double rel, double *depth, int32_t *id,
                 double *normal, double *albedo, double *rough, double *metal, uint8_t *ambiguous) {
    const int W = cam->width, H = cam->height;
    const double *M = cam->world_to_cam;
    double o[3];  /* camera position -R^T t */
    for (int c = 0; c < 3; ++c) o[c] = -(M[c] * M[3] + M[4 + c] * M[7] + M[8 + c] * M[11]);
    size_t plane_px = (size_t)W * H;
#pragma omp parallel for schedule(dynamic, 4)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            size_t p = (size_t)y * W + x;
            double v[3] = {(x + 0.5 - cam->cx) / cam->fx, -(y + 0.5 - cam->cy) / cam->fy, -1.0};
            double d[3];
            for (int c = 0; c < 3; ++c) d[c] = M[c] * v[0] + M[4 + c] * v[1] + M[8 + c] * v[2];
            double best = INFINITY;
            int who = -1, amb = 0;
            double aa = dot3(d, d);
            for (int k = 0; k < s->n; ++k) {
                const double *ck = s->center + 3 * k;
                double oc[3] = {o[0] - ck[0], o[1] - ck[1], o[2] - ck[2]};
                double b = dot3(d, oc);
                double c0 = dot3(oc, oc) - s->radius[k] * s->radius[k];
                double disc = b * b - aa * c0;
                if (fabs(disc) <= rel * fmax(b * b, fabs(aa * c0))) amb = 1;  /* grazing */
                if (disc < 0.0) continue;
                double t = (-b - sqrt(disc)) / aa;
                if (!(t > 0.0)) continue;
                if (fabs(t - best) <= rel * fmin(t, best)) amb = 1;  /* near tie */
                if (t < best) { best = t; who = k; }
            }
            if (s->plane && d[1] < 0.0) {
                double t = -o[1] / d[1];
                if (t > 0.0) {
                    if (fabs(t - best) <= rel * fmin(t, best)) amb = 1;
                    if (t < best) { best = t; who = s->n; }
                }
            }
            depth[p] = best;
            id[p] = who;
            if (ambiguous) ambiguous[p] = (uint8_t)amb;
            if (!normal) continue;
            double nr[3] = {0, 0, 0}, al[3] = {0, 0, 0}, rg = 0, mt = 0;
            if (who >= 0 && who < s->n) {
                const double *ck = s->center + 3 * who;
                for (int c = 0; c < 3; ++c) nr[c] = (o[c] + best * d[c] - ck[c]) / s->radius[who];
                normalize3(nr);
                for (int c = 0; c < 3; ++c) al[c] = s->albedo[3 * who + c];
                rg = s->rough[who];
                mt = s->metal[who];
            } else if (who == s->n) {
                nr[1] = 1.0;
                for (int c = 0; c < 3; ++c) al[c] = s->plane_albedo[c];
                rg = s->plane_rough;
                mt = s->plane_metal;
            }
            for (int c = 0; c < 3; ++c) {
                normal[c * plane_px + p] = nr[c];
                albedo[c * plane_px + p] = al[c];
            }
            rough[p] = rg;
            metal[p] = mt;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* surfel G-buffer (Sec. 4.4): overlapping surfels add their attributes and  */
/* a weight; the compose pass first divides by that weight                   */
/* ------------------------------------------------------------------------ */

/* Normalises the accumulated normal, albedo, roughness and metalness of every
 * pixel with weight > 0 by that weight, in place; pixels with weight <= 0 are
 * left as they are (no surfel covered them). */
void orc_normalize_gbuffer(const double *weight, int W, int H, double *normal, double *albedo,
                           double *rough, double *metal) {
    size_t n = (size_t)W * H;
    for (size_t p = 0; p < n; ++p) {
        double w = weight[p];
        if (!(w > 0.0)) continue;
        for (int c = 0; c < 3; ++c) {
            normal[c * n + p] /= w;
            albedo[c * n + p] /= w;
        }
        rough[p] /= w;
        metal[p] /= w;
    }
}

/* ------------------------------------------------------------------------ */
/* a4: deferred shading (Sec. 3, 3.1, 4, 5.1, 5.4)                           */
/* ------------------------------------------------------------------------ */

/* Lit fraction of a 3x3 percentage-closer patch around the projection of the
 * world point Pw into a light's depth map, as an interval over ties; cam_pos
 * is the position of the camera whose depth the point was reconstructed from
 * (it sets the magnitude scale of the float decisions). */
static void pcf_shadow(const orc_light *L, const double Pw[3], const double cam_pos[3],
                       const orc_tie *tie, double *slo, double *shi) {
    const orc_camera *c = &L->shadow_cam;
    double Pl[3];
    rot(c->world_to_cam, Pw, Pl);
    Pl[0] += c->world_to_cam[3]; Pl[1] += c->world_to_cam[7]; Pl[2] += c->world_to_cam[11];
    double dl = -Pl[2];
    /* magnitude scales: distances point - camera and camera - light camera */
    double lt[3] = {c->world_to_cam[3], c->world_to_cam[7], c->world_to_cam[11]}, lpos[3];
    rot_t(c->world_to_cam, lt, lpos);
    double pc[3] = {Pw[0] - cam_pos[0], Pw[1] - cam_pos[1], Pw[2] - cam_pos[2]};
    double cl[3] = {cam_pos[0] + lpos[0], cam_pos[1] + lpos[1], cam_pos[2] + lpos[2]};
    double dist = sqrt(dot3(pc, pc)) + sqrt(dot3(cl, cl));
    double dtie = tie->pcf_depth * (dist + fabs(dl) + fabs(L->shadow_bias));
    double lo = INFINITY, hi = -INFINITY;
    if (dl <= dtie) { lo = 1.0; hi = 1.0; } /* behind the light camera: lit */
    if (dl > 0.0) {
        int w = c->width, h = c->height;
        double u = c->cx + c->fx * Pl[0] / dl;
        double v = c->cy - c->fy * Pl[1] / dl;
        double bu = tie->pcf_coord * (c->fx * dist / dl + fabs(u - c->cx) + fabs(c->cx));
        double bv = tie->pcf_coord * (c->fy * dist / dl + fabs(v - c->cy) + fabs(c->cy));
        int cu[2], cv[2];
        int nu = floor_candidates(u, bu, cu);
        int nv = floor_candidates(v, bv, cv);
        for (int a = 0; a < nu; ++a)
            for (int b = 0; b < nv; ++b) {
                int i0 = cu[a], j0 = cv[b];
                if (i0 < 0 || i0 >= w || j0 < 0 || j0 >= h) { /* outside the map: lit */
                    lo = mind(lo, 1.0); hi = maxd(hi, 1.0);
                    continue;
                }
                int sure = 0, maybe = 0;
                double ref = dl - L->shadow_bias;
                for (int dj = -1; dj <= 1; ++dj)
                    for (int di = -1; di <= 1; ++di) {
                        int ti = i0 + di, tj = j0 + dj;
                        if (ti < 0 || ti >= w || tj < 0 || tj >= h) { ++sure; continue; }
                        double sd = L->shadow_map[(size_t)tj * w + ti];
                        double m = sd - ref; /* lit iff ref <= sd */
                        if (isinf(sd) || m >= dtie) ++sure;
                        else if (m > -dtie) ++maybe;
                    }
                lo = mind(lo, sure / 9.0);
                hi = maxd(hi, (sure + maybe) / 9.0);
            }
    }
    *slo = lo;
    *shi = hi;
}

/* Bilinear lookup in a 2-channel LUT at (x, y) in [0, 1]^2 texel-centre space. */
static void lut_bilinear(const double *lut, int size, double x, double y, double out[2]) {
    double fx = x * size - 0.5, fy = y * size - 0.5;
    double x0f = floor(fx), y0f = floor(fy);
    double wx = fx - x0f, wy = fy - y0f;
    int x0 = (int)x0f, y0 = (int)y0f;
    int xa = x0 < 0 ? 0 : (x0 > size - 1 ? size - 1 : x0);
    int xb = x0 + 1 < 0 ? 0 : (x0 + 1 > size - 1 ? size - 1 : x0 + 1);
    int ya = y0 < 0 ? 0 : (y0 > size - 1 ? size - 1 : y0);
    int yb = y0 + 1 < 0 ? 0 : (y0 + 1 > size - 1 ? size - 1 : y0 + 1);
    for (int c = 0; c < 2; ++c) {
        double v00 = lut[((size_t)ya * size + xa) * 2 + c], v10 = lut[((size_t)ya * size + xb) * 2 + c];
        double v01 = lut[((size_t)yb * size + xa) * 2 + c], v11 = lut[((size_t)yb * size + xb) * 2 + c];
        out[c] = (1 - wy) * ((1 - wx) * v00 + wx * v10) + wy * ((1 - wx) * v01 + wx * v11);
    }
}

/* Half-resolution AO bilinearly upsampled at full-resolution pixel (x, y):
 * sample point (x / 2, y / 2) in half-resolution texel space, clamped. */
static double ao_upsample(const double *ao, int Wh, int Hh, int x, int y) {
    double fx = x * 0.5, fy = y * 0.5;
    int x0 = (int)floor(fx), y0 = (int)floor(fy);
    double wx = fx - x0, wy = fy - y0;
    int x1 = x0 + 1 < Wh ? x0 + 1 : Wh - 1;
    int y1 = y0 + 1 < Hh ? y0 + 1 : Hh - 1;
    double a = ao[(size_t)y0 * Wh + x0], b = ao[(size_t)y0 * Wh + x1];
    double c = ao[(size_t)y1 * Wh + x0], d = ao[(size_t)y1 * Wh + x1];
    return (1 - wy) * ((1 - wx) * a + wx * b) + wy * ((1 - wx) * c + wx * d);
}

void orc_shade(const double *depth, const double *normal, const double *albedo,
               const double *rough, const double *metal, const orc_camera *cam,
               const double *ao_lo, const double *ao_hi, const orc_light *lights, int n_lights,
               const double *irradiance, int irr_size, const double *pref_lo, const double *pref_hi,
               int pref_base, int pref_levels, const double *lut, int lut_size, const double *env,
               int env_size, const orc_tie *tie, double *hdr_lo, double *hdr_hi) {
    int W = cam->width, H = cam->height;
    int Wh = (W + 1) / 2, Hh = (H + 1) / 2;
    size_t plane = (size_t)W * H;
    const double *M = cam->world_to_cam;
    double tvec[3] = {M[3], M[7], M[11]};
    double cam_pos[3];
    rot_t(M, tvec, cam_pos);
    for (int c = 0; c < 3; ++c) cam_pos[c] = -cam_pos[c];
#pragma omp parallel for schedule(dynamic)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t p = (size_t)y * W + x;
            double d = depth[p];
            double dirv[3] = {(x + 0.5 - cam->cx) / cam->fx, -(y + 0.5 - cam->cy) / cam->fy, -1.0};
            double lo[3], hi[3];
            if (isinf(d)) {
                /* background: the environment along the view ray */
                double dw[3];
                rot_t(M, dirv, dw);
                cube_bilinear_iv(env, env_size, dw, tie->face, lo, hi);
            } else {
                /* position from depth (Sec. 4): world point and unit view vector */
                double Pv[3] = {dirv[0] * d, dirv[1] * d, -d};
                double Pr[3], Pw[3], V[3];
                rot_t(M, Pv, Pr); /* world point relative to the camera */
                for (int c = 0; c < 3; ++c) { Pw[c] = Pr[c] + cam_pos[c]; V[c] = -Pr[c]; }
                normalize3(V);
                double n[3] = {normal[p], normal[plane + p], normal[2 * plane + p]};
                normalize3(n);
                double alb[3] = {albedo[p], albedo[plane + p], albedo[2 * plane + p]};
                double r = rough[p], mt = metal[p];
                double nv_raw = dot3(n, V);
                double NoV = clampd(nv_raw, 1e-4, 1.0);
                double F0[3], cd[3];
                for (int c = 0; c < 3; ++c) {
                    F0[c] = 0.04 * (1.0 - mt) + alb[c] * mt;
                    cd[c] = alb[c] * (1.0 - mt);
                }
                double alpha = r * r;
                double kd = (r + 1.0) * (r + 1.0) / 8.0;
                /* direct light: Cook-Torrance GGX / Smith-Schlick / Schlick (Sec. 3) */
                double Llo[3] = {0, 0, 0}, Lhi[3] = {0, 0, 0};
                for (int li = 0; li < n_lights; ++li) {
                    const orc_light *L = &lights[li];
                    double l[3] = {L->pos[0] - Pw[0], L->pos[1] - Pw[1], L->pos[2] - Pw[2]};
                    double dist2 = dot3(l, l);
                    normalize3(l);
                    double NoL = dot3(n, l);
                    if (NoL <= 0.0) continue;
                    double h[3] = {V[0] + l[0], V[1] + l[1], V[2] + l[2]};
                    normalize3(h);
                    double NoH = dot3(n, h), VoH = maxd(0.0, dot3(V, h));
                    double D = orc_ggx_D(NoH, alpha);
                    double G = smith_g1(NoL, kd) * smith_g1(NoV, kd);
                    double fc = pow5(1.0 - VoH);
                    double slo = 1.0, shi = 1.0;
                    if (L->shadow_map) pcf_shadow(L, Pw, cam_pos, tie, &slo, &shi);
                    for (int c = 0; c < 3; ++c) {
                        double F = F0[c] + (1.0 - F0[c]) * fc;
                        double f = cd[c] / PI + D * G * F / (4.0 * NoL * NoV);
                        double rad = L->color[c] * L->intensity / dist2;
                        double e = f * rad * NoL;
                        Llo[c] += e * slo;
                        Lhi[c] += e * shi;
                    }
                }
                /* ambient: split-sum IBL with multiple scattering (Sec. 3.1) */
                double AB[2];
                lut_bilinear(lut, lut_size, NoV, r, AB);
                double Elo[3], Ehi[3], Plo[3], Phi[3];
                cube_bilinear_iv(irradiance, irr_size, n, tie->face, Elo, Ehi);
                double R[3] = {2.0 * nv_raw * n[0] - V[0], 2.0 * nv_raw * n[1] - V[1],
                               2.0 * nv_raw * n[2] - V[2]};
                double Pa[3], Pb[3];
                chain_trilinear_iv(pref_lo, pref_base, pref_levels, R, r * (pref_levels - 1),
                                   tie->face, Plo, Pa);
                chain_trilinear_iv(pref_hi, pref_base, pref_levels, R, r * (pref_levels - 1),
                                   tie->face, Pb, Phi);
                for (int c = 0; c < 3; ++c) { Plo[c] = mind(Plo[c], Pb[c]); Phi[c] = maxd(Phi[c], Pa[c]); }
                double aol = ao_upsample(ao_lo, Wh, Hh, x, y);
                double aoh = ao_upsample(ao_hi, Wh, Hh, x, y);
                double fc5 = pow5(1.0 - NoV);
                for (int c = 0; c < 3; ++c) {
                    double kS = F0[c] + (maxd(1.0 - r, F0[c]) - F0[c]) * fc5;
                    double FssEss = kS * AB[0] + AB[1];
                    double Ess = AB[0] + AB[1];
                    double Ems = 1.0 - Ess;
                    double Favg = F0[c] + (1.0 - F0[c]) / 21.0;
                    double Fms = FssEss * Favg / (1.0 - Ems * Favg);
                    double kD = cd[c] * (1.0 - FssEss - Fms * Ems);
                    double ce = Fms * Ems + kD;
                    double amb_lo = FssEss * Plo[c] + ce * Elo[c];
                    double amb_hi = FssEss * Phi[c] + ce * Ehi[c];
                    lo[c] = Llo[c] + aol * amb_lo;
                    hi[c] = Lhi[c] + aoh * amb_hi;
                }
            }
            for (int c = 0; c < 3; ++c) {
                hdr_lo[c * plane + p] = lo[c];
                hdr_hi[c * plane + p] = hi[c];
            }
        }
}

/* ------------------------------------------------------------------------ */
/* Eye-dome lighting of depth-only renders such as point clouds (Sec. 4.3):  */
/* the compositing step darkens a pixel by how far it lies behind the pixels  */
/* around it in screen space, using nothing but the depth map.               */
/* ------------------------------------------------------------------------ */

/* The neighbourhood: n_dirs directions 2 pi k / n_dirs around the pixel, each
 * taken radius pixels away and rounded to the nearest pixel (x right, y down),
 * halves away from zero; a coordinate within 1e-9 of a half counts as the half
 * (sin 30 degrees is not exactly 1/2 in floating point). */
static int edl_round(double v) {
    double m = floor(fabs(v) + 0.5 + 1e-9);
    return (int)(v < 0 ? -m : m);
}
void orc_edl_offsets(int radius, int n_dirs, int *dx, int *dy) {
    for (int k = 0; k < n_dirs; ++k) {
        double a = 2.0 * PI * (double)k / (double)n_dirs;
        dx[k] = edl_round(radius * cos(a));
        dy[k] = edl_round(radius * sin(a));
    }
}

/* Depth on the logarithmic scale the comparison uses; background (+inf) and
 * anything farther than far_depth count as far_depth. */
static double edl_log_depth(double d, double far_depth) { return log2(d < far_depth ? d : far_depth); }

/* Per pixel p: response = (1 / n) sum over the in-image neighbours q of
 * max(0, log2 d_p - log2 d_q) (neighbours outside the image add nothing);
 * shade = 2^(-strength * response).  Foreground pixels return shade * AO *
 * colour (AO upsampled as in shading; NULL means 1), background pixels shade
 * times the environment along the view ray (NULL environment: black). */
void orc_edl(const double *depth, const double *color, const orc_camera *cam, const double *ao_lo,
             const double *ao_hi, int radius, int n_dirs, double strength, double far_depth,
             const double *env, int env_size, double tie_rel, double *hdr_lo, double *hdr_hi) {
    int W = cam->width, H = cam->height;
    int Wh = (W + 1) / 2, Hh = (H + 1) / 2;
    size_t plane = (size_t)W * H;
    const double *M = cam->world_to_cam;
    int dx[64], dy[64];
    orc_edl_offsets(radius, n_dirs, dx, dy);
#pragma omp parallel for schedule(dynamic)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t p = (size_t)y * W + x;
            double zp = edl_log_depth(depth[p], far_depth);
            double response = 0.0;
            for (int k = 0; k < n_dirs; ++k) {
                int qx = x + dx[k], qy = y + dy[k];
                if (qx < 0 || qx >= W || qy < 0 || qy >= H) continue;
                response += maxd(0.0, zp - edl_log_depth(depth[(size_t)qy * W + qx], far_depth));
            }
            response /= n_dirs;
            double shade = exp2(-strength * response);
            double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
            if (isinf(depth[p])) {
                if (env) {
                    double dirv[3] = {(x + 0.5 - cam->cx) / cam->fx, -(y + 0.5 - cam->cy) / cam->fy, -1.0};
                    double dw[3];
                    rot_t(M, dirv, dw);
                    cube_bilinear_iv(env, env_size, dw, tie_rel, lo, hi);
                }
                for (int c = 0; c < 3; ++c) { lo[c] *= shade; hi[c] *= shade; }
            } else {
                double aol = ao_lo ? ao_upsample(ao_lo, Wh, Hh, x, y) : 1.0;
                double aoh = ao_hi ? ao_upsample(ao_hi, Wh, Hh, x, y) : 1.0;
                for (int c = 0; c < 3; ++c) {
                    lo[c] = shade * aol * color[c * plane + p];
                    hi[c] = shade * aoh * color[c * plane + p];
                }
            }
            for (int c = 0; c < 3; ++c) {
                hdr_lo[c * plane + p] = lo[c];
                hdr_hi[c * plane + p] = hi[c];
            }
        }
}

/* ------------------------------------------------------------------------ */
/* a5 / a6: bloom pyramid, composite, ACES tonemap, gamma, 8 bit             */
/* ------------------------------------------------------------------------ */

/* ACES filmic curve, Narkowicz rational fit. */
double orc_aces(double x) {
    return (x * (2.51 * x + 0.03)) / (x * (2.43 * x + 0.59) + 0.14);
}

/* Exposure, ACES, clamp to [0, 1], gamma 1/g, round half up to 8 bits. */
/* Reinhard's global operator, per channel (the paper's second tone curve). */
double orc_reinhard(double x) { return x / (1.0 + x); }

int orc_encode_u8_op(double x, double exposure, double gamma, int tonemap) {
    double e = exposure * x;
    double y = clampd(tonemap == 1 ? orc_reinhard(e) : orc_aces(e), 0.0, 1.0);
    double g = pow(y, 1.0 / gamma);
    int q = (int)floor(255.0 * g + 0.5);
    return q < 0 ? 0 : (q > 255 ? 255 : q);
}

int orc_encode_u8(double x, double exposure, double gamma) {
    double y = clampd(orc_aces(exposure * x), 0.0, 1.0);
    double g = pow(y, 1.0 / gamma);
    int q = (int)floor(255.0 * g + 0.5);
    return q < 0 ? 0 : (q > 255 ? 255 : q);
}

/* one 5-tap binomial pass, clamp to edge; horizontal if dx == 1 */
static void binomial_pass(const double *src, double *dst, int w, int h, int horizontal) {
    static const double k[5] = {1.0 / 16, 4.0 / 16, 6.0 / 16, 4.0 / 16, 1.0 / 16};
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            double s = 0.0;
            for (int t = -2; t <= 2; ++t) {
                int xx = x, yy = y;
                if (horizontal) xx = x + t < 0 ? 0 : (x + t > w - 1 ? w - 1 : x + t);
                else yy = y + t < 0 ? 0 : (y + t > h - 1 ? h - 1 : y + t);
                s += k[t + 2] * src[(size_t)yy * w + xx];
            }
            dst[(size_t)y * w + x] = s;
        }
}

void orc_bloom_tonemap(const double *hdr, int W, int H, int levels, double threshold,
                       double strength, double exposure, double gamma, int tonemap, uint8_t *ldr,
                       double *composite, double *pyramid) {
    size_t plane = (size_t)W * H;
    int nl = levels - 1; /* levels 1 .. levels-1 are built, blurred and added back */
    int *lw = malloc(sizeof(int) * (levels + 1)), *lh = malloc(sizeof(int) * (levels + 1));
    double **lvl = malloc(sizeof(double *) * (levels + 1));
    lw[0] = W; lh[0] = H;
    /* level 0: the bright map, c max(Y - T, 0) / Y with Rec. 709 luminance Y */
    lvl[0] = malloc(sizeof(double) * 3 * plane);
    for (size_t p = 0; p < plane; ++p) {
        double R = hdr[p], G = hdr[plane + p], B = hdr[2 * plane + p];
        double Y = 0.2126 * R + 0.7152 * G + 0.0722 * B;
        double s = Y > 0.0 ? maxd(Y - threshold, 0.0) / Y : 0.0;
        lvl[0][p] = R * s; lvl[0][plane + p] = G * s; lvl[0][2 * plane + p] = B * s;
    }
    /* levels 1..: mean of the in-range children of the previous level */
    for (int l = 1; l <= nl; ++l) {
        int pw = lw[l - 1], ph = lh[l - 1];
        int w = (pw + 1) / 2, h = (ph + 1) / 2;
        lw[l] = w; lh[l] = h;
        size_t pp = (size_t)pw * ph, cp = (size_t)w * h;
        lvl[l] = malloc(sizeof(double) * 3 * cp);
        for (int c = 0; c < 3; ++c)
            for (int y = 0; y < h; ++y)
                for (int x = 0; x < w; ++x) {
                    double s = 0; int n = 0;
                    for (int b = 0; b < 2; ++b)
                        for (int a = 0; a < 2; ++a) {
                            int xx = 2 * x + a, yy = 2 * y + b;
                            if (xx < pw && yy < ph) { s += lvl[l - 1][c * pp + (size_t)yy * pw + xx]; ++n; }
                        }
                    lvl[l][c * cp + (size_t)y * w + x] = s / n;
                }
    }
    /* blur levels 1.. with the separable [1 4 6 4 1] / 16 kernel */
    double **blur = malloc(sizeof(double *) * (levels + 1));
    size_t poff = 0;
    for (int l = 1; l <= nl; ++l) {
        int w = lw[l], h = lh[l];
        size_t cp = (size_t)w * h;
        blur[l] = malloc(sizeof(double) * 3 * cp);
        double *tmp = malloc(sizeof(double) * cp);
        for (int c = 0; c < 3; ++c) {
            binomial_pass(lvl[l] + c * cp, tmp, w, h, 1);
            binomial_pass(tmp, blur[l] + c * cp, w, h, 0);
        }
        free(tmp);
        if (pyramid) {
            memcpy(pyramid + poff, blur[l], sizeof(double) * 3 * cp);
            poff += 3 * cp;
        }
    }
    /* composite: HDR + strength * sum of bilinearly upsampled blurred levels */
#pragma omp parallel for schedule(dynamic)
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t p = (size_t)y * W + x;
            double C[3] = {hdr[p], hdr[plane + p], hdr[2 * plane + p]};
            for (int l = 1; l <= nl; ++l) {
                int w = lw[l], h = lh[l];
                size_t cp = (size_t)w * h;
                double sc = (double)(1 << l);
                double fx = (x + 0.5) / sc - 0.5, fy = (y + 0.5) / sc - 0.5;
                double x0f = floor(fx), y0f = floor(fy);
                double wx = fx - x0f, wy = fy - y0f;
                int x0 = (int)x0f, y0 = (int)y0f;
                int xa = x0 < 0 ? 0 : (x0 > w - 1 ? w - 1 : x0);
                int xb = x0 + 1 < 0 ? 0 : (x0 + 1 > w - 1 ? w - 1 : x0 + 1);
                int ya = y0 < 0 ? 0 : (y0 > h - 1 ? h - 1 : y0);
                int yb = y0 + 1 < 0 ? 0 : (y0 + 1 > h - 1 ? h - 1 : y0 + 1);
                for (int c = 0; c < 3; ++c) {
                    const double *b = blur[l] + c * cp;
                    double v = (1 - wy) * ((1 - wx) * b[(size_t)ya * w + xa] + wx * b[(size_t)ya * w + xb]) +
                               wy * ((1 - wx) * b[(size_t)yb * w + xa] + wx * b[(size_t)yb * w + xb]);
                    C[c] += strength * v;
                }
            }
            for (int c = 0; c < 3; ++c) {
                if (composite) composite[c * plane + p] = C[c];
                ldr[4 * p + c] = (uint8_t)orc_encode_u8_op(C[c], exposure, gamma, tonemap);
            }
            ldr[4 * p + 3] = 255;
        }
    for (int l = 0; l <= nl; ++l) free(lvl[l]);
    for (int l = 1; l <= nl; ++l) free(blur[l]);
    free(lvl); free(blur); free(lw); free(lh);
}

/* Threads of the parallel loops (timing the oracle on 1 and on all cores). */
void orc_set_threads(int n) {
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}
