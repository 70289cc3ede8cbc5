/*
 * FP64 CPU oracle of the EasyPBR deferred screen-space shading pass.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the HIP implementation.
 *
 * Every routine is the plain, slow reading of the method in double precision:
 * no blocking, fusion or reordering beyond what the method states.  The paper
 * names the methods and cites them; the formulas below follow those published
 * methods, and every point the paper leaves open is read the same way as in the
 * design notes (conventions, constants, tie-breaks).
 *
 * Decisions taken by a floating-point comparison (an SSAO depth test, a PCF
 * depth test, a nearest-texel floor, a cube-face choice) may legitimately come
 * out differently in a float32 implementation when the operands are within
 * rounding distance of the threshold.  Where an operand lies within the tie
 * margin the oracle evaluates every outcome and reports the smallest and the
 * largest result ("lo" and "hi").  All later steps are monotone in these values,
 * so the interval propagates exactly.  Away from ties lo == hi.
 *
 * Layouts (all row-major, y down):
 *   planar image   [c][H][W]
 *   cube map       [face][S][S][4]   faces +X,-X,+Y,-Y,+Z,-Z, RGBA (A unused)
 *   mip chain      levels concatenated, level m of size base >> m
 *   BRDF LUT       [size][size][2]   row = roughness, column = N.V, (A, B)
 */
#ifndef EPB_ORACLE_H
#define EPB_ORACLE_H
#include <stdint.h>

typedef struct {
    double world_to_cam[12]; /* row-major 3x4 [R | t] */
    double fx, fy, cx, cy;
    int32_t width, height;
} orc_camera;

/* Half-widths of the ambiguous bands of the float decisions.  A float32
 * implementation forms each decision's operand from terms whose magnitudes
 * add up to a scale S; its rounding error is then a small multiple of
 * 2^-24 S.  Each field below is that multiple (as a fraction of S), and the
 * oracle treats an operand within field * S of the threshold as a tie:
 *   ssao_coord  floors and in-image tests of an SSAO sample's half-resolution
 *               coordinate h = u/2 + 1/4 (v alike), formed as the pixel's own
 *               coordinate plus the sample's offset:
 *               S = 1 + D (|w_x| + |a_x w_z| + |w| + g) + |h| / 8, with
 *               D = f_x r / (2 z_q), w the view-space offset of the kernel
 *               vector s, a_x the pixel's view-ray slope (P_x / d) and
 *               g = (|s_x| + |s_y|) / |r_perp|, the amplification of the
 *               tangent's error by the Gram-Schmidt step (r_perp: the noise
 *               vector minus its normal part, before normalisation);
 *   ssao_depth  the SSAO depth test d_s <= z_q - bias, formed as the difference
 *               of the sampled and the pixel's own depth against the sample's
 *               offset: S = |d_s - d| + r (1 + g) + |bias|; the in-front test
 *               z_q > 0: S = d + r (1 + g) + |bias|;
 *   pcf_coord   the floors and in-map tests of the light-map coordinate u (v
 *               alike) of a point reconstructed from camera depth:
 *               S = f_l (|P - c| + |c - l|) / d_l + |u - c_l| + |c_l|, with P
 *               the point, c the camera position, l the light camera's
 *               position, f_l, c_l the light camera's focal length and
 *               principal point;
 *   pcf_depth   the PCF depth test d_l - bias <= map and the in-front test
 *               d_l > 0: S = |P - c| + |c - l| + |d_l| + |bias|;
 *   face        cube-face choices: S = the largest component magnitude. */
typedef struct {
    double ssao_coord, ssao_depth, pcf_coord, pcf_depth, face;
} orc_tie;

typedef struct {
    double pos[3], color[3], intensity;
    const double *shadow_map; /* [h][w] linear depth, +inf = empty; NULL = no shadow */
    orc_camera shadow_cam;
    double shadow_bias;
} orc_light;

/* conventions */
void orc_cube_texel_dir(int face, int i, int j, int S, double d[3]);
double orc_texel_solid_angle(int i, int j, int S);

/* building blocks exported for the pin tests */
double orc_ggx_D(double NoH, double alpha);
void orc_brdf_lut_point(double NoV, double rough, int samples, double AB[2]);
double orc_aces(double x);
double orc_reinhard(double x);
int orc_encode_u8(double x, double exposure, double gamma);
/* tonemap 0: ACES, 1: Reinhard */
int orc_encode_u8_op(double x, double exposure, double gamma, int tonemap);

/* a1 image-based-lighting precompute */
void orc_env_downsample(const double *src, int S, double *dst);
void orc_irradiance(const double *src, int S_src, double *out, int S_out);
/* fis != 0: filtered importance sampling (each sample reads the environment's
 * solid-angle-weighted mip chain at the level its pdf asks for). */
void orc_prefilter(const double *env, int S, double *out_lo, double *out_hi, int base, int levels,
                   int samples, double tie_rel, int fis);
void orc_brdf_lut(double *out, int size, int samples);

/* a2 / a3 screen-space ambient occlusion */
void orc_ssao_raw(const double *depth, const double *normal, const orc_camera *cam,
                  const double *kernel, int n_samples, const double *noise, double radius,
                  double bias, const orc_tie *tie, double *lo, double *hi);
void orc_ssao_blur(const double *raw_lo, const double *raw_hi, const double *depth, int W,
                   int H, double tau, double *lo, double *hi);

/* a4 shading */
/* Surfel G-buffer (Sec. 4.4): divides the accumulated normal, albedo,
 * roughness and metalness by the accumulated weight (pixels with weight > 0),
 * in place; the shading step then proceeds as for any G-buffer. */
void orc_normalize_gbuffer(const double *weight, int W, int H, double *normal, double *albedo,
                           double *rough, double *metal);

void orc_shade(const double *depth, const double *normal, const double *albedo,
               const double *rough, const double *metal, const orc_camera *cam,
               const double *ao_lo, const double *ao_hi, const orc_light *lights, int n_lights,
               const double *irradiance, int irr_size, const double *pref_lo, const double *pref_hi,
               int pref_base, int pref_levels, const double *lut, int lut_size, const double *env,
               int env_size, const orc_tie *tie, double *hdr_lo, double *hdr_hi);

/* ---- the G-buffer and shadow-map pass on sphere fields (stand-in for the
 * rasterised geometry pass, Sec. 4, and the depth renders of Sec. 5.1) ---- */
typedef struct {
    int32_t n;
    const double *center;  /* [n][3] */
    const double *radius;  /* [n] */
    const double *albedo;  /* [n][3] */
    const double *rough;   /* [n] */
    const double *metal;   /* [n] */
    int32_t plane;         /* 1: the plane y = 0 (normal +y) behind every sphere */
    double plane_albedo[3], plane_rough, plane_metal;
} orc_scene;

/* Nearest-hit ray cast of every pixel of cam.  Pixel (x, y) casts o + t d with
 * o the camera position and d = R^T ((x + .5 - cx) / fx, -(y + .5 - cy) / fy, -1),
 * so t is the linear view depth.  A sphere is hit at the nearer root of
 * |o + t d - c| = r when that root is positive; the plane where d.y < 0 at
 * t = -o.y / d.y > 0.  The nearest hit wins, spheres in index order first and
 * the plane last, an equal t keeping the earlier object.
 *   depth [H][W] (+inf: no hit), id [H][W] (-1 none, n = plane);
 *   normal, albedo [3][H][W], rough, metal [H][W] (NULL: depth and id only);
 *   ambiguous [H][W] (may be NULL): 1 where the decision is within the tie
 *   margin -- two candidate hits within rel * t of each other, or a sphere
 *   whose discriminant is within rel of its terms (a grazing ray). */
void orc_raycast(const orc_scene *s, const orc_camera *cam, double rel, double *depth, int32_t *id,
                 double *normal, double *albedo, double *rough, double *metal, uint8_t *ambiguous);

/* Eye-dome lighting (Sec. 4.3) of a depth map with per-pixel colour: shade =
 * 2^(-strength * mean over n_dirs neighbours at radius pixels of
 * max(0, log2 d_p - log2 d_q)), depths capped at far_depth (background too);
 * foreground = shade * AO * colour, background = shade * environment.
 * ao_lo / ao_hi and env may be NULL.  n_dirs <= 64. */
void orc_edl_offsets(int radius, int n_dirs, int *dx, int *dy);
void orc_edl(const double *depth, const double *color, const orc_camera *cam, const double *ao_lo,
             const double *ao_hi, int radius, int n_dirs, double strength, double far_depth,
             const double *env, int env_size, double tie_rel, double *hdr_lo, double *hdr_hi);

/* a5 / a6 bloom, composite, tonemap.  pyramid (optional) receives the blurred
 * levels 1..levels-1 as planar [3][H_l][W_l] blocks one after another. */
void orc_bloom_tonemap(const double *hdr, int W, int H, int levels, double threshold,
                       double strength, double exposure, double gamma, int tonemap, uint8_t *ldr,
                       double *composite, double *pyramid);

/* Threads used by the OpenMP loops of the oracle. */
void orc_set_threads(int n);

#endif
