/*
 * epb.h -- C ABI of an MI355X (gfx950) implementation of the deferred
 * screen-space shading pass of EasyPBR (Rosu and Behnke, "EasyPBR: A
 * Lightweight Physically-Based Renderer", GRAPP 2021).
 *
 * The paper's renderer writes a G-buffer (Sec. 4, Tab. 1), runs effect passes
 * on it (shadows, SSAO, bloom; Sec. 4.2, Sec. 5) and composes everything with
 * PBR and image-based lighting (Sec. 3, 3.1, 4.2) before tone mapping (Sec. 5.4).
 * This library implements that shading pass as four stream-ordered calls:
 *
 *   epb_precompute_ibl  -- once per environment map (Sec. 3.1)
 *   epb_ssao            -- half-resolution SSAO + bilateral blur (Sec. 5.2)
 *   epb_shade           -- position from depth, direct light with PCF shadows,
 *                          split-sum IBL with multiple scattering, AO (Sec. 3,
 *                          3.1, 4, 5.1)
 *   epb_bloom_tonemap   -- bright-map pyramid bloom, ACES, gamma, 8 bit
 *                          (Sec. 5.3, 5.4)
 *
 * epb_shade_post runs the last two as one call, forming bloom level 1 inside
 * the shading pass (bitwise the same results).
 *
 * Beside them: a batched form of the per-frame calls, a device ray caster of
 * sphere fields (the G-buffer and shadow-map pass before shading) and
 * eye-dome lighting, the compositing step of depth-only point-cloud renders
 * (Sec. 4.3).
 *
 * Conventions (the paper leaves them open; every call uses the same ones):
 *  - Images are row-major, y down.  Multi-channel images are planar [c][H][W].
 *  - Pinhole cameras: pixel centres at (x + 0.5, y + 0.5); the view-space point
 *    of pixel (x, y) at linear depth d is
 *      ((x + 0.5 - cx) / fx * d, -(y + 0.5 - cy) / fy * d, -d);
 *    world_to_cam is a row-major 3x4 rigid transform [R | t].
 *  - Depth is the linear view depth d > 0; +inf marks background (Sec. 4 keeps
 *    only depth and reconstructs positions from it).
 *  - Normals are world-space (renormalised on read), albedo is linear.
 *  - Cube maps are [level][face][S][S][4] float RGBA (A unused), faces ordered
 *    +X, -X, +Y, -Y, +Z, -Z; texel (i, j) has s = 2 (i + .5) / S - 1,
 *    t = 2 (j + .5) / S - 1 and points along +X (1,-t,-s), -X (-1,-t,s),
 *    +Y (s,1,t), -Y (s,-1,-t), +Z (s,-t,1), -Z (-s,-t,-1).  Lookups pick the
 *    major axis (ties z, then y, then x) and filter bilinearly with
 *    clamp-to-edge inside the face; every filtered level has faces of at
 *    least 2x2 texels.
 *  - Half resolution is Wh = ceil(W / 2), Hh = ceil(H / 2); half-resolution
 *    texel (i, j) is the full-resolution pixel (2 i, 2 j).
 *
 * Memory and ownership: every data pointer is a device pointer owned by the
 * caller and must be 16-byte aligned.  The library allocates nothing: calls
 * that need temporary device memory take a caller-provided scratch buffer of
 * at least epb_scratch_bytes() bytes.  Struct arguments are read on the host
 * during the call; device buffers are read or written by the enqueued work
 * until the stream reaches it.  Nothing is retained after the call returns.
 *
 * Errors: arguments are validated on the host before anything is enqueued; a
 * validation failure returns a negative epb_status and enqueues nothing (the
 * outputs are untouched).  A failed launch returns EPB_ERR_HIP and
 * epb_last_hip_error() gives the HIP error code of the calling thread.
 * Faults inside kernels surface at the caller's next stream synchronisation.
 * No call aborts, exits or throws.
 *
 * Concurrency: all work is enqueued on the given stream, with no device-wide
 * synchronisation.  Calls are reentrant; calls on different streams must use
 * different scratch buffers.  Results are deterministic for fixed inputs (no
 * floating-point atomics).
 */
#ifndef EPB_H
#define EPB_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EPB_OK = 0,
    EPB_ERR_NULL = -1,    /* a required pointer is NULL                      */
    EPB_ERR_SIZE = -2,    /* an image / cube / table size is out of range     */
    EPB_ERR_DTYPE = -3,   /* unsupported storage type                         */
    EPB_ERR_ALIGN = -4,   /* a device pointer is not 16-byte aligned          */
    EPB_ERR_SCRATCH = -5, /* scratch buffer missing or smaller than required  */
    EPB_ERR_PARAM = -6,   /* a scalar parameter is out of range               */
    EPB_ERR_HIP = -7,     /* a HIP launch failed; see epb_last_hip_error()    */
    EPB_ERR_TIMEOUT = -8  /* a wait of the persistent batch launch gave up    */
} epb_status;

/* Storage type of G-buffer attribute planes, AO and HDR images.  Arithmetic
 * is always float32; EPB_F16 stores IEEE half (HDR saturates at 65504). */
typedef enum { EPB_F32 = 0, EPB_F16 = 1 } epb_dtype;

#define EPB_MAX_LIGHTS 8
#define EPB_MAX_SSAO_SAMPLES 256
#define EPB_MAX_BLOOM_LEVELS 6 /* "up to six levels" (Sec. 5.3) */
#define EPB_MAX_IMAGE_SIZE 16384

/* Pinhole camera (see conventions above). */
typedef struct {
    float world_to_cam[12]; /* row-major 3x4 [R | t], R orthonormal */
    float fx, fy, cx, cy;   /* focal lengths and principal point, pixels */
    int32_t width, height;
} epb_camera;

/* G-buffer (Sec. 4, Tab. 1): depth is always float32 (the paper's R32 target);
 * the attribute planes use `dtype`.  A surfel-splatted G-buffer (Sec. 4.4)
 * holds accumulated attributes and their accumulated weight: shading first
 * divides albedo, roughness and metalness by the weight on pixels whose weight
 * is > 0 (the normal is renormalised anyway, so its division is implied); with
 * weight == NULL the attributes are used as they are. */
typedef struct {
    int32_t width, height;
    epb_dtype dtype;      /* of normal, albedo, roughness, metalness, weight */
    const float *depth;   /* [H][W] linear view depth, +inf = background    */
    const void *normal;   /* [3][H][W] world-space normal                   */
    const void *albedo;   /* [3][H][W] linear base colour in [0, 1]         */
    const void *roughness;/* [H][W] perceptual roughness in (0, 1]          */
    const void *metalness;/* [H][W] in [0, 1]                               */
    const void *weight;   /* [H][W] accumulated surfel weight, or NULL      */
} epb_gbuffer;

/* A float32 cube map with `levels` mip levels of sizes size >> m (size <= 4096). */
typedef struct {
    int32_t size;
    int32_t levels;
    float *data; /* [level][6][s][s][4]; read-only where the call only reads */
} epb_cube;

/* Image-based-lighting precompute sizes (Sec. 3.1). */
typedef struct {
    int32_t irr_size;     /* irradiance map face size (e.g. 32)                    */
    int32_t irr_src_size; /* irradiance source face size; the environment is
                             averaged down to min(env size, this) (e.g. 64)         */
    int32_t pref_size;    /* prefiltered base size cap: base = min(env, this) (128) */
    int32_t pref_levels;  /* prefiltered mip levels, roughness m / (levels-1) (5)  */
    int32_t pref_samples; /* GGX samples per prefiltered texel (1024)              */
    int32_t lut_size;     /* BRDF table size (256)                                 */
    int32_t lut_samples;  /* GGX samples per table entry (1024)                    */
    int32_t pref_fis;     /* 1: filtered importance sampling of the prefilter (each
                             sample reads the environment's mip chain at the level
                             its pdf asks for; needs a power-of-two size); 0: every
                             sample reads level 0 (the default)                    */
} epb_ibl_params;

/* Outputs of epb_precompute_ibl, inputs of epb_shade. */
typedef struct {
    epb_cube irradiance;  /* 1 level of irr_size: cosine-weighted mean radiance  */
    epb_cube prefiltered; /* pref_levels levels from base = min(env, pref_size)  */
    float *brdf_lut;      /* [lut_size][lut_size][2] = (A, B); row = roughness,
                             column = N.V, both sampled at texel centres          */
    int32_t lut_size;
} epb_ibl_maps;

/* Screen-space ambient occlusion (Sec. 5.2). */
typedef struct {
    int32_t n_samples;    /* 1 .. EPB_MAX_SSAO_SAMPLES                         */
    const float *kernel;  /* device [n][3] tangent-space hemisphere vectors   */
    const float *noise;   /* device [4][4][2] rotation vectors (view xy)      */
    float radius;         /* world units (e.g. 0.5)                           */
    float bias;           /* depth bias, world units (e.g. 0.025)             */
    float blur_tau;       /* relative depth tolerance of the blur (e.g. 0.1)  */
    int32_t blur;         /* 1: apply the 4x4 bilateral blur, 0: raw AO       */
    epb_dtype out_dtype;  /* storage of the AO image                          */
} epb_ssao_params;

/* Storage layouts of a shadow map (epb_light.shadow_layout). */
#define EPB_MAP_ROWS 0  /* [h][w] row-major                                        */
#define EPB_MAP_TILES 1 /* the tiled form written by epb_shadow_tiles (below)      */

/* Point light (Sec. 5.1) with an optional depth map rendered from the light. */
typedef struct {
    float pos[3];
    float color[3];
    float intensity;          /* radiance at distance r is color * intensity / r^2 */
    const float *shadow_map;  /* device linear depth (+inf empty) of w x h texels
                                 (w, h from shadow_cam, at least 3x3) in
                                 shadow_layout, or NULL                           */
    epb_camera shadow_cam;    /* camera the map was rendered with                 */
    float shadow_bias;        /* depth bias of the shadow test (e.g. 0.02)        */
    int32_t shadow_layout;    /* EPB_MAP_ROWS or EPB_MAP_TILES (same results; the
                                 tiled form fetches faster)                       */
} epb_light;

/*
 * Tiled form of a shadow map.  The 3x3 percentage-closer test (Sec. 5.1)
 * reads a 3x3 texel patch around each shaded point's projection; neighbouring
 * pixels project onto a rotated strip of the map, so in row-major order one
 * wavefront's patch rows fall on many different cache lines.  The tiled form
 * pads the map with a one-texel apron of +inf (empty, so lit), cuts the padded
 * map into tiles of 6x6 texels and stores each as an 8x8 block of floats that
 * repeats the next two columns and rows: the patch of any point projecting
 * inside the map then lies inside one block, its three rows 8 floats apart,
 * with no border case, and a strip of the map covers far fewer lines.  One
 * more block of +inf follows the tiles (points outside the map read it).
 *
 *   nx = ceil(w / 6) tiles across, ny = ceil(h / 6) down, tiles in row-major
 *   order; float (p nx + q) 64 + 8 j + i (0 <= i, j < 8) holds
 *   map[6 p + j - 1][6 q + i - 1], +inf where that index is outside the map;
 *   floats 64 nx ny .. 64 nx ny + 63 are +inf.
 *
 * epb_shadow_tiles_bytes(w, h) = 256 (nx ny + 1) (0 unless 3 <= w, h <=
 * EPB_MAX_IMAGE_SIZE).  epb_shadow_tiles copies the row-major [h][w] `map`
 * into `tiles` (>= epb_shadow_tiles_bytes bytes, not overlapping `map`) on
 * `stream`; a renderer calls it whenever it re-renders a map.  Statuses:
 * EPB_ERR_NULL, EPB_ERR_SIZE (sizes out of range or `tiles` too small),
 * EPB_ERR_ALIGN, EPB_ERR_PARAM (the two buffers overlap).
 */
size_t epb_shadow_tiles_bytes(int32_t width, int32_t height);
int epb_shadow_tiles(const float *map, int32_t width, int32_t height, float *tiles, size_t tiles_bytes,
                     hipStream_t stream);

/* Bloom and tone mapping (Sec. 5.3, 5.4). */
typedef struct {
    int32_t bloom_levels; /* pyramid levels including the full-resolution bright
                             map; levels 1 .. bloom_levels-1 are blurred and added
                             (1 .. EPB_MAX_BLOOM_LEVELS)                      */
    float threshold;      /* luminance above which light blooms (1.0)           */
    float strength;       /* weight of each added level (0.04)                  */
    float exposure;       /* multiplies HDR before the ACES curve (1.0)         */
    float gamma;          /* display gamma (2.2)                                */
    epb_dtype pyr_dtype;  /* storage of the bloom pyramid in scratch            */
    int32_t tonemap;      /* EPB_TONEMAP_ACES (0, the default) or
                             EPB_TONEMAP_REINHARD (1)                          */
} epb_post_params;

/* Tone-mapping operators of the final compositing step (Sec. 5.4). */
#define EPB_TONEMAP_ACES 0
#define EPB_TONEMAP_REINHARD 1

/* A field of spheres with an optional ground plane y = 0: the geometry the
 * ray caster turns into G-buffers and shadow maps (a stand-in for the paper's
 * rasterised geometry pass, Sec. 4, and its depth renders from each light,
 * Sec. 5.1).  Geometry is double precision; materials are float. */
#define EPB_MAX_SPHERES 65536
typedef struct {
    int32_t n;              /* 0 .. EPB_MAX_SPHERES                              */
    const double *center;   /* device [n][3] (finite)                            */
    const double *radius;   /* device [n] (> 0)                                  */
    const float *albedo;    /* device [n][3]                                     */
    const float *rough;     /* device [n]                                        */
    const float *metal;     /* device [n]                                        */
    int32_t plane;          /* 1: the plane y = 0 with normal +y                 */
    float plane_albedo[3], plane_rough, plane_metal;
} epb_sphere_scene;

/* Operation ids for epb_scratch_bytes. */
typedef enum {
    EPB_OP_PRECOMPUTE_IBL = 0,
    EPB_OP_SSAO = 1,
    EPB_OP_BLOOM_TONEMAP = 2,
    EPB_OP_RAYCAST = 3 /* params: epb_sphere_scene */
} epb_op;

/*
 * epb_precompute_ibl -- image-based-lighting tables of one environment
 * (Sec. 3.1: blurred cube maps for diffuse light, split-sum prefiltered
 * specular chain and BRDF table).
 *
 *   env      cube with levels >= 1 of size S; S = irr_src * 2^k for some k >= 0
 *            where irr_src = min(S, params->irr_src_size)
 *   out      irradiance (size irr_size, 1 level), prefiltered (size
 *            min(S, pref_size), pref_levels levels), brdf_lut (lut_size^2 x 2),
 *            all caller-allocated
 *   scratch  >= epb_scratch_bytes(EPB_OP_PRECOMPUTE_IBL, S, S, params)
 *
 * Irradiance: E(n) = sum L max(0, n.w) dW / sum max(0, n.w) dW over the texels
 * of the solid-angle-weighted average of env at size irr_src.  Prefiltered level
 * m: the N.L-weighted mean of env level 0 over pref_samples GGX reflection
 * samples (Hammersley) with N = V = R the texel direction and roughness
 * m / (pref_levels - 1).  With pref_fis, a sample reads instead the mip chain
 * of env (level k = solid-angle-weighted 2x2 means of level k - 1, down to 2x2
 * faces) trilinearly at lod = 1/2 log2(omega_s / omega_p) + 1, clamped to the
 * chain, where omega_s = 1 / (N pdf) is the sample's solid angle (pdf = D / 4
 * for V = N) and omega_p = 4 pi / (6 S^2) (Krivanek and Colbert's filtered
 * importance sampling).  BRDF table: the Karis scale and bias integrals
 * (k = alpha / 2) at N.V = (i + .5) / lut_size, roughness = (j + .5) / lut_size.
 * Sums are Kahan-compensated in float32.
 */
int epb_precompute_ibl(const epb_cube *env, const epb_ibl_params *params, epb_ibl_maps *out,
                       void *scratch, size_t scratch_bytes, hipStream_t stream);

/*
 * epb_ssao -- normal-oriented hemisphere ambient occlusion at half resolution,
 * bilaterally blurred (Sec. 5.2).
 *
 *   gbuf, cam  G-buffer and the camera it was rendered with (same W, H)
 *   ao_out     [Hh][Wh] of params->out_dtype
 *   scratch    >= epb_scratch_bytes(EPB_OP_SSAO, W, H, params)
 *
 * Per half-resolution texel p (background: AO = 1): view-space position P and
 * normal n; the noise vector of (i mod 4, j mod 4) Gram-Schmidt-orthogonalised
 * to n gives t and b = n x t; each kernel vector s gives Q = P + radius (t sx +
 * b sy + n sz), projected to the nearest half-resolution texel q; the sample is
 * occluded by smoothstep(0, 1, radius / |d_p - d_q|) when d_q <= -Q.z - bias.
 * AO = 1 - mean occlusion.  The blur is the mean over offsets -2..1 in x and y
 * weighted by max(0, 1 - |d_q - d_p| / (blur_tau d_p)).
 */
int epb_ssao(const epb_gbuffer *gbuf, const epb_camera *cam, const epb_ssao_params *params,
             void *ao_out, void *scratch, size_t scratch_bytes, hipStream_t stream);

/*
 * epb_ssao_static -- epb_ssao for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation and results, bit for bit, with the scratch
 * taken from an array the library holds on every GPU it runs on
 * (EPB_SSAO_STATIC_SCRATCH_BYTES, kept until the process ends).  Nothing is
 * allocated; the caller passes inputs and outputs as for epb_ssao, on the
 * current device.  Images whose SSAO scratch (epb_scratch_bytes(EPB_OP_SSAO,
 * ...), two planes of ceil(W/2) x ceil(H/2) floats) exceeds the array return
 * EPB_ERR_SIZE (3840 x 2160 fits); a failed device-address lookup returns
 * EPB_ERR_HIP.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (concurrent streams) race, so callers serialise them.
 * Nothing in the array needs to start at zero (every value is written before
 * it is read within the call).
 */
#define EPB_SSAO_STATIC_SCRATCH_BYTES (16u << 20)
int epb_ssao_static(const epb_gbuffer *gbuf, const epb_camera *cam, const epb_ssao_params *params,
                    void *ao_out, hipStream_t stream);

/*
 * epb_shade -- the compose pass (Sec. 4.2) with PBR (Sec. 3) and IBL (Sec. 3.1).
 *
 *   gbuf, cam   G-buffer and camera (same W, H)
 *   ao, ao_dtype  [Hh][Wh] ambient occlusion (e.g. from epb_ssao), or NULL for 1
 *   lights      host array of n_lights (0 .. EPB_MAX_LIGHTS) lights
 *   ibl         tables from epb_precompute_ibl
 *   env         environment cube (level 0 is shown behind the scene)
 *   hdr_out     [3][H][W] linear radiance of hdr_dtype
 *
 * Per pixel: world position from depth; Cook-Torrance with GGX, Smith-Schlick
 * (k = (r + 1)^2 / 8) and Schlick Fresnel, F0 = mix(0.04, albedo, metal),
 * Lambert diffuse albedo (1 - metal) / pi, N.V clamped to [1e-4, 1]; per light
 * the 3x3 percentage-closer shadow test of the light's depth map (taps outside
 * the map are lit).  Ambient = split-sum specular and irradiance with the
 * Fdez-Aguera multiple-scattering terms, times the bilinearly upsampled AO.
 * Background pixels show the environment along the view ray.
 */
int epb_shade(const epb_gbuffer *gbuf, const epb_camera *cam, const void *ao,
              epb_dtype ao_dtype, const epb_light *lights, int32_t n_lights,
              const epb_ibl_maps *ibl, const epb_cube *env, void *hdr_out, epb_dtype hdr_dtype,
              hipStream_t stream);

/*
 * epb_bloom_tonemap -- bloom (Sec. 5.3) and final compositing with ACES tone
 * mapping and gamma correction (Sec. 5.4).
 *
 *   hdr       [3][H][W] of hdr_dtype
 *   ldr_out   [H][W][4] uint8 RGBA (A = 255)
 *   scratch   >= epb_scratch_bytes(EPB_OP_BLOOM_TONEMAP, W, H, params); on
 *             return its first part holds the blurred levels 1 .. L-1, each
 *             [H_l][W_l][4] of params->pyr_dtype (RGB + unused), level after level
 *
 * Bright map b = c max(Y - threshold, 0) / Y (Rec. 709 luminance Y, the
 * division as a float32 reciprocal; pixels with Y below 2^-126 add nothing);
 * level 1 sums each 2x2 block as two horizontal pairs, then the rows; level l
 * of size ceil(W / 2^l) x ceil(H / 2^l) is the mean of the in-range children of
 * level l - 1; levels 1 .. L-1 are blurred with the separable [1 4 6 4 1] / 16
 * kernel (clamp to edge) and added, times strength, bilinearly upsampled; the
 * result goes through exposure, the tone curve -- the ACES fit x (2.51 x + .03) /
 * (x (2.43 x + .59) + .14), or the global Reinhard operator x / (1 + x) -- per
 * channel, clamp to [0, 1], x^(1 / gamma) and rounding to 8 bits.
 */
int epb_bloom_tonemap(const void *hdr, epb_dtype hdr_dtype, int32_t width, int32_t height,
                      const epb_post_params *params, uint8_t *ldr_out, void *scratch,
                      size_t scratch_bytes, hipStream_t stream);

/*
 * epb_shade_post -- epb_shade followed by epb_bloom_tonemap in one call, with
 * level 1 of the bloom pyramid (Sec. 5.3) formed in the shading pass: each
 * 2x2 block of shaded pixels is bright-passed and averaged from the HDR values
 * as stored while they are still in registers, so the bloom pass does not read
 * the HDR image back to build it.  Arguments are those of the two calls (the
 * bloom pass takes W, H from cam and its HDR input is hdr_out); the same
 * validation and statuses.  hdr_out, ldr_out and scratch hold bitwise what
 * epb_shade then epb_bloom_tonemap leave there.
 */
int epb_shade_post(const epb_gbuffer *gbuf, const epb_camera *cam, const void *ao, epb_dtype ao_dtype,
                   const epb_light *lights, int32_t n_lights, const epb_ibl_maps *ibl, const epb_cube *env,
                   void *hdr_out, epb_dtype hdr_dtype, const epb_post_params *params, uint8_t *ldr_out,
                   void *scratch, size_t scratch_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Batched form: the whole pass (SSAO, shading, bloom and tone mapping) of many
 * views of any sizes with one launch per stage (seven launches per batch, not
 * seven per view), or all of it in one persistent launch (epb_schedule).  Every stage walks the work items (tiles) of all views, so
 * small views do not leave the device idle and a batch is a fixed sequence of
 * launches that can be captured in a HIP graph and replayed.
 *
 * Use: fill one epb_view per view; size the scratch with
 * epb_batch_scratch_bytes() and the table with epb_batch_table_bytes();
 * epb_batch_build() validates every view and writes the batch table into host
 * memory; copy those table bytes to device memory (16-byte aligned); then
 * epb_render_batch() enqueues the frame.  The table holds the device addresses
 * of every input, output and scratch buffer and may be reused (and its device
 * copy replayed) for as long as those buffers stay where they are.
 * Each view's results are bitwise identical to the single-view calls
 * epb_ssao -> epb_shade -> epb_bloom_tonemap on the same inputs with the same
 * schedule choices (tile shapes do not change results; see epb_schedule).
 * ------------------------------------------------------------------------ */

#define EPB_MAX_BATCH_VIEWS 4096

typedef struct {
    epb_gbuffer gbuf;             /* the view's G-buffer                        */
    epb_camera cam;               /* its camera (same W, H)                     */
    const epb_light *lights;      /* host array of n_lights lights              */
    int32_t n_lights;             /* 0 .. EPB_MAX_LIGHTS                        */
    const epb_ibl_maps *ibl;      /* host struct: tables of epb_precompute_ibl  */
    const epb_cube *env;          /* host struct: environment cube              */
    const epb_ssao_params *ssao;  /* host struct                                */
    const epb_post_params *post;  /* host struct                                */
    epb_dtype hdr_dtype;          /* storage of the HDR image                   */
    void *ao;                     /* [Hh][Wh] AO output, or NULL: kept in scratch */
    void *hdr;                    /* [3][H][W] HDR output, or NULL: in scratch  */
    uint8_t *ldr;                 /* [H][W][4] RGBA8 output (required)          */
    void *scratch;                /* this view's own scratch of at least
                                     epb_view_scratch_bytes(view) bytes, or NULL:
                                     a region of the batch scratch             */
} epb_view;

/* Launch shapes of a batch.  They change the speed, never the results: every
 * output value is computed by the same arithmetic whatever the shape. */
typedef struct {
    int32_t shade_tile;    /* shading pixel tile: 0 = 32x8, 1 = 64x4, 2 = 16x16 */
    int32_t ssao_tile;     /* SSAO half-resolution tile: 0 = 16x8, 1 = 32x4,
                              2 = 16x16, its depth and a 32-texel halo staged
                              in LDS                                          */
    int32_t ssao_batch;    /* SSAO depth gathers in flight: 0 = 8, 1 = 16        */
    int32_t blocks_per_cu; /* 0: one workgroup per work item (persistent
                              launch: as many as fit); k in 1..64: a grid of k
                              workgroups per compute unit that loops over the
                              work                                             */
    int32_t persistent;    /* 0: one launch per stage (seven per batch);
                              k in 1..EPB_MAX_PERSISTENT_CHUNK: the whole batch
                              in one launch whose work items are k tiles of one
                              view and stage (requires one storage type for
                              G-buffer, AO, HDR and pyramid; else EPB_ERR_DTYPE) */
    int32_t wait_limit;    /* persistent: polls of a dependency before a
                              workgroup gives up (0: 2^22, about seconds); a
                              negative value -k makes every wait give up after k
                              polls (for testing the error path)               */
    int32_t fuse_bloom;    /* 1: the shading stage also forms bloom level 1, as
                              epb_shade_post does (stage launches with shading
                              tile 0 only; else EPB_ERR_PARAM)                  */
} epb_schedule;

#define EPB_MAX_PERSISTENT_CHUNK 4096

/* Bytes of the batch table for n_views views (0 if n_views is out of range). */
size_t epb_batch_table_bytes(int32_t n_views);

/* Bytes of device scratch one view needs: the SSAO and bloom scratch of the
 * single-view calls, plus AO and HDR images when the view leaves them NULL.
 * 0 for invalid arguments. */
size_t epb_view_scratch_bytes(const epb_view *view);

/* Bytes of batch scratch a batch of these views needs: the sum of
 * epb_view_scratch_bytes over the views that bring no scratch of their own
 * (0 when all do, or for invalid arguments). */
size_t epb_batch_scratch_bytes(const epb_view *views, int32_t n_views);

/*
 * epb_batch_build -- validate n_views views (1 .. EPB_MAX_BATCH_VIEWS) and
 * write the batch table into the host buffer `table`.
 *
 *   views     host array; each view is checked as the single-view calls check
 *             their arguments (same status codes)
 *   schedule  launch shapes, or NULL for all zeros
 *   scratch   device buffer of >= epb_batch_scratch_bytes(views, n_views);
 *             may be NULL when every view brings its own scratch
 *   table     host buffer of >= epb_batch_table_bytes(n_views)
 *
 * All views must share the G-buffer dtype, the AO dtype, the HDR dtype, the
 * bloom pyramid dtype (else EPB_ERR_DTYPE) and the SSAO blur flag (else
 * EPB_ERR_PARAM).  Enqueues nothing; returns EPB_OK or a validation status.
 */
int epb_batch_build(const epb_view *views, int32_t n_views, const epb_schedule *schedule,
                    void *scratch, size_t scratch_bytes, void *table, size_t table_bytes);

/*
 * epb_render_batch -- enqueue the batch described by `table` (host copy, as
 * written by epb_batch_build) on `stream`; `table_dev` is a device copy of
 * the same bytes that stays unchanged until the enqueued work has run.
 * Launches exactly the kernels of one frame: no copies, allocations or
 * memsets, so the call may be captured into a HIP graph.  Returns
 * EPB_ERR_PARAM for a table that epb_batch_build did not write.
 *
 * With a persistent schedule the frame is one launch (after a one-block clear
 * of the table's work counters): the device copy must then stay writable, as
 * its last bytes hold the counters (the host copy is not changed), and two
 * renders of one device table must not overlap.
 * Work items are handed out in stage order, and an item waits, bounded by the
 * schedule's wait_limit, until its view's previous stage is complete; a wait
 * that gives up stops the launch early (its outputs are then incomplete) and
 * is reported by epb_batch_status().
 */
int epb_render_batch(const void *table, const void *table_dev, hipStream_t stream);

/*
 * epb_batch_status -- after epb_render_batch of a persistent table: waits for
 * `stream` and returns EPB_ERR_TIMEOUT if a dependency wait of the last render
 * of `table_dev` gave up, else EPB_OK (also for tables of stage launches,
 * which never wait).  EPB_ERR_PARAM for a table epb_batch_build did not write;
 * EPB_ERR_HIP if the copy of the status word fails.
 */
int epb_batch_status(const void *table, const void *table_dev, hipStream_t stream);

/*
 * epb_raycast -- G-buffer (or depth map) of a sphere field seen by `cam`: the
 * pass before shading, on the device, so that a renderer can take new cameras
 * and re-render shadow maps when lights or objects move.
 *
 *   out      destination planes of cam's size; out->depth is required; with
 *            out->normal == NULL only depth is written (a shadow map), else
 *            normal, albedo, roughness and metalness too, in out->dtype;
 *            out->weight must be NULL
 *   scratch  >= epb_scratch_bytes(EPB_OP_RAYCAST, W, H, scene)
 *
 * Pixel (x, y) casts o + t d, o the camera position, d = R^T ((x + .5 - cx) /
 * fx, -(y + .5 - cy) / fy, -1), so that t is the linear view depth.  A sphere is
 * hit at the nearer root of |o + t d - c| = r when it is positive; the plane
 * where d.y < 0 at t = -o.y / d.y > 0.  The nearest hit wins (spheres in index
 * order, then the plane; an equal t keeps the earlier object); no hit gives
 * depth +inf and zero attributes.  The normal is the unit (p - c) / r (plane:
 * +y); albedo, roughness and metalness are the hit object's.  Intersections
 * are computed in double precision and stored rounded to the destination type.
 */
int epb_raycast(const epb_sphere_scene *scene, const epb_camera *cam, const epb_gbuffer *out,
                void *scratch, size_t scratch_bytes, hipStream_t stream);

/* Eye-dome lighting (Sec. 4.3) of depth-only renders such as point clouds. */
#define EPB_MAX_EDL_RADIUS 16
#define EPB_MAX_EDL_DIRS 32
typedef struct {
    int32_t radius;   /* neighbour distance in pixels, 1 .. EPB_MAX_EDL_RADIUS     */
    int32_t n_dirs;   /* neighbours on the circle, 1 .. EPB_MAX_EDL_DIRS           */
    float strength;   /* shade = 2^(-strength * response), finite and >= 0         */
    float far_depth;  /* depth given to background and depths beyond it, > 0       */
} epb_edl_params;

/*
 * epb_edl -- the compositing step for depth-only renders (Sec. 4.3): no normals,
 * so no PBR; pixels are darkened where their depth jumps behind their
 * neighbours.
 *
 *   depth        [H][W] linear view depth, +inf = background (H, W from cam)
 *   color        [3][H][W] linear colour of the points, of color_dtype
 *   cam          the camera of the render (background view directions)
 *   ao, ao_dtype [Hh][Wh] ambient occlusion (e.g. from epb_ssao), or NULL for 1
 *   env          environment cube shown behind the points (level 0), or NULL
 *                for black
 *   hdr_out      [3][H][W] of hdr_dtype
 *
 * Neighbour k of n_dirs is the pixel offset (round(radius cos a_k),
 * round(radius sin a_k)), a_k = 2 pi k / n_dirs, x right and y down, rounded
 * half away from zero (within 1e-9 of a half counts as the half).  With
 * z = log2(min(d, far_depth)) (background: log2 far_depth), the response of
 * pixel p is (1 / n_dirs) sum over the neighbours q inside the image of
 * max(0, z_p - z_q), and shade = 2^(-strength * response).  Foreground pixels
 * get shade * AO * colour (AO bilinearly upsampled as in epb_shade),
 * background pixels shade * env along the view ray, so the background next to
 * the points receives a dark outline.
 */
int epb_edl(const float *depth, const void *color, epb_dtype color_dtype, const epb_camera *cam,
            const void *ao, epb_dtype ao_dtype, const epb_edl_params *params, const epb_cube *env,
            void *hdr_out, epb_dtype hdr_dtype, hipStream_t stream);

/* Bytes of scratch the operation needs for a W x H image (for
 * EPB_OP_PRECOMPUTE_IBL pass the environment size as W and H and an
 * epb_ibl_params; for EPB_OP_SSAO an epb_ssao_params or NULL; for
 * EPB_OP_BLOOM_TONEMAP an epb_post_params; for EPB_OP_RAYCAST an
 * epb_sphere_scene).  Returns 0 for invalid arguments. */
size_t epb_scratch_bytes(int32_t op, int32_t width, int32_t height, const void *params);

/* Static description of a status code (never NULL). */
const char *epb_status_str(int status);

/* HIP error code of the last EPB_ERR_HIP returned on the calling thread. */
int epb_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EPB_H */
