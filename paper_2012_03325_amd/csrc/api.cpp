// C ABI of the shading pass: argument validation (before anything is
// enqueued), scratch sizing, camera/light parameter set-up, and dispatch to
// the kernels.  Declarations and the full contract are in include/epb.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstring>

#include "../../include/epb.h"
#include "launch.hpp"

namespace {

thread_local int g_last_hip_error = 0;

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }
bool finite(float v) { return std::isfinite(v); }
bool valid_dtype(int d) { return d == EPB_F32 || d == EPB_F16; }
bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int hip_status(hipError_t e) {
    if (e == hipSuccess) return EPB_OK;
    g_last_hip_error = (int)e;
    return EPB_ERR_HIP;
}

// Camera checks: positive finite intrinsics, finite transform, sizes in range.
int check_camera(const epb_camera *c) {
    if (c->width < 1 || c->height < 1 || c->width > EPB_MAX_IMAGE_SIZE || c->height > EPB_MAX_IMAGE_SIZE)
        return EPB_ERR_SIZE;
    for (float v : c->world_to_cam)
        if (!finite(v)) return EPB_ERR_PARAM;
    if (!(c->fx > 0) || !(c->fy > 0) || !finite(c->fx) || !finite(c->fy) || !finite(c->cx) || !finite(c->cy))
        return EPB_ERR_PARAM;
    return EPB_OK;
}

epb::HostCam host_cam(const epb_camera *c) {
    epb::HostCam h{};
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) h.R[3 * r + k] = c->world_to_cam[4 * r + k];
        h.t[r] = c->world_to_cam[4 * r + 3];
    }
    h.fx = c->fx; h.fy = c->fy; h.cx = c->cx; h.cy = c->cy;
    h.inv_fx = (float)(1.0 / (double)c->fx);
    h.inv_fy = (float)(1.0 / (double)c->fy);
    h.w = c->width; h.h = c->height;
    return h;
}

int check_gbuffer(const epb_gbuffer *g, const epb_camera *cam) {
    if (!g->depth || !g->normal || !g->albedo || !g->roughness || !g->metalness) return EPB_ERR_NULL;
    if (g->width != cam->width || g->height != cam->height) return EPB_ERR_SIZE;
    if (!valid_dtype(g->dtype)) return EPB_ERR_DTYPE;
    if (!aligned16(g->depth) || !aligned16(g->normal) || !aligned16(g->albedo) || !aligned16(g->roughness) ||
        !aligned16(g->metalness) || (g->weight && !aligned16(g->weight)))
        return EPB_ERR_ALIGN;
    return EPB_OK;
}

// Cubes that are filtered bilinearly must have faces of at least 2x2 on every level.
int check_cube(const epb_cube *c, int min_levels, int min_face = 1) {
    if (!c->data) return EPB_ERR_NULL;
    if (c->size < 1 || c->size > 4096 || c->levels < min_levels || c->levels > 16) return EPB_ERR_SIZE;
    if ((c->size >> (c->levels - 1)) < min_face) return EPB_ERR_SIZE;
    if (!aligned16(c->data)) return EPB_ERR_ALIGN;
    return EPB_OK;
}

int check_ibl_params(int S, const epb_ibl_params *p) {
    if (p->irr_size < 2 || p->irr_size > 1024 || p->irr_src_size < 1 || p->pref_size < 2 || p->pref_levels < 1 ||
        p->pref_levels > 8 || p->lut_size < 2 || p->lut_size > 4096 || S < 2)
        return EPB_ERR_SIZE;
    if (p->pref_samples < 1 || p->pref_samples > (1 << 20) || p->lut_samples < 1 || p->lut_samples > (1 << 20))
        return EPB_ERR_PARAM;
    if (p->pref_fis != 0 && p->pref_fis != 1) return EPB_ERR_PARAM;
    if (p->pref_fis && !is_pow2(S)) return EPB_ERR_SIZE;  // the mip chain halves exactly
    int src = S < p->irr_src_size ? S : p->irr_src_size;
    if (S % src != 0 || !is_pow2(S / src)) return EPB_ERR_SIZE;
    int base = S < p->pref_size ? S : p->pref_size;
    if ((base >> (p->pref_levels - 1)) < 2) return EPB_ERR_SIZE;
    return EPB_OK;
}

// ---- per-stage validation and descriptor set-up (shared by the single-view
// calls and the batch builder) -------------------------------------------------
int build_ssao(const epb_gbuffer *gbuf, const epb_camera *cam, const epb_ssao_params *params, void *ao_out,
               void *scratch, size_t scratch_bytes, epb::SsaoDesc *out) {
    if (!gbuf || !cam || !params || !ao_out) return EPB_ERR_NULL;
    int st = check_camera(cam);
    if (st) return st;
    st = check_gbuffer(gbuf, cam);
    if (st) return st;
    if (!params->kernel || !params->noise) return EPB_ERR_NULL;
    if (params->n_samples < 1 || params->n_samples > EPB_MAX_SSAO_SAMPLES) return EPB_ERR_PARAM;
    if (!(params->radius > 0) || !finite(params->radius) || !finite(params->bias) ||
        (params->blur && (!(params->blur_tau > 0) || !finite(params->blur_tau))))
        return EPB_ERR_PARAM;
    if (!valid_dtype(params->out_dtype)) return EPB_ERR_DTYPE;
    if (!aligned16(ao_out) || !aligned16(params->kernel) || !aligned16(params->noise)) return EPB_ERR_ALIGN;
    epb::SsaoPlan plan = epb::ssao_plan(cam->width, cam->height);
    if (!scratch || scratch_bytes < plan.bytes) return EPB_ERR_SCRATCH;
    if (!aligned16(scratch)) return EPB_ERR_ALIGN;
    *out = epb::ssao_desc(plan, gbuf->depth, gbuf->normal, host_cam(cam), params->kernel, params->n_samples,
                          params->noise, params->radius, params->bias, params->blur_tau, params->blur ? 1 : 0,
                          ao_out, scratch);
    return EPB_OK;
}

int build_shade(const epb_gbuffer *gbuf, const epb_camera *cam, const void *ao, epb_dtype ao_dtype,
                const epb_light *lights, int32_t n_lights, const epb_ibl_maps *ibl, const epb_cube *env,
                void *hdr_out, epb_dtype hdr_dtype, epb::ShadeArgs *out) {
    if (!gbuf || !cam || !ibl || !env || !hdr_out) return EPB_ERR_NULL;
    if (n_lights < 0 || n_lights > EPB_MAX_LIGHTS) return EPB_ERR_PARAM;
    if (n_lights > 0 && !lights) return EPB_ERR_NULL;
    int st = check_camera(cam);
    if (st) return st;
    st = check_gbuffer(gbuf, cam);
    if (st) return st;
    if (!valid_dtype(ao_dtype) || !valid_dtype(hdr_dtype)) return EPB_ERR_DTYPE;
    if ((ao && !aligned16(ao)) || !aligned16(hdr_out)) return EPB_ERR_ALIGN;
    if ((st = check_cube(&ibl->irradiance, 1, 2)) || (st = check_cube(&ibl->prefiltered, 1, 2)) ||
        (st = check_cube(env, 1, 2)))
        return st;
    if (ibl->prefiltered.levels > 8) return EPB_ERR_SIZE;
    if (!ibl->brdf_lut) return EPB_ERR_NULL;
    if (ibl->lut_size < 2 || ibl->lut_size > 4096) return EPB_ERR_SIZE;
    if (!aligned16(ibl->brdf_lut)) return EPB_ERR_ALIGN;
    epb::ShadeArgs a{};
    a.depth = gbuf->depth;
    a.normal = gbuf->normal; a.albedo = gbuf->albedo; a.rough = gbuf->roughness; a.metal = gbuf->metalness;
    a.weight = gbuf->weight;
    a.gdtype = gbuf->dtype;
    a.W = cam->width; a.H = cam->height;
    a.cam = host_cam(cam);
    // camera position -R^T t (double on the host, once per call)
    double cp[3];
    for (int c = 0; c < 3; ++c) {
        cp[c] = 0;
        for (int r = 0; r < 3; ++r) cp[c] -= (double)cam->world_to_cam[4 * r + c] * cam->world_to_cam[4 * r + 3];
        a.cam_pos[c] = (float)cp[c];
    }
    a.ao = ao;
    a.ao_dtype = ao_dtype;
    a.n_lights = n_lights;
    for (int i = 0; i < n_lights; ++i) {
        const epb_light &L = lights[i];
        epb::DevLight &h = a.lights[i];
        for (int c = 0; c < 3; ++c) {
            if (!finite(L.pos[c]) || !finite(L.color[c]) || L.color[c] < 0) return EPB_ERR_PARAM;
            h.pos[c] = L.pos[c];
            h.rad[c] = L.color[c] * L.intensity;
        }
        if (!finite(L.intensity) || L.intensity < 0) return EPB_ERR_PARAM;
        h.map = L.shadow_map;
        if (L.shadow_map) {
            if (!aligned16(L.shadow_map)) return EPB_ERR_ALIGN;
            if ((st = check_camera(&L.shadow_cam))) return st;
            if (L.shadow_cam.width < 3 || L.shadow_cam.height < 3) return EPB_ERR_SIZE;
            if (!finite(L.shadow_bias)) return EPB_ERR_PARAM;
            // light view from camera view: P_l = R_l (R^T (P_v - t) ) + t_l = M P_v + o, the
            // rows of x and y scaled by fx and -fy so that they give (u - cx) d_l and (v - cy) d_l
            const float *A = L.shadow_cam.world_to_cam, *B = cam->world_to_cam;
            const double row_scale[3] = {(double)L.shadow_cam.fx, -(double)L.shadow_cam.fy, 1.0};
            for (int r = 0; r < 3; ++r) {
                for (int c = 0; c < 3; ++c) {
                    double s = 0;
                    for (int k = 0; k < 3; ++k) s += (double)A[4 * r + k] * B[4 * c + k];
                    h.M[3 * r + c] = (float)(row_scale[r] * s);
                }
                double o = A[4 * r + 3];
                for (int k = 0; k < 3; ++k) o += (double)A[4 * r + k] * cp[k];
                h.o[r] = (float)(row_scale[r] * o);
            }
            h.cx = L.shadow_cam.cx; h.cy = L.shadow_cam.cy;
            h.w = L.shadow_cam.width; h.h = L.shadow_cam.height;
            h.fw = (float)h.w; h.fh = (float)h.h;
            h.bias = L.shadow_bias;
            if (L.shadow_layout != EPB_MAP_ROWS && L.shadow_layout != EPB_MAP_TILES) return EPB_ERR_PARAM;
            h.tiles = L.shadow_layout == EPB_MAP_TILES;
            epb::ShadowTilesPlan tp = epb::shadow_tiles_plan(h.w, h.h);
            h.tile_pitch = h.tiles ? tp.pitch : 0u;
            h.sentinel = h.tiles ? tp.sentinel : 0u;
        }
    }
    a.irr = ibl->irradiance.data; a.irr_size = ibl->irradiance.size;
    a.pref = ibl->prefiltered.data; a.pref_base = ibl->prefiltered.size; a.pref_levels = ibl->prefiltered.levels;
    a.lut = ibl->brdf_lut; a.lut_size = ibl->lut_size;
    a.env = env->data; a.env_size = env->size;
    a.hdr = hdr_out;
    a.hdr_dtype = hdr_dtype;
    *out = a;
    return EPB_OK;
}

int check_post_params(const epb_post_params *params) {
    if (params->bloom_levels < 1 || params->bloom_levels > EPB_MAX_BLOOM_LEVELS) return EPB_ERR_PARAM;
    if (!finite(params->threshold) || !finite(params->strength) || !(params->exposure > 0) ||
        !finite(params->exposure) || !(params->gamma > 0) || !finite(params->gamma))
        return EPB_ERR_PARAM;
    if (params->tonemap != EPB_TONEMAP_ACES && params->tonemap != EPB_TONEMAP_REINHARD) return EPB_ERR_PARAM;
    if (!valid_dtype(params->pyr_dtype)) return EPB_ERR_DTYPE;
    return EPB_OK;
}

int build_post(const void *hdr, epb_dtype hdr_dtype, int32_t width, int32_t height, const epb_post_params *params,
               uint8_t *ldr_out, void *scratch, size_t scratch_bytes, epb::PostDesc *out) {
    if (!hdr || !params || !ldr_out) return EPB_ERR_NULL;
    if (width < 1 || height < 1 || width > EPB_MAX_IMAGE_SIZE || height > EPB_MAX_IMAGE_SIZE) return EPB_ERR_SIZE;
    if (!valid_dtype(hdr_dtype)) return EPB_ERR_DTYPE;
    int st = check_post_params(params);
    if (st) return st;
    if (!aligned16(hdr) || !aligned16(ldr_out)) return EPB_ERR_ALIGN;
    epb::PostPlan plan = epb::post_plan(width, height, params->bloom_levels, params->pyr_dtype);
    if (!scratch || scratch_bytes < plan.bytes) return EPB_ERR_SCRATCH;
    if (!aligned16(scratch)) return EPB_ERR_ALIGN;
    *out = epb::post_desc(plan, hdr, params->threshold, params->strength, params->exposure, params->gamma,
                          params->tonemap, ldr_out, scratch);
    return EPB_OK;
}

// ---- batched form ------------------------------------------------------------
size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Scratch of one view of a batch: [SSAO][bloom pyramid][AO if not given][HDR if not given].
struct ViewScratch {
    size_t ssao, post, ao, hdr, total;
};

int view_scratch(const epb_view &v, ViewScratch *out) {
    if (!v.ssao || !v.post) return EPB_ERR_NULL;
    int W = v.cam.width, H = v.cam.height;
    if (W < 1 || H < 1 || W > EPB_MAX_IMAGE_SIZE || H > EPB_MAX_IMAGE_SIZE) return EPB_ERR_SIZE;
    if (!valid_dtype(v.ssao->out_dtype) || !valid_dtype(v.hdr_dtype)) return EPB_ERR_DTYPE;
    int st = check_post_params(v.post);
    if (st) return st;
    ViewScratch s{};
    s.ssao = align256(epb::ssao_plan(W, H).bytes);
    s.post = align256(epb::post_plan(W, H, v.post->bloom_levels, v.post->pyr_dtype).bytes);
    size_t ao_elt = v.ssao->out_dtype == EPB_F16 ? 2 : 4, hdr_elt = v.hdr_dtype == EPB_F16 ? 2 : 4;
    s.ao = v.ao ? 0 : align256((size_t)((W + 1) / 2) * ((H + 1) / 2) * ao_elt);
    s.hdr = v.hdr ? 0 : align256((size_t)3 * W * H * hdr_elt);
    s.total = s.ssao + s.post + s.ao + s.hdr;
    *out = s;
    return EPB_OK;
}

int batch_scratch(const epb_view *views, int32_t n, size_t *bytes) {
    if (!views) return EPB_ERR_NULL;
    if (n < 1 || n > EPB_MAX_BATCH_VIEWS) return EPB_ERR_SIZE;
    size_t total = 0;
    for (int i = 0; i < n; ++i) {
        ViewScratch s;
        int st = view_scratch(views[i], &s);
        if (st) return st;
        if (!views[i].scratch) total += s.total;
    }
    *bytes = total;
    return EPB_OK;
}

int check_schedule(const epb_schedule &q) {
    if (q.shade_tile < 0 || q.shade_tile > 2 || q.ssao_tile < 0 || q.ssao_tile > 2 || q.ssao_batch < 0 ||
        q.ssao_batch > 1 || q.blocks_per_cu < 0 || q.blocks_per_cu > 64 || q.persistent < 0 ||
        q.persistent > EPB_MAX_PERSISTENT_CHUNK || q.wait_limit < -(1 << 30) || q.fuse_bloom < 0 ||
        q.fuse_bloom > 1)
        return EPB_ERR_PARAM;
    // the fused bloom epilogue needs the 32 x 8 shading tile of the stage launches
    if (q.fuse_bloom && (q.shade_tile != 0 || q.persistent)) return EPB_ERR_PARAM;
    return EPB_OK;
}

// Work items of one view's stages in the persistent launch (256-thread tiles).
void persistent_items(const epb::ViewDesc &d, int items[epb::kStages]) {
    using namespace epb;
    int st = kPersistSsaoT;
    items[kStPrep] = ssao_items(d.ssao, kStPrep, 0);
    items[kStRaw] = ceil_div(d.ssao.Wh, st) * ceil_div(d.ssao.Hh, st);
    items[kStBlur] = d.ssao.blur ? items[kStRaw] : 0;
    items[kStShade] = shade_items(d.shade, 0);
    items[kStDown] = post_items(d.post, kStDown);
    items[kStBloomBlur] = post_items(d.post, kStBloomBlur);
    items[kStComposite] = ceil_div(post_items(d.post, kStComposite), kPersistCompositeTiles);
}

}  // namespace

extern "C" {

const char *epb_status_str(int status) {
    switch (status) {
    case EPB_OK: return "ok";
    case EPB_ERR_NULL: return "a required pointer is NULL";
    case EPB_ERR_SIZE: return "size out of range";
    case EPB_ERR_DTYPE: return "unsupported storage type";
    case EPB_ERR_ALIGN: return "device pointer not 16-byte aligned";
    case EPB_ERR_SCRATCH: return "scratch buffer missing or too small";
    case EPB_ERR_PARAM: return "parameter out of range";
    case EPB_ERR_HIP: return "HIP launch failed";
    case EPB_ERR_TIMEOUT: return "a dependency wait of the persistent launch gave up";
    default: return "unknown status";
    }
}

int epb_last_hip_error(void) { return g_last_hip_error; }

// Neighbour offsets of eye-dome lighting: the direction 2 pi k / n rounded to the
// nearest pixel at the radius, halves away from zero (1e-9 slack at halves).
static int edl_round(double v) {
    double m = std::floor(std::fabs(v) + 0.5 + 1e-9);
    return (int)(v < 0 ? -m : m);
}

int epb_edl(const float *depth, const void *color, epb_dtype color_dtype, const epb_camera *cam,
            const void *ao, epb_dtype ao_dtype, const epb_edl_params *params, const epb_cube *env,
            void *hdr_out, epb_dtype hdr_dtype, hipStream_t stream) {
    if (!depth || !color || !cam || !params || !hdr_out) return EPB_ERR_NULL;
    int st = check_camera(cam);
    if (st) return st;
    if (!valid_dtype(color_dtype) || !valid_dtype(ao_dtype) || !valid_dtype(hdr_dtype)) return EPB_ERR_DTYPE;
    if (params->radius < 1 || params->radius > EPB_MAX_EDL_RADIUS || params->n_dirs < 1 ||
        params->n_dirs > EPB_MAX_EDL_DIRS)
        return EPB_ERR_PARAM;
    if (!finite(params->strength) || params->strength < 0 || !finite(params->far_depth) || !(params->far_depth > 0))
        return EPB_ERR_PARAM;
    if (env && (st = check_cube(env, 1, 2))) return st;
    if (!aligned16(depth) || !aligned16(color) || (ao && !aligned16(ao)) || !aligned16(hdr_out))
        return EPB_ERR_ALIGN;
    epb::HostCam hc = host_cam(cam);
    epb::EdlDesc c{};
    c.depth = depth; c.color = color; c.ao = ao; c.hdr = hdr_out;
    c.env = env ? (const float4 *)env->data : nullptr;
    for (int i = 0; i < 9; ++i) c.R[i] = hc.R[i];
    c.cx = hc.cx; c.cy = hc.cy; c.inv_fx = hc.inv_fx; c.inv_fy = hc.inv_fy;
    c.W = cam->width; c.H = cam->height; c.Wh = (c.W + 1) / 2; c.Hh = (c.H + 1) / 2;
    c.env_size = env ? env->size : 0;
    c.env_dims = epb::face_dims(c.env_size);
    c.radius = params->radius;
    c.n_dirs = params->n_dirs;
    c.neg_strength_over_n = (float)(-(double)params->strength / params->n_dirs);
    c.far_depth = params->far_depth;
    const double two_pi = 6.283185307179586476925286766559;
    int pitch = 32 + 2 * params->radius;  // LDS tile pitch of the kernel (32-pixel rows + halo)
    for (int k = 0; k < params->n_dirs; ++k) {
        double a = two_pi * k / params->n_dirs;
        int dx = edl_round(params->radius * std::cos(a)), dy = edl_round(params->radius * std::sin(a));
        if (dx < -params->radius || dx > params->radius || dy < -params->radius || dy > params->radius)
            return EPB_ERR_PARAM;  // cannot happen: |round(r cos a)| <= r
        c.loff[k] = dy * pitch + dx;
    }
    return hip_status(epb::launch_edl(c, color_dtype, ao_dtype, hdr_dtype, stream));
}

size_t epb_shadow_tiles_bytes(int32_t width, int32_t height) {
    if (width < 3 || height < 3 || width > EPB_MAX_IMAGE_SIZE || height > EPB_MAX_IMAGE_SIZE) return 0;
    return epb::shadow_tiles_plan(width, height).bytes;
}

int epb_shadow_tiles(const float *map, int32_t width, int32_t height, float *tiles, size_t tiles_bytes,
                     hipStream_t stream) {
    if (!map || !tiles) return EPB_ERR_NULL;
    size_t need = epb_shadow_tiles_bytes(width, height);
    if (!need || tiles_bytes < need) return EPB_ERR_SIZE;
    if (!aligned16(map) || !aligned16(tiles)) return EPB_ERR_ALIGN;
    uintptr_t m0 = (uintptr_t)map, m1 = m0 + (size_t)width * (size_t)height * 4u;
    uintptr_t t0 = (uintptr_t)tiles, t1 = t0 + need;
    if (m0 < t1 && t0 < m1) return EPB_ERR_PARAM;
    return hip_status(epb::launch_shadow_tiles(map, width, height, tiles, stream));
}

size_t epb_scratch_bytes(int32_t op, int32_t width, int32_t height, const void *params) {
    if (width < 1 || height < 1 || width > EPB_MAX_IMAGE_SIZE || height > EPB_MAX_IMAGE_SIZE) return 0;
    switch (op) {
    case EPB_OP_PRECOMPUTE_IBL: {
        if (!params || width != height) return 0;
        const epb_ibl_params *p = (const epb_ibl_params *)params;
        if (check_ibl_params(width, p) != EPB_OK) return 0;
        return epb::ibl_plan(width, *p).bytes;
    }
    case EPB_OP_SSAO:
        return epb::ssao_plan(width, height).bytes;
    case EPB_OP_RAYCAST: {
        if (!params) return 0;
        const epb_sphere_scene *sc = (const epb_sphere_scene *)params;
        if (sc->n < 0 || sc->n > EPB_MAX_SPHERES) return 0;
        return align256((size_t)16 * (sc->n > 0 ? sc->n : 1));
    }
    case EPB_OP_BLOOM_TONEMAP: {
        if (!params) return 0;
        const epb_post_params *p = (const epb_post_params *)params;
        if (check_post_params(p) != EPB_OK) return 0;
        return epb::post_plan(width, height, p->bloom_levels, p->pyr_dtype).bytes;
    }
    default:
        return 0;
    }
}

int epb_precompute_ibl(const epb_cube *env, const epb_ibl_params *params, epb_ibl_maps *out, void *scratch,
                       size_t scratch_bytes, hipStream_t stream) {
    if (!env || !params || !out) return EPB_ERR_NULL;
    int st = check_cube(env, 1);
    if (st) return st;
    st = check_ibl_params(env->size, params);
    if (st) return st;
    if (!out->irradiance.data || !out->prefiltered.data || !out->brdf_lut) return EPB_ERR_NULL;
    int base = env->size < params->pref_size ? env->size : params->pref_size;
    if (out->irradiance.size != params->irr_size || out->irradiance.levels < 1 || out->prefiltered.size != base ||
        out->prefiltered.levels != params->pref_levels || out->lut_size != params->lut_size)
        return EPB_ERR_SIZE;
    if (!aligned16(out->irradiance.data) || !aligned16(out->prefiltered.data) || !aligned16(out->brdf_lut))
        return EPB_ERR_ALIGN;
    epb::IblPlan plan = epb::ibl_plan(env->size, *params);
    if (!scratch || scratch_bytes < plan.bytes) return EPB_ERR_SCRATCH;
    if (!aligned16(scratch)) return EPB_ERR_ALIGN;
    return hip_status(epb::launch_precompute_ibl(plan, env->data, out->irradiance.data, out->prefiltered.data,
                                                 out->brdf_lut, scratch, stream));
}

int epb_ssao(const epb_gbuffer *gbuf, const epb_camera *cam, const epb_ssao_params *params, void *ao_out,
             void *scratch, size_t scratch_bytes, hipStream_t stream) {
    epb::SsaoDesc d;
    int st = build_ssao(gbuf, cam, params, ao_out, scratch, scratch_bytes, &d);
    if (st) return st;
    return hip_status(epb::launch_ssao(d, gbuf->dtype, params->out_dtype, stream));
}

int epb_ssao_static(const epb_gbuffer *gbuf, const epb_camera *cam, const epb_ssao_params *params,
                    void *ao_out, hipStream_t stream) {
    if (!gbuf || !cam || !params || !ao_out) return EPB_ERR_NULL;
    int st = check_camera(cam);
    if (st) return st;
    if (epb::ssao_plan(cam->width, cam->height).bytes > (size_t)EPB_SSAO_STATIC_SCRATCH_BYTES) return EPB_ERR_SIZE;
    void *scratch = nullptr;
    st = hip_status(epb::ssao_static_scratch(&scratch));
    if (st) return st;
    epb::SsaoDesc d;
    st = build_ssao(gbuf, cam, params, ao_out, scratch, EPB_SSAO_STATIC_SCRATCH_BYTES, &d);
    if (st) return st;
    return hip_status(epb::launch_ssao(d, gbuf->dtype, params->out_dtype, stream));
}

int epb_shade(const epb_gbuffer *gbuf, const epb_camera *cam, const void *ao, epb_dtype ao_dtype,
              const epb_light *lights, int32_t n_lights, const epb_ibl_maps *ibl, const epb_cube *env,
              void *hdr_out, epb_dtype hdr_dtype, hipStream_t stream) {
    epb::ShadeArgs a;
    int st = build_shade(gbuf, cam, ao, ao_dtype, lights, n_lights, ibl, env, hdr_out, hdr_dtype, &a);
    if (st) return st;
    return hip_status(epb::launch_shade(a, stream));
}

int epb_bloom_tonemap(const void *hdr, epb_dtype hdr_dtype, int32_t width, int32_t height,
                      const epb_post_params *params, uint8_t *ldr_out, void *scratch, size_t scratch_bytes,
                      hipStream_t stream) {
    epb::PostDesc d;
    int st = build_post(hdr, hdr_dtype, width, height, params, ldr_out, scratch, scratch_bytes, &d);
    if (st) return st;
    return hip_status(epb::launch_bloom_tonemap(d, hdr_dtype, params->pyr_dtype, stream));
}

int epb_shade_post(const epb_gbuffer *gbuf, const epb_camera *cam, const void *ao, epb_dtype ao_dtype,
                   const epb_light *lights, int32_t n_lights, const epb_ibl_maps *ibl, const epb_cube *env,
                   void *hdr_out, epb_dtype hdr_dtype, const epb_post_params *params, uint8_t *ldr_out,
                   void *scratch, size_t scratch_bytes, hipStream_t stream) {
    epb::ShadeArgs a;
    int st = build_shade(gbuf, cam, ao, ao_dtype, lights, n_lights, ibl, env, hdr_out, hdr_dtype, &a);
    if (st) return st;
    epb::PostDesc d;
    if ((st = build_post(hdr_out, hdr_dtype, cam->width, cam->height, params, ldr_out, scratch, scratch_bytes, &d)))
        return st;
    hipError_t e = epb::launch_shade(a, stream, &d);
    if (e != hipSuccess) return hip_status(e);
    return hip_status(epb::launch_bloom_tonemap(d, hdr_dtype, params->pyr_dtype, stream, d.nl >= 1));
}

size_t epb_batch_table_bytes(int32_t n_views) {
    if (n_views < 1 || n_views > EPB_MAX_BATCH_VIEWS) return 0;
    return epb::batch_table_bytes(n_views);
}

size_t epb_view_scratch_bytes(const epb_view *view) {
    ViewScratch s;
    if (!view || view_scratch(*view, &s) != EPB_OK) return 0;
    return s.total;
}

size_t epb_batch_scratch_bytes(const epb_view *views, int32_t n_views) {
    size_t bytes = 0;
    return batch_scratch(views, n_views, &bytes) == EPB_OK ? bytes : 0;
}

int epb_raycast(const epb_sphere_scene *scene, const epb_camera *cam, const epb_gbuffer *out, void *scratch,
                size_t scratch_bytes, hipStream_t stream) {
    if (!scene || !cam || !out || !out->depth) return EPB_ERR_NULL;
    int st = check_camera(cam);
    if (st) return st;
    if (out->width != cam->width || out->height != cam->height) return EPB_ERR_SIZE;
    if (scene->n < 0 || scene->n > EPB_MAX_SPHERES) return EPB_ERR_SIZE;
    if (scene->n > 0 && (!scene->center || !scene->radius || !scene->albedo || !scene->rough || !scene->metal))
        return EPB_ERR_NULL;
    if (scene->n > 0 && (!aligned16(scene->center) || !aligned16(scene->radius) || !aligned16(scene->albedo) ||
                         !aligned16(scene->rough) || !aligned16(scene->metal)))
        return EPB_ERR_ALIGN;
    for (float v : scene->plane_albedo)
        if (!finite(v)) return EPB_ERR_PARAM;
    if (!finite(scene->plane_rough) || !finite(scene->plane_metal)) return EPB_ERR_PARAM;
    if (out->weight) return EPB_ERR_PARAM;
    bool attrs = out->normal != nullptr;
    if (attrs && (!out->albedo || !out->roughness || !out->metalness)) return EPB_ERR_NULL;
    if (attrs && !valid_dtype(out->dtype)) return EPB_ERR_DTYPE;
    if (!aligned16(out->depth) ||
        (attrs && (!aligned16(out->normal) || !aligned16(out->albedo) || !aligned16(out->roughness) ||
                   !aligned16(out->metalness))))
        return EPB_ERR_ALIGN;
    size_t need = align256((size_t)16 * (scene->n > 0 ? scene->n : 1));
    if (!scratch || scratch_bytes < need) return EPB_ERR_SCRATCH;
    if (!aligned16(scratch)) return EPB_ERR_ALIGN;
    epb::RayScene s{};
    s.n = scene->n;
    s.center = scene->center; s.radius = scene->radius;
    s.albedo = scene->albedo; s.rough = scene->rough; s.metal = scene->metal;
    s.plane = scene->plane ? 1 : 0;
    for (int k = 0; k < 3; ++k) s.plane_albedo[k] = scene->plane_albedo[k];
    s.plane_rough = scene->plane_rough; s.plane_metal = scene->plane_metal;
    epb::RayCam c{};
    for (int k = 0; k < 12; ++k) c.M[k] = cam->world_to_cam[k];
    c.fx = cam->fx; c.fy = cam->fy; c.cx = cam->cx; c.cy = cam->cy;
    c.W = cam->width; c.H = cam->height;
    epb::RayOut o{};
    o.depth = (float *)out->depth;
    if (attrs) {
        o.normal = (void *)out->normal; o.albedo = (void *)out->albedo;
        o.rough = (void *)out->roughness; o.metal = (void *)out->metalness;
    }
    return hip_status(epb::launch_raycast(s, c, o, attrs ? out->dtype : EPB_F32, scratch, stream));
}

int epb_batch_build(const epb_view *views, int32_t n_views, const epb_schedule *schedule, void *scratch,
                    size_t scratch_bytes, void *table, size_t table_bytes) {
    if (!views || !table) return EPB_ERR_NULL;
    if (n_views < 1 || n_views > EPB_MAX_BATCH_VIEWS) return EPB_ERR_SIZE;
    epb_schedule q{};
    if (schedule) q = *schedule;
    int st = check_schedule(q);
    if (st) return st;
    if (table_bytes < epb::batch_table_bytes(n_views)) return EPB_ERR_SIZE;
    size_t need = 0;
    if ((st = batch_scratch(views, n_views, &need))) return st;
    if (need > 0 && (!scratch || scratch_bytes < need)) return EPB_ERR_SCRATCH;
    if (need > 0 && !aligned16(scratch)) return EPB_ERR_ALIGN;
    const epb_view &v0 = views[0];
    for (int i = 0; i < n_views; ++i) {
        const epb_view &v = views[i];
        if (v.gbuf.dtype != v0.gbuf.dtype || v.ssao->out_dtype != v0.ssao->out_dtype ||
            v.hdr_dtype != v0.hdr_dtype || v.post->pyr_dtype != v0.post->pyr_dtype)
            return EPB_ERR_DTYPE;
        if ((v.ssao->blur != 0) != (v0.ssao->blur != 0)) return EPB_ERR_PARAM;
    }
    // the persistent launch is built for one storage type throughout
    if (q.persistent && (v0.ssao->out_dtype != v0.gbuf.dtype || v0.hdr_dtype != v0.gbuf.dtype ||
                         v0.post->pyr_dtype != v0.gbuf.dtype))
        return EPB_ERR_DTYPE;
    // descriptors first (validating every view), then the header and item prefix sums
    epb::ViewDesc *vd = (epb::ViewDesc *)((char *)table + epb::batch_views_offset(n_views));
    char *sc = (char *)scratch;
    long long total[epb::kStages] = {}, chunks[epb::kStages] = {};
    int *start = (int *)((char *)table + epb::batch_start_offset());
    int *cstart = (int *)((char *)table + epb::batch_cstart_offset(n_views));
    for (int i = 0; i < n_views; ++i) {
        const epb_view &v = views[i];
        ViewScratch vs;
        view_scratch(v, &vs);
        if (v.scratch && !aligned16(v.scratch)) return EPB_ERR_ALIGN;
        char *base = v.scratch ? (char *)v.scratch : sc;
        if (!v.scratch) sc += vs.total;
        char *s_ssao = base, *s_post = base + vs.ssao;
        void *ao = v.ao ? v.ao : (void *)(s_post + vs.post);
        void *hdr = v.hdr ? v.hdr : (void *)(s_post + vs.post + vs.ao);
        epb::ViewDesc d;
        std::memset(&d, 0, sizeof(d));
        if ((st = build_ssao(&v.gbuf, &v.cam, v.ssao, ao, s_ssao, vs.ssao, &d.ssao))) return st;
        epb::ShadeArgs a;
        if ((st = build_shade(&v.gbuf, &v.cam, ao, v.ssao->out_dtype, v.lights, v.n_lights, v.ibl, v.env, hdr,
                              v.hdr_dtype, &a)))
            return st;
        d.shade = epb::shade_desc(a);
        if ((st = build_post(hdr, v.hdr_dtype, v.cam.width, v.cam.height, v.post, v.ldr, s_post, vs.post, &d.post)))
            return st;
        if (q.fuse_bloom && d.post.nl >= 1) {  // the shading stage writes bloom level 1
            d.shade.bloom1 = d.post.raw[1];
            d.shade.bloom1_half = d.post.texel_half;
            d.shade.bloom_threshold = d.post.threshold;
        }
        int items[epb::kStages];
        if (q.persistent) {
            persistent_items(d, items);
        } else {
            items[epb::kStPrep] = epb::ssao_items(d.ssao, epb::kStPrep, q.ssao_tile);
            items[epb::kStRaw] = epb::ssao_items(d.ssao, epb::kStRaw, q.ssao_tile);
            items[epb::kStBlur] = d.ssao.blur ? epb::ssao_items(d.ssao, epb::kStBlur, q.ssao_tile) : 0;
            items[epb::kStShade] = epb::shade_items(d.shade, q.shade_tile);
            items[epb::kStDown] = epb::post_items(d.post, epb::kStDown);
            items[epb::kStBloomBlur] = epb::post_items(d.post, epb::kStBloomBlur);
            items[epb::kStComposite] = epb::post_items(d.post, epb::kStComposite);
        }
        for (int k = 0; k < epb::kStages; ++k) {
            if (total[k] + items[k] > 0x7fffffffLL) return EPB_ERR_SIZE;
            start[k * (n_views + 1) + i] = (int)total[k];
            total[k] += items[k];
            long long nc = q.persistent ? (items[k] + q.persistent - 1) / q.persistent : 0;
            cstart[k * (n_views + 1) + i] = (int)chunks[k];
            chunks[k] += nc;
        }
        std::memcpy(&vd[i], &d, sizeof(d));
    }
    epb::BatchHeader h{};
    h.magic = epb::kBatchMagic;
    h.n_views = n_views;
    h.gdtype = v0.gbuf.dtype;
    h.ao_dtype = v0.ssao->out_dtype;
    h.hdr_dtype = v0.hdr_dtype;
    h.pyr_dtype = v0.post->pyr_dtype;
    h.blur = v0.ssao->blur ? 1 : 0;
    h.has_ao = 1;
    h.shade_tile = q.shade_tile;
    h.ssao_tile = q.ssao_tile;
    h.ssao_batch = q.ssao_batch;
    h.blocks_per_cu = q.blocks_per_cu;
    h.fuse_bloom = q.fuse_bloom;
    for (int k = 0; k < epb::kStages; ++k) {
        h.total[k] = (int)total[k];
        start[k * (n_views + 1) + n_views] = (int)total[k];
        cstart[k * (n_views + 1) + n_views] = (int)chunks[k];
    }
    h.persistent = q.persistent ? 1 : 0;
    h.chunk = q.persistent;
    h.gate = q.wait_limit < 0 ? 0 : 1;
    h.wait_limit = q.wait_limit < 0 ? -q.wait_limit : (q.wait_limit > 0 ? q.wait_limit : (1 << 22));
    long long first = 0;
    for (int k = 0; k < epb::kStages; ++k) {
        h.chunk_first[k] = (int)first;
        first += chunks[k];
        if (first > 0x7fffffffLL) return EPB_ERR_SIZE;
    }
    h.chunk_first[epb::kStages] = (int)first;
    h.total_chunks = (int)first;
    std::memset((char *)table + epb::batch_state_offset(n_views), 0,
                epb::batch_table_bytes(n_views) - epb::batch_state_offset(n_views));
    std::memset(table, 0, epb::batch_start_offset());
    std::memcpy(table, &h, sizeof(h));
    return EPB_OK;
}

int epb_render_batch(const void *table, const void *table_dev, hipStream_t stream) {
    if (!table || !table_dev) return EPB_ERR_NULL;
    if (!aligned16(table_dev)) return EPB_ERR_ALIGN;
    epb::BatchHeader h;
    std::memcpy(&h, table, sizeof(h));
    if (h.magic != epb::kBatchMagic || h.n_views < 1 || h.n_views > EPB_MAX_BATCH_VIEWS) return EPB_ERR_PARAM;
    if (h.persistent) return hip_status(epb::launch_persistent(h, table_dev, stream));
    hipError_t e = epb::launch_ssao_batch(h, table_dev, stream);
    if (e == hipSuccess) e = epb::launch_shade_batch(h, table_dev, stream);
    if (e == hipSuccess) e = epb::launch_post_batch(h, table_dev, stream);
    return hip_status(e);
}

int epb_batch_status(const void *table, const void *table_dev, hipStream_t stream) {
    if (!table || !table_dev) return EPB_ERR_NULL;
    if (!aligned16(table_dev)) return EPB_ERR_ALIGN;
    epb::BatchHeader h;
    std::memcpy(&h, table, sizeof(h));
    if (h.magic != epb::kBatchMagic || h.n_views < 1 || h.n_views > EPB_MAX_BATCH_VIEWS) return EPB_ERR_PARAM;
    if (!h.persistent) return EPB_OK;  // the stage launches have nothing that can give up
    int err = 0;
    const char *word = (const char *)table_dev + epb::batch_state_offset(h.n_views) + offsetof(epb::PersistState, error);
    hipError_t e = hipMemcpyAsync(&err, word, sizeof(int), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_status(e);
    return err ? EPB_ERR_TIMEOUT : EPB_OK;
}

}  // extern "C"
