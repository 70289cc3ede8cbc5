// C ABI of the shading pass: argument validation (before anything is
// enqueued), scratch sizing, camera/light parameter set-up, and dispatch to
// the kernels.  Declarations and the full contract are in include/epb.h.
#include <hip/hip_runtime.h>

#include <cmath>
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
        !aligned16(g->metalness))
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
    int src = S < p->irr_src_size ? S : p->irr_src_size;
    if (S % src != 0 || !is_pow2(S / src)) return EPB_ERR_SIZE;
    int base = S < p->pref_size ? S : p->pref_size;
    if ((base >> (p->pref_levels - 1)) < 2) return EPB_ERR_SIZE;
    return EPB_OK;
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
    default: return "unknown status";
    }
}

int epb_last_hip_error(void) { return g_last_hip_error; }

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
    case EPB_OP_BLOOM_TONEMAP: {
        if (!params) return 0;
        const epb_post_params *p = (const epb_post_params *)params;
        if (p->bloom_levels < 1 || p->bloom_levels > EPB_MAX_BLOOM_LEVELS || !valid_dtype(p->pyr_dtype)) return 0;
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
    return hip_status(epb::launch_ssao(plan, gbuf->depth, gbuf->normal, gbuf->dtype, host_cam(cam),
                                       params->kernel, params->n_samples, params->noise, params->radius,
                                       params->bias, params->blur_tau, params->blur, ao_out, params->out_dtype,
                                       scratch, stream));
}

int epb_shade(const epb_gbuffer *gbuf, const epb_camera *cam, const void *ao, epb_dtype ao_dtype,
              const epb_light *lights, int32_t n_lights, const epb_ibl_maps *ibl, const epb_cube *env,
              void *hdr_out, epb_dtype hdr_dtype, hipStream_t stream) {
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
        epb::HostLight &h = a.lights[i];
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
            // light view from camera view: P_l = R_l (R^T (P_v - t) ) + t_l = M P_v + o
            const float *A = L.shadow_cam.world_to_cam, *B = cam->world_to_cam;
            for (int r = 0; r < 3; ++r) {
                for (int c = 0; c < 3; ++c) {
                    double s = 0;
                    for (int k = 0; k < 3; ++k) s += (double)A[4 * r + k] * B[4 * c + k];
                    h.M[3 * r + c] = (float)s;
                }
                double o = A[4 * r + 3];
                for (int k = 0; k < 3; ++k) o += (double)A[4 * r + k] * cp[k];
                h.o[r] = (float)o;
            }
            h.fx = L.shadow_cam.fx; h.fy = L.shadow_cam.fy; h.cx = L.shadow_cam.cx; h.cy = L.shadow_cam.cy;
            h.w = L.shadow_cam.width; h.h = L.shadow_cam.height;
            h.bias = L.shadow_bias;
        }
    }
    a.irr = ibl->irradiance.data; a.irr_size = ibl->irradiance.size;
    a.pref = ibl->prefiltered.data; a.pref_base = ibl->prefiltered.size; a.pref_levels = ibl->prefiltered.levels;
    a.lut = ibl->brdf_lut; a.lut_size = ibl->lut_size;
    a.env = env->data; a.env_size = env->size;
    a.hdr = hdr_out;
    a.hdr_dtype = hdr_dtype;
    return hip_status(epb::launch_shade(a, stream));
}

int epb_bloom_tonemap(const void *hdr, epb_dtype hdr_dtype, int32_t width, int32_t height,
                      const epb_post_params *params, uint8_t *ldr_out, void *scratch, size_t scratch_bytes,
                      hipStream_t stream) {
    if (!hdr || !params || !ldr_out) return EPB_ERR_NULL;
    if (width < 1 || height < 1 || width > EPB_MAX_IMAGE_SIZE || height > EPB_MAX_IMAGE_SIZE) return EPB_ERR_SIZE;
    if (!valid_dtype(hdr_dtype)) return EPB_ERR_DTYPE;
    if (params->bloom_levels < 1 || params->bloom_levels > EPB_MAX_BLOOM_LEVELS) return EPB_ERR_PARAM;
    if (!finite(params->threshold) || !finite(params->strength) || !(params->exposure > 0) ||
        !finite(params->exposure) || !(params->gamma > 0) || !finite(params->gamma))
        return EPB_ERR_PARAM;
    if (!valid_dtype(params->pyr_dtype)) return EPB_ERR_DTYPE;
    if (!aligned16(hdr) || !aligned16(ldr_out)) return EPB_ERR_ALIGN;
    epb::PostPlan plan = epb::post_plan(width, height, params->bloom_levels, params->pyr_dtype);
    if (!scratch || scratch_bytes < plan.bytes) return EPB_ERR_SCRATCH;
    if (!aligned16(scratch)) return EPB_ERR_ALIGN;
    return hip_status(epb::launch_bloom_tonemap(plan, hdr, hdr_dtype, params->threshold, params->strength,
                                                params->exposure, params->gamma, ldr_out, scratch, stream));
}

}  // extern "C"
