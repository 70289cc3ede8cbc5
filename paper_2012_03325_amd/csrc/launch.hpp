// Internal launch interface between the C ABI (api.cpp) and the kernels.
// Arguments are already validated when these are called; each launcher
// returns the hipError_t of its launches.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/epb.h"
#include "desc.hpp"

namespace epb {

struct HostCam {
    float R[9], t[3];
    float fx, fy, cx, cy, inv_fx, inv_fy;
    int w, h;
};

// Grid of a batched stage: one block per item, or a persistent grid of
// blocks_per_cu blocks per CU.
int batch_grid(int total, int blocks_per_cu);

// ---- image-based lighting (ibl.hip) ---------------------------------------
struct IblPlan {
    int S;          // environment face size
    int src;        // irradiance source size
    int irr;        // irradiance output size
    int pref_base, pref_levels, pref_samples;
    int lut, lut_samples;
    int chunks;     // split of the irradiance source sum
    int fis;        // filtered importance sampling of the prefilter
    int chain_last; // last level of the environment mip chain (faces >= 2x2)
    size_t off_src, off_tab, off_part, off_chain, off_ggx, off_rgb, off_ppart, bytes;  // scratch layout
};
IblPlan ibl_plan(int S, const epb_ibl_params &p);
hipError_t launch_precompute_ibl(const IblPlan &plan, const float *env, float *irr, float *pref,
                                 float *lut, void *scratch, hipStream_t s);

// ---- SSAO (ssao.hip) --------------------------------------------------------
struct SsaoPlan {
    int W, H, Wh, Hh;
    size_t off_hdepth, off_raw, bytes;
};
SsaoPlan ssao_plan(int W, int H);
SsaoDesc ssao_desc(const SsaoPlan &q, const float *depth, const void *normal, const HostCam &cam,
                   const float *kernel, int n_samples, const float *noise, float radius, float bias,
                   float tau, int blur, void *ao_out, void *scratch);
int ssao_items(const SsaoDesc &c, int stage, int ssao_tile);
hipError_t launch_ssao(const SsaoDesc &c, epb_dtype gdtype, epb_dtype ao_dtype, hipStream_t s);
hipError_t launch_ssao_batch(const BatchHeader &h, const void *table, hipStream_t s);
// Device address of the library's own SSAO scratch array on the current device
// (EPB_SSAO_STATIC_SCRATCH_BYTES bytes), looked up once per device.
hipError_t ssao_static_scratch(void **addr);

// ---- shading (shade.hip) ----------------------------------------------------
struct ShadeArgs {
    const float *depth;
    const void *normal, *albedo, *rough, *metal;
    const void *weight;  // accumulated surfel weight, or null
    epb_dtype gdtype;
    int W, H;
    HostCam cam;
    float cam_pos[3];
    const void *ao;
    epb_dtype ao_dtype;
    int n_lights;
    DevLight lights[EPB_MAX_LIGHTS];
    const float *irr;
    int irr_size;
    const float *pref;
    int pref_base, pref_levels;
    const float *lut;
    int lut_size;
    const float *env;
    int env_size;
    void *hdr;
    epb_dtype hdr_dtype;
};
ShadeDesc shade_desc(const ShadeArgs &a);
int shade_items(const ShadeDesc &c, int shade_tile);
// with `bloom` (the fused form), level 1 of its pyramid is written as well
hipError_t launch_shade(const ShadeArgs &a, hipStream_t s, const PostDesc *bloom = nullptr);

// Tiled form of a w x h shadow map (w, h >= 3) padded with a +inf apron:
// nx x ny tiles of 6x6 texels, each stored as 8x8 floats, then one all-+inf
// tile; pitch and sentinel are DevLight::tile_pitch and DevLight::sentinel.
struct ShadowTilesPlan {
    int nx, ny;
    size_t bytes;
    unsigned pitch, sentinel;
};
ShadowTilesPlan shadow_tiles_plan(int w, int h);
hipError_t launch_shadow_tiles(const float *map, int w, int h, float *tiles, hipStream_t s);
hipError_t launch_shade_batch(const BatchHeader &h, const void *table, hipStream_t s);

// ---- bloom + tonemap (post.hip) ----------------------------------------------
struct PostPlan {
    int W, H, levels;
    int texel_bytes;  // 16 (float4) or 8 (half4) per pyramid texel
    int lw[EPB_MAX_BLOOM_LEVELS], lh[EPB_MAX_BLOOM_LEVELS];
    size_t off_blur[EPB_MAX_BLOOM_LEVELS];  // blurred level l
    size_t off_raw[EPB_MAX_BLOOM_LEVELS];   // unblurred level l
    size_t bytes;
};
PostPlan post_plan(int W, int H, int levels, epb_dtype pyr_dtype);
PostDesc post_desc(const PostPlan &q, const void *hdr, float threshold, float strength, float exposure,
                   float gamma, int tonemap, uint8_t *ldr, void *scratch);
int post_items(const PostDesc &c, int stage);
// level1_given: the shading pass has written pyramid level 1 (the fused form)
hipError_t launch_bloom_tonemap(const PostDesc &c, epb_dtype hdr_dtype, epb_dtype pyr_dtype, hipStream_t s,
                                bool level1_given = false);
hipError_t launch_post_batch(const BatchHeader &h, const void *table, hipStream_t s);

// persistent.hip: the whole batch in one launch (the table's persistent schedule); the
// table must be the device copy, whose work counters it clears and updates
hipError_t launch_persistent(const BatchHeader &h, const void *table, hipStream_t s);

// ---- eye-dome lighting (edl.hip) ---------------------------------------------
hipError_t launch_edl(const EdlDesc &c, epb_dtype cdtype, epb_dtype ao_dtype, epb_dtype hdr_dtype, hipStream_t s);

// ---- ray-cast G-buffers and depth maps (raycast.hip) ------------------------
hipError_t launch_raycast(const RayScene &s, const RayCam &c, const RayOut &out, epb_dtype dtype, void *scratch,
                          hipStream_t st);

}  // namespace epb
