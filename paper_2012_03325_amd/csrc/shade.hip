// Compose pass (paper Sec. 4.2): surfel G-buffers normalised by their
// accumulated weight (Sec. 4.4), position from depth (Sec. 4), Cook-Torrance
// direct lighting in the Unreal Engine 4 variant (Sec. 3) with 3x3
// percentage-closer shadow tests (Sec. 5.1), split-sum image-based lighting
// with multiple-scattering compensation (Sec. 3.1) scaled by ambient
// occlusion (Sec. 5.2), environment behind the scene.
//
// gfx950 mapping: one thread per pixel, 32x8 pixel tiles (a wavefront covers
// 32x2 pixels: two 128-byte row segments of every planar G-buffer channel),
// consecutive tiles on the same XCD so that the shadow-map and IBL texels a
// band of rows touches stay in that XCD's L2.  Lights travel in the kernel
// argument segment and are read with scalar loads.
//
// Float32 care where the reference is float64:
//  * GGX: 1 - (N.H)^2 is taken as |H - (N.H) N|^2 (= |N x H|^2 for unit
//    vectors), exact to rounding near the highlight peak where the
//    subtraction would cancel (roughness 0.05 gives alpha^2 = 6e-6).
//  * Smith-Schlick visibility G / (4 N.L N.V) is evaluated as
//    1 / (4 (N.L(1-k)+k)(N.V(1-k)+k)): no division by a clamped N.V.
//  * The view vector is -normalize(R^T P_view), free of the cancellation of
//    camera_position - world_position for distant pixels.
#include "device_common.hpp"
#include "launch.hpp"
#include "shade_tiles.hpp"

namespace epb {

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
// Minimum waves per SIMD: 7, the FP32 kernel's natural 65 VGPRs (69 with the
// bloom epilogue).  At 8 (64 VGPRs) the FP16 kernel spills and runs 3 us
// slower at 1080p; the batched kernel, with the view lookup on top, would
// settle at 6.
constexpr int kShadeMinWaves = 7;

template <int TX, int TY, bool kBloom1, typename TG, typename TA, typename TH>
__global__ void __launch_bounds__(TX *TY) __attribute__((amdgpu_waves_per_eu(kShadeMinWaves)))
k_shade(const ShadeDesc c, int tiles) {
    shade_tile<TX, TY, kBloom1, TG, TA, TH>(c, xcd_tile(blockIdx.x, tiles));
}

template <int TX, int TY, bool kBloom1, typename TG, typename TA, typename TH>
__global__ void __launch_bounds__(TX *TY) __attribute__((amdgpu_waves_per_eu(kShadeMinWaves)))
k_shade_batch(const void *__restrict__ table) {
    const BatchHeader *h = (const BatchHeader *)table;
    const int *start = batch_start(table, kStShade);
    const ViewDesc *views = batch_views(table);
    XcdRange w = xcd_range(h->total[kStShade]);
    for (int it = w.lb; it < w.count; it += w.stride) {
        int g = w.first + it;
        int v = find_view(start, h->n_views, g);
        shade_tile<TX, TY, kBloom1, TG, TA, TH>(views[v].shade, g - start[v]);
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
ShadeDesc shade_desc(const ShadeArgs &a) {
    ShadeDesc k{};
    k.depth = a.depth;
    k.normal = a.normal; k.albedo = a.albedo; k.rough = a.rough; k.metal = a.metal;
    k.weight = a.weight;
    k.ao = a.ao;
    k.hdr = a.hdr;
    k.irr = (const float4 *)a.irr;
    k.pref = (const float4 *)a.pref;
    k.env = (const float4 *)a.env;
    k.lut = (const float2 *)a.lut;
    for (int i = 0; i < 9; ++i) k.R[i] = a.cam.R[i];
    for (int i = 0; i < 3; ++i) k.cam_pos[i] = a.cam_pos[i];
    k.cx = a.cam.cx; k.cy = a.cam.cy; k.inv_fx = a.cam.inv_fx; k.inv_fy = a.cam.inv_fy;
    k.W = a.W; k.H = a.H; k.Wh = (a.W + 1) / 2; k.Hh = (a.H + 1) / 2;
    k.irr_size = a.irr_size; k.pref_base = a.pref_base; k.pref_levels = a.pref_levels;
    k.lut_size = a.lut_size; k.env_size = a.env_size;
    k.irr_dims = face_dims(a.irr_size); k.lut_dims = face_dims(a.lut_size); k.env_dims = face_dims(a.env_size);
    k.f_levels1 = (float)(a.pref_levels - 1);
    int off = 0;
    for (int m = 0; m < 8; ++m) {
        int sm = m < a.pref_levels ? a.pref_base >> m : 2;
        k.pref_off[m] = off;
        if (m < a.pref_levels) off += 6 * sm * sm;
    }
    k.n_lights = a.n_lights;
    for (int i = 0; i < a.n_lights; ++i) k.lights[i] = a.lights[i];
    return k;
}

int shade_items(const ShadeDesc &c, int shade_tile) {
    TileShape t = kShadeTiles[shade_tile];
    return ceil_div(c.W, t.tx) * ceil_div(c.H, t.ty);
}

template <typename TG, typename TA, typename TH>
static void go(const ShadeDesc &k, hipStream_t s) {
    int tiles = shade_items(k, 0);
    if (k.bloom1)
        hipLaunchKernelGGL((k_shade<32, 8, true, TG, TA, TH>), dim3(tiles), dim3(256), 0, s, k, tiles);
    else
        hipLaunchKernelGGL((k_shade<32, 8, false, TG, TA, TH>), dim3(tiles), dim3(256), 0, s, k, tiles);
}
template <int TX, int TY, bool kBloom1, typename TG, typename TA, typename TH>
static void go_batch(const BatchHeader &h, const void *table, hipStream_t s) {
    hipLaunchKernelGGL((k_shade_batch<TX, TY, kBloom1, TG, TA, TH>),
                       dim3(batch_grid(h.total[kStShade], h.blocks_per_cu)), dim3(TX * TY), 0, s, table);
}
template <typename TG, typename TA, typename TH>
static void go_shape(const BatchHeader *h, const void *table, const ShadeDesc *k, hipStream_t s) {
    if (!h) {
        go<TG, TA, TH>(*k, s);
        return;
    }
    if (h->fuse_bloom) {  // 32 x 8 tiles only (rows 2k, 2k + 1 in one wavefront; checked on the host)
        go_batch<32, 8, true, TG, TA, TH>(*h, table, s);
        return;
    }
    switch (h->shade_tile) {
    case 1: go_batch<64, 4, false, TG, TA, TH>(*h, table, s); break;
    case 2: go_batch<16, 16, false, TG, TA, TH>(*h, table, s); break;
    default: go_batch<32, 8, false, TG, TA, TH>(*h, table, s); break;
    }
}
template <typename TG, typename TA>
static void go_h(const BatchHeader *h, const void *table, const ShadeDesc *k, epb_dtype hd, hipStream_t s) {
    if (hd == EPB_F32) go_shape<TG, TA, float>(h, table, k, s);
    else go_shape<TG, TA, __half>(h, table, k, s);
}
template <typename TG>
static void go_a(const BatchHeader *h, const void *table, const ShadeDesc *k, epb_dtype ad, epb_dtype hd,
                 hipStream_t s) {
    if (ad == EPB_F32) go_h<TG, float>(h, table, k, hd, s);
    else go_h<TG, __half>(h, table, k, hd, s);
}

hipError_t launch_shade(const ShadeArgs &a, hipStream_t s, const PostDesc *bloom) {
    ShadeDesc k = shade_desc(a);
    if (bloom && bloom->nl >= 1) {  // the fused form writes bloom level 1 as well
        k.bloom1 = bloom->raw[1];
        k.bloom1_half = bloom->texel_half;
        k.bloom_threshold = bloom->threshold;
    }
    if (a.gdtype == EPB_F32) go_a<float>(nullptr, nullptr, &k, a.ao_dtype, a.hdr_dtype, s);
    else go_a<__half>(nullptr, nullptr, &k, a.ao_dtype, a.hdr_dtype, s);
    return hipGetLastError();
}

// Tiled form of a shadow map: one thread per stored float, one row of tiles per
// blockIdx.y (the last row holds the all-+inf tile); consecutive threads write
// consecutive floats and read runs of 8 texels of a map row.  Stored float
// (p nx + q) 64 + 8 j + i is texel (6 q + i - 1, 6 p + j - 1) of the map, +inf
// outside it.
__global__ void __launch_bounds__(256) k_shadow_tiles(const float *__restrict__ map, int w, int h, int nx, int ny,
                                                      float *__restrict__ tiles) {
    unsigned t = blockIdx.x * 256u + threadIdx.x;  // float index inside this row of tiles
    unsigned p = blockIdx.y;
    if (t >= (p < (unsigned)ny ? (unsigned)nx * 64u : 64u)) return;
    unsigned q = t >> 6, j = (t >> 3) & 7u, i = t & 7u;
    int x = (int)(6u * q + i) - 1, y = (int)(6u * p + j) - 1;
    float v = __builtin_inff();
    if (p < (unsigned)ny && x >= 0 && x < w && y >= 0 && y < h) v = map[(size_t)y * (unsigned)w + (unsigned)x];
    tiles[(size_t)p * nx * 64u + t] = v;
}

ShadowTilesPlan shadow_tiles_plan(int w, int h) {
    ShadowTilesPlan t{};
    t.nx = ceil_div(w, 6);
    t.ny = ceil_div(h, 6);
    t.bytes = ((size_t)t.nx * (size_t)t.ny + 1u) * 256u;
    t.pitch = 256u * (unsigned)t.nx - 192u;
    t.sentinel = (unsigned)t.nx * (unsigned)t.ny * 256u;
    return t;
}

hipError_t launch_shadow_tiles(const float *map, int w, int h, float *tiles, hipStream_t s) {
    ShadowTilesPlan t = shadow_tiles_plan(w, h);
    dim3 grid(ceil_div(t.nx * 64, 256), t.ny + 1);
    k_shadow_tiles<<<grid, 256, 0, s>>>(map, w, h, t.nx, t.ny, tiles);
    return hipGetLastError();
}

hipError_t launch_shade_batch(const BatchHeader &h, const void *table, hipStream_t s) {
    epb_dtype ad = (epb_dtype)h.ao_dtype, hd = (epb_dtype)h.hdr_dtype;
    if (h.gdtype == EPB_F32) go_a<float>(&h, table, nullptr, ad, hd, s);
    else go_a<__half>(&h, table, nullptr, ad, hd, s);
    return hipGetLastError();
}

}  // namespace epb
