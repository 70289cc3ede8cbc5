// Plain descriptors shared by host set-up code and kernels: one view's inputs,
// outputs and scratch for each stage of the shading pass, and the layout of
// the batch table that carries many views to the batched kernels.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "../../include/epb.h"

namespace epb {

// Sizes of a face of S x S texels as the bilinear lookups use them; all exact
// in float.  Kernels take them precomputed (kernel arguments, scalar
// registers) where S is the same for every lane.
struct FaceDims {
    int S;
    float half, off, hi, hi1;  // S / 2, S / 2 - 1/2, S - 1, S - 2
};
__host__ __device__ inline FaceDims face_dims(int S) {
    float fS = (float)S;
    return FaceDims{S, 0.5f * fS, 0.5f * fS - 0.5f, fS - 1.0f, fS - 2.0f};
}

// Rigid camera with precomputed reciprocals.
struct DevCam {
    float R[9];  // row-major rotation
    float t[3];
    float fx, fy, cx, cy;
    float inv_fx, inv_fy;
    int w, h;
};

// Point light with an optional depth map, transforms composed on the host.
struct DevLight {
    float pos[3], rad[3];  // rad = colour * intensity
    const float *map;      // may be null
    // light view from camera view, P_l = R P_v + t, with the rows of x and y scaled
    // by fx and -fy (the map's v axis points down): M P_v + o = ((u - cx) d_l,
    // (v - cy) d_l, -d_l) for the map coordinates (u, v) and light depth d_l
    float M[9], o[3];
    float cx, cy;
    int w, h;
    float fw, fh;          // w, h as floats
    float bias;
    int tiles;             // map in the tiled form (6x6 texels per 8x8 block, +inf apron)
    unsigned tile_pitch;   // byte step per row of tiles minus 6 block rows: 256 nx - 192
    unsigned sentinel;     // byte offset of the tiled form's all-+inf tile
};

struct SsaoDesc {
    DevCam cam;
    float radius, bias, tau, inv_n;
    int n, blur;
    int W, H, Wh, Hh;
    const float *depth;
    const void *normal;
    const float *kernel;  // [n][3]
    const float *noise;   // [4][4][2]
    float *hdepth;        // scratch: compact half-resolution depth
    void *raw;            // raw AO: scratch when blurred, else the output
    void *out;            // AO output
};

struct ShadeDesc {
    const float *depth;
    const void *normal, *albedo, *rough, *metal;
    const void *weight;  // accumulated surfel weight, or null
    const void *ao;  // may be null
    void *hdr;
    const float4 *irr, *pref, *env;
    const float2 *lut;
    float R[9];
    float cam_pos[3];
    float cx, cy, inv_fx, inv_fy;
    int W, H, Wh, Hh;
    int irr_size, pref_base, pref_levels, lut_size, env_size;
    FaceDims irr_dims, lut_dims, env_dims;  // sizes of the lookups (host-computed)
    float f_levels1;                        // levels - 1
    int pref_off[8];                       // texel offset of each prefiltered level
    int n_lights;
    DevLight lights[EPB_MAX_LIGHTS];
    void *bloom1;           // bloom level 1, written by the fused form; null otherwise
    int bloom1_half;        // its texels are four halves (else float4)
    float bloom_threshold;
};

struct PostDesc {
    int W, H, nl;  // nl = number of pyramid levels >= 1
    int texel_half;  // pyramid texels are four halves (else float4)
    int lw[EPB_MAX_BLOOM_LEVELS], lh[EPB_MAX_BLOOM_LEVELS];
    void *raw[EPB_MAX_BLOOM_LEVELS];   // unblurred level texels (pyramid storage type)
    void *blur[EPB_MAX_BLOOM_LEVELS];  // blurred level texels
    int blk_start[EPB_MAX_BLOOM_LEVELS + 1];  // first blur work item of each level
    float threshold, strength, exposure, inv_gamma;
    int tonemap;  // EPB_TONEMAP_ACES or EPB_TONEMAP_REINHARD
    const void *hdr;
    uint32_t *ldr;
};

// Eye-dome lighting of a depth map with per-pixel colour.
struct EdlDesc {
    const float *depth;
    const void *color;  // [3][H][W]
    const void *ao;     // half resolution, may be null
    void *hdr;
    const float4 *env;  // level 0 shown behind the cloud, may be null
    float R[9];
    float cx, cy, inv_fx, inv_fy;
    int W, H, Wh, Hh;
    int env_size;
    FaceDims env_dims;
    int radius, n_dirs;
    float neg_strength_over_n;  // -strength / n_dirs
    float far_depth;
    int loff[EPB_MAX_EDL_DIRS];  // LDS index delta of each neighbour (tile pitch 32 + 2 radius)
};

// Ray-cast pass: sphere field, double-precision camera, destination planes.
struct RayScene {
    int n;
    const double *center, *radius;
    const float *albedo, *rough, *metal;
    int plane;
    float plane_albedo[3], plane_rough, plane_metal;
};
struct RayCam {
    double M[12];  // row-major [R | t]
    double fx, fy, cx, cy;
    int W, H;
};
struct RayOut {
    float *depth;
    void *normal, *albedo, *rough, *metal;  // null normal: depth only
};

// ---------------------------------------------------------------------------
// tile shapes
// ---------------------------------------------------------------------------
constexpr int kSsaoPrepW = 256;           // half-resolution texels per prep item
constexpr int kBlurTx = 16, kBlurTy = 8;  // SSAO blur tile
constexpr int kPostTx = 64, kPostTy = 8;  // composite: one wavefront, a column of 8 pixels per thread
constexpr int kBloomTx = 32, kBloomTy = 16;  // bloom-blur tile
constexpr int kDownTile = 16;             // bloom_down: 16x16 level-1 texels (32x32 pixels)

// Selectable shapes (the schedule picks one per stage).
struct TileShape {
    int tx, ty;
};
constexpr TileShape kShadeTiles[3] = {{32, 8}, {64, 4}, {16, 16}};
constexpr TileShape kSsaoTiles[3] = {{16, 8}, {32, 4}, {16, 16}};  // the last one stages its window in LDS
constexpr int kSsaoLdsTile = 16, kSsaoHalo = 32;                     // LDS variant: tile and halo
constexpr int kSsaoLdsW = kSsaoLdsTile + 2 * kSsaoHalo;             // window side: 80 texels, 25.6 KB
constexpr int kSsaoBatches[2] = {8, 16};

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// batch table: [BatchHeader][int start[kStages][n + 1]][int cstart[kStages][n + 1]]
// [pad to 16][ViewDesc[n]][pad to 256][PersistState][int done[n][kStages]]
// ---------------------------------------------------------------------------
enum Stage { kStPrep = 0, kStRaw, kStBlur, kStShade, kStDown, kStBloomBlur, kStComposite, kStages };

struct ViewDesc {
    SsaoDesc ssao;
    ShadeDesc shade;
    PostDesc post;
};

struct BatchHeader {
    uint32_t magic;
    int n_views;
    int gdtype, ao_dtype, hdr_dtype, pyr_dtype;
    int blur, has_ao;
    int shade_tile, ssao_tile, ssao_batch, blocks_per_cu;
    int fuse_bloom;      // the shading stage writes bloom level 1; the down stage starts from it
    int total[kStages];  // work items of each stage over all views
    // one persistent launch (persistent != 0): work items are chunks of `chunk`
    // tiles of one view and stage, handed out in stage-major order
    int persistent, chunk;
    int wait_limit;                 // polls of a dependency before the block gives up
    int gate;                       // 1; 0 makes every dependency wait give up (error-path tests)
    int total_chunks;
    int chunk_first[kStages + 1];   // first chunk of each stage
};

// Work counters of the persistent launch, in the device copy of the table; the
// launch clears them first.  done[v][s] (after this struct) counts the finished
// chunks of view v's stage s.
struct PersistState {
    int head;                 // next chunk to hand out
    int error;                // a dependency wait gave up
    int stage_done[kStages];  // finished chunks of each stage over all views
    int pad[16 - 2 - kStages];
};
static_assert(sizeof(PersistState) == 64, "one 64-byte block");

// Persistent launch: tile shapes of the stages whose single-view / batched tile
// is not 256 threads (SSAO raw and blur: 16 x 16 texels; composite: 4 tiles of
// 64 x 8 pixels, one per wavefront).
constexpr int kPersistSsaoT = 16;
constexpr int kPersistCompositeTiles = 4;

constexpr uint32_t kBatchMagic = 0x45504232u;  // "EPB2"

__host__ __device__ inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
__host__ __device__ inline size_t batch_start_offset() { return align_up(sizeof(BatchHeader), 16); }
__host__ __device__ inline size_t batch_cstart_offset(int n) {
    return batch_start_offset() + sizeof(int) * kStages * (size_t)(n + 1);
}
__host__ __device__ inline size_t batch_views_offset(int n) {
    return align_up(batch_cstart_offset(n) + sizeof(int) * kStages * (size_t)(n + 1), 16);
}
__host__ __device__ inline size_t batch_state_offset(int n) {
    return align_up(batch_views_offset(n) + sizeof(ViewDesc) * (size_t)n, 256);
}
__host__ __device__ inline size_t batch_table_bytes(int n) {
    return batch_state_offset(n) + sizeof(PersistState) + sizeof(int) * kStages * (size_t)n;
}

__host__ __device__ inline const int *batch_start(const void *table, int stage) {
    const BatchHeader *h = (const BatchHeader *)table;
    return (const int *)((const char *)table + batch_start_offset()) + stage * (h->n_views + 1);
}
__host__ __device__ inline const int *batch_cstart(const void *table, int stage) {
    const BatchHeader *h = (const BatchHeader *)table;
    return (const int *)((const char *)table + batch_cstart_offset(h->n_views)) + stage * (h->n_views + 1);
}
__host__ __device__ inline const ViewDesc *batch_views(const void *table) {
    const BatchHeader *h = (const BatchHeader *)table;
    return (const ViewDesc *)((const char *)table + batch_views_offset(h->n_views));
}

}  // namespace epb
