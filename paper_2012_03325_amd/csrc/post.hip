// Bloom (paper Sec. 5.3) and final compositing with ACES tone mapping and
// gamma correction (Sec. 5.4).
//
// gfx950 mapping:
//  * bloom_down: one workgroup per 32x32-pixel tile reads the HDR planes
//    once (one level-1 texel per thread, its twelve loads in flight together),
//    forms the bright map and its 2x2 means, and builds pyramid levels 1..5 of
//    that tile in LDS (16x16 level-1 texels halve down to one at level 5),
//    writing every level once.
//  * bloom_blur: all levels in one launch; each workgroup stages the 36x20
//    texel footprint of its 32x16 tile in LDS and applies the separable
//    [1 4 6 4 1] / 16 binomial (clamp to edge) horizontally then vertically.
//  * composite: a wavefront covers 64 columns x 8 rows, a thread one column
//    of 8 pixels; every blurred level is interpolated at the column (rows
//    first, then between two rows per pixel) in registers; each thread adds
//    the upsampled levels to its pixels, applies exposure, the ACES fit,
//    gamma and 8-bit rounding, and writes one 32-bit RGBA word per pixel.
//  * pyramid texels are float4, or four halves in the FP16 form.
//  * every stage has a single-view kernel and a batched kernel that walks the
//    work items of many views.
#include "device_common.hpp"
#include "launch.hpp"
#include "post_tiles.hpp"

namespace epb {

// ---------------------------------------------------------------------------
// kernels: single view (XCD-aware tile order) and batched (persistent range)
// ---------------------------------------------------------------------------
template <typename TH, typename TP>
__global__ void __launch_bounds__(256) k_bloom_down(const PostDesc c, int tiles) {
    __shared__ DownLds sm;
    bloom_down_tile<TH, TP>(c, xcd_tile(blockIdx.x, tiles), sm);
}

template <typename TP>
__global__ void __launch_bounds__(256) k_bloom_down_from1(const PostDesc c, int tiles) {
    __shared__ DownLds sm;
    bloom_down_from1_tile<TP>(c, xcd_tile(blockIdx.x, tiles), sm);
}

template <typename TP>
__global__ void __launch_bounds__(256) k_bloom_blur(const PostDesc c) {
    __shared__ BlurLds sm;
    bloom_blur_item<TP>(c, blockIdx.x, sm);
}

template <typename TH, typename TP>
__global__ void __launch_bounds__(kPostTx) __attribute__((amdgpu_waves_per_eu(5))) k_composite(const PostDesc c, int tiles) {
    composite_tile<TH, TP>(c, xcd_tile(blockIdx.x, tiles), (int)threadIdx.x);
}

template <typename TH, typename TP>
__global__ void __launch_bounds__(256) k_bloom_down_batch(const void *__restrict__ table) {
    __shared__ DownLds sm;
    const BatchHeader *h = (const BatchHeader *)table;
    const int *start = batch_start(table, kStDown);
    const ViewDesc *views = batch_views(table);
    XcdRange w = xcd_range(h->total[kStDown]);
    for (int it = w.lb; it < w.count; it += w.stride) {
        int g = w.first + it;
        int v = find_view(start, h->n_views, g);
        bloom_down_tile<TH, TP>(views[v].post, g - start[v], sm);
    }
}

template <typename TP>
__global__ void __launch_bounds__(256) k_bloom_down_from1_batch(const void *__restrict__ table) {
    __shared__ DownLds sm;
    const BatchHeader *h = (const BatchHeader *)table;
    const int *start = batch_start(table, kStDown);
    const ViewDesc *views = batch_views(table);
    XcdRange w = xcd_range(h->total[kStDown]);
    for (int it = w.lb; it < w.count; it += w.stride) {
        int g = w.first + it;
        int v = find_view(start, h->n_views, g);
        bloom_down_from1_tile<TP>(views[v].post, g - start[v], sm);
    }
}

template <typename TP>
__global__ void __launch_bounds__(256) k_bloom_blur_batch(const void *__restrict__ table) {
    __shared__ BlurLds sm;
    const BatchHeader *h = (const BatchHeader *)table;
    const int *start = batch_start(table, kStBloomBlur);
    const ViewDesc *views = batch_views(table);
    XcdRange w = xcd_range(h->total[kStBloomBlur]);
    for (int it = w.lb; it < w.count; it += w.stride) {
        int g = w.first + it;
        int v = find_view(start, h->n_views, g);
        bloom_blur_item<TP>(views[v].post, g - start[v], sm);
    }
}

template <typename TH, typename TP>
__global__ void __launch_bounds__(kPostTx) __attribute__((amdgpu_waves_per_eu(5))) k_composite_batch(const void *__restrict__ table) {
    const BatchHeader *h = (const BatchHeader *)table;
    const int *start = batch_start(table, kStComposite);
    const ViewDesc *views = batch_views(table);
    XcdRange w = xcd_range(h->total[kStComposite]);
    for (int it = w.lb; it < w.count; it += w.stride) {
        int g = w.first + it;
        int v = find_view(start, h->n_views, g);
        composite_tile<TH, TP>(views[v].post, g - start[v], (int)threadIdx.x);
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
PostPlan post_plan(int W, int H, int levels, epb_dtype pyr_dtype) {
    PostPlan q{};
    q.W = W;
    q.H = H;
    q.levels = levels;
    q.texel_bytes = pyr_dtype == EPB_F16 ? 8 : 16;
    q.lw[0] = W;
    q.lh[0] = H;
    for (int l = 1; l < levels; ++l) {
        q.lw[l] = (q.lw[l - 1] + 1) / 2;
        q.lh[l] = (q.lh[l - 1] + 1) / 2;
    }
    size_t off = 0;
    for (int l = 1; l < levels; ++l) {  // blurred levels first (documented scratch layout)
        q.off_blur[l] = off;
        off += (size_t)q.lw[l] * q.lh[l] * q.texel_bytes;
    }
    off = (off + 255) & ~size_t(255);
    for (int l = 1; l < levels; ++l) {
        q.off_raw[l] = off;
        off += (size_t)q.lw[l] * q.lh[l] * q.texel_bytes;
    }
    q.bytes = (off + 255) & ~size_t(255);
    if (q.bytes == 0) q.bytes = 256;
    return q;
}

PostDesc post_desc(const PostPlan &q, const void *hdr, float threshold, float strength, float exposure,
                   float gamma, int tonemap, uint8_t *ldr, void *scratch) {
    PostDesc c{};
    c.W = q.W;
    c.H = q.H;
    c.nl = q.levels - 1;
    c.texel_half = q.texel_bytes == 8;
    char *sc = (char *)scratch;
    for (int l = 0; l < q.levels; ++l) {
        c.lw[l] = q.lw[l];
        c.lh[l] = q.lh[l];
        if (l >= 1) {
            c.raw[l] = sc + q.off_raw[l];
            c.blur[l] = sc + q.off_blur[l];
        }
    }
    int nb = 0;
    for (int l = 1; l <= c.nl; ++l) {
        c.blk_start[l] = nb;
        nb += ceil_div(c.lw[l], kBloomTx) * ceil_div(c.lh[l], kBloomTy);
    }
    c.blk_start[c.nl + 1] = nb;
    c.threshold = threshold;
    c.strength = strength;
    c.exposure = exposure;
    c.inv_gamma = 1.0f / gamma;
    c.tonemap = tonemap;
    c.hdr = hdr;
    c.ldr = (uint32_t *)ldr;
    return c;
}

int post_items(const PostDesc &c, int stage) {
    if (stage == kStDown) return c.nl >= 1 ? ceil_div(c.lw[1], kDownTile) * ceil_div(c.lh[1], kDownTile) : 0;
    if (stage == kStBloomBlur) return c.nl >= 1 ? c.blk_start[c.nl + 1] : 0;
    return ceil_div(c.W, kPostTx) * ceil_div(c.H, kPostTy);
}

template <typename TH, typename TP>
static void launch_post(const PostDesc &c, bool level1_given, hipStream_t s) {
    if (c.nl >= 1) {
        int tiles = post_items(c, kStDown);
        if (!level1_given)
            hipLaunchKernelGGL((k_bloom_down<TH, TP>), dim3(tiles), dim3(256), 0, s, c, tiles);
        else if (c.nl >= 2)
            hipLaunchKernelGGL(k_bloom_down_from1<TP>, dim3(tiles), dim3(256), 0, s, c, tiles);
        hipLaunchKernelGGL(k_bloom_blur<TP>, dim3(post_items(c, kStBloomBlur)), dim3(256), 0, s, c);
    }
    int tiles = post_items(c, kStComposite);
    hipLaunchKernelGGL((k_composite<TH, TP>), dim3(tiles), dim3(kPostTx), 0, s, c, tiles);
}

template <typename TH, typename TP>
static void launch_post_batch_t(const BatchHeader &h, const void *table, hipStream_t s) {
    if (h.total[kStDown] > 0 && h.fuse_bloom)  // level 1 came from the shading stage
        hipLaunchKernelGGL(k_bloom_down_from1_batch<TP>, dim3(batch_grid(h.total[kStDown], h.blocks_per_cu)),
                           dim3(256), 0, s, table);
    else if (h.total[kStDown] > 0)
        hipLaunchKernelGGL((k_bloom_down_batch<TH, TP>), dim3(batch_grid(h.total[kStDown], h.blocks_per_cu)),
                           dim3(256), 0, s, table);
    if (h.total[kStBloomBlur] > 0)
        hipLaunchKernelGGL(k_bloom_blur_batch<TP>, dim3(batch_grid(h.total[kStBloomBlur], h.blocks_per_cu)),
                           dim3(256), 0, s, table);
    hipLaunchKernelGGL((k_composite_batch<TH, TP>), dim3(batch_grid(h.total[kStComposite], h.blocks_per_cu)),
                       dim3(kPostTx), 0, s, table);
}

hipError_t launch_bloom_tonemap(const PostDesc &c, epb_dtype hdr_dtype, epb_dtype pyr_dtype, hipStream_t s,
                                bool level1_given) {
    bool h16 = hdr_dtype == EPB_F16, p16 = pyr_dtype == EPB_F16;
    if (!h16 && !p16) launch_post<float, float4>(c, level1_given, s);
    else if (!h16 && p16) launch_post<float, Half4>(c, level1_given, s);
    else if (h16 && !p16) launch_post<__half, float4>(c, level1_given, s);
    else launch_post<__half, Half4>(c, level1_given, s);
    return hipGetLastError();
}

hipError_t launch_post_batch(const BatchHeader &h, const void *table, hipStream_t s) {
    bool h16 = h.hdr_dtype == EPB_F16, p16 = h.pyr_dtype == EPB_F16;
    if (!h16 && !p16) launch_post_batch_t<float, float4>(h, table, s);
    else if (!h16 && p16) launch_post_batch_t<float, Half4>(h, table, s);
    else if (h16 && !p16) launch_post_batch_t<__half, float4>(h, table, s);
    else launch_post_batch_t<__half, Half4>(h, table, s);
    return hipGetLastError();
}

}  // namespace epb
