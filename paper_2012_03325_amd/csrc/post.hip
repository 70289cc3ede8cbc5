// Bloom (paper Sec. 5.3) and final compositing with ACES tone mapping and
// gamma correction (Sec. 5.4).
//
// gfx950 mapping:
//  * bloom_down: one workgroup per 64x64-pixel tile reads the HDR planes
//    once, forms the bright map and its 2x2 means, and builds pyramid levels
//    1..5 of that tile in LDS (a level-1 tile of 32x32 texels halves down to
//    2x2 at level 5), writing every level once.
//  * bloom_blur: all levels in one launch; each workgroup stages a 36x12
//    texel footprint of its 32x8 tile in LDS and applies the separable
//    [1 4 6 4 1] / 16 binomial (clamp to edge) horizontally then vertically.
//  * composite: the footprint of a 32x8 pixel tile on every blurred level
//    (at most 252 texels) is staged in LDS; each thread adds the bilinearly
//    upsampled levels to its pixel, applies exposure, the ACES fit, gamma and
//    8-bit rounding, and writes one 32-bit RGBA word.
//  * pyramid texels are float4, or four halves in the FP16 form.
//  * every stage has a single-view kernel and a batched kernel that walks the
//    work items of many views.
#include "device_common.hpp"
#include "launch.hpp"

namespace epb {

__device__ __forceinline__ float4 add4(float4 a, float4 b) {
    return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, 0.0f);
}
__device__ __forceinline__ float4 scale4(float4 a, float s) { return make_float4(a.x * s, a.y * s, a.z * s, 0.0f); }

// Pyramid texel storage: float4, or four halves (saturating at 65504).
struct alignas(8) Half4 {
    __half x, y, z, w;
};
__device__ __forceinline__ float4 unpack(float4 v) { return v; }
__device__ __forceinline__ float4 unpack(Half4 v) {
    return make_float4(__half2float(v.x), __half2float(v.y), __half2float(v.z), 0.0f);
}
template <typename TP> __device__ __forceinline__ TP pack(float4 v);
template <> __device__ __forceinline__ float4 pack<float4>(float4 v) { return v; }
template <> __device__ __forceinline__ Half4 pack<Half4>(float4 v) {
    Half4 h;
    h.x = __float2half_rn(fminf(v.x, 65504.0f));
    h.y = __float2half_rn(fminf(v.y, 65504.0f));
    h.z = __float2half_rn(fminf(v.z, 65504.0f));
    h.w = __float2half_rn(0.0f);
    return h;
}

// ---------------------------------------------------------------------------
// bloom_down: one 32x32 level-1 tile -> levels 1..5 of that tile
// ---------------------------------------------------------------------------
struct DownLds {
    float4 s1[32][33];
    float4 s2[16][17];
    float4 s3[8][9];
    float4 s4[4][5];
};

// Level L texel (lx, ly) of tile (bx, by) as the mean of its in-range
// children in `src`; kept in `dst` for the next level when that is non-null.
template <int L, int N, typename TP, typename SRC, typename DST>
__device__ __forceinline__ void down_level(const PostDesc &c, int bx, int by, SRC src, DST dst) {
    int t = threadIdx.x;
    if (t >= N * N) return;
    int lx = t % N, ly = t / N;
    int X = bx * N + lx, Y = by * N + ly;
    float4 v = make_float4(0, 0, 0, 0);
    if (X < c.lw[L] && Y < c.lh[L]) {
        float n = 0.0f;
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a)
                if (2 * X + a < c.lw[L - 1] && 2 * Y + b < c.lh[L - 1]) {
                    v = add4(v, src[2 * ly + b][2 * lx + a]);
                    n += 1.0f;
                }
        v = scale4(v, 1.0f / n);
        ((TP *)c.raw[L])[(size_t)Y * c.lw[L] + X] = pack<TP>(v);
    }
    if (dst) dst[ly][lx] = v;
}

template <typename TH, typename TP>
__device__ __forceinline__ void bloom_down_tile(const PostDesc &c, int tile, DownLds &sm) {
    int tiles_x = (c.lw[1] + kDownTile - 1) / kDownTile;
    int by = tile / tiles_x, bx = tile - by * tiles_x;
    int t = threadIdx.x;
    const TH *hdr = (const TH *)c.hdr;
    unsigned plane = (unsigned)c.W * (unsigned)c.H;
    // level 1: bright map averaged over the in-range 2x2 children
    int lx = t % 32;
#pragma unroll
    for (int ly = t / 32; ly < 32; ly += 8) {
        int X = bx * 32 + lx, Y = by * 32 + ly;
        float4 v = make_float4(0, 0, 0, 0);
        if (X < c.lw[1] && Y < c.lh[1]) {
            float n = 0.0f;
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    int px = 2 * X + a, py = 2 * Y + b;
                    if (px < c.W && py < c.H) {
                        unsigned p = __umul24((unsigned)py, (unsigned)c.W) + (unsigned)px;
                        float R = ldf(hdr, p), G = ldf(hdr, plane + p), B = ldf(hdr, 2 * plane + p);
                        float Yl = fmaf(0.2126f, R, fmaf(0.7152f, G, 0.0722f * B));
                        float sc = Yl > 0.0f ? fmaxf(Yl - c.threshold, 0.0f) / Yl : 0.0f;
                        v.x = fmaf(R, sc, v.x);
                        v.y = fmaf(G, sc, v.y);
                        v.z = fmaf(B, sc, v.z);
                        n += 1.0f;
                    }
                }
            v = scale4(v, 1.0f / n);
            ((TP *)c.raw[1])[(size_t)Y * c.lw[1] + X] = pack<TP>(v);
        }
        sm.s1[ly][lx] = v;
    }
    __syncthreads();
    // levels 2..5 inside the tile (the level count is uniform: barriers are safe)
    if (c.nl >= 2) {
        down_level<2, 16, TP>(c, bx, by, sm.s1, sm.s2);
        __syncthreads();
    }
    if (c.nl >= 3) {
        down_level<3, 8, TP>(c, bx, by, sm.s2, sm.s3);
        __syncthreads();
    }
    if (c.nl >= 4) {
        down_level<4, 4, TP>(c, bx, by, sm.s3, sm.s4);
        __syncthreads();
    }
    if (c.nl >= 5) down_level<5, 2, TP>(c, bx, by, sm.s4, (float4(*)[5]) nullptr);
    __syncthreads();  // the next item of a batched launch refills the LDS
}

// ---------------------------------------------------------------------------
// bloom_blur: one 32x8 tile of one level
// ---------------------------------------------------------------------------
struct BlurLds {
    float4 in[12][36];
    float4 h[12][32];
};

template <typename TP>
__device__ __forceinline__ void bloom_blur_item(const PostDesc &c, int item, BlurLds &sm) {
    int L = 1;
    while (L < c.nl && item >= c.blk_start[L + 1]) ++L;
    int local = item - c.blk_start[L];
    int w = c.lw[L], h = c.lh[L];
    int tx = (w + kPostTx - 1) / kPostTx;
    int X0 = (local % tx) * kPostTx, Y0 = (local / tx) * kPostTy;
    const TP *src = (const TP *)c.raw[L];
    int t = threadIdx.x;
    for (int q = t; q < 12 * 36; q += 256) {
        int r = q / 36, cc = q % 36;
        int gy = min(max(Y0 + r - 2, 0), h - 1);
        int gx = min(max(X0 + cc - 2, 0), w - 1);
        sm.in[r][cc] = unpack(src[(size_t)gy * w + gx]);
    }
    __syncthreads();
    for (int q = t; q < 12 * 32; q += 256) {
        int r = q / 32, cc = q % 32;
        float4 a = sm.in[r][cc], bb = sm.in[r][cc + 1], m = sm.in[r][cc + 2], d = sm.in[r][cc + 3],
               e = sm.in[r][cc + 4];
        sm.h[r][cc] = make_float4((a.x + e.x + 4.0f * (bb.x + d.x) + 6.0f * m.x) * 0.0625f,
                                  (a.y + e.y + 4.0f * (bb.y + d.y) + 6.0f * m.y) * 0.0625f,
                                  (a.z + e.z + 4.0f * (bb.z + d.z) + 6.0f * m.z) * 0.0625f, 0.0f);
    }
    __syncthreads();
    int ox = t % 32, oy = t / 32;
    int X = X0 + ox, Y = Y0 + oy;
    if (X < w && Y < h) {
        float4 a = sm.h[oy][ox], bb = sm.h[oy + 1][ox], m = sm.h[oy + 2][ox], d = sm.h[oy + 3][ox],
               e = sm.h[oy + 4][ox];
        ((TP *)c.blur[L])[(size_t)Y * w + X] =
            pack<TP>(make_float4((a.x + e.x + 4.0f * (bb.x + d.x) + 6.0f * m.x) * 0.0625f,
                                 (a.y + e.y + 4.0f * (bb.y + d.y) + 6.0f * m.y) * 0.0625f,
                                 (a.z + e.z + 4.0f * (bb.z + d.z) + 6.0f * m.z) * 0.0625f, 0.0f));
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// composite + tone mapping: one 32x8 pixel tile
// ---------------------------------------------------------------------------
__device__ __forceinline__ float aces(float x) {
    return x * fmaf(2.51f, x, 0.03f) * rcp(fmaf(x, fmaf(2.43f, x, 0.59f), 0.14f));
}
__device__ __forceinline__ uint32_t encode8(float x, float exposure, float inv_gamma) {
    float y = clamp01(aces(exposure * x));
    float g = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(y) * inv_gamma);
    float q = floorf(fmaf(255.0f, g, 0.5f));
    return (uint32_t)fminf(fmaxf(q, 0.0f), 255.0f);
}

// Texel footprint of a 32x8 pixel tile on level l (scale 2^-l): from
// floor((X0 + .5) 2^-l - .5) to floor((X0 + 31.5) 2^-l - .5) + 1, i.e. at most
// 32 / 2^l + 2 columns and 8 / 2^l + 2 rows (+1 for rounding).
constexpr int kCompLds = (19 * 7) + (11 * 5) + (7 * 4) + (5 * 4) + (4 * 4);

template <typename TH, typename TP>
__device__ __forceinline__ void composite_tile(const PostDesc &c, int tile, float4 *sb) {
    int tiles_x = (c.W + kPostTx - 1) / kPostTx;
    int ty = tile / tiles_x;
    int X0 = (tile - ty * tiles_x) * kPostTx, Y0 = ty * kPostTy;
    int x = X0 + (int)(threadIdx.x % kPostTx);
    int y = Y0 + (int)(threadIdx.x / kPostTx);
    bool live = x < c.W && y < c.H;
    unsigned p = live ? __umul24((unsigned)y, (unsigned)c.W) + (unsigned)x : 0u;
    unsigned plane = (unsigned)c.W * (unsigned)c.H;
    const TH *hdr = (const TH *)c.hdr;
    // the pixel's HDR first (in flight while the pyramid footprint is staged)
    float R0 = ldf(hdr, p), G0 = ldf(hdr, plane + p), B0 = ldf(hdr, 2 * plane + p);
    // stage the clamped footprint of every blurred level; a footprint is at
    // most 19 x 7 texels, one texel per thread (row = thread / 32, col = thread % 32)
    int base[EPB_MAX_BLOOM_LEVELS], sx0[EPB_MAX_BLOOM_LEVELS], sy0[EPB_MAX_BLOOM_LEVELS],
        cols[EPB_MAX_BLOOM_LEVELS];
    int off = 0;
    int tr = threadIdx.x / 32, tc = threadIdx.x % 32;
#pragma unroll
    for (int L = 1; L < EPB_MAX_BLOOM_LEVELS; ++L) {
        if (L > c.nl) break;
        const float sc = 1.0f / (float)(1 << L);
        int w = c.lw[L], h = c.lh[L];
        int ax = (int)floorf(fmaf((float)X0 + 0.5f, sc, -0.5f));
        int ay = (int)floorf(fmaf((float)Y0 + 0.5f, sc, -0.5f));
        int bx = (int)floorf(fmaf((float)X0 + 31.5f, sc, -0.5f)) + 1;
        int by = (int)floorf(fmaf((float)Y0 + 7.5f, sc, -0.5f)) + 1;
        int nc = bx - ax + 1, nr = by - ay + 1;
        if (tc < nc && tr < nr) {
            int gx = min(max(ax + tc, 0), w - 1), gy = min(max(ay + tr, 0), h - 1);
            sb[off + tr * nc + tc] = unpack(((const TP *)c.blur[L])[(size_t)gy * w + gx]);
        }
        base[L] = off;
        sx0[L] = ax;
        sy0[L] = ay;
        cols[L] = nc;
        off += nc * nr;
    }
    __syncthreads();
    if (live) {
        float sx = 0.0f, sy = 0.0f, sz = 0.0f;
#pragma unroll
        for (int L = 1; L < EPB_MAX_BLOOM_LEVELS; ++L) {
            if (L > c.nl) break;
            const float sc = 1.0f / (float)(1 << L);
            float fx = fmaf((float)x + 0.5f, sc, -0.5f), fy = fmaf((float)y + 0.5f, sc, -0.5f);
            float x0f = floorf(fx), y0f = floorf(fy);
            float wx = fx - x0f, wy = fy - y0f;
            int lx = (int)x0f - sx0[L], ly = (int)y0f - sy0[L];
            const float4 *r0 = sb + base[L] + ly * cols[L] + lx;
            const float4 *r1 = r0 + cols[L];
            float4 v = lerp4(lerp4(r0[0], r0[1], wx), lerp4(r1[0], r1[1], wx), wy);
            sx += v.x;
            sy += v.y;
            sz += v.z;
        }
        float R = fmaf(c.strength, sx, R0);
        float G = fmaf(c.strength, sy, G0);
        float Bc = fmaf(c.strength, sz, B0);
        uint32_t word = encode8(R, c.exposure, c.inv_gamma) | (encode8(G, c.exposure, c.inv_gamma) << 8) |
                        (encode8(Bc, c.exposure, c.inv_gamma) << 16) | (255u << 24);
        sto(c.ldr, p * 4u, word);
    }
    __syncthreads();  // the next item of a batched launch refills the LDS
}

// ---------------------------------------------------------------------------
// kernels: single view (XCD-aware tile order) and batched (persistent range)
// ---------------------------------------------------------------------------
template <typename TH, typename TP>
__global__ void __launch_bounds__(256) k_bloom_down(const PostDesc c, int tiles) {
    __shared__ DownLds sm;
    bloom_down_tile<TH, TP>(c, xcd_tile(blockIdx.x, tiles), sm);
}

template <typename TP>
__global__ void __launch_bounds__(256) k_bloom_blur(const PostDesc c) {
    __shared__ BlurLds sm;
    bloom_blur_item<TP>(c, blockIdx.x, sm);
}

template <typename TH, typename TP>
__global__ void __launch_bounds__(256) k_composite(const PostDesc c, int tiles) {
    __shared__ float4 sb[kCompLds];
    composite_tile<TH, TP>(c, xcd_tile(blockIdx.x, tiles), sb);
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
__global__ void __launch_bounds__(256) k_composite_batch(const void *__restrict__ table) {
    __shared__ float4 sb[kCompLds];
    const BatchHeader *h = (const BatchHeader *)table;
    const int *start = batch_start(table, kStComposite);
    const ViewDesc *views = batch_views(table);
    XcdRange w = xcd_range(h->total[kStComposite]);
    for (int it = w.lb; it < w.count; it += w.stride) {
        int g = w.first + it;
        int v = find_view(start, h->n_views, g);
        composite_tile<TH, TP>(views[v].post, g - start[v], sb);
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
                   float gamma, uint8_t *ldr, void *scratch) {
    PostDesc c{};
    c.W = q.W;
    c.H = q.H;
    c.nl = q.levels - 1;
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
        nb += ceil_div(c.lw[l], kPostTx) * ceil_div(c.lh[l], kPostTy);
    }
    c.blk_start[c.nl + 1] = nb;
    c.threshold = threshold;
    c.strength = strength;
    c.exposure = exposure;
    c.inv_gamma = 1.0f / gamma;
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
static void launch_post(const PostDesc &c, hipStream_t s) {
    if (c.nl >= 1) {
        int tiles = post_items(c, kStDown);
        hipLaunchKernelGGL((k_bloom_down<TH, TP>), dim3(tiles), dim3(256), 0, s, c, tiles);
        hipLaunchKernelGGL(k_bloom_blur<TP>, dim3(post_items(c, kStBloomBlur)), dim3(256), 0, s, c);
    }
    int tiles = post_items(c, kStComposite);
    hipLaunchKernelGGL((k_composite<TH, TP>), dim3(tiles), dim3(256), 0, s, c, tiles);
}

template <typename TH, typename TP>
static void launch_post_batch_t(const BatchHeader &h, const void *table, hipStream_t s) {
    if (h.total[kStDown] > 0)
        hipLaunchKernelGGL((k_bloom_down_batch<TH, TP>), dim3(batch_grid(h.total[kStDown], h.blocks_per_cu)),
                           dim3(256), 0, s, table);
    if (h.total[kStBloomBlur] > 0)
        hipLaunchKernelGGL(k_bloom_blur_batch<TP>, dim3(batch_grid(h.total[kStBloomBlur], h.blocks_per_cu)),
                           dim3(256), 0, s, table);
    hipLaunchKernelGGL((k_composite_batch<TH, TP>), dim3(batch_grid(h.total[kStComposite], h.blocks_per_cu)),
                       dim3(256), 0, s, table);
}

hipError_t launch_bloom_tonemap(const PostDesc &c, epb_dtype hdr_dtype, epb_dtype pyr_dtype, hipStream_t s) {
    bool h16 = hdr_dtype == EPB_F16, p16 = pyr_dtype == EPB_F16;
    if (!h16 && !p16) launch_post<float, float4>(c, s);
    else if (!h16 && p16) launch_post<float, Half4>(c, s);
    else if (h16 && !p16) launch_post<__half, float4>(c, s);
    else launch_post<__half, Half4>(c, s);
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
