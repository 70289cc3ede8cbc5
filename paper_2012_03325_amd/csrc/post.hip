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
//  * composite: the footprint of a 32x8 pixel tile on every blurred level
//    (at most 252 texels) is staged in LDS and interpolated separably (rows
//    at the tile's columns, then per pixel between two rows); each thread adds
//    the upsampled levels to its pixel, applies exposure, the ACES fit, gamma
//    and 8-bit rounding, and writes one 32-bit RGBA word.
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
// bloom_down: one 16x16 level-1 tile (32x32 pixels) -> levels 1..5 of that tile
// ---------------------------------------------------------------------------
struct DownLds {
    float4 s1[16][17];
    float4 s2[8][9];
    float4 s3[4][5];
    float4 s4[2][3];
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
    // level 1, one texel per thread: the bright map averaged over its in-range 2x2 children
    int lx = t % kDownTile, ly = t / kDownTile;
    int X = bx * kDownTile + lx, Y = by * kDownTile + ly;
    float4 v = make_float4(0, 0, 0, 0);
    if (X < c.lw[1] && Y < c.lh[1]) {
        float R[4], G[4], B[4];
        bool in[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {  // all twelve loads in flight together
            int px = 2 * X + (k & 1), py = 2 * Y + (k >> 1);
            in[k] = px < c.W && py < c.H;
            unsigned p = in[k] ? __umul24((unsigned)py, (unsigned)c.W) + (unsigned)px : 0u;
            R[k] = ldf(hdr, p);
            G[k] = ldf(hdr, plane + p);
            B[k] = ldf(hdr, 2 * plane + p);
        }
        float n = 0.0f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (!in[k]) continue;
            float Yl = fmaf(0.2126f, R[k], fmaf(0.7152f, G[k], 0.0722f * B[k]));
            float sc = Yl > 0.0f ? fmaxf(Yl - c.threshold, 0.0f) / Yl : 0.0f;
            v.x = fmaf(R[k], sc, v.x);
            v.y = fmaf(G[k], sc, v.y);
            v.z = fmaf(B[k], sc, v.z);
            n += 1.0f;
        }
        v = scale4(v, 1.0f / n);
        ((TP *)c.raw[1])[(size_t)Y * c.lw[1] + X] = pack<TP>(v);
    }
    sm.s1[ly][lx] = v;
    __syncthreads();
    // levels 2..5 inside the tile (the level count is uniform: barriers are safe)
    if (c.nl >= 2) {
        down_level<2, 8, TP>(c, bx, by, sm.s1, sm.s2);
        __syncthreads();
    }
    if (c.nl >= 3) {
        down_level<3, 4, TP>(c, bx, by, sm.s2, sm.s3);
        __syncthreads();
    }
    if (c.nl >= 4) {
        down_level<4, 2, TP>(c, bx, by, sm.s3, sm.s4);
        __syncthreads();
    }
    if (c.nl >= 5) down_level<5, 1, TP>(c, bx, by, sm.s4, (float4(*)[3]) nullptr);
    __syncthreads();  // the next item of a batched launch refills the LDS
}

// ---------------------------------------------------------------------------
// bloom_blur: one 32x16 tile of one level
// ---------------------------------------------------------------------------
struct Rgb {
    float x, y, z;
};
constexpr int kBbW = kBloomTx + 4, kBbH = kBloomTy + 4;  // footprint with the 2-texel halo
struct BlurLds {
    Rgb in[kBbH][kBbW];
    Rgb h[kBbH][kBloomTx];
};

__device__ __forceinline__ Rgb binomial5(Rgb a, Rgb b, Rgb m, Rgb d, Rgb e) {
    return Rgb{(a.x + e.x + 4.0f * (b.x + d.x) + 6.0f * m.x) * 0.0625f,
               (a.y + e.y + 4.0f * (b.y + d.y) + 6.0f * m.y) * 0.0625f,
               (a.z + e.z + 4.0f * (b.z + d.z) + 6.0f * m.z) * 0.0625f};
}

template <typename TP>
__device__ __forceinline__ void bloom_blur_item(const PostDesc &c, int item, BlurLds &sm) {
    int L = 1;
    while (L < c.nl && item >= c.blk_start[L + 1]) ++L;
    int local = item - c.blk_start[L];
    int w = c.lw[L], h = c.lh[L];
    int tx = (w + kBloomTx - 1) / kBloomTx;
    int ty = local / tx;
    int X0 = (local - ty * tx) * kBloomTx, Y0 = ty * kBloomTy;
    const TP *src = (const TP *)c.raw[L];
    int t = threadIdx.x;
    for (int q = t; q < kBbH * kBbW; q += 256) {  // every load of the footprint in flight together
        int r = q / kBbW, cc = q - r * kBbW;
        int gy = min(max(Y0 + r - 2, 0), h - 1);
        int gx = min(max(X0 + cc - 2, 0), w - 1);
        float4 v = unpack(ldo(src, (__umul24((unsigned)gy, (unsigned)w) + (unsigned)gx) * (unsigned)sizeof(TP)));
        sm.in[r][cc] = Rgb{v.x, v.y, v.z};
    }
    __syncthreads();
    for (int q = t; q < kBbH * kBloomTx; q += 256) {
        int r = q / kBloomTx, cc = q % kBloomTx;
        sm.h[r][cc] = binomial5(sm.in[r][cc], sm.in[r][cc + 1], sm.in[r][cc + 2], sm.in[r][cc + 3], sm.in[r][cc + 4]);
    }
    __syncthreads();
    for (int q = t; q < kBloomTy * kBloomTx; q += 256) {
        int oy = q / kBloomTx, ox = q % kBloomTx;
        int X = X0 + ox, Y = Y0 + oy;
        if (X < w && Y < h) {
            Rgb v = binomial5(sm.h[oy][ox], sm.h[oy + 1][ox], sm.h[oy + 2][ox], sm.h[oy + 3][ox], sm.h[oy + 4][ox]);
            ((TP *)c.blur[L])[(size_t)Y * w + X] = pack<TP>(make_float4(v.x, v.y, v.z, 0.0f));
        }
    }
    __syncthreads();  // the next item of a batched launch refills the LDS
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

// Level l samples pixel x at (x + 1/2) 2^-l - 1/2 = v / 2^(l+1) with v = 2x + 1 - 2^l:
// the texel is v >> (l+1) (an arithmetic shift floors) and the weight is the
// remainder (v & (2^(l+1) - 1)) / 2^(l+1), exact in float -- the same numbers as
// the float form, without floor or conversions.  A 32x8 pixel tile reads at
// most 32 / 2^l + 2 columns and 8 / 2^l + 2 rows of level l (+1 for rounding).
// The bilinear upsampling is done separably: every footprint row is first
// interpolated at the tile's 32 pixel columns (one item per thread and level,
// as a footprint has at most 7 rows), then each pixel interpolates its two rows
// -- the same two-step lerp per pixel, with the horizontal steps shared by the
// pixels of a column.
constexpr int kCompLds = (19 * 7) + (11 * 5) + (7 * 4) + (5 * 4) + (4 * 4);
constexpr int kCompRows = 7 + 5 + 4 + 4 + 4;
struct CompLds {
    float4 tex[kCompLds];            // level footprints
    float4 row[kCompRows][kPostTx];  // footprint rows interpolated at the tile's columns
};

template <typename TH, typename TP>
__device__ __forceinline__ void composite_tile(const PostDesc &c, int tile, CompLds &sm) {
    int tiles_x = (c.W + kPostTx - 1) / kPostTx;
    int ty = tile / tiles_x;
    int X0 = (tile - ty * tiles_x) * kPostTx, Y0 = ty * kPostTy;
    int tc = (int)(threadIdx.x % kPostTx), tr = (int)(threadIdx.x / kPostTx);
    int x = X0 + tc, y = Y0 + tr;
    bool live = x < c.W && y < c.H;
    unsigned p = live ? __umul24((unsigned)y, (unsigned)c.W) + (unsigned)x : 0u;
    unsigned plane = (unsigned)c.W * (unsigned)c.H;
    const TH *hdr = (const TH *)c.hdr;
    // the pixel's HDR first (in flight while the pyramid footprint is staged)
    float R0 = ldf(hdr, p), G0 = ldf(hdr, plane + p), B0 = ldf(hdr, 2 * plane + p);
    // stage the clamped footprint of every blurred level, one texel per thread
    int base[EPB_MAX_BLOOM_LEVELS], rbase[EPB_MAX_BLOOM_LEVELS], ax[EPB_MAX_BLOOM_LEVELS],
        ay[EPB_MAX_BLOOM_LEVELS], cols[EPB_MAX_BLOOM_LEVELS], rows[EPB_MAX_BLOOM_LEVELS];
    int off = 0, roff = 0;
#pragma unroll
    for (int L = 1; L < EPB_MAX_BLOOM_LEVELS; ++L) {
        if (L > c.nl) break;
        const int sh = L + 1, o = 1 - (1 << L);
        int w = c.lw[L], h = c.lh[L];
        ax[L] = (2 * X0 + o) >> sh;
        ay[L] = (2 * Y0 + o) >> sh;
        int nc = ((2 * (X0 + kPostTx - 1) + o) >> sh) + 2 - ax[L];
        int nr = ((2 * (Y0 + kPostTy - 1) + o) >> sh) + 2 - ay[L];
        if (tc < nc && tr < nr) {
            int gx = min(max(ax[L] + tc, 0), w - 1), gy = min(max(ay[L] + tr, 0), h - 1);
            unsigned t = __umul24((unsigned)gy, (unsigned)w) + (unsigned)gx;
            sm.tex[off + __mul24(tr, nc) + tc] = unpack(ldo((const TP *)c.blur[L], t * (unsigned)sizeof(TP)));
        }
        base[L] = off;
        rbase[L] = roff;
        cols[L] = nc;
        rows[L] = nr;
        off += nc * nr;
        roff += nr;
    }
    __syncthreads();
    // horizontal step: footprint row tr of each level at this thread's column
#pragma unroll
    for (int L = 1; L < EPB_MAX_BLOOM_LEVELS; ++L) {
        if (L > c.nl) break;
        if (tr < rows[L]) {
            const int sh = L + 1, o = 1 - (1 << L), m = (1 << sh) - 1;
            const float inv = 1.0f / (float)(1 << sh);
            int vx = 2 * x + o;
            float wx = (float)(vx & m) * inv;
            const float4 *t0 = sm.tex + base[L] + __mul24(tr, cols[L]) + ((vx >> sh) - ax[L]);
            sm.row[rbase[L] + tr][tc] = lerp4(t0[0], t0[1], wx);
        }
    }
    __syncthreads();
    if (live) {
        float sx = 0.0f, sy = 0.0f, sz = 0.0f;
#pragma unroll
        for (int L = 1; L < EPB_MAX_BLOOM_LEVELS; ++L) {
            if (L > c.nl) break;
            const int sh = L + 1, o = 1 - (1 << L), m = (1 << sh) - 1;
            const float inv = 1.0f / (float)(1 << sh);
            int vy = 2 * y + o;
            float wy = (float)(vy & m) * inv;
            int r0 = rbase[L] + ((vy >> sh) - ay[L]);
            float4 v = lerp4(sm.row[r0][tc], sm.row[r0 + 1][tc], wy);
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
    __shared__ CompLds sm;
    composite_tile<TH, TP>(c, xcd_tile(blockIdx.x, tiles), sm);
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
    __shared__ CompLds sm;
    const BatchHeader *h = (const BatchHeader *)table;
    const int *start = batch_start(table, kStComposite);
    const ViewDesc *views = batch_views(table);
    XcdRange w = xcd_range(h->total[kStComposite]);
    for (int it = w.lb; it < w.count; it += w.stride) {
        int g = w.first + it;
        int v = find_view(start, h->n_views, g);
        composite_tile<TH, TP>(views[v].post, g - start[v], sm);
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
        nb += ceil_div(c.lw[l], kBloomTx) * ceil_div(c.lh[l], kBloomTy);
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
