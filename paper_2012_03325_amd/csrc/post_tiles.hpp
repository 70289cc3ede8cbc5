// Per-tile device functions of bloom and compositing (paper Sec. 5.3, 5.4);
// shared by the single-view, batched and persistent kernels.
#pragma once

#include "device_common.hpp"

namespace epb {

__device__ __forceinline__ float4 add4(float4 a, float4 b) {
    return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, 0.0f);
}
__device__ __forceinline__ float4 scale4(float4 a, float s) { return make_float4(a.x * s, a.y * s, a.z * s, 0.0f); }

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
        // child (2X, 2Y) is always in range (each level is the previous one halved,
        // rounded up); 1 / n for n = 1, 2 or 4 children is a product of halves, exact
        bool x1 = 2 * X + 1 < c.lw[L - 1], y1 = 2 * Y + 1 < c.lh[L - 1];
        v = add4(v, src[2 * ly][2 * lx]);
        if (x1) v = add4(v, src[2 * ly][2 * lx + 1]);
        if (y1) v = add4(v, src[2 * ly + 1][2 * lx]);
        if (x1 && y1) v = add4(v, src[2 * ly + 1][2 * lx + 1]);
        v = scale4(v, (x1 ? 0.5f : 1.0f) * (y1 ? 0.5f : 1.0f));
        sto((TP *)c.raw[L], (unsigned)(Y * c.lw[L] + X) * (unsigned)sizeof(TP), pack<TP>(v));
    }
    if (dst) dst[ly][lx] = v;
}

// Levels 2..5 of tile (bx, by) from its level-1 texels in sm.s1 (the level
// count is uniform: barriers are safe).
template <typename TP>
__device__ __forceinline__ void down_levels_2_to_5(const PostDesc &c, int bx, int by, DownLds &sm) {
    __syncthreads();
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

// Two horizontally adjacent pixels of a plane (index p even, so the pair is
// 8-byte aligned in float32 and 4-byte aligned in half): one load.
__device__ __forceinline__ void ld_pair(const float *b, unsigned p, float &u, float &v) {
    float2 q = ldo((const float2 *)b, p * 4u);
    u = q.x;
    v = q.y;
}
struct alignas(4) HalfPair {
    __half a, b;
};
__device__ __forceinline__ void ld_pair(const __half *b, unsigned p, float &u, float &v) {
    HalfPair q = ldo((const HalfPair *)b, p * 2u);
    u = __half2float(q.a);
    v = __half2float(q.b);
}

template <typename TH, typename TP>
__device__ __forceinline__ void bloom_down_tile(const PostDesc &c, int tile, DownLds &sm) {
    int tiles_x = (c.lw[1] + kDownTile - 1) / kDownTile;
    int by = tile / tiles_x, bx = tile - by * tiles_x;
    int t = threadIdx.x;
    const TH *hdr = (const TH *)c.hdr;
    unsigned plane = (unsigned)c.W * (unsigned)c.H;
    // level 1, one texel per thread: the bright map averaged over its in-range 2x2
    // children, summed as horizontal pairs and then the two rows (the order the
    // fused shading epilogue uses)
    int lx = t % kDownTile, ly = t / kDownTile;
    int X = bx * kDownTile + lx, Y = by * kDownTile + ly;
    float4 v = make_float4(0, 0, 0, 0);
    if (X < c.lw[1] && Y < c.lh[1]) {
        float R[4], G[4], B[4];
        bool in[4];
        if (!(c.W & 1)) {  // even width: a row's two children are one pair (six loads in flight)
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                int py = 2 * Y + r;
                in[2 * r] = in[2 * r + 1] = py < c.H;
                unsigned p = in[2 * r] ? __umul24((unsigned)py, (unsigned)c.W) + (unsigned)(2 * X) : 0u;
                ld_pair(hdr, p, R[2 * r], R[2 * r + 1]);
                ld_pair(hdr, plane + p, G[2 * r], G[2 * r + 1]);
                ld_pair(hdr, 2 * plane + p, B[2 * r], B[2 * r + 1]);
            }
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) {  // all twelve loads in flight together
                int px = 2 * X + (k & 1), py = 2 * Y + (k >> 1);
                in[k] = px < c.W && py < c.H;
                unsigned p = in[k] ? __umul24((unsigned)py, (unsigned)c.W) + (unsigned)px : 0u;
                R[k] = ldf(hdr, p);
                G[k] = ldf(hdr, plane + p);
                B[k] = ldf(hdr, 2 * plane + p);
            }
        }
        float cr[4], cg[4], cb[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {  // an out-of-image child adds an exact zero
            float sc = bright_scale(R[k], G[k], B[k], c.threshold);
            cr[k] = in[k] ? R[k] * sc : 0.0f;
            cg[k] = in[k] ? G[k] * sc : 0.0f;
            cb[k] = in[k] ? B[k] * sc : 0.0f;
        }
        float inv_n = (in[1] ? 0.5f : 1.0f) * (in[2] ? 0.5f : 1.0f);
        v = make_float4(((cr[0] + cr[1]) + (cr[2] + cr[3])) * inv_n, ((cg[0] + cg[1]) + (cg[2] + cg[3])) * inv_n,
                        ((cb[0] + cb[1]) + (cb[2] + cb[3])) * inv_n, 0.0f);
        TP st = pack<TP>(v);
        sto((TP *)c.raw[1], (unsigned)(Y * c.lw[1] + X) * (unsigned)sizeof(TP), st);
        v = unpack(st);  // the next levels average what level 1 holds
    }
    sm.s1[ly][lx] = v;
    down_levels_2_to_5<TP>(c, bx, by, sm);
}

// Levels 2..5 when the shading pass has written level 1 (the fused form).
template <typename TP>
__device__ __forceinline__ void bloom_down_from1_tile(const PostDesc &c, int tile, DownLds &sm) {
    int tiles_x = (c.lw[1] + kDownTile - 1) / kDownTile;
    int by = tile / tiles_x, bx = tile - by * tiles_x;
    int t = threadIdx.x;
    int lx = t % kDownTile, ly = t / kDownTile;
    int X = bx * kDownTile + lx, Y = by * kDownTile + ly;
    float4 v = make_float4(0, 0, 0, 0);
    if (X < c.lw[1] && Y < c.lh[1])
        v = unpack(ldo((const TP *)c.raw[1], (unsigned)(Y * c.lw[1] + X) * (unsigned)sizeof(TP)));
    sm.s1[ly][lx] = v;
    down_levels_2_to_5<TP>(c, bx, by, sm);
}

// ---------------------------------------------------------------------------
// bloom_blur: one 32x16 tile of one level
// ---------------------------------------------------------------------------
struct Rgb {
    float x, y, z;
};
constexpr int kBbW = kBloomTx + 4, kBbH = kBloomTy + 4;  // footprint with the 2-texel halo
constexpr int kBbLdsRows = ((kBbH * kBbW + 255) / 256 * 256 + kBbW - 1) / kBbW;  // padding for whole rounds
struct BlurLds {
    Rgb in[kBbLdsRows][kBbW];
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
    // every load of the footprint in flight together: all issued before the first LDS store
    constexpr int kN = kBbH * kBbW, kIt = (kN + 255) / 256;
    TP v[kIt];
#pragma unroll
    for (int i = 0; i < kIt; ++i) {
        int q = min(t + 256 * i, kN - 1);  // clamped: every lane issues every load
        int r = q / kBbW, cc = q - r * kBbW;
        int gy = min(max(Y0 + r - 2, 0), h - 1);
        int gx = min(max(X0 + cc - 2, 0), w - 1);
        v[i] = ldo(src, (__umul24((unsigned)gy, (unsigned)w) + (unsigned)gx) * (unsigned)sizeof(TP));
    }
#pragma unroll
    for (int i = 0; i < kIt; ++i) {  // unconditional: entries past the footprint land in the padding rows
        float4 f = unpack(v[i]);
        (&sm.in[0][0])[t + 256 * i] = Rgb{f.x, f.y, f.z};
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
            sto((TP *)c.blur[L], (unsigned)(Y * w + X) * (unsigned)sizeof(TP), pack<TP>(make_float4(v.x, v.y, v.z, 0.0f)));
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
// Reinhard's global operator on each channel (the paper's alternative curve).
__device__ __forceinline__ float reinhard(float x) { return x * rcp(1.0f + x); }
template <bool kReinhard>
__device__ __forceinline__ uint32_t encode8(float x, float exposure, float inv_gamma) {
    float e = exposure * x;
    float y = clamp01(kReinhard ? reinhard(e) : aces(e));
    float g = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(y) * inv_gamma);
    float q = floorf(fmaf(255.0f, g, 0.5f));
    return (uint32_t)fminf(fmaxf(q, 0.0f), 255.0f);
}

// Level L samples pixel x at (x + 1/2) 2^-L - 1/2 = v / 2^(L+1) with v = 2x + 1 - 2^L:
// the texel is v >> (L+1) (an arithmetic shift floors) and the weight is the
// remainder (v & (2^(L+1) - 1)) / 2^(L+1), exact in float -- the same numbers as
// the float form, without floor or conversions.
//
// A thread owns one pixel column of an 8-row strip (the strip starts at a
// multiple of 8).  For each blurred level it first interpolates, at its column,
// the level rows under the strip (6, 4, 3, 2, 2 rows for levels 1..5: two texel
// loads per row, neighbouring lanes share cache lines), then every pixel of
// the column interpolates between two of those rows.  Because the strip starts
// at a multiple of 8, which rows a pixel uses is fixed at compile time (levels
// 1..3), or is the first pair for all eight pixels (levels 4 and 5, where the
// strip lies inside one texel row pair and the remainder grows by 2 per pixel
// without wrapping); the weights of levels 1..3 are compile-time constants as
// well.  Everything stays in registers: no LDS, no barriers, and the strip's
// 24 HDR loads are in flight while the pyramid is read.
template <int L>
struct LevelRows {
    static constexpr int sh = L + 1, o = 1 - (1 << L), m = (1 << sh) - 1;
    static constexpr int n = L == 1 ? 6 : L == 2 ? 4 : L == 3 ? 3 : 2;
    static constexpr float inv = 1.0f / (float)(1 << sh);
    // first row (relative to the strip's first footprint row) of pixel j
    static constexpr int rel(int j) { return L <= 3 ? ((2 * j + o) >> sh) - (o >> sh) : 0; }
    // weight of pixel j (levels 1..3)
    static constexpr float wy(int j) { return (float)((2 * j + o) & m) * inv; }
};

// The level-L rows under the strip, interpolated at the thread's column.
template <int L, typename TP>
__device__ __forceinline__ void level_rows(const PostDesc &c, int x, int Y0, float (&rows)[LevelRows<L>::n][3]) {
    using LR = LevelRows<L>;
    const int w = c.lw[L], h = c.lh[L];
    const TP *lvl = (const TP *)c.blur[L];
    int vx = 2 * x + LR::o;
    float wx = (float)(vx & LR::m) * LR::inv;
    int cx = vx >> LR::sh;
    unsigned c0 = (unsigned)min(max(cx, 0), w - 1), c1 = (unsigned)min(max(cx + 1, 0), w - 1);
    int ay = (2 * Y0 + LR::o) >> LR::sh;
    // all the level's texel loads issued before any is used (one memory round trip per level)
    TP ta[LR::n], tb[LR::n];
#pragma unroll
    for (int r = 0; r < LR::n; ++r) {
        unsigned gy = (unsigned)min(max(ay + r, 0), h - 1);
        unsigned base = __umul24(gy, (unsigned)w);
        ta[r] = ldo(lvl, (base + c0) * (unsigned)sizeof(TP));
        tb[r] = ldo(lvl, (base + c1) * (unsigned)sizeof(TP));
    }
    __builtin_amdgcn_sched_barrier(0);  // keep the scheduler from interleaving the loads with their uses
#pragma unroll
    for (int r = 0; r < LR::n; ++r) {
        float4 a = unpack(ta[r]), b = unpack(tb[r]);
        rows[r][0] = fmaf(wx, b.x - a.x, a.x);
        rows[r][1] = fmaf(wx, b.y - a.y, a.y);
        rows[r][2] = fmaf(wx, b.z - a.z, a.z);
    }
}

// Levels 4 and 5, which start the strip's sums: each pixel of the strip adds
// a_L + w_L(j) (b_L - a_L) for the one row pair (a_L, b_L) under the strip, with
// w_L(j) = w_L(0) + 2 j / 2^(L+1); the two a_L are summed once per thread and
// enter as the first addend, so a pixel spends one FMA per level and channel.
// Absent levels contribute nothing (their difference and weight are 0).
template <typename TP>
__device__ __forceinline__ void init_coarse(const PostDesc &c, int x, int Y0, float (&acc)[kPostTy][3]) {
    float base[3] = {0.0f, 0.0f, 0.0f}, d4[3] = {0.0f, 0.0f, 0.0f}, d5[3] = {0.0f, 0.0f, 0.0f};
    float w4 = 0.0f, w5 = 0.0f;
    if (c.nl >= 4) {
        float rows[2][3];
        level_rows<4, TP>(c, x, Y0, rows);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            base[ch] = rows[0][ch];
            d4[ch] = rows[1][ch] - rows[0][ch];
        }
        w4 = (float)((2 * Y0 + LevelRows<4>::o) & LevelRows<4>::m) * LevelRows<4>::inv;
    }
    if (c.nl >= 5) {
        float rows[2][3];
        level_rows<5, TP>(c, x, Y0, rows);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            base[ch] += rows[0][ch];
            d5[ch] = rows[1][ch] - rows[0][ch];
        }
        w5 = (float)((2 * Y0 + LevelRows<5>::o) & LevelRows<5>::m) * LevelRows<5>::inv;
    }
#pragma unroll
    for (int j = 0; j < kPostTy; ++j) {
        float wj4 = w4 + (float)(2 * j) * LevelRows<4>::inv, wj5 = w5 + (float)(2 * j) * LevelRows<5>::inv;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) acc[j][ch] = fmaf(wj5, d5[ch], fmaf(wj4, d4[ch], base[ch]));
    }
}

// Levels 1..3: (1 - w) a + w b for the pixel's row pair, two FMAs per channel.
template <int L, typename TP>
__device__ __forceinline__ void add_fine(const PostDesc &c, int x, int Y0, float (&acc)[kPostTy][3]) {
    using LR = LevelRows<L>;
    float rows[LR::n][3];
    level_rows<L, TP>(c, x, Y0, rows);
#pragma unroll
    for (int j = 0; j < kPostTy; ++j) {
        const int r0 = LR::rel(j);
        const float w = LR::wy(j);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) acc[j][ch] = fmaf(w, rows[r0 + 1][ch], fmaf(1.0f - w, rows[r0][ch], acc[j][ch]));
    }
}

// Bloom added to the strip's HDR, tone mapped and stored as RGBA8.
template <bool kReinhard>
__device__ __forceinline__ void store_strip(const PostDesc &c, int x, int Y0, const float (&px)[kPostTy][3],
                                            const float (&acc)[kPostTy][3]) {
#pragma unroll
    for (int j = 0; j < kPostTy; ++j) {
        if (Y0 + j >= c.H) break;
        float R = fmaf(c.strength, acc[j][0], px[j][0]);
        float G = fmaf(c.strength, acc[j][1], px[j][1]);
        float Bc = fmaf(c.strength, acc[j][2], px[j][2]);
        uint32_t word = encode8<kReinhard>(R, c.exposure, c.inv_gamma) |
                        (encode8<kReinhard>(G, c.exposure, c.inv_gamma) << 8) |
                        (encode8<kReinhard>(Bc, c.exposure, c.inv_gamma) << 16) | (255u << 24);
        unsigned p = __umul24((unsigned)(Y0 + j), (unsigned)c.W) + (unsigned)x;
        sto(c.ldr, p * 4u, word);
    }
}

// One 64 x 8 tile by one wavefront; `lane` is the thread's lane (its column).
template <typename TH, typename TP>
__device__ __forceinline__ void composite_tile(const PostDesc &c, int tile, int lane) {
    int tiles_x = (c.W + kPostTx - 1) / kPostTx;
    int ty = tile / tiles_x;
    int x = (tile - ty * tiles_x) * kPostTx + lane, Y0 = ty * kPostTy;
    if (x >= c.W) return;
    unsigned plane = (unsigned)c.W * (unsigned)c.H;
    const TH *hdr = (const TH *)c.hdr;
    // the strip's HDR first (in flight while the pyramid is read); rows below the image are
    // clamped to the last row and not stored
    float px[kPostTy][3];
#pragma unroll
    for (int j = 0; j < kPostTy; ++j) {
        unsigned p = __umul24((unsigned)min(Y0 + j, c.H - 1), (unsigned)c.W) + (unsigned)x;
        px[j][0] = ldf(hdr, p);
        px[j][1] = ldf(hdr, plane + p);
        px[j][2] = ldf(hdr, 2 * plane + p);
    }
    // the bloom sum of levels 5, 4 (one row pair for the whole strip), then 1 .. 3
    // (nl is uniform)
    float acc[kPostTy][3];
    init_coarse<TP>(c, x, Y0, acc);
    if (c.nl >= 1) add_fine<1, TP>(c, x, Y0, acc);
    if (c.nl >= 2) add_fine<2, TP>(c, x, Y0, acc);
    if (c.nl >= 3) add_fine<3, TP>(c, x, Y0, acc);
    if (c.tonemap == EPB_TONEMAP_REINHARD) store_strip<true>(c, x, Y0, px, acc);
    else store_strip<false>(c, x, Y0, px, acc);
}

}  // namespace epb
