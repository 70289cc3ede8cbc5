// Bloom (paper Sec. 5.3) and final compositing with ACES tone mapping and
// gamma correction (Sec. 5.4).
//
// gfx950 mapping:
//  * k_bloom_down: one workgroup per 64x64-pixel tile reads the HDR planes
//    once, forms the bright map and its 2x2 means, and builds pyramid levels
//    1..5 of that tile in LDS (a level-1 tile of 32x32 texels halves down to
//    2x2 at level 5), writing every level once.
//  * k_bloom_blur: all levels in one launch; each workgroup stages a 36x12
//    texel footprint of its 32x8 tile in LDS and applies the separable
//    [1 4 6 4 1] / 16 binomial (clamp to edge) horizontally then vertically.
//  * k_composite: one thread per pixel adds the bilinearly upsampled blurred
//    levels (float4 texels, L2-resident), applies exposure, the ACES fit,
//    gamma and 8-bit rounding, and writes one 32-bit RGBA word.
#include "device_common.hpp"
#include "launch.hpp"

namespace epb {

struct PostK {
    int W, H, nl;  // nl = number of levels >= 1
    int lw[EPB_MAX_BLOOM_LEVELS], lh[EPB_MAX_BLOOM_LEVELS];
    void *raw[EPB_MAX_BLOOM_LEVELS];   // level texels of the pyramid storage type
    void *blur[EPB_MAX_BLOOM_LEVELS];
    int blk_start[EPB_MAX_BLOOM_LEVELS + 1];  // blur launch: first block of each level
    float threshold, strength, exposure, inv_gamma;
    int tiles_x, tiles;
};

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

template <typename TH, typename TP>
__global__ void __launch_bounds__(256) k_bloom_down(const PostK c, const TH *__restrict__ hdr) {
    __shared__ float4 s1[32][33];
    __shared__ float4 s2[16][17];
    __shared__ float4 s3[8][9];
    __shared__ float4 s4[4][5];
    int tile = xcd_tile(blockIdx.x, c.tiles);
    int bx = tile % c.tiles_x, by = tile / c.tiles_x;
    int t = threadIdx.x;
    unsigned plane = (unsigned)c.W * (unsigned)c.H;
    // level 1: bright map averaged over the in-range 2x2 children
    {
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
            s1[ly][lx] = v;
        }
    }
    __syncthreads();
    // levels 2..5 inside the tile; a texel averages its in-range children
#define EPB_LEVEL(L, SRC, DST, N)                                                                   \
    if (c.nl >= L) {                                                                                \
        if (t < N * N) {                                                                            \
            int lx = t % N, ly = t / N;                                                             \
            int X = bx * N + lx, Y = by * N + ly;                                                   \
            float4 v = make_float4(0, 0, 0, 0);                                                     \
            if (X < c.lw[L] && Y < c.lh[L]) {                                                       \
                float n = 0.0f;                                                                     \
                for (int b = 0; b < 2; ++b)                                                         \
                    for (int a = 0; a < 2; ++a)                                                     \
                        if (2 * X + a < c.lw[L - 1] && 2 * Y + b < c.lh[L - 1]) {                   \
                            v = add4(v, SRC[2 * ly + b][2 * lx + a]);                               \
                            n += 1.0f;                                                              \
                        }                                                                           \
                v = scale4(v, 1.0f / n);                                                            \
                ((TP *)c.raw[L])[(size_t)Y * c.lw[L] + X] = pack<TP>(v);                            \
            }                                                                                       \
            DST[ly][lx] = v;                                                                        \
        }                                                                                           \
        __syncthreads();                                                                            \
    }
    EPB_LEVEL(2, s1, s2, 16)
    EPB_LEVEL(3, s2, s3, 8)
    EPB_LEVEL(4, s3, s4, 4)
    if (c.nl >= 5 && t < 4) {
        int lx = t % 2, ly = t / 2;
        int X = bx * 2 + lx, Y = by * 2 + ly;
        if (X < c.lw[5] && Y < c.lh[5]) {
            float4 v = make_float4(0, 0, 0, 0);
            float n = 0.0f;
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a)
                    if (2 * X + a < c.lw[4] && 2 * Y + b < c.lh[4]) {
                        v = add4(v, s4[2 * ly + b][2 * lx + a]);
                        n += 1.0f;
                    }
            ((TP *)c.raw[5])[(size_t)Y * c.lw[5] + X] = pack<TP>(scale4(v, 1.0f / n));
        }
    }
#undef EPB_LEVEL
}

template <typename TP>
__global__ void __launch_bounds__(256) k_bloom_blur(const PostK c) {
    __shared__ float4 sin_[12][36];
    __shared__ float4 sh[12][32];
    int b = blockIdx.x;
    int L = 1;
    while (L < c.nl && b >= c.blk_start[L + 1]) ++L;
    int local = b - c.blk_start[L];
    int w = c.lw[L], h = c.lh[L];
    int tx = (w + 31) / 32;
    int X0 = (local % tx) * 32, Y0 = (local / tx) * 8;
    const TP *src = (const TP *)c.raw[L];
    int t = threadIdx.x;
    for (int q = t; q < 12 * 36; q += 256) {
        int r = q / 36, cc = q % 36;
        int gy = min(max(Y0 + r - 2, 0), h - 1);
        int gx = min(max(X0 + cc - 2, 0), w - 1);
        sin_[r][cc] = unpack(src[(size_t)gy * w + gx]);
    }
    __syncthreads();
    for (int q = t; q < 12 * 32; q += 256) {
        int r = q / 32, cc = q % 32;
        float4 a = sin_[r][cc], bb = sin_[r][cc + 1], m = sin_[r][cc + 2], d = sin_[r][cc + 3], e = sin_[r][cc + 4];
        sh[r][cc] = make_float4((a.x + e.x + 4.0f * (bb.x + d.x) + 6.0f * m.x) * 0.0625f,
                                (a.y + e.y + 4.0f * (bb.y + d.y) + 6.0f * m.y) * 0.0625f,
                                (a.z + e.z + 4.0f * (bb.z + d.z) + 6.0f * m.z) * 0.0625f, 0.0f);
    }
    __syncthreads();
    int ox = t % 32, oy = t / 32;
    int X = X0 + ox, Y = Y0 + oy;
    if (X < w && Y < h) {
        float4 a = sh[oy][ox], bb = sh[oy + 1][ox], m = sh[oy + 2][ox], d = sh[oy + 3][ox], e = sh[oy + 4][ox];
        ((TP *)c.blur[L])[(size_t)Y * w + X] = pack<TP>(
            make_float4((a.x + e.x + 4.0f * (bb.x + d.x) + 6.0f * m.x) * 0.0625f,
                        (a.y + e.y + 4.0f * (bb.y + d.y) + 6.0f * m.y) * 0.0625f,
                        (a.z + e.z + 4.0f * (bb.z + d.z) + 6.0f * m.z) * 0.0625f, 0.0f));
    }
}

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
__global__ void __launch_bounds__(256) k_composite(const PostK c, const TH *__restrict__ hdr,
                                                   uint32_t *__restrict__ ldr) {
    __shared__ float4 sb[kCompLds];
    int tile = xcd_tile(blockIdx.x, c.tiles);
    int X0 = (tile % c.tiles_x) * 32, Y0 = (tile / c.tiles_x) * 8;
    int x = X0 + (int)(threadIdx.x % 32);
    int y = Y0 + (int)(threadIdx.x / 32);
    bool live = x < c.W && y < c.H;
    unsigned p = live ? __umul24((unsigned)y, (unsigned)c.W) + (unsigned)x : 0u;
    unsigned plane = (unsigned)c.W * (unsigned)c.H;
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
    if (!live) return;
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
    sto(ldr, p * 4u, word);
}

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

template <typename TH, typename TP>
static void launch_post(const PostK &c0, const void *hdr, uint8_t *ldr, hipStream_t s) {
    PostK c = c0;
    if (c.nl >= 1) {
        c.tiles_x = (c.lw[1] + 31) / 32;
        c.tiles = c.tiles_x * ((c.lh[1] + 31) / 32);
        hipLaunchKernelGGL((k_bloom_down<TH, TP>), dim3(c.tiles), dim3(256), 0, s, c, (const TH *)hdr);
        int nb = 0;
        for (int l = 1; l <= c.nl; ++l) {
            c.blk_start[l] = nb;
            nb += ((c.lw[l] + 31) / 32) * ((c.lh[l] + 7) / 8);
        }
        c.blk_start[c.nl + 1] = nb;
        hipLaunchKernelGGL(k_bloom_blur<TP>, dim3(nb), dim3(256), 0, s, c);
    }
    c.tiles_x = (c.W + 31) / 32;
    c.tiles = c.tiles_x * ((c.H + 7) / 8);
    hipLaunchKernelGGL((k_composite<TH, TP>), dim3(c.tiles), dim3(256), 0, s, c, (const TH *)hdr, (uint32_t *)ldr);
}

hipError_t launch_bloom_tonemap(const PostPlan &q, const void *hdr, epb_dtype hdr_dtype, float threshold,
                                float strength, float exposure, float gamma, uint8_t *ldr, void *scratch,
                                hipStream_t s) {
    PostK c{};
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
    c.threshold = threshold;
    c.strength = strength;
    c.exposure = exposure;
    c.inv_gamma = 1.0f / gamma;
    bool h16 = hdr_dtype == EPB_F16, p16 = q.texel_bytes == 8;
    if (!h16 && !p16) launch_post<float, float4>(c, hdr, ldr, s);
    else if (!h16 && p16) launch_post<float, Half4>(c, hdr, ldr, s);
    else if (h16 && !p16) launch_post<__half, float4>(c, hdr, ldr, s);
    else launch_post<__half, Half4>(c, hdr, ldr, s);
    return hipGetLastError();
}

}  // namespace epb
