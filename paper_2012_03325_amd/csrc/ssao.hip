// Screen-space ambient occlusion at half resolution with a bilateral blur
// (paper Sec. 5.2: normal-oriented hemisphere, Bavoil and Sainz).
//
// gfx950 mapping:
//  * prep compacts the half-resolution depth (the depth at (2i, 2j)) into a
//    dense Wh x Hh plane: 2 MB at 1080p, resident in one XCD's 4 MB L2, so
//    the sample gathers hit L2 instead of striding the full-resolution plane.
//    It stores h = (d + bias) / radius: the occlusion test d_s <= z_q - bias
//    becomes h_s <= z_q / radius and the range term radius / |d - d_s| becomes
//    1 / |h - h_s|, two instructions fewer per sample.
//  * raw: one thread per half-resolution texel; the sample kernel is read with
//    scalar loads (wave-uniform).  A sample's depth and projected texel
//    coordinates, in units of the radius, are affine in the kernel vector
//    (three plane equations per pixel), so a sample costs 9 FMA, one
//    reciprocal, two multiplies, two floor-converts, a range test, one
//    gathered depth and 5 instructions of smoothstep and sum; gathers are
//    issued a batch at a time before any is consumed, through a buffer
//    resource whose range check makes an out-of-image offset read 0 (the
//    sample is discarded by its range test).
//  * blur: 4x4 bilateral mean; the 19x11 depth/AO footprint of a 16x8 tile is
//    staged through LDS.
//  * every stage has a single-view kernel (one block per tile, XCD-aware
//    order) and a batched kernel that walks the tiles of many views.
#include "device_common.hpp"
#include "launch.hpp"

namespace epb {

// ---------------------------------------------------------------------------
// per-item work
// ---------------------------------------------------------------------------
// Stored form of a half-resolution depth: (d + bias) / radius (+inf stays +inf).
__device__ __forceinline__ float ssao_h(const SsaoDesc &c, float d) { return (d + c.bias) * c.inv_radius; }

__device__ __forceinline__ void ssao_prep_item(const SsaoDesc &c, int item) {
    int chunks = (c.Wh + kSsaoPrepW - 1) / kSsaoPrepW;
    int j = item / chunks;
    int i = (item - j * chunks) * kSsaoPrepW + (int)threadIdx.x;
    if (i >= c.Wh) return;
    stf(c.hdepth, __umul24((unsigned)j, (unsigned)c.Wh) + (unsigned)i,
        ssao_h(c, ldf(c.depth, __umul24((unsigned)(2 * j), (unsigned)c.W) + (unsigned)(2 * i))));
}

// KB samples of one pixel: all gathers issued before any is used.  `kern` points
// at the batch's first kernel vector; with `ragged`, only the first `m` samples
// exist (the others repeat the last one and are discarded).
template <int KB, bool ragged>
__device__ __forceinline__ float ssao_batch(const SsaoDesc &c, const ConstFloat *kern, int m, v3 Xv, v3 Yv, v3 Zv,
                                            float X0, float Y0, float Z0, float hp, __amdgpu_buffer_rsrc_t hdepth,
                                            float occ) {
    float hs[KB], zqs[KB];
    bool ok[KB];
#pragma unroll
    for (int b = 0; b < KB; ++b) {
        int k = ragged ? min(b, m - 1) : b;  // wave-uniform: scalar loads
        float sx = kern[3 * k], sy = kern[3 * k + 1], sz = kern[3 * k + 2];
        float zq = fmaf(Zv.x, sx, fmaf(Zv.y, sy, fmaf(Zv.z, sz, Z0)));
        float nx = fmaf(Xv.x, sx, fmaf(Xv.y, sy, fmaf(Xv.z, sz, X0)));
        float ny = fmaf(Yv.x, sx, fmaf(Yv.y, sy, fmaf(Yv.z, sz, Y0)));
        float iz = rcp(zq);
        // floor-convert: 0 <= hx < Wh exactly when 0 <= floor(hx) < Wh (one unsigned
        // compare; out-of-range values saturate outside the range, and a NaN
        // (converted to 0) only arises with zq <= 0 or a NaN input, rejected by zq > 0)
        int ix = floor_to_int(nx * iz), iy = floor_to_int(ny * iz);
        ok[b] = (!ragged || b < m) && zq > 0.0f && (unsigned)ix < (unsigned)c.Wh && (unsigned)iy < (unsigned)c.Hh;
        // unchecked offset: when !ok it may point anywhere (a load past the plane
        // reads 0, one inside it an unrelated texel) and the sample is discarded
        hs[b] = buf_ldf(hdepth, (__umul24((unsigned)iy, (unsigned)c.Wh) + (unsigned)ix) * 4u);
        zqs[b] = zq;
    }
#pragma unroll
    for (int b = 0; b < KB; ++b) {
        // smoothstep(radius / |d - d_s|) = u^2 (3 - 2u), u = clamp(1 / |h - h_s|)
        float u = clamp01(rcp(fabsf(hp - hs[b])));
        float u2 = u * u, w = fmaf(-2.0f, u, 3.0f);
        occ = fmaf(u2, (ok[b] && hs[b] <= zqs[b]) ? w : 0.0f, occ);  // d_s <= z_q - bias
    }
    return occ;
}

template <int TX, int TY, int KB, typename TG, typename TA>
__device__ __forceinline__ void ssao_raw_tile(const SsaoDesc &c, int tile) {
    int tiles_x = (c.Wh + TX - 1) / TX;
    int ty = tile / tiles_x;
    int i = (tile - ty * tiles_x) * TX + (int)(threadIdx.x % TX);
    int j = ty * TY + (int)(threadIdx.x / TX);
    if (i >= c.Wh || j >= c.Hh) return;
    int x = 2 * i, y = 2 * j;
    unsigned p = __umul24((unsigned)y, (unsigned)c.W) + (unsigned)x;
    float d = ldf(c.depth, p);
    unsigned o = __umul24((unsigned)j, (unsigned)c.Wh) + (unsigned)i;
    TA *out = (TA *)c.raw;
    if (__builtin_isinf(d)) {
        stf(out, o, 1.0f);
        return;
    }
    unsigned plane = (unsigned)c.W * (unsigned)c.H;
    const TG *normal = (const TG *)c.normal;
    // view-space position and normal
    v3 P = mk3(((float)x + 0.5f - c.cam.cx) * c.cam.inv_fx * d, -((float)y + 0.5f - c.cam.cy) * c.cam.inv_fy * d, -d);
    v3 nw = mk3(ldf(normal, p), ldf(normal, plane + p), ldf(normal, 2 * plane + p));
    v3 nv = normalize(mul_R(c.cam.R, nw));
    // rotation noise, Gram-Schmidt against the normal
    unsigned rn = 2u * (unsigned)((j & 3) * 4 + (i & 3));
    v3 r = mk3(ldf(c.noise, rn), ldf(c.noise, rn + 1u), 0.0f);
    v3 t = normalize(r - nv * dot(nv, r));
    v3 bb = cross(nv, t);
    // Sample s of the kernel lands at Q = P + radius (t sx + b sy + n sz).  In
    // units of the radius its depth zq = -Q.z / radius and the numerators of its
    // half-resolution texel coordinates hx = u / 2 + 1/4 = (fx/2 Q.x + (cx/2 +
    // 1/4) (-Q.z)) / (-Q.z) (hy alike, y flipped) are affine in s: three plane
    // equations per pixel.
    float ax = 0.5f * c.cam.fx, bx = 0.5f * c.cam.cx + 0.25f;
    float ay = -0.5f * c.cam.fy, by = 0.5f * c.cam.cy + 0.25f;
    v3 Pr = P * c.inv_radius;
    v3 Mx = mk3(t.x, bb.x, nv.x), My = mk3(t.y, bb.y, nv.y);
    v3 Zv = mk3(-t.z, -bb.z, -nv.z);
    float Z0 = -Pr.z;
    v3 Xv = Mx * ax + Zv * bx, Yv = My * ay + Zv * by;
    float X0 = fmaf(ax, Pr.x, bx * Z0), Y0 = fmaf(ay, Pr.y, by * Z0);
    float hp = ssao_h(c, d);  // the pixel's own stored depth, as prep computed it
    __amdgpu_buffer_rsrc_t hdepth = raw_buffer(c.hdepth, (unsigned)c.Wh * (unsigned)c.Hh * 4u);
    float occ = 0.0f;
    // whole batches of KB samples (their 3 KB kernel floats in one run of scalar
    // loads), then the ragged last batch with its sample index clamped
    int nfull = c.n - c.n % KB;
    const ConstFloat *kern = as_constant(c.kernel);
    for (int k0 = 0; k0 < nfull; k0 += KB)
        occ = ssao_batch<KB, false>(c, kern + 3 * k0, KB, Xv, Yv, Zv, X0, Y0, Z0, hp, hdepth, occ);
    if (nfull < c.n)
        occ = ssao_batch<KB, true>(c, kern + 3 * nfull, c.n - nfull, Xv, Yv, Zv, X0, Y0, Z0, hp, hdepth, occ);
    stf(out, o, 1.0f - occ * c.inv_n);
}

// LDS rows of the blur footprint (11 rows of 19) plus padding, so that every
// thread's staging stores are unconditional (the last ones land in the padding)
constexpr int kBlurLdsRows = ((kBlurTy + 3) * (kBlurTx + 3) + kBlurTx * kBlurTy - 1) / (kBlurTx * kBlurTy) *
                                 (kBlurTx * kBlurTy) / (kBlurTx + 3) + 1;

template <typename TA>
__device__ __forceinline__ void ssao_blur_tile(const SsaoDesc &c, int tile, float (*sd)[kBlurTx + 3],
                                               float (*sa)[kBlurTx + 3]) {
    constexpr int LW = kBlurTx + 3, LH = kBlurTy + 3;  // offsets -2 .. +1
    int tiles_x = (c.Wh + kBlurTx - 1) / kBlurTx;
    int ty = tile / tiles_x;
    int i0 = (tile - ty * tiles_x) * kBlurTx, j0 = ty * kBlurTy;
    const float *raw = (const float *)c.raw;
    // every load of the footprint in flight together: all issued before the first LDS store
    constexpr int kN = LW * LH, kThreads = kBlurTx * kBlurTy, kIt = (kN + kThreads - 1) / kThreads;
    float dq[kIt], aq[kIt];
    bool in[kIt];
#pragma unroll
    for (int k = 0; k < kIt; ++k) {
        int q = min((int)threadIdx.x + kThreads * k, kN - 1);
        int li = q % LW, lj = q / LW;
        int gi = i0 + li - 2, gj = j0 + lj - 2;
        in[k] = gi >= 0 && gi < c.Wh && gj >= 0 && gj < c.Hh;
        unsigned g = in[k] ? __umul24((unsigned)gj, (unsigned)c.Wh) + (unsigned)gi : 0u;
        dq[k] = ldf(c.hdepth, g);
        aq[k] = ldf(raw, g);
    }
#pragma unroll
    for (int k = 0; k < kIt; ++k) {  // unconditional: entries past the footprint land in the padding rows
        int q = (int)threadIdx.x + kThreads * k;
        (&sd[0][0])[q] = in[k] ? dq[k] : __builtin_inff();  // out of range: weight 0
        (&sa[0][0])[q] = in[k] ? aq[k] : 0.0f;
    }
    __syncthreads();
    int ti = threadIdx.x % kBlurTx, tj = threadIdx.x / kBlurTx;
    int i = i0 + ti, j = j0 + tj;
    if (i < c.Wh && j < c.Hh) {
        float dp = sd[tj + 2][ti + 2];  // stored form h = (d + bias) / radius
        float v = 1.0f;
        if (!__builtin_isinf(dp)) {
            // |d_q - d_p| / (tau d_p) = |h_q - h_p| radius / (tau d_p)
            float inv = c.radius / (c.tau * fmaf(dp, c.radius, -c.bias));
            float s = 0.0f, sw = 0.0f;
#pragma unroll
            for (int dy = 0; dy < 4; ++dy)
#pragma unroll
                for (int dx = 0; dx < 4; ++dx) {
                    float dq = sd[tj + dy][ti + dx];
                    float w = __builtin_isinf(dq) ? 0.0f : fmaxf(0.0f, 1.0f - fabsf(dq - dp) * inv);
                    s = fmaf(w, sa[tj + dy][ti + dx], s);
                    sw += w;
                }
            v = s / sw;
        }
        stf((TA *)c.out, __umul24((unsigned)j, (unsigned)c.Wh) + (unsigned)i, v);
    }
    __syncthreads();  // the tile's LDS may be refilled by the next item
}

// ---------------------------------------------------------------------------
// single-view kernels
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kSsaoPrepW) k_ssao_prep(const SsaoDesc c, int items) {
    ssao_prep_item(c, xcd_tile(blockIdx.x, items));
}

template <int TX, int TY, int KB, typename TG, typename TA>
__global__ void __launch_bounds__(TX *TY) k_ssao_raw(const SsaoDesc c, int tiles) {
    ssao_raw_tile<TX, TY, KB, TG, TA>(c, xcd_tile(blockIdx.x, tiles));
}

template <typename TA>
__global__ void __launch_bounds__(kBlurTx *kBlurTy) k_ssao_blur(const SsaoDesc c, int tiles) {
    __shared__ float sd[kBlurLdsRows][kBlurTx + 3];
    __shared__ float sa[kBlurLdsRows][kBlurTx + 3];
    ssao_blur_tile<TA>(c, xcd_tile(blockIdx.x, tiles), sd, sa);
}

// ---------------------------------------------------------------------------
// batched kernels: work items of all views, XCD-aware persistent walk
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kSsaoPrepW) k_ssao_prep_batch(const void *__restrict__ table) {
    const BatchHeader *h = (const BatchHeader *)table;
    const int *start = batch_start(table, kStPrep);
    const ViewDesc *views = batch_views(table);
    XcdRange w = xcd_range(h->total[kStPrep]);
    for (int it = w.lb; it < w.count; it += w.stride) {
        int g = w.first + it;
        int v = find_view(start, h->n_views, g);
        ssao_prep_item(views[v].ssao, g - start[v]);
    }
}

template <int TX, int TY, int KB, typename TG, typename TA>
__global__ void __launch_bounds__(TX *TY) k_ssao_raw_batch(const void *__restrict__ table) {
    const BatchHeader *h = (const BatchHeader *)table;
    const int *start = batch_start(table, kStRaw);
    const ViewDesc *views = batch_views(table);
    XcdRange w = xcd_range(h->total[kStRaw]);
    for (int it = w.lb; it < w.count; it += w.stride) {
        int g = w.first + it;
        int v = find_view(start, h->n_views, g);
        ssao_raw_tile<TX, TY, KB, TG, TA>(views[v].ssao, g - start[v]);
    }
}

template <typename TA>
__global__ void __launch_bounds__(kBlurTx *kBlurTy) k_ssao_blur_batch(const void *__restrict__ table) {
    __shared__ float sd[kBlurLdsRows][kBlurTx + 3];
    __shared__ float sa[kBlurLdsRows][kBlurTx + 3];
    const BatchHeader *h = (const BatchHeader *)table;
    const int *start = batch_start(table, kStBlur);
    const ViewDesc *views = batch_views(table);
    XcdRange w = xcd_range(h->total[kStBlur]);
    for (int it = w.lb; it < w.count; it += w.stride) {
        int g = w.first + it;
        int v = find_view(start, h->n_views, g);
        ssao_blur_tile<TA>(views[v].ssao, g - start[v], sd, sa);
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
SsaoPlan ssao_plan(int W, int H) {
    SsaoPlan q{};
    q.W = W;
    q.H = H;
    q.Wh = (W + 1) / 2;
    q.Hh = (H + 1) / 2;
    size_t n = (size_t)q.Wh * q.Hh * 4;
    n = (n + 255) & ~size_t(255);
    q.off_hdepth = 0;
    q.off_raw = n;
    q.bytes = 2 * n;
    return q;
}

int ssao_items(const SsaoDesc &c, int stage, int ssao_tile) {
    switch (stage) {
    case kStPrep: return c.Hh * ceil_div(c.Wh, kSsaoPrepW);
    case kStRaw: {
        TileShape t = kSsaoTiles[ssao_tile];
        return ceil_div(c.Wh, t.tx) * ceil_div(c.Hh, t.ty);
    }
    default: return ceil_div(c.Wh, kBlurTx) * ceil_div(c.Hh, kBlurTy);
    }
}

SsaoDesc ssao_desc(const SsaoPlan &q, const float *depth, const void *normal, const HostCam &cam, const float *kernel,
                   int n_samples, const float *noise, float radius, float bias, float tau, int blur, void *ao_out,
                   void *scratch) {
    SsaoDesc c{};
    for (int k = 0; k < 9; ++k) c.cam.R[k] = cam.R[k];
    for (int k = 0; k < 3; ++k) c.cam.t[k] = cam.t[k];
    c.cam.fx = cam.fx; c.cam.fy = cam.fy; c.cam.cx = cam.cx; c.cam.cy = cam.cy;
    c.cam.inv_fx = cam.inv_fx; c.cam.inv_fy = cam.inv_fy;
    c.cam.w = cam.w; c.cam.h = cam.h;
    c.radius = radius;
    c.inv_radius = (float)(1.0 / (double)radius);
    c.bias = bias;
    c.tau = tau;
    c.n = n_samples;
    c.inv_n = 1.0f / (float)n_samples;
    c.blur = blur;
    c.W = q.W; c.H = q.H; c.Wh = q.Wh; c.Hh = q.Hh;
    c.depth = depth;
    c.normal = normal;
    c.kernel = kernel;
    c.noise = noise;
    char *sc = (char *)scratch;
    c.hdepth = (float *)(sc + q.off_hdepth);
    // raw AO goes to scratch when blurred, straight to the output otherwise
    c.raw = blur ? (void *)(sc + q.off_raw) : ao_out;
    c.out = ao_out;
    return c;
}

template <int TX, int TY, int KB, typename TG, typename TA>
static void go_raw(const SsaoDesc &c, hipStream_t s) {
    int tiles = ceil_div(c.Wh, TX) * ceil_div(c.Hh, TY);
    hipLaunchKernelGGL((k_ssao_raw<TX, TY, KB, TG, TA>), dim3(tiles), dim3(TX * TY), 0, s, c, tiles);
}

hipError_t launch_ssao(const SsaoDesc &c, epb_dtype gdtype, epb_dtype ao_dtype, hipStream_t s) {
    int prep = ssao_items(c, kStPrep, 0);
    hipLaunchKernelGGL(k_ssao_prep, dim3(prep), dim3(kSsaoPrepW), 0, s, c, prep);
    // the raw pass writes float32 into scratch when a blur follows
    epb_dtype raw_dt = c.blur ? EPB_F32 : ao_dtype;
    if (gdtype == EPB_F32) {
        if (raw_dt == EPB_F32) go_raw<16, 8, 8, float, float>(c, s);
        else go_raw<16, 8, 8, float, __half>(c, s);
    } else {
        if (raw_dt == EPB_F32) go_raw<16, 8, 8, __half, float>(c, s);
        else go_raw<16, 8, 8, __half, __half>(c, s);
    }
    if (c.blur) {
        int tiles = ssao_items(c, kStBlur, 0);
        if (ao_dtype == EPB_F32)
            hipLaunchKernelGGL(k_ssao_blur<float>, dim3(tiles), dim3(kBlurTx * kBlurTy), 0, s, c, tiles);
        else
            hipLaunchKernelGGL(k_ssao_blur<__half>, dim3(tiles), dim3(kBlurTx * kBlurTy), 0, s, c, tiles);
    }
    return hipGetLastError();
}

// Grid of a batched stage: one block per item, or a persistent grid of
// blocks_per_cu blocks per CU (at least 8, so that every XCD has a block).
int batch_grid(int total, int blocks_per_cu) {
    if (blocks_per_cu <= 0) return total;
    int g = blocks_per_cu * 256;
    if (g < 8) g = 8;
    return total < g ? total : g;
}

template <int TX, int TY, int KB, typename TG, typename TA>
static void go_raw_batch(const BatchHeader &h, const void *table, hipStream_t s) {
    int grid = batch_grid(h.total[kStRaw], h.blocks_per_cu);
    hipLaunchKernelGGL((k_ssao_raw_batch<TX, TY, KB, TG, TA>), dim3(grid), dim3(TX * TY), 0, s, table);
}

template <typename TG, typename TA>
static void pick_raw_batch(const BatchHeader &h, const void *table, hipStream_t s) {
    int shape = h.ssao_tile, kb = h.ssao_batch;
    if (shape == 0 && kb == 0) go_raw_batch<16, 8, 8, TG, TA>(h, table, s);
    else if (shape == 0) go_raw_batch<16, 8, 16, TG, TA>(h, table, s);
    else if (kb == 0) go_raw_batch<32, 4, 8, TG, TA>(h, table, s);
    else go_raw_batch<32, 4, 16, TG, TA>(h, table, s);
}

hipError_t launch_ssao_batch(const BatchHeader &h, const void *table, hipStream_t s) {
    hipLaunchKernelGGL(k_ssao_prep_batch, dim3(batch_grid(h.total[kStPrep], h.blocks_per_cu)), dim3(kSsaoPrepW), 0,
                       s, table);
    epb_dtype raw_dt = h.blur ? EPB_F32 : (epb_dtype)h.ao_dtype;
    if (h.gdtype == EPB_F32) {
        if (raw_dt == EPB_F32) pick_raw_batch<float, float>(h, table, s);
        else pick_raw_batch<float, __half>(h, table, s);
    } else {
        if (raw_dt == EPB_F32) pick_raw_batch<__half, float>(h, table, s);
        else pick_raw_batch<__half, __half>(h, table, s);
    }
    if (h.blur) {
        int grid = batch_grid(h.total[kStBlur], h.blocks_per_cu);
        if (h.ao_dtype == EPB_F32)
            hipLaunchKernelGGL(k_ssao_blur_batch<float>, dim3(grid), dim3(kBlurTx * kBlurTy), 0, s, table);
        else
            hipLaunchKernelGGL(k_ssao_blur_batch<__half>, dim3(grid), dim3(kBlurTx * kBlurTy), 0, s, table);
    }
    return hipGetLastError();
}

}  // namespace epb
