// Screen-space ambient occlusion at half resolution with a bilateral blur
// (paper Sec. 5.2: normal-oriented hemisphere, Bavoil and Sainz).
//
// gfx950 mapping:
//  * prep compacts the half-resolution depth (the depth at (2i, 2j)) into a
//    dense Wh x Hh plane: 2 MB at 1080p, resident in one XCD's 4 MB L2, so
//    the sample gathers hit L2 instead of striding the full-resolution plane.
//  * raw: one thread per half-resolution texel; the sample kernel is read with
//    scalar loads (wave-uniform).  Every float decision is formed from small
//    quantities, so that its rounding error does not grow with the depth or
//    the image size:
//      - the sample's texel coordinate is the pixel's own coordinate plus the
//        sample's offset, offset = (f/2) r (w_x + a_x w_z) / z_q (w the
//        view-space kernel vector, a_x the pixel's view-ray slope), added in
//        one fused multiply-add, so its error is a few roundings of the offset
//        plus one of the sum;
//      - the depth test d_s <= z_q - bias becomes (d_s - d) <= -(r w_z + bias),
//        where d_s - d is exact whenever the two depths lie within a factor of
//        two of each other (Sterbenz) and r w_z + bias is of the order of the
//        radius; the range term radius / |d - d_s| uses the same difference.
//    A sample costs 12 FMA for the offset numerators and r w_z + bias, one
//    subtraction for z_q, one reciprocal, two fused offsets, two
//    floor-converts, a range test, one gathered depth and 8 instructions of
//    smoothstep and sum; gathers are issued a batch at a time before any is
//    consumed, through a buffer resource whose range check makes an
//    out-of-image offset read 0 (the sample is discarded by its range test).
//  * blur: 4x4 bilateral mean; the 19x11 depth/AO footprint of a 16x8 tile is
//    staged through LDS.
//  * every stage has a single-view kernel (one block per tile, XCD-aware
//    order) and a batched kernel that walks the tiles of many views.
#include <mutex>

#include "device_common.hpp"
#include "launch.hpp"

namespace epb {

// ---------------------------------------------------------------------------
// per-item work
// ---------------------------------------------------------------------------
__device__ __forceinline__ void ssao_prep_item(const SsaoDesc &c, int item) {
    int chunks = (c.Wh + kSsaoPrepW - 1) / kSsaoPrepW;
    int j = item / chunks;
    int i = (item - j * chunks) * kSsaoPrepW + (int)threadIdx.x;
    if (i >= c.Wh) return;
    stf(c.hdepth, __umul24((unsigned)j, (unsigned)c.Wh) + (unsigned)i,
        ldf(c.depth, __umul24((unsigned)(2 * j), (unsigned)c.W) + (unsigned)(2 * i)));
}

// Per-pixel constants of the sample loop: the kernel vector s enters through
// three dot products, e = r w_z + bias (Ev, bias), and the numerators of the
// texel-coordinate offsets in x and y (Xv, Yv).
struct SsaoPix {
    v3 Ev, Xv, Yv;
    float d, dpb, hx0, hy0;  // own depth, d + bias, own half-resolution coordinates + 1/2
};

// Half-resolution depth staged in LDS for a tile and its halo: lds[ly * kSsaoLdsW + lx]
// holds texel (ox + lx, oy + ly) of the compact plane (clamped to the image:
// entries outside it are never used, a sample landing there is discarded).
struct LdsWindow {
    const float *lds;
    int ox, oy;
};

// KB samples of one pixel: all gathers issued before any is used.  `kern` points
// at the batch's first kernel vector; with `ragged`, only the first `m` samples
// exist (the others repeat the last one and are discarded).  With kLds, a sample
// inside the LDS window reads it there; the lanes with a kept sample outside it
// read all KB from the plane in L2 (the same texels, so the same values).
template <int KB, bool ragged, bool kLds>
__device__ __forceinline__ float ssao_batch(const SsaoDesc &c, const ConstFloat *kern, int m, const SsaoPix &q,
                                            __amdgpu_buffer_rsrc_t hdepth, LdsWindow win, float occ) {
    float ds[KB], es[KB];
    bool ok[KB];
    unsigned off[KB];
    bool miss = false;
#pragma unroll
    for (int b = 0; b < KB; ++b) {
        int k = ragged ? min(b, m - 1) : b;  // wave-uniform: scalar loads
        float sx = kern[3 * k], sy = kern[3 * k + 1], sz = kern[3 * k + 2];
        float e = fmaf(q.Ev.x, sx, fmaf(q.Ev.y, sy, fmaf(q.Ev.z, sz, c.bias)));  // r w_z + bias
        float zq = q.dpb - e;                                                   // d - r w_z
        float nx = fmaf(q.Xv.x, sx, fmaf(q.Xv.y, sy, q.Xv.z * sz));
        float ny = fmaf(q.Yv.x, sx, fmaf(q.Yv.y, sy, q.Yv.z * sz));
        float iz = rcp(zq);
        // floor-convert: 0 <= h < Wh exactly when 0 <= floor(h) < Wh (one unsigned
        // compare; out-of-range values saturate outside the range, and a NaN
        // (converted to 0) only arises with zq <= 0 or a NaN input, rejected by zq > 0)
        int ix = floor_to_int(fmaf(nx, iz, q.hx0)), iy = floor_to_int(fmaf(ny, iz, q.hy0));
        ok[b] = (!ragged || b < m) && zq > 0.0f && (unsigned)ix < (unsigned)c.Wh && (unsigned)iy < (unsigned)c.Hh;
        // unchecked offset: when !ok it may point anywhere (a load past the plane
        // reads 0, one inside it an unrelated texel) and the sample is discarded
        off[b] = (__umul24((unsigned)iy, (unsigned)c.Wh) + (unsigned)ix) * 4u;
        if constexpr (kLds) {
            unsigned lx = (unsigned)(ix - win.ox), ly = (unsigned)(iy - win.oy);
            bool in = max(lx, ly) < (unsigned)kSsaoLdsW;
            ds[b] = win.lds[in ? __umul24(ly, (unsigned)kSsaoLdsW) + lx : 0u];
            miss |= ok[b] && !in;
        } else {
            ds[b] = buf_ldf(hdepth, off[b]);
        }
        es[b] = e;
    }
    if constexpr (kLds) {
        if (miss) {
#pragma unroll
            for (int b = 0; b < KB; ++b) ds[b] = buf_ldf(hdepth, off[b]);
        }
    }
#pragma unroll
    for (int b = 0; b < KB; ++b) {
        float dd = ds[b] - q.d;  // exact when the depths are within a factor of two
        // smoothstep(radius / |d - d_s|) = u^2 (3 - 2u), u = clamp(radius / |d - d_s|)
        float u = clamp01(c.radius * rcp(fabsf(dd)));
        float u2 = u * u, w = fmaf(-2.0f, u, 3.0f);
        occ = fmaf(u2, (ok[b] && dd <= -es[b]) ? w : 0.0f, occ);  // d_s <= z_q - bias
    }
    return occ;
}

// Raw AO of half-resolution texel (i, j), whose pixel (2i, 2j) at plane index p
// has the finite depth d: the kernel's samples in batches of KB.
template <int KB, bool kLds, typename TG>
__device__ __forceinline__ float ssao_texel(const SsaoDesc &c, int i, int j, unsigned p, float d, LdsWindow win) {
    int x = 2 * i, y = 2 * j;
    unsigned plane = (unsigned)c.W * (unsigned)c.H;
    const TG *normal = (const TG *)c.normal;
    // view-ray slopes of the pixel (its point is d (ax, ay, -1)) and view-space normal
    float ax = ((float)x + 0.5f - c.cam.cx) * c.cam.inv_fx, ay = -((float)y + 0.5f - c.cam.cy) * c.cam.inv_fy;
    v3 nw = mk3(ldf(normal, p), ldf(normal, plane + p), ldf(normal, 2 * plane + p));
    v3 nv = normalize(mul_R(c.cam.R, nw));
    // rotation noise, Gram-Schmidt against the normal
    unsigned rn = 2u * (unsigned)((j & 3) * 4 + (i & 3));
    v3 r = mk3(ldf(c.noise, rn), ldf(c.noise, rn + 1u), 0.0f);
    v3 t = normalize(r - nv * dot(nv, r));
    v3 bb = cross(nv, t);
    // The sample lands at Q = P + radius w, w = t sx + b sy + n sz, depth
    // z_q = d - radius w_z; its half-resolution coordinate is the pixel's own,
    // i + 1/2, plus (fx radius / 2) (w_x + ax w_z) / z_q (y alike, flipped).
    SsaoPix q;
    q.Ev = mk3(t.z, bb.z, nv.z) * c.radius;
    float sx = 0.5f * c.cam.fx * c.radius, sy = -0.5f * c.cam.fy * c.radius;
    q.Xv = mk3(fmaf(ax, t.z, t.x), fmaf(ax, bb.z, bb.x), fmaf(ax, nv.z, nv.x)) * sx;
    q.Yv = mk3(fmaf(ay, t.z, t.y), fmaf(ay, bb.z, bb.y), fmaf(ay, nv.z, nv.y)) * sy;
    q.d = d;
    q.dpb = d + c.bias;
    q.hx0 = (float)i + 0.5f;
    q.hy0 = (float)j + 0.5f;
    __amdgpu_buffer_rsrc_t hdepth = raw_buffer(c.hdepth, (unsigned)c.Wh * (unsigned)c.Hh * 4u);
    float occ = 0.0f;
    // whole batches of KB samples (their 3 KB kernel floats in one run of scalar
    // loads), then the ragged last batch with its sample index clamped
    int nfull = c.n - c.n % KB;
    const ConstFloat *kern = as_constant(c.kernel);
    for (int k0 = 0; k0 < nfull; k0 += KB)
        occ = ssao_batch<KB, false, kLds>(c, kern + 3 * k0, KB, q, hdepth, win, occ);
    if (nfull < c.n)
        occ = ssao_batch<KB, true, kLds>(c, kern + 3 * nfull, c.n - nfull, q, hdepth, win, occ);
    return 1.0f - occ * c.inv_n;
}

template <int TX, int TY, int KB, typename TG, typename TA>
__device__ __forceinline__ void ssao_raw_tile(const SsaoDesc &c, int tile) {
    int tiles_x = (c.Wh + TX - 1) / TX;
    int ty = tile / tiles_x;
    int i = (tile - ty * tiles_x) * TX + (int)(threadIdx.x % TX);
    int j = ty * TY + (int)(threadIdx.x / TX);
    if (i >= c.Wh || j >= c.Hh) return;
    unsigned p = __umul24((unsigned)(2 * j), (unsigned)c.W) + (unsigned)(2 * i);
    float d = ldf(c.depth, p);
    unsigned o = __umul24((unsigned)j, (unsigned)c.Wh) + (unsigned)i;
    stf((TA *)c.raw, o, __builtin_isinf(d) ? 1.0f : ssao_texel<KB, false, TG>(c, i, j, p, d, LdsWindow{}));
}

// The LDS-staged variant: a kSsaoLdsTile^2 tile stages its footprint and a
// kSsaoHalo-texel halo of the compact depth plane (kSsaoLdsW^2 floats), then
// samples as above.  Every thread reaches both barriers; the first one also
// keeps a persistent block from overwriting the window that the previous item
// still reads.
template <int KB, typename TG, typename TA>
__device__ __forceinline__ void ssao_raw_tile_lds(const SsaoDesc &c, int tile, float *lds) {
    constexpr int T = kSsaoLdsTile, NT = T * T, N = kSsaoLdsW * kSsaoLdsW, IT = N / NT;
    static_assert(N % NT == 0, "the window is whole rounds of the block");
    int tiles_x = (c.Wh + T - 1) / T;
    int ty = tile / tiles_x;
    LdsWindow win{lds, (tile - ty * tiles_x) * T - kSsaoHalo, ty * T - kSsaoHalo};
    float st[IT];
#pragma unroll
    for (int k = 0; k < IT; ++k) {  // all loads in flight before the first store
        int q = (int)threadIdx.x + NT * k;
        int ly = q / kSsaoLdsW, lx = q - ly * kSsaoLdsW;
        int gi = min(max(win.ox + lx, 0), c.Wh - 1), gj = min(max(win.oy + ly, 0), c.Hh - 1);
        st[k] = ldf(c.hdepth, __umul24((unsigned)gj, (unsigned)c.Wh) + (unsigned)gi);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < IT; ++k) lds[(int)threadIdx.x + NT * k] = st[k];
    __syncthreads();
    int i = win.ox + kSsaoHalo + (int)(threadIdx.x % T), j = win.oy + kSsaoHalo + (int)(threadIdx.x / T);
    if (i >= c.Wh || j >= c.Hh) return;
    unsigned p = __umul24((unsigned)(2 * j), (unsigned)c.W) + (unsigned)(2 * i);
    float d = ldf(c.depth, p);
    unsigned o = __umul24((unsigned)j, (unsigned)c.Wh) + (unsigned)i;
    stf((TA *)c.raw, o, __builtin_isinf(d) ? 1.0f : ssao_texel<KB, true, TG>(c, i, j, p, d, win));
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
        float dp = sd[tj + 2][ti + 2];
        float v = 1.0f;
        if (!__builtin_isinf(dp)) {
            float inv = 1.0f / (c.tau * dp);  // weight 1 - |d_q - d_p| / (tau d_p)
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

template <int KB, typename TG, typename TA>
__global__ void __launch_bounds__(kSsaoLdsTile *kSsaoLdsTile) k_ssao_raw_batch_lds(const void *__restrict__ table) {
    __shared__ float lds[kSsaoLdsW * kSsaoLdsW];
    const BatchHeader *h = (const BatchHeader *)table;
    const int *start = batch_start(table, kStRaw);
    const ViewDesc *views = batch_views(table);
    XcdRange w = xcd_range(h->total[kStRaw]);
    for (int it = w.lb; it < w.count; it += w.stride) {  // the bounds are block-uniform
        int g = w.first + it;
        int v = find_view(start, h->n_views, g);
        ssao_raw_tile_lds<KB, TG, TA>(views[v].ssao, g - start[v], lds);
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

// ---------------------------------------------------------------------------
// scratch held by the library (epb_ssao_static): one array per GPU, for callers
// that cannot allocate.  In host code the array's name is only a stand-in; its
// device address is looked up once per device and used everywhere instead.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char static_scratch[EPB_SSAO_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void *g_static_addr[kMaxDevices];  // device address of static_scratch, per device
}  // namespace

hipError_t ssao_static_scratch(void **addr) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_addr[dev]) {  // first call on this device, which is current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(static_scratch));
        if (e != hipSuccess) return e;
        g_static_addr[dev] = p;
    }
    *addr = g_static_addr[dev];
    return hipSuccess;
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

template <int KB, typename TG, typename TA>
static void go_raw_batch_lds(const BatchHeader &h, const void *table, hipStream_t s) {
    int grid = batch_grid(h.total[kStRaw], h.blocks_per_cu);
    hipLaunchKernelGGL((k_ssao_raw_batch_lds<KB, TG, TA>), dim3(grid), dim3(kSsaoLdsTile * kSsaoLdsTile), 0, s,
                       table);
}

template <typename TG, typename TA>
static void pick_raw_batch(const BatchHeader &h, const void *table, hipStream_t s) {
    int shape = h.ssao_tile, kb = h.ssao_batch;
    if (shape == 0 && kb == 0) go_raw_batch<16, 8, 8, TG, TA>(h, table, s);
    else if (shape == 0) go_raw_batch<16, 8, 16, TG, TA>(h, table, s);
    else if (shape == 1 && kb == 0) go_raw_batch<32, 4, 8, TG, TA>(h, table, s);
    else if (shape == 1) go_raw_batch<32, 4, 16, TG, TA>(h, table, s);
    else if (kb == 0) go_raw_batch_lds<8, TG, TA>(h, table, s);
    else go_raw_batch_lds<16, TG, TA>(h, table, s);
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
