// Per-tile device functions of the SSAO stages (paper Sec. 5.2): depth
// compaction, raw AO of a tile (L2 gathers or an LDS window) and the bilateral
// blur; shared by the single-view, batched and persistent kernels.
#pragma once

#include "device_common.hpp"

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
    return clamp01(1.0f - occ * c.inv_n);  // (1/n rounded up could take a fully occluded texel below 0)
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

// LDS rows of a TX x TY blur tile's footprint ((TY + 3) rows of TX + 3) plus
// padding, so that every thread's staging stores are unconditional (the last
// ones land in the padding)
template <int TX, int TY>
constexpr int blur_lds_rows() {
    return ((TY + 3) * (TX + 3) + TX * TY - 1) / (TX * TY) * (TX * TY) / (TX + 3) + 1;
}

// 4x4 bilateral mean of one TX x TY tile of half-resolution texels (TX * TY
// threads); the same arithmetic per texel for every tile shape.
template <int TX, int TY, typename TA>
__device__ __forceinline__ void ssao_blur_tile(const SsaoDesc &c, int tile, float (*sd)[TX + 3], float (*sa)[TX + 3]) {
    constexpr int LW = TX + 3, LH = TY + 3;  // offsets -2 .. +1
    int tiles_x = (c.Wh + TX - 1) / TX;
    int ty = tile / tiles_x;
    int i0 = (tile - ty * tiles_x) * TX, j0 = ty * TY;
    const float *raw = (const float *)c.raw;
    // every load of the footprint in flight together: all issued before the first LDS store
    constexpr int kN = LW * LH, kThreads = TX * TY, kIt = (kN + kThreads - 1) / kThreads;
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
    int ti = threadIdx.x % TX, tj = threadIdx.x / TX;
    int i = i0 + ti, j = j0 + tj;
    if (i < c.Wh && j < c.Hh) {
        float dp = sd[tj + 2][ti + 2];
        float v = 1.0f;
        if (!__builtin_isinf(dp)) {
            float inv = rcp(c.tau * dp);  // weight 1 - |d_q - d_p| / (tau d_p)
            float s = 0.0f, sw = 0.0f;
#pragma unroll
            for (int dy = 0; dy < 4; ++dy)
#pragma unroll
                for (int dx = 0; dx < 4; ++dx) {
                    // a background or out-of-range neighbour (+inf) gets max(0, -inf) = 0
                    float dq = sd[tj + dy][ti + dx];
                    float w = fmaxf(0.0f, 1.0f - fabsf(dq - dp) * inv);
                    s = fmaf(w, sa[tj + dy][ti + dx], s);
                    sw += w;
                }
            // s / sw (sw >= 1: the centre's own weight) from the reciprocal and one
            // correction with the exact residual s - sw q: exactly 1 where s == sw, and
            // kept in [0, 1] (a weighted mean of values in [0, 1]) by the free clamp
            float r = rcp(sw), q = s * r;
            v = clamp01(fmaf(fmaf(-sw, q, s), r, q));
        }
        stf((TA *)c.out, __umul24((unsigned)j, (unsigned)c.Wh) + (unsigned)i, v);
    }
    __syncthreads();  // the tile's LDS may be refilled by the next item
}

}  // namespace epb
