// Screen-space ambient occlusion at half resolution with a bilateral blur
// (paper Sec. 5.2: normal-oriented hemisphere, Bavoil and Sainz).
//
// gfx950 mapping:
//  * k_ssao_prep compacts the half-resolution depth (the depth at (2i, 2j))
//    into a dense Wh x Hh plane: 2 MB at 1080p, resident in one XCD's 4 MB
//    L2, so the sample gathers hit L2 instead of striding through the
//    full-resolution plane.
//  * k_ssao_raw: one thread per half-resolution texel; the sample kernel is
//    staged once per workgroup in LDS and read as wave-uniform broadcasts; the
//    per-sample work is a 3x3 frame transform, one reciprocal, a floor and one
//    gathered depth.
//  * k_ssao_blur: 4x4 bilateral mean; the 19x11 depth/AO footprint of a 16x8
//    tile is staged through LDS.
//  * 16x8 tiles, consecutive tiles on the same XCD.
#include "device_common.hpp"
#include "launch.hpp"

namespace epb {

constexpr int kTx = 16, kTy = 8;  // 128 threads per workgroup

__global__ void __launch_bounds__(256) k_ssao_prep(const float *__restrict__ depth, int W, int Wh, int Hh,
                                                   float *__restrict__ hdepth) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y;
    if (i >= Wh) return;
    hdepth[(size_t)j * Wh + i] = depth[(size_t)(2 * j) * W + 2 * i];
}

struct SsaoConst {
    DevCam cam;
    float radius, bias;
    int n;
    float inv_n;
    int W, H, Wh, Hh;
    int tiles_x, tiles;
};

template <typename TG, typename TA>
__global__ void __launch_bounds__(kTx *kTy) k_ssao_raw(SsaoConst c, const float *__restrict__ depth,
                                                       const TG *__restrict__ normal,
                                                       const float *__restrict__ hdepth,
                                                       const float *__restrict__ kern,
                                                       const float *__restrict__ noise, TA *__restrict__ out) {
    __shared__ float sk[EPB_MAX_SSAO_SAMPLES * 3];
    for (int q = threadIdx.x; q < c.n * 3; q += blockDim.x) sk[q] = kern[q];
    __syncthreads();
    int tile = xcd_tile(blockIdx.x, c.tiles);
    int ti = threadIdx.x % kTx, tj = threadIdx.x / kTx;
    int i = (tile % c.tiles_x) * kTx + ti;
    int j = (tile / c.tiles_x) * kTy + tj;
    if (i >= c.Wh || j >= c.Hh) return;
    int x = 2 * i, y = 2 * j;
    unsigned p = __umul24((unsigned)y, (unsigned)c.W) + (unsigned)x;
    float d = ldf(depth, p);
    unsigned o = __umul24((unsigned)j, (unsigned)c.Wh) + (unsigned)i;
    if (__builtin_isinf(d)) {
        stf(out, o, 1.0f);
        return;
    }
    unsigned plane = (unsigned)c.W * (unsigned)c.H;
    // view-space position and normal
    v3 P = mk3(((float)x + 0.5f - c.cam.cx) * c.cam.inv_fx * d, -((float)y + 0.5f - c.cam.cy) * c.cam.inv_fy * d, -d);
    v3 nw = mk3(ldf(normal, p), ldf(normal, plane + p), ldf(normal, 2 * plane + p));
    v3 nv = normalize(mul_R(c.cam.R, nw));
    // rotation noise, Gram-Schmidt against the normal
    const float *rn = noise + 2 * ((j & 3) * 4 + (i & 3));
    v3 r = mk3(rn[0], rn[1], 0.0f);
    v3 t = normalize(r - nv * dot(nv, r));
    v3 bb = cross(nv, t);
    // Sample s of the kernel lands at Q = P + radius (t sx + b sy + n sz).  Its
    // depth zq = -Q.z and the numerators of its half-resolution texel
    // coordinates hx = u / 2 + 1/4 = (fx/2 Q.x + (cx/2 + 1/4) zq) / zq (hy alike,
    // y flipped) are affine in s: three plane equations per pixel.
    float ax = 0.5f * c.cam.fx, bx = 0.5f * c.cam.cx + 0.25f;
    float ay = -0.5f * c.cam.fy, by = 0.5f * c.cam.cy + 0.25f;
    v3 Mx = mk3(t.x, bb.x, nv.x) * c.radius, My = mk3(t.y, bb.y, nv.y) * c.radius,
       Mz = mk3(t.z, bb.z, nv.z) * c.radius;
    v3 Zv = mk3(-Mz.x, -Mz.y, -Mz.z);
    float Z0 = -P.z;
    v3 Xv = Mx * ax + Zv * bx, Yv = My * ay + Zv * by;
    float X0 = fmaf(ax, P.x, bx * Z0), Y0 = fmaf(ay, P.y, by * Z0);
    float fWh = (float)c.Wh, fHh = (float)c.Hh;
    // samples in batches of 8: every gather of a batch is issued (at index 0
    // for samples that miss the image) before any is consumed
    constexpr int kB = 8;
    float occ = 0.0f;
    for (int k0 = 0; k0 < c.n; k0 += kB) {
        float ds[kB], zqs[kB];
        bool ok[kB];
#pragma unroll
        for (int b = 0; b < kB; ++b) {
            int k = min(k0 + b, c.n - 1);
            float sx = sk[3 * k], sy = sk[3 * k + 1], sz = sk[3 * k + 2];
            float zq = fmaf(Zv.x, sx, fmaf(Zv.y, sy, fmaf(Zv.z, sz, Z0)));
            float nx = fmaf(Xv.x, sx, fmaf(Xv.y, sy, fmaf(Xv.z, sz, X0)));
            float ny = fmaf(Yv.x, sx, fmaf(Yv.y, sy, fmaf(Yv.z, sz, Y0)));
            float iz = rcp(zq);
            float hx = nx * iz, hy = ny * iz;
            ok[b] = (k0 + b < c.n) && zq > 0.0f && hx >= 0.0f && hx < fWh && hy >= 0.0f && hy < fHh;
            // truncation is floor on the accepted (non-negative) range
            unsigned idx = ok[b] ? __umul24((unsigned)(int)hy, (unsigned)c.Wh) + (unsigned)(int)hx : 0u;
            ds[b] = ldf(hdepth, idx);
            zqs[b] = zq;
        }
#pragma unroll
        for (int b = 0; b < kB; ++b) {
            float u = clamp01(c.radius * rcp(fabsf(d - ds[b])));
            float sm = u * u * (3.0f - 2.0f * u);
            occ += (ok[b] && ds[b] <= zqs[b] - c.bias) ? sm : 0.0f;
        }
    }
    stf(out, o, 1.0f - occ * c.inv_n);
}

template <typename TA>
__global__ void __launch_bounds__(kTx *kTy) k_ssao_blur(const float *__restrict__ hdepth,
                                                        const float *__restrict__ raw, int Wh, int Hh, float tau,
                                                        int tiles_x, int tiles, TA *__restrict__ out) {
    constexpr int LW = kTx + 3, LH = kTy + 3;  // offsets -2 .. +1
    __shared__ float sd[LH][LW];
    __shared__ float sa[LH][LW];
    int tile = xcd_tile(blockIdx.x, tiles);
    int i0 = (tile % tiles_x) * kTx, j0 = (tile / tiles_x) * kTy;
    for (int q = threadIdx.x; q < LW * LH; q += blockDim.x) {
        int li = q % LW, lj = q / LW;
        int gi = i0 + li - 2, gj = j0 + lj - 2;
        bool in = gi >= 0 && gi < Wh && gj >= 0 && gj < Hh;
        size_t g = (size_t)gj * Wh + gi;
        sd[lj][li] = in ? hdepth[g] : __builtin_inff();  // out of range: weight 0
        sa[lj][li] = in ? raw[g] : 0.0f;
    }
    __syncthreads();
    int ti = threadIdx.x % kTx, tj = threadIdx.x / kTx;
    int i = i0 + ti, j = j0 + tj;
    if (i >= Wh || j >= Hh) return;
    float dp = sd[tj + 2][ti + 2];
    float v = 1.0f;
    if (!__builtin_isinf(dp)) {
        float inv = 1.0f / (tau * dp);
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
    st(out + (size_t)j * Wh + i, v);
}

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

template <typename TG, typename TA>
static void launch_raw(const SsaoPlan &q, SsaoConst c, const float *depth, const void *normal,
                       const float *hdepth, const float *kernel, const float *noise, void *out, hipStream_t s) {
    hipLaunchKernelGGL((k_ssao_raw<TG, TA>), dim3(c.tiles), dim3(kTx * kTy), 0, s, c, depth, (const TG *)normal,
                       hdepth, kernel, noise, (TA *)out);
}

hipError_t launch_ssao(const SsaoPlan &q, const float *depth, const void *normal, epb_dtype gdtype,
                       const HostCam &cam, const float *kernel, int n_samples, const float *noise, float radius,
                       float bias, float tau, int blur, void *ao_out, epb_dtype ao_dtype, void *scratch,
                       hipStream_t s) {
    char *sc = (char *)scratch;
    float *hdepth = (float *)(sc + q.off_hdepth);
    float *raw = (float *)(sc + q.off_raw);
    hipLaunchKernelGGL(k_ssao_prep, dim3((q.Wh + 255) / 256, q.Hh), dim3(256), 0, s, depth, q.W, q.Wh, q.Hh, hdepth);
    SsaoConst c{};
    for (int k = 0; k < 9; ++k) c.cam.R[k] = cam.R[k];
    for (int k = 0; k < 3; ++k) c.cam.t[k] = cam.t[k];
    c.cam.fx = cam.fx; c.cam.fy = cam.fy; c.cam.cx = cam.cx; c.cam.cy = cam.cy;
    c.cam.inv_fx = cam.inv_fx; c.cam.inv_fy = cam.inv_fy;
    c.cam.w = cam.w; c.cam.h = cam.h;
    c.radius = radius;
    c.bias = bias;
    c.n = n_samples;
    c.inv_n = 1.0f / (float)n_samples;
    c.W = q.W; c.H = q.H; c.Wh = q.Wh; c.Hh = q.Hh;
    c.tiles_x = (q.Wh + kTx - 1) / kTx;
    c.tiles = c.tiles_x * ((q.Hh + kTy - 1) / kTy);
    // raw AO goes to scratch when blurred, straight to the output otherwise
    bool direct = !blur;
    void *raw_dst = direct ? ao_out : (void *)raw;
    epb_dtype raw_dt = direct ? ao_dtype : EPB_F32;
    if (gdtype == EPB_F32) {
        if (raw_dt == EPB_F32) launch_raw<float, float>(q, c, depth, normal, hdepth, kernel, noise, raw_dst, s);
        else launch_raw<float, __half>(q, c, depth, normal, hdepth, kernel, noise, raw_dst, s);
    } else {
        if (raw_dt == EPB_F32) launch_raw<__half, float>(q, c, depth, normal, hdepth, kernel, noise, raw_dst, s);
        else launch_raw<__half, __half>(q, c, depth, normal, hdepth, kernel, noise, raw_dst, s);
    }
    if (!direct) {
        if (ao_dtype == EPB_F32)
            hipLaunchKernelGGL(k_ssao_blur<float>, dim3(c.tiles), dim3(kTx * kTy), 0, s, hdepth, raw, q.Wh, q.Hh,
                               tau, c.tiles_x, c.tiles, (float *)ao_out);
        else
            hipLaunchKernelGGL(k_ssao_blur<__half>, dim3(c.tiles), dim3(kTx * kTy), 0, s, hdepth, raw, q.Wh, q.Hh,
                               tau, c.tiles_x, c.tiles, (__half *)ao_out);
    }
    return hipGetLastError();
}

}  // namespace epb
