// Compose pass (paper Sec. 4.2): position from depth (Sec. 4), Cook-Torrance
// direct lighting in the Unreal Engine 4 variant (Sec. 3) with 3x3
// percentage-closer shadow tests (Sec. 5.1), split-sum image-based lighting
// with multiple-scattering compensation (Sec. 3.1) scaled by ambient
// occlusion (Sec. 5.2), environment behind the scene.
//
// gfx950 mapping: one thread per pixel, 32x8 pixel tiles (a wavefront covers
// 32x2 pixels: two 128-byte row segments of every planar G-buffer channel),
// consecutive tiles on the same XCD so that the shadow-map and IBL texels a
// band of rows touches stay in that XCD's L2.  Lights travel in the kernel
// argument segment and are read with scalar loads.
//
// Float32 care where the reference is float64:
//  * GGX: 1 - (N.H)^2 is taken as |N x H|^2, exact to rounding near the
//    highlight peak where the subtraction would cancel (roughness 0.05 gives
//    alpha^2 = 6e-6).
//  * Smith-Schlick visibility G / (4 N.L N.V) is evaluated as
//    1 / (4 (N.L(1-k)+k)(N.V(1-k)+k)): no division by a clamped N.V.
//  * The view vector is -normalize(R^T P_view), free of the cancellation of
//    camera_position - world_position for distant pixels.
#include "device_common.hpp"
#include "launch.hpp"

namespace epb {

constexpr int kShTx = 32, kShTy = 8;

struct DevLight {
    float pos[3], rad[3];
    const float *map;
    float M[9], o[3];  // light view from camera view: P_l = M P_v + o
    float fx, fy, cx, cy;
    int w, h;
    float bias;
};

struct ShadeK {
    const float *depth;
    const void *normal, *albedo, *rough, *metal;
    const void *ao;
    void *hdr;
    const float4 *irr, *pref, *env;
    const float2 *lut;
    float R[9];
    float cam_pos[3];
    float cx, cy, inv_fx, inv_fy;
    int W, H, Wh, Hh;
    int tiles_x, tiles;
    int irr_size, pref_base, pref_levels, lut_size, env_size;
    int pref_off[8];
    int n_lights;
    DevLight lights[EPB_MAX_LIGHTS];
};

__device__ __forceinline__ float2 lut_bilinear(const float2 *__restrict__ lut, int size, float u, float v) {
    float fx = fmaf(u, (float)size, -0.5f), fy = fmaf(v, (float)size, -0.5f);
    float x0f = floorf(fx), y0f = floorf(fy);
    float wx = fx - x0f, wy = fy - y0f;
    int x0 = (int)x0f, y0 = (int)y0f;
    int xa = min(max(x0, 0), size - 1), xb = min(max(x0 + 1, 0), size - 1);
    int ya = min(max(y0, 0), size - 1), yb = min(max(y0 + 1, 0), size - 1);
    float2 a = lut[ya * size + xa], b = lut[ya * size + xb];
    float2 c = lut[yb * size + xa], d = lut[yb * size + xb];
    float ax = fmaf(wx, b.x - a.x, a.x), ay = fmaf(wx, b.y - a.y, a.y);
    float cx = fmaf(wx, d.x - c.x, c.x), cy = fmaf(wx, d.y - c.y, c.y);
    return make_float2(fmaf(wy, cx - ax, ax), fmaf(wy, cy - ay, ay));
}

// Lit fraction of the 3x3 patch around the projection of view point Pv.
// The nine taps are fetched at clamped (always valid) addresses with no
// branch between them, so they are in flight together; taps outside the map
// and points outside the light frustum are lit.
__device__ __forceinline__ float pcf(const DevLight &L, v3 Pv) {
    v3 Pl = mul_R(L.M, Pv) + mk3(L.o[0], L.o[1], L.o[2]);
    float dl = -Pl.z;
    float idl = rcp(dl);
    float u = fmaf(L.fx * Pl.x, idl, L.cx);
    float v = fmaf(-L.fy * Pl.y, idl, L.cy);
    bool inside = dl > 0.0f && u >= 0.0f && u < (float)L.w && v >= 0.0f && v < (float)L.h;
    int i0 = (int)fminf(fmaxf(u, 0.0f), (float)(L.w - 1));  // == floor(u) when inside
    int j0 = (int)fminf(fmaxf(v, 0.0f), (float)(L.h - 1));
    float ref = dl - L.bias;
    float tap[9];
    bool in[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        int ti = i0 + k % 3 - 1, tj = j0 + k / 3 - 1;
        in[k] = ti >= 0 && ti < L.w && tj >= 0 && tj < L.h;
        int ci = min(max(ti, 0), L.w - 1), cj = min(max(tj, 0), L.h - 1);
        tap[k] = L.map[(size_t)cj * L.w + ci];
    }
    int lit = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) lit += (!in[k] || ref <= tap[k]) ? 1 : 0;
    return inside ? (float)lit * (1.0f / 9.0f) : 1.0f;
}

template <typename TG, typename TA, typename TH>
__global__ void __launch_bounds__(kShTx *kShTy) k_shade(const ShadeK c) {
    int tile = xcd_tile(blockIdx.x, c.tiles);
    int x = (tile % c.tiles_x) * kShTx + (int)(threadIdx.x % kShTx);
    int y = (tile / c.tiles_x) * kShTy + (int)(threadIdx.x / kShTx);
    if (x >= c.W || y >= c.H) return;
    size_t p = (size_t)y * c.W + x;
    size_t plane = (size_t)c.W * c.H;
    float d = c.depth[p];
    float dvx = ((float)x + 0.5f - c.cx) * c.inv_fx;
    float dvy = -((float)y + 0.5f - c.cy) * c.inv_fy;
    float out[3];
    if (__builtin_isinf(d)) {
        v3 dw = mul_Rt(c.R, mk3(dvx, dvy, -1.0f));
        float4 e = cube_bilinear(c.env, c.env_size, dw);
        out[0] = e.x; out[1] = e.y; out[2] = e.z;
    } else {
        const TG *nrm = (const TG *)c.normal, *alb = (const TG *)c.albedo;
        v3 Pv = mk3(dvx * d, dvy * d, -d);
        v3 Pr = mul_Rt(c.R, Pv);  // world position relative to the camera
        v3 Pw = Pr + mk3(c.cam_pos[0], c.cam_pos[1], c.cam_pos[2]);
        v3 V = normalize(mk3(-Pr.x, -Pr.y, -Pr.z));
        v3 n = normalize(mk3(ldc(nrm + p), ldc(nrm + plane + p), ldc(nrm + 2 * plane + p)));
        float a[3] = {ldc(alb + p), ldc(alb + plane + p), ldc(alb + 2 * plane + p)};
        float r = ldc((const TG *)c.rough + p);
        float mt = ldc((const TG *)c.metal + p);
        float nv_raw = dot(n, V);
        float NoV = fminf(fmaxf(nv_raw, 1e-4f), 1.0f);
        float F0[3], cd[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            F0[ch] = fmaf(mt, a[ch] - 0.04f, 0.04f);
            cd[ch] = a[ch] * (1.0f - mt);
        }
        float alpha = r * r, a2 = alpha * alpha;
        float kd = (r + 1.0f) * (r + 1.0f) * 0.125f;
        float gv = fmaf(NoV, 1.0f - kd, kd);
        // ambient inputs first: their gathers overlap the direct-light math
        float2 AB = lut_bilinear(c.lut, c.lut_size, NoV, r);
        float4 E = cube_bilinear(c.irr, c.irr_size, n);
        v3 Rf = n * (2.0f * nv_raw) - V;
        float lod = fminf(fmaxf(r * (float)(c.pref_levels - 1), 0.0f), (float)(c.pref_levels - 1));
        int l0 = (int)lod;
        int l1 = min(l0 + 1, c.pref_levels - 1);
        float fl = lod - (float)l0;
        FaceST fs = cube_face(Rf);
        float4 P0 = face_bilinear(c.pref + c.pref_off[l0], c.pref_base >> l0, fs);
        float4 P1 = face_bilinear(c.pref + c.pref_off[l1], c.pref_base >> l1, fs);
        float ao = 1.0f;
        if (c.ao) {
            const TA *aop = (const TA *)c.ao;
            int x0 = x >> 1, y0 = y >> 1;
            int x1 = min(x0 + 1, c.Wh - 1), y1 = min(y0 + 1, c.Hh - 1);
            float wx = (x & 1) ? 0.5f : 0.0f, wy = (y & 1) ? 0.5f : 0.0f;
            float a00 = ldc(aop + (size_t)y0 * c.Wh + x0), a10 = ldc(aop + (size_t)y0 * c.Wh + x1);
            float a01 = ldc(aop + (size_t)y1 * c.Wh + x0), a11 = ldc(aop + (size_t)y1 * c.Wh + x1);
            float top = fmaf(wx, a10 - a00, a00), bot = fmaf(wx, a11 - a01, a01);
            ao = fmaf(wy, bot - top, top);
        }
        // direct light
        float Lo[3] = {0.0f, 0.0f, 0.0f};
        for (int li = 0; li < c.n_lights; ++li) {
            const DevLight &L = c.lights[li];
            v3 lv = mk3(L.pos[0], L.pos[1], L.pos[2]) - Pw;
            float dist2 = dot(lv, lv);
            float il = rsq(dist2);
            v3 l = lv * il;
            float NoL = dot(n, l);
            if (!(NoL > 0.0f)) continue;
            float sh = L.map ? pcf(L, Pv) : 1.0f;
            v3 h = normalize(V + l);
            float NoH = dot(n, h);
            float VoH = fmaxf(dot(V, h), 0.0f);
            v3 nxh = cross(n, h);
            float q = fmaf(NoH * NoH, a2, dot(nxh, nxh));
            float D = a2 * rcp(kPi * q * q);
            float vis = 0.25f * rcp(fmaf(NoL, 1.0f - kd, kd) * gv);
            float spec = D * vis;
            float fc = pow5(1.0f - VoH);
            float e = il * il * NoL * sh;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float F = fmaf(1.0f - F0[ch], fc, F0[ch]);
                float f = fmaf(spec, F, cd[ch] * (1.0f / kPi));
                Lo[ch] = fmaf(f, L.rad[ch] * e, Lo[ch]);
            }
        }
        float4 P = lerp4(P0, P1, fl);
        float fc5 = pow5(1.0f - NoV);
        float Pc[3] = {P.x, P.y, P.z}, Ec[3] = {E.x, E.y, E.z};
        float Ess = AB.x + AB.y, Ems = 1.0f - Ess;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float kS = fmaf(fmaxf(1.0f - r, F0[ch]) - F0[ch], fc5, F0[ch]);
            float FssEss = fmaf(kS, AB.x, AB.y);
            float Favg = fmaf(1.0f - F0[ch], 1.0f / 21.0f, F0[ch]);
            float Fms = FssEss * Favg * rcp(1.0f - Ems * Favg);
            float msE = Fms * Ems;
            float kD = cd[ch] * (1.0f - FssEss - msE);
            float amb = fmaf(FssEss, Pc[ch], (msE + kD) * Ec[ch]);
            out[ch] = fmaf(ao, amb, Lo[ch]);
        }
    }
    TH *hdr = (TH *)c.hdr;
    st(hdr + p, out[0]);
    st(hdr + plane + p, out[1]);
    st(hdr + 2 * plane + p, out[2]);
}

template <typename TG, typename TA, typename TH>
static void go(const ShadeK &k, hipStream_t s) {
    hipLaunchKernelGGL((k_shade<TG, TA, TH>), dim3(k.tiles), dim3(kShTx * kShTy), 0, s, k);
}
template <typename TG, typename TA>
static void go_h(const ShadeK &k, epb_dtype hd, hipStream_t s) {
    if (hd == EPB_F32) go<TG, TA, float>(k, s);
    else go<TG, TA, __half>(k, s);
}
template <typename TG>
static void go_a(const ShadeK &k, epb_dtype ad, epb_dtype hd, hipStream_t s) {
    if (ad == EPB_F32) go_h<TG, float>(k, hd, s);
    else go_h<TG, __half>(k, hd, s);
}

hipError_t launch_shade(const ShadeArgs &a, hipStream_t s) {
    ShadeK k{};
    k.depth = a.depth;
    k.normal = a.normal; k.albedo = a.albedo; k.rough = a.rough; k.metal = a.metal;
    k.ao = a.ao;
    k.hdr = a.hdr;
    k.irr = (const float4 *)a.irr;
    k.pref = (const float4 *)a.pref;
    k.env = (const float4 *)a.env;
    k.lut = (const float2 *)a.lut;
    for (int i = 0; i < 9; ++i) k.R[i] = a.cam.R[i];
    for (int i = 0; i < 3; ++i) k.cam_pos[i] = a.cam_pos[i];
    k.cx = a.cam.cx; k.cy = a.cam.cy; k.inv_fx = a.cam.inv_fx; k.inv_fy = a.cam.inv_fy;
    k.W = a.W; k.H = a.H; k.Wh = (a.W + 1) / 2; k.Hh = (a.H + 1) / 2;
    k.tiles_x = (a.W + kShTx - 1) / kShTx;
    k.tiles = k.tiles_x * ((a.H + kShTy - 1) / kShTy);
    k.irr_size = a.irr_size; k.pref_base = a.pref_base; k.pref_levels = a.pref_levels;
    k.lut_size = a.lut_size; k.env_size = a.env_size;
    int off = 0;
    for (int m = 0; m < 8; ++m) {
        k.pref_off[m] = off;
        if (m < a.pref_levels) off += 6 * (a.pref_base >> m) * (a.pref_base >> m);
    }
    k.n_lights = a.n_lights;
    for (int i = 0; i < a.n_lights; ++i) {
        const HostLight &h = a.lights[i];
        DevLight &d = k.lights[i];
        for (int j = 0; j < 3; ++j) { d.pos[j] = h.pos[j]; d.rad[j] = h.rad[j]; d.o[j] = h.o[j]; }
        for (int j = 0; j < 9; ++j) d.M[j] = h.M[j];
        d.map = h.map;
        d.fx = h.fx; d.fy = h.fy; d.cx = h.cx; d.cy = h.cy;
        d.w = h.w; d.h = h.h;
        d.bias = h.bias;
    }
    if (a.gdtype == EPB_F32) go_a<float>(k, a.ao_dtype, a.hdr_dtype, s);
    else go_a<__half>(k, a.ao_dtype, a.hdr_dtype, s);
    return hipGetLastError();
}

}  // namespace epb
