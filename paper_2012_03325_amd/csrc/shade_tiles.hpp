// Per-tile device functions of the shading pass (paper Sec. 3, 3.1, 4, 5.1):
// PCF, one pixel's radiance and the optional bloom level-1 epilogue; shared by
// the single-view, batched and persistent kernels.
#pragma once

#include "device_common.hpp"

namespace epb {

struct Row3 {
    float v[3];
};

// Bilinear lookup of the (size >= 2) BRDF table, clamp to edge (sizes as for
// a cube face: the table is one size x size face).
__device__ __forceinline__ float2 lut_bilinear(const float2 *__restrict__ lut, const FaceDims &g, float u, float v) {
    float fsize = (float)g.S;
    float fx = clamp_to(fmaf(u, fsize, -0.5f), g.hi);
    float fy = clamp_to(fmaf(v, fsize, -0.5f), g.hi);
    float x0f = fminf(floorf(fx), g.hi1), y0f = fminf(floorf(fy), g.hi1);
    float wx = fx - x0f, wy = fy - y0f;
    unsigned o0 = (__umul24((unsigned)y0f, (unsigned)g.S) + (unsigned)x0f) * 8u;
    unsigned o1 = o0 + (unsigned)g.S * 8u;
    float2 a = ldo(lut, o0), b = ldo(lut + 1, o0), c = ldo(lut, o1), d = ldo(lut + 1, o1);
    float ax = fmaf(wx, b.x - a.x, a.x), ay = fmaf(wx, b.y - a.y, a.y);
    float cx = fmaf(wx, d.x - c.x, c.x), cy = fmaf(wx, d.y - c.y, c.y);
    return make_float2(fmaf(wy, cx - ax, ax), fmaf(wy, cy - ay, ay));
}

// Lit fraction of the 3x3 patch around the projection of view point Pv
// (maps of at least 3x3); points outside the light's frustum are lit.
//
// Tiled form: the map is padded with a +inf (lit) apron, so the patch of any
// point that projects inside the map, top-left texel (i0 - 1, j0 - 1), is the
// block at padded coordinates (i0, j0) and lies inside one 8x8 stored block
// (tile (j0 / 6, i0 / 6)); its rows sit at fixed +32/+64-byte offsets, taken
// from the base pointer so that they fold into the load instructions.  A point
// outside the map or behind the light reads the form's all-+inf tile: all nine
// taps lit, no border case and no select of the result.
//
// Row-major form: one 3x3 block that lies wholly inside the map is fetched
// through three row loads (fixed +1/+2 column offsets, all nine loads in
// flight together); when the true patch sticks out of the map the block is
// shifted inwards by one texel and the columns/rows that do not belong to the
// patch are dropped, the missing taps counting as lit.
__device__ __forceinline__ float pcf(const DevLight &L, float dvx, float dvy, float d) {
    // M P_v + o = ((u - cx) d_l, (v - cy) d_l, -d_l) with P_v = d (dvx, dvy, -1)
    v3 Md = mk3(fmaf(L.M[0], dvx, fmaf(L.M[1], dvy, -L.M[2])), fmaf(L.M[3], dvx, fmaf(L.M[4], dvy, -L.M[5])),
                fmaf(L.M[6], dvx, fmaf(L.M[7], dvy, -L.M[8])));
    v3 Pl = mk3(fmaf(Md.x, d, L.o[0]), fmaf(Md.y, d, L.o[1]), fmaf(Md.z, d, L.o[2]));
    float dl = -Pl.z;
    float idl = rcp(dl);
    float u = fmaf(Pl.x, idl, L.cx);
    float v = fmaf(Pl.y, idl, L.cy);
    float ref = dl - L.bias;
    const Row3 *map = reinterpret_cast<const Row3 *>(L.map);
    if (L.tiles) {
        // floor-convert: 0 <= u < w exactly when 0 <= floor(u) < w (one unsigned
        // compare; +-inf saturate outside; u is finite whenever d_l > 0)
        int i0 = floor_to_int(u), j0 = floor_to_int(v);
        bool inside = dl > 0.0f && (unsigned)i0 < (unsigned)L.w && (unsigned)j0 < (unsigned)L.h;
        unsigned x = (unsigned)i0, y = (unsigned)j0;
        unsigned tq = __umulhi(x, 0x2AAAAAABu), tp = __umulhi(y, 0x2AAAAAABu);  // x / 6, y / 6 (exact below 2^31)
        unsigned q0 = inside ? __umul24(tp, L.tile_pitch) + __umul24(tq, 232u) + y * 32u + x * 4u : L.sentinel;
        const char *base = reinterpret_cast<const char *>(L.map);  // wave-uniform: the row offsets are scalar adds
        Row3 a = ldo(map, q0), b = ldo(reinterpret_cast<const Row3 *>(base + 32), q0),
             e = ldo(reinterpret_cast<const Row3 *>(base + 64), q0);
        float t[9] = {a.v[0], a.v[1], a.v[2], b.v[0], b.v[1], b.v[2], e.v[0], e.v[1], e.v[2]};
        int lit = 0;
#pragma unroll
        for (int k = 0; k < 9; ++k) lit += t[k] < ref ? 0 : 1;  // lit iff ref <= t
        return (float)lit * (1.0f / 9.0f);
    }
    bool inside = dl > 0.0f && u >= 0.0f && u < L.fw && v >= 0.0f && v < L.fh;
    int i0 = inside ? (int)u : 1, j0 = inside ? (int)v : 1;  // truncation == floor when inside
    int bi = min(max(i0, 1), L.w - 2), bj = min(max(j0, 1), L.h - 2);
    // three 12-byte row loads (dword aligned) cover the 3x3 block
    unsigned q0 = (__umul24((unsigned)(bj - 1), (unsigned)L.w) + (unsigned)(bi - 1)) * 4u;
    unsigned row = (unsigned)L.w * 4u;
    Row3 a = ldo(map, q0), b = ldo(map, q0 + row), e = ldo(map, q0 + 2u * row);
    float t[9] = {a.v[0], a.v[1], a.v[2], b.v[0], b.v[1], b.v[2], e.v[0], e.v[1], e.v[2]};
    int lit = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) lit += ref <= t[k] ? 1 : 0;
    int si = i0 - bi, sj = j0 - bj;  // -1, 0 or +1; non-zero only next to the map border
    if (si | sj) {
        bool kc[3] = {si <= 0, true, si >= 0};
        bool kr[3] = {sj <= 0, true, sj >= 0};
        int nc = 1 + (si <= 0) + (si >= 0), nr = 1 + (sj <= 0) + (sj >= 0);
        lit = 9 - nc * nr;  // taps outside the map
#pragma unroll
        for (int k = 0; k < 9; ++k) lit += (kr[k / 3] && kc[k % 3] && ref <= t[k]) ? 1 : 0;
    }
    return inside ? (float)lit * (1.0f / 9.0f) : 1.0f;
}

// One pixel's radiance: shading of the surface, or the environment behind it.
template <typename TG, typename TA, typename TH>
__device__ __forceinline__ void shade_pixel(const ShadeDesc &c, int x, int y, float (&out)[3]) {
    unsigned p = __umul24((unsigned)y, (unsigned)c.W) + (unsigned)x;
    unsigned plane = (unsigned)c.W * (unsigned)c.H;
    float d = ldf(c.depth, p);
    float dvx = ((float)x + 0.5f - c.cx) * c.inv_fx;
    float dvy = -((float)y + 0.5f - c.cy) * c.inv_fy;
    if (__builtin_isinf(d)) {
        v3 dw = mul_Rt(c.R, mk3(dvx, dvy, -1.0f));
        float4 e = cube_bilinear(c.env, c.env_dims, dw);
        out[0] = e.x; out[1] = e.y; out[2] = e.z;
    } else {
        const TG *nrm = (const TG *)c.normal, *alb = (const TG *)c.albedo;
        v3 Pv = mk3(dvx * d, dvy * d, -d);
        v3 Pr = mul_Rt(c.R, Pv);  // world position relative to the camera
        v3 Pw = Pr + mk3(c.cam_pos[0], c.cam_pos[1], c.cam_pos[2]);
        v3 V = normalize(mk3(-Pr.x, -Pr.y, -Pr.z));
        v3 n = normalize(mk3(ldf(nrm, p), ldf(nrm, plane + p), ldf(nrm, 2 * plane + p)));
        float a[3] = {ldf(alb, p), ldf(alb, plane + p), ldf(alb, 2 * plane + p)};
        float r = ldf((const TG *)c.rough, p);
        float mt = ldf((const TG *)c.metal, p);
        if (c.weight) {  // surfel G-buffer: accumulated attributes over their weight
            float w = ldf((const TG *)c.weight, p);
            if (w > 0.0f) {
                float iw = rcp(w);
                a[0] *= iw; a[1] *= iw; a[2] *= iw;
                r *= iw;
                mt *= iw;
            }
        }
        float nv_raw = dot(n, V);
        float NoV = __builtin_amdgcn_fmed3f(nv_raw, 1e-4f, 1.0f);
        float F0[3], cd[3], omF0[3], cdpi[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            F0[ch] = fmaf(mt, a[ch] - 0.04f, 0.04f);
            cd[ch] = a[ch] * (1.0f - mt);
            omF0[ch] = 1.0f - F0[ch];
            cdpi[ch] = cd[ch] * (1.0f / kPi);
        }
        float alpha = r * r, a2 = alpha * alpha;
        float kd = (r + 1.0f) * (r + 1.0f) * 0.125f;
        float gv = fmaf(NoV, 1.0f - kd, kd);
        float ao = 1.0f;
        if (c.ao) {
            const TA *aop = (const TA *)c.ao;
            unsigned x0 = x >> 1, y0 = y >> 1;
            unsigned dx = (x & 1) && (int)x0 + 1 < c.Wh ? 1u : 0u;
            unsigned dy = (y & 1) && (int)y0 + 1 < c.Hh ? (unsigned)c.Wh : 0u;
            unsigned q = __umul24(y0, (unsigned)c.Wh) + x0;
            float a00 = ldf(aop, q), a10 = ldf(aop, q + dx), a01 = ldf(aop, q + dy), a11 = ldf(aop, q + dy + dx);
            float wx = (x & 1) ? 0.5f : 0.0f, wy = (y & 1) ? 0.5f : 0.0f;
            float top = fmaf(wx, a10 - a00, a00), bot = fmaf(wx, a11 - a01, a01);
            ao = fmaf(wy, bot - top, top);
        }
        // direct light
        float Lo[3] = {0.0f, 0.0f, 0.0f};
        for (int li = 0; li < c.n_lights; ++li) {
            const DevLight L = c.lights[li];  // a copy: its fields load into scalar registers together
            v3 lv = mk3(L.pos[0], L.pos[1], L.pos[2]) - Pw;
            float dist2 = dot(lv, lv);
            float il = rsq(dist2);
            float NoL = dot(n, lv) * il;  // (l = lv il is never formed)
            if (!(NoL > 0.0f)) continue;
            float sh = L.map ? pcf(L, dvx, dvy, d) : 1.0f;
            // The half vector h = s / |s| is never formed: with s = V + l (both unit
            // vectors) N.H = (N.V + N.L) / |s|, 1 - (N.H)^2 = |s - (n.s) n|^2 / |s|^2
            // (the part of s off the normal, no cancellation at the peak) and
            // V.H = |s| / 2, so the GGX denominator q = (N.H)^2 alpha^2 + 1 - (N.H)^2
            // is qs / |s|^2 with qs = (n.s)^2 alpha^2 + |s - (n.s) n|^2.
            v3 sv = mk3(fmaf(lv.x, il, V.x), fmaf(lv.y, il, V.y), fmaf(lv.z, il, V.z));
            float s2 = dot(sv, sv);
            float ns = nv_raw + NoL;
            v3 sp = mk3(fmaf(-ns, n.x, sv.x), fmaf(-ns, n.y, sv.y), fmaf(-ns, n.z, sv.z));
            float qs = fmaf(ns * ns, a2, dot(sp, sp));
            // D * G / (4 NoL NoV) = alpha^2 / (pi q^2) * 1 / (4 (NoL(1-k)+k)(NoV(1-k)+k))
            float spec = (0.25f / kPi) * a2 * (s2 * s2) * rcp(qs * qs * fmaf(NoL, 1.0f - kd, kd) * gv);
            float fc = pow5(fmaf(-0.5f, __builtin_amdgcn_sqrtf(s2), 1.0f));  // (1 - V.H)^5
            float e = il * il * NoL * sh;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float F = fmaf(omF0[ch], fc, F0[ch]);
                float f = fmaf(spec, F, cdpi[ch]);
                Lo[ch] = fmaf(f, L.rad[ch] * e, Lo[ch]);
            }
        }
        // ambient inputs after the light loop: gathered before it, their taps would stay live
        // through the loop (123 VGPRs, 4 waves/SIMD); here the kernel needs 65 (7 waves/SIMD)
        float2 AB = lut_bilinear(c.lut, c.lut_dims, NoV, r);
        float4 E = cube_bilinear(c.irr, c.irr_dims, n);
        v3 Rf = n * (2.0f * nv_raw) - V;
        float lod = clamp_to(r * c.f_levels1, c.f_levels1);
        int l0 = (int)lod;
        int l1 = min(l0 + 1, c.pref_levels - 1);
        float fl = lod - (float)l0;
        FaceST fs = cube_face(Rf);
        int s0 = c.pref_base >> l0, s1 = c.pref_base >> l1;
        float4 P0 = face_bilinear(c.pref, c.pref_off[l0], face_dims(s0), fs);
        float4 P1 = face_bilinear(c.pref, c.pref_off[l1], face_dims(s1), fs);
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
    stf(hdr, p, out[0]);
    stf(hdr, plane + p, out[1]);
    stf(hdr, 2 * plane + p, out[2]);
}

// Level 1 of the bloom pyramid from the shaded pixels of this wave: the texel
// (x / 2, y / 2) is the mean of the bright-pass values of its in-image 2x2
// children, summed as horizontal pairs, then the two rows (the order of the
// unfused bloom pass, so the two agree bitwise), from the HDR values as
// stored.  A TX-wide tile (TX = 16 or 32) puts rows 2k and 2k + 1 of a tile in
// one wave, at lanes l and l ^ TX; every lane of the wave takes part.
template <int TX, typename TH>
__device__ __forceinline__ void bloom1_epilogue(const ShadeDesc &c, int x, int y, bool in, const float (&o)[3]) {
    float cr = 0.0f, cg = 0.0f, cb = 0.0f;
    if (in) {
        float r = stored_as(o[0], (const TH *)nullptr), g = stored_as(o[1], (const TH *)nullptr),
              b = stored_as(o[2], (const TH *)nullptr);
        float sc = bright_scale(r, g, b, c.bloom_threshold);
        cr = r * sc;
        cg = g * sc;
        cb = b * sc;
    }
    cr = add_row_pair<TX>(add_lane_pair(cr));
    cg = add_row_pair<TX>(add_lane_pair(cg));
    cb = add_row_pair<TX>(add_lane_pair(cb));
    if (in && !(x & 1) && !(y & 1)) {
        float inv_n = (x + 1 < c.W ? 0.5f : 1.0f) * (y + 1 < c.H ? 0.5f : 1.0f);
        unsigned t = __umul24((unsigned)(y >> 1), (unsigned)c.Wh) + (unsigned)(x >> 1);
        float4 v = make_float4(cr * inv_n, cg * inv_n, cb * inv_n, 0.0f);
        if (c.bloom1_half) sto((Half4 *)c.bloom1, t * 8u, pack_half4(v));
        else sto((float4 *)c.bloom1, t * 16u, v);
    }
}

template <int TX, int TY, bool kBloom1, typename TG, typename TA, typename TH>
__device__ __forceinline__ void shade_tile(const ShadeDesc &c, int tile) {
    int tiles_x = (c.W + TX - 1) / TX;
    int ty = tile / tiles_x;
    int x = (tile - ty * tiles_x) * TX + (int)(threadIdx.x % TX);
    int y = ty * TY + (int)(threadIdx.x / TX);
    bool in = x < c.W && y < c.H;
    float out[3] = {0.0f, 0.0f, 0.0f};
    // (with kBloom1 every lane reaches the epilogue; otherwise out-of-image lanes leave here)
    if (!kBloom1 && !in) return;
    if (in) shade_pixel<TG, TA, TH>(c, x, y, out);
    if constexpr (kBloom1) {
        if (c.bloom1) bloom1_epilogue<TX, TH>(c, x, y, in, out);  // (uniform: null for a view without bloom)
    }
}

}  // namespace epb
