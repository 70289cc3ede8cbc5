// Image-based-lighting precompute (paper Sec. 3.1): a solid-angle-weighted
// average of the environment, the diffuse irradiance map, the split-sum
// prefiltered specular chain and the environment BRDF table.
//
// gfx950 mapping:
//  * irradiance: 6*32^2 outputs x 6*64^2 source texels.  One thread per
//    output, source texels staged through LDS in blocks of 256 and broadcast
//    to all lanes; the source range is split across workgroups so that the
//    grid gives every CU about four, and the per-split Kahan partials are combined in
//    a fixed order by a second kernel (deterministic, no atomics).
//  * a GGX sample's tangent-frame half vector depends on the sample and the
//    roughness only, and its square roots, reciprocal and sine/cosine are most
//    of a sample's instructions, so it is made once per level (prefilter) or
//    per table row (BRDF table) and only turned into each texel's frame.
//  * prefilter from the full-resolution environment: one wavefront per output
//    texel, the 64 lanes split the samples, whose taps then stay within the
//    texel's GGX lobe (a few cache lines at the rough levels' narrow lobes);
//    per-lane Kahan sums, compensated wave reduction through cross-lane
//    shuffles; a lane takes two samples at a time (both lookups' taps in
//    flight), their half vectors from the level's table one iteration ahead,
//    the taps from a packed RGB copy of the environment (the texture data path
//    bounds this kernel, and the fourth channel is never used).
//  * prefilter with filtered importance sampling (taps on the mip level that
//    matches each sample's footprint): one wavefront per 8x8 tile of output
//    texels and chunk of the samples; all lanes take the same sample at once,
//    so its half vector is a uniform (scalar) table load and neighbouring
//    texels' taps share cache lines; per-lane Kahan sums per chunk, the chunks
//    added in a fixed order by a second kernel (deterministic, no atomics).
//  * BRDF table: one wavefront per entry, the 64 lanes split the Hammersley
//    samples (per-lane Kahan sums, compensated wave reduction through
//    cross-lane shuffles); a block makes its row's half vectors into LDS, and
//    a lane Kahan-adds its (non-negative) terms four at a time.
//  * roughness-0 prefilter level: every GGX half vector equals the normal, so
//    the N.L-weighted mean is the environment along the texel direction; one
//    bilinear lookup per texel.
#include <cmath>

#include "device_common.hpp"
#include "launch.hpp"

namespace epb {

// Solid angle of texel (i, j) of a face of size S.  The texel is a planar
// quadrilateral at unit distance whose edges project to great circles; split
// along its diagonal into two spherical triangles, each is evaluated with the
// Van Oosterom-Strackee formula tan(W / 2) = |a.(b x c)| / (|a||b||c| +
// (a.b)|c| + (a.c)|b| + (b.c)|a|).  For corners (x0,y0,1), (x1,y0,1),
// (x1,y1,1), (x0,y1,1) the triple products are exactly dx dy and the
// denominators are sums of positive terms, so no cancellation occurs even for
// texels of 1e-5 sr.
__device__ float texel_solid_angle(int i, int j, int S) {
    float inv = 1.0f / (float)S;
    float x0 = (float)(2 * i - S) * inv, x1 = (float)(2 * i + 2 - S) * inv;
    float y0 = (float)(2 * j - S) * inv, y1 = (float)(2 * j + 2 - S) * inv;
    float num = (x1 - x0) * (y1 - y0);
    v3 a = mk3(x0, y0, 1.0f), b = mk3(x1, y0, 1.0f), c = mk3(x1, y1, 1.0f), d = mk3(x0, y1, 1.0f);
    float la = sqrtf(dot(a, a)), lb = sqrtf(dot(b, b)), lc = sqrtf(dot(c, c)), ld_ = sqrtf(dot(d, d));
    float den1 = la * lb * lc + dot(a, b) * lc + dot(a, c) * lb + dot(b, c) * la;
    float den2 = la * lc * ld_ + dot(a, c) * ld_ + dot(a, d) * lc + dot(c, d) * la;
    return 2.0f * (atan2f(num, den1) + atan2f(num, den2));
}

// Compensated sum over aligned segments of `width` lanes (a power of two <= 64):
// Knuth two-sums down a butterfly, the rounding errors carried beside.
__device__ __forceinline__ float segment_sum_compensated(float v, int width) {
    float comp = 0.0f;
    for (int off = width >> 1; off >= 1; off >>= 1) {
        float o = __shfl_xor(v, off, 64);
        float oc = __shfl_xor(comp, off, 64);
        float s, e;
        two_sum(v, o, s, e);
        v = s;
        comp = comp + oc + e;
    }
    return v + comp;
}

// Irradiance source: texel (f, i, j) of size Ss is the solid-angle-weighted mean
// of the k x k environment texels it covers (k = S / Ss).  Because solid angles
// add, this equals repeated 2x2 weighted halving.  Also writes the source
// table entry (unit direction, solid angle at size Ss).
// A segment of lpt lanes (the k x k block rounded up to a power of two, at most
// 64) per source texel: each lane sums its share of the block with Kahan, the
// segment adds the lanes' sums compensated.  lpt is uniform.
__global__ void __launch_bounds__(256) k_ibl_source(const float4 *__restrict__ env, int S, int Ss, int lpt,
                                                    float4 *__restrict__ src, float4 *__restrict__ tab) {
    int t = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    int o = t / lpt, sub = t - o * lpt;
    int nsrc = 6 * Ss * Ss;
    // (the segment stays together: nsrc * lpt threads fill whole segments)
    bool live = o < nsrc;
    int oc = live ? o : nsrc - 1;
    int f = oc / (Ss * Ss), j = (oc / Ss) % Ss, i = oc % Ss;
    int k = S / Ss;
    Kahan r{0, 0}, g{0, 0}, b{0, 0}, w{0, 0};
    const float4 *face = env + (size_t)f * S * S;
    for (int q = sub; q < k * k; q += lpt) {
        int bj = q / k, bi = q - bj * k;
        int ci = i * k + bi, cj = j * k + bj;
        float dw = k == 1 ? 1.0f : texel_solid_angle(ci, cj, S);
        float4 L = face[(size_t)cj * S + ci];
        kahan_add(r, L.x * dw);
        kahan_add(g, L.y * dw);
        kahan_add(b, L.z * dw);
        kahan_add(w, dw);
    }
    float R = segment_sum_compensated(kahan_value(r), lpt);
    float G = segment_sum_compensated(kahan_value(g), lpt);
    float Bv = segment_sum_compensated(kahan_value(b), lpt);
    float W = segment_sum_compensated(kahan_value(w), lpt);
    if (live && sub == 0) {
        float iw = 1.0f / W;
        src[o] = make_float4(R * iw, G * iw, Bv * iw, 0.0f);
        v3 d = normalize(cube_texel_dir(f, i, j, Ss));
        tab[o] = make_float4(d.x, d.y, d.z, texel_solid_angle(i, j, Ss));
    }
}

// Partial irradiance sums over source chunk blockIdx.y for 256 outputs.
// part layout: [chunk][output][8] = Kahan (s, c) of R, G, B, weight.
__global__ void __launch_bounds__(256) k_irradiance_partial(const float4 *__restrict__ src,
                                                            const float4 *__restrict__ tab, int nsrc,
                                                            int chunk_len, int irr, float *__restrict__ part) {
    __shared__ float4 sL[256];
    __shared__ float4 sT[256];
    int nout = 6 * irr * irr;
    int o = blockIdx.x * 256 + threadIdx.x;
    v3 n = mk3(0, 0, 1);
    if (o < nout) {
        int f = o / (irr * irr), j = (o / irr) % irr, i = o % irr;
        n = normalize(cube_texel_dir(f, i, j, irr));
    }
    Kahan r{0, 0}, g{0, 0}, b{0, 0}, w{0, 0};
    int beg = blockIdx.y * chunk_len;
    int end = min(beg + chunk_len, nsrc);
    for (int base = beg; base < end; base += 256) {
        int t = base + threadIdx.x;
        if (t < end) {
            sL[threadIdx.x] = src[t];
            sT[threadIdx.x] = tab[t];
        }
        __syncthreads();
        int cnt = min(256, end - base);
        // Every term is >= 0, so a group of four summed in plain float and then
        // Kahan-added keeps the whole sum within about 3 units of rounding of
        // its value (each group's error is bounded by its own terms), as with
        // a Kahan add per term, at a quarter of the compensation work.
        int q = 0;
        for (; q + 4 <= cnt; q += 4) {
            float c[4], lr[4], lg[4], lb[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                float4 T = sT[q + u];
                c[u] = fmaxf(0.0f, fmaf(n.x, T.x, fmaf(n.y, T.y, n.z * T.z))) * T.w;
                float4 L = sL[q + u];
                lr[u] = L.x;
                lg[u] = L.y;
                lb[u] = L.z;
            }
            kahan_add(r, fmaf(lr[3], c[3], fmaf(lr[2], c[2], fmaf(lr[1], c[1], lr[0] * c[0]))));
            kahan_add(g, fmaf(lg[3], c[3], fmaf(lg[2], c[2], fmaf(lg[1], c[1], lg[0] * c[0]))));
            kahan_add(b, fmaf(lb[3], c[3], fmaf(lb[2], c[2], fmaf(lb[1], c[1], lb[0] * c[0]))));
            kahan_add(w, ((c[0] + c[1]) + c[2]) + c[3]);
        }
        for (; q < cnt; ++q) {
            float4 T = sT[q];
            float c = fmaxf(0.0f, fmaf(n.x, T.x, fmaf(n.y, T.y, n.z * T.z))) * T.w;
            float4 L = sL[q];
            kahan_add(r, L.x * c);
            kahan_add(g, L.y * c);
            kahan_add(b, L.z * c);
            kahan_add(w, c);
        }
        __syncthreads();
    }
    if (o < nout) {
        float *p = part + ((size_t)blockIdx.y * nout + o) * 8;
        p[0] = r.s; p[1] = g.s; p[2] = b.s; p[3] = w.s;
        p[4] = r.c; p[5] = g.c; p[6] = b.c; p[7] = w.c;
    }
}

__global__ void __launch_bounds__(256) k_irradiance_final(const float *__restrict__ part, int chunks,
                                                          int irr, float4 *__restrict__ out) {
    int nout = 6 * irr * irr;
    int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= nout) return;
    Kahan acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    // (unrolled: several chunks' loads in flight ahead of the serial adds)
#pragma unroll 8
    for (int c = 0; c < chunks; ++c) {
        const float *p = part + ((size_t)c * nout + o) * 8;
        for (int q = 0; q < 4; ++q) {
            kahan_add(acc[q], p[q]);
            kahan_add(acc[q], -p[4 + q]);
        }
    }
    float iw = 1.0f / kahan_value(acc[3]);
    out[o] = make_float4(kahan_value(acc[0]) * iw, kahan_value(acc[1]) * iw, kahan_value(acc[2]) * iw, 0.0f);
}

// Roughness-0 level: the environment along each texel direction.
__global__ void __launch_bounds__(256) k_prefilter_mirror(const float4 *__restrict__ env, int S, int sm,
                                                          float4 *__restrict__ out) {
    int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= 6 * sm * sm) return;
    int f = o / (sm * sm), j = (o / sm) % sm, i = o % sm;
    v3 n = normalize(cube_texel_dir(f, i, j, sm));
    out[o] = cube_bilinear(env, face_dims(S), n);
}

// Environment mip chain for filtered importance sampling.  Level 0 is a copy
// of the environment so that every level sits at a closed-form offset of one
// buffer: level k (faces S >> k, S a power of two) starts at texel
// 8 (S^2 - (S >> k)^2) = 6 (S^2 + (S/2)^2 + ... + (S >> (k-1))^2).
__device__ __forceinline__ unsigned chain_offset_pow2(int S, int k) {
    unsigned s = (unsigned)S, sk = (unsigned)(S >> k);
    return 8u * (s * s - sk * sk);
}

__global__ void __launch_bounds__(256) k_env_copy(const float4 *__restrict__ env, int n, float4 *__restrict__ dst) {
    int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o < n) dst[o] = env[o];
}

// Level 0 of the environment as packed RGB texels (12 bytes) for the
// prefilter, whose taps use only the colour: each tap then moves three quarters
// of the bytes through the texture data path, the unit that bounds it.
struct Rgb {
    float r, g, b;
};
__global__ void __launch_bounds__(256) k_env_rgb(const float4 *__restrict__ env, int n, Rgb *__restrict__ dst) {
    int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o < n) {
        float4 v = env[o];
        sto(dst, (unsigned)o * 12u, Rgb{v.x, v.y, v.z});
    }
}

// face_bilinear over packed RGB texels, split into its loads and its
// interpolation (so that a caller can have several lookups' loads in flight):
// the same coordinates, taps and interpolation, so the same values.
struct RgbTaps {
    Rgb a, b, c, d;
    float wx, wy;
};
__device__ __forceinline__ RgbTaps rgb_taps(const Rgb *__restrict__ lvl, const FaceDims &g, FaceST f) {
    RgbTaps q;
    float x = clamp_to(fmaf(f.s, g.half, g.off), g.hi);
    float y = clamp_to(fmaf(f.t, g.half, g.off), g.hi);
    float x0f = fminf(floorf(x), g.hi1), y0f = fminf(floorf(y), g.hi1);
    q.wx = x - x0f;
    q.wy = y - y0f;
    unsigned idx = __umul24((unsigned)fmaf(f.face, (float)g.S, y0f), (unsigned)g.S) + (unsigned)x0f;
    unsigned o0 = idx * 12u, o1 = o0 + (unsigned)g.S * 12u;
    q.a = ldo(lvl, o0);
    q.b = ldo(lvl + 1, o0);
    q.c = ldo(lvl, o1);
    q.d = ldo(lvl + 1, o1);
    return q;
}
__device__ __forceinline__ float4 rgb_bilinear(const RgbTaps &q) {
    float4 A = make_float4(q.a.r, q.a.g, q.a.b, 0.0f), B = make_float4(q.b.r, q.b.g, q.b.b, 0.0f);
    float4 C = make_float4(q.c.r, q.c.g, q.c.b, 0.0f), D = make_float4(q.d.r, q.d.g, q.d.b, 0.0f);
    return lerp4(lerp4(A, B, q.wx), lerp4(C, D, q.wx), q.wy);
}

// Level k from level k - 1 (face size Sp = 2 Sd): solid-angle-weighted mean of
// the 2x2 children, as the irradiance source is built.
__global__ void __launch_bounds__(256) k_env_down(const float4 *__restrict__ src, int Sp,
                                                  float4 *__restrict__ dst) {
    int Sd = Sp >> 1;
    int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= 6 * Sd * Sd) return;
    int f = o / (Sd * Sd), j = (o / Sd) % Sd, i = o % Sd;
    const float4 *face = src + (size_t)f * Sp * Sp;
    float r = 0.0f, g = 0.0f, b = 0.0f, w = 0.0f;
    for (int bj = 0; bj < 2; ++bj)
        for (int bi = 0; bi < 2; ++bi) {
            int ci = 2 * i + bi, cj = 2 * j + bj;
            float dw = texel_solid_angle(ci, cj, Sp);
            float4 L = face[(size_t)cj * Sp + ci];
            r = fmaf(L.x, dw, r);
            g = fmaf(L.y, dw, g);
            b = fmaf(L.z, dw, b);
            w += dw;
        }
    float iw = 1.0f / w;
    dst[o] = make_float4(r * iw, g * iw, b * iw, 0.0f);
}

// The GGX samples of the prefiltered levels (one launch, blockIdx.y = level):
// entry k of level m is the tangent-frame half vector of Hammersley sample k for
// roughness^2 = alpha_m and, for filtered importance sampling, the environment
// chain level that sample reads (w; 0 otherwise).  That level is lod0 - log2(den)
// clamped to [0, last], where den = (1 - u2) + alpha^2 u2 is the GGX sampling
// denominator: for V = N the pdf of l is D / 4 = den^2 / (4 pi alpha^2), so
// 1/2 log2(omega_s / omega_p) + 1 = 1/2 log2(6 S^2 alpha^2 / N) + 1 - log2(den)
// (lod0 is that constant part, computed on the host in double precision).
// Levels with alpha = 0 (the mirror level) have no table.
struct GgxLevels {
    float alpha[8], lod0[8];
};
__global__ void __launch_bounds__(256) k_ggx_table(GgxLevels lv, int samples, int fis, int last,
                                                   float4 *__restrict__ tables) {
    int k = (int)blockIdx.x * 256 + (int)threadIdx.x, m = (int)blockIdx.y;
    float alpha = lv.alpha[m];
    if (k >= samples || alpha == 0.0f) return;
    float a2 = alpha * alpha;
    float inv_n = 1.0f / (float)samples;
    float u2 = radical_inverse2((uint32_t)k);
    float4 t = ggx_tangent((float)k * inv_n, u2, a2);
    if (fis) {
        float den = fmaf(a2, u2, 1.0f - u2);
        t.w = fminf(fmaxf(lv.lod0[m] - __log2f(den), 0.0f), (float)last);
    }
    tables[(size_t)m * samples + k] = t;
}

// One wavefront per prefiltered texel of a level (roughness > 0), from level 0
// of the environment (its packed RGB copy): sample k's half vector from the table, its direction l
// the half vector reflected about the texel normal n; with N.L > 0 it adds
// L(l) N.L and N.L.  A lane takes its samples k and k + 64 together: both
// lookups' taps are in flight before either is added (the adds keep the order
// k, k + 64, k + 128, ...), and the next pair's table entries load one
// iteration ahead, with the current pair's taps.
__global__ void __launch_bounds__(256) k_prefilter(const Rgb *__restrict__ env, int S, int sm,
                                                   const float4 *__restrict__ table, int samples,
                                                   float4 *__restrict__ out) {
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // XCD-aware: each XCD's blocks take a contiguous run of texels, whose lobes
    // cover a fraction of the environment that its own L2 can hold
    int o = xcd_tile((int)blockIdx.x, (int)gridDim.x) * 4 + wave;
    if (o >= 6 * sm * sm) return;  // whole wavefront leaves together
    int f = o / (sm * sm), j = (o / sm) % sm, i = o % sm;
    v3 n = normalize(cube_texel_dir(f, i, j, sm));
    v3 T, B;
    tangent_frame(n, T, B);
    FaceDims dims = face_dims(S);
    Kahan r{0, 0}, g{0, 0}, b{0, 0}, w{0, 0};
    int last = samples - 1;
    float4 na = table[min(lane, last)], nb = table[min(lane + 64, last)];
    for (int k = lane; k < samples; k += 128) {
        float4 ta = na, tb = nb;
        if (k + 128 < samples) {
            na = table[k + 128];
            nb = table[min(k + 192, last)];
        }
        v3 ha = ggx_to_world(ta, n, T, B), hb = ggx_to_world(tb, n, T, B);
        float vha = dot(n, ha), vhb = dot(n, hb);
        v3 la = ha * (2.0f * vha) - n, lb = hb * (2.0f * vhb) - n;
        float nla = dot(n, la), nlb = dot(n, lb);
        bool ua = nla > 0.0f, ub = k + 64 < samples && nlb > 0.0f;
        RgbTaps qa{}, qb{};
        if (ua) qa = rgb_taps(env, dims, cube_face(la));
        if (ub) qb = rgb_taps(env, dims, cube_face(lb));
        float4 La = rgb_bilinear(qa), Lb = rgb_bilinear(qb);
        if (ua) {
            kahan_add(r, La.x * nla);
            kahan_add(g, La.y * nla);
            kahan_add(b, La.z * nla);
            kahan_add(w, nla);
        }
        if (ub) {
            kahan_add(r, Lb.x * nlb);
            kahan_add(g, Lb.y * nlb);
            kahan_add(b, Lb.z * nlb);
            kahan_add(w, nlb);
        }
    }
    float R = wave_sum_compensated(kahan_value(r));
    float G = wave_sum_compensated(kahan_value(g));
    float Bv = wave_sum_compensated(kahan_value(b));
    float W = wave_sum_compensated(kahan_value(w));
    if (lane == 0) {
        float iw = 1.0f / W;
        out[o] = make_float4(R * iw, G * iw, Bv * iw, 0.0f);
    }
}

// Partial sums of a prefiltered level (roughness > 0) with filtered importance
// sampling.  Wavefront w of the grid takes tile w / chunks (8x8 texels of one
// face) and chunk w % chunks of the samples; its lanes are the tile's texels (a
// lane past the face edge computes a clamped texel and writes nothing).  Sample
// k's direction l is its half vector reflected about the texel normal n; with
// N.L > 0 it adds L(l) N.L and N.L, L read trilinearly from the environment
// chain at the sample's level.  part: [chunk][texel][8] = Kahan (s, c) of R,
// G, B and the weight, as k_irradiance_final sums them.
__global__ void __launch_bounds__(256) k_prefilter_fis(const float4 *__restrict__ chain, int S, int last, int sm,
                                                       const float4 *__restrict__ table, int samples, int chunks,
                                                       float *__restrict__ part) {
    // wave-uniform by construction; readfirstlane tells the compiler, so the
    // sample loop and its table loads are scalar
    // (not XCD-aware: the matched mip levels are small enough for every L2,
    // and the XCD-contiguous order measured slower here)
    int w = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + (int)(threadIdx.x >> 6));
    int lane = threadIdx.x & 63;
    int tpf = (sm + 7) >> 3;
    if (w >= 6 * tpf * tpf * chunks) return;  // whole wavefront leaves together
    int tile = w / chunks, chunk = w - tile * chunks;
    int f = tile / (tpf * tpf), t = tile - f * (tpf * tpf);
    int i = (t % tpf) * 8 + (lane & 7), j = (t / tpf) * 8 + (lane >> 3);
    v3 n = normalize(cube_texel_dir(f, min(i, sm - 1), min(j, sm - 1), sm));
    v3 T, B;
    tangent_frame(n, T, B);
    Kahan r{0, 0}, g{0, 0}, b{0, 0}, wt{0, 0};
    // (samples <= 2^20 and chunks <= 16: the products fit in 32 bits)
    int k0 = chunk * samples / chunks, k1 = (chunk + 1) * samples / chunks;
    for (int k = k0; k < k1; ++k) {
        float4 tk = table[k];
        v3 h = ggx_to_world(tk, n, T, B);
        float vh = dot(n, h);
        v3 l = h * (2.0f * vh) - n;
        float nl = dot(n, l);
        if (nl > 0.0f) {
            float lod = tk.w;
            int l0 = (int)lod;
            int l1 = min(l0 + 1, last);
            float fl = lod - (float)l0;
            FaceST fs = cube_face(l);
            int s0 = S >> l0, s1 = S >> l1;
            float4 L0 = face_bilinear(chain, chain_offset_pow2(S, l0), face_dims(s0), fs);
            float4 L1 = face_bilinear(chain, chain_offset_pow2(S, l1), face_dims(s1), fs);
            float4 L = lerp4(L0, L1, fl);
            kahan_add(r, L.x * nl);
            kahan_add(g, L.y * nl);
            kahan_add(b, L.z * nl);
            kahan_add(wt, nl);
        }
    }
    if (i < sm && j < sm) {
        int nout = 6 * sm * sm;
        int o = f * sm * sm + j * sm + i;
        float *p = part + ((size_t)chunk * nout + o) * 8;
        p[0] = r.s; p[1] = g.s; p[2] = b.s; p[3] = wt.s;
        p[4] = r.c; p[5] = g.c; p[6] = b.c; p[7] = wt.c;
    }
}

// One wavefront per BRDF table entry: N = +z, V = (sqrt(1 - NoV^2), 0, NoV).
// G_vis = G VoH / (NoH NoV) with G = G1(NoL) G1(NoV), G1(x) = x / (x(1-k)+k),
// written without the division by NoV: NoL VoH / (NoH (NoL(1-k)+k)(NoV(1-k)+k)).
__global__ void __launch_bounds__(256) k_brdf_lut(int size, int samples, float2 *__restrict__ out) {
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int o = blockIdx.x * 4 + wave;
    if (o >= size * size) return;
    int j = o / size, i = o % size;
    float NoV = ((float)i + 0.5f) / (float)size;
    float rough = ((float)j + 0.5f) / (float)size;
    float alpha = rough * rough, a2 = alpha * alpha, k = 0.5f * alpha;
    v3 V = mk3(sqrtf(fmaxf(0.0f, 1.0f - NoV * NoV)), 0.0f, NoV);
    v3 n = mk3(0.0f, 0.0f, 1.0f), T, B;
    tangent_frame(n, T, B);
    float gv = fmaf(NoV, 1.0f - k, k);
    float inv_n = 1.0f / (float)samples;
    Kahan A{0, 0}, Bs{0, 0};
    for (int s = lane; s < samples; s += 64) {
        v3 h = ggx_half((float)s * inv_n, radical_inverse2((uint32_t)s), a2, n, T, B);
        float vh = dot(V, h);
        float nl = fmaf(2.0f * vh, h.z, -V.z);
        if (nl > 0.0f) {
            float gvis = nl * vh / (h.z * fmaf(nl, 1.0f - k, k) * gv);
            float fc = pow5(1.0f - vh);
            kahan_add(A, (1.0f - fc) * gvis);
            kahan_add(Bs, fc * gvis);
        }
    }
    float a = wave_sum_compensated(kahan_value(A));
    float b = wave_sum_compensated(kahan_value(Bs));
    if (lane == 0) out[o] = make_float2(a * inv_n, b * inv_n);
}

// The same entries with the row's GGX half vectors made once into LDS (for up
// to kLutLdsSamples samples): block b takes kLutRowSlice entries of one row (one
// roughness), each wavefront a quarter of them in turn, its lanes splitting
// the samples as in k_brdf_lut (the same order); G_vis from a reciprocal, the
// compensated sums over groups of four samples.
constexpr int kLutLdsSamples = 2048, kLutRowSlice = 32;
__global__ void __launch_bounds__(256) k_brdf_lut_rows(int size, int samples, float2 *__restrict__ out) {
    extern __shared__ float4 tab[];  // samples entries (launched with samples * 16 bytes)
    int slices = (size + kLutRowSlice - 1) / kLutRowSlice;
    int j = (int)blockIdx.x / slices, i0 = ((int)blockIdx.x - j * slices) * kLutRowSlice;
    float rough = ((float)j + 0.5f) / (float)size;
    float alpha = rough * rough, a2 = alpha * alpha, k = 0.5f * alpha;
    float inv_n = 1.0f / (float)samples;
    for (int s = (int)threadIdx.x; s < samples; s += 256)
        tab[s] = ggx_tangent((float)s * inv_n, radical_inverse2((uint32_t)s), a2);
    __syncthreads();
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    v3 n = mk3(0.0f, 0.0f, 1.0f), T, B;
    tangent_frame(n, T, B);
    for (int q = wave; q < kLutRowSlice; q += 4) {
        int i = i0 + q;
        if (i >= size) break;  // wave-uniform
        float NoV = ((float)i + 0.5f) / (float)size;
        v3 V = mk3(sqrtf(fmaxf(0.0f, 1.0f - NoV * NoV)), 0.0f, NoV);
        float gv = fmaf(NoV, 1.0f - k, k);
        // Sample s's two terms, both >= 0: with N.L clamped at 0, a sample
        // below the horizon gets G_vis = 0 (N.L is a factor, the denominator
        // stays positive: h.z > 0, k > 0) and adds nothing, as if skipped.
        auto terms = [&](int s, float &ta, float &tb) {
            v3 h = ggx_to_world(tab[s], n, T, B);
            float vh = dot(V, h);
            float nl = fmaxf(fmaf(2.0f * vh, h.z, -V.z), 0.0f);
            float gvis = nl * vh * rcp(h.z * fmaf(nl, 1.0f - k, k) * gv);
            float fc = pow5(1.0f - vh);
            ta = (1.0f - fc) * gvis;
            tb = fc * gvis;
        };
        // a lane's samples in groups of four summed in plain float, each group
        // Kahan-added (the whole sum stays within a few units of rounding, as
        // for the irradiance), then the ones left over one by one
        Kahan A{0, 0}, Bs{0, 0};
        int s = lane;
        for (; s + 192 < samples; s += 256) {
            float a0, b0, a1, b1, a2, b2, a3, b3;
            terms(s, a0, b0);
            terms(s + 64, a1, b1);
            terms(s + 128, a2, b2);
            terms(s + 192, a3, b3);
            kahan_add(A, ((a0 + a1) + a2) + a3);
            kahan_add(Bs, ((b0 + b1) + b2) + b3);
        }
        for (; s < samples; s += 64) {
            float ta, tb;
            terms(s, ta, tb);
            kahan_add(A, ta);
            kahan_add(Bs, tb);
        }
        float a = wave_sum_compensated(kahan_value(A));
        float b = wave_sum_compensated(kahan_value(Bs));
        if (lane == 0) out[j * size + i] = make_float2(a * inv_n, b * inv_n);
    }
}

// Sample chunks of a prefiltered level of face size sm: enough wavefronts to
// fill the chip (about 8192, 32 per CU) without splitting a tile's samples
// more than 16 ways.
static int prefilter_chunks(int sm) {
    int tpf = (sm + 7) / 8;
    int tiles = 6 * tpf * tpf;
    int c = (8192 + tiles - 1) / tiles;
    return c < 1 ? 1 : (c > 16 ? 16 : c);
}

IblPlan ibl_plan(int S, const epb_ibl_params &p) {
    IblPlan q{};
    q.S = S;
    q.src = S < p.irr_src_size ? S : p.irr_src_size;
    q.irr = p.irr_size;
    q.pref_base = S < p.pref_size ? S : p.pref_size;
    q.pref_levels = p.pref_levels;
    q.pref_samples = p.pref_samples;
    q.lut = p.lut_size;
    q.lut_samples = p.lut_samples;
    q.fis = p.pref_fis;
    q.chain_last = 0;
    while ((S >> (q.chain_last + 1)) >= 2) ++q.chain_last;
    int nsrc = 6 * q.src * q.src;
    int nout = 6 * q.irr * q.irr;
    int out_blocks = (nout + 255) / 256;
    // about four workgroups per CU (one per SIMD is too few to hide the serial
    // Kahan chains; eight gain nothing more), chunks of >= 256 sources
    int chunks = (1024 + out_blocks - 1) / out_blocks;
    int max_chunks = (nsrc + 255) / 256;
    if (chunks > max_chunks) chunks = max_chunks;
    if (chunks < 1) chunks = 1;
    q.chunks = chunks;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    };
    q.off_src = take((size_t)nsrc * 16);
    q.off_tab = take((size_t)nsrc * 16);
    q.off_part = take((size_t)chunks * nout * 8 * 4);
    // environment mip chain for filtered importance sampling: levels 0 .. last
    // contiguous, level k at texel offset 8 (S^2 - (S >> k)^2)
    q.off_chain = take(q.fis ? (size_t)8 * S * S * 16 : 0);
    // the prefilter's GGX sample table and partial sums, one level at a time
    size_t part = 0;
    for (int m = 1; q.fis && m < q.pref_levels; ++m) {  // (level 0 has roughness 0: no samples)
        int sm = q.pref_base >> m;
        size_t need = (size_t)prefilter_chunks(sm) * 6 * sm * sm * 8 * 4;
        if (need > part) part = need;
    }
    q.off_ggx = take(q.pref_levels > 1 ? (size_t)q.pref_levels * q.pref_samples * 16 : 0);  // a table per level
    q.off_rgb = take(!q.fis && q.pref_levels > 1 ? (size_t)6 * S * S * 12 : 0);  // level 0 as packed RGB
    q.off_ppart = take(part);
    q.bytes = off;
    return q;
}

hipError_t launch_precompute_ibl(const IblPlan &q, const float *env, float *irr, float *pref, float *lut,
                                 void *scratch, hipStream_t s) {
    char *sc = (char *)scratch;
    float4 *src = (float4 *)(sc + q.off_src);
    float4 *tab = (float4 *)(sc + q.off_tab);
    float *part = (float *)(sc + q.off_part);
    const float4 *env4 = (const float4 *)env;
    int nsrc = 6 * q.src * q.src;
    int nout = 6 * q.irr * q.irr;
    int kk = (q.S / q.src) * (q.S / q.src), lpt = 1;
    while (lpt < kk && lpt < 64) lpt *= 2;
    long long threads = (long long)nsrc * lpt;
    hipLaunchKernelGGL(k_ibl_source, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, env4, q.S, q.src,
                       lpt, src, tab);
    int chunk_len = (nsrc + q.chunks - 1) / q.chunks;
    hipLaunchKernelGGL(k_irradiance_partial, dim3((nout + 255) / 256, q.chunks), dim3(256), 0, s, src, tab,
                       nsrc, chunk_len, q.irr, part);
    hipLaunchKernelGGL(k_irradiance_final, dim3((nout + 255) / 256), dim3(256), 0, s, part, q.chunks, q.irr,
                       (float4 *)irr);
    float4 *chain = (float4 *)(sc + q.off_chain);
    float4 *ggx = (float4 *)(sc + q.off_ggx);
    float *ppart = (float *)(sc + q.off_ppart);
    if (q.fis) {
        int n0 = 6 * q.S * q.S;
        hipLaunchKernelGGL(k_env_copy, dim3((n0 + 255) / 256), dim3(256), 0, s, env4, n0, chain);
        for (int k = 1; k <= q.chain_last; ++k) {
            int Sd = q.S >> k;
            hipLaunchKernelGGL(k_env_down, dim3((6 * Sd * Sd + 255) / 256), dim3(256), 0, s,
                               (const float4 *)(chain + 8u * ((unsigned)q.S * q.S - (unsigned)(2 * Sd) * (2 * Sd))),
                               2 * Sd, chain + 8u * ((unsigned)q.S * q.S - (unsigned)Sd * Sd));
        }
    }
    GgxLevels lv{};
    for (int m = 0; m < q.pref_levels; ++m) {
        float rough = q.pref_levels > 1 ? (float)m / (float)(q.pref_levels - 1) : 0.0f;
        lv.alpha[m] = rough * rough;
        if (q.fis && lv.alpha[m] != 0.0f) {
            double a2 = (double)lv.alpha[m] * lv.alpha[m];
            lv.lod0[m] = (float)(0.5 * std::log2(6.0 * q.S * q.S * a2 / q.pref_samples) + 1.0);
        }
    }
    Rgb *rgb = (Rgb *)(sc + q.off_rgb);
    if (!q.fis && q.pref_levels > 1) {
        int n0 = 6 * q.S * q.S;
        hipLaunchKernelGGL(k_env_rgb, dim3((n0 + 255) / 256), dim3(256), 0, s, env4, n0, rgb);
    }
    if (q.pref_levels > 1)
        hipLaunchKernelGGL(k_ggx_table, dim3((q.pref_samples + 255) / 256, q.pref_levels), dim3(256), 0, s, lv,
                           q.pref_samples, q.fis, q.chain_last, ggx);
    size_t off = 0;
    for (int m = 0; m < q.pref_levels; ++m) {
        int sm = q.pref_base >> m;
        float alpha = lv.alpha[m];
        const float4 *table = ggx + (size_t)m * q.pref_samples;
        int n = 6 * sm * sm;
        float4 *dst = (float4 *)pref + off;
        if (alpha == 0.0f) {
            hipLaunchKernelGGL(k_prefilter_mirror, dim3((n + 255) / 256), dim3(256), 0, s, env4, q.S, sm, dst);
        } else {
            // (stream order: the previous level's kernels are done with the partials)
            if (q.fis) {
                int chunks = prefilter_chunks(sm), tpf = (sm + 7) / 8;
                int waves = 6 * tpf * tpf * chunks;
                hipLaunchKernelGGL(k_prefilter_fis, dim3((waves + 3) / 4), dim3(256), 0, s, chain, q.S,
                                   q.chain_last, sm, table, q.pref_samples, chunks, ppart);
                hipLaunchKernelGGL(k_irradiance_final, dim3((n + 255) / 256), dim3(256), 0, s, ppart, chunks, sm,
                                   dst);
            } else {
                hipLaunchKernelGGL(k_prefilter, dim3((n + 3) / 4), dim3(256), 0, s, (const Rgb *)rgb, q.S, sm,
                                   table, q.pref_samples, dst);
            }
        }
        off += (size_t)n;
    }
    if (q.lut_samples <= kLutLdsSamples) {
        int slices = (q.lut + kLutRowSlice - 1) / kLutRowSlice;
        hipLaunchKernelGGL(k_brdf_lut_rows, dim3(q.lut * slices), dim3(256), (size_t)q.lut_samples * sizeof(float4), s,
                           q.lut, q.lut_samples, (float2 *)lut);
    } else {
        int nl = q.lut * q.lut;
        hipLaunchKernelGGL(k_brdf_lut, dim3((nl + 3) / 4), dim3(256), 0, s, q.lut, q.lut_samples, (float2 *)lut);
    }
    return hipGetLastError();
}

}  // namespace epb
