// Image-based-lighting precompute (paper Sec. 3.1): a solid-angle-weighted
// average of the environment, the diffuse irradiance map, the split-sum
// prefiltered specular chain and the environment BRDF table.
//
// gfx950 mapping:
//  * irradiance: 6*32^2 outputs x 6*64^2 source texels.  One thread per
//    output, source texels staged through LDS in blocks of 256 and broadcast
//    to all lanes; the source range is split across workgroups so that the
//    grid fills all 256 CUs, and the per-split Kahan partials are combined in
//    a fixed order by a second kernel (deterministic, no atomics).
//  * prefilter and BRDF table: one wavefront per output texel, the 64 lanes
//    split the Hammersley samples, per-lane Kahan sums, compensated wave
//    reduction through cross-lane shuffles.
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

// Irradiance source: texel (f, i, j) of size Ss is the solid-angle-weighted mean
// of the k x k environment texels it covers (k = S / Ss).  Because solid angles
// add, this equals repeated 2x2 weighted halving.  Also writes the source
// table entry (unit direction, solid angle at size Ss).
__global__ void __launch_bounds__(256) k_ibl_source(const float4 *__restrict__ env, int S, int Ss,
                                                    float4 *__restrict__ src, float4 *__restrict__ tab) {
    int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= 6 * Ss * Ss) return;
    int f = o / (Ss * Ss), j = (o / Ss) % Ss, i = o % Ss;
    int k = S / Ss;
    Kahan r{0, 0}, g{0, 0}, b{0, 0}, w{0, 0};
    const float4 *face = env + (size_t)f * S * S;
    for (int bj = 0; bj < k; ++bj)
        for (int bi = 0; bi < k; ++bi) {
            int ci = i * k + bi, cj = j * k + bj;
            float dw = k == 1 ? 1.0f : texel_solid_angle(ci, cj, S);
            float4 L = face[(size_t)cj * S + ci];
            kahan_add(r, L.x * dw);
            kahan_add(g, L.y * dw);
            kahan_add(b, L.z * dw);
            kahan_add(w, dw);
        }
    float iw = 1.0f / kahan_value(w);
    src[o] = make_float4(kahan_value(r) * iw, kahan_value(g) * iw, kahan_value(b) * iw, 0.0f);
    v3 d = normalize(cube_texel_dir(f, i, j, Ss));
    tab[o] = make_float4(d.x, d.y, d.z, texel_solid_angle(i, j, Ss));
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
        for (int q = 0; q < cnt; ++q) {
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

// One wavefront per prefiltered texel of a level with roughness^2 = alpha > 0.
__global__ void __launch_bounds__(256) k_prefilter(const float4 *__restrict__ env, int S, int sm, float alpha,
                                                   int samples, float4 *__restrict__ out) {
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int o = blockIdx.x * 4 + wave;
    if (o >= 6 * sm * sm) return;  // whole wavefront leaves together
    int f = o / (sm * sm), j = (o / sm) % sm, i = o % sm;
    v3 n = normalize(cube_texel_dir(f, i, j, sm));
    v3 T, B;
    tangent_frame(n, T, B);
    float a2 = alpha * alpha;
    float inv_n = 1.0f / (float)samples;
    FaceDims dims = face_dims(S);
    Kahan r{0, 0}, g{0, 0}, b{0, 0}, w{0, 0};
    for (int k = lane; k < samples; k += 64) {
        v3 h = ggx_half((float)k * inv_n, radical_inverse2((uint32_t)k), a2, n, T, B);
        float vh = dot(n, h);
        v3 l = h * (2.0f * vh) - n;
        float nl = dot(n, l);
        if (nl > 0.0f) {
            float4 L = cube_bilinear(env, dims, l);
            kahan_add(r, L.x * nl);
            kahan_add(g, L.y * nl);
            kahan_add(b, L.z * nl);
            kahan_add(w, nl);
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

// Filtered importance sampling: as k_prefilter, but sample l reads the chain
// trilinearly at lod = lod0 - log2(den) clamped to [0, last], where den =
// (1 - u2) + alpha^2 u2 is the GGX sampling denominator: for V = N the pdf of l
// is D / 4 = den^2 / (4 pi alpha^2), so 1/2 log2(omega_s / omega_p) + 1 =
// 1/2 log2(6 S^2 alpha^2 / N) + 1 - log2(den) (lod0 is that constant part,
// computed on the host in double precision).
__global__ void __launch_bounds__(256) k_prefilter_fis(const float4 *__restrict__ chain, int S, int last,
                                                       int sm, float alpha, int samples, float lod0,
                                                       float4 *__restrict__ out) {
    int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int o = blockIdx.x * 4 + wave;
    if (o >= 6 * sm * sm) return;  // whole wavefront leaves together
    int f = o / (sm * sm), j = (o / sm) % sm, i = o % sm;
    v3 n = normalize(cube_texel_dir(f, i, j, sm));
    v3 T, B;
    tangent_frame(n, T, B);
    float a2 = alpha * alpha;
    float inv_n = 1.0f / (float)samples;
    float flast = (float)last;
    Kahan r{0, 0}, g{0, 0}, b{0, 0}, w{0, 0};
    for (int k = lane; k < samples; k += 64) {
        float u2 = radical_inverse2((uint32_t)k);
        v3 h = ggx_half((float)k * inv_n, u2, a2, n, T, B);
        float vh = dot(n, h);
        v3 l = h * (2.0f * vh) - n;
        float nl = dot(n, l);
        if (nl > 0.0f) {
            float den = fmaf(a2, u2, 1.0f - u2);
            float lod = fminf(fmaxf(lod0 - __log2f(den), 0.0f), flast);
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
            kahan_add(w, nl);
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
    // enough workgroups to cover the 256 CUs at least twice, chunks of >= 256 sources
    int chunks = (512 + out_blocks - 1) / out_blocks;
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
    hipLaunchKernelGGL(k_ibl_source, dim3((nsrc + 255) / 256), dim3(256), 0, s, env4, q.S, q.src, src, tab);
    int chunk_len = (nsrc + q.chunks - 1) / q.chunks;
    hipLaunchKernelGGL(k_irradiance_partial, dim3((nout + 255) / 256, q.chunks), dim3(256), 0, s, src, tab,
                       nsrc, chunk_len, q.irr, part);
    hipLaunchKernelGGL(k_irradiance_final, dim3((nout + 255) / 256), dim3(256), 0, s, part, q.chunks, q.irr,
                       (float4 *)irr);
    float4 *chain = (float4 *)(sc + q.off_chain);
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
    size_t off = 0;
    for (int m = 0; m < q.pref_levels; ++m) {
        int sm = q.pref_base >> m;
        float rough = q.pref_levels > 1 ? (float)m / (float)(q.pref_levels - 1) : 0.0f;
        float alpha = rough * rough;
        int n = 6 * sm * sm;
        float4 *dst = (float4 *)pref + off;
        if (alpha == 0.0f) {
            hipLaunchKernelGGL(k_prefilter_mirror, dim3((n + 255) / 256), dim3(256), 0, s, env4, q.S, sm, dst);
        } else if (q.fis) {
            double a2 = (double)alpha * alpha;
            float lod0 = (float)(0.5 * std::log2(6.0 * q.S * q.S * a2 / q.pref_samples) + 1.0);
            hipLaunchKernelGGL(k_prefilter_fis, dim3((n + 3) / 4), dim3(256), 0, s, chain, q.S, q.chain_last, sm,
                               alpha, q.pref_samples, lod0, dst);
        } else
            hipLaunchKernelGGL(k_prefilter, dim3((n + 3) / 4), dim3(256), 0, s, env4, q.S, sm, alpha,
                               q.pref_samples, dst);
        off += (size_t)n;
    }
    int nl = q.lut * q.lut;
    hipLaunchKernelGGL(k_brdf_lut, dim3((nl + 3) / 4), dim3(256), 0, s, q.lut, q.lut_samples, (float2 *)lut);
    return hipGetLastError();
}

}  // namespace epb
