// Device-side helpers shared by the gfx950 kernels of the shading pass:
// small vector algebra, storage conversions, camera projection, cube-map
// addressing and filtering, compensated summation and the XCD-aware block
// order.  Nothing here is host code.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "desc.hpp"

namespace epb {

constexpr float kPi = 3.14159265358979323846f;
constexpr int kNumXcd = 8;  // MI355X: 256 CUs in 8 accelerator complex dies

// ---------------------------------------------------------------------------
// storage
// ---------------------------------------------------------------------------
// Loads and stores at a 32-bit byte offset from a wave-uniform base: the
// compiler then emits the scalar-base + 32-bit vector-offset form (with the
// constant part folded into the immediate) instead of 64-bit address
// arithmetic per lane.  Callers keep every offset below 2^32 (sizes are
// validated on the host).
// The access is made through the global address space: every buffer handed to
// the library is device memory, and a pointer read from a batch table would
// otherwise be a generic (flat) address, loaded per lane with 64-bit
// arithmetic.  Values move as 16- or 32-bit words (class types cannot be
// copied through a pointer of another address space).
template <typename T>
__device__ __forceinline__ T ldo(const T *base, unsigned byte_off) {
    typedef __attribute__((address_space(1))) const char GC;
    typedef __attribute__((address_space(1))) const unsigned GU;
    typedef __attribute__((address_space(1))) const unsigned short GS;
    GC *a = (GC *)base + byte_off;
    T r;
    if constexpr (sizeof(T) % 4 == 0) {
        unsigned w[sizeof(T) / 4];
#pragma unroll
        for (unsigned k = 0; k < sizeof(T) / 4; ++k) w[k] = ((GU *)a)[k];
        __builtin_memcpy(&r, w, sizeof(T));
    } else {
        static_assert(sizeof(T) == 2, "16-bit or whole 32-bit words");
        unsigned short h = *(GS *)a;
        __builtin_memcpy(&r, &h, 2);
    }
    return r;
}
template <typename T>
__device__ __forceinline__ void sto(T *base, unsigned byte_off, T v) {
    typedef __attribute__((address_space(1))) char GC;
    typedef __attribute__((address_space(1))) unsigned GU;
    typedef __attribute__((address_space(1))) unsigned short GS;
    GC *a = (GC *)base + byte_off;
    if constexpr (sizeof(T) % 4 == 0) {
        unsigned w[sizeof(T) / 4];
        __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
        for (unsigned k = 0; k < sizeof(T) / 4; ++k) ((GU *)a)[k] = w[k];
    } else {
        static_assert(sizeof(T) == 2, "16-bit or whole 32-bit words");
        unsigned short h;
        __builtin_memcpy(&h, &v, 2);
        *(GS *)a = h;
    }
}
__device__ __forceinline__ float ldf(const float *base, unsigned i) { return ldo(base, i * 4u); }
__device__ __forceinline__ float ldf(const __half *base, unsigned i) { return __half2float(ldo(base, i * 2u)); }
__device__ __forceinline__ void stf(float *base, unsigned i, float v) { sto(base, i * 4u, v); }
__device__ __forceinline__ void stf(__half *base, unsigned i, float v) {
    sto(base, i * 2u, __float2half_rn(fminf(v, 65504.0f)));  // saturate (HDR peaks can exceed 65504)
}

// Raw buffer resource over the first `bytes` bytes at `base`.  A load through it
// at a byte offset at or past `bytes` returns 0 without touching memory (the
// buffer unit's range check), so a gather can be issued from an unchecked
// offset and its result discarded when the offset was not valid.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_buffer(const void *base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float buf_ldf(__amdgpu_buffer_rsrc_t r, unsigned byte_off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}

// Read-only data that every lane of a wavefront reads at the same address (a
// sample kernel, a table): through the constant address space the compiler
// issues scalar loads, also where the pointer itself was read from memory (the
// batch table), which it otherwise treats as a generic per-lane address.
typedef __attribute__((address_space(4))) const float ConstFloat;
__device__ __forceinline__ const ConstFloat *as_constant(const float *p) { return (const ConstFloat *)p; }

__device__ __forceinline__ float ldc(const float *p) { return *p; }
__device__ __forceinline__ float ldc(const __half *p) { return __half2float(*p); }

__device__ __forceinline__ void st(float *p, float v) { *p = v; }
__device__ __forceinline__ void st(__half *p, float v) {
    // saturate instead of overflowing to inf (HDR peaks can exceed 65504)
    *p = __float2half_rn(fminf(v, 65504.0f));
}

// ---------------------------------------------------------------------------
// vectors
// ---------------------------------------------------------------------------
struct v3 {
    float x, y, z;
};
__device__ __forceinline__ v3 mk3(float x, float y, float z) { return v3{x, y, z}; }
__device__ __forceinline__ v3 operator+(v3 a, v3 b) { return mk3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ v3 operator-(v3 a, v3 b) { return mk3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ v3 operator*(v3 a, float s) { return mk3(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ float dot(v3 a, v3 b) { return fmaf(a.x, b.x, fmaf(a.y, b.y, a.z * b.z)); }
__device__ __forceinline__ v3 cross(v3 a, v3 b) {
    return mk3(fmaf(a.y, b.z, -a.z * b.y), fmaf(a.z, b.x, -a.x * b.z), fmaf(a.x, b.y, -a.y * b.x));
}
__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
// floor and convert to int in one VALU instruction.  (int)floorf(x) is two
// (v_floor, v_cvt), because the fused v_cvt_flr_i32_f32 is only selected under
// finite-math, which these kernels cannot assume (+inf marks background).
// Results agree for every input: both saturate out of range, NaN gives 0.
__device__ __forceinline__ int floor_to_int(float x) {
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ v3 normalize(v3 a) { return a * rsq(dot(a, a)); }
__device__ __forceinline__ float clamp01(float x) { return fminf(fmaxf(x, 0.0f), 1.0f); }
// x clamped to [0, hi] in one instruction (median of three; equal to the
// min/max pair for every non-NaN x)
__device__ __forceinline__ float clamp_to(float x, float hi) { return __builtin_amdgcn_fmed3f(x, 0.0f, hi); }
__device__ __forceinline__ float pow5(float x) {
    float x2 = x * x;
    return x2 * x2 * x;
}

__device__ __forceinline__ v3 mul_R(const float *R, v3 v) {
    return mk3(fmaf(R[0], v.x, fmaf(R[1], v.y, R[2] * v.z)), fmaf(R[3], v.x, fmaf(R[4], v.y, R[5] * v.z)),
               fmaf(R[6], v.x, fmaf(R[7], v.y, R[8] * v.z)));
}
__device__ __forceinline__ v3 mul_Rt(const float *R, v3 v) {
    return mk3(fmaf(R[0], v.x, fmaf(R[3], v.y, R[6] * v.z)), fmaf(R[1], v.x, fmaf(R[4], v.y, R[7] * v.z)),
               fmaf(R[2], v.x, fmaf(R[5], v.y, R[8] * v.z)));
}

// ---------------------------------------------------------------------------
// cube maps: [face][S][S] float4 texels, faces +X -X +Y -Y +Z -Z
// ---------------------------------------------------------------------------
struct FaceST {
    float face;  // 0 .. 5 (+X, -X, +Y, -Y, +Z, -Z), as the cube instructions return it
    float s, t;  // in [-1, 1] on the face
};

// Face and in-face coordinates of direction d by the CDNA cube instructions:
// the major axis with ties broken z, then y, then x; a zero component counts
// as positive; cubesc / cubetc give the OpenGL s and t numerators and cubema
// twice the signed major component, so s = sc / |major| = sc * (2 / |ma|).
// Four instructions and no branches (lanes look along different axes).
__device__ __forceinline__ FaceST cube_face(v3 d) {
    FaceST r;
    r.face = __builtin_amdgcn_cubeid(d.x, d.y, d.z);
    float inv = 2.0f * rcp(fabsf(__builtin_amdgcn_cubema(d.x, d.y, d.z)));  // == rcp(|major|)
    r.s = __builtin_amdgcn_cubesc(d.x, d.y, d.z) * inv;
    r.t = __builtin_amdgcn_cubetc(d.x, d.y, d.z) * inv;
    return r;
}

__device__ __forceinline__ float4 ld4(const float4 *p) { return *p; }
__device__ __forceinline__ float4 lerp4(float4 a, float4 b, float w) {
    return make_float4(fmaf(w, b.x - a.x, a.x), fmaf(w, b.y - a.y, a.y), fmaf(w, b.z - a.z, a.z), 0.0f);
}

// Bilinear, clamp-to-edge inside one face of one level (S >= 2).  Clamping
// the coordinate to [0, S-1] and the left tap to S-2 gives the same result as
// clamping both taps (at an edge one weight is 0 or 1), and keeps the second
// column at a fixed +1 offset from the first (taken from the base pointer, so
// that it folds into the load instructions).  `lvl` is wave-uniform and the
// texel index a 32-bit offset (24-bit multiplies; S <= 8192).
__device__ __forceinline__ float4 face_bilinear(const float4 *__restrict__ lvl, unsigned off, const FaceDims &g,
                                                FaceST f) {
    float x = clamp_to(fmaf(f.s, g.half, g.off), g.hi);
    float y = clamp_to(fmaf(f.t, g.half, g.off), g.hi);
    float x0f = fminf(floorf(x), g.hi1), y0f = fminf(floorf(y), g.hi1);
    float wx = x - x0f, wy = y - y0f;
    // row of the texel in the level: face S + y0, exact in float (below 2^24)
    unsigned idx = off + __umul24((unsigned)fmaf(f.face, (float)g.S, y0f), (unsigned)g.S) + (unsigned)x0f;
    unsigned o0 = idx * 16u, o1 = o0 + (unsigned)g.S * 16u;
    float4 a = ldo(lvl, o0), b = ldo(lvl + 1, o0);
    float4 c = ldo(lvl, o1), d = ldo(lvl + 1, o1);
    return lerp4(lerp4(a, b, wx), lerp4(c, d, wx), wy);
}

__device__ __forceinline__ float4 cube_bilinear(const float4 *__restrict__ lvl, const FaceDims &g, v3 d) {
    return face_bilinear(lvl, 0u, g, cube_face(d));
}

// Offset (in texels) of level m of a chain with base size `base`.
__device__ __forceinline__ size_t chain_offset(int base, int m) {
    size_t off = 0;
    for (int k = 0; k < m; ++k) off += (size_t)6 * (base >> k) * (base >> k);
    return off;
}

// ---------------------------------------------------------------------------
// compensated (Kahan) summation; contraction must stay off inside
// ---------------------------------------------------------------------------
struct Kahan {
    float s, c;
};
__device__ __forceinline__ void kahan_add(Kahan &k, float x) {
#pragma clang fp contract(off)
    float y = x - k.c;
    float t = k.s + y;
    k.c = (t - k.s) - y;
    k.s = t;
}
__device__ __forceinline__ float kahan_value(const Kahan &k) {
#pragma clang fp contract(off)
    return k.s - k.c;
}

// Error-free sum of two floats (Knuth): a + b = s + e exactly.
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
#pragma clang fp contract(off)
    s = a + b;
    float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Compensated sum over the 64 lanes of a wavefront; every lane gets the total.
__device__ __forceinline__ float wave_sum_compensated(float v) {
    float comp = 0.0f;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        float o = __shfl_xor(v, off, 64);
        float oc = __shfl_xor(comp, off, 64);
        float s, e;
        two_sum(v, o, s, e);
        v = s;
        comp = comp + oc + e;
    }
    return v + comp;
}

// ---------------------------------------------------------------------------
// bloom bright pass and the 2x2 sums of its first level
// ---------------------------------------------------------------------------
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

__device__ __forceinline__ Half4 pack_half4(float4 v) { return pack<Half4>(v); }

// The value that storing v to a buffer of T leaves there, read back as float.
__device__ __forceinline__ float stored_as(float v, const float *) { return v; }
__device__ __forceinline__ float stored_as(float v, const __half *) {
    return __half2float(__float2half_rn(fminf(v, 65504.0f)));
}

// Bright-pass weight max(Y - threshold, 0) / Y of a pixel (Rec. 709 luminance
// Y), with a reciprocal; a luminance below the smallest normal float blooms
// nothing (its reciprocal would overflow).
__device__ __forceinline__ float bright_scale(float r, float g, float b, float threshold) {
    float Y = fmaf(0.2126f, r, fmaf(0.7152f, g, 0.0722f * b));
    float m = Y - threshold;
    return m > 0.0f && Y >= 1.17549435e-38f ? m * rcp(Y) : 0.0f;
}

// v plus the value of the neighbouring lane (lanes 2k and 2k + 1 pair up);
// both lanes get the same sum.
__device__ __forceinline__ float add_lane_pair(float v) {
    int n = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1, 0xF, 0xF, true);  // quad_perm 1,0,3,2
    return v + __builtin_bit_cast(float, n);
}

// v plus the value of lane l ^ S, S = 16 or 32: the lane's row of S lanes and
// the paired row (rows 2k and 2k + 1).  A permlane swap of v with itself puts
// the even row's values in the first result and the odd row's in the second.
// (The results are copied out before the bit casts: a bit cast of a vector
// element reads element 0 with this compiler.)
template <int S>
__device__ __forceinline__ float add_row_pair(float v) {
    static_assert(S == 16 || S == 32, "rows of 16 or 32 lanes");
    unsigned u = __builtin_bit_cast(unsigned, v), even, odd;
    if constexpr (S == 32) {
        auto p = __builtin_amdgcn_permlane32_swap(u, u, false, false);
        even = p[0];
        odd = p[1];
    } else {
        auto p = __builtin_amdgcn_permlane16_swap(u, u, false, false);
        even = p[0];
        odd = p[1];
    }
    return __builtin_bit_cast(float, even) + __builtin_bit_cast(float, odd);
}

// ---------------------------------------------------------------------------
// launch order: consecutive tiles go to the same XCD (own L2)
// ---------------------------------------------------------------------------
// The dispatcher hands workgroup b to XCD b % 8.  Remap so that XCD k
// processes a contiguous range of tiles (a bijection for any grid size).
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    int q = nb / kNumXcd, r = nb % kNumXcd;
    int x = b % kNumXcd, local = b / kNumXcd;
    return x < r ? x * (q + 1) + local : r * (q + 1) + (x - r) * q + local;
}

// Work distribution of persistent (or one-item-per-block) grids: XCD x (the
// blocks b with b mod 8 == x) owns a contiguous share of the items, visited by
// its blocks in turn.  With one block per item this is the bijection above.
// The trip count depends on blockIdx only, so loops may contain barriers.
struct XcdRange {
    int first, count, lb, stride;
};
__device__ __forceinline__ XcdRange xcd_range(int total) {
    int nb = gridDim.x, b = blockIdx.x;
    int x = b % kNumXcd;
    int q = total / kNumXcd, r = total % kNumXcd;
    XcdRange w;
    w.first = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    w.count = q + (x < r ? 1 : 0);
    w.stride = nb / kNumXcd + (x < nb % kNumXcd ? 1 : 0);
    w.lb = b / kNumXcd;
    return w;
}

// View owning work item g: start[v] <= g < start[v + 1] (binary search; uniform).
__device__ __forceinline__ int find_view(const int *start, int n, int g) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (start[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

// GGX half vector for the point (u1, u2) around normal n with tangent frame
// (T, B): phi = 2 pi u1, cos^2 = (1 - u2) / den, sin^2 = alpha^2 u2 / den,
// den = (1 - u2) + alpha^2 u2 (both fractions without cancellation).
// The GGX half vector of sample (u1, u2) in the tangent frame: (sin t cos p,
// sin t sin p, cos t) with p = 2 pi u1 and cos^2 t = (1 - u2) / (1 + (a2 - 1) u2).
// It depends on the sample and the roughness only, so kernels that reuse one
// sample set for many texels take it from a table made by this function.
__device__ __forceinline__ float4 ggx_tangent(float u1, float u2, float a2) {
    float om = 1.0f - u2;
    float den = fmaf(a2, u2, om);
    float inv = rcp(den);
    float ct = sqrtf(om * inv);
    float st = sqrtf(a2 * u2 * inv);
    float sp, cp;
    sincospif(2.0f * u1, &sp, &cp);
    return make_float4(st * cp, st * sp, ct, 0.0f);
}
// A tangent-frame half vector t (x, y, z) in the frame (T, B, n).
__device__ __forceinline__ v3 ggx_to_world(float4 t, v3 n, v3 T, v3 B) {
    return mk3(fmaf(T.x, t.x, fmaf(B.x, t.y, n.x * t.z)), fmaf(T.y, t.x, fmaf(B.y, t.y, n.y * t.z)),
               fmaf(T.z, t.x, fmaf(B.z, t.y, n.z * t.z)));
}
__device__ __forceinline__ v3 ggx_half(float u1, float u2, float a2, v3 n, v3 T, v3 B) {
    return ggx_to_world(ggx_tangent(u1, u2, a2), n, T, B);
}

// Tangent frame: up = +z unless |n.z| >= 0.999, then +x; T = norm(up x n), B = n x T.
__device__ __forceinline__ void tangent_frame(v3 n, v3 &T, v3 &B) {
    v3 up = fabsf(n.z) < 0.999f ? mk3(0.0f, 0.0f, 1.0f) : mk3(1.0f, 0.0f, 0.0f);
    T = normalize(cross(up, n));
    B = cross(n, T);
}

__device__ __forceinline__ float radical_inverse2(uint32_t k) {
    return (float)__builtin_bitreverse32(k) * 2.3283064365386963e-10f;  // 2^-32
}

// Texel-centre direction of cube texel (i, j) on a face of size S (not unit).
__device__ __forceinline__ v3 cube_texel_dir(int face, int i, int j, int S) {
    float inv = 1.0f / (float)S;
    float s = (float)(2 * i + 1 - S) * inv;
    float t = (float)(2 * j + 1 - S) * inv;
    switch (face) {
    case 0: return mk3(1.0f, -t, -s);
    case 1: return mk3(-1.0f, -t, s);
    case 2: return mk3(s, 1.0f, t);
    case 3: return mk3(s, -1.0f, -t);
    case 4: return mk3(s, -t, 1.0f);
    default: return mk3(-s, -t, -1.0f);
    }
}

}  // namespace epb
