// Eye-dome lighting (paper Sec. 4.3): the compositing step for depth-only
// renders such as point clouds, where no normals exist for PBR.  A pixel is
// darkened by how far it lies behind its screen-space neighbours on a log
// depth scale: shade = 2^(-strength * mean_k max(0, log2 d_p - log2 d_q)) over
// n_dirs neighbours at a fixed pixel radius (neighbours outside the image add
// nothing); background and depths beyond far_depth count as far_depth, so the
// background right next to the cloud gets a dark outline.  Foreground pixels
// return shade * AO * colour, background pixels shade * environment.
//
// gfx950 mapping: 32x16 pixel tiles, 256 threads, two pixels per thread (8
// rows apart; a wavefront's rows are 128-byte segments of every plane); the tile's log depths
// plus a halo of the radius are computed once per texel into LDS (log2 taken
// once per texel, not once per neighbour read), texels outside the image hold
// +inf so that they add max(0, z - inf) = 0 without a branch.  The neighbour
// offsets are LDS index deltas precomputed on the host for the tile pitch and
// read from the kernel arguments with scalar loads.  A block is short-lived,
// so its memory round trips set its time: the pixel's own depth, colour and AO
// are fetched before the barrier, in flight together with the halo fill.  The
// kernel streams depth + colour + AO in and HDR out once: HBM-bound.
#include "device_common.hpp"
#include "launch.hpp"

namespace epb {

// A block of 256 threads covers a 32 x (8 PPT) pixel tile, each thread PPT
// pixels of one column, 8 rows apart (rows of a wavefront stay 128-byte
// segments).  More pixels per thread put more independent fetches in flight
// per wavefront at the same occupancy.
constexpr int kEdlTx = 32, kEdlRows = 8, kEdlPpt = 2, kEdlTy = kEdlRows * kEdlPpt;
constexpr int kEdlThreads = kEdlTx * kEdlRows;
constexpr int kEdlPitchMax = kEdlTx + 2 * EPB_MAX_EDL_RADIUS;
constexpr int kEdlRowsMax = kEdlTy + 2 * EPB_MAX_EDL_RADIUS;

// Log depth of halo-tile texel q (row-major, pitch = 32 + 2r) or +inf outside
// the image; the load address is clamped so that every lane may issue it.
struct HaloTexel {
    unsigned idx;
    bool in;
};
__device__ __forceinline__ HaloTexel halo_texel(const EdlDesc &c, int X0, int Y0, int pitch, int q) {
    int ry = q / pitch, rx = q - ry * pitch;
    int gx = X0 - c.radius + rx, gy = Y0 - c.radius + ry;
    bool in = gx >= 0 && gx < c.W && gy >= 0 && gy < c.H;
    return HaloTexel{in ? __umul24((unsigned)gy, (unsigned)c.W) + (unsigned)gx : 0u, in};
}

template <typename TG, typename TA, typename TH>
__global__ void __launch_bounds__(kEdlThreads) k_edl(const EdlDesc c, int tiles) {
    constexpr int kEarly = 4;  // halo texels per thread fetched up front (all of them for radius <= 4)
    __shared__ float z[kEdlPitchMax * kEdlRowsMax];
    int tile = xcd_tile(blockIdx.x, tiles);
    int tiles_x = (c.W + kEdlTx - 1) / kEdlTx;
    int ty = tile / tiles_x;
    int X0 = (tile - ty * tiles_x) * kEdlTx, Y0 = ty * kEdlTy;
    int t = (int)threadIdx.x;
    int r = c.radius, pitch = kEdlTx + 2 * r, area = pitch * (kEdlTy + 2 * r);
    int lx = t % kEdlTx, ly = t / kEdlTx;
    int x = X0 + lx;
    unsigned plane = (unsigned)c.W * (unsigned)c.H;
    // Issue order: the pixels' depths, then the first halo texels, then (once
    // a depth says its pixel holds a point) that pixel's colour and AO taps --
    // all before the barrier, so that the pixels' own fetches overlap the halo's.
    bool valid[kEdlPpt], fg[kEdlPpt];
    unsigned p[kEdlPpt];
    float d[kEdlPpt];
#pragma unroll
    for (int k = 0; k < kEdlPpt; ++k) {
        int y = Y0 + ly + k * kEdlRows;
        valid[k] = x < c.W && y < c.H;
        p[k] = valid[k] ? __umul24((unsigned)y, (unsigned)c.W) + (unsigned)x : 0u;
        d[k] = ldf(c.depth, p[k]);
    }
    float hv[kEarly];
    bool hin[kEarly];
#pragma unroll
    for (int e = 0; e < kEarly; ++e) {
        int q = t + e * kEdlThreads;
        HaloTexel h = halo_texel(c, X0, Y0, pitch, q < area ? q : 0);
        hin[e] = h.in && q < area;
        hv[e] = ldf(c.depth, h.idx);
    }
    float col[kEdlPpt][3];
    float a00[kEdlPpt], a10[kEdlPpt], a01[kEdlPpt], a11[kEdlPpt];
#pragma unroll
    for (int k = 0; k < kEdlPpt; ++k) {
        fg[k] = valid[k] && !__builtin_isinf(d[k]);
        col[k][0] = col[k][1] = col[k][2] = 0.0f;
        a00[k] = a10[k] = a01[k] = a11[k] = 1.0f;
        if (fg[k]) {
            const TG *cp = (const TG *)c.color;
            col[k][0] = ldf(cp, p[k]);
            col[k][1] = ldf(cp, plane + p[k]);
            col[k][2] = ldf(cp, 2 * plane + p[k]);
            if (c.ao) {  // taps of the bilinear upsampling at (x / 2, y / 2), clamped, as in shading
                int y = Y0 + ly + k * kEdlRows;
                const TA *aop = (const TA *)c.ao;
                unsigned x0 = x >> 1, y0 = y >> 1;
                unsigned dx = (x & 1) && (int)x0 + 1 < c.Wh ? 1u : 0u;
                unsigned dy = (y & 1) && (int)y0 + 1 < c.Hh ? (unsigned)c.Wh : 0u;
                unsigned q = __umul24(y0, (unsigned)c.Wh) + x0;
                a00[k] = ldf(aop, q); a10[k] = ldf(aop, q + dx);
                a01[k] = ldf(aop, q + dy); a11[k] = ldf(aop, q + dy + dx);
            }
        }
    }
    // log depths of the tile and its halo (one log2 per texel; +inf outside the image)
#pragma unroll
    for (int e = 0; e < kEarly; ++e) {
        int q = t + e * kEdlThreads;
        if (q < area) z[q] = hin[e] ? log2f(fminf(hv[e], c.far_depth)) : __builtin_inff();
    }
    for (int q = t + kEarly * kEdlThreads; q < area; q += kEdlThreads) {  // radius > 4 only
        HaloTexel h = halo_texel(c, X0, Y0, pitch, q);
        z[q] = h.in ? log2f(fminf(ldf(c.depth, h.idx), c.far_depth)) : __builtin_inff();
    }
    __syncthreads();
    TH *hdr = (TH *)c.hdr;
#pragma unroll
    for (int k = 0; k < kEdlPpt; ++k) {
        if (!valid[k]) continue;
        int y = Y0 + ly + k * kEdlRows;
        int centre = (ly + k * kEdlRows + r) * pitch + lx + r;
        float zp = z[centre];
        float acc = 0.0f;
        for (int n = 0; n < c.n_dirs; ++n) acc += fmaxf(zp - z[centre + c.loff[n]], 0.0f);
        float shade = exp2f(c.neg_strength_over_n * acc);
        float out[3] = {0.0f, 0.0f, 0.0f};
        if (!fg[k]) {
            if (c.env) {
                float dvx = ((float)x + 0.5f - c.cx) * c.inv_fx;
                float dvy = -((float)y + 0.5f - c.cy) * c.inv_fy;
                v3 dw = mul_Rt(c.R, mk3(dvx, dvy, -1.0f));
                float4 e = cube_bilinear(c.env, c.env_dims, dw);
                out[0] = shade * e.x; out[1] = shade * e.y; out[2] = shade * e.z;
            }
        } else {
            float ao = 1.0f;
            if (c.ao) {
                float wx = (x & 1) ? 0.5f : 0.0f, wy = (y & 1) ? 0.5f : 0.0f;
                float top = fmaf(wx, a10[k] - a00[k], a00[k]), bot = fmaf(wx, a11[k] - a01[k], a01[k]);
                ao = fmaf(wy, bot - top, top);
            }
            float sv = shade * ao;
            out[0] = sv * col[k][0];
            out[1] = sv * col[k][1];
            out[2] = sv * col[k][2];
        }
        stf(hdr, p[k], out[0]);
        stf(hdr, plane + p[k], out[1]);
        stf(hdr, 2 * plane + p[k], out[2]);
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
template <typename TG, typename TA>
static void go_h(const EdlDesc &c, epb_dtype hd, int tiles, hipStream_t s) {
    if (hd == EPB_F32) hipLaunchKernelGGL((k_edl<TG, TA, float>), dim3(tiles), dim3(kEdlThreads), 0, s, c, tiles);
    else hipLaunchKernelGGL((k_edl<TG, TA, __half>), dim3(tiles), dim3(kEdlThreads), 0, s, c, tiles);
}
template <typename TG>
static void go_a(const EdlDesc &c, epb_dtype ad, epb_dtype hd, int tiles, hipStream_t s) {
    if (ad == EPB_F32) go_h<TG, float>(c, hd, tiles, s);
    else go_h<TG, __half>(c, hd, tiles, s);
}

hipError_t launch_edl(const EdlDesc &c, epb_dtype cdtype, epb_dtype ao_dtype, epb_dtype hdr_dtype, hipStream_t s) {
    int tiles = ceil_div(c.W, kEdlTx) * ceil_div(c.H, kEdlTy);
    if (cdtype == EPB_F32) go_a<float>(c, ao_dtype, hdr_dtype, tiles, s);
    else go_a<__half>(c, ao_dtype, hdr_dtype, tiles, s);
    return hipGetLastError();
}

}  // namespace epb
