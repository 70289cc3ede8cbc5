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
#include "ssao_tiles.hpp"

namespace epb {

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
    __shared__ float sd[blur_lds_rows<kBlurTx, kBlurTy>()][kBlurTx + 3];
    __shared__ float sa[blur_lds_rows<kBlurTx, kBlurTy>()][kBlurTx + 3];
    ssao_blur_tile<kBlurTx, kBlurTy, TA>(c, xcd_tile(blockIdx.x, tiles), sd, sa);
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
    __shared__ float sd[blur_lds_rows<kBlurTx, kBlurTy>()][kBlurTx + 3];
    __shared__ float sa[blur_lds_rows<kBlurTx, kBlurTy>()][kBlurTx + 3];
    const BatchHeader *h = (const BatchHeader *)table;
    const int *start = batch_start(table, kStBlur);
    const ViewDesc *views = batch_views(table);
    XcdRange w = xcd_range(h->total[kStBlur]);
    for (int it = w.lb; it < w.count; it += w.stride) {
        int g = w.first + it;
        int v = find_view(start, h->n_views, g);
        ssao_blur_tile<kBlurTx, kBlurTy, TA>(views[v].ssao, g - start[v], sd, sa);
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
