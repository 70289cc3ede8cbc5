// G-buffer and depth-map pass on sphere fields: the stand-in for the paper's
// rasterised geometry pass (Sec. 4) and its depth renders from each light
// (Sec. 5.1), on the device so that cameras and lights can change per frame.
//
// gfx950 mapping:
//  * k_sphere_boxes: one thread per sphere writes a conservative pixel box: the
//    projected corners of the sphere's bounding cube plus a texel of margin
//    (the cube lies wholly in front of the camera there, so the hull of its
//    corners contains the sphere's image); a sphere crossing the camera plane
//    covers the screen, one behind it nothing.
//  * k_raycast: one workgroup per 16x16 pixel tile.  Spheres are taken 256 at a
//    time in index order; each thread tests one box against the tile and the
//    overlapping indices are compacted into LDS in order (wave ballot and
//    prefix counts).  Every pixel then intersects the list; the list index is
//    wave-uniform, so sphere data come through scalar loads.  Candidates arrive
//    in index order and only a strictly nearer hit replaces the current one,
//    so an equal distance keeps the earlier object.
//  * intersections are double precision with contraction off (IEEE sqrt and
//    division), the results rounded to the destination types on store.
#include "device_common.hpp"
#include "launch.hpp"

namespace epb {

constexpr int kRayTile = 16;

__device__ __forceinline__ void camera_position(const RayCam &c, double o[3]) {
#pragma clang fp contract(off)
    for (int k = 0; k < 3; ++k) o[k] = -(c.M[k] * c.M[3] + c.M[4 + k] * c.M[7] + c.M[8 + k] * c.M[11]);
}

__global__ void __launch_bounds__(256) k_sphere_boxes(const RayScene s, const RayCam c, int4 *__restrict__ box) {
#pragma clang fp contract(off)
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= s.n) return;
    double cc[3] = {s.center[3 * k], s.center[3 * k + 1], s.center[3 * k + 2]};
    double r = s.radius[k];
    double v[3];
    for (int i = 0; i < 3; ++i) v[i] = c.M[4 * i] * cc[0] + c.M[4 * i + 1] * cc[1] + c.M[4 * i + 2] * cc[2] + c.M[4 * i + 3];
    const double eps = 1e-3;
    int4 b;
    if (-(v[2] + r) <= eps && -(v[2] - r) <= eps) {
        b = make_int4(0, 0, 0, 0);  // behind the camera
    } else if (-(v[2] + r) <= eps) {
        b = make_int4(0, c.W, 0, c.H);  // crosses the camera plane
    } else {
        double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
        for (int q = 0; q < 8; ++q) {
            double px3 = v[0] + ((q & 1) ? r : -r), py3 = v[1] + ((q & 2) ? r : -r), pz3 = v[2] + ((q & 4) ? r : -r);
            double z = -pz3;
            double px = c.cx + c.fx * px3 / z - 0.5, py = c.cy - c.fy * py3 / z - 0.5;
            x0 = fmin(x0, px); x1 = fmax(x1, px);
            y0 = fmin(y0, py); y1 = fmax(y1, py);
        }
        // clamp in double before converting (far-off boxes would overflow int)
        b.x = (int)fmax(floor(x0) - 1.0, 0.0);
        b.y = (int)fmin(ceil(x1) + 2.0, (double)c.W);
        b.z = (int)fmax(floor(y0) - 1.0, 0.0);
        b.w = (int)fmin(ceil(y1) + 2.0, (double)c.H);
    }
    box[k] = b;
}

template <typename TG>
__global__ void __launch_bounds__(kRayTile *kRayTile) k_raycast(const RayScene s, const RayCam c,
                                                                const int4 *__restrict__ box, RayOut out, int tiles) {
#pragma clang fp contract(off)
    __shared__ int list[256];
    __shared__ int wave_count[4];
    int tile = xcd_tile(blockIdx.x, tiles);
    int tiles_x = (c.W + kRayTile - 1) / kRayTile;
    int ty = tile / tiles_x;
    int X0 = (tile - ty * tiles_x) * kRayTile, Y0 = ty * kRayTile;
    int t = threadIdx.x;
    int x = X0 + (t % kRayTile), y = Y0 + (t / kRayTile);
    double o[3];
    camera_position(c, o);
    double v0 = ((double)x + 0.5 - c.cx) / c.fx, v1 = -(((double)y + 0.5 - c.cy) / c.fy), v2 = -1.0;
    double d[3];
    for (int k = 0; k < 3; ++k) d[k] = c.M[k] * v0 + c.M[4 + k] * v1 + c.M[8 + k] * v2;
    double aa = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    double best = __builtin_inf();
    int who = -1;
    int lane = t & 63, wv = t >> 6;
    for (int base = 0; base < s.n; base += 256) {
        int k = base + t;
        bool in = false;
        if (k < s.n) {
            int4 b = box[k];
            in = b.x < X0 + kRayTile && b.y > X0 && b.z < Y0 + kRayTile && b.w > Y0;
        }
        unsigned long long m = __ballot(in);
        int pre = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wave_count[wv] = __popcll(m);
        __syncthreads();
        int off = 0, total = 0;
        for (int w = 0; w < 4; ++w) {
            off += w < wv ? wave_count[w] : 0;
            total += wave_count[w];
        }
        if (in) list[off + pre] = k;
        __syncthreads();
        for (int i = 0; i < total; ++i) {
            int kk = __builtin_amdgcn_readfirstlane(list[i]);
            double oc0 = o[0] - s.center[3 * kk], oc1 = o[1] - s.center[3 * kk + 1], oc2 = o[2] - s.center[3 * kk + 2];
            double r = s.radius[kk];
            double b = d[0] * oc0 + d[1] * oc1 + d[2] * oc2;
            double c0 = (oc0 * oc0 + oc1 * oc1 + oc2 * oc2) - r * r;
            double disc = b * b - aa * c0;
            if (disc < 0.0) continue;
            double tt = (-b - sqrt(disc)) / aa;
            if (tt > 0.0 && tt < best) {
                best = tt;
                who = kk;
            }
        }
        __syncthreads();  // the list is refilled by the next chunk
    }
    if (s.plane && d[1] < 0.0) {
        double tt = -o[1] / d[1];
        if (tt > 0.0 && tt < best) {
            best = tt;
            who = s.n;
        }
    }
    if (x >= c.W || y >= c.H) return;
    unsigned p = __umul24((unsigned)y, (unsigned)c.W) + (unsigned)x;
    stf(out.depth, p, (float)best);
    if (!out.normal) return;
    float nr[3] = {0.0f, 0.0f, 0.0f}, al[3] = {0.0f, 0.0f, 0.0f}, rg = 0.0f, mt = 0.0f;
    if (who >= 0 && who < s.n) {
        double r = s.radius[who];
        double n3[3];
        for (int k = 0; k < 3; ++k) n3[k] = (o[k] + best * d[k] - s.center[3 * who + k]) / r;
        double len = sqrt(n3[0] * n3[0] + n3[1] * n3[1] + n3[2] * n3[2]);
        for (int k = 0; k < 3; ++k) nr[k] = (float)(n3[k] / len);
        for (int k = 0; k < 3; ++k) al[k] = s.albedo[3 * who + k];
        rg = s.rough[who];
        mt = s.metal[who];
    } else if (who == s.n) {
        nr[1] = 1.0f;
        for (int k = 0; k < 3; ++k) al[k] = s.plane_albedo[k];
        rg = s.plane_rough;
        mt = s.plane_metal;
    }
    unsigned plane = (unsigned)c.W * (unsigned)c.H;
    TG *nrm = (TG *)out.normal, *alb = (TG *)out.albedo;
    for (int k = 0; k < 3; ++k) {
        stf(nrm, k * plane + p, nr[k]);
        stf(alb, k * plane + p, al[k]);
    }
    stf((TG *)out.rough, p, rg);
    stf((TG *)out.metal, p, mt);
}

hipError_t launch_raycast(const RayScene &s, const RayCam &c, const RayOut &out, epb_dtype dtype, void *scratch,
                          hipStream_t st) {
    int4 *box = (int4 *)scratch;
    if (s.n > 0) hipLaunchKernelGGL(k_sphere_boxes, dim3(ceil_div(s.n, 256)), dim3(256), 0, st, s, c, box);
    int tiles = ceil_div(c.W, kRayTile) * ceil_div(c.H, kRayTile);
    if (dtype == EPB_F32)
        hipLaunchKernelGGL(k_raycast<float>, dim3(tiles), dim3(kRayTile * kRayTile), 0, st, s, c, box, out, tiles);
    else
        hipLaunchKernelGGL(k_raycast<__half>, dim3(tiles), dim3(kRayTile * kRayTile), 0, st, s, c, box, out, tiles);
    return hipGetLastError();
}

}  // namespace epb
