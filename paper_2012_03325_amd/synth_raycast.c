/* Nearest-hit ray casting of sphere fields (and the plane y = 0) for the
 * seeded input generator: linear view depth and per-object surface attributes
 * per pixel.  Input synthesis only -- no shading arithmetic.  Double precision;
 * rows are cast in parallel with OpenMP.
 *
 * Pixel (x, y) casts the world-space ray o + t d with d = R^T ((x + .5 - cx)/fx,
 * -(y + .5 - cy)/fy, -1), so t is the linear view depth.  Spheres are tested in
 * index order within their pixel bounding boxes and the plane last; a hit
 * replaces the current one only when strictly nearer. */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

void syn_raycast(int n, const double *centers, const double *radii, const double *albedo,
                 const double *rough, const double *metal, int plane, const double *plane_albedo,
                 double plane_rough, double plane_metal, const double *R, const double *o, double fx,
                 double fy, double cx, double cy, int W, int H, const int32_t *bbox, float *depth_out,
                 float *normal_out, float *albedo_out, float *rough_out, float *metal_out) {
    size_t plane_px = (size_t)W * H;
#pragma omp parallel
    {
        double *dir = (double *)malloc(sizeof(double) * 3 * (size_t)W);
        double *t = (double *)malloc(sizeof(double) * (size_t)W);
        int *id = (int *)malloc(sizeof(int) * (size_t)W);
#pragma omp for schedule(dynamic, 4)
        for (int y = 0; y < H; ++y) {
            double vy = -(y + 0.5 - cy) / fy;
            for (int x = 0; x < W; ++x) {
                double vx = (x + 0.5 - cx) / fx, vz = -1.0;
                for (int j = 0; j < 3; ++j) dir[3 * x + j] = vx * R[j] + vy * R[3 + j] + vz * R[6 + j];
                t[x] = INFINITY;
                id[x] = -1;
            }
            for (int k = 0; k < n; ++k) {
                const int32_t *bb = bbox + 4 * k; /* x0, x1, y0, y1 */
                if (y < bb[2] || y >= bb[3]) continue;
                const double *c = centers + 3 * k;
                double oc[3] = {o[0] - c[0], o[1] - c[1], o[2] - c[2]};
                double cc = oc[0] * oc[0] + oc[1] * oc[1] + oc[2] * oc[2] - radii[k] * radii[k];
                for (int x = bb[0]; x < bb[1]; ++x) {
                    const double *d = dir + 3 * x;
                    double a = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                    double b = d[0] * oc[0] + d[1] * oc[1] + d[2] * oc[2];
                    double disc = b * b - a * cc;
                    if (disc < 0.0) continue;
                    double tt = (-b - sqrt(disc)) / a;
                    if (tt > 0.0 && tt < t[x]) {
                        t[x] = tt;
                        id[x] = k;
                    }
                }
            }
            if (plane) {
                for (int x = 0; x < W; ++x) {
                    double dy = dir[3 * x + 1];
                    if (!(dy < 0.0)) continue;
                    double tt = -o[1] / dy;
                    if (tt > 0.0 && tt < t[x]) {
                        t[x] = tt;
                        id[x] = n;
                    }
                }
            }
            for (int x = 0; x < W; ++x) {
                size_t p = (size_t)y * W + x;
                depth_out[p] = (float)t[x];
                if (!normal_out) continue;
                double nr[3] = {0, 0, 0}, al[3] = {0, 0, 0}, rg = 0.0, mt = 0.0;
                int k = id[x];
                if (k >= 0 && k < n) {
                    const double *d = dir + 3 * x, *c = centers + 3 * k;
                    for (int j = 0; j < 3; ++j) nr[j] = (o[j] + t[x] * d[j] - c[j]) / radii[k];
                    for (int j = 0; j < 3; ++j) al[j] = albedo[3 * k + j];
                    rg = rough[k];
                    mt = metal[k];
                } else if (k == n) {
                    nr[1] = 1.0;
                    for (int j = 0; j < 3; ++j) al[j] = plane_albedo[j];
                    rg = plane_rough;
                    mt = plane_metal;
                }
                if (k >= 0) {
                    double ln = sqrt(nr[0] * nr[0] + nr[1] * nr[1] + nr[2] * nr[2]);
                    for (int j = 0; j < 3; ++j) nr[j] /= ln;
                }
                for (int j = 0; j < 3; ++j) {
                    normal_out[j * plane_px + p] = (float)nr[j];
                    albedo_out[j * plane_px + p] = (float)al[j];
                }
                rough_out[p] = (float)rg;
                metal_out[p] = (float)mt;
            }
        }
        free(dir);
        free(t);
        free(id);
    }
}
