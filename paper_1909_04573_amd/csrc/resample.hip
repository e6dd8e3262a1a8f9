// Bilinear resampling.
//  * Mixed-media matching: a still image's residual is resized (and cropped)
//    to the geometry of a video fingerprint before the two are correlated
//    (Sec. V-B).  Output pixel (y, x) samples the source at
//      ((y + oy + 0.5) / scale - 0.5, (x + ox + 0.5) / scale - 0.5)
//    (pixel centres).
//  * Stabilised video: the stabiliser shifts, rotates or zooms each frame
//    (Sec. II-B); the affine warp samples plane k % n_src at column
//    u = m0 x + m1 y + m2 and row v = m3 x + m4 y + m5 of its own matrix.
// Coordinates are computed in double and clamped to the plane (edge
// replication).  One thread per output pixel; pure gather (HBM / L2 bound).

#include "internal.h"
#include "stage_dev.h"

namespace prnu {
namespace {

constexpr int NT = 256;

__global__ __launch_bounds__(NT) void resample_bilinear_kernel(const float *__restrict__ src, int H, int W,
                                                               double inv_scale, int oy, int ox, int oh, int ow,
                                                               float *__restrict__ out) {
    const int p = (int)blockIdx.y;
    const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (e >= (int64_t)oh * ow) return;
    const int y = (int)(e / ow), x = (int)(e - (e / ow) * ow);
    // sample coordinates in double: exact to far below a pixel at any size
    double fy = ((double)(y + oy) + 0.5) * inv_scale - 0.5;
    double fx = ((double)(x + ox) + 0.5) * inv_scale - 0.5;
    fy = fmin(fmax(fy, 0.0), (double)(H - 1));
    fx = fmin(fmax(fx, 0.0), (double)(W - 1));
    const int y0 = (int)fy, x0 = (int)fx;
    const int y1 = y0 + 1 < H ? y0 + 1 : H - 1, x1 = x0 + 1 < W ? x0 + 1 : W - 1;
    const float wy = (float)(fy - (double)y0), wx = (float)(fx - (double)x0);
    const PRNU_GLOBAL float *sp = gmem(src) + (int64_t)p * H * W;
    const float a = sp[(int64_t)y0 * W + x0], b = sp[(int64_t)y0 * W + x1];
    const float c = sp[(int64_t)y1 * W + x0], d = sp[(int64_t)y1 * W + x1];
    const float top = a + wx * (b - a), bot = c + wx * (d - c);
    gmem(out)[(int64_t)p * oh * ow + e] = top + wy * (bot - top);
}

__global__ __launch_bounds__(NT) void warp_affine_kernel(const float *__restrict__ src, int n_src, int H, int W,
                                                         const double *__restrict__ affine, int oh, int ow,
                                                         float *__restrict__ out) {
    const int p = (int)blockIdx.y;
    const int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (e >= (int64_t)oh * ow) return;
    const int y = (int)(e / ow), x = (int)(e - (e / ow) * ow);
    const PRNU_GLOBAL double *m = gmem(affine) + 6 * (int64_t)p;  // uniform: scalar loads
    double fx = m[0] * (double)x + m[1] * (double)y + m[2];
    double fy = m[3] * (double)x + m[4] * (double)y + m[5];
    fy = fmin(fmax(fy, 0.0), (double)(H - 1));
    fx = fmin(fmax(fx, 0.0), (double)(W - 1));
    const int y0 = (int)fy, x0 = (int)fx;
    const int y1 = y0 + 1 < H ? y0 + 1 : H - 1, x1 = x0 + 1 < W ? x0 + 1 : W - 1;
    const float wy = (float)(fy - (double)y0), wx = (float)(fx - (double)x0);
    const PRNU_GLOBAL float *sp = gmem(src) + (int64_t)(p % n_src) * H * W;
    const float a = sp[(int64_t)y0 * W + x0], b = sp[(int64_t)y0 * W + x1];
    const float c = sp[(int64_t)y1 * W + x0], d = sp[(int64_t)y1 * W + x1];
    const float top = a + wx * (b - a), bot = c + wx * (d - c);
    gmem(out)[(int64_t)p * oh * ow + e] = top + wy * (bot - top);
}

}  // namespace

hipError_t launch_warp_affine(const float *src, int n_src, int H, int W, const double *affine, int n, int oh, int ow,
                              float *out, hipStream_t s) {
    const int64_t N = (int64_t)oh * ow;
    KernelTimer kt("warp_affine", (double)n * N * 8.0, s);
    warp_affine_kernel<<<dim3((unsigned)((N + NT - 1) / NT), (unsigned)n), NT, 0, s>>>(src, n_src, H, W, affine, oh,
                                                                                      ow, out);
    return hipGetLastError();
}

hipError_t launch_resample_bilinear(const float *src, int n, int H, int W, double scale, int oy, int ox, int oh,
                                    int ow, float *out, hipStream_t s) {
    const int64_t N = (int64_t)oh * ow;
    KernelTimer kt("resample_bilinear", (double)n * N * 8.0, s);
    resample_bilinear_kernel<<<dim3((unsigned)((N + NT - 1) / NT), (unsigned)n), NT, 0, s>>>(
        src, H, W, 1.0 / scale, oy, ox, oh, ow, out);
    return hipGetLastError();
}

}  // namespace prnu
