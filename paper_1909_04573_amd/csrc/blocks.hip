// Block gather for the block-wise PCE protocol: fingerprints and test
// residuals are divided into disjoint b x b blocks and corresponding blocks
// are correlated (Sec. IV).  The gather writes the blocks of n planes
// block-major, out[k][p][r][c] = src[p][(k / nbc) b + r][(k % nbc) b + c], so
// the n planes of one block index are one contiguous batch for the PCE entry
// point.  Rows and columns past the last whole block are not used.
//
// grid.x runs over (block, plane) pairs and grid.y strides over the b*b
// elements of one block; consecutive threads copy consecutive elements of a
// block row.  Pure data movement (HBM bound).

#include "internal.h"
#include "stage_dev.h"

namespace prnu {
namespace {

constexpr int NT = 256;

__global__ __launch_bounds__(NT) void extract_blocks_kernel(const float *__restrict__ src, int n, int H, int W,
                                                            int b, int nbc, float *__restrict__ out) {
    const int kp = (int)blockIdx.x;  // block index * n + plane
    const int k = kp / n, p = kp - (kp / n) * n;
    const int br = k / nbc, bc = k - (k / nbc) * nbc;
    const int64_t bb = (int64_t)b * b;
    const PRNU_GLOBAL float *sp = gmem(src) + (int64_t)p * H * W + (int64_t)br * b * W + (int64_t)bc * b;
    PRNU_GLOBAL float *op = gmem(out) + (int64_t)kp * bb;
    const int64_t e0 = (int64_t)blockIdx.y * NT + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.y * NT;
    for (int64_t e = e0; e < bb; e += stride) {
        const int r = (int)(e / b), c = (int)(e - (e / b) * b);
        op[e] = sp[(int64_t)r * W + c];
    }
}

}  // namespace

hipError_t launch_extract_blocks(const float *src, int n, int H, int W, int b, float *out, hipStream_t s) {
    const int nbr = H / b, nbc = W / b;
    const int64_t bb = (int64_t)b * b;
    int gy = (int)((bb + NT - 1) / NT);
    if (gy > 64) gy = 64;
    KernelTimer kt("extract_blocks", 8.0 * (double)n * nbr * nbc * bb, s);
    extract_blocks_kernel<<<dim3((unsigned)(nbr * nbc * n), (unsigned)gy), NT, 0, s>>>(src, n, H, W, b, nbc, out);
    return hipGetLastError();
}

}  // namespace prnu
