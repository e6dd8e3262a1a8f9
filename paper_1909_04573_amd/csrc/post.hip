// Fingerprint finalisation kernels: the MLE ratio K = A / B (Sec. III-A/B),
// per-channel zero-mean (row means, then column means), ITU-R BT.601 luma,
// per-plane variance, and the DFT-domain Wiener step applied to |F|/sqrt(N).
//
// All reductions are two-stage with a fixed order (per-block partials in
// double, then one block combining them), so results are deterministic.

#include "internal.h"
#include "stage_dev.h"
#include "wiener_dev.h"

namespace prnu {
namespace {

constexpr int NT = 256;
constexpr float kLuma[3] = {0.299f, 0.587f, 0.114f};

__device__ __forceinline__ float bf16f(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }

template <int ACC>
__global__ __launch_bounds__(NT) void ratio_kernel(const void *__restrict__ Av, const void *__restrict__ Bv,
                                                   int64_t n, float *__restrict__ K) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    double a, b;
    if (ACC == PRNU_ACC_F64) {
        a = static_cast<const double *>(Av)[i];
        b = static_cast<const double *>(Bv)[i];
    } else if (ACC == PRNU_ACC_F32) {
        a = static_cast<const float *>(Av)[i];
        b = static_cast<const float *>(Bv)[i];
    } else {  // value + compensation planes
        const float *A = static_cast<const float *>(Av);
        const float *B = static_cast<const float *>(Bv);
        a = (double)A[i] + (double)A[i + n];
        b = (double)B[i] + (double)B[i + n];
    }
    K[i] = b > 0.0 ? (float)(a / b) : 0.f;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block-wide sum in a fixed order; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) r += sh[k];
    __syncthreads();
    return r;
}

// Both sums below add their terms one by one in a fixed order; the loads of
// a batch of ZB terms are issued before the first add (a term past the end
// reads element 0 and adds an exact 0.0), so each thread keeps ZB loads in
// flight instead of waiting for every term in turn.
constexpr int ZB = 8;

// Row means: one wave per row of a plane.  rm[c*H + r] = mean of row r; lane
// l adds elements l, l + 64, ... in order, then the lanes are added by a
// fixed shuffle tree.
__global__ __launch_bounds__(NT) void row_mean_kernel(const float *__restrict__ x, int rows, int W,
                                                      double *__restrict__ rm) {
    const int row = blockIdx.x * (NT / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= rows) return;
    const float *p = x + (int64_t)row * W;
    double s = 0.0;
    for (int i0 = lane; i0 < W; i0 += 64 * ZB) {
        float v[ZB];
#pragma unroll
        for (int k = 0; k < ZB; ++k) {
            const int i = i0 + 64 * k;
            v[k] = p[i < W ? i : 0];
        }
#pragma unroll
        for (int k = 0; k < ZB; ++k) s += i0 + 64 * k < W ? (double)v[k] : 0.0;
    }
    s = wave_sum(s);
    if (lane == 0) rm[row] = s / (double)W;
}

// Column partial sums over chunks of RCH rows: colpart[c][chunk][col], the
// rows of a chunk added in order.
constexpr int RCH = 64;
__global__ __launch_bounds__(NT) void col_part_kernel(const float *__restrict__ x, int H, int W,
                                                      double *__restrict__ colpart) {
    const int col = blockIdx.x * NT + threadIdx.x;
    const int chunk = blockIdx.y, c = blockIdx.z;
    if (col >= W) return;
    const int nch = gridDim.y;
    const float *p = x + (int64_t)c * H * W + col;
    const int r0 = chunk * RCH, r1 = min(H, r0 + RCH);
    double s = 0.0;
    for (int rb = r0; rb < r1; rb += ZB) {
        float v[ZB];
#pragma unroll
        for (int k = 0; k < ZB; ++k) {
            const int r = rb + k;
            v[k] = p[(int64_t)(r < r1 ? r : r0) * W];
        }
#pragma unroll
        for (int k = 0; k < ZB; ++k) s += rb + k < r1 ? (double)v[k] : 0.0;
    }
    colpart[((int64_t)c * nch + chunk) * W + col] = s;
}

// adj[c][col] = column mean of the plane minus the mean of its row means.
__global__ __launch_bounds__(NT) void col_finish_kernel(const double *__restrict__ colpart, int nch,
                                                        const double *__restrict__ rm, int H, int W,
                                                        double *__restrict__ adj) {
    __shared__ double sh[NT / 64];
    __shared__ double mu;
    const int c = blockIdx.y;
    double s = 0.0;
    for (int r = threadIdx.x; r < H; r += NT) s += rm[(int64_t)c * H + r];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) mu = s / (double)H;
    __syncthreads();
    const int col = blockIdx.x * NT + threadIdx.x;
    if (col >= W) return;
    double t = 0.0;
    for (int k = 0; k < nch; ++k) t += colpart[((int64_t)c * nch + k) * W + col];
    adj[(int64_t)c * W + col] = t / (double)H - mu;
}

// out = x - rm[r] - adj[col] per channel, then luma (LUMA, C == 3).  Block
// (column block, row group, frame): the row index comes from the grid (no
// division per pixel) and the row means are uniform across the block.  CC:
// the channel count when it is 1 or 3 (loops unrolled), else 0 (runtime C).
template <int CC, bool LUMA, bool ZM>
__global__ __launch_bounds__(NT) void zm_apply_kernel(const float *__restrict__ x, int Cr, int H, int W,
                                                      const double *__restrict__ rm,
                                                      const double *__restrict__ adj,
                                                      float *__restrict__ out) {
    const int C = CC > 0 ? CC : Cr;
    const int col = blockIdx.x * NT + threadIdx.x;
    if (col >= W) return;
    const int64_t N = (int64_t)H * W;
    const int f = blockIdx.z;  // frame: planes f*C .. f*C + C-1
    x += (int64_t)f * C * N;
    out += (int64_t)f * (LUMA ? 1 : C) * N;
    if (ZM) {
        rm += (int64_t)f * C * H;
        adj += (int64_t)f * C * W;
    }
    for (int r = blockIdx.y; r < H; r += gridDim.y) {
        const int64_t i = (int64_t)r * W + col;
        if (LUMA) {
            double acc = 0.0;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                double v = (double)x[c * N + i];
                if (ZM) v -= rm[(int64_t)c * H + r] + adj[(int64_t)c * W + col];
                acc += (double)kLuma[c] * v;
            }
            out[i] = (float)acc;
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                double v = (double)x[c * N + i];
                if (ZM) v -= rm[(int64_t)c * H + r] + adj[(int64_t)c * W + col];
                out[c * N + i] = (float)v;
            }
        }
    }
}

template <int DT>
__global__ __launch_bounds__(NT) void luma_frames_kernel(const void *__restrict__ frames, int64_t npx,
                                                         int C, float *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    const int f = blockIdx.y;
    if (i >= npx) return;
    const int64_t e = ((int64_t)f * npx + i) * C;
    float v[3];
    for (int c = 0; c < C; ++c) {
        if (DT == PRNU_U8) v[c] = (float)static_cast<const uint8_t *>(frames)[e + c];
        else if (DT == PRNU_BF16) v[c] = bf16f(static_cast<const uint16_t *>(frames)[e + c]);
        else v[c] = static_cast<const float *>(frames)[e + c];
    }
    float r;
    if (C == 3) r = (float)((double)kLuma[0] * v[0] + (double)kLuma[1] * v[1] + (double)kLuma[2] * v[2]);
    else r = v[0];
    out[(int64_t)f * npx + i] = r;
}

// Interleaved u8 RGB frames, four pixels per thread: three aligned dwords in
// (12 bytes), one float4 out, the luma formed as in luma_frames_kernel.
// Needs npx % 4 == 0 and 4-byte aligned frames, 16-byte aligned out.
__global__ __launch_bounds__(NT) void luma_u8x4_kernel(const uint32_t *__restrict__ frames, int64_t npx,
                                                       float *__restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * NT + threadIdx.x;  // pixel quad
    const int f = blockIdx.y;
    if (4 * q >= npx) return;
    const uint32_t *src = frames + ((int64_t)f * npx / 4 + q) * 3;
    const uint32_t w0 = src[0], w1 = src[1], w2 = src[2];
    auto byte = [&](int b) {
        const uint32_t w = b < 4 ? w0 : b < 8 ? w1 : w2;
        return (float)((w >> (8 * (b & 3))) & 0xffu);
    };
    float r[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float v0 = byte(3 * k), v1 = byte(3 * k + 1), v2 = byte(3 * k + 2);
        r[k] = (float)((double)kLuma[0] * v0 + (double)kLuma[1] * v1 + (double)kLuma[2] * v2);
    }
    *reinterpret_cast<float4 *>(out + (int64_t)f * npx + 4 * q) = make_float4(r[0], r[1], r[2], r[3]);
}

// ---- per-plane sums: partials[p][blk] -------------------------------------
constexpr int RBLK = 64;  // blocks per plane

__global__ __launch_bounds__(NT) void plane_partial_kernel(const float *__restrict__ x, int64_t N,
                                                           const double *__restrict__ mean,
                                                           double *__restrict__ part) {
    __shared__ double sh[NT / 64];
    const int p = blockIdx.y;
    const float *xp = x + (int64_t)p * N;
    const double mu = mean ? mean[p] : 0.0;
    // the thread's terms in order, ZB loads in flight (a term past the end is 0)
    constexpr int64_t STRIDE = (int64_t)RBLK * NT;
    double s = 0.0;
    for (int64_t i0 = (int64_t)blockIdx.x * NT + threadIdx.x; i0 < N; i0 += ZB * STRIDE) {
        float x[ZB];
#pragma unroll
        for (int k = 0; k < ZB; ++k) x[k] = xp[i0 + k * STRIDE < N ? i0 + k * STRIDE : 0];
#pragma unroll
        for (int k = 0; k < ZB; ++k) {
            const double v = i0 + k * STRIDE < N ? (double)x[k] - mu : 0.0;
            s += mean ? v * v : v;
        }
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[(int64_t)p * RBLK + blockIdx.x] = s;
}

__global__ void plane_finish_kernel(const double *__restrict__ part, int n, int64_t N,
                                    double *__restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double s = 0.0;
    for (int k = 0; k < RBLK; ++k) s += part[(int64_t)p * RBLK + k];
    out[p] = s / (double)N;
}

// DFT-domain Wiener: tile of T x T bins with a 4-bin margin; q = |F|^2 / N
// (zero outside the array), G = F * rho.
constexpr int WT = 32, WH = 4, WNC = WT + 2 * WH, WNCS = WNC + 1;
__global__ __launch_bounds__(NT) void spectral_wiener_kernel(const float2 *__restrict__ F, int h, int w,
                                                             const double *__restrict__ var,
                                                             float sigma2, int tiles_c,
                                                             float2 *__restrict__ G) {
    __shared__ float q[WNC * WNCS];
    const int p = blockIdx.y;
    const int tr = blockIdx.x / tiles_c, tc = blockIdx.x - (blockIdx.x / tiles_c) * tiles_c;
    const int r0 = tr * WT - WH, c0 = tc * WT - WH;
    const int64_t N = (int64_t)h * w;
    const float2 *Fp = F + (int64_t)p * N;
    float2 *Gp = G + (int64_t)p * N;
    const float invN = (float)(1.0 / (double)N);
    staged_copy<NT, 8, float>(
        threadIdx.x, WNC * WNC,
        [&](int e) {
            const int i = e / WNC, j = e - (e / WNC) * WNC;
            const int gr = r0 + i, gc = c0 + j;
            const float2 z = Fp[(int64_t)min(max(gr, 0), h - 1) * w + min(max(gc, 0), w - 1)];
            const float v = (z.x * z.x + z.y * z.y) * invN;
            return gr >= 0 && gr < h && gc >= 0 && gc < w ? v : 0.f;
        },
        [&](int e, float v) { q[(e / WNC) * WNCS + e - (e / WNC) * WNC] = v; });
    __syncthreads();
    const float s2 = sigma2 >= 0.f ? sigma2 : (float)var[p];
    if (threadIdx.x < 2 * WT) {
        const int half = threadIdx.x / WT, kcl = threadIdx.x & (WT - 1);
        const int gc = tc * WT + kcl;
        auto load = [&](int r, int c) { return q[r * WNCS + c]; };
        auto emit = [&](int ko, float rho, float) {
            const int gr = r0 + ko;
            if (gr < h && gc < w) {
                const float2 z = Fp[(int64_t)gr * w + gc];
                Gp[(int64_t)gr * w + gc] = make_float2(z.x * rho, z.y * rho);
            }
        };
        wiener_column<WT / 2>(half * (WT / 2), kcl, s2, load, emit);
    }
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + NT - 1) / NT); }

}  // namespace

hipError_t launch_ratio(const void *A, const void *B, int acc_mode, int64_t n, float *K, hipStream_t s) {
    KernelTimer kt("ratio", (double)n * ((acc_mode == PRNU_ACC_F32 ? 8.0 : 16.0) + 4.0), s);
    if (acc_mode == PRNU_ACC_F64) ratio_kernel<PRNU_ACC_F64><<<blocks(n), NT, 0, s>>>(A, B, n, K);
    else if (acc_mode == PRNU_ACC_F32) ratio_kernel<PRNU_ACC_F32><<<blocks(n), NT, 0, s>>>(A, B, n, K);
    else ratio_kernel<PRNU_ACC_KAHAN_F32><<<blocks(n), NT, 0, s>>>(A, B, n, K);
    return hipGetLastError();
}

size_t zm_scratch_doubles(int nf, int C, int H, int W) {
    const int nch = (H + RCH - 1) / RCH;
    const size_t P = (size_t)nf * C;
    return P * H + P * nch * W + P * W;
}

hipError_t launch_zero_mean(const float *in, int nf, int C, int H, int W, bool zm, bool luma, float *out,
                            double *scratch, hipStream_t s) {
    const int nch = (H + RCH - 1) / RCH;
    const int P = nf * C;
    double *rm = scratch;
    double *colpart = rm + (size_t)P * H;
    double *adj = colpart + (size_t)P * nch * W;
    const int nout = luma ? 1 : C;
    KernelTimer kt("zero_mean", (double)nf * H * W * 4.0 * (C * (zm ? 3.0 : 1.0) + nout), s);
    if (zm) {
        row_mean_kernel<<<(unsigned)((P * H + 3) / 4), NT, 0, s>>>(in, P * H, W, rm);
        col_part_kernel<<<dim3(blocks(W), nch, P), NT, 0, s>>>(in, H, W, colpart);
        col_finish_kernel<<<dim3(blocks(W), P), NT, 0, s>>>(colpart, nch, rm, H, W, adj);
    }
    const dim3 g(blocks(W), (unsigned)(H < 65535 ? H : 65535), (unsigned)nf);
#define PRNU_ZM_APPLY(CC, L, Z) zm_apply_kernel<CC, L, Z><<<g, NT, 0, s>>>(in, C, H, W, rm, adj, out)
    if (luma) {  // C == 3
        if (zm) PRNU_ZM_APPLY(3, true, true);
        else PRNU_ZM_APPLY(3, true, false);
    } else if (C == 1) {
        if (zm) PRNU_ZM_APPLY(1, false, true);
        else PRNU_ZM_APPLY(1, false, false);
    } else if (C == 3) {
        if (zm) PRNU_ZM_APPLY(3, false, true);
        else PRNU_ZM_APPLY(3, false, false);
    } else {
        if (zm) PRNU_ZM_APPLY(0, false, true);
        else PRNU_ZM_APPLY(0, false, false);
    }
#undef PRNU_ZM_APPLY
    return hipGetLastError();
}

hipError_t launch_luma_frames(const void *frames, int dtype, int n, int H, int W, int C, float *out,
                              hipStream_t s) {
    const int64_t npx = (int64_t)H * W;
    dim3 g(blocks(npx), (unsigned)n);
    KernelTimer kt("luma_frames", (double)n * npx * (C * (dtype == PRNU_U8 ? 1.0 : dtype == PRNU_BF16 ? 2.0 : 4.0) + 4.0), s);
    const bool quads = dtype == PRNU_U8 && C == 3 && npx % 4 == 0 &&
                       (reinterpret_cast<uintptr_t>(frames) & 3) == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0;
    if (quads)
        luma_u8x4_kernel<<<dim3(blocks(npx / 4), (unsigned)n), NT, 0, s>>>(static_cast<const uint32_t *>(frames), npx,
                                                                          out);
    else if (dtype == PRNU_U8) luma_frames_kernel<PRNU_U8><<<g, NT, 0, s>>>(frames, npx, C, out);
    else if (dtype == PRNU_BF16) luma_frames_kernel<PRNU_BF16><<<g, NT, 0, s>>>(frames, npx, C, out);
    else luma_frames_kernel<PRNU_F32><<<g, NT, 0, s>>>(frames, npx, C, out);
    return hipGetLastError();
}

size_t reduce_scratch_doubles(int n, int64_t) { return (size_t)n * RBLK + (size_t)n; }

hipError_t launch_plane_variance(const float *x, int n, int64_t N, double *var, double *scratch,
                                 hipStream_t s) {
    double *part = scratch;
    double *mean = scratch + (size_t)n * RBLK;
    dim3 g(RBLK, (unsigned)n);
    KernelTimer kt("plane_variance", 8.0 * (double)n * N, s);
    plane_partial_kernel<<<g, NT, 0, s>>>(x, N, nullptr, part);
    plane_finish_kernel<<<(n + 63) / 64, 64, 0, s>>>(part, n, N, mean);
    plane_partial_kernel<<<g, NT, 0, s>>>(x, N, mean, part);
    plane_finish_kernel<<<(n + 63) / 64, 64, 0, s>>>(part, n, N, var);
    return hipGetLastError();
}

hipError_t launch_spectral_wiener(const float2 *F, int n, int h, int w, const double *var, float sigma2,
                                  float2 *G, hipStream_t s) {
    const int tr = (h + WT - 1) / WT, tc = (w + WT - 1) / WT;
    KernelTimer kt("spectral_wiener", 16.0 * (double)n * h * w, s);
    spectral_wiener_kernel<<<dim3((unsigned)(tr * tc), (unsigned)n), NT, 0, s>>>(F, h, w, var, sigma2,
                                                                                  tc, G);
    return hipGetLastError();
}

}  // namespace prnu
