// Hand-written adjoint of the differentiable chain (zero-mean fingerprints,
// fixed-peak PCE) with respect to the shrinkage noise variances s_l.
//
// Denoiser: with r = c s / max(s, m) per detail coefficient (m the smallest
// 3/5/7/9 window mean of c^2), dr/ds = [m > s] c / m, checkpointed by the
// forward kernel.  The residual is a cropped periodised synthesis of the r's,
// so the gradient of the r's is the periodised analysis of the zero-embedded
// gradient of W; dwt_vjp runs that analysis level by level (approximation
// to the next level, details dotted with the checkpoint) and leaves one
// FP64 partial sum per tile.
//
// PCE (peak at 0): C(s) = sum_t xc(t+s) yc(t), E = sum_{s outside N} C^2 /
// (N - n^2), PCE = sign(C0) C0^2 / E.  dPCE/dC = alpha C~ + beta delta_0 with
// C~ = C masked on N, alpha = -2 sign(C0) C0^2 / (E^2 (N - n^2)),
// beta = 2 |C0| / E; then dPCE/dyc = corr(gC, xc) and dPCE/dxc = conv(gC, yc),
// both through the FFT with the DC bin cleared (the centring's adjoint).

#include <cfloat>

#include "fft_dev.h"
#include "internal.h"
#include "stage_dev.h"

namespace prnu {
namespace {

constexpr int NT = 256;
constexpr int VT = 32;  // coefficients per tile side

template <int TAPS>
struct VjpGeom {
    static constexpr int IN = 2 * VT + TAPS - 2;
    static constexpr int INS = (IN + 3) / 4 * 4;
};

// Periodic wrap into [0, n), then the crop's adjoint: outside the stored
// window [off, off + stored) the padded plane is zero (-1 marks that).
__device__ __forceinline__ int map_zero(int p, int n, int off, int stored) {
    int pm = p % n;
    if (pm < 0) pm += n;
    const int q = pm - off;
    return (q >= 0 && q < stored) ? q : -1;
}

template <int TAPS>
__global__ __launch_bounds__(NT) void dwt_vjp(const float *__restrict__ src, int64_t src_stride, int src_rows,
                                              int src_cols, const float *__restrict__ mul, int64_t mul_stride,
                                              const float *__restrict__ div, int n_r, int n_c, int off_r, int off_c,
                                              float *__restrict__ ll_out, const float *__restrict__ ckpt,
                                              int64_t ckpt_stride, double *__restrict__ part, int tiles_c, Filter f) {
    using G = VjpGeom<TAPS>;
    constexpr int IN = G::IN, INS = G::INS, NC = VT;
    __shared__ __align__(16) float tile[IN * INS];
    __shared__ __align__(16) float rlo[IN * NC];
    __shared__ __align__(16) float rhi[IN * NC];
    __shared__ int rmap[IN];
    __shared__ int cmap[IN];
    __shared__ double red[NT / 64];
    const int hk = n_r >> 1, wk = n_c >> 1;
    const int tr = blockIdx.x / tiles_c, tc = blockIdx.x - (blockIdx.x / tiles_c) * tiles_c;
    const int k0r = tr * VT, k0c = tc * VT;
    const int tid = threadIdx.x;
    const float *sp = src + (int64_t)blockIdx.y * src_stride;
    const float *mp = mul ? mul + (int64_t)blockIdx.y * mul_stride : nullptr;
    if (tid < IN)
        rmap[tid] = map_zero(2 * k0r + tid, n_r, off_r, src_rows);
    else if (tid < 2 * IN)
        cmap[tid - IN] = map_zero(2 * k0c + tid - IN, n_c, off_c, src_cols);
    __syncthreads();
    staged_copy<NT, 8, float>(
        tid, IN * IN,
        [&](int e) {
            const int i = e / IN, j = e - (e / IN) * IN;
            const int r = rmap[i], c = cmap[j];
            const int64_t o = (int64_t)max(r, 0) * src_cols + max(c, 0);
            float v = sp[o];
            if (mp) v *= mp[o];
            if (div) {
                const float d = div[o];
                v = d > 0.f ? v / d : 0.f;
            }
            return r >= 0 && c >= 0 ? v : 0.f;
        },
        [&](int e, float v) { tile[(e / IN) * INS + e - (e / IN) * IN] = v; });
    __syncthreads();
    constexpr int NQ = NC / 4;
    for (int it = tid; it < IN * NQ; it += NT) {
        const int i = it / NQ, kq = it - (it / NQ) * NQ;
        float x[TAPS + 6];
#pragma unroll
        for (int t = 0; t < TAPS + 6; ++t) x[t] = tile[i * INS + 8 * kq + t];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            float lo = 0.f, hi = 0.f;
#pragma unroll
            for (int j = 0; j < TAPS; ++j) {
                lo = fmaf(f.h[j], x[2 * u + j], lo);
                hi = fmaf(f.g[j], x[2 * u + j], hi);
            }
            rlo[i * NC + 4 * kq + u] = lo;
            rhi[i * NC + 4 * kq + u] = hi;
        }
    }
    __syncthreads();
    const int64_t band = (int64_t)hk * wk;
    const float *cp = ckpt + (int64_t)blockIdx.y * ckpt_stride;
    double acc = 0.0;
    for (int it = tid; it < NC * (NC / 2); it += NT) {
        const int kc = it % NC, kp = it / NC;
        float xl[TAPS + 2], xh[TAPS + 2];
#pragma unroll
        for (int t = 0; t < TAPS + 2; ++t) {
            xl[t] = rlo[(4 * kp + t) * NC + kc];
            xh[t] = rhi[(4 * kp + t) * NC + kc];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            float ll = 0.f, hl = 0.f, lh = 0.f, hh = 0.f;
#pragma unroll
            for (int j = 0; j < TAPS; ++j) {
                ll = fmaf(f.h[j], xl[2 * u + j], ll);
                hl = fmaf(f.g[j], xl[2 * u + j], hl);
                lh = fmaf(f.h[j], xh[2 * u + j], lh);
                hh = fmaf(f.g[j], xh[2 * u + j], hh);
            }
            const int gr = k0r + 2 * kp + u, gc = k0c + kc;
            if (gr < hk && gc < wk) {
                const int64_t o = (int64_t)gr * wk + gc;
                if (ll_out) ll_out[(int64_t)blockIdx.y * band + o] = ll;
                acc += (double)lh * cp[o] + (double)hl * cp[band + o] + (double)hh * cp[2 * band + o];
            }
        }
    }
    // block sum in fixed order
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int k = 0; k < NT / 64; ++k) s += red[k];
        part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
    }
}

__global__ void vjp_finish(const double *__restrict__ part, int64_t n, double *__restrict__ out) {
    __shared__ double red[NT / 64];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += NT) s += part[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < NT / 64; ++k) t += red[k];
        *out += t;
    }
}

// ---- PCE adjoint -------------------------------------------------------------
struct PvjpCoef {
    double alpha, beta, pce;
};

// Per pair: total energy (partials in fixed order) and the neighbourhood,
// then alpha, beta, PCE.  z holds N * C in its real part.
__global__ __launch_bounds__(NT) void pvjp_coef(const float2 *__restrict__ z, int h, int w, int nbhd, int p0,
                                                PvjpCoef *__restrict__ coef, double *__restrict__ pce) {
    __shared__ double red[NT / 64];
    __shared__ double s_tot;
    const int64_t N = (int64_t)h * w;
    const float2 *zp = z + (int64_t)blockIdx.x * N;
    double e = 0.0;
    for (int64_t i = threadIdx.x; i < N; i += NT) {
        const double v = zp[i].x;
        e += v * v;
    }
    e = block_sum_f64(e, red);
    if (threadIdx.x == 0) s_tot = e;
    __syncthreads();
    const int r = nbhd / 2;
    double n11 = 0.0;
    for (int t = threadIdx.x; t < nbhd * nbhd; t += NT) {
        const int dy = t / nbhd - r, dx = t % nbhd - r;
        const int yy = (dy % h + h) % h, xx = (dx % w + w) % w;
        const double v = zp[(int64_t)yy * w + xx].x;
        n11 += v * v;
    }
    n11 = block_sum_f64(n11, red);
    if (threadIdx.x == 0) {
        const double invN = 1.0 / (double)N;
        const double den = (double)(N - (int64_t)nbhd * nbhd);
        const double c0 = (double)zp[0].x * invN;
        const double E = (s_tot - n11) * invN * invN / den;
        PvjpCoef k{0.0, 0.0, 0.0};
        if (E > 0.0) {
            const double sg = c0 >= 0.0 ? 1.0 : -1.0;
            k.pce = sg * c0 * c0 / E;
            k.alpha = -2.0 * sg * c0 * c0 / (E * E * den);
            k.beta = 2.0 * fabs(c0) / E;
        }
        coef[blockIdx.x] = k;
        if (pce) pce[p0 + blockIdx.x] = k.pce;
    }
}

// z <- alpha * C~ + beta * delta_0 (real), C~ = C with the n x n block around 0 cleared.
__global__ __launch_bounds__(NT) void pvjp_gc(float2 *__restrict__ z, int h, int w, int nbhd,
                                              const PvjpCoef *__restrict__ coef) {
    const int64_t N = (int64_t)h * w;
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= N) return;
    const PvjpCoef k = coef[blockIdx.y];
    float2 *zp = z + (int64_t)blockIdx.y * N;
    const int y = (int)(i / w), x = (int)(i - (int64_t)(i / w) * w);
    const int r = nbhd / 2;
    const bool inN = (y <= r || y >= h - r) && (x <= r || x >= w - r);
    const double c = (double)zp[i].x / (double)N;
    double g = inN ? 0.0 : k.alpha * c;
    if (i == 0) g += k.beta;
    zp[i] = make_float2((float)g, 0.f);
}

// t1 = conj(G) X^_q (-> gradient of yc), t2 = G V (-> gradient of xc); DC cleared.
__global__ __launch_bounds__(NT) void pvjp_products(const float2 *__restrict__ G, const float2 *__restrict__ Xs,
                                                    const float2 *__restrict__ V, int ny, int p0, int64_t N,
                                                    float2 *__restrict__ t1, float2 *__restrict__ t2) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= N) return;
    const int q = (p0 + (int)blockIdx.y) / ny;
    const int64_t o = (int64_t)blockIdx.y * N + i;
    const float2 g = G[o], x = Xs[(int64_t)q * N + i], v = V[o];
    float2 a = make_float2(g.x * x.x + g.y * x.y, g.x * x.y - g.y * x.x);  // conj(g) * x
    float2 b = make_float2(g.x * v.x - g.y * v.y, g.x * v.y + g.y * v.x);  // g * v
    if (i == 0) {
        a = make_float2(0.f, 0.f);
        b = make_float2(0.f, 0.f);
    }
    t1[o] = a;
    t2[o] = b;
}

// gX[q] += w * Re(t2)/N, gY[j] += w * mod_q * Re(t1)/N over the chunk's pairs in order.
__global__ __launch_bounds__(NT) void pvjp_accum(const float2 *__restrict__ t1, const float2 *__restrict__ t2,
                                                 const double *__restrict__ wts, const float *__restrict__ mod,
                                                 int n, int ny, int p0, int64_t N, float *__restrict__ gX,
                                                 float *__restrict__ gY) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= N) return;
    const float invN = (float)(1.0 / (double)N);
    for (int p = 0; p < n; ++p) {
        const int pid = p0 + p;
        const int q = pid / ny, j = pid % ny;
        const float wt = (float)wts[pid];
        if (wt == 0.f) continue;
        const int64_t o = (int64_t)p * N + i;
        gX[(int64_t)q * N + i] += wt * t2[o].x * invN;
        const float m = mod ? mod[(int64_t)q * N + i] : 1.f;
        gY[(int64_t)j * N + i] += wt * m * t1[o].x * invN;
    }
}

__global__ __launch_bounds__(NT) void fill_zero(float *__restrict__ x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i < n) x[i] = 0.f;
}

inline unsigned ublocks(int64_t n) { return (unsigned)((n + NT - 1) / NT); }

}  // namespace

int dwt_vjp_tiles(int hk, int wk) { return ((hk + VT - 1) / VT) * ((wk + VT - 1) / VT); }

hipError_t launch_dwt_vjp(int taps, const Filter &f, const float *src, int64_t src_stride, int src_rows,
                          int src_cols, const float *mul, int64_t mul_stride, const float *div, int n_r, int n_c,
                          int off_r, int off_c, float *ll_out, const float *ckpt, int64_t ckpt_stride, int planes,
                          double *part, hipStream_t s) {
    const int hk = n_r / 2, wk = n_c / 2;
    const int tc = (wk + VT - 1) / VT;
    dim3 grid((unsigned)dwt_vjp_tiles(hk, wk), (unsigned)planes);
    KernelTimer kt(taps == 16 ? "dwt_vjp<16>" : "dwt_vjp<8>",
                   (double)planes * 4.0 * ((double)src_rows * src_cols + 4.0 * hk * wk), s);
    if (taps == 16)
        dwt_vjp<16><<<grid, NT, 0, s>>>(src, src_stride, src_rows, src_cols, mul, mul_stride, div, n_r, n_c, off_r,
                                        off_c, ll_out, ckpt, ckpt_stride, part, tc, f);
    else
        dwt_vjp<8><<<grid, NT, 0, s>>>(src, src_stride, src_rows, src_cols, mul, mul_stride, div, n_r, n_c, off_r,
                                       off_c, ll_out, ckpt, ckpt_stride, part, tc, f);
    return hipGetLastError();
}

hipError_t launch_vjp_finish(const double *part, int64_t n, double *out, hipStream_t s) {
    vjp_finish<<<1, NT, 0, s>>>(part, n, out);
    return hipGetLastError();
}

size_t pvjp_coef_bytes(int n) { return (size_t)n * sizeof(PvjpCoef); }

hipError_t launch_pvjp(float2 *Z, float2 *V, float2 *T1, float2 *T2, const float2 *Xs, int n, int h, int w,
                       int nbhd, int ny, int p0, const FftPlan &ph, const FftPlan &pw, const float2 *tw_h,
                       const float2 *tw_w, void *coef, const double *wts, const float *mod, double *pce, float *gX,
                       float *gY, hipStream_t s) {
    // Z holds X^ conj(V) transformed back: N * C per pair.
    const int64_t N = (int64_t)h * w;
    PvjpCoef *k = static_cast<PvjpCoef *>(coef);
    pvjp_coef<<<(unsigned)n, NT, 0, s>>>(Z, h, w, nbhd, p0, k, pce);
    pvjp_gc<<<dim3(ublocks(N), (unsigned)n), NT, 0, s>>>(Z, h, w, nbhd, k);
    hipError_t e = launch_fft2(Z, n, h, w, ph, pw, tw_h, tw_w, -1, s);
    if (e != hipSuccess) return e;
    pvjp_products<<<dim3(ublocks(N), (unsigned)n), NT, 0, s>>>(Z, Xs, V, ny, p0, N, T1, T2);
    e = launch_fft2(T1, n, h, w, ph, pw, tw_h, tw_w, +1, s);
    if (e != hipSuccess) return e;
    e = launch_fft2(T2, n, h, w, ph, pw, tw_h, tw_w, +1, s);
    if (e != hipSuccess) return e;
    pvjp_accum<<<ublocks(N), NT, 0, s>>>(T1, T2, wts, mod, n, ny, p0, N, gX, gY);
    return hipGetLastError();
}

hipError_t launch_fill_zero(float *x, int64_t n, hipStream_t s) {
    fill_zero<<<ublocks(n), NT, 0, s>>>(x, n);
    return hipGetLastError();
}

}  // namespace prnu
