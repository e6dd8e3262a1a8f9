// Device helpers of the mixed-radix Stockham FFT (see fft.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace prnu {

constexpr int FNT = 512;    // threads per FFT workgroup (8 waves hide LDS latency; the in-place transforms of 1080p planes take 30-50 KB of LDS, three to five workgroups per CU)
constexpr int FCAP = 5120;  // longest transform
constexpr int FVEC = 2560;  // vectors per workgroup: as many as keep nvec * N within this

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// sigma * i * z
__device__ __forceinline__ float2 cmuli(float2 z, float sigma) { return make_float2(-sigma * z.y, sigma * z.x); }
__device__ __forceinline__ float2 cscale(float2 z, float s) { return make_float2(z.x * s, z.y * s); }

// R-point DFT in place, y_k = sum_r x_r exp(sigma 2 pi i r k / R).
template <int R>
__device__ __forceinline__ void dft(float2 *x, float sigma);

template <>
__device__ __forceinline__ void dft<2>(float2 *x, float) {
    const float2 a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
}

template <>
__device__ __forceinline__ void dft<3>(float2 *x, float sigma) {
    constexpr float S3 = 0.866025403784438646763723170752936f;  // sin(2 pi / 3)
    const float2 t1 = cadd(x[1], x[2]), t2 = csub(x[1], x[2]);
    const float2 m = csub(x[0], cscale(t1, 0.5f));
    const float2 s = cmuli(cscale(t2, S3), sigma);
    x[0] = cadd(x[0], t1);
    x[1] = cadd(m, s);
    x[2] = csub(m, s);
}

template <>
__device__ __forceinline__ void dft<4>(float2 *x, float sigma) {
    const float2 a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
    const float2 c = cadd(x[1], x[3]), d = cmuli(csub(x[1], x[3]), sigma);
    x[0] = cadd(a, c);
    x[2] = csub(a, c);
    x[1] = cadd(b, d);
    x[3] = csub(b, d);
}

template <>
__device__ __forceinline__ void dft<5>(float2 *x, float sigma) {
    constexpr float C1 = 0.309016994374947424102293417182819f;   // cos(2 pi / 5)
    constexpr float C2 = -0.809016994374947424102293417182819f;  // cos(4 pi / 5)
    constexpr float S1 = 0.951056516295153572116439333379382f;   // sin(2 pi / 5)
    constexpr float S2 = 0.587785252292473129168705954639073f;   // sin(4 pi / 5)
    const float2 t1 = cadd(x[1], x[4]), t2 = cadd(x[2], x[3]);
    const float2 t3 = csub(x[1], x[4]), t4 = csub(x[2], x[3]);
    const float2 a1 = cadd(x[0], cadd(cscale(t1, C1), cscale(t2, C2)));
    const float2 a2 = cadd(x[0], cadd(cscale(t1, C2), cscale(t2, C1)));
    const float2 b1 = cmuli(cadd(cscale(t3, S1), cscale(t4, S2)), sigma);
    const float2 b2 = cmuli(csub(cscale(t3, S2), cscale(t4, S1)), sigma);
    x[0] = cadd(x[0], cadd(t1, t2));
    x[1] = cadd(a1, b1);
    x[4] = csub(a1, b1);
    x[2] = cadd(a2, b2);
    x[3] = csub(a2, b2);
}

// Exact j / d for 0 <= j < 2^20 and d >= 1 (float estimate plus correction).
__device__ __forceinline__ int udiv_small(int j, int d, float inv_d) {
    int q = (int)((float)j * inv_d);
    if (q * d > j) --q;
    if ((q + 1) * d <= j) ++q;
    return q;
}

template <int R>
__device__ __forceinline__ void stockham_pass(const float2 *__restrict__ src, float2 *__restrict__ dst, int N,
                                              int nvec, int lvec, int Ns, const float2 *__restrict__ tw,
                                              float sigma) {
    // KB butterflies per thread per batch: their LDS reads are issued together
    constexpr int KB = R == 5 ? 3 : 4;
    const int NR = N / R;
    const int nb = NR * nvec;
    const int tws = N / (Ns * R);
    const float inv_ns = 1.0f / (float)Ns;
    for (int idx0 = threadIdx.x; idx0 < nb; idx0 += KB * FNT) {
        float2 v[KB][R];
        int kk[KB], d0[KB];
#pragma unroll
        for (int b = 0; b < KB; ++b) {
            const int idx = idx0 + b * FNT;
            if (idx < nb) {
                const int vv = idx & (nvec - 1), j = idx >> lvec;
                const int jq = udiv_small(j, Ns, inv_ns);
                const int k = j - jq * Ns;
                kk[b] = k;
                d0[b] = (jq * Ns * R + k) * nvec + vv;
#pragma unroll
                for (int r = 0; r < R; ++r) v[b][r] = src[(j + r * NR) * nvec + vv];
            }
        }
#pragma unroll
        for (int b = 0; b < KB; ++b) {
            const int idx = idx0 + b * FNT;
            if (idx < nb) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    float2 w = tw[kk[b] * r * tws];
                    w.y *= -sigma;  // table holds exp(-2 pi i k / N); the inverse uses its conjugate
                    v[b][r] = cmul(v[b][r], w);
                }
                dft<R>(v[b], sigma);
#pragma unroll
                for (int r = 0; r < R; ++r) dst[d0[b] + r * Ns * nvec] = v[b][r];
            }
        }
    }
    __syncthreads();
}

// Transform the nvec vectors in b0 (layout [n][nvec]); returns the buffer
// holding the result (b0 or b1).
__device__ __forceinline__ const float2 *fft_lds(float2 *b0, float2 *b1, const FftPlan &plan,
                                                 const float2 *__restrict__ tw, float sigma) {
    float2 *src = b0, *dst = b1;
    int Ns = 1;
    for (int p = 0; p < plan.nrad; ++p) {
        const int R = plan.rad[p];
        if (R == 4)
            stockham_pass<4>(src, dst, plan.n, plan.nvec, plan.lvec, Ns, tw, sigma);
        else if (R == 2)
            stockham_pass<2>(src, dst, plan.n, plan.nvec, plan.lvec, Ns, tw, sigma);
        else if (R == 3)
            stockham_pass<3>(src, dst, plan.n, plan.nvec, plan.lvec, Ns, tw, sigma);
        else
            stockham_pass<5>(src, dst, plan.n, plan.nvec, plan.lvec, Ns, tw, sigma);
        float2 *t = src;
        src = dst;
        dst = t;
        Ns *= R;
    }
    return src;
}

// ---------------------------------------------------------------------------
// The same transform for a length N and vector count NV fixed at compile
// time: every loop bound, index division and twiddle stride is a constant, so
// the per-butterfly index arithmetic of the passes folds away.  Radices are
// taken in the order make_fft_plan uses (fours, a two, threes, fives).
struct Radices {
    int n;
    int r[16];
};
constexpr Radices radices_of(int N) {
    Radices L{0, {}};
    int m = N;
    while (m % 4 == 0 && L.n < 16) { L.r[L.n++] = 4; m /= 4; }
    while (m % 2 == 0 && L.n < 16) { L.r[L.n++] = 2; m /= 2; }
    while (m % 3 == 0 && L.n < 16) { L.r[L.n++] = 3; m /= 3; }
    while (m % 5 == 0 && L.n < 16) { L.r[L.n++] = 5; m /= 5; }
    return L;
}
constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

// The passes run in place in one LDS buffer: every thread first takes all
// of its butterflies' inputs into registers and transforms them, and writes
// them back after a barrier, so a workgroup needs half the LDS of the
// two-buffer passes of the runtime plan (more workgroups per CU).
template <int N, int R, int NS, int NV>
__device__ __forceinline__ void stockham_inplace(float2 *buf, const float2 *__restrict__ tw, float sigma) {
    constexpr int NR = N / R, NB = NR * NV, TWS = N / (NS * R);
    constexpr int ITER = (NB + FNT - 1) / FNT;
    float2 v[ITER][R];
    unsigned d0[ITER];
#pragma unroll
    for (int i = 0; i < ITER; ++i) {
        const unsigned idx = threadIdx.x + (unsigned)(i * FNT);
        if ((i + 1) * FNT <= NB || idx < (unsigned)NB) {
            const unsigned vv = idx % NV, j = idx / NV;
            const unsigned k = j % NS, jq = j / NS;
            d0[i] = (jq * (NS * R) + k) * NV + vv;
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = buf[(j + r * NR) * NV + vv];
            if (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    float2 w = tw[k * (r * TWS)];
                    w.y *= -sigma;
                    v[i][r] = cmul(v[i][r], w);
                }
            }
            dft<R>(v[i], sigma);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITER; ++i) {
        const unsigned idx = threadIdx.x + (unsigned)(i * FNT);
        if ((i + 1) * FNT <= NB || idx < (unsigned)NB) {
#pragma unroll
            for (int r = 0; r < R; ++r) buf[d0[i] + r * NS * NV] = v[i][r];
        }
    }
    __syncthreads();
}

template <int N, int NV, int P = 0, int NS = 1>
__device__ __forceinline__ void fft_fixed_inplace(float2 *buf, const float2 *__restrict__ tw, float sigma) {
    constexpr Radices L = radices_of(N);
    if constexpr (P < L.n) {
        constexpr int R = L.r[P];
        stockham_inplace<N, R, NS, NV>(buf, tw, sigma);
        fft_fixed_inplace<N, NV, P + 1, NS * R>(buf, tw, sigma);
    }
}

// Runtime plan for N = 0 (two buffers, the result in either), the
// compile-time passes in place in b0 otherwise (b1 unused).
template <int N, int NV>
__device__ __forceinline__ const float2 *fft_run(float2 *b0, float2 *b1, const FftPlan &plan,
                                                 const float2 *__restrict__ tw, float sigma) {
    if constexpr (N == 0) {
        return fft_lds(b0, b1, plan, tw, sigma);
    } else {
        fft_fixed_inplace<N, NV>(b0, tw, sigma);
        return b0;
    }
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block-wide sum in a fixed order; the result is valid in thread 0.  Every
// thread of the block must call it.
__device__ __forceinline__ double block_sum_f64(double v, double *sh) {
    v = wave_sum_f64(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) r += sh[k];
    __syncthreads();
    return r;
}

}  // namespace prnu
