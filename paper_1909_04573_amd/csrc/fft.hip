// Mixed-radix complex FFT for gfx950 (radices 2, 3, 4, 5), used by the
// DFT-domain Wiener step and by the PCE correlation surfaces.
//
// A workgroup transforms `nvec` vectors of length N held in LDS as
// buf[n * nvec + v].  Each pass is a Stockham (self-sorting) step: with Ns the
// product of the radices already applied, butterfly j (k = j mod Ns) reads
// x[j + r N/R] for r < R, multiplies by the twiddle W_N^{k r N/(Ns R)},
// does an R-point DFT and writes y[(j / Ns) Ns R + k + r Ns].  Every thread
// keeps its butterflies' values in registers across one barrier, so the
// pass runs in place in a single LDS buffer.  Twiddles W_N^k = exp(-2 pi i k/N)
// are rounded to float from double-precision sincospi once per size.
//
// 2-D transforms are a pass along rows (vectors = rows) and a pass along
// columns (vectors = columns, coalesced across the nvec neighbouring columns).

#include <cmath>

#include "internal.h"

namespace prnu {
namespace {

constexpr int FNT = 256;
constexpr int LDS_CAP = 8704;  // complex elements per workgroup (68 KiB)

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

template <int R>
struct MaxB {
    static constexpr int v = (LDS_CAP / R + FNT - 1) / FNT;
};

template <int R>
__device__ __forceinline__ void stockham_pass(float2 *buf, int N, int nvec, int Ns,
                                              const float2 *__restrict__ tw, float sigma) {
    constexpr int MB = MaxB<R>::v;
    const int nb = (N / R) * nvec;
    const int NR = N / R;
    const int tws = N / (Ns * R);
    float2 v[MB][R];
    int dst[MB];
#pragma unroll
    for (int b = 0; b < MB; ++b) {
        const int idx = threadIdx.x + b * FNT;
        if (idx < nb) {
            const int vv = idx % nvec, j = idx / nvec;
            const int k = j % Ns;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float2 x = buf[(j + r * NR) * nvec + vv];
                if (r > 0) {
                    float2 w = tw[k * r * tws];
                    w.y *= -sigma;  // table holds exp(-2 pi i k / N); inverse uses the conjugate
                    x = cmul(x, make_float2(w.x, w.y));
                }
                v[b][r] = x;
            }
            dft<R>(v[b], sigma);
            dst[b] = ((j / Ns) * Ns * R + k) * nvec + vv;
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < MB; ++b) {
        const int idx = threadIdx.x + b * FNT;
        if (idx < nb) {
#pragma unroll
            for (int r = 0; r < R; ++r) buf[dst[b] + r * Ns * nvec] = v[b][r];
        }
    }
    __syncthreads();
}

// One batch of 1-D transforms: vectors v0 .. v0+nvec-1 of `count`, element n
// of vector v at base[v * vs + n * es].
__global__ __launch_bounds__(FNT) void fft_1d(float2 *__restrict__ data, int N, int count, int64_t es,
                                              int64_t vs, int64_t plane_stride, FftPlan plan,
                                              const float2 *__restrict__ tw, float sigma) {
    __shared__ float2 buf[LDS_CAP];
    const int nvec = plan.nvec;
    const int v0 = blockIdx.x * nvec;
    float2 *base = data + (int64_t)blockIdx.y * plane_stride;
    const int tot = N * nvec;
    for (int e = threadIdx.x; e < tot; e += FNT) {
        const int v = e % nvec, n = e / nvec;
        buf[e] = (v0 + v < count) ? base[(int64_t)(v0 + v) * vs + (int64_t)n * es] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    int Ns = 1;
    for (int p = 0; p < plan.nrad; ++p) {
        const int R = plan.rad[p];
        if (R == 4)
            stockham_pass<4>(buf, N, nvec, Ns, tw, sigma);
        else if (R == 2)
            stockham_pass<2>(buf, N, nvec, Ns, tw, sigma);
        else if (R == 3)
            stockham_pass<3>(buf, N, nvec, Ns, tw, sigma);
        else
            stockham_pass<5>(buf, N, nvec, Ns, tw, sigma);
        Ns *= R;
    }
    for (int e = threadIdx.x; e < tot; e += FNT) {
        const int v = e % nvec, n = e / nvec;
        if (v0 + v < count) base[(int64_t)(v0 + v) * vs + (int64_t)n * es] = buf[e];
    }
}

__global__ void twiddle_kernel(int n, float2 *tw) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double s, c;
    sincospi(-2.0 * (double)k / (double)n, &s, &c);
    tw[k] = make_float2((float)c, (float)s);
}

}  // namespace

bool make_fft_plan(int n, FftPlan *p) {
    if (n < 1 || n > LDS_CAP) return false;
    int m = n, k = 0;
    while (m % 4 == 0 && k < 16) { p->rad[k++] = 4; m /= 4; }
    while (m % 2 == 0 && k < 16) { p->rad[k++] = 2; m /= 2; }
    while (m % 3 == 0 && k < 16) { p->rad[k++] = 3; m /= 3; }
    while (m % 5 == 0 && k < 16) { p->rad[k++] = 5; m /= 5; }
    if (m != 1) return false;
    p->n = n;
    p->nrad = k;
    int nv = 16;
    while (nv > 1 && n * nv > LDS_CAP) nv /= 2;
    p->nvec = nv;
    return true;
}

size_t fft_twiddle_floats(int n) { return (size_t)2 * n; }

hipError_t launch_twiddles(int n, float2 *tw, hipStream_t s) {
    twiddle_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, tw);
    return hipGetLastError();
}

hipError_t launch_fft2(float2 *data, int batch, int h, int w, const FftPlan &ph, const FftPlan &pw,
                       const float2 *tw_h, const float2 *tw_w, int dir, hipStream_t s) {
    const float sigma = dir < 0 ? -1.f : 1.f;
    const int64_t plane = (int64_t)h * w;
    const double bytes = 16.0 * (double)batch * plane;  // read + write every complex element
    // rows: h vectors of length w
    dim3 gr((unsigned)((h + pw.nvec - 1) / pw.nvec), (unsigned)batch);
    {
        KernelTimer kt("fft_1d", bytes, s);
        fft_1d<<<gr, FNT, 0, s>>>(data, w, h, 1, w, plane, pw, tw_w, sigma);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // columns: w vectors of length h
    dim3 gc((unsigned)((w + ph.nvec - 1) / ph.nvec), (unsigned)batch);
    {
        KernelTimer kt("fft_1d", bytes, s);
        fft_1d<<<gc, FNT, 0, s>>>(data, h, w, w, 1, plane, ph, tw_h, sigma);
    }
    return hipGetLastError();
}

}  // namespace prnu
