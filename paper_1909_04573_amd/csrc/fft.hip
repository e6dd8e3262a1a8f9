// Mixed-radix FFTs for gfx950 (radices 2, 3, 4, 5), used by the DFT-domain
// Wiener step and by PCE.
//
// A workgroup transforms `nvec` vectors of length N held in LDS as
// buf[n * nvec + v].  Each pass is a Stockham (self-sorting) step: with Ns the
// product of the radices already applied, butterfly j (k = j mod Ns) reads
// x[j + r N/R] for r < R, multiplies by the twiddle W_N^{k r N/(Ns R)},
// does an R-point DFT and writes y[(j / Ns) Ns R + k + r Ns].  For the
// lengths compiled in (those of 1080p, 720p, 2160p and 512 x 512 planes) a
// pass runs in place in one LDS buffer: a thread reads and transforms all of
// its butterflies, and writes them back after a barrier.  Other lengths run
// a plan read at run time whose passes ping-pong between two LDS buffers.
// Twiddles W_N^k = exp(-2 pi i k / N) are rounded to float from
// double-precision sincospi once per size and staged into LDS with the data,
// so a pass touches no global memory.  LDS is sized per launch: one or two
// data buffers of N * nvec plus the twiddle table(s).
//
// Kernels:
//   fft_1d          complex transform of rows or columns, in place in HBM
//   rfft_rows       real rows (optionally scaled elementwise by a second
//                   field) -> half spectrum of w/2+1 bins, through one
//                   complex transform of length w/2
//   fft_cols_power  column transform of half spectra; the epilogue either
//                   stores |Y_k|^2 or reduces sum_k |X_k|^2 |Y_k|^2 over the
//                   full (Hermitian) spectrum without the DC bin
//
// Half spectra and power tables of h rows x Mc bins are held in column
// groups of G = 2^lg bins, G being the column transform's vectors per
// workgroup: bin (n, c) at ((c >> lg) h + n) G + (c & (G - 1)), a plane of
// h * ceil(Mc / G) * G elements (bins past Mc are padding, never read as
// values).  A column workgroup then stages one contiguous block instead of
// G adjacent values from each of h rows.

#include <cmath>

#include "fft_dev.h"
#include "internal.h"
#include "stage_dev.h"

namespace prnu {
namespace {

// One batch of 1-D transforms: vectors v0 .. v0+nvec-1 of `count`, element n
// of vector v at base[v * vs + n * es].
// FN, FV: length and vectors per workgroup fixed at compile time (FN = 0: the
// runtime plan).  With rin the input is real (rin at the same element
// offsets, imaginary part 0); with rout only the real part, times rscale, is
// stored, to rout at the same offsets.
template <int FN, int FV>
__global__ __launch_bounds__(FNT) void fft_1d(float2 *__restrict__ data, int Nrt, int count, int64_t es,
                                              int64_t vs, int64_t plane_stride, FftPlan plan,
                                              const float2 *__restrict__ tw, float sigma,
                                              const float *__restrict__ rin, float *__restrict__ rout,
                                              float rscale) {
    extern __shared__ float2 smem[];
    int blk, pl;
    grid_tile(blk, pl);  // neighbouring vector groups on one XCD: they share cache lines
    const int N = FN ? FN : Nrt;
    const int nvec = FN ? FV : plan.nvec, lvec = FN ? ilog2c(FV) : plan.lvec;
    const int v0 = blk * nvec;
    float2 *base = data + (int64_t)pl * plane_stride;
    const int tot = N * nvec;
    // compile-time lengths transform in place (data, twiddles); the runtime
    // plan ping-pongs between two data buffers
    float2 *b0 = smem, *b1 = smem + tot, *twl = FN ? smem + tot : smem + 2 * tot;
    staged_copy<FNT, 4, float2>(threadIdx.x, N, [&](int e) { return tw[e]; }, [&](int e, float2 z) { twl[e] = z; });
    // vector groups inside the batch (all but a ragged last one) stage without
    // a bounds select, which the compiler would turn into a branch around the loads
    auto elem = [&](int e, bool in) {
        const int v = e & (nvec - 1), n = e >> lvec;
        const int64_t o = (int64_t)min(v0 + v, count - 1) * vs + (int64_t)n * es;
        const float2 z = rin ? make_float2(rin[(int64_t)pl * plane_stride + o], 0.f) : base[o];
        return in || v0 + v < count ? z : make_float2(0.f, 0.f);
    };
    if (v0 + nvec <= count)
        staged_copy<FNT, 8, float2>(threadIdx.x, tot, [&](int e) { return elem(e, true); },
                                    [&](int e, float2 z) { b0[e] = z; });
    else
        staged_copy<FNT, 8, float2>(threadIdx.x, tot, [&](int e) { return elem(e, false); },
                                    [&](int e, float2 z) { b0[e] = z; });
    __syncthreads();
    const float2 *res = fft_run<FN, FV>(b0, b1, plan, twl, sigma);
    for (int e = threadIdx.x; e < tot; e += FNT) {
        const int v = e & (nvec - 1), n = e >> lvec;
        const int64_t o = (int64_t)(v0 + v) * vs + (int64_t)n * es;
        if (v0 + v < count) {
            if (rout)
                rout[(int64_t)pl * plane_stride + o] = res[e].x * rscale;
            else
                base[o] = res[e];
        }
    }
}

// Real rows -> half spectra.  Plane p of the batch is y = Y[(p0+p) % ny]
// (times mod[(p0+p) / ny] if given, minus `mean[p]` if given); its bins
// k = 0 .. w/2 go to out[p] in column groups of 2^lg bins.
template <int FN, int FV, bool MOD>
__global__ __launch_bounds__(FNT) void rfft_rows(const float *__restrict__ Y, const float *__restrict__ mod,
                                                 int ny, int p0, const double *__restrict__ mean, int h,
                                                 int wrt, FftPlan plan, const float2 *__restrict__ tw_half,
                                                 const float2 *__restrict__ tw_full, int lg,
                                                 float2 *__restrict__ out) {
    extern __shared__ float2 smem[];
    const int w = FN ? 2 * FN : wrt;
    const int M = w / 2;
    const int nvec = FN ? FV : plan.nvec, lvec = FN ? ilog2c(FV) : plan.lvec;
    // the pairs of one row block run together on one XCD: the fingerprint and
    // modulation rows they share are fetched into its L2 once
    int rb, pl;
    grid_plane_major(rb, pl);
    const int r0 = rb * nvec;
    const int pid = p0 + pl;
    const int64_t N = (int64_t)h * w;
    const float *yp = Y + (int64_t)(pid % ny) * N;
    const float *mp = MOD ? mod + (int64_t)(pid / ny) * N : nullptr;
    const float mu = mean ? (float)mean[pl] : 0.f;
    const int tot = M * nvec;
    float2 *b0 = smem, *b1 = smem + tot, *twh = FN ? smem + tot : smem + 2 * tot, *twf = twh + M;
    staged_copy<FNT, 4, float2>(threadIdx.x, M, [&](int e) { return tw_half[e]; },
                                [&](int e, float2 z) { twh[e] = z; });
    staged_copy<FNT, 4, float2>(threadIdx.x, M + 1, [&](int e) { return tw_full[e]; },
                                [&](int e, float2 z) { twf[e] = z; });
    // rows of a block inside the plane (all but a ragged last block) stage
    // without a bounds select: the compiler would turn it into a branch
    // around the loads and wait for each pair of loads in turn
    auto row_pair = [&](int e, bool in) {
        const int v = e & (nvec - 1), n = e >> lvec;
        const int64_t o = (int64_t)min(r0 + v, h - 1) * w + 2 * n;
        float a = yp[o], b = yp[o + 1];
        if constexpr (MOD) {  // a separate instantiation: no branch around the loads
            a *= mp[o];
            b *= mp[o + 1];
        }
        return in || r0 + v < h ? make_float2(a - mu, b - mu) : make_float2(0.f, 0.f);
    };
    if (r0 + nvec <= h)
        staged_copy<FNT, 8, float2>(threadIdx.x, tot, [&](int e) { return row_pair(e, true); },
                                    [&](int e, float2 z) { b0[e] = z; });
    else
        staged_copy<FNT, 8, float2>(threadIdx.x, tot, [&](int e) { return row_pair(e, false); },
                                    [&](int e, float2 z) { b0[e] = z; });
    __syncthreads();
    const float2 *res = fft_run<FN, FV>(b0, b1, plan, twh, -1.f);
    // Split the even/odd-sample spectra: Y[k] = E[k] + W_w^k O[k], stored in
    // column groups of 2^lg bins.
    const int G = 1 << lg;
    float2 *op = out + (int64_t)pl * h * ((M + G) >> lg << lg);
    const int tot2 = (M + 1) * nvec;
    for (int e = threadIdx.x; e < tot2; e += FNT) {
        const int v = e % nvec, k = e / nvec;
        if (r0 + v >= h) continue;
        const float2 zk = res[(k % M) * nvec + v];
        const float2 zm = res[((M - k) % M) * nvec + v];
        // E = (zk + conj zm) / 2 ; O = (zk - conj zm) / (2i)
        const float2 E = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
        const float2 O = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
        const float2 tO = cmul(twf[k], O);  // exp(-2 pi i k / w), k <= w/2
        op[((int64_t)(k >> lg) * h + r0 + v) * G + (k & (G - 1))] = make_float2(E.x + tO.x, E.y + tO.y);
    }
}

// Column transforms of half spectra (h rows x Mc = w/2 + 1 bins, column groups).
//   POWER_STORE: Pout[p][k] = |S_k|^2 (DC bin 0)
//   POWER_DOT:   part[p][b] = sum_k wgt(k) Px[q][k] |S_k|^2 over column group b
//                (wgt = 1 on the first and the Nyquist column, 2 between;
//                DC bin excluded), q = (p0 + p) / ny.
template <bool DOT, int FN, int FV>
__global__ __launch_bounds__(FNT) void fft_cols_power(const float2 *__restrict__ S, int hrt, int Mc, FftPlan plan,
                                                      const float2 *__restrict__ tw, const float *__restrict__ Px,
                                                      int ny, int p0, float *__restrict__ Pout,
                                                      double *__restrict__ part) {
    extern __shared__ float2 smem[];
    int blk, pl;
    // the pairs of one column group run together on one XCD: a query's power
    // weights of the group are fetched into its L2 once for all its pairs
    grid_plane_major(blk, pl);
    const int h = FN ? FN : hrt;
    const int nvec = FN ? FV : plan.nvec, lvec = FN ? ilog2c(FV) : plan.lvec;
    const int c0 = blk * nvec;
    const int tot = h * nvec;
    // column groups of nvec bins: this workgroup's block is contiguous
    const int64_t plane = (int64_t)gridDim.x * tot;
    const float2 *sp = S + (int64_t)pl * plane + (int64_t)blk * tot;
    float2 *b0 = smem, *b1 = smem + tot, *twl = FN ? smem + tot : smem + 2 * tot;
    staged_copy<FNT, 4, float2>(threadIdx.x, h, [&](int e) { return tw[e]; }, [&](int e, float2 z) { twl[e] = z; });
    // column groups inside the half spectrum (all but the last) stage without a
    // bounds select, which the compiler would turn into a branch around the
    // loads; the last group's padding bins are read and replaced by 0
    auto col_elem = [&](int e, bool in) {
        const int v = e & (nvec - 1);
        const float2 z = sp[e];
        return in || c0 + v < Mc ? z : make_float2(0.f, 0.f);
    };
    if (c0 + nvec <= Mc)
        staged_copy<FNT, 8, float2>(threadIdx.x, tot, [&](int e) { return col_elem(e, true); },
                                    [&](int e, float2 z) { b0[e] = z; });
    else
        staged_copy<FNT, 8, float2>(threadIdx.x, tot, [&](int e) { return col_elem(e, false); },
                                    [&](int e, float2 z) { b0[e] = z; });
    const int pid = p0 + pl;
    const float *pq = DOT ? Px + (int64_t)(pid / ny) * plane + (int64_t)blk * tot : nullptr;
    // With a compile-time length the power weights of this thread's elements
    // are loaded now, so they arrive while the transform runs.
    constexpr int PXN = (DOT && FN) ? (FN * FV + FNT - 1) / FNT : 1;
    float pxr[PXN];
    if constexpr (DOT && FN != 0) {
#pragma unroll
        for (int k = 0; k < PXN; ++k) {
            const int e = threadIdx.x + k * FNT;
            // clamped to the block (used only where e and the column are in range)
            pxr[k] = pq[min(e, tot - 1)];
        }
    }
    __syncthreads();
    const float2 *res = fft_run<FN, FV>(b0, b1, plan, twl, -1.f);
    double acc = 0.0;
    if constexpr (DOT && FN != 0) {
#pragma unroll
        for (int k = 0; k < PXN; ++k) {
            const int e = threadIdx.x + k * FNT;
            const int v = e & (nvec - 1), n = e >> lvec;
            const int col = c0 + v;
            if (e >= tot || col >= Mc) continue;
            const float2 z = res[e];
            float pw = z.x * z.x + z.y * z.y;
            if (n == 0 && col == 0) pw = 0.f;
            const float wgt = (col == 0 || col == Mc - 1) ? 1.f : 2.f;
            acc += (double)(wgt * pw) * (double)pxr[k];
        }
    }
    constexpr int KB = 8;  // the power weights of KB elements are loaded before they are used
    for (int e0 = threadIdx.x; e0 < ((DOT && FN) ? 0 : tot); e0 += KB * FNT) {
        float px[KB];
        if (DOT) {
#pragma unroll
            for (int k = 0; k < KB; ++k) {
                const int e = e0 + k * FNT;
                px[k] = pq[e < tot ? e : 0];  // read where e and the column are in range
            }
        }
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const int e = e0 + k * FNT;
            const int v = e & (nvec - 1), n = e >> lvec;
            const int col = c0 + v;
            if (e >= tot || col >= Mc) continue;
            const float2 z = res[e];
            float pw = z.x * z.x + z.y * z.y;
            if (n == 0 && col == 0) pw = 0.f;
            if (DOT) {
                const float wgt = (col == 0 || col == Mc - 1) ? 1.f : 2.f;
                acc += (double)(wgt * pw) * (double)px[k];
            } else {
                Pout[(int64_t)pl * plane + (int64_t)blk * tot + e] = pw;
            }
        }
    }
    if (DOT) {
        // the twiddles (compile-time lengths) or the buffer not holding the
        // result are free for the reduction: the last pass ended in a barrier
        double *red = reinterpret_cast<double *>(FN ? twl : (res == b0 ? b1 : b0));
        acc = block_sum_f64(acc, red);
        if (threadIdx.x == 0) part[(int64_t)pl * gridDim.x + blk] = acc;
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

bool make_fft_plan(int n, FftPlan *p, bool columns) {
    if (n < 1 || n > FCAP) return false;
    int m = n, k = 0;
    while (m % 4 == 0 && k < 16) { p->rad[k++] = 4; m /= 4; }
    while (m % 2 == 0 && k < 16) { p->rad[k++] = 2; m /= 2; }
    while (m % 3 == 0 && k < 16) { p->rad[k++] = 3; m /= 3; }
    while (m % 5 == 0 && k < 16) { p->rad[k++] = 5; m /= 5; }
    if (m != 1) return false;
    p->n = n;
    p->nrad = k;
    // Column transforms read nvec adjacent complex values per row: they keep
    // up to twice as many vectors per workgroup for longer contiguous reads.
    const int target = columns ? 2 * FVEC : FVEC;
    int nv = 16, lv = 4;
    while (nv > 1 && n * nv > target) {
        nv /= 2;
        --lv;
    }
    p->nvec = nv;
    p->lvec = lv;
    return true;
}

size_t fft_twiddle_floats(int n) { return (size_t)2 * n; }

// Dynamic LDS of a transform workgroup: one data buffer (compile-time
// lengths, in place) or two (runtime plan) and `tw` twiddles (at most
// 2 * 5120 + 5121 complex values, 123 KB, for one vector of 5120).
unsigned fft_lds_bytes(const FftPlan &p, int tw, bool in_place) {
    return (unsigned)(sizeof(float2) * ((size_t)(in_place ? 1 : 2) * p.n * p.nvec + (size_t)tw));
}

// Allows a kernel the dynamic LDS of its launch.
template <typename K>
hipError_t allow_lds(K kernel, unsigned bytes) {
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

// Lengths with compile-time transforms, each with the vector count its plan
// gets: full rows, half rows and columns of 1920x1080, 1280x720, 3840x2160
// and 512x512 planes.  Every other length runs the runtime plan.
using Fft1dKernel = decltype(&fft_1d<0, 0>);
using RowsKernel = decltype(&rfft_rows<0, 0, false>);
using ColsKernel = decltype(&fft_cols_power<true, 0, 0>);

static Fft1dKernel pick_fft_1d(const FftPlan &p) {
#define PRNU_CASE(N, V) \
    if (p.n == N && p.nvec == V) return fft_1d<N, V>;
    PRNU_CASE(1920, 1) PRNU_CASE(1080, 4) PRNU_CASE(1280, 2) PRNU_CASE(720, 4) PRNU_CASE(3840, 1)
    PRNU_CASE(2160, 2) PRNU_CASE(512, 4) PRNU_CASE(512, 8)
#undef PRNU_CASE
    return fft_1d<0, 0>;
}

static RowsKernel pick_rfft_rows(const FftPlan &p, bool mod) {
#define PRNU_CASE(N, V) \
    if (p.n == N && p.nvec == V) return mod ? rfft_rows<N, V, true> : rfft_rows<N, V, false>;
    PRNU_CASE(960, 4) PRNU_CASE(640, 8) PRNU_CASE(1920, 2) PRNU_CASE(256, 16)
#undef PRNU_CASE
    return mod ? rfft_rows<0, 0, true> : rfft_rows<0, 0, false>;
}

template <bool DOT>
static ColsKernel pick_fft_cols(const FftPlan &p) {
#define PRNU_CASE(N, V) \
    if (p.n == N && p.nvec == V) return fft_cols_power<DOT, N, V>;
    PRNU_CASE(1080, 4) PRNU_CASE(720, 4) PRNU_CASE(2160, 2) PRNU_CASE(512, 8)
#undef PRNU_CASE
    return fft_cols_power<DOT, 0, 0>;
}

hipError_t launch_twiddles(int n, float2 *tw, hipStream_t s) {
    twiddle_kernel<<<(n + 255) / 256, 256, 0, s>>>(n, tw);
    return hipGetLastError();
}

hipError_t launch_fft2(float2 *data, int batch, int h, int w, const FftPlan &ph, const FftPlan &pw,
                       const float2 *tw_h, const float2 *tw_w, int dir, hipStream_t s, const float *rin,
                       float *rout, float rscale) {
    const float sigma = dir < 0 ? -1.f : 1.f;
    const int64_t plane = (int64_t)h * w;
    // read + write every element: complex 8 B, real input or output 4 B
    const double bytes_rows = (rin ? 12.0 : 16.0) * (double)batch * plane;
    const double bytes_cols = (rout ? 12.0 : 16.0) * (double)batch * plane;
    // rows: h vectors of length w
    dim3 gr((unsigned)((h + pw.nvec - 1) / pw.nvec), (unsigned)batch);
    {
        KernelTimer kt("fft_1d", bytes_rows, s);
        const Fft1dKernel k = pick_fft_1d(pw);
        const unsigned lds = fft_lds_bytes(pw, pw.n, k != fft_1d<0, 0>);
        hipError_t e = allow_lds(k, lds);
        if (e != hipSuccess) return e;
        k<<<gr, FNT, lds, s>>>(data, w, h, 1, w, plane, pw, tw_w, sigma, rin, nullptr, 1.f);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // columns: w vectors of length h
    dim3 gc((unsigned)((w + ph.nvec - 1) / ph.nvec), (unsigned)batch);
    {
        KernelTimer kt("fft_1d", bytes_cols, s);
        const Fft1dKernel k = pick_fft_1d(ph);
        const unsigned lds = fft_lds_bytes(ph, ph.n, k != fft_1d<0, 0>);
        e = allow_lds(k, lds);
        if (e != hipSuccess) return e;
        k<<<gc, FNT, lds, s>>>(data, h, w, w, 1, plane, ph, tw_h, sigma, nullptr, rout, rscale);
    }
    return hipGetLastError();
}

hipError_t launch_rfft_rows(const float *Y, const float *mod, int ny, int p0, int n, const double *mean,
                            int h, int w, const FftPlan &phalf, const float2 *tw_half, const float2 *tw_full,
                            const FftPlan &pcol, float2 *out, hipStream_t s) {
    const double bytes = (double)n * h * ((mod ? 8.0 : 4.0) * w + 8.0 * (w / 2 + 1));
    KernelTimer kt("rfft_rows", bytes, s);
    dim3 g((unsigned)((h + phalf.nvec - 1) / phalf.nvec), (unsigned)n);
    const RowsKernel k = pick_rfft_rows(phalf, mod != nullptr);
    const unsigned lds =
        fft_lds_bytes(phalf, 2 * phalf.n + 1, k != rfft_rows<0, 0, false> && k != rfft_rows<0, 0, true>);
    const hipError_t e = allow_lds(k, lds);
    if (e != hipSuccess) return e;
    k<<<g, FNT, lds, s>>>(Y, mod, ny, p0, mean, h, w, phalf, tw_half, tw_full, pcol.lvec, out);
    return hipGetLastError();
}

int fft_cols_power_blocks(int Mc, const FftPlan &ph) { return (Mc + ph.nvec - 1) / ph.nvec; }
int64_t half_plane_elems(int h, int Mc, const FftPlan &ph) {
    return (int64_t)h * fft_cols_power_blocks(Mc, ph) * ph.nvec;
}

hipError_t launch_fft_cols_power(const float2 *S, int n, int h, int Mc, const FftPlan &ph, const float2 *tw_h,
                                 const float *Px, int ny, int p0, float *Pout, double *part, hipStream_t s) {
    const double bytes = (double)n * h * Mc * (8.0 + 4.0);
    dim3 g((unsigned)fft_cols_power_blocks(Mc, ph), (unsigned)n);
    const unsigned lds = fft_lds_bytes(ph, ph.n, pick_fft_cols<true>(ph) != fft_cols_power<true, 0, 0>);
    if (Px) {
        const ColsKernel k = pick_fft_cols<true>(ph);
        const hipError_t e = allow_lds(k, lds);
        if (e != hipSuccess) return e;
        KernelTimer kt("fft_cols_power_dot", bytes, s);
        k<<<g, FNT, lds, s>>>(S, h, Mc, ph, tw_h, Px, ny, p0, nullptr, part);
    } else {
        const ColsKernel k = pick_fft_cols<false>(ph);
        const hipError_t e = allow_lds(k, lds);
        if (e != hipSuccess) return e;
        KernelTimer kt("fft_cols_power_store", bytes, s);
        k<<<g, FNT, lds, s>>>(S, h, Mc, ph, tw_h, nullptr, ny, p0, Pout, nullptr);
    }
    return hipGetLastError();
}

}  // namespace prnu
