// NCC / PCE of query residuals against fingerprints (Sec. II-A: the query's
// residual is correlated with the fingerprint; Sec. IV: PCE above 60 means
// "same camera").
//
// Per pair p = (q, j) of a chunk: y = modulate[q] * Y[j] (or Y[j]) is centred
// and transformed, its spectrum is multiplied into X^[q] * conj(Y^), and the
// inverse transform gives N * C(s).  The surface is reduced in two fixed-order
// stages: per-block partials (sum of C^2 in double, first maximum), then one
// block per pair adds the partials, subtracts the nbhd x nbhd block around the
// peak from the energy and forms PCE and NCC.

#include <cfloat>
#include <climits>

#include "internal.h"
#include "stage_dev.h"

namespace prnu {
namespace {

constexpr int NT = 256;
constexpr int RB = 64;  // reduction blocks per plane

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double block_sum(double v, double *sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < NT / 64; ++k) r += sh[k];
    __syncthreads();
    return r;
}

// plane p of the chunk: y = Y[(p0+p) % ny] times modulate[(p0+p) / ny] if given.
struct PairSel {
    const float *Y;
    const float *mod;
    int ny;
    int p0;
    __device__ __forceinline__ void planes(int64_t N, const float *&y, const float *&m) const {
        const int pid = p0 + (int)blockIdx.y;
        y = Y + (int64_t)(pid % ny) * N;
        m = mod ? mod + (int64_t)(pid / ny) * N : nullptr;
    }
};

// pass 0: partial sums of y; pass 1: partial sums of (y - mean)^2
__global__ __launch_bounds__(NT) void stats_partial(PairSel sel, int64_t N, const double *__restrict__ mean,
                                                    double *__restrict__ part) {
    __shared__ double sh[NT / 64];
    const float *y, *m;
    sel.planes(N, y, m);
    const double mu = mean ? mean[blockIdx.y] : 0.0;
    // the thread's terms in order, SB loads in flight (a term past the end is 0)
    constexpr int SB = 8;
    constexpr int64_t STRIDE = (int64_t)RB * NT;
    double s = 0.0;
    for (int64_t i0 = (int64_t)blockIdx.x * NT + threadIdx.x; i0 < N; i0 += SB * STRIDE) {
        float v[SB];
#pragma unroll
        for (int k = 0; k < SB; ++k) {
            const int64_t i = i0 + k * STRIDE < N ? i0 + k * STRIDE : 0;
            v[k] = m ? m[i] * y[i] : y[i];
        }
#pragma unroll
        for (int k = 0; k < SB; ++k) {
            const double d = i0 + k * STRIDE < N ? (double)v[k] - mu : 0.0;
            s += mean ? d * d : d;
        }
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.y * RB + blockIdx.x] = s;
}

__global__ void stats_finish(const double *__restrict__ part, int n, double scale, double *__restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double s = 0.0;
    for (int k = 0; k < RB; ++k) s += part[(int64_t)p * RB + k];
    out[p] = s * scale;
}

__global__ __launch_bounds__(NT) void center_complex(PairSel sel, int64_t N, const double *__restrict__ mean,
                                                     float2 *__restrict__ z) {
    const float *y, *m;
    sel.planes(N, y, m);
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= N) return;
    const float v = m ? m[i] * y[i] : y[i];
    z[(int64_t)blockIdx.y * N + i] = make_float2((float)((double)v - mean[blockIdx.y]), 0.f);
}

// z[p] = X^[q] * conj(S), S = z[p] (in place) or Ycache[j].
__global__ __launch_bounds__(NT) void cross_spectrum(const float2 *__restrict__ Xs, const float2 *Ycache,
                                                     int ny, int p0, int64_t N, float2 *z) {
    const int pid = p0 + (int)blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (i >= N) return;
    const float2 a = Xs[(int64_t)(pid / ny) * N + i];
    const float2 b = Ycache ? Ycache[(int64_t)(pid % ny) * N + i] : z[(int64_t)blockIdx.y * N + i];
    // a * conj(b)
    z[(int64_t)blockIdx.y * N + i] = make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

struct PcePart {
    double e2;   // sum of v^2
    float vmax;  // first maximum of v
    int imax;
};

__global__ __launch_bounds__(NT) void pce_partial(const float2 *__restrict__ z, int64_t N,
                                                  PcePart *__restrict__ part) {
    __shared__ double sh[NT / 64];
    __shared__ float sv[NT];
    __shared__ int si[NT];
    const float2 *zp = z + (int64_t)blockIdx.y * N;
    double e = 0.0;
    float best = -FLT_MAX;
    int bi = INT_MAX;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < N; i += (int64_t)RB * NT) {
        const float v = zp[i].x;
        e += (double)v * (double)v;
        if (v > best || (v == best && (int)i < bi)) {
            best = v;
            bi = (int)i;
        }
    }
    sv[threadIdx.x] = best;
    si[threadIdx.x] = bi;
    e = block_sum(e, sh);  // contains barriers
    for (int st = NT / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            const float ov = sv[threadIdx.x + st];
            const int oi = si[threadIdx.x + st];
            if (ov > sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi < si[threadIdx.x])) {
                sv[threadIdx.x] = ov;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.y * RB + blockIdx.x] = {e, sv[0], si[0]};
}

__global__ __launch_bounds__(NT) void pce_finish(const float2 *__restrict__ z, int h, int w, int nbhd,
                                                 int peak_mode, const PcePart *__restrict__ part,
                                                 const double *__restrict__ xn2, const double *__restrict__ yn2,
                                                 int yn2_by_j, int ny, int p0, double *__restrict__ pce,
                                                 double *__restrict__ ncc, int32_t *__restrict__ peak) {
    __shared__ double sh[NT / 64];
    __shared__ int s_peak;
    __shared__ double s_tot;
    const int p = blockIdx.x;
    const int pid = p0 + p;
    const int64_t N = (int64_t)h * w;
    const float2 *zp = z + (int64_t)p * N;
    if (threadIdx.x == 0) {
        double tot = 0.0;
        float best = -FLT_MAX;
        int bi = INT_MAX;
        for (int k = 0; k < RB; ++k) {
            const PcePart q = part[(int64_t)p * RB + k];
            tot += q.e2;
            if (q.vmax > best || (q.vmax == best && q.imax < bi)) {
                best = q.vmax;
                bi = q.imax;
            }
        }
        s_tot = tot;
        if (bi < 0 || (int64_t)bi >= N) bi = 0;  // no comparable value (e.g. all NaN)
        s_peak = peak_mode == PRNU_PEAK_ARGMAX ? bi : 0;
    }
    __syncthreads();
    const int pk = s_peak;
    const int py = pk / w, px = pk - (pk / w) * w;
    const int r = nbhd / 2;
    double e = 0.0;
    for (int t = threadIdx.x; t < nbhd * nbhd; t += NT) {
        const int dy = t / nbhd - r, dx = t % nbhd - r;
        const int yy = ((py + dy) % h + h) % h, xx = ((px + dx) % w + w) % w;
        const double v = zp[(int64_t)yy * w + xx].x;
        e += v * v;
    }
    e = block_sum(e, sh);
    if (threadIdx.x == 0) {
        const double invN = 1.0 / (double)N;
        const double cp = (double)zp[pk].x * invN;
        const double energy = (s_tot - e) * invN * invN / (double)(N - (int64_t)nbhd * nbhd);
        const double val = energy > 0.0 ? (cp >= 0.0 ? 1.0 : -1.0) * cp * cp / energy : 0.0;
        const int q = pid / ny, j = pid % ny;
        pce[pid] = val;
        if (ncc) {
            const double c0 = (double)zp[0].x * invN;
            const double den = sqrt(xn2[q] * yn2[yn2_by_j ? j : p]);
            ncc[pid] = den > 0.0 ? c0 / den : 0.0;
        }
        if (peak) {
            peak[2 * (int64_t)pid] = py;
            peak[2 * (int64_t)pid + 1] = px;
        }
    }
}

// ---- fixed-peak fast path ---------------------------------------------------
// C(s) for the (2*DRAD+1)^2 shifts around 0, computed directly:
//   D(s) = sum_t xc(t + s) y(t),  xc = X[q] - mean[q] (circular in t + s),
// with y = mod[q] * Y[j] (or Y[j]); plus sum y, sum y^2 and sum xc.
// A thread owns 4 consecutive pixels of a 16 x 64 tile; the centred x tile
// with a DRAD halo sits in LDS; the 121 sums stay in registers across the
// block's tiles and are reduced once per block.
constexpr int DRAD = 5;
constexpr int DNS = 2 * DRAD + 1;
constexpr int DSTAT = DNS * DNS + 3;  // D(s), sum y, sum y^2, sum xc
static_assert(DSTAT == kPceDirectStats, "partial layout shared with the host plan");
constexpr int DTY = 16, DTX = 64;
constexpr int XTH = DTY + 2 * DRAD, XTW = DTX + 2 * DRAD, XTWS = 76;

__global__ __launch_bounds__(NT) void pce_direct(const float *__restrict__ X, const double *__restrict__ xmean,
                                                 PairSel sel, int h, int w, int tiles_x, int ntiles,
                                                 double *__restrict__ part) {
    __shared__ float xs[XTH * XTWS];
    __shared__ float red[NT / 64][DSTAT];
    const int64_t N = (int64_t)h * w;
    const int pid = sel.p0 + (int)blockIdx.y;
    const int q = pid / sel.ny;
    const float *xp = X + (int64_t)q * N;
    const float mux = (float)xmean[q];
    const float *yp = sel.Y + (int64_t)(pid % sel.ny) * N;
    const float *mp = sel.mod ? sel.mod + (int64_t)q * N : nullptr;
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tq = tid & 15;
    float acc[DNS][DNS];
#pragma unroll
    for (int a = 0; a < DNS; ++a)
#pragma unroll
        for (int b = 0; b < DNS; ++b) acc[a][b] = 0.f;
    float sy = 0.f, syy = 0.f, sx = 0.f;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int ty0 = (tile / tiles_x) * DTY, tx0 = (tile % tiles_x) * DTX;
        __syncthreads();
        staged_copy<NT, 4, float>(
            tid, XTH * XTW,
            [&](int e) {
                const int i = e / XTW, jj = e - (e / XTW) * XTW;
                int gr = (ty0 - DRAD + i) % h;
                gr = gr < 0 ? gr + h : gr;
                int gc = (tx0 - DRAD + jj) % w;
                gc = gc < 0 ? gc + w : gc;
                return xp[(int64_t)gr * w + gc] - mux;
            },
            [&](int e, float v) { xs[(e / XTW) * XTWS + e - (e / XTW) * XTW] = v; });
        __syncthreads();
        const int gy = ty0 + ty, gx = tx0 + 4 * tq;
        float yv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            float v = 0.f;
            if (gy < h && gx + u < w) {
                const int64_t o = (int64_t)gy * w + gx + u;
                v = mp ? mp[o] * yp[o] : yp[o];
                sx += xs[(ty + DRAD) * XTWS + 4 * tq + u + DRAD];
            }
            yv[u] = v;
            sy += v;
            syy = fmaf(v, v, syy);
        }
#pragma unroll
        for (int dy = 0; dy < DNS; ++dy) {
            const float *row = &xs[(ty + dy) * XTWS + 4 * tq];
            float xr[4 + 2 * DRAD];
#pragma unroll
            for (int t = 0; t < 4 + 2 * DRAD; ++t) xr[t] = row[t];
#pragma unroll
            for (int dx = 0; dx < DNS; ++dx)
#pragma unroll
                for (int u = 0; u < 4; ++u) acc[dy][dx] = fmaf(xr[u + dx], yv[u], acc[dy][dx]);
        }
    }
    // block reduction: wave shuffles, then across the waves in fixed order
    const int lane = tid & 63, wv = tid >> 6;
    auto wsum = [](float v) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        return v;
    };
#pragma unroll
    for (int a = 0; a < DNS; ++a)
#pragma unroll
        for (int b = 0; b < DNS; ++b) {
            const float v = wsum(acc[a][b]);
            if (lane == 0) red[wv][a * DNS + b] = v;
        }
    {
        const float v0 = wsum(sy), v1 = wsum(syy), v2 = wsum(sx);
        if (lane == 0) {
            red[wv][DNS * DNS] = v0;
            red[wv][DNS * DNS + 1] = v1;
            red[wv][DNS * DNS + 2] = v2;
        }
    }
    __syncthreads();
    if (tid < DSTAT) {
        double t = 0.0;
        for (int k = 0; k < NT / 64; ++k) t += (double)red[k][tid];
        part[((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * DSTAT + tid] = t;
    }
}

// ---- fixed-peak direct sums on the matrix cores ------------------------------
// For one query q and 16 fingerprints j0 .. j0+15 the 121 shifted sums are
// one product D[s][j] = sum_t xc(t + s) y_j(t) whose inner dimension runs over
// the pixels t.  v_mfma_f32_16x16x4f32 multiplies 16 shifts x 4 pixels (A:
// the centred query tile in LDS, read through per-lane shift offsets) by
// 4 pixels x 16 fingerprints (B: the modulated fingerprint tile in LDS); eight
// such products per pixel quad cover 128 rows: the 121 shifts, an all-ones row
// (giving sum y) and 6 unused rows; each of the four waves owns two of the
// eight shift blocks for every pixel of the tile.  Lane layout (checked on
// the device): A[i][k] and B[k][n] at lane 16 k + i / 16 k + n,
// C[4 (l / 16) + r][l % 16] in slot r of lane l.  Each tile's fp32 products
// are added to FP64 accumulators; sum y^2 and sum xc are plain FP64 sums.
// The all-ones row reads a block of ones kept in LDS below the query tile,
// so the loop has no per-lane select; sum y^2, which only the NCC needs, is
// formed only when SYY is set.
constexpr int MTY = 8, MTX = 64;                              // pixel tile
// query tile with the shift halo; row stride 16 banks (mod 64): the 16 shifts
// of a block span at most three rows, whose reads then fall in disjoint banks
constexpr int MXH = MTY + 2 * DRAD, MXW = MTX + 2 * DRAD, MXWS = 80;
constexpr int MNJ = 16, MNS = 8;                              // fingerprints, shift blocks of 16
constexpr int MYS = MTY * MTX + 4;                            // fingerprint stride in LDS (bank offset 4)
constexpr int MONES = DNS * DNS;                              // row 121: all ones
constexpr int SBW = MNS / (NT / 64);                          // shift blocks per wave
typedef float v4f __attribute__((ext_vector_type(4)));

template <bool SYY>
__global__ __launch_bounds__(NT) void pce_direct_mfma(const float *__restrict__ X, const double *__restrict__ xmean,
                                                      const float *__restrict__ Y, const float *__restrict__ mod,
                                                      int ny, int q0, int h, int w, int tiles_x, int ntiles,
                                                      double *__restrict__ part) {
    __shared__ float xs[(MXH + MTY) * MXWS];  // query tile, then MTY rows of ones
    __shared__ float ms[MTY * MTX];                // modulation per tile pixel, 0 outside the image
    __shared__ __align__(16) float ys[MNJ * MYS];
    __shared__ double sred[NT / 64];
    __shared__ double yred[NT / 64][MNJ];
    const int q = q0 + (int)blockIdx.y;
    const int j0 = (int)blockIdx.z * MNJ;
    const int nblk = gridDim.x, blk = blockIdx.x;
    const int64_t N = (int64_t)h * w;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const PRNU_GLOBAL float *xp = gmem(X) + (int64_t)q * N;
    const float mux = (float)xmean[q];
    const PRNU_GLOBAL float *mp = mod ? gmem(mod) + (int64_t)q * N : nullptr;
    // A operand: row i = lane % 16 of shift block sb is shift m = 16 sb + i (rows past the
    // ones row read shift (0,0) and are dropped), column k = lane / 16 is pixel k of the quad.
    // The modulation belongs to the pixel t, so it scales B: y(t) = mod(t) * K(t),
    // formed once per tile pixel and fingerprint when the tile is staged.
    // Wave wv computes shift blocks SBW wv .. SBW wv + SBW - 1 over all the
    // tile's pixels, so it holds complete sums for its shifts (no cross-wave
    // reduction, a quarter of the accumulators).
    int aoff[SBW];
#pragma unroll
    for (int i = 0; i < SBW; ++i) {
        const int m = 16 * (SBW * wv + i) + (lane & 15);
        const int mm = m < DNS * DNS ? m : (DNS * DNS) / 2;
        // the ones row reads 16 columns in, in banks no shift of its block uses
        aoff[i] = m == MONES ? MXH * MXWS + 16 + (lane >> 4) : (mm / DNS) * MXWS + (mm % DNS) + (lane >> 4);
    }
    // the ones (tile staging writes only the rows above them)
    for (int e = tid; e < MTY * MXWS; e += NT) xs[MXH * MXWS + e] = 1.f;
    const int boff = (lane & 15) * MYS + (lane >> 4);  // B: fingerprint n = lane % 16, pixel k = lane / 16
    // staging of the fingerprint tile: thread -> fingerprint sn, columns sc + 16 u
    const int sn = tid >> 4, sc = tid & 15;
    const PRNU_GLOBAL float *yp = j0 + sn < ny ? gmem(Y) + (int64_t)(j0 + sn) * N : nullptr;
    double acc[SBW][4];
#pragma unroll
    for (int i = 0; i < SBW; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[i][r] = 0.0;
    double syy = 0.0, sx = 0.0;

    // The next tile's global loads are issued before the current tile's
    // products and land in registers while the matrix cores run.
    constexpr int KX = (MXH * MXW + NT - 1) / NT, KM = MTY * MTX / NT, KY = MTY * MTX * MNJ / NT;
    static_assert(KM * NT == MTY * MTX && KY * NT == MTY * MTX * MNJ, "tile staging");
    float rx[KX], rm[KM], ry[KY];
    auto fetch = [&](int tile) {
        const int ty0 = (tile / tiles_x) * MTY, tx0 = (tile % tiles_x) * MTX;
#pragma unroll
        for (int k = 0; k < KX; ++k) {
            const int e = tid + k * NT;
            rx[k] = 0.f;
            if (e < MXH * MXW) {
                const int i = e / MXW, jj = e - (e / MXW) * MXW;
                int gr = (ty0 - DRAD + i) % h;
                gr = gr < 0 ? gr + h : gr;
                int gc = (tx0 - DRAD + jj) % w;
                gc = gc < 0 ? gc + w : gc;
                rx[k] = xp[(int64_t)gr * w + gc];
            }
        }
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            const int e = tid + k * NT, gy = ty0 + e / MTX, gx = tx0 + e % MTX;
            const bool in = gy < h && gx < w;
            rm[k] = in ? (mp ? mp[(int64_t)gy * w + gx] : 1.f) : 0.f;
        }
#pragma unroll
        for (int k = 0; k < KY; ++k) {
            const int r = k >> 2, c = sc + 16 * (k & 3), gy = ty0 + r, gx = tx0 + c;
            ry[k] = (yp && gy < h && gx < w) ? yp[(int64_t)gy * w + gx] : 0.f;
        }
    };
    auto put = [&]() {
#pragma unroll
        for (int k = 0; k < KX; ++k) {
            const int e = tid + k * NT;
            if (e < MXH * MXW) xs[(e / MXW) * MXWS + e - (e / MXW) * MXW] = rx[k] - mux;
        }
#pragma unroll
        for (int k = 0; k < KM; ++k) ms[tid + k * NT] = rm[k];
        __syncthreads();  // the modulation of every tile pixel is in LDS
        // the fingerprint tile goes to LDS already modulated: y = mod * K
#pragma unroll
        for (int k = 0; k < KY; ++k) {
            const int o = (k >> 2) * MTX + sc + 16 * (k & 3);
            ys[sn * MYS + o] = ry[k] * ms[o];
        }
    };

    if (blk < ntiles) fetch(blk);
    for (int tile = blk; tile < ntiles; tile += nblk) {
        const int ty0 = (tile / tiles_x) * MTY, tx0 = (tile % tiles_x) * MTX;
        __syncthreads();  // previous tile's LDS reads are done
        put();
        __syncthreads();
        if (tile + nblk < ntiles) fetch(tile + nblk);
        // sum of the centred query over this tile's pixels inside the image
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int t = tid + u * NT, r = t / MTX, c = t % MTX;
            if (ty0 + r < h && tx0 + c < w) sx += (double)xs[(r + DRAD) * MXWS + c + DRAD];
        }
        // every pixel row, sixteen quads each; sum y^2 of rows wv and wv + 4
        v4f cacc[SBW];
#pragma unroll
        for (int i = 0; i < SBW; ++i) cacc[i] = v4f{0.f, 0.f, 0.f, 0.f};
        float ssq = 0.f;
#pragma unroll 16
        for (int g = 0; g < MTY * 16; ++g) {
            const int r = g >> 4, c4 = (g & 15) * 4;
            const float b = ys[boff + r * MTX + c4];  // the modulated fingerprint y
            if (SYY && (r & 3) == wv) ssq = fmaf(b, b, ssq);
            const int xb = r * MXWS + c4;
#pragma unroll
            for (int i = 0; i < SBW; ++i)
                cacc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(xs[xb + aoff[i]], b, cacc[i], 0, 0, 0);
        }
        syy += (double)ssq;
#pragma unroll
        for (int i = 0; i < SBW; ++i)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[i][r] += (double)cacc[i][r];
    }
    const int64_t prow = (int64_t)(q - q0) * ny;
    {
        const int n = lane & 15;
        if (j0 + n < ny) {
            double *dst = part + ((prow + j0 + n) * nblk + blk) * DSTAT;
#pragma unroll
            for (int i = 0; i < SBW; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = 16 * (SBW * wv + i) + 4 * (lane >> 4) + r;
                    if (m <= MONES) dst[m] = acc[i][r];
                }
        }
    }
    // sum y^2 per fingerprint n = lane % 16: the four lanes of n in each wave (a
    // fixed shuffle tree), then the four waves in order
    syy += __shfl_xor(syy, 16, 64);
    syy += __shfl_xor(syy, 32, 64);
    if (lane < MNJ) yred[wv][lane] = syy;
    // sum xc, the same for every fingerprint
    sx = wave_sum(sx);
    if (lane == 0) sred[wv] = sx;
    __syncthreads();
    if (tid < MNJ && j0 + tid < ny) {
        double t = 0.0, u = 0.0;
        for (int k = 0; k < NT / 64; ++k) {
            t += sred[k];
            u += yred[k][tid];
        }
        part[((prow + j0 + tid) * nblk + blk) * DSTAT + MONES + 1] = u;
        part[((prow + j0 + tid) * nblk + blk) * DSTAT + MONES + 2] = t;
    }
}

// part[p][blk] = sum over the half spectrum of wgt * Px[q] * Py[j] (DC excluded),
// the bins taken in row-major order; Px and Py are held in column groups of
// 2^lg bins (planes of h * ceil(Mc / 2^lg) * 2^lg).
__global__ __launch_bounds__(NT) void power_dot(const float *__restrict__ Px, const float *__restrict__ Py,
                                                int ny, int p0, int h, int Mc, int lg, double *__restrict__ part) {
    __shared__ double sh[NT / 64];
    const int pid = p0 + (int)blockIdx.y;
    const int64_t M = (int64_t)h * Mc;
    const int G = 1 << lg;
    const int64_t Mg = (int64_t)h * ((Mc + G - 1) >> lg << lg);
    const float *a = Px + (int64_t)(pid / ny) * Mg;
    const float *b = Py + (int64_t)(pid % ny) * Mg;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < M; i += (int64_t)gridDim.x * NT) {
        const int n = (int)(i / Mc), col = (int)(i - (int64_t)n * Mc);
        const int64_t o = ((int64_t)(col >> lg) * h + n) * G + (col & (G - 1));
        const float wgt = (col == 0 || col == Mc - 1) ? 1.f : 2.f;
        acc += (i == 0) ? 0.0 : (double)(wgt * a[o] * b[o]);
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = acc;
}

__global__ void pce_finish_fixed(const double *__restrict__ dpart, int nblk_d, const double *__restrict__ spart,
                                 int nblk_s, int64_t N, int nbhd, const double *__restrict__ xn2, int ny, int p0,
                                 double *__restrict__ pce, double *__restrict__ ncc,
                                 int32_t *__restrict__ peak) {
    __shared__ double st[DSTAT];
    const int p = blockIdx.x;
    const int pid = p0 + p;
    for (int t = threadIdx.x; t < DSTAT; t += blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nblk_d; ++b) s += dpart[((int64_t)p * nblk_d + b) * DSTAT + t];
        st[t] = s;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double dot = 0.0;
    for (int b = 0; b < nblk_s; ++b) dot += spart[(int64_t)p * nblk_s + b];
    const double dN = (double)N;
    const double sy = st[DNS * DNS], syy = st[DNS * DNS + 1], sx = st[DNS * DNS + 2];
    const double muy = sy / dN;
    const int r = nbhd / 2;
    double n11 = 0.0;
    for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) {
            const double c = st[(dy + DRAD) * DNS + (dx + DRAD)] - muy * sx;
            n11 += c * c;
        }
    const double c0 = st[DRAD * DNS + DRAD] - muy * sx;
    const double total = dot / dN;
    const double energy = (total - n11) / (dN - (double)nbhd * nbhd);
    pce[pid] = energy > 0.0 ? (c0 >= 0.0 ? 1.0 : -1.0) * c0 * c0 / energy : 0.0;
    if (ncc) {
        const int q = pid / ny;
        const double yn = syy - sy * sy / dN;
        const double den = sqrt(xn2[q] * (yn > 0.0 ? yn : 0.0));
        ncc[pid] = den > 0.0 ? c0 / den : 0.0;
    }
    if (peak) {
        peak[2 * (int64_t)pid] = 0;
        peak[2 * (int64_t)pid + 1] = 0;
    }
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + NT - 1) / NT); }

}  // namespace

size_t pce_part_bytes(int npairs) { return (size_t)npairs * RB * sizeof(PcePart); }
size_t stats_part_doubles(int n) { return (size_t)n * RB; }

// Means and centred squared norms of the chunk's planes (pairs p0 .. p0+n-1,
// or plain planes when mod == nullptr and ny >= p0 + n).
hipError_t launch_pair_stats(const float *Y, const float *mod, int ny, int p0, int n, int64_t N,
                             double *mean, double *nrm2, double *part, hipStream_t s) {
    PairSel sel{Y, mod, ny, p0};
    dim3 g(RB, (unsigned)n);
    KernelTimer kt("pair_stats", 2.0 * (double)n * N * (mod ? 8.0 : 4.0), s);
    stats_partial<<<g, NT, 0, s>>>(sel, N, nullptr, part);
    stats_finish<<<(n + 63) / 64, 64, 0, s>>>(part, n, 1.0 / (double)N, mean);
    if (nrm2) {
        stats_partial<<<g, NT, 0, s>>>(sel, N, mean, part);
        stats_finish<<<(n + 63) / 64, 64, 0, s>>>(part, n, 1.0, nrm2);
    }
    return hipGetLastError();
}

hipError_t launch_pair_center(const float *Y, const float *mod, int ny, int p0, int n, int64_t N,
                              const double *mean, float2 *z, hipStream_t s) {
    PairSel sel{Y, mod, ny, p0};
    KernelTimer kt("center_complex", (double)n * N * ((mod ? 8.0 : 4.0) + 8.0), s);
    center_complex<<<dim3(blocks(N), (unsigned)n), NT, 0, s>>>(sel, N, mean, z);
    return hipGetLastError();
}

hipError_t launch_cross(const float2 *Xs, const float2 *Ycache, int ny, int p0, int n, int64_t N,
                        float2 *z, hipStream_t s) {
    KernelTimer kt("cross_spectrum", (double)n * N * 24.0, s);
    cross_spectrum<<<dim3(blocks(N), (unsigned)n), NT, 0, s>>>(Xs, Ycache, ny, p0, N, z);
    return hipGetLastError();
}

hipError_t launch_pce_reduce(const float2 *z, int n, int h, int w, int nbhd, int peak_mode,
                             const double *xn2, const double *yn2, bool yn2_by_j, int ny, int p0,
                             double *pce, double *ncc, int32_t *peak, void *part, hipStream_t s) {
    const int64_t N = (int64_t)h * w;
    PcePart *pp = static_cast<PcePart *>(part);
    KernelTimer kt("pce_reduce", (double)n * N * 8.0, s);
    pce_partial<<<dim3(RB, (unsigned)n), NT, 0, s>>>(z, N, pp);
    pce_finish<<<(unsigned)n, NT, 0, s>>>(z, h, w, nbhd, peak_mode, pp, xn2, yn2,
                                                yn2_by_j ? 1 : 0, ny, p0, pce, ncc, peak);
    return hipGetLastError();
}

}  // namespace prnu

namespace prnu {

int pce_direct_blocks(int h, int w) {
    const int tiles = ((h + DTY - 1) / DTY) * ((w + DTX - 1) / DTX);
    int nb = (tiles + 31) / 32;
    return nb < 1 ? 1 : nb;
}
size_t pce_direct_part_doubles(int npairs, int h, int w) {
    return (size_t)npairs * pce_direct_blocks(h, w) * DSTAT;
}
int pce_dot_blocks() { return 64; }

hipError_t launch_pce_direct(const float *X, const double *xmean, const float *Y, const float *mod, int ny,
                             int p0, int n, int h, int w, double *part, hipStream_t s) {
    const int tiles_x = (w + DTX - 1) / DTX;
    const int ntiles = tiles_x * ((h + DTY - 1) / DTY);
    PairSel sel{Y, mod, ny, p0};
    KernelTimer kt("pce_direct", (double)n * h * w * (mod ? 12.0 : 8.0), s);
    pce_direct<<<dim3((unsigned)pce_direct_blocks(h, w), (unsigned)n), NT, 0, s>>>(X, xmean, sel, h, w,
                                                                                  tiles_x, ntiles, part);
    return hipGetLastError();
}

int pce_mfma_tiles(int h, int w) { return ((h + MTY - 1) / MTY) * ((w + MTX - 1) / MTX); }

int pce_mfma_blocks(int nq, int ny, int h, int w) {
    const int64_t groups = (int64_t)nq * ((ny + MNJ - 1) / MNJ);
    int64_t nb = (2048 + groups - 1) / groups;  // about eight workgroups per CU in all
    const int tiles = pce_mfma_tiles(h, w);
    if (nb > 64) nb = 64;
    if (nb > tiles) nb = tiles;
    return nb < 1 ? 1 : (int)nb;
}

hipError_t launch_pce_direct_mfma(const float *X, const double *xmean, const float *Y, const float *mod, int ny,
                                  int q0, int nq, int h, int w, int nblk, bool syy, double *part, hipStream_t s) {
    const int tiles_x = (w + MTX - 1) / MTX;
    const int ntiles = pce_mfma_tiles(h, w);
    const int ng = (ny + MNJ - 1) / MNJ;
    // algorithmic bytes: every query pixel once, every fingerprint (and modulation) pixel once per query
    KernelTimer kt("pce_direct_mfma", (double)nq * h * w * (4.0 + ny * (mod ? 8.0 : 4.0)), s,
                   2.0 * (DNS * DNS + 1) * (double)nq * ny * h * w);  // 121 shifted sums and the plain sum
    const dim3 grid((unsigned)nblk, (unsigned)nq, (unsigned)ng);
    if (syy)
        pce_direct_mfma<true><<<grid, NT, 0, s>>>(X, xmean, Y, mod, ny, q0, h, w, tiles_x, ntiles, part);
    else
        pce_direct_mfma<false><<<grid, NT, 0, s>>>(X, xmean, Y, mod, ny, q0, h, w, tiles_x, ntiles, part);
    return hipGetLastError();
}

hipError_t launch_power_dot(const float *Px, const float *Py, int ny, int p0, int n, int h, int Mc, int lg,
                            double *part, hipStream_t s) {
    KernelTimer kt("power_dot", (double)n * h * Mc * 8.0, s);
    power_dot<<<dim3((unsigned)pce_dot_blocks(), (unsigned)n), NT, 0, s>>>(Px, Py, ny, p0, h, Mc, lg, part);
    return hipGetLastError();
}

hipError_t launch_pce_finish_fixed(const double *dpart, int nblk_d, const double *spart, int nblk_s, int n,
                                   int h, int w, int nbhd, const double *xn2, int ny, int p0, double *pce,
                                   double *ncc, int32_t *peak, hipStream_t s) {
    pce_finish_fixed<<<(unsigned)n, 64, 0, s>>>(dpart, nblk_d, spart, nblk_s, (int64_t)h * w, nbhd, xn2, ny, p0,
                                                pce, ncc, peak);
    return hipGetLastError();
}

}  // namespace prnu
