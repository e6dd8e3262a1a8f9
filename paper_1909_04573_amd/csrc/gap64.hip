// FP64 mode of the differentiated chain: the matched-minus-unmatched PCE gap
// of Sec. II-A / Sec. IV and its gradient with respect to the denoiser's
// noise variances (sigma0, lambda_1..4), every step in double precision.
//
// The chain (same definitions as the FP32 path and its adjoint):
//   per camera: SDA means of d frames (Sec. III-B) -> residual W = I - F(I)
//               (periodised 4-level DWT, detail coefficients replaced by
//               r = c s / max(s, m), m the smallest 3/5/7/9 window mean of
//               c^2, zero approximation, inverse) -> K = sum W I / sum I^2
//               (Sec. III-B MLE) -> zero-mean
//   per query:  residual -> zero-mean -> x;  y = I_q K_j
//   per pair:   fixed-peak PCE of the centred x, y through the DFT
//   loss:       mean PCE over matched pairs - mean over unmatched pairs
// and backward: dPCE/dC -> gradients of x and y through the DFT -> zero-mean
// (self-adjoint) -> MLE -> the residual's adjoint (the periodised analysis of
// the zero-embedded gradient, dotted with the checkpointed dr/ds = [m > s]
// c / m per level).
//
// The kernels are plain: one thread per output value, direct window sums,
// a Stockham FFT with radices 2..5, block reductions in a fixed order (the
// results do not depend on scheduling).  This mode exists to check the
// gradient at full sizes against an FP64 reference, not for speed.

#include <cmath>

#include "internal.h"
#include "stage_dev.h"

namespace prnu {
namespace {

constexpr int T64 = 256;

inline unsigned blocks(int64_t n) { return (unsigned)((n + T64 - 1) / T64); }

__device__ __forceinline__ int64_t gid() { return blockIdx.x * (int64_t)blockDim.x + threadIdx.x; }

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// ---- SDA, widening, padding ---------------------------------------------------
// out[c][gi][p] = sum_{f in group gi} fr[c][f][p] / count  (frames summed in order)
__global__ void sda64(const float *__restrict__ fr, int m, int d, int g, int64_t npx, int ncam,
                      double *__restrict__ out) {
    const int64_t e = gid();
    if (e >= (int64_t)ncam * g * npx) return;
    const int64_t p = e % npx;
    const int64_t cg = e / npx;
    const int c = (int)(cg / g), gi = (int)(cg - (int64_t)c * g);
    const int f0 = gi * d, cnt = min(d, m - f0);
    double s = 0.0;
    for (int f = 0; f < cnt; ++f) s += (double)fr[((int64_t)c * m + f0 + f) * npx + p];
    out[e] = s / (double)cnt;
}

__global__ void widen64(const float *__restrict__ x, int64_t n, double *__restrict__ y) {
    const int64_t e = gid();
    if (e < n) y[e] = (double)x[e];
}

// Edge-including mirror padding: [P][H][W] -> [P][Hp][Wp], t rows before, l columns before.
__global__ void pad64(const double *__restrict__ x, int H, int W, int t, int l, int Hp, int Wp, int64_t P,
                      double *__restrict__ y) {
    const int64_t e = gid();
    if (e >= P * Hp * Wp) return;
    const int64_t pl = e / ((int64_t)Hp * Wp);
    const int rem = (int)(e - pl * Hp * Wp), r = rem / Wp, c = rem - (rem / Wp) * Wp;
    int sr = r - t, sc = c - l;
    sr = sr < 0 ? -1 - sr : (sr >= H ? 2 * H - 1 - sr : sr);
    sc = sc < 0 ? -1 - sc : (sc >= W ? 2 * W - 1 - sc : sc);
    y[e] = x[(pl * H + sr) * W + sc];
}

// crop (embed = 0): [P][Hp][Wp] -> [P][H][W];  embed (= 1): the crop's adjoint, zero outside.
__global__ void crop64(const double *__restrict__ x, int H, int W, int t, int l, int Hp, int Wp, int64_t P,
                       int embed, double *__restrict__ y) {
    const int64_t e = gid();
    if (embed) {
        if (e >= P * Hp * Wp) return;
        const int64_t pl = e / ((int64_t)Hp * Wp);
        const int rem = (int)(e - pl * Hp * Wp), r = rem / Wp - t, c = rem - (rem / Wp) * Wp - l;
        y[e] = (r >= 0 && r < H && c >= 0 && c < W) ? x[(pl * H + r) * W + c] : 0.0;
    } else {
        if (e >= P * H * W) return;
        const int64_t pl = e / ((int64_t)H * W);
        const int rem = (int)(e - pl * H * W), r = rem / W, c = rem - (rem / W) * W;
        y[e] = x[(pl * Hp + r + t) * Wp + c + l];
    }
}

// ---- wavelet steps ---------------------------------------------------------------
// Periodised analysis of [P][R][C] along axis 1 (rows: a, d are [P][R][C/2])
// or axis 0 (columns: a, d are [P][R/2][C]): a[k] = sum_j h[j] x[(2k+j) mod n].
__global__ void ana64(const double *__restrict__ x, int R, int C, int axis, int64_t P, Filter64 f,
                      double *__restrict__ a, double *__restrict__ d) {
    const int Ro = axis ? R : R / 2, Co = axis ? C / 2 : C;
    const int64_t e = gid();
    if (e >= P * Ro * Co) return;
    const int64_t pl = e / ((int64_t)Ro * Co);
    const int rem = (int)(e - pl * Ro * Co), r = rem / Co, c = rem - (rem / Co) * Co;
    const double *xp = x + pl * R * C;
    double sa = 0.0, sd = 0.0;
    for (int j = 0; j < f.taps; ++j) {
        const double v = axis ? xp[(int64_t)r * C + (2 * c + j) % C] : xp[(int64_t)((2 * r + j) % R) * C + c];
        sa = fma(f.h[j], v, sa);
        sd = fma(f.g[j], v, sd);
    }
    a[e] = sa;
    d[e] = sd;
}

// Synthesis (the analysis' adjoint) into [P][R][C] along axis 1 (a, d of
// [P][R][C/2]) or axis 0 (a, d of [P][R/2][C]): output i gathers h[j] a[k] +
// g[j] d[k] over the taps j with 2k + j = i (mod n).
__global__ void syn64(const double *__restrict__ a, const double *__restrict__ d, int R, int C, int axis,
                      int64_t P, Filter64 f, double *__restrict__ x) {
    const int64_t e = gid();
    if (e >= P * R * C) return;
    const int64_t pl = e / ((int64_t)R * C);
    const int rem = (int)(e - pl * R * C), r = rem / C, c = rem - (rem / C) * C;
    const int n = axis ? C : R, i = axis ? c : r, m = n / 2;
    double s = 0.0;
    for (int j = (i & 1); j < f.taps; j += 2) {  // 2k + j = i (mod n) needs j = i (mod 2)
        const int k = (((i - j) % n + n) % n) / 2;
        const int64_t o = axis ? (pl * R + r) * m + k : (pl * m + k) * C + c;
        s = fma(f.h[j], a[o], fma(f.g[j], d[o], s));
    }
    x[e] = s;
}

// Shrinkage of one detail band [P][R][C] at noise variance s2: r = c s2 / max(s2, m)
// and the checkpoint dr/ds2 = [m > s2] c / m, m the smallest centred 3/5/7/9
// window mean of c^2 (zero outside the band).
__global__ void wiener64(const double *__restrict__ cb, int R, int C, int64_t P, double s2, double *__restrict__ r,
                         double *__restrict__ sens) {
    const int64_t e = gid();
    if (e >= P * R * C) return;
    const int64_t pl = e / ((int64_t)R * C);
    const int rem = (int)(e - pl * R * C), y = rem / C, x = rem - (rem / C) * C;
    const double *cp = cb + pl * R * C;
    double m = 0.0;
    for (int w = 3; w <= 9; w += 2) {
        const int h = w / 2;
        double s = 0.0;
        for (int dy = -h; dy <= h; ++dy) {
            const int yy = y + dy;
            if (yy < 0 || yy >= R) continue;
            for (int dx = -h; dx <= h; ++dx) {
                const int xx = x + dx;
                if (xx < 0 || xx >= C) continue;
                const double v = cp[(int64_t)yy * C + xx];
                s = fma(v, v, s);
            }
        }
        const double mw = s / (double)(w * w);
        m = w == 3 ? mw : fmin(m, mw);
    }
    const double c = cp[(int64_t)y * C + x];
    const bool act = m > s2;
    r[e] = act ? c * s2 / m : c;
    sens[e] = act ? c / m : 0.0;
}

// ---- MLE, zero-mean, elementwise -------------------------------------------------
// Camera c: A = sum_i W_i I_i, B = sum_i I_i^2 over its g SDA frames in order;
// K = A / B (0 where B = 0); B kept for the backward pass.
__global__ void mle64(const double *__restrict__ Wr, const double *__restrict__ I, int g, int64_t npx, int ncam,
                      double *__restrict__ K, double *__restrict__ B) {
    const int64_t e = gid();
    if (e >= (int64_t)ncam * npx) return;
    const int64_t c = e / npx, p = e - c * npx;
    double a = 0.0, b = 0.0;
    for (int i = 0; i < g; ++i) {
        const int64_t o = (c * g + i) * npx + p;
        a += Wr[o] * I[o];
        b += I[o] * I[o];
    }
    K[e] = b > 0.0 ? a / b : 0.0;
    B[e] = b;
}

// Zero-mean step 1: subtract each row's mean (one block per row, tree sum).
__global__ __launch_bounds__(T64) void zm_rows64(double *__restrict__ x, int W) {
    __shared__ double red[T64];
    double *row = x + (int64_t)blockIdx.x * W;
    double s = 0.0;
    for (int c = threadIdx.x; c < W; c += T64) s += row[c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = T64 / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    const double mean = red[0] / (double)W;
    for (int c = threadIdx.x; c < W; c += T64) row[c] -= mean;
}

// Zero-mean step 2: subtract each column's mean (one thread per column, rows in order).
__global__ void zm_cols64(double *__restrict__ x, int H, int W, int64_t P) {
    const int64_t e = gid();
    if (e >= P * W) return;
    const int64_t pl = e / W;
    const int c = (int)(e - pl * W);
    double *xp = x + pl * H * W + c;
    double s = 0.0;
    for (int r = 0; r < H; ++r) s += xp[(int64_t)r * W];
    const double mean = s / (double)H;
    for (int r = 0; r < H; ++r) xp[(int64_t)r * W] -= mean;
}

// Per-plane sums in a fixed order: part[p][b] over chunk b of plane p (tree
// inside the block), then sums[p] = the partials in order.
// mode 0: x, 1: x*x, 2: x*y.
__global__ __launch_bounds__(T64) void red64_part(const double *__restrict__ x, const double *__restrict__ y,
                                                  int64_t n, int nblk, int mode, double *__restrict__ part) {
    __shared__ double red[T64];
    const int64_t pl = blockIdx.y;
    const int64_t chunk = (n + nblk - 1) / nblk;
    const int64_t b0 = blockIdx.x * chunk, b1 = min(n, b0 + chunk);
    const double *xp = x + pl * n;
    const double *yp = y ? y + pl * n : nullptr;
    double s = 0.0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += T64) {
        const double v = xp[i];
        s += mode == 0 ? v : (mode == 1 ? v * v : v * yp[i]);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = T64 / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[pl * nblk + blockIdx.x] = red[0];
}

__global__ void red64_finish(const double *__restrict__ part, int nblk, int64_t P, double scale,
                             double *__restrict__ out) {
    const int64_t p = gid();
    if (p >= P) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[p * nblk + b];
    out[p] = s * scale;
}

// y[p][i] = a[p][i] * (b ? b[p % nbm][i] : 1) - (mean ? mean[p] : 0)
__global__ void axpm64(const double *__restrict__ a, const double *__restrict__ b, int nbm, const double *mean,
                       int64_t n, int64_t P, double *__restrict__ y) {
    const int64_t e = gid();
    if (e >= P * n) return;
    const int64_t p = e / n, i = e - p * n;
    double v = a[e];
    if (b) v *= b[(p % nbm) * n + i];
    y[e] = mean ? v - mean[p] : v;
}

// ---- DFT ---------------------------------------------------------------------------
// One radix-R pass of length-n complex transforms in Stockham order (p = the
// product of the radices before this pass; the last pass leaves natural
// order).  Transform b's element e is at (b / inner) * outer + (b % inner) *
// istride + e * estride.  sign -1 forward, +1 inverse (unscaled).
template <int R>
__global__ void fft64_pass(const double2 *__restrict__ x, double2 *__restrict__ y, int n, int p, int64_t nbt,
                           int64_t inner, int64_t outer, int64_t istride, int64_t estride, double sign) {
    const int T = n / R;
    const int64_t e = gid();
    if (e >= nbt * T) return;
    const int64_t b = e / T;
    const int i = (int)(e - b * T);
    const int64_t off = (b / inner) * outer + (b % inner) * istride;
    const int k = i % p;
    double2 u[R];
#pragma unroll
    for (int j = 0; j < R; ++j) u[j] = x[off + (int64_t)(i + j * T) * estride];
#pragma unroll
    for (int j = 1; j < R; ++j) {
        const int q = (j * k) % (p * R);
        double s, c;
        sincospi(sign * 2.0 * (double)q / (double)(p * R), &s, &c);
        u[j] = cmul(u[j], make_double2(c, s));
    }
    const int o = (i - k) * R + k;
#pragma unroll
    for (int mm = 0; mm < R; ++mm) {
        double2 v = u[0];
#pragma unroll
        for (int j = 1; j < R; ++j) {
            double s, c;
            sincospi(sign * 2.0 * (double)((j * mm) % R) / (double)R, &s, &c);
            const double2 t = cmul(u[j], make_double2(c, s));
            v.x += t.x;
            v.y += t.y;
        }
        y[off + (int64_t)(o + mm * p) * estride] = v;
    }
}

// complex planes from real ones: z = (x - mean[p], 0)
__global__ void to_complex64(const double *__restrict__ x, const double *mean, int64_t n, int64_t P,
                             double2 *__restrict__ z) {
    const int64_t e = gid();
    if (e >= P * n) return;
    z[e] = make_double2(x[e] - (mean ? mean[e / n] : 0.0), 0.0);
}

// z[p] = op(A[p % na], B[p % nb]): mode 0: A conj(B), 1: A B, 2: conj(A) B
__global__ void cprod64(const double2 *A, int na, const double2 *B, int nb, int64_t n, int64_t P, int mode,
                        double2 *z) {
    const int64_t e = gid();
    if (e >= P * n) return;
    const int64_t p = e / n, i = e - p * n;
    double2 a = A[(p % na) * n + i], b = B[(p % nb) * n + i];
    if (mode == 0) b.y = -b.y;
    if (mode == 2) a.y = -a.y;
    z[e] = cmul(a, b);
}

__global__ void real_part64(const double2 *__restrict__ z, int64_t n, double scale, double *__restrict__ x) {
    const int64_t e = gid();
    if (e < n) x[e] = z[e].x * scale;
}

// ---- PCE and its derivative ---------------------------------------------------------
// Pair k (query q, camera j): c0 = C(0,0), E = (sum C^2 - sum over the
// nbhd x nbhd block around 0 of C^2) / (N - nbhd^2), PCE = sign(c0) c0^2 / E;
// coef[k] = (alpha, beta) of dPCE/dC = alpha Ct + beta delta_0 with Ct = C
// cleared on the block.  One thread per pair (the block in row-major order).
__global__ void pce_stats64(const double *__restrict__ C, const double *__restrict__ sumsq, int h, int w, int nbhd,
                            int64_t npair, double *__restrict__ pce, double2 *__restrict__ coef) {
    const int64_t k = gid();
    if (k >= npair) return;
    const double *Cp = C + k * h * w;
    const int r = nbhd / 2;
    double blk = 0.0;
    for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx) {
            const double v = Cp[(int64_t)(((dy % h) + h) % h) * w + ((dx % w) + w) % w];
            blk = fma(v, v, blk);
        }
    const double denom = (double)h * w - (double)nbhd * nbhd;
    const double E = (sumsq[k] - blk) / denom;
    const double c0 = Cp[0];
    const double sg = c0 > 0.0 ? 1.0 : (c0 < 0.0 ? -1.0 : 0.0);
    pce[k] = sg * c0 * c0 / E;
    coef[k] = make_double2(-sg * c0 * c0 / (E * E) * 2.0 / denom, 2.0 * fabs(c0) / E);
}

// gC[k] = alpha_k * C[k] off the block, 0 on it, plus beta_k at (0, 0); as complex.
__global__ void pce_gc64(const double *__restrict__ C, const double2 *__restrict__ coef, int h, int w, int nbhd,
                         int64_t npair, double2 *__restrict__ z) {
    const int64_t e = gid();
    const int64_t n = (int64_t)h * w;
    if (e >= npair * n) return;
    const int64_t k = e / n;
    const int i = (int)(e - k * n), y = i / w, x = i - (i / w) * w;
    const int r = nbhd / 2;
    const int dy = y <= h / 2 ? y : y - h, dx = x <= w / 2 ? x : x - w;
    const bool in = dy >= -r && dy <= r && dx >= -r && dx <= r;
    double v = in ? 0.0 : coef[k].x * C[e];
    if (i == 0) v += coef[k].y;
    z[e] = make_double2(v, 0.0);
}

// Gradients of one query's pairs, summed over its cameras j = 0..nc-1 in order:
// gxq += sum_j w_j (gx_j - mean gx_j);  gK_j += w_j Iq (gy_j - mean gy_j).
__global__ void pce_accum64(const double *__restrict__ gx, const double *__restrict__ gxm,
                            const double *__restrict__ gy, const double *__restrict__ gym, const double *__restrict__ wq,
                            const double *__restrict__ Iq, int nc, int64_t n, double *__restrict__ gxq,
                            double *__restrict__ gK) {
    const int64_t i = gid();
    if (i >= n) return;
    double sx = gxq[i];
    for (int j = 0; j < nc; ++j) {
        sx += wq[j] * (gx[j * n + i] - gxm[j]);
        gK[j * n + i] += wq[j] * Iq[i] * (gy[j * n + i] - gym[j]);
    }
    gxq[i] = sx;
}

// Backward through the MLE: gW[c][i] = B > 0 ? gK[c] I_i / B : 0.
__global__ void mle_back64(const double *__restrict__ gK, const double *__restrict__ I, const double *__restrict__ B,
                           int g, int64_t npx, int ncam, double *__restrict__ gW) {
    const int64_t e = gid();
    if (e >= (int64_t)ncam * g * npx) return;
    const int64_t p = e % npx, c = e / npx / g;
    const double b = B[c * npx + p];
    gW[e] = b > 0.0 ? gK[c * npx + p] * I[e] / b : 0.0;
}

// Pair weights from the query cameras: 1/#matched on matched pairs, -1/#unmatched otherwise.
__global__ void gap_weights64(const int *__restrict__ qcam, int nq, int nc, double *__restrict__ w) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int nm = 0;
    for (int q = 0; q < nq; ++q) nm += (qcam[q] >= 0 && qcam[q] < nc) ? 1 : 0;
    const int nu = nq * nc - nm;
    for (int q = 0; q < nq; ++q)
        for (int j = 0; j < nc; ++j)
            w[q * nc + j] = qcam[q] == j ? 1.0 / (double)(nm > 0 ? nm : 1) : -1.0 / (double)(nu > 0 ? nu : 1);
}

// out = (loss, dL/dsigma0, dL/dlambda_1..4): loss = sum w P; dL/ds_l summed over
// the planes in order; chain rule s_l = lambda_l sigma0^2.
__global__ void gap_finish64(const double *__restrict__ w, const double *__restrict__ pce, int npair,
                             const double *__restrict__ dlds_pl, int nplane, int levels, double sigma0, double l0,
                             double l1, double l2, double l3, double *__restrict__ out) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double L = 0.0;
    for (int k = 0; k < npair; ++k) L += w[k] * pce[k];
    const double lam[4] = {l0, l1, l2, l3};
    double g0 = 0.0;
    out[0] = L;
    for (int l = 0; l < 4; ++l) {
        double ds = 0.0;
        if (l < levels)
            for (int p = 0; p < nplane; ++p) ds += dlds_pl[(int64_t)p * levels + l];
        g0 += ds * 2.0 * lam[l] * sigma0;
        out[2 + l] = ds * sigma0 * sigma0;
    }
    out[1] = g0;
}


__global__ void copy64c(const double2 *__restrict__ x, int64_t n, double2 *__restrict__ y) {
    const int64_t e = gid();
    if (e < n) y[e] = x[e];
}

__global__ void copy64(const double *__restrict__ x, int64_t n, double *__restrict__ y) {
    const int64_t e = gid();
    if (e < n) y[e] = x[e];
}

__global__ void zero64(double *__restrict__ x, int64_t n) {
    const int64_t e = gid();
    if (e < n) x[e] = 0.0;
}

// Band [NP][bsz] <-> its slot at offset off of each plane's checkpoint [NP][ssz].
__global__ void band_to_slot64(const double *__restrict__ r, const double *__restrict__ ds, int64_t bsz, int64_t NP,
                               int64_t ssz, int64_t off, double *__restrict__ rd, double *__restrict__ sens) {
    const int64_t e = gid();
    if (e >= NP * bsz) return;
    const int64_t p = e / bsz, i = e - p * bsz;
    rd[p * ssz + off + i] = r[e];
    sens[p * ssz + off + i] = ds[e];
}

__global__ void slot_to_band64(const double *__restrict__ src, int64_t bsz, int64_t NP, int64_t ssz, int64_t off,
                               double *__restrict__ band) {
    const int64_t e = gid();
    if (e >= NP * bsz) return;
    const int64_t p = e / bsz, i = e - p * bsz;
    band[e] = src[p * ssz + off + i];
}

// dlds[p][lv] = sum over the level's three bands (lh, hl, hh) of plane p
__global__ void add_level64(const double *__restrict__ prod, int64_t NP, int levels, int lv, double *__restrict__ dlds) {
    const int64_t p = gid();
    if (p >= NP) return;
    dlds[p * levels + lv] = prod[p] + prod[NP + p] + prod[2 * NP + p];
}



// ---------------------------------------------------------------------------------------
// Host side.

int radix_of(int n) { return n % 4 == 0 ? 4 : n % 2 == 0 ? 2 : n % 3 == 0 ? 3 : n % 5 == 0 ? 5 : 0; }

// Passes of a length-n transform over nbt transforms (layout as in
// fft64_pass), ping-ponging between *cur and *other; on return *cur holds
// the result.
hipError_t fft64_axis(double2 **cur, double2 **other, int n, int64_t nbt, int64_t inner, int64_t outer,
                      int64_t istride, int64_t estride, double sign, hipStream_t s) {
    int p = 1, rest = n;
    while (rest > 1) {
        const int R = radix_of(rest);
        if (R == 0) return hipErrorInvalidValue;
        const int64_t work = nbt * (n / R);
        double2 *src = *cur, *dst = *other;
        if (R == 2)
            fft64_pass<2><<<blocks(work), T64, 0, s>>>(src, dst, n, p, nbt, inner, outer, istride, estride, sign);
        else if (R == 3)
            fft64_pass<3><<<blocks(work), T64, 0, s>>>(src, dst, n, p, nbt, inner, outer, istride, estride, sign);
        else if (R == 4)
            fft64_pass<4><<<blocks(work), T64, 0, s>>>(src, dst, n, p, nbt, inner, outer, istride, estride, sign);
        else
            fft64_pass<5><<<blocks(work), T64, 0, s>>>(src, dst, n, p, nbt, inner, outer, istride, estride, sign);
        p *= R;
        rest /= R;
        *cur = dst;
        *other = src;
    }
    return hipGetLastError();
}

// Unscaled 2-D transform of P planes [P][h][w] in place in x (tmp: scratch of
// the same size): every row, then every column.
hipError_t fft2d64(double2 *x, double2 *tmp, int64_t P, int h, int w, double sign, hipStream_t s) {
    double2 *cur = x, *other = tmp;
    // rows: transform b = (plane, row) at b * w, elements contiguous
    hipError_t e = fft64_axis(&cur, &other, w, P * h, P * h, 0, w, 1, sign, s);
    // columns: transform b = (plane, column) at plane * h * w + column, elements w apart
    if (e == hipSuccess) e = fft64_axis(&cur, &other, h, P * w, w, (int64_t)h * w, 1, w, sign, s);
    if (e == hipSuccess && cur != x) {
        copy64c<<<blocks(P * h * w), T64, 0, s>>>(cur, P * h * w, x);
        e = hipGetLastError();
    }
    return e;
}

// out[p] = scale * sum_i op(x[p][i], y[p][i]) for P planes of n values (op as red64_part).
void plane_sums64(const double *x, const double *y, int64_t n, int64_t P, int mode, double scale, double *part,
                  double *out, hipStream_t s) {
    red64_part<<<dim3((unsigned)kRedBlocks64, (unsigned)P), T64, 0, s>>>(x, y, n, kRedBlocks64, mode, part);
    red64_finish<<<blocks(P), T64, 0, s>>>(part, kRedBlocks64, P, scale, out);
}

void zero_mean64(double *x, int64_t P, int H, int W, hipStream_t s) {
    zm_rows64<<<(unsigned)(P * H), T64, 0, s>>>(x, W);
    zm_cols64<<<blocks(P * W), T64, 0, s>>>(x, H, W, P);
}

struct Carve64 {
    char *base;
    size_t off = 0;
    template <class T>
    T *take(int64_t n) {
        off = (off + 255) / 256 * 256;
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += (size_t)n * sizeof(T);
        return p;
    }
};

struct Ws64 {
    double *img, *res, *sens, *rd, *X0, *lo, *hi, *ll, *bands, *K, *B, *gK, *gx, *gW;
    double *wts, *pce, *part, *small, *dlds, *C, *gxp, *gyp, *prod;
    double2 *XQ, *Y, *Z, *T, *coef;
    size_t bytes;
};

// One carving pass sizes the workspace (base = nullptr), the next hands out pointers.
void carve64(char *base, const Gap64Dims &D, Ws64 *w) {
    Carve64 cv{base};
    const int64_t npx = (int64_t)D.H * D.W, ppx = (int64_t)D.Hp * D.Wp, nc = D.ncam;
    const int64_t NP = nc * D.g + D.nq;
    w->img = cv.take<double>(NP * npx);
    w->res = cv.take<double>(NP * npx);
    w->sens = cv.take<double>(NP * D.ssz);
    w->rd = cv.take<double>(NP * D.ssz);
    w->X0 = cv.take<double>(NP * ppx);
    w->lo = cv.take<double>(NP * ppx / 2);
    w->hi = cv.take<double>(NP * ppx / 2);
    w->ll = cv.take<double>(NP * ppx / 4);
    w->bands = cv.take<double>(NP * ppx / 4 * 3);
    w->K = cv.take<double>(nc * npx);
    w->B = cv.take<double>(nc * npx);
    w->gK = cv.take<double>(nc * npx);
    w->gx = cv.take<double>((int64_t)D.nq * npx);
    w->gW = cv.take<double>(NP * npx);
    w->wts = cv.take<double>((int64_t)D.nq * nc);
    w->pce = cv.take<double>((int64_t)D.nq * nc);
    w->part = cv.take<double>((NP > nc ? NP : nc) * kRedBlocks64);
    w->small = cv.take<double>(4 * nc + 4);
    w->dlds = cv.take<double>(NP * D.levels);
    w->C = cv.take<double>(nc * npx);
    w->gxp = cv.take<double>(nc * npx);
    w->gyp = cv.take<double>(nc * npx);
    w->prod = cv.take<double>(3 * NP);
    w->XQ = cv.take<double2>(npx);
    w->Y = cv.take<double2>(nc * npx);
    w->Z = cv.take<double2>(nc * npx);
    w->T = cv.take<double2>(nc * npx);
    w->coef = cv.take<double2>(nc);
    w->bytes = cv.off;
}

// Residuals of the NP planes in w.img: pad, L analysis levels with the
// shrinkage of each detail band (r into w.rd, dr/ds into w.sens, per plane
// level by level as [lh | hl | hh]), synthesis from a zero approximation,
// crop into w.res.
void residuals64(const Gap64Dims &D, const Filter64 &f, const double *s2, const Ws64 &w, hipStream_t s) {
    const int64_t NP = (int64_t)D.ncam * D.g + D.nq;
    pad64<<<blocks(NP * D.Hp * D.Wp), T64, 0, s>>>(w.img, D.H, D.W, D.t, D.l, D.Hp, D.Wp, NP, w.X0);
    int h = D.Hp, wd = D.Wp;
    int64_t soff = 0;
    for (int lv = 0; lv < D.levels; ++lv) {
        const int h2 = h / 2, w2 = wd / 2;
        const int64_t bsz = (int64_t)h2 * w2;
        double *lh = w.bands, *hl = lh + NP * bsz, *hh = hl + NP * bsz;
        ana64<<<blocks(NP * h * w2), T64, 0, s>>>(w.X0, h, wd, 1, NP, f, w.lo, w.hi);
        ana64<<<blocks(NP * bsz), T64, 0, s>>>(w.lo, h, w2, 0, NP, f, w.ll, hl);  // ll, hl from lo1
        ana64<<<blocks(NP * bsz), T64, 0, s>>>(w.hi, h, w2, 0, NP, f, lh, hh);    // lh, hh from hi1
        for (int b = 0; b < 3; ++b) {
            const double *cb = b == 0 ? lh : (b == 1 ? hl : hh);
            wiener64<<<blocks(NP * bsz), T64, 0, s>>>(cb, h2, w2, NP, s2[lv], w.lo, w.hi);
            band_to_slot64<<<blocks(NP * bsz), T64, 0, s>>>(w.lo, w.hi, bsz, NP, D.ssz, soff + b * bsz, w.rd, w.sens);
        }
        soff += 3 * bsz;
        copy64<<<blocks(NP * bsz), T64, 0, s>>>(w.ll, NP * bsz, w.X0);  // next level's input
        h = h2;
        wd = w2;
    }
    zero64<<<blocks(NP * h * wd), T64, 0, s>>>(w.ll, NP * h * wd);  // approximation set to zero
    for (int lv = D.levels - 1; lv >= 0; --lv) {
        const int64_t bsz = (int64_t)h * wd;
        soff -= 3 * bsz;
        double *lh = w.bands, *hl = lh + NP * bsz, *hh = hl + NP * bsz;
        slot_to_band64<<<blocks(NP * bsz), T64, 0, s>>>(w.rd, bsz, NP, D.ssz, soff, lh);
        slot_to_band64<<<blocks(NP * bsz), T64, 0, s>>>(w.rd, bsz, NP, D.ssz, soff + bsz, hl);
        slot_to_band64<<<blocks(NP * bsz), T64, 0, s>>>(w.rd, bsz, NP, D.ssz, soff + 2 * bsz, hh);
        // lo1 = syn0(ll, hl), hi1 = syn0(lh, hh): [2h][wd]; x = syn1(lo1, hi1): [2h][2wd]
        syn64<<<blocks(NP * 2 * h * wd), T64, 0, s>>>(w.ll, hl, 2 * h, wd, 0, NP, f, w.lo);
        syn64<<<blocks(NP * 2 * h * wd), T64, 0, s>>>(lh, hh, 2 * h, wd, 0, NP, f, w.hi);
        syn64<<<blocks(NP * 4 * h * wd), T64, 0, s>>>(w.lo, w.hi, 2 * h, 2 * wd, 1, NP, f, w.X0);
        h *= 2;
        wd *= 2;
        if (lv > 0) copy64<<<blocks(NP * h * wd), T64, 0, s>>>(w.X0, NP * h * wd, w.ll);
    }
    crop64<<<blocks(NP * D.H * D.W), T64, 0, s>>>(w.X0, D.H, D.W, D.t, D.l, D.Hp, D.Wp, NP, 0, w.res);
}

// dL/ds_l per plane from dL/dW of every plane (w.gW): embed (the crop's
// adjoint), the periodised analysis (the synthesis' adjoint), and per level
// the sum of the detail gradients times the checkpointed dr/ds.
void residual_vjp64(const Gap64Dims &D, const Filter64 &f, const Ws64 &w, hipStream_t s) {
    const int64_t NP = (int64_t)D.ncam * D.g + D.nq;
    crop64<<<blocks(NP * D.Hp * D.Wp), T64, 0, s>>>(w.gW, D.H, D.W, D.t, D.l, D.Hp, D.Wp, NP, 1, w.X0);
    int h = D.Hp, wd = D.Wp;
    int64_t soff = 0;
    for (int lv = 0; lv < D.levels; ++lv) {
        const int h2 = h / 2, w2 = wd / 2;
        const int64_t bsz = (int64_t)h2 * w2;
        double *lh = w.bands, *hl = lh + NP * bsz, *hh = hl + NP * bsz;
        ana64<<<blocks(NP * h * w2), T64, 0, s>>>(w.X0, h, wd, 1, NP, f, w.lo, w.hi);
        ana64<<<blocks(NP * bsz), T64, 0, s>>>(w.lo, h, w2, 0, NP, f, w.ll, hl);
        ana64<<<blocks(NP * bsz), T64, 0, s>>>(w.hi, h, w2, 0, NP, f, lh, hh);
        for (int b = 0; b < 3; ++b) {
            const double *gb = b == 0 ? lh : (b == 1 ? hl : hh);
            slot_to_band64<<<blocks(NP * bsz), T64, 0, s>>>(w.sens, bsz, NP, D.ssz, soff + b * bsz, w.lo);
            plane_sums64(gb, w.lo, bsz, NP, 2, 1.0, w.part, w.prod + b * NP, s);
        }
        add_level64<<<blocks(NP), T64, 0, s>>>(w.prod, NP, D.levels, lv, w.dlds);
        soff += 3 * bsz;
        copy64<<<blocks(NP * bsz), T64, 0, s>>>(w.ll, NP * bsz, w.X0);
        h = h2;
        wd = w2;
    }
}

}  // namespace

bool gap64_fft_length_ok(int n) {
    if (n < 1) return false;
    while (n > 1) {
        const int R = radix_of(n);
        if (R == 0) return false;
        n /= R;
    }
    return true;
}

size_t gap64_workspace_bytes(const Gap64Dims &D) {
    Ws64 w;
    carve64(nullptr, D, &w);
    return w.bytes;
}

hipError_t gap64_run(const Gap64Dims &D, const Filter64 &f, const double *theta, const float *cams,
                     const float *queries, const int *qcam, void *ws, double *out, double *pce_out, hipStream_t s) {
    Ws64 w;
    carve64(static_cast<char *>(ws), D, &w);
    const int nc = D.ncam, nq = D.nq, H = D.H, W = D.W;
    const int64_t npx = (int64_t)H * W, NP = (int64_t)nc * D.g + nq;
    const double N = (double)npx, sigma0 = theta[0];
    double s2[4];
    for (int l = 0; l < 4; ++l) s2[l] = theta[1 + l] * sigma0 * sigma0;
    // forward: SDA means and query planes, residuals with checkpoints
    sda64<<<blocks((int64_t)nc * D.g * npx), T64, 0, s>>>(cams, D.m, D.d, D.g, npx, nc, w.img);
    widen64<<<blocks((int64_t)nq * npx), T64, 0, s>>>(queries, (int64_t)nq * npx, w.img + (int64_t)nc * D.g * npx);
    residuals64(D, f, s2, w, s);
    // fingerprints K_j (zero-mean) and query residuals x_q (zero-mean)
    mle64<<<blocks((int64_t)nc * npx), T64, 0, s>>>(w.res, w.img, D.g, npx, nc, w.K, w.B);
    zero_mean64(w.K, nc, H, W, s);
    double *xq = w.res + (int64_t)nc * D.g * npx;
    zero_mean64(xq, nq, H, W, s);
    gap_weights64<<<1, 64, 0, s>>>(qcam, nq, nc, w.wts);
    zero64<<<blocks((int64_t)nc * npx), T64, 0, s>>>(w.gK, (int64_t)nc * npx);
    zero64<<<blocks((int64_t)nq * npx), T64, 0, s>>>(w.gx, (int64_t)nq * npx);
    double *ym = w.small, *sq = ym + nc, *gxm = sq + nc, *gym = gxm + nc, *xm = gym + nc;
    hipError_t e = hipSuccess;
    for (int q = 0; q < nq && e == hipSuccess; ++q) {
        const double *x = xq + (int64_t)q * npx, *Iq = w.img + ((int64_t)nc * D.g + q) * npx;
        // X = DFT(x - mean x);  Y_j = DFT(y_j - mean y_j), y_j = I_q K_j
        plane_sums64(x, nullptr, npx, 1, 0, 1.0 / N, w.part, xm, s);
        to_complex64<<<blocks(npx), T64, 0, s>>>(x, xm, npx, 1, w.XQ);
        e = fft2d64(w.XQ, w.T, 1, H, W, -1.0, s);
        axpm64<<<blocks((int64_t)nc * npx), T64, 0, s>>>(w.K, Iq, 1, nullptr, npx, nc, w.C);
        plane_sums64(w.C, nullptr, npx, nc, 0, 1.0 / N, w.part, ym, s);
        to_complex64<<<blocks((int64_t)nc * npx), T64, 0, s>>>(w.C, ym, npx, nc, w.Y);
        if (e == hipSuccess) e = fft2d64(w.Y, w.T, nc, H, W, -1.0, s);
        // C_j = Re IDFT(X conj(Y_j)) / N, its energy, PCE and dPCE/dC
        cprod64<<<blocks((int64_t)nc * npx), T64, 0, s>>>(w.XQ, 1, w.Y, nc, npx, nc, 0, w.Z);
        if (e == hipSuccess) e = fft2d64(w.Z, w.T, nc, H, W, 1.0, s);
        real_part64<<<blocks((int64_t)nc * npx), T64, 0, s>>>(w.Z, (int64_t)nc * npx, 1.0 / N, w.C);
        plane_sums64(w.C, nullptr, npx, nc, 1, 1.0, w.part, sq, s);
        pce_stats64<<<blocks(nc), T64, 0, s>>>(w.C, sq, H, W, D.nbhd, nc, w.pce + (int64_t)q * nc, w.coef);
        pce_gc64<<<blocks((int64_t)nc * npx), T64, 0, s>>>(w.C, w.coef, H, W, D.nbhd, nc, w.Z);
        if (e == hipSuccess) e = fft2d64(w.Z, w.T, nc, H, W, -1.0, s);  // G_j
        // gx_j = Re IDFT(G_j Y_j) / N,  gy_j = Re IDFT(conj(G_j) X) / N
        cprod64<<<blocks((int64_t)nc * npx), T64, 0, s>>>(w.Z, nc, w.Y, nc, npx, nc, 1, w.Y);
        cprod64<<<blocks((int64_t)nc * npx), T64, 0, s>>>(w.Z, nc, w.XQ, 1, npx, nc, 2, w.Z);
        if (e == hipSuccess) e = fft2d64(w.Y, w.T, nc, H, W, 1.0, s);
        if (e == hipSuccess) e = fft2d64(w.Z, w.T, nc, H, W, 1.0, s);
        real_part64<<<blocks((int64_t)nc * npx), T64, 0, s>>>(w.Y, (int64_t)nc * npx, 1.0 / N, w.gxp);
        real_part64<<<blocks((int64_t)nc * npx), T64, 0, s>>>(w.Z, (int64_t)nc * npx, 1.0 / N, w.gyp);
        plane_sums64(w.gxp, nullptr, npx, nc, 0, 1.0 / N, w.part, gxm, s);
        plane_sums64(w.gyp, nullptr, npx, nc, 0, 1.0 / N, w.part, gym, s);
        pce_accum64<<<blocks(npx), T64, 0, s>>>(w.gxp, gxm, w.gyp, gym, w.wts + (int64_t)q * nc, Iq, nc, npx,
                                               w.gx + (int64_t)q * npx, w.gK);
        if (e == hipSuccess) e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    // backward: zero-mean (self-adjoint), the MLE, the query residuals
    zero_mean64(w.gK, nc, H, W, s);
    mle_back64<<<blocks((int64_t)nc * D.g * npx), T64, 0, s>>>(w.gK, w.img, w.B, D.g, npx, nc, w.gW);
    zero_mean64(w.gx, nq, H, W, s);
    copy64<<<blocks((int64_t)nq * npx), T64, 0, s>>>(w.gx, (int64_t)nq * npx, w.gW + (int64_t)nc * D.g * npx);
    residual_vjp64(D, f, w, s);
    gap_finish64<<<1, 64, 0, s>>>(w.wts, w.pce, nq * nc, w.dlds, (int)NP, D.levels, sigma0, theta[1], theta[2],
                                  theta[3], theta[4], out);
    if (pce_out) copy64<<<blocks((int64_t)nq * nc), T64, 0, s>>>(w.pce, (int64_t)nq * nc, pce_out);
    return hipGetLastError();
}

}  // namespace prnu
