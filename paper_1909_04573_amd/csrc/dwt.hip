// Wavelet denoiser levels for gfx950: the residual W = I - F(I) of Sec. II-A
// with F the locally adaptive wavelet denoiser named in Sec. IV.
//
// Forward level (analysis + Wiener shrinkage, one launch per level):
//   a workgroup owns a T x T tile of every subband.  It stages the
//   (2(T+2*HALO)+L-2)^2 input samples the tile and a HALO-wide Wiener margin
//   need into LDS (periodic wrap, plus symmetric padding at level 1), filters
//   rows then columns in LDS with register-blocked taps held in scalar
//   registers, keeps the three detail subbands of the (T+2*HALO)^2 region in
//   LDS, and shrinks the T x T core:
//       var = min_{w=3,5,7,9} max(0, box_w(c^2)/w^2 - s2)   (zero outside the band)
//       r   = c * s2 / (var + s2)
//   It writes the approximation (input of the next level) and the residual
//   detail coefficients r; the shrunk coefficients never touch HBM.
//
// Inverse level (synthesis): a workgroup owns a 2T x 2T output tile, stages
//   the (T+L/2-1)^2 coefficients of the four subbands it needs, synthesises
//   columns then rows in LDS and either stores the plane (next level up),
//   stores the cropped residual, or (level 1 of the fingerprint path) folds
//   the MLE sums  A += W*I, B += I^2  over a batch of SDA frames in registers
//   before one read-modify-write of the accumulators.

#include "internal.h"
#include "wiener_dev.h"

namespace prnu {
namespace {

constexpr int T = 32;     // subband coefficients per tile side
constexpr int HALO = 4;   // half of the largest Wiener window (9)
constexpr int NT = 256;   // threads per workgroup

template <int TAPS>
struct FwdGeom {
    static constexpr int NC = T + 2 * HALO;       // coefficients per side incl. margin (40)
    static constexpr int IN = 2 * NC + TAPS - 2;  // input samples per side (94 for 16 taps)
    static constexpr int INS = (IN + 3) / 4 * 4;  // LDS row stride, 16-byte aligned rows
    static constexpr int QSZ = 3 * NC * NC + 3 * T * T;  // masked squares + core coefficients
    static constexpr int TILE = IN * INS > QSZ ? IN * INS : QSZ;
};

template <int TAPS>
struct InvGeom {
    static constexpr int NK = T + TAPS / 2 - 1;  // coefficients per side
    static constexpr int NKS = NK + 1;
    static constexpr int NO = 2 * T;             // outputs per side
};

// Periodic wrap into [0, n), then symmetric (edge-including) reflection of
// the padded index into the stored [0, stored) range.
__device__ __forceinline__ int map_index(int p, int n, int off, int stored) {
    int pm = p % n;
    if (pm < 0) pm += n;
    int q = pm - off;
    if (q < 0) q = -q - 1;
    if (q >= stored) q = 2 * stored - q - 1;
    return q;
}

template <int TAPS>
__global__ __launch_bounds__(NT) void dwt_fwd_wiener(const float *__restrict__ src, int64_t src_stride,
                                                     int src_rows, int src_cols, int n_r, int n_c,
                                                     int off_r, int off_c, float *__restrict__ out,
                                                     float s2, int tiles_c, int write_ll, Filter f,
                                                     float *__restrict__ ckpt, int64_t ckpt_stride) {
    using G = FwdGeom<TAPS>;
    constexpr int IN = G::IN, INS = G::INS, NC = G::NC;
    __shared__ __align__(16) float tile[G::TILE];  // input samples; later squares + core coefficients
    __shared__ __align__(16) float rlo[IN * NC];
    __shared__ __align__(16) float rhi[IN * NC];
    __shared__ int rmap[IN];
    __shared__ int cmap[IN];

    const int hk = n_r >> 1, wk = n_c >> 1;
    const int tr = blockIdx.x / tiles_c, tc = blockIdx.x - (blockIdx.x / tiles_c) * tiles_c;
    const int k0r = tr * T, k0c = tc * T;
    const float *sp = src + (int64_t)blockIdx.y * src_stride;
    float *op = out + (int64_t)blockIdx.y * 4 * hk * wk;
    const int64_t band = (int64_t)hk * wk;
    const int tid = threadIdx.x;

    if (tid < IN)
        rmap[tid] = map_index(2 * (k0r - HALO) + tid, n_r, off_r, src_rows);
    else if (tid < 2 * IN)
        cmap[tid - IN] = map_index(2 * (k0c - HALO) + tid - IN, n_c, off_c, src_cols);
    __syncthreads();

    // Stage the input tile: pairs of contiguous samples where the tile's columns
    // need neither the periodic wrap nor the reflection, single samples otherwise.
    const int c_src0 = 2 * (k0c - HALO) - off_c;
    const bool cfast = c_src0 >= 0 && c_src0 + IN <= src_cols && (c_src0 & 1) == 0 && (src_cols & 1) == 0 &&
                       (src_stride & 1) == 0;
    if (cfast) {
        constexpr int IN2 = IN / 2;
        for (int e = tid; e < IN * IN2; e += NT) {
            const int i = e / IN2, j2 = e - (e / IN2) * IN2;
            const float2 v = *reinterpret_cast<const float2 *>(sp + (int64_t)rmap[i] * src_cols + c_src0 + 2 * j2);
            *reinterpret_cast<float2 *>(&tile[i * INS + 2 * j2]) = v;
        }
    } else {
        for (int e = tid; e < IN * IN; e += NT) {
            const int i = e / IN, j = e - (e / IN) * IN;
            tile[i * INS + j] = sp[(int64_t)rmap[i] * src_cols + cmap[j]];
        }
    }
    __syncthreads();

    // Rows: lo/hi along axis 1, four coefficients per item, 16-byte LDS traffic.
    constexpr int NQ = NC / 4;
    constexpr int NX = TAPS + 8;  // TAPS + 6 samples, rounded up to whole float4s
    for (int it = tid; it < IN * NQ; it += NT) {
        const int i = it / NQ, kq = it - (it / NQ) * NQ;
        const float4 *row = reinterpret_cast<const float4 *>(&tile[i * INS + 8 * kq]);
        float x[NX];
#pragma unroll
        for (int t = 0; t < NX / 4; ++t) {
            const float4 v = row[t];
            x[4 * t] = v.x;
            x[4 * t + 1] = v.y;
            x[4 * t + 2] = v.z;
            x[4 * t + 3] = v.w;
        }
        float lo[4], hi[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            lo[u] = 0.f;
            hi[u] = 0.f;
#pragma unroll
            for (int j = 0; j < TAPS; ++j) {
                lo[u] = fmaf(f.h[j], x[2 * u + j], lo[u]);
                hi[u] = fmaf(f.g[j], x[2 * u + j], hi[u]);
            }
        }
        *reinterpret_cast<float4 *>(&rlo[i * NC + 4 * kq]) = make_float4(lo[0], lo[1], lo[2], lo[3]);
        *reinterpret_cast<float4 *>(&rhi[i * NC + 4 * kq]) = make_float4(hi[0], hi[1], hi[2], hi[3]);
    }
    __syncthreads();

    // Columns: a quad of coefficient columns by a pair of coefficient rows per
    // item.  Every detail coefficient's square goes to q (zero outside the
    // band: the Wiener windows' zero extension); the core coefficients to cb.
    float *qb = tile;                // [3][NC][NC]
    float *cb = tile + 3 * NC * NC;  // [3][T][T]
    const int gr0 = k0r - HALO, gc0 = k0c - HALO;
    for (int it = tid; it < NQ * (NC / 2); it += NT) {
        const int cq = it % NQ, kp = it / NQ;
        bool cv[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) cv[c] = gc0 + 4 * cq + c >= 0 && gc0 + 4 * cq + c < wk;
        const bool core_c = cq >= HALO / 4 && cq < (HALO + T) / 4;
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
            const float *rb = pass == 0 ? rlo : rhi;
            float4 xv[TAPS + 2];
#pragma unroll
            for (int t = 0; t < TAPS + 2; ++t) xv[t] = *reinterpret_cast<const float4 *>(&rb[(4 * kp + t) * NC + 4 * cq]);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                float a[4] = {0.f, 0.f, 0.f, 0.f}, d[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int j = 0; j < TAPS; ++j) {
                    const float4 v = xv[2 * u + j];
                    a[0] = fmaf(f.h[j], v.x, a[0]);
                    a[1] = fmaf(f.h[j], v.y, a[1]);
                    a[2] = fmaf(f.h[j], v.z, a[2]);
                    a[3] = fmaf(f.h[j], v.w, a[3]);
                    d[0] = fmaf(f.g[j], v.x, d[0]);
                    d[1] = fmaf(f.g[j], v.y, d[1]);
                    d[2] = fmaf(f.g[j], v.z, d[2]);
                    d[3] = fmaf(f.g[j], v.w, d[3]);
                }
                const int kr = 2 * kp + u;
                const bool rv = gr0 + kr >= 0 && gr0 + kr < hk;
                const bool core = core_c && kr >= HALO && kr < HALO + T;
                // pass 0 (row low-pass): a = ll, d = hl (band 2); pass 1: a = lh (band 1), d = hh (band 3)
                if (pass == 0) {
                    if (write_ll && core) {
                        const int gr = gr0 + kr;
                        if (gr < hk)
#pragma unroll
                            for (int c = 0; c < 4; ++c)
                                if (cv[c]) op[(int64_t)gr * wk + gc0 + 4 * cq + c] = a[c];
                    }
                } else {
                    *reinterpret_cast<float4 *>(&qb[(0 * NC + kr) * NC + 4 * cq]) =
                        make_float4(rv && cv[0] ? a[0] * a[0] : 0.f, rv && cv[1] ? a[1] * a[1] : 0.f,
                                    rv && cv[2] ? a[2] * a[2] : 0.f, rv && cv[3] ? a[3] * a[3] : 0.f);
                    if (core)
                        *reinterpret_cast<float4 *>(&cb[(0 * T + kr - HALO) * T + 4 * cq - HALO]) =
                            make_float4(a[0], a[1], a[2], a[3]);
                }
                const int sb = pass == 0 ? 1 : 2;  // hl -> band index 1 of q/cb, hh -> 2
                *reinterpret_cast<float4 *>(&qb[(sb * NC + kr) * NC + 4 * cq]) =
                    make_float4(rv && cv[0] ? d[0] * d[0] : 0.f, rv && cv[1] ? d[1] * d[1] : 0.f,
                                rv && cv[2] ? d[2] * d[2] : 0.f, rv && cv[3] ? d[3] * d[3] : 0.f);
                if (core)
                    *reinterpret_cast<float4 *>(&cb[(sb * T + kr - HALO) * T + 4 * cq - HALO]) =
                        make_float4(d[0], d[1], d[2], d[3]);
            }
        }
    }
    __syncthreads();

    // Wiener shrinkage of the T x T core of each detail band: one thread per
    // (band, core column, half of the core rows).  Band s of q/cb is lh, hl,
    // hh for s = 0, 1, 2, stored as subbands 1, 2, 3.
    if (tid < 3 * 2 * T) {
        const int s = tid / (2 * T), half = (tid / T) & 1, kcl = tid & (T - 1);
        const float *Q = qb + s * NC * NC;
        const float *Cc = cb + s * T * T;
        float *ob = op + (int64_t)(s + 1) * band;
        const int gco = k0c + kcl;
        float *cp = ckpt ? ckpt + (int64_t)blockIdx.y * ckpt_stride + (int64_t)s * band : nullptr;
        auto load = [&](int kr, int kc) { return Q[kr * NC + kc]; };
        auto emit = [&](int ko, float rho, float den) {
            const int gro = gr0 + ko;
            if (gro < hk && gco < wk) {
                const float c = Cc[(ko - HALO) * T + kcl];
                ob[(int64_t)gro * wk + gco] = c * rho;
                // sensitivity dr/ds = c / m where the window mean m exceeds s2, else 0
                if (cp) cp[(int64_t)gro * wk + gco] = den > s2 ? c * __builtin_amdgcn_rcpf(den) : 0.f;
            }
        };
        wiener_column<T / 2>(half * (T / 2), kcl, s2, load, emit);
    }
}

// ---------------------------------------------------------------------------
// Inverse level.

template <int TAPS>
__device__ __forceinline__ void inv_load(const float *__restrict__ lp, int hk, int wk, int k0r,
                                         int k0c, bool zero_approx, float *sb, int *rmap,
                                         int *cmap) {
    using G = InvGeom<TAPS>;
    constexpr int NK = G::NK, NKS = G::NKS;
    const int tid = threadIdx.x;
    const int64_t band = (int64_t)hk * wk;
    for (int e = tid; e < 4 * NK * NK; e += NT) {
        const int s = e / (NK * NK);
        const int rem = e - s * NK * NK;
        const int kr = rem / NK, kc = rem - (rem / NK) * NK;
        float v = 0.f;
        if (!(s == 0 && zero_approx)) v = lp[s * band + (int64_t)rmap[kr] * wk + cmap[kc]];
        sb[(s * NK + kr) * NKS + kc] = v;
    }
}

// Columns (axis 0): lo1/hi1[n][kc] for the 2T output rows.
template <int TAPS>
__device__ __forceinline__ void inv_cols(const float *sb, float *lo1, float *hi1, const Filter &f) {
    using G = InvGeom<TAPS>;
    constexpr int NK = G::NK, NKS = G::NKS, HT = TAPS / 2;
    const int tid = threadIdx.x;
    // item: column kc, quad of output rows n = 4pp .. 4pp+3 (coefficient rows 2pp .. 2pp+HT)
    for (int it = tid; it < NK * (T / 2); it += NT) {
        const int pp = it / NK, kc = it - (it / NK) * NK;
        float a[HT + 1], lh[HT + 1], hl[HT + 1], hh[HT + 1];
#pragma unroll
        for (int t = 0; t <= HT; ++t) {
            const int kr = 2 * pp + t;
            a[t] = sb[(0 * NK + kr) * NKS + kc];
            lh[t] = sb[(1 * NK + kr) * NKS + kc];
            hl[t] = sb[(2 * NK + kr) * NKS + kc];
            hh[t] = sb[(3 * NK + kr) * NKS + kc];
        }
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int par = 0; par < 2; ++par) {
                float lo = 0.f, hi = 0.f;
#pragma unroll
                for (int i = 0; i < HT; ++i) {
                    const int t = v - i + HT - 1;
                    const float hj = f.h[2 * i + par], gj = f.g[2 * i + par];
                    lo = fmaf(hj, a[t], fmaf(gj, hl[t], lo));
                    hi = fmaf(hj, lh[t], fmaf(gj, hh[t], hi));
                }
                const int n = 4 * pp + 2 * v + par;
                lo1[n * NKS + kc] = lo;
                hi1[n * NKS + kc] = hi;
            }
    }
}

// Rows (axis 1): four consecutive outputs x[n][4mq .. 4mq+3].
template <int TAPS>
__device__ __forceinline__ void inv_row_quad(const float *lo1, const float *hi1, int n, int mq,
                                             const Filter &f, float out[4]) {
    using G = InvGeom<TAPS>;
    constexpr int NKS = G::NKS, HT = TAPS / 2;
    float l[HT + 1], h[HT + 1];
#pragma unroll
    for (int t = 0; t <= HT; ++t) {
        l[t] = lo1[n * NKS + 2 * mq + t];
        h[t] = hi1[n * NKS + 2 * mq + t];
    }
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int par = 0; par < 2; ++par) {
            float x = 0.f;
#pragma unroll
            for (int i = 0; i < HT; ++i) {
                const int t = v - i + HT - 1;
                x = fmaf(f.h[2 * i + par], l[t], fmaf(f.g[2 * i + par], h[t], x));
            }
            out[2 * v + par] = x;
        }
}

template <int TAPS, int EPI>
__global__ __launch_bounds__(NT) void dwt_inv(const float *__restrict__ lvl, int hk, int wk,
                                              int zero_approx, int tiles_c, float *__restrict__ out,
                                              int H, int W, int off_r, int off_c, Filter f) {
    using G = InvGeom<TAPS>;
    constexpr int NK = G::NK, NKS = G::NKS, NO = G::NO, HT = TAPS / 2;
    __shared__ float sb[4 * NK * NKS];
    __shared__ float lo1[NO * NKS];
    __shared__ float hi1[NO * NKS];
    __shared__ int rmap[NK];
    __shared__ int cmap[NK];
    const int tid = threadIdx.x;
    const int tr = blockIdx.x / tiles_c, tc = blockIdx.x - (blockIdx.x / tiles_c) * tiles_c;
    const int k0r = tr * T, k0c = tc * T;
    if (tid < NK) {
        int k = (k0r - (HT - 1) + tid) % hk;
        rmap[tid] = k < 0 ? k + hk : k;
    } else if (tid < 2 * NK) {
        int k = (k0c - (HT - 1) + tid - NK) % wk;
        cmap[tid - NK] = k < 0 ? k + wk : k;
    }
    __syncthreads();
    const float *lp = lvl + (int64_t)blockIdx.y * 4 * hk * wk;
    inv_load<TAPS>(lp, hk, wk, k0r, k0c, zero_approx != 0, sb, rmap, cmap);
    __syncthreads();
    inv_cols<TAPS>(sb, lo1, hi1, f);
    __syncthreads();
    const int nr = 2 * hk, nc = 2 * wk;
    for (int it = tid; it < NO * (NO / 4); it += NT) {
        const int n = it / (NO / 4), mq = it - (it / (NO / 4)) * (NO / 4);
        float x[4];
        inv_row_quad<TAPS>(lo1, hi1, n, mq, f, x);
        const int gr = 2 * k0r + n;
        if (gr >= nr) continue;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int gc = 2 * k0c + 4 * mq + u;
            if (gc >= nc) continue;
            if (EPI == INV_PLANE) {
                out[(int64_t)blockIdx.y * 4 * nr * nc + (int64_t)gr * nc + gc] = x[u];
            } else {
                const int y = gr - off_r, xx = gc - off_c;
                if (y >= 0 && y < H && xx >= 0 && xx < W)
                    out[(int64_t)blockIdx.y * H * W + (int64_t)y * W + xx] = x[u];
            }
        }
    }
}

// Level 1 with the MLE epilogue over nb SDA frames of one channel.
template <int TAPS, int ACC>
__global__ __launch_bounds__(NT) void dwt_inv_mle(const float *__restrict__ lvl, int hk, int wk,
                                                  int zero_approx, int tiles_c, int nb, int C,
                                                  const float *__restrict__ means, int H, int W,
                                                  int off_r, int off_c, void *__restrict__ Av,
                                                  void *__restrict__ Bv, Filter f) {
    using G = InvGeom<TAPS>;
    constexpr int NK = G::NK, NKS = G::NKS, NO = G::NO, HT = TAPS / 2;
    constexpr int ITEMS = NO * (NO / 4) / NT;  // 4
    static_assert(NO * (NO / 4) == ITEMS * NT, "items per thread");
    __shared__ float sb[4 * NK * NKS];
    __shared__ float lo1[NO * NKS];
    __shared__ float hi1[NO * NKS];
    __shared__ int rmap[NK];
    __shared__ int cmap[NK];
    const int tid = threadIdx.x;
    const int c = blockIdx.y;
    const int tr = blockIdx.x / tiles_c, tc = blockIdx.x - (blockIdx.x / tiles_c) * tiles_c;
    const int k0r = tr * T, k0c = tc * T;
    if (tid < NK) {
        int k = (k0r - (HT - 1) + tid) % hk;
        rmap[tid] = k < 0 ? k + hk : k;
    } else if (tid < 2 * NK) {
        int k = (k0c - (HT - 1) + tid - NK) % wk;
        cmap[tid - NK] = k < 0 ? k + wk : k;
    }
    const int64_t npx = (int64_t)H * W;
    // per-thread partial sums: ITEMS row quads of 4 pixels
    double sa[ITEMS][4], sbb[ITEMS][4];  // ACC_F64 partials
    float ka[ITEMS][4], kc_[ITEMS][4];   // float partial of A (+ compensation for KAHAN)
    float kb[ITEMS][4], kbc[ITEMS][4];   // ... and of B
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            sa[k][u] = 0.0;
            sbb[k][u] = 0.0;
            ka[k][u] = kc_[k][u] = kb[k][u] = kbc[k][u] = 0.f;
        }
    for (int fr = 0; fr < nb; ++fr) {
        __syncthreads();  // maps ready / previous frame's LDS reads done
        const float *lp = lvl + (int64_t)(fr * C + c) * 4 * hk * wk;
        inv_load<TAPS>(lp, hk, wk, k0r, k0c, zero_approx != 0, sb, rmap, cmap);
        __syncthreads();
        inv_cols<TAPS>(sb, lo1, hi1, f);
        __syncthreads();
        const float *Ip = means + (int64_t)(fr * C + c) * npx;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int it = tid + k * NT;
            const int n = it / (NO / 4), mq = it - (it / (NO / 4)) * (NO / 4);
            float x[4];
            inv_row_quad<TAPS>(lo1, hi1, n, mq, f, x);
            const int y = 2 * k0r + n - off_r;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int xx = 2 * k0c + 4 * mq + u - off_c;
                if (y >= 0 && y < H && xx >= 0 && xx < W) {
                    const float I = Ip[(int64_t)y * W + xx];
                    if (ACC == PRNU_ACC_KAHAN_F32) {
                        // two-sum accumulation of W*I and I*I
                        const float pa = x[u] * I, pb = I * I;
                        float t = ka[k][u] + pa;
                        float z = t - ka[k][u];
                        kc_[k][u] += (ka[k][u] - (t - z)) + (pa - z);
                        ka[k][u] = t;
                        t = kb[k][u] + pb;
                        z = t - kb[k][u];
                        kbc[k][u] += (kb[k][u] - (t - z)) + (pb - z);
                        kb[k][u] = t;
                    } else if (ACC == PRNU_ACC_F32) {
                        ka[k][u] = fmaf(x[u], I, ka[k][u]);
                        kb[k][u] = fmaf(I, I, kb[k][u]);
                    } else {
                        sa[k][u] = fma((double)x[u], (double)I, sa[k][u]);
                        sbb[k][u] = fma((double)I, (double)I, sbb[k][u]);
                    }
                }
            }
        }
    }
    // one read-modify-write of the accumulators per pixel
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int it = tid + k * NT;
        const int n = it / (NO / 4), mq = it - (it / (NO / 4)) * (NO / 4);
        const int y = 2 * k0r + n - off_r;
        if (y < 0 || y >= H) continue;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int xx = 2 * k0c + 4 * mq + u - off_c;
            if (xx < 0 || xx >= W) continue;
            const int64_t o = (int64_t)c * npx + (int64_t)y * W + xx;
            if (ACC == PRNU_ACC_F64) {
                double *A = static_cast<double *>(Av);
                double *B = static_cast<double *>(Bv);
                A[o] += sa[k][u];
                B[o] += sbb[k][u];
            } else if (ACC == PRNU_ACC_F32) {
                float *A = static_cast<float *>(Av);
                float *B = static_cast<float *>(Bv);
                A[o] += ka[k][u];
                B[o] += kb[k][u];
            } else {
                // value plane [0], compensation plane [1]
                float *A = static_cast<float *>(Av);
                float *B = static_cast<float *>(Bv);
                const int64_t cs = (int64_t)C * npx;
                float s = A[o], t = s + ka[k][u], z = t - s;
                A[o + cs] += kc_[k][u] + ((s - (t - z)) + (ka[k][u] - z));
                A[o] = t;
                s = B[o];
                t = s + kb[k][u];
                z = t - s;
                B[o + cs] += kbc[k][u] + ((s - (t - z)) + (kb[k][u] - z));
                B[o] = t;
            }
        }
    }
}

inline unsigned ceil_div(int a, int b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

hipError_t launch_dwt_fwd(int taps, const Filter &f, const float *src, int64_t src_stride,
                          int src_rows, int src_cols, int n_r, int n_c, int off_r, int off_c,
                          float *out, int planes, float s2, bool write_ll, hipStream_t s, float *ckpt,
                          int64_t ckpt_stride) {
    const int hk = n_r / 2, wk = n_c / 2;
    const int tr = (int)ceil_div(hk, T), tc = (int)ceil_div(wk, T);
    dim3 grid((unsigned)(tr * tc), (unsigned)planes);
    const double bytes = (double)planes * 4.0 *
                         ((double)src_rows * src_cols + (write_ll ? 4.0 : 3.0) * (double)hk * wk);
    KernelTimer kt(taps == 16 ? "dwt_fwd_wiener<16>" : "dwt_fwd_wiener<8>", bytes, s);
    if (taps == 16)
        dwt_fwd_wiener<16><<<grid, NT, 0, s>>>(src, src_stride, src_rows, src_cols, n_r, n_c, off_r,
                                               off_c, out, s2, tc, write_ll ? 1 : 0, f, ckpt, ckpt_stride);
    else
        dwt_fwd_wiener<8><<<grid, NT, 0, s>>>(src, src_stride, src_rows, src_cols, n_r, n_c, off_r,
                                              off_c, out, s2, tc, write_ll ? 1 : 0, f, ckpt, ckpt_stride);
    return hipGetLastError();
}

hipError_t launch_dwt_inv(int taps, const Filter &f, const float *lvl, int hk, int wk,
                          bool zero_approx, int planes, int epi, float *out, int H, int W,
                          int off_r, int off_c, hipStream_t s) {
    const int tr = (int)ceil_div(hk, T), tc = (int)ceil_div(wk, T);
    dim3 grid((unsigned)(tr * tc), (unsigned)planes);
    const int za = zero_approx ? 1 : 0;
    const double outpx = epi == INV_PLANE ? 4.0 * hk * wk : (double)H * W;
    const double bytes = (double)planes * 4.0 * ((zero_approx ? 3.0 : 4.0) * (double)hk * wk + outpx);
    static const char *names[2][2] = {{"dwt_inv<8,plane>", "dwt_inv<8,resid>"},
                                      {"dwt_inv<16,plane>", "dwt_inv<16,resid>"}};
    KernelTimer kt(names[taps == 16][epi == INV_PLANE ? 0 : 1], bytes, s);
#define PRNU_INV(TP, EP)                                                                        \
    dwt_inv<TP, EP><<<grid, NT, 0, s>>>(lvl, hk, wk, za, tc, out, H, W, off_r, off_c, f)
    if (taps == 16) {
        if (epi == INV_PLANE) PRNU_INV(16, INV_PLANE); else PRNU_INV(16, INV_RESID);
    } else {
        if (epi == INV_PLANE) PRNU_INV(8, INV_PLANE); else PRNU_INV(8, INV_RESID);
    }
#undef PRNU_INV
    return hipGetLastError();
}

hipError_t launch_dwt_inv_mle(int taps, const Filter &f, const float *lvl, int hk, int wk,
                              bool zero_approx, int nb, int C, const float *means, int H, int W,
                              int off_r, int off_c, int acc_mode, void *A, void *B, hipStream_t s) {
    const int tr = (int)ceil_div(hk, T), tc = (int)ceil_div(wk, T);
    dim3 grid((unsigned)(tr * tc), (unsigned)C);
    const int za = zero_approx ? 1 : 0;
    const double accb = acc_mode == PRNU_ACC_F32 ? 16.0 : 32.0;  // A and B, read + write
    const double bytes = (double)nb * C * 4.0 * ((zero_approx ? 3.0 : 4.0) * (double)hk * wk + (double)H * W) +
                         (double)C * H * W * accb;
    KernelTimer kt(taps == 16 ? "dwt_inv_mle<16>" : "dwt_inv_mle<8>", bytes, s);
#define PRNU_MLE(TP, AC)                                                                          \
    dwt_inv_mle<TP, AC><<<grid, NT, 0, s>>>(lvl, hk, wk, za, tc, nb, C, means, H, W, off_r, off_c, \
                                            A, B, f)
    if (taps == 16) {
        if (acc_mode == PRNU_ACC_F64) PRNU_MLE(16, PRNU_ACC_F64);
        else if (acc_mode == PRNU_ACC_KAHAN_F32) PRNU_MLE(16, PRNU_ACC_KAHAN_F32);
        else PRNU_MLE(16, PRNU_ACC_F32);
    } else {
        if (acc_mode == PRNU_ACC_F64) PRNU_MLE(8, PRNU_ACC_F64);
        else if (acc_mode == PRNU_ACC_KAHAN_F32) PRNU_MLE(8, PRNU_ACC_KAHAN_F32);
        else PRNU_MLE(8, PRNU_ACC_F32);
    }
#undef PRNU_MLE
    return hipGetLastError();
}

}  // namespace prnu
