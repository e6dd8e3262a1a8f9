// Wavelet denoiser levels for gfx950: the residual W = I - F(I) of Sec. II-A
// with F the locally adaptive wavelet denoiser named in Sec. IV.
//
// Forward level (analysis + Wiener shrinkage, one launch per level):
//   a workgroup owns a TT x TT tile of every subband (TT = 16 or 32).  It
//   stages the (2(TT+2*HALO)+L-2)^2 input samples the tile and a HALO-wide
//   Wiener margin need into LDS (periodic wrap, plus symmetric padding at
//   level 1), filters rows then columns in LDS with register-blocked taps held
//   in scalar registers, keeps the squares of the three detail bands over the
//   (TT+2*HALO)^2 region (zero outside the band) in LDS, and shrinks the core:
//       var = min_{w=3,5,7,9} max(0, box_w(c^2)/w^2 - s2)
//       r   = c * s2 / (var + s2)
//   It writes the approximation (input of the next level) and the residual
//   detail coefficients r; the shrunk coefficients never touch HBM.  One LDS
//   area holds in turn the input samples, the row-filtered bands and the
//   squares, each pass keeping its results in registers across a barrier.
//   Level 1 reads float planes or, at SDA depth 1, one channel of the u8
//   frames themselves.
//
// Inverse level (synthesis): a workgroup owns a 2TT x 2TT output tile, stages
//   the (TT+L/2-1)^2 coefficients of the four subbands it needs, synthesises
//   columns then rows in LDS and either stores the plane (next level up),
//   stores the cropped residual, or (level 1 of the fingerprint path) folds
//   the MLE sums  A += W*I, B += I^2  over a batch of SDA frames in registers
//   (I the SDA means, or the u8 frames at depth 1) before one
//   read-modify-write of the accumulators.
//
// Each level body is a device function of (tile, plane) working in an LDS
// area handed to it, so the per-plane kernels (tile and plane from blockIdx)
// and the batched work-queue kernels (planes of many cameras of different
// sizes in one launch) run the same code.

#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "internal.h"
#include "stage_dev.h"
#include "wiener_dev.h"

namespace prnu {
namespace {

constexpr int HALO = 4;  // half of the largest Wiener window (9)
constexpr int NT = 256;  // threads per workgroup
// Forward-level workgroups with 32 x 32 tiles take 36 KB of LDS (four per
// CU); 512 threads give each of them eight waves.
constexpr int FWD_NT32 = 512;
constexpr int fwd_nt(int tt) { return tt == 32 ? FWD_NT32 : NT; }
// Row parts per core column in the forward level's Wiener stage: each part
// re-reads eight halo rows, so few long parts beat many short ones once other
// workgroups on the CU cover the idle threads.
constexpr int WIENER_SPLIT = 2;
// Inverse levels with 32 x 32 tiles run 512 threads per workgroup.
constexpr int INV_NT32 = 512;
constexpr int inv_nt(int tt) { return tt == 32 ? INV_NT32 : NT; }

template <int TAPS, int TT>
struct FwdGeom {
    static constexpr int NC = TT + 2 * HALO;              // coefficients per side incl. margin
    static constexpr int IN = 2 * NC + TAPS - 2;          // input samples per side
    static constexpr int INS = (IN + 3) / 4 * 4;          // LDS row stride, 16-byte aligned rows
    static constexpr int QSZ = 3 * NC * NC + 3 * TT * TT;  // masked squares + core coefficients
    static constexpr int RL = IN * NC;                    // one row-filtered band
    // One area holds, in turn, the input samples, the two row-filtered bands
    // and the squares + core coefficients: each pass keeps its results in
    // registers until every thread has read its inputs.
    static constexpr int TILE = IN * INS > QSZ ? (IN * INS > 2 * RL ? IN * INS : 2 * RL) : (QSZ > 2 * RL ? QSZ : 2 * RL);
    static constexpr int LDS = TILE + 2 * IN;             // floats; the two index maps at the end
    static_assert(TILE % 4 == 0 && RL % 4 == 0 && NC % 4 == 0, "16-byte aligned LDS areas");
};

template <int TAPS, int TT>
struct InvGeom {
    static constexpr int NK = TT + TAPS / 2 - 1;  // coefficients per side
    static constexpr int NKS = NK + 1;
    static constexpr int NO = 2 * TT;             // outputs per side
    static constexpr int SB = 4 * NK * NKS;
    static constexpr int L1 = NO * NKS;
    static constexpr int LDS = SB + 2 * L1 + 2 * NK;
};

// The thread index as a value the compiler cannot hoist out of a persistent
// loop: the per-thread index arithmetic of a level body is recomputed for
// every tile instead of being kept live in registers across tiles.
__device__ __forceinline__ int opaque_tid() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

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

// ---------------------------------------------------------------------------
// Forward level: staging of a tile's input samples.  maps() writes the
// periodic/reflected source row and column of every tile sample to LDS;
// fetch() issues the tile's global loads into registers (pairs of contiguous
// samples where the tile's columns need neither the periodic wrap nor the
// reflection, single samples otherwise); put() stores them to LDS.  Threads
// form CX columns x RY rows: a thread looks up its column offsets once and one
// row offset per row it reads, so each load costs an address add, and every
// load of a thread is issued before the first LDS store.  Splitting fetch and
// put keeps the register staging separate from the LDS layout.
template <int TAPS, int TT>
struct FwdStage {
    using G = FwdGeom<TAPS, TT>;
    static constexpr int NTH = fwd_nt(TT), IN = G::IN, INS = G::INS, IN2 = IN / 2;
    static constexpr int CXF = IN2 <= 32 ? 32 : 64, RYF = NTH / CXF, NRGF = (IN + RYF - 1) / RYF;
    static constexpr int CXS = 32, RYS = NTH / CXS, NCGS = (IN + CXS - 1) / CXS, NRGS = (IN + RYS - 1) / RYS;
    static constexpr int NV = 2 * NRGF > NRGS * NCGS ? 2 * NRGF : NRGS * NCGS;
    float v[NV];
    bool fast;

    static __device__ __forceinline__ void maps(const FwdArgs &a, int tile, int tid, int *rmap, int *cmap) {
        const int tr = tile / a.tiles_c, tc = tile - (tile / a.tiles_c) * a.tiles_c;
        if (tid < IN)  // row offsets in elements (< 2^30: a plane has at most 2^15 x 2^15 samples)
            rmap[tid] = map_index(2 * (tr * TT - HALO) + tid, a.n_r, a.off_r, a.src_rows) * a.src_cols;
        else if (tid < 2 * IN)
            cmap[tid - IN] = map_index(2 * (tc * TT - HALO) + tid - IN, a.n_c, a.off_c, a.src_cols);
    }
    __device__ __forceinline__ void fetch(const FwdArgs &a, int tile, int plane, int tid, const int *rmap,
                                          const int *cmap) {
        const int tc = tile - (tile / a.tiles_c) * a.tiles_c;
        const PRNU_GLOBAL float *sp = gmem(a.src) + (int64_t)plane * a.src_stride;
        const int c_src0 = 2 * (tc * TT - HALO) - a.off_c;
        fast = !a.src8 && c_src0 >= 0 && c_src0 + IN <= a.src_cols && (c_src0 & 1) == 0 &&
               (a.src_cols & 1) == 0 && (a.src_stride & 1) == 0;
        if (fast) {
            const int tx = tid % CXF, ty = tid / CXF;
            const PRNU_GLOBAL float *cp0 = sp + c_src0 + 2 * tx;
#pragma unroll
            for (int i = 0; i < NRGF; ++i) {
                const int r = ty + i * RYF;
                if (tx < IN2 && r < IN) {
                    const float2 t = ld2(cp0 + (unsigned)rmap[r]);
                    v[2 * i] = t.x;
                    v[2 * i + 1] = t.y;
                }
            }
        } else {
            const int tx = tid % CXS, ty = tid / CXS;
            int coff[NCGS];
#pragma unroll
            for (int g = 0; g < NCGS; ++g) coff[g] = tx + g * CXS < IN ? cmap[tx + g * CXS] : 0;
            if (a.src8) {
                // one channel of interleaved u8 frames (exact in float)
                const int C8 = a.src8_c;
                const PRNU_GLOBAL unsigned char *bp =
                    gmem(a.src8) + (int64_t)(plane / C8) * a.src_rows * a.src_cols * C8 + plane % C8;
#pragma unroll
                for (int i = 0; i < NRGS; ++i) {
                    const int r = ty + i * RYS;
                    const unsigned ro = r < IN ? (unsigned)rmap[r] : 0u;
#pragma unroll
                    for (int g = 0; g < NCGS; ++g)
                        if (r < IN && tx + g * CXS < IN) v[i * NCGS + g] = (float)bp[(ro + (unsigned)coff[g]) * (unsigned)C8];
                }
            } else {
#pragma unroll
                for (int i = 0; i < NRGS; ++i) {
                    const int r = ty + i * RYS;
                    const PRNU_GLOBAL float *rp = sp + (unsigned)(r < IN ? rmap[r] : 0);
#pragma unroll
                    for (int g = 0; g < NCGS; ++g)
                        if (r < IN && tx + g * CXS < IN) v[i * NCGS + g] = rp[coff[g]];
                }
            }
        }
    }
    __device__ __forceinline__ void put(float *tbuf, int tid) const {
        if (fast) {
            const int tx = tid % CXF, ty = tid / CXF;
#pragma unroll
            for (int i = 0; i < NRGF; ++i) {
                const int r = ty + i * RYF;
                if (tx < IN2 && r < IN)
                    *reinterpret_cast<float2 *>(&tbuf[r * INS + 2 * tx]) = make_float2(v[2 * i], v[2 * i + 1]);
            }
        } else {
            const int tx = tid % CXS, ty = tid / CXS;
#pragma unroll
            for (int i = 0; i < NRGS; ++i)
#pragma unroll
                for (int g = 0; g < NCGS; ++g) {
                    const int r = ty + i * RYS;
                    if (r < IN && tx + g * CXS < IN) tbuf[r * INS + tx + g * CXS] = v[i * NCGS + g];
                }
        }
    }
};

// Forward level work on a staged tile (`tile` of plane `plane`, input samples
// in LDS): row pass, column pass, Wiener shrinkage of the detail bands.
template <int TAPS, int TT>
__device__ __forceinline__ void fwd_compute(const FwdArgs &a, int tile, int plane, float *lds, const Filter &f) {
    using G = FwdGeom<TAPS, TT>;
    constexpr int NTH = fwd_nt(TT);
    constexpr int IN = G::IN, INS = G::INS, NC = G::NC;
    float *tbuf = lds;             // input samples, then the row bands, then squares + core coefficients
    float *rlo = lds;              // row low-pass
    float *rhi = lds + G::RL;      // row high-pass
    const int hk = a.n_r >> 1, wk = a.n_c >> 1;
    const int tr = tile / a.tiles_c, tc = tile - (tile / a.tiles_c) * a.tiles_c;
    const int k0r = tr * TT, k0c = tc * TT;
    PRNU_GLOBAL float *op = gmem(a.out) + (int64_t)plane * 4 * hk * wk;
    const int64_t band = (int64_t)hk * wk;
    const int tid = opaque_tid();

    // Rows: lo/hi along axis 1, four coefficients per item, 16-byte LDS traffic.
    constexpr int NQ = NC / 4;
    constexpr int NX = TAPS + 8;  // TAPS + 6 samples, rounded up to whole float4s
    constexpr int RITEMS = IN * NQ, RIT = (RITEMS + NTH - 1) / NTH;
    float rl[RIT][4], rh[RIT][4];
#pragma unroll
    for (int k = 0; k < RIT; ++k) {
        const int it = tid + k * NTH;
        if (it < RITEMS) {
            const int i = it / NQ, kq = it - (it / NQ) * NQ;
            const float4 *row = reinterpret_cast<const float4 *>(&tbuf[i * INS + 8 * kq]);
            float x[NX];
#pragma unroll
            for (int t = 0; t < NX / 4; ++t) {
                const float4 v = row[t];
                x[4 * t] = v.x;
                x[4 * t + 1] = v.y;
                x[4 * t + 2] = v.z;
                x[4 * t + 3] = v.w;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                rl[k][u] = 0.f;
                rh[k][u] = 0.f;
#pragma unroll
                for (int j = 0; j < TAPS; ++j) {
                    rl[k][u] = fmaf(f.h[j], x[2 * u + j], rl[k][u]);
                    rh[k][u] = fmaf(f.g[j], x[2 * u + j], rh[k][u]);
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < RIT; ++k) {
        const int it = tid + k * NTH;
        if (it < RITEMS) {
            const int i = it / NQ, kq = it - (it / NQ) * NQ;
            *reinterpret_cast<float4 *>(&rlo[i * NC + 4 * kq]) = make_float4(rl[k][0], rl[k][1], rl[k][2], rl[k][3]);
            *reinterpret_cast<float4 *>(&rhi[i * NC + 4 * kq]) = make_float4(rh[k][0], rh[k][1], rh[k][2], rh[k][3]);
        }
    }
    __syncthreads();

    // Columns: a pair of coefficient columns by a pair of coefficient rows of
    // one row band per item.  Every detail coefficient's square goes to q
    // (zero outside the band: the Wiener windows' zero extension); the core
    // coefficients to cb.  Row band 0 (low-pass) gives ll (stored at once)
    // and hl (q band 1); row band 1 gives lh (q band 0) and hh (q band 2).
    float *qb = tbuf;                // [3][NC][NC]
    float *cb = tbuf + 3 * NC * NC;  // [3][TT][TT]
    const int gr0 = k0r - HALO, gc0 = k0c - HALO;
    constexpr int NP = NC / 2;
    constexpr int CITEMS = 2 * NP * NP, CIT = (CITEMS + NTH - 1) / NTH;
    float cl[CIT][2][2], ch[CIT][2][2];  // [item][row][column]
#pragma unroll
    for (int k = 0; k < CIT; ++k) {
        const int it = tid + k * NTH;
        if (it < CITEMS) {
            const int cp = it % NP, kp = (it / NP) % NP, pass = it / (NP * NP);
            const float *rb = pass == 0 ? rlo : rhi;
            float2 xv[TAPS + 2];
#pragma unroll
            for (int t = 0; t < TAPS + 2; ++t)
                xv[t] = *reinterpret_cast<const float2 *>(&rb[(4 * kp + t) * NC + 2 * cp]);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                float l0 = 0.f, l1 = 0.f, h0 = 0.f, h1 = 0.f;
#pragma unroll
                for (int j = 0; j < TAPS; ++j) {
                    const float2 v = xv[2 * u + j];
                    l0 = fmaf(f.h[j], v.x, l0);
                    l1 = fmaf(f.h[j], v.y, l1);
                    h0 = fmaf(f.g[j], v.x, h0);
                    h1 = fmaf(f.g[j], v.y, h1);
                }
                cl[k][u][0] = l0;
                cl[k][u][1] = l1;
                ch[k][u][0] = h0;
                ch[k][u][1] = h1;
                const int kr = 2 * kp + u;
                const bool core = cp >= HALO / 2 && cp < (HALO + TT) / 2 && kr >= HALO && kr < HALO + TT;
                if (pass == 0 && a.write_ll && core) {
                    const int gr = gr0 + kr, gc = gc0 + 2 * cp;
                    if (gr < hk) {
                        if (gc < wk) op[(int64_t)gr * wk + gc] = l0;
                        if (gc + 1 < wk) op[(int64_t)gr * wk + gc + 1] = l1;
                    }
                }
            }
        }
    }
    __syncthreads();
    // Tiles whose margin lies inside the band (most of them) store the
    // squares without the per-coefficient range masks.
    const bool inside = gr0 >= 0 && gr0 + NC <= hk && gc0 >= 0 && gc0 + NC <= wk;
    auto store_cols = [&](auto masked) {
#pragma unroll
        for (int k = 0; k < CIT; ++k) {
            const int it = tid + k * NTH;
            if (it < CITEMS) {
                const int cp = it % NP, kp = (it / NP) % NP, pass = it / (NP * NP);
                const bool cv0 = !masked || (gc0 + 2 * cp >= 0 && gc0 + 2 * cp < wk);
                const bool cv1 = !masked || (gc0 + 2 * cp + 1 >= 0 && gc0 + 2 * cp + 1 < wk);
                const bool core_c = cp >= HALO / 2 && cp < (HALO + TT) / 2;
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int kr = 2 * kp + u;
                    const bool rv = !masked || (gr0 + kr >= 0 && gr0 + kr < hk);
                    const bool core = core_c && kr >= HALO && kr < HALO + TT;
                    auto put = [&](int sb, float c0, float c1) {
                        float2 q2 = make_float2(c0 * c0, c1 * c1);
                        if (masked) q2 = make_float2(rv && cv0 ? q2.x : 0.f, rv && cv1 ? q2.y : 0.f);
                        *reinterpret_cast<float2 *>(&qb[(sb * NC + kr) * NC + 2 * cp]) = q2;
                        if (core)
                            *reinterpret_cast<float2 *>(&cb[(sb * TT + kr - HALO) * TT + 2 * cp - HALO]) =
                                make_float2(c0, c1);
                    };
                    if (pass == 0) {
                        put(1, ch[k][u][0], ch[k][u][1]);
                    } else {
                        put(0, cl[k][u][0], cl[k][u][1]);
                        put(2, ch[k][u][0], ch[k][u][1]);
                    }
                }
            }
        }
    };
    if (inside)
        store_cols(std::false_type{});
    else
        store_cols(std::true_type{});
    __syncthreads();

    // Wiener shrinkage of the TT x TT core of each detail band: one thread per
    // (band, core column, WS-th part of the core rows).  Band s of q/cb is lh,
    // hl, hh for s = 0, 1, 2, stored as subbands 1, 2, 3.
    constexpr int WS = WIENER_SPLIT;
    static_assert(3 * WS * TT <= NTH, "one Wiener column part per thread");
    if (tid < 3 * WS * TT) {
        const int s = tid / (WS * TT), part = (tid / TT) % WS, kcl = tid & (TT - 1);
        const float *Q = qb + s * NC * NC;
        const float *Cc = cb + s * TT * TT;
        PRNU_GLOBAL float *ob = op + (int64_t)(s + 1) * band;
        PRNU_GLOBAL float *cp = a.ckpt ? gmem(a.ckpt) + (int64_t)plane * a.ckpt_stride + (int64_t)s * band : nullptr;
        const int gco = k0c + kcl;
        const float s2 = a.s2;
        // this thread's outputs: core rows part*TT/WS + i of column kcl
        const int grow0 = k0r + part * (TT / WS);
        PRNU_GLOBAL float *orow = ob + (int64_t)grow0 * wk + gco;
        PRNU_GLOBAL float *crow = cp ? cp + (int64_t)grow0 * wk + gco : nullptr;
        const float *ccol = Cc + part * (TT / WS) * TT + kcl;
        auto load = [&](int kr, int kc) { return Q[kr * NC + kc]; };
        auto emit = [&](int ko, float rho, float den) {
            const int i = ko - HALO - part * (TT / WS);
            if (grow0 + i < hk && gco < wk) {
                const float c = ccol[i * TT];
                orow[i * wk] = c * rho;
                // sensitivity dr/ds = c / m where the window mean m exceeds s2, else 0
                if (crow) crow[i * wk] = den > s2 ? c * __builtin_amdgcn_rcpf(den) : 0.f;
            }
        };
        wiener_column<TT / WS>(part * (TT / WS), kcl, s2, load, emit);
    }
}

// Forward level body: subband tile `tile` of plane `plane`.
template <int TAPS, int TT>
__device__ __forceinline__ void fwd_body(const FwdArgs &a, int tile, int plane, float *lds, const Filter &f) {
    using G = FwdGeom<TAPS, TT>;
    int *rmap = reinterpret_cast<int *>(lds + G::TILE);
    int *cmap = rmap + G::IN;
    const int tid = opaque_tid();
    FwdStage<TAPS, TT>::maps(a, tile, tid, rmap, cmap);
    __syncthreads();
    FwdStage<TAPS, TT> st;
    st.fetch(a, tile, plane, tid, rmap, cmap);
    st.put(lds, tid);
    __syncthreads();
    fwd_compute<TAPS, TT>(a, tile, plane, lds, f);
}

// ---------------------------------------------------------------------------
// Inverse level pieces.
template <int TAPS, int TT>
__device__ __forceinline__ void inv_maps(int tid, int hk, int wk, int k0r, int k0c, int *rmap, int *cmap) {
    constexpr int NK = InvGeom<TAPS, TT>::NK, HT = TAPS / 2;
    if (tid < NK) {
        int k = (k0r - (HT - 1) + tid) % hk;
        rmap[tid] = k < 0 ? k + hk : k;
    } else if (tid < 2 * NK) {
        int k = (k0c - (HT - 1) + tid - NK) % wk;
        cmap[tid - NK] = k < 0 ? k + wk : k;
    }
}

// Staging of the (TT+L/2-1)^2 coefficients of the four subbands (subband 0
// as zeros with zero_approx).  Threads form 32 columns x (threads/32) rows: a
// thread looks up its column and row offsets once (they are the same for
// every plane of a level) and then reads the same positions of every
// subband, so each load costs one address add; a wave's lanes read
// consecutive columns of two rows.  fetch() issues a plane's loads into
// registers, put() stores them to LDS, so a caller can have the next plane's
// loads in flight while it works on the current one.
template <int TAPS, int TT>
struct InvStage {
    static constexpr int NK = InvGeom<TAPS, TT>::NK, NKS = InvGeom<TAPS, TT>::NKS;
    static constexpr int CX = 32, RY = inv_nt(TT) / CX;
    static constexpr int NCG = (NK + CX - 1) / CX, NRG = (NK + RY - 1) / RY;
    int tx, ty, coff[NCG], roff[NRG];
    float v[4][NRG][NCG];

    // rmap/cmap must be in LDS (after the barrier that follows inv_maps)
    __device__ __forceinline__ void offsets(int tid, int wk, const int *rmap, const int *cmap) {
        tx = tid % CX;
        ty = tid / CX;
#pragma unroll
        for (int g = 0; g < NCG; ++g) coff[g] = tx + g * CX < NK ? cmap[tx + g * CX] : 0;
#pragma unroll
        for (int i = 0; i < NRG; ++i) roff[i] = ty + i * RY < NK ? rmap[ty + i * RY] * wk : 0;
    }
    __device__ __forceinline__ void fetch(const float *__restrict__ lpp, int64_t band, bool zero_approx) {
        const PRNU_GLOBAL float *lp = gmem(lpp);
#pragma unroll
        for (int sbd = 0; sbd < 4; ++sbd)
#pragma unroll
            for (int i = 0; i < NRG; ++i)
#pragma unroll
                for (int g = 0; g < NCG; ++g) {
                    v[sbd][i][g] = 0.f;
                    if (ty + i * RY < NK && tx + g * CX < NK && !(sbd == 0 && zero_approx))
                        v[sbd][i][g] = lp[sbd * band + roff[i] + coff[g]];
                }
    }
    __device__ __forceinline__ void put(float *sb) const {
#pragma unroll
        for (int sbd = 0; sbd < 4; ++sbd)
#pragma unroll
            for (int i = 0; i < NRG; ++i)
#pragma unroll
                for (int g = 0; g < NCG; ++g)
                    if (ty + i * RY < NK && tx + g * CX < NK)
                        sb[(sbd * NK + ty + i * RY) * NKS + tx + g * CX] = v[sbd][i][g];
    }
};

// Columns (axis 0): lo1/hi1[n][kc] for the 2TT output rows.
template <int TAPS, int TT>
__device__ __forceinline__ void inv_cols(int tid, const float *sb, float *lo1, float *hi1, const Filter &f) {
    constexpr int NK = InvGeom<TAPS, TT>::NK, NKS = InvGeom<TAPS, TT>::NKS, HT = TAPS / 2;
    // item: column kc, quad of output rows n = 4pp .. 4pp+3 (coefficient rows 2pp .. 2pp+HT)
    for (int it = tid; it < NK * (TT / 2); it += inv_nt(TT)) {
        const int pp = it / NK, kc = it - (it / NK) * NK;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            // half 0: a and hl give lo1; half 1: lh and hh give hi1
            const int s0 = half == 0 ? 0 : 1, s1 = half == 0 ? 2 : 3;
            float p[HT + 1], q[HT + 1];
#pragma unroll
            for (int t = 0; t <= HT; ++t) {
                const int kr = 2 * pp + t;
                p[t] = sb[(s0 * NK + kr) * NKS + kc];
                q[t] = sb[(s1 * NK + kr) * NKS + kc];
            }
            float *dst = half == 0 ? lo1 : hi1;
#pragma unroll
            for (int v = 0; v < 2; ++v)
#pragma unroll
                for (int par = 0; par < 2; ++par) {
                    float acc = 0.f;
#pragma unroll
                    for (int i = 0; i < HT; ++i) {
                        const int t = v - i + HT - 1;
                        acc = fmaf(f.h[2 * i + par], p[t], fmaf(f.g[2 * i + par], q[t], acc));
                    }
                    dst[(4 * pp + 2 * v + par) * NKS + kc] = acc;
                }
        }
    }
}

// Rows (axis 1): four consecutive outputs x[n][4mq .. 4mq+3].
template <int TAPS, int TT>
__device__ __forceinline__ void inv_row_quad(const float *lo1, const float *hi1, int n, int mq, const Filter &f,
                                             float out[4]) {
    constexpr int NKS = InvGeom<TAPS, TT>::NKS, HT = TAPS / 2;
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

template <int TAPS, int TT, int EPI>
__device__ __forceinline__ void inv_body(const InvArgs &a, int tile, int plane, float *lds, const Filter &f) {
    using G = InvGeom<TAPS, TT>;
    constexpr int NO = G::NO;
    float *sb = lds, *lo1 = lds + G::SB, *hi1 = lo1 + G::L1;
    int *rmap = reinterpret_cast<int *>(hi1 + G::L1);
    int *cmap = rmap + G::NK;
    const int tid = opaque_tid();
    const int tr = tile / a.tiles_c, tc = tile - (tile / a.tiles_c) * a.tiles_c;
    const int k0r = tr * TT, k0c = tc * TT;
    inv_maps<TAPS, TT>(tid, a.hk, a.wk, k0r, k0c, rmap, cmap);
    __syncthreads();
    {
        InvStage<TAPS, TT> st;
        st.offsets(tid, a.wk, rmap, cmap);
        st.fetch(a.lvl + (int64_t)plane * 4 * a.hk * a.wk, (int64_t)a.hk * a.wk, a.zero_approx != 0);
        st.put(sb);
    }
    __syncthreads();
    inv_cols<TAPS, TT>(tid, sb, lo1, hi1, f);
    __syncthreads();
    const int nr = 2 * a.hk, nc = 2 * a.wk;
    PRNU_GLOBAL float *out = gmem(a.out);
    for (int it = tid; it < NO * (NO / 4); it += inv_nt(TT)) {
        const int n = it / (NO / 4), mq = it - (it / (NO / 4)) * (NO / 4);
        float x[4];
        inv_row_quad<TAPS, TT>(lo1, hi1, n, mq, f, x);
        const int gr = 2 * k0r + n;
        if (gr >= nr) continue;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int gc = 2 * k0c + 4 * mq + u;
            if (gc >= nc) continue;
            if (EPI == INV_PLANE) {
                out[(int64_t)plane * 4 * nr * nc + (int64_t)gr * nc + gc] = x[u];
            } else {
                const int y = gr - a.off_r, xx = gc - a.off_c;
                if (y >= 0 && y < a.H && xx >= 0 && xx < a.W)
                    out[(int64_t)plane * a.H * a.W + (int64_t)y * a.W + xx] = x[u];
            }
        }
    }
}

// Level 1 with the MLE epilogue over the a.nb SDA frames of channel c
// (planes [nb][C], means [nb][C][H][W]).
template <int TAPS, int TT, int ACC, bool U8I = false>
__device__ __forceinline__ void mle_body(const MleArgs &a, int tile, int c, float *lds, const Filter &f) {
    using G = InvGeom<TAPS, TT>;
    constexpr int NO = G::NO;
    constexpr int ITEMS = NO * (NO / 4) / inv_nt(TT);  // row quads per thread
    static_assert(NO * (NO / 4) == ITEMS * inv_nt(TT), "items per thread");
    float *sb = lds, *lo1 = lds + G::SB, *hi1 = lo1 + G::L1;
    int *rmap = reinterpret_cast<int *>(hi1 + G::L1);
    int *cmap = rmap + G::NK;
    const int tid = opaque_tid();
    const int tr = tile / a.tiles_c, tc = tile - (tile / a.tiles_c) * a.tiles_c;
    const int k0r = tr * TT, k0c = tc * TT;
    const int H = a.H, W = a.W, C = a.C;
    inv_maps<TAPS, TT>(tid, a.hk, a.wk, k0r, k0c, rmap, cmap);
    const int64_t npx = (int64_t)H * W;
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
    // subband loads of frame fr + 1 are in flight while frame fr is transformed
    __syncthreads();  // maps ready
    InvStage<TAPS, TT> st;
    st.offsets(tid, a.wk, rmap, cmap);
    const int64_t band = (int64_t)a.hk * a.wk;
    st.fetch(a.lvl + (int64_t)c * 4 * band, band, a.zero_approx != 0);
    for (int fr = 0; fr < a.nb; ++fr) {
        // this frame's SDA means, loaded ahead of the subband staging (kept
        // in registers only where a thread owns a single row quad)
        const PRNU_GLOBAL float *Ip = gmem(a.means) + (int64_t)(fr * C + c) * npx;
        // U8I: SDA depth 1, the means are the u8 frames (a.means8) themselves
        const PRNU_GLOBAL unsigned char *I8 = U8I ? gmem(a.means8) + (int64_t)fr * npx * C + c : nullptr;
        auto load_I = [&](int y, int xx) {
            if constexpr (U8I)
                return (float)I8[((int64_t)y * W + xx) * C];
            else
                return Ip[(int64_t)y * W + xx];
        };
        constexpr int PF = ITEMS == 1 ? 1 : 0;
        float Iv[PF ? ITEMS : 1][4];
#pragma unroll
        for (int k = 0; k < (PF ? ITEMS : 0); ++k) {
            const int it = tid + k * inv_nt(TT);
            const int n = it / (NO / 4), mq = it - (it / (NO / 4)) * (NO / 4);
            const int y = 2 * k0r + n - a.off_r;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int xx = 2 * k0c + 4 * mq + u - a.off_c;
                Iv[k][u] = (y >= 0 && y < H && xx >= 0 && xx < W) ? load_I(y, xx) : 0.f;
            }
        }
        // The previous frame's column pass finished reading sb before the
        // barrier that precedes its row pass, and this frame's column pass
        // writes lo1/hi1 only after the next barrier, which every thread
        // reaches after its row pass: one barrier per hand-over suffices.
        st.put(sb);
        __syncthreads();
        if (fr + 1 < a.nb) st.fetch(a.lvl + (int64_t)((fr + 1) * C + c) * 4 * band, band, a.zero_approx != 0);
        const int tf = opaque_tid();  // index arithmetic per frame, not live across the frame loop
        inv_cols<TAPS, TT>(tf, sb, lo1, hi1, f);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int it = tid + k * inv_nt(TT);
            const int n = it / (NO / 4), mq = it - (it / (NO / 4)) * (NO / 4);
            float x[4];
            inv_row_quad<TAPS, TT>(lo1, hi1, n, mq, f, x);
            const int y = 2 * k0r + n - a.off_r;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int xx = 2 * k0c + 4 * mq + u - a.off_c;
                if (y >= 0 && y < H && xx >= 0 && xx < W) {
                    const float I = PF ? Iv[PF ? k : 0][u] : load_I(y, xx);
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
        const int it = tid + k * inv_nt(TT);
        const int n = it / (NO / 4), mq = it - (it / (NO / 4)) * (NO / 4);
        const int y = 2 * k0r + n - a.off_r;
        if (y < 0 || y >= H) continue;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int xx = 2 * k0c + 4 * mq + u - a.off_c;
            if (xx < 0 || xx >= W) continue;
            const int64_t o = (int64_t)c * npx + (int64_t)y * W + xx;
            if (ACC == PRNU_ACC_F64) {
                PRNU_GLOBAL double *A = gmem(static_cast<double *>(a.A));
                PRNU_GLOBAL double *B = gmem(static_cast<double *>(a.B));
                A[o] += sa[k][u];
                B[o] += sbb[k][u];
            } else if (ACC == PRNU_ACC_F32) {
                PRNU_GLOBAL float *A = gmem(static_cast<float *>(a.A));
                PRNU_GLOBAL float *B = gmem(static_cast<float *>(a.B));
                A[o] += ka[k][u];
                B[o] += kb[k][u];
            } else {
                // value plane [0], compensation plane [1]
                PRNU_GLOBAL float *A = gmem(static_cast<float *>(a.A));
                PRNU_GLOBAL float *B = gmem(static_cast<float *>(a.B));
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

// ---------------------------------------------------------------------------
// Per-plane kernels.
template <int TAPS, int TT>
__global__ __launch_bounds__(fwd_nt(TT)) void dwt_fwd_wiener(FwdArgs a, Filter f) {
    __shared__ __align__(16) float lds[FwdGeom<TAPS, TT>::LDS];
    int tile, plane;
    if (a.src8 && a.src8_c > 1)
        grid_tile_channels(tile, plane, a.src8_c);
    else
        grid_tile(tile, plane);
    fwd_body<TAPS, TT>(a, tile, plane, lds, f);
}

template <int TAPS, int TT, int EPI>
__global__ __launch_bounds__(inv_nt(TT)) void dwt_inv(InvArgs a, Filter f) {
    __shared__ __align__(16) float lds[InvGeom<TAPS, TT>::LDS];
    int tile, plane;
    grid_tile(tile, plane);
    inv_body<TAPS, TT, EPI>(a, tile, plane, lds, f);
}

template <int TAPS, int TT, int ACC, bool U8I>
__global__ __launch_bounds__(inv_nt(TT)) void dwt_inv_mle(MleArgs a, Filter f) {
    __shared__ __align__(16) float lds[InvGeom<TAPS, TT>::LDS];
    int tile, c;
    grid_tile(tile, c);
    mle_body<TAPS, TT, ACC, U8I>(a, tile, c, lds, f);
}

// ---------------------------------------------------------------------------
// Work-queue kernels: a persistent grid takes virtual blocks from a counter;
// virtual block vb belongs to the last descriptor whose block0 <= vb (binary
// search; block0 ascending, first 0) and is (tile, plane) of that level, tile
// fastest.  Every workgroup leaves once the counter has passed `total`, so
// the grid drains whatever its size; the host keeps total + grid < 2^31.
template <typename D>
__device__ __forceinline__ int find_desc(const D *__restrict__ d, int nd, int vb) {
    int lo = 0, hi = nd - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].block0 <= vb)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// One thread takes the next virtual block for the workgroup (vector atomic on
// the global counter), the barrier publishes it through LDS.
__device__ __forceinline__ int next_block(int *ctr, int *slot) {
    __syncthreads();  // the previous block's LDS use is over
    if (threadIdx.x == 0) *slot = atomicAdd(ctr, 1);
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(*slot);  // uniform: descriptor fields go to scalar registers
}

template <int TAPS, int TT>
__global__ __launch_bounds__(fwd_nt(TT)) void dwt_fwd_multi(const FwdDesc *__restrict__ d, int nd, int total, int *ctr,
                                                    Filter f) {
    __shared__ __align__(16) float lds[FwdGeom<TAPS, TT>::LDS];
    __shared__ int slot;
    for (;;) {
        const int vb = next_block(ctr, &slot);
        if (vb >= total) break;
        const FwdDesc &D = d[find_desc(d, nd, vb)];
        const int local = vb - (int)D.block0;
        fwd_body<TAPS, TT>(D.a, local % D.tiles, local / D.tiles, lds, f);
    }
}

template <int TAPS, int TT>
__global__ __launch_bounds__(inv_nt(TT)) void dwt_inv_multi(const InvDesc *__restrict__ d, int nd, int total, int *ctr,
                                                    Filter f) {
    __shared__ __align__(16) float lds[InvGeom<TAPS, TT>::LDS];
    __shared__ int slot;
    for (;;) {
        const int vb = next_block(ctr, &slot);
        if (vb >= total) break;
        const InvDesc &D = d[find_desc(d, nd, vb)];
        const int local = vb - (int)D.block0;
        inv_body<TAPS, TT, INV_PLANE>(D.a, local % D.tiles, local / D.tiles, lds, f);
    }
}

template <int TAPS, int TT, int ACC>
__global__ __launch_bounds__(inv_nt(TT)) void dwt_mle_multi(const MleDesc *__restrict__ d, int nd, int total, int *ctr,
                                                    Filter f) {
    __shared__ __align__(16) float lds[InvGeom<TAPS, TT>::LDS];
    __shared__ int slot;
    for (;;) {
        const int vb = next_block(ctr, &slot);
        if (vb >= total) break;
        const MleDesc &D = d[find_desc(d, nd, vb)];
        const int local = vb - (int)D.block0;
        mle_body<TAPS, TT, ACC>(D.a, local % D.tiles, local / D.tiles, lds, f);
    }
}

__global__ void zero_ints(int *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Grey levels in [40, 220] from an integer hash of the index (timing input).
__global__ void fill_pattern(float *x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t h = (uint32_t)i * 2654435761u;
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    x[i] = 40.f + (float)(h & 0xFFFFu) * (180.f / 65535.f);
}

inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

std::mutex g_tile_mu;
std::map<std::tuple<int, int, int, int>, int> g_tile;

template <typename K>
int occupancy_of(K kernel, int threads = NT) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, threads, 0) != hipSuccess || n < 1) n = 1;
    return n;
}

}  // namespace

int device_cus() {
    static std::mutex mu;
    static std::map<int, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 256;
    cache[dev] = n;
    return n;
}

int tile_choice(int kind, int taps, int hk, int wk) {
    std::lock_guard<std::mutex> lk(g_tile_mu);
    auto it = g_tile.find(std::make_tuple(kind, taps, hk, wk));
    return it == g_tile.end() ? 32 : it->second;
}

void set_tile_choice(int kind, int taps, int hk, int wk, int tt) {
    std::lock_guard<std::mutex> lk(g_tile_mu);
    g_tile[std::make_tuple(kind, taps, hk, wk)] = tt == 16 ? 16 : 32;
}

hipError_t launch_dwt_fwd(int taps, const Filter &f, const float *src, int64_t src_stride, int src_rows,
                          int src_cols, int n_r, int n_c, int off_r, int off_c, float *out, int planes, float s2,
                          bool write_ll, hipStream_t s, float *ckpt, int64_t ckpt_stride, const unsigned char *src8,
                          int src8_c) {
    const int hk = n_r / 2, wk = n_c / 2;
    const int tt = tile_choice(TK_FWD, taps, hk, wk);
    FwdArgs a{src, src_stride, src_rows, src_cols, n_r, n_c, off_r, off_c, out, s2,
              ceil_div(wk, tt), write_ll ? 1 : 0, ckpt, ckpt_stride, src8, src8_c};
    dim3 grid((unsigned)tiles_for(tt, hk, wk), (unsigned)planes);
    const double bytes = (double)planes * ((src8 ? 1.0 : 4.0) * (double)src_rows * src_cols +
                                           4.0 * (write_ll ? 4.0 : 3.0) * (double)hk * wk);
    KernelTimer kt(taps == 16 ? "dwt_fwd_wiener<16>" : "dwt_fwd_wiener<8>", bytes, s,
                   (double)planes * n_r * n_c * fwd_flops_per_px(taps));
    if (taps == 16) {
        if (tt == 16) dwt_fwd_wiener<16, 16><<<grid, fwd_nt(16), 0, s>>>(a, f);
        else dwt_fwd_wiener<16, 32><<<grid, fwd_nt(32), 0, s>>>(a, f);
    } else {
        if (tt == 16) dwt_fwd_wiener<8, 16><<<grid, fwd_nt(16), 0, s>>>(a, f);
        else dwt_fwd_wiener<8, 32><<<grid, fwd_nt(32), 0, s>>>(a, f);
    }
    return hipGetLastError();
}

hipError_t launch_dwt_inv(int taps, const Filter &f, const float *lvl, int hk, int wk, bool zero_approx, int planes,
                          int epi, float *out, int H, int W, int off_r, int off_c, hipStream_t s) {
    const int tt = tile_choice(TK_INV, taps, hk, wk);
    InvArgs a{lvl, hk, wk, zero_approx ? 1 : 0, ceil_div(wk, tt), out, H, W, off_r, off_c};
    dim3 grid((unsigned)tiles_for(tt, hk, wk), (unsigned)planes);
    const double outpx = epi == INV_PLANE ? 4.0 * hk * wk : (double)H * W;
    const double bytes = (double)planes * 4.0 * ((zero_approx ? 3.0 : 4.0) * (double)hk * wk + outpx);
    static const char *names[2][2] = {{"dwt_inv<8,plane>", "dwt_inv<8,resid>"},
                                      {"dwt_inv<16,plane>", "dwt_inv<16,resid>"}};
    KernelTimer kt(names[taps == 16][epi == INV_PLANE ? 0 : 1], bytes, s,
                   (double)planes * 4.0 * hk * wk * inv_flops_per_px(taps));
#define PRNU_INV(TP, T_)                                                  \
    do {                                                                  \
        if (epi == INV_PLANE) dwt_inv<TP, T_, INV_PLANE><<<grid, inv_nt(T_), 0, s>>>(a, f); \
        else dwt_inv<TP, T_, INV_RESID><<<grid, inv_nt(T_), 0, s>>>(a, f);        \
    } while (0)
    if (taps == 16) {
        if (tt == 16) PRNU_INV(16, 16); else PRNU_INV(16, 32);
    } else {
        if (tt == 16) PRNU_INV(8, 16); else PRNU_INV(8, 32);
    }
#undef PRNU_INV
    return hipGetLastError();
}

hipError_t launch_dwt_inv_mle(int taps, const Filter &f, const float *lvl, int hk, int wk, bool zero_approx, int nb,
                              int C, const float *means, int H, int W, int off_r, int off_c, int acc_mode, void *A,
                              void *B, hipStream_t s, const unsigned char *means8) {
    const int tt = tile_choice(TK_MLE, taps, hk, wk);
    MleArgs a{lvl, hk, wk, zero_approx ? 1 : 0, ceil_div(wk, tt), nb, C, means, H, W, off_r, off_c, A, B, means8};
    dim3 grid((unsigned)tiles_for(tt, hk, wk), (unsigned)C);
    const double accb = acc_mode == PRNU_ACC_F32 ? 16.0 : 32.0;  // A and B, read + write
    const double bytes = (double)nb * C *
                             (4.0 * (zero_approx ? 3.0 : 4.0) * (double)hk * wk + (means8 ? 1.0 : 4.0) * H * W) +
                         (double)C * H * W * accb;
    KernelTimer kt(taps == 16 ? "dwt_inv_mle<16>" : "dwt_inv_mle<8>", bytes, s,
                   (double)nb * C * (4.0 * hk * wk * inv_flops_per_px(taps) + 4.0 * H * W));
#define PRNU_MLE_U(TP, T_, U)                                                                              \
    do {                                                                                                   \
        if (acc_mode == PRNU_ACC_F64) dwt_inv_mle<TP, T_, PRNU_ACC_F64, U><<<grid, inv_nt(T_), 0, s>>>(a, f); \
        else if (acc_mode == PRNU_ACC_KAHAN_F32)                                                           \
            dwt_inv_mle<TP, T_, PRNU_ACC_KAHAN_F32, U><<<grid, inv_nt(T_), 0, s>>>(a, f);                  \
        else dwt_inv_mle<TP, T_, PRNU_ACC_F32, U><<<grid, inv_nt(T_), 0, s>>>(a, f);                       \
    } while (0)
#define PRNU_MLE(TP, T_)                        \
    do {                                        \
        if (means8) PRNU_MLE_U(TP, T_, true);   \
        else PRNU_MLE_U(TP, T_, false);         \
    } while (0)
    if (taps == 16) {
        if (tt == 16) PRNU_MLE(16, 16); else PRNU_MLE(16, 32);
    } else {
        if (tt == 16) PRNU_MLE(8, 16); else PRNU_MLE(8, 32);
    }
#undef PRNU_MLE
#undef PRNU_MLE_U
    return hipGetLastError();
}

hipError_t launch_fwd_multi(int taps, int tt, const Filter &f, const FwdDesc *d, int nd, int total, int *ctr,
                            int grid, hipStream_t s) {
    if (total <= 0 || nd <= 0) return hipSuccess;
    if (taps == 16) {
        if (tt == 16) dwt_fwd_multi<16, 16><<<grid, fwd_nt(16), 0, s>>>(d, nd, total, ctr, f);
        else dwt_fwd_multi<16, 32><<<grid, fwd_nt(32), 0, s>>>(d, nd, total, ctr, f);
    } else {
        if (tt == 16) dwt_fwd_multi<8, 16><<<grid, fwd_nt(16), 0, s>>>(d, nd, total, ctr, f);
        else dwt_fwd_multi<8, 32><<<grid, fwd_nt(32), 0, s>>>(d, nd, total, ctr, f);
    }
    return hipGetLastError();
}

hipError_t launch_inv_multi(int taps, int tt, const Filter &f, const InvDesc *d, int nd, int total, int *ctr,
                            int grid, hipStream_t s) {
    if (total <= 0 || nd <= 0) return hipSuccess;
    if (taps == 16) {
        if (tt == 16) dwt_inv_multi<16, 16><<<grid, inv_nt(16), 0, s>>>(d, nd, total, ctr, f);
        else dwt_inv_multi<16, 32><<<grid, inv_nt(32), 0, s>>>(d, nd, total, ctr, f);
    } else {
        if (tt == 16) dwt_inv_multi<8, 16><<<grid, inv_nt(16), 0, s>>>(d, nd, total, ctr, f);
        else dwt_inv_multi<8, 32><<<grid, inv_nt(32), 0, s>>>(d, nd, total, ctr, f);
    }
    return hipGetLastError();
}

hipError_t launch_mle_multi(int taps, int tt, int acc_mode, const Filter &f, const MleDesc *d, int nd, int total,
                            int *ctr, int grid, hipStream_t s) {
    if (total <= 0 || nd <= 0) return hipSuccess;
#define PRNU_MM(TP, T_)                                                                                  \
    do {                                                                                                 \
        if (acc_mode == PRNU_ACC_F64)                                                                    \
            dwt_mle_multi<TP, T_, PRNU_ACC_F64><<<grid, inv_nt(T_), 0, s>>>(d, nd, total, ctr, f);               \
        else if (acc_mode == PRNU_ACC_KAHAN_F32)                                                         \
            dwt_mle_multi<TP, T_, PRNU_ACC_KAHAN_F32><<<grid, inv_nt(T_), 0, s>>>(d, nd, total, ctr, f);         \
        else                                                                                             \
            dwt_mle_multi<TP, T_, PRNU_ACC_F32><<<grid, inv_nt(T_), 0, s>>>(d, nd, total, ctr, f);               \
    } while (0)
    if (taps == 16) {
        if (tt == 16) PRNU_MM(16, 16); else PRNU_MM(16, 32);
    } else {
        if (tt == 16) PRNU_MM(8, 16); else PRNU_MM(8, 32);
    }
#undef PRNU_MM
    return hipGetLastError();
}

hipError_t launch_zero_ints(int *p, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    zero_ints<<<(n + 255) / 256, 256, 0, s>>>(p, n);
    return hipGetLastError();
}

hipError_t launch_fill_pattern(float *x, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    fill_pattern<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, n);
    return hipGetLastError();
}

int fwd_multi_occupancy(int taps, int tt) {
    if (taps == 16)
        return tt == 16 ? occupancy_of(dwt_fwd_multi<16, 16>, fwd_nt(16))
                        : occupancy_of(dwt_fwd_multi<16, 32>, fwd_nt(32));
    return tt == 16 ? occupancy_of(dwt_fwd_multi<8, 16>, fwd_nt(16)) : occupancy_of(dwt_fwd_multi<8, 32>, fwd_nt(32));
}
int inv_multi_occupancy(int taps, int tt) {
    if (taps == 16)
        return tt == 16 ? occupancy_of(dwt_inv_multi<16, 16>, inv_nt(16))
                        : occupancy_of(dwt_inv_multi<16, 32>, inv_nt(32));
    return tt == 16 ? occupancy_of(dwt_inv_multi<8, 16>, inv_nt(16)) : occupancy_of(dwt_inv_multi<8, 32>, inv_nt(32));
}
int mle_multi_occupancy(int taps, int tt, int acc_mode) {
#define PRNU_OCC(TP, T_)                                                                              \
    return acc_mode == PRNU_ACC_F64 ? occupancy_of(dwt_mle_multi<TP, T_, PRNU_ACC_F64>, inv_nt(T_))          \
           : acc_mode == PRNU_ACC_KAHAN_F32 ? occupancy_of(dwt_mle_multi<TP, T_, PRNU_ACC_KAHAN_F32>, inv_nt(T_)) \
                                            : occupancy_of(dwt_mle_multi<TP, T_, PRNU_ACC_F32>, inv_nt(T_))
    if (taps == 16) {
        if (tt == 16) PRNU_OCC(16, 16);
        PRNU_OCC(16, 32);
    }
    if (tt == 16) PRNU_OCC(8, 16);
    PRNU_OCC(8, 32);
#undef PRNU_OCC
}

}  // namespace prnu
