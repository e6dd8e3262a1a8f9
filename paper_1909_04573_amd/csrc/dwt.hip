// Wavelet denoiser levels for gfx950: the residual W = I - F(I) of Sec. II-A
// with F the locally adaptive wavelet denoiser named in Sec. IV.
//
// Forward level (analysis + Wiener shrinkage, one launch per level):
//   a workgroup owns a strip of TC = 64 (or 32) subband columns of one plane
//   and walks down a segment of its rows, 16 coefficient rows per step.  Per
//   step it stages 32 new input rows in LDS (periodic wrap, plus symmetric
//   padding at level 1), filters them along the rows into a ring of
//   row-filtered rows (the last TAPS - 2 rows carry over to the next step),
//   filters the ring along the columns into 16 new coefficient rows of the
//   four subbands over the strip and a 4-column Wiener margin each side, and
//   advances the Wiener window sums of every detail column, held in
//   registers across steps:
//       var = min_{w=3,5,7,9} max(0, box_w(c^2)/w^2 - s2)
//       r   = c * s2 / (var + s2)
//   It writes the approximation (input of the next level) and the residual
//   detail coefficients r; the shrunk coefficients never touch HBM.  Along
//   the streamed direction nothing is filtered twice: the halo is paid once
//   per segment, not once per tile.  Level 1 reads float planes or, at SDA
//   depth 1, one channel of the u8 frames themselves.
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
// Inverse levels with 32 x 32 tiles run 512 threads per workgroup.
constexpr int INV_NT32 = 512;
constexpr int inv_nt(int tt) { return tt == 32 ? INV_NT32 : NT; }

template <int TAPS, int TT>
struct InvGeom {
    static constexpr int NK = TT + TAPS / 2 - 1;  // coefficients per side
    // odd row stride: the row pass's lanes read every other column of two
    // consecutive rows, which then fall in banks of opposite parity
    static constexpr int NKS = NK | 1;
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
// Forward level, streamed by strips.  A workgroup owns a strip of TC subband
// columns of one plane and walks down a segment of its rows, SR coefficient
// rows per step.  Per step it
//   P  stores the 2 SR input rows it prefetched into registers to LDS,
//   R  filters them along the rows (low and high pass, NC = TC + 2 HALO
//      coefficient columns: the strip and its Wiener margins) into a ring of
//      row-filtered rows, and issues the next step's input loads,
//   C  filters the ring along the columns: SR new coefficient rows of the four
//      subbands; the approximation goes straight to HBM, the squares of the
//      three detail bands (zero outside the band) and the strip's detail
//      coefficients to LDS,
//   W  advances each detail column's Wiener window sums by SR rows: one thread
//      per (band, strip column) keeps the horizontal 3/5/7/9 sums of the last
//      rows and their pair sums in registers across steps and shrinks the
//      coefficient four rows behind the newest square row; meanwhile the
//      remaining threads move the last TAPS - 2 ring rows to the ring's start
//      for the next step's column pass.
// Nothing is filtered twice along the streamed direction: the vertical halo
// is paid once per segment instead of once per tile.
constexpr int SR = 16;  // coefficient rows per step; also the period of the Wiener register ring (>= 9)

// High-pass tap j as the quadrature mirror of the low-pass, g[j] =
// (-1)^j h[TAPS-1-j] (exactly the host's g): the sign becomes a source
// modifier of the FMA, so only the TAPS low-pass taps occupy scalar registers.
template <int TAPS>
__device__ __forceinline__ float qmf_g(const Filter &f, int j) {
    return (j & 1) ? -f.h[TAPS - 1 - j] : f.h[TAPS - 1 - j];
}

template <int TAPS, int TC>
struct StripGeom {
    static constexpr int NTH = 4 * TC;             // threads: 3 TC Wiener columns + TC helpers
    static constexpr int NW = 3 * TC;              // Wiener threads
    static constexpr int NEW = 2 * SR;             // input rows staged per step
    static constexpr int CARRY = TAPS - 2;         // row-filtered rows the next step's column pass reuses
    static constexpr int RR = NEW + CARRY;         // rows of the row-filtered ring
    static constexpr int NC = TC + 2 * HALO;       // coefficient columns incl. the Wiener margins
    static constexpr int NP = NC / 2;              // column pairs
    static constexpr int INC = 2 * NC + TAPS - 2;  // input columns
    static constexpr int INCQ = (INC + 3) / 4 * 4; // input columns read (whole 16-byte quads)
    // LDS row stride of the staged input: 4 (mod 32) floats, so the row pass's
    // 16-byte reads by consecutive rows fall in distinct banks
    static constexpr int INCS = (INCQ + 27) / 32 * 32 + 4;
    static constexpr int NQ4 = INCQ / 4;
    static constexpr int RING = 2 * RR * NC;       // [row band lo, hi][RR][NC]
    static constexpr int QF = 3 * SR * NC;         // squares [3][SR][NC]
    static constexpr int CF = 3 * SR * TC;         // strip coefficients [3][SR][TC]
    static constexpr int SF = NEW * INCS;          // staged input [NEW][INCS]
    // the staged input and the squares + coefficients share one area: the row
    // pass has read the input before the column pass writes the squares
    static constexpr int AREA = QF + CF > SF ? QF + CF : SF;
    static constexpr int LDS = RING + AREA + 2 * NEW + INCS;  // floats, then two row maps and the column map
    static_assert(INCQ >= INC + 2 && INCS >= INCQ && INCS % 32 == 4, "staged row layout");
    static_assert(NC % 4 == 0 && RING % 4 == 0 && QF % 4 == 0 && AREA % 4 == 0, "16-byte aligned LDS areas");
    static_assert(NTH - NW >= 32, "helper threads for the ring move");
    static_assert((SR & (SR - 1)) == 0, "SR a power of two");
};

// Strips per plane, segment rows and virtual blocks of a forward level of
// hk x wk coefficients with strips of tc columns over `planes` planes: long
// segments keep the vertical halo small, short ones keep enough workgroups
// (about six per CU per launch) to fill the chip and shorten its tail.
__host__ __device__ inline void strip_layout(int tc, int hk, int wk, int64_t planes, int cus, int per_cu,
                                             int *strips, int *seg, int *tiles) {
    const int ns = (wk + tc - 1) / tc;
    const int64_t base = (int64_t)ns * (planes > 0 ? planes : 1);
    const int64_t want = (int64_t)per_cu * (cus > 0 ? cus : 256);
    int64_t nseg = (want + base - 1) / base;
    // segments of at least 16 rows: the small levels (68 and 136 rows at
    // 1080p) need several to give the chip enough workgroups
    const int max_seg = hk / 16 > 1 ? hk / 16 : 1;
    if (nseg > max_seg) nseg = max_seg;
    if (nseg < (hk + 503) / 504) nseg = (hk + 503) / 504;  // and at most about 500
    int S = (int)((hk + nseg - 1) / nseg);
    S = ((S + 2 * HALO + SR - 1) / SR) * SR - 2 * HALO;  // whole steps: S + 2 HALO rows computed
    if (S < 1) S = 1;
    *strips = ns;
    *seg = S;
    *tiles = ns * ((hk + S - 1) / S);
}

__device__ __forceinline__ float4 ld4(const PRNU_GLOBAL float *p) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    const v4 t = *(const PRNU_GLOBAL v4 *)p;
    return make_float4(t.x, t.y, t.z, t.w);
}

// Staging modes of a strip's input rows (uniform per strip): float planes
// whose strip needs neither the periodic wrap nor the reflection in its
// columns are read as 16-byte quads; other float planes and u8 frames one
// sample per load through the column map.
enum StageMode { ST_QUAD = 0, ST_F32 = 1, ST_U8 = 2 };

// Staging of NR input rows of a strip: fetch() issues the global loads into
// registers, put() stores them to the LDS rows.  Quads: slot e = row-major
// quad index; samples: threads form 32 columns x NTH/32 rows (u8 frames: one
// channel of interleaved frames, kept as bytes until put(), exact in float).
// Neither branches on the slot: slots past the end repeat the last valid one
// (the same value lands in the same LDS word twice), so every thread issues
// the same loads and the compiler can count the memory operations in flight.
template <int TAPS, int TC, int NR, int MODE>
struct StripStage {
    using G = StripGeom<TAPS, TC>;
    static constexpr int NTH = G::NTH, INC = G::INC, INCS = G::INCS, NQ4 = G::NQ4;
    static constexpr int NVF = (NR * NQ4 + NTH - 1) / NTH;
    static constexpr int CX = 32, RY = NTH / CX;
    static constexpr int NCG = (INC + CX - 1) / CX, NRG = (NR + RY - 1) / RY;
    static constexpr int NV = MODE == ST_QUAD ? 4 * NVF : NRG * NCG;
    using V = typename std::conditional<MODE == ST_U8, unsigned, float>::type;
    V v[NV];

    static __device__ __forceinline__ int slot(int tid, int k) {
        const int e = tid + k * NTH;
        return e < NR * NQ4 ? e : NR * NQ4 - 1;
    }
    static __device__ __forceinline__ int srow(int ty, int i) {
        const int r = ty + i * RY;
        return r < NR ? r : NR - 1;
    }
    static __device__ __forceinline__ int scol(int tx, int g) {
        const int x = tx + g * CX;
        return x < INC ? x : INC - 1;
    }

    __device__ __forceinline__ void fetch(const FwdArgs &a, int plane, int tid, int c_src0, const int *rmap,
                                          const int *cmap) {
        if constexpr (MODE == ST_QUAD) {
            const PRNU_GLOBAL float *sp = gmem(a.src) + (int64_t)plane * a.src_stride + c_src0;
#pragma unroll
            for (int k = 0; k < NVF; ++k) {
                const int e = slot(tid, k);
                const int r = e / NQ4, q = e - (e / NQ4) * NQ4;
                const float4 t = ld4(sp + (unsigned)(rmap[r] + 4 * q));
                v[4 * k] = t.x;
                v[4 * k + 1] = t.y;
                v[4 * k + 2] = t.z;
                v[4 * k + 3] = t.w;
            }
        } else {
            const int tx = tid % CX, ty = tid / CX;
            int coff[NCG];
#pragma unroll
            for (int g = 0; g < NCG; ++g) coff[g] = cmap[scol(tx, g)];
            if constexpr (MODE == ST_U8) {
                const int C8 = a.src8_c;
                const PRNU_GLOBAL unsigned char *bp =
                    gmem(a.src8) + (int64_t)(plane / C8) * a.src_rows * a.src_cols * C8 + plane % C8;
#pragma unroll
                for (int g = 0; g < NCG; ++g) coff[g] *= C8;
#pragma unroll
                for (int i = 0; i < NRG; ++i) {
                    const unsigned ro = (unsigned)rmap[srow(ty, i)] * (unsigned)C8;
#pragma unroll
                    for (int g = 0; g < NCG; ++g) v[i * NCG + g] = bp[ro + (unsigned)coff[g]];
                }
            } else {
                const PRNU_GLOBAL float *sp = gmem(a.src) + (int64_t)plane * a.src_stride;
#pragma unroll
                for (int i = 0; i < NRG; ++i) {
                    const PRNU_GLOBAL float *rp = sp + (unsigned)rmap[srow(ty, i)];
#pragma unroll
                    for (int g = 0; g < NCG; ++g) v[i * NCG + g] = rp[coff[g]];
                }
            }
        }
    }
    __device__ __forceinline__ void put(float *S, int tid) const {
        if constexpr (MODE == ST_QUAD) {
#pragma unroll
            for (int k = 0; k < NVF; ++k) {
                const int e = slot(tid, k);
                const int r = e / NQ4, q = e - (e / NQ4) * NQ4;
                *reinterpret_cast<float4 *>(&S[r * INCS + 4 * q]) =
                    make_float4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
            }
        } else {
            const int tx = tid % CX, ty = tid / CX;
#pragma unroll
            for (int i = 0; i < NRG; ++i)
#pragma unroll
                for (int g = 0; g < NCG; ++g) S[srow(ty, i) * INCS + scol(tx, g)] = (float)v[i * NCG + g];
        }
    }
};

// Staging mode of the strip whose input starts at column c_src0 of the source.
__device__ __forceinline__ int strip_mode(const FwdArgs &a, int c_src0, int incq) {
    if (a.src8) return ST_U8;
    const bool quad = c_src0 >= 0 && c_src0 + incq <= a.src_cols && (c_src0 & 3) == 0 && (a.src_cols & 3) == 0 &&
                      (a.src_stride & 3) == 0 && (reinterpret_cast<uintptr_t>(a.src) & 15) == 0;
    return quad ? ST_QUAD : ST_F32;
}

// Row pass over NR staged rows: low and high pass of four consecutive
// coefficient columns of one row per item into ring rows row0 .. row0 + NR - 1.
template <int TAPS, int TC, int NR>
__device__ __forceinline__ void strip_rows(int tid, const float *S, float *ring, int row0, const Filter &f) {
    using G = StripGeom<TAPS, TC>;
    constexpr int NC = G::NC, NQ = NC / 4, NX = TAPS + 8, ITEMS = NR * NQ;
    float *rlo = ring, *rhi = ring + G::RR * NC;
#pragma unroll 1
    for (int k = 0; k < (ITEMS + G::NTH - 1) / G::NTH; ++k) {
        const int it = tid + k * G::NTH;
        if (it < ITEMS) {
            // consecutive lanes filter consecutive rows (distinct LDS banks)
            const int i = it % NR, kq = it / NR;
            const float4 *row = reinterpret_cast<const float4 *>(&S[i * G::INCS + 8 * kq]);
            float x[NX];
#pragma unroll
            for (int t = 0; t < NX / 4; ++t) {
                const float4 v = row[t];
                x[4 * t] = v.x;
                x[4 * t + 1] = v.y;
                x[4 * t + 2] = v.z;
                x[4 * t + 3] = v.w;
            }
            float rl[4], rh[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                rl[u] = 0.f;
                rh[u] = 0.f;
#pragma unroll
                for (int j = 0; j < TAPS; ++j) {
                    rl[u] = fmaf(f.h[j], x[2 * u + j], rl[u]);
                    rh[u] = fmaf(qmf_g<TAPS>(f, j), x[2 * u + j], rh[u]);
                }
            }
            *reinterpret_cast<float4 *>(&rlo[(row0 + i) * NC + 4 * kq]) = make_float4(rl[0], rl[1], rl[2], rl[3]);
            *reinterpret_cast<float4 *>(&rhi[(row0 + i) * NC + 4 * kq]) = make_float4(rh[0], rh[1], rh[2], rh[3]);
        }
    }
}

// Wiener state of one (band, strip column): horizontal window sums h of the
// last rows and the pair sums p of consecutive rows, ring index = row mod SR.
struct WienerRing {
    float h3[SR], h5[SR], h7[SR], h9[SR];
    float p3[SR], p5[SR], p7[SR], p9[SR];
    float c[SR];  // the column's coefficients, shrunk four rows later
};

// Forward level body: strip tile % tiles_c, segment tile / tiles_c of plane
// `plane`, in the LDS area `lds` (StripGeom::LDS floats).  CK: also store the
// sensitivity checkpoint (a.ckpt).
template <int TAPS, int TC, bool CK, int MODE>
__device__ __forceinline__ void fwd_strip(const FwdArgs &a, int tile, int plane, float *lds, const Filter &f) {
    using G = StripGeom<TAPS, TC>;
    constexpr int NTH = G::NTH, NC = G::NC, NP = G::NP, RR = G::RR, NEW = G::NEW, CARRY = G::CARRY;
    float *ring = lds;
    float *S = lds + G::RING;           // staged input rows ...
    float *Q = S;                       // ... later the squares [3][SR][NC]
    float *Cb = S + G::QF;              // and the strip coefficients [3][SR][TC]
    int *rmap = reinterpret_cast<int *>(lds + G::RING + G::AREA);  // [2][NEW] row offsets (elements)
    int *cmap = rmap + 2 * NEW;                                     // [INC] source columns
    const int tid = opaque_tid();
    const int hk = a.n_r >> 1, wk = a.n_c >> 1;
    const int sc = tile % a.tiles_c, sg = tile / a.tiles_c;
    const int C0 = sc * TC, R0 = sg * a.seg_rows;
    const int K0 = R0 - HALO, J0 = C0 - HALO;
    const int oend = min(R0 + a.seg_rows, hk);
    const int T = (oend - R0 + 2 * HALO + SR - 1) / SR;
    float *op = a.out + (int64_t)plane * 4 * hk * wk;
    const int64_t band = (int64_t)hk * wk;
    // Outputs go through buffer stores whose out-of-range lanes the hardware
    // drops: every thread issues the same stores each step (no branches around
    // them), so the wait for the next step's input loads counts exactly the
    // stores behind them instead of draining them.  Byte ranges: subband 0,
    // then the three detail bands (and the checkpoint's three bands).
    const unsigned ll_bytes = (unsigned)(band * 4), det_bytes = (unsigned)(3 * band * 4);
    const __amdgpu_buffer_rsrc_t ll_rs = __builtin_amdgcn_make_buffer_rsrc(op, 0, (int)ll_bytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t det_rs = __builtin_amdgcn_make_buffer_rsrc(op + band, 0, (int)det_bytes, 0x00020000);
    const __amdgpu_buffer_rsrc_t ck_rs = __builtin_amdgcn_make_buffer_rsrc(
        CK ? a.ckpt + (int64_t)plane * a.ckpt_stride : op, 0, (int)det_bytes, 0x00020000);
    const int c_src0 = 2 * J0 - a.off_c;
    auto row_of = [&](int y) { return map_index(y, a.n_r, a.off_r, a.src_rows) * a.src_cols; };

    // prologue: the first CARRY row-filtered rows go straight to the ring's
    // start, then step 0's rows are staged
    if (tid < G::INC) cmap[tid] = map_index(2 * J0 + tid, a.n_c, a.off_c, a.src_cols);
    if (tid < CARRY) rmap[NEW + tid] = row_of(2 * K0 + tid);
    __syncthreads();
    {
        StripStage<TAPS, TC, CARRY, MODE> pro;
        pro.fetch(a, plane, tid, c_src0, rmap + NEW, cmap);
        pro.put(S, tid);
    }
    if (tid < NEW) rmap[tid] = row_of(2 * K0 + CARRY + tid);
    __syncthreads();
    strip_rows<TAPS, TC, CARRY>(tid, S, ring, 0, f);
    StripStage<TAPS, TC, NEW, MODE> st;
    st.fetch(a, plane, tid, c_src0, rmap, cmap);
    __syncthreads();
    st.put(S, tid);
    if (tid < NEW) rmap[NEW + tid] = row_of(2 * K0 + 2 * SR + CARRY + tid);
    __syncthreads();

    const bool cols_in = J0 >= 0 && J0 + NC <= wk;
    // Column-pass items of this thread, the same every step: (row band b,
    // coefficient row pair kp, column pair cp) -> LDS addresses of its ring
    // reads and of its square / coefficient writes, and its approximation
    // offset relative to the step's first row.  Kept in registers.
    typedef __attribute__((address_space(3))) float lds_rw;
    typedef float v2f __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(3))) v2f lds_rw2;
    constexpr int CITEMS = 2 * NP * (SR / 2), NCI = (CITEMS + NTH - 1) / NTH;
    lds_rw *ci_rd[NCI], *ci_qh[NCI], *ci_ql[NCI], *ci_ch[NCI], *ci_cl[NCI];
    int ci_ll[NCI], ci_meta[NCI];  // meta: bit 0 valid, 1 b, 2 core column, 3 col 0 in band, 4 col 1 in band; kp << 8
#pragma unroll
    for (int k = 0; k < NCI; ++k) {
        const int it = tid + k * NTH;
        const int q8 = it / NP, cp = it - (it / NP) * NP, kp = q8 & (SR / 2 - 1), b = (q8 / (SR / 2)) & 1;
        const int gc = J0 + 2 * cp;
        const bool core_c = cp >= HALO / 2 && cp < (HALO + TC) / 2;
        ci_rd[k] = (lds_rw *)(ring + b * RR * NC + 4 * kp * NC + 2 * cp);
        ci_qh[k] = (lds_rw *)(Q + ((1 + b) * SR + 2 * kp) * NC + 2 * cp);
        ci_ql[k] = (lds_rw *)(Q + (2 * kp) * NC + 2 * cp);
        ci_ch[k] = (lds_rw *)(Cb + ((1 + b) * SR + 2 * kp) * TC + 2 * cp - HALO);
        ci_cl[k] = (lds_rw *)(Cb + (2 * kp) * TC + 2 * cp - HALO);
        ci_ll[k] = 2 * kp * wk + gc;
        ci_meta[k] = (it < CITEMS ? 1 : 0) | (b << 1) | (core_c ? 4 : 0) | (gc >= 0 && gc < wk ? 8 : 0) |
                     (gc + 1 >= 0 && gc + 1 < wk ? 16 : 0) | (kp << 8);
    }
    WienerRing wr;
#pragma unroll
    for (int i = 0; i < SR; ++i) {
        wr.h3[i] = wr.h5[i] = wr.h7[i] = wr.h9[i] = 0.f;
        wr.p3[i] = wr.p5[i] = wr.p7[i] = wr.p9[i] = 0.f;
        wr.c[i] = 0.f;
    }
    // Step t: R (row pass of the staged rows; the next step's loads issued),
    // C, W (with this step's stores), then P: the next step's rows to LDS.
    // The last step fetches and stages one more step of rows it does not
    // use (valid rows): the loads stay unconditional.
    for (int t = 0; t < T; ++t) {
        strip_rows<TAPS, TC, NEW>(tid, S, ring, CARRY, f);
        st.fetch(a, plane, tid, c_src0, rmap + ((t + 1) & 1) * NEW, cmap);
        __syncthreads();
        // C: column pass, coefficient rows kb .. kb + SR - 1
        const int kb = K0 + SR * t;
        const int kbwk = kb * wk;
        const bool inside = cols_in && kb >= 0 && kb + SR <= hk;
        auto cols = [&](auto masked) {
#pragma unroll
            for (int k = 0; k < NCI; ++k) {
                __builtin_amdgcn_sched_barrier(0);  // one item at a time: registers
                const int meta = ci_meta[k];
                if (!(meta & 1)) continue;
                const int b = (meta >> 1) & 1, kp = meta >> 8;
                const bool core_c = (meta & 4) != 0;
                const bool cv0 = !masked || (meta & 8), cv1 = !masked || (meta & 16);
                const lds_rw *rb = ci_rd[k];
                float2 xv[TAPS + 2];
#pragma unroll
                for (int u = 0; u < TAPS + 2; ++u) {
                    const v2f t2 = *(const lds_rw2 *)(&rb[u * NC]);
                    xv[u] = make_float2(t2.x, t2.y);
                }
                // approximation (row low-pass items, strip columns, the segment's rows) to HBM
                const bool llc = b == 0 && a.write_ll && core_c;
                const unsigned ll0 = llc ? (unsigned)(kbwk + ci_ll[k]) * 4u : ll_bytes;
                // the high-pass output goes to band 1 (hl) from row low-pass items, band 2 (hh)
                // from row high-pass ones; the low-pass output of row high-pass items to band 0 (lh)
                lds_rw *qh = ci_qh[k], *ql = ci_ql[k], *ch = ci_ch[k], *cl = ci_cl[k];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    float l0 = 0.f, l1 = 0.f, h0 = 0.f, h1 = 0.f;
#pragma unroll
                    for (int j = 0; j < TAPS; ++j) {
                        const float2 v = xv[2 * u + j];
                        l0 = fmaf(f.h[j], v.x, l0);
                        l1 = fmaf(f.h[j], v.y, l1);
                        h0 = fmaf(qmf_g<TAPS>(f, j), v.x, h0);
                        h1 = fmaf(qmf_g<TAPS>(f, j), v.y, h1);
                    }
                    const int kr = kb + 2 * kp + u;
                    const bool rv = !masked || (kr >= 0 && kr < hk);
                    auto sq = [&](float c0, float c1) {
                        v2f q2 = v2f{c0 * c0, c1 * c1};
                        if (masked) q2 = v2f{rv && cv0 ? q2.x : 0.f, rv && cv1 ? q2.y : 0.f};
                        return q2;
                    };
                    const bool llr = kr >= R0 && kr < oend;
                    const unsigned lo = ll0 + (unsigned)u * (unsigned)wk * 4u;
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(l0), ll_rs, llr && cv0 ? lo : ll_bytes, 0, 0);
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(l1), ll_rs, llr && cv1 ? lo + 4u : ll_bytes,
                                                          0, 0);
                    *(lds_rw2 *)(&qh[u * NC]) = sq(h0, h1);
                    if (core_c) *(lds_rw2 *)(&ch[u * TC]) = v2f{h0, h1};
                    if (b == 1) {
                        *(lds_rw2 *)(&ql[u * NC]) = sq(l0, l1);
                        if (core_c) *(lds_rw2 *)(&cl[u * TC]) = v2f{l0, l1};
                    }
                }
            }
        };
        if (inside)
            cols(std::false_type{});
        else
            cols(std::true_type{});
        __syncthreads();
        // W: Wiener shrinkage of the strip's detail columns, four rows behind
        float res[SR], sen[CK ? SR : 1];
        const int ob = R0 + SR * t - 2 * HALO;  // output row of the step's row i is ob + i (from row R0 on)
        // byte offset of output row ob of this thread's column in the detail
        // bands; out of range for helper threads and columns past the band
        unsigned obase = det_bytes;
        if (tid < G::NW) {
            const int s = tid / TC, jc = tid - (tid / TC) * TC;
            // the column's LDS addresses as opaque registers: every load is
            // then that register plus an immediate offset (the compiler would
            // otherwise rebuild the area's base address for each pair of loads)
            typedef __attribute__((address_space(3))) const float lds_f32;
            lds_f32 *Qs = (lds_f32 *)(Q + s * SR * NC + jc);
            lds_f32 *Cs = (lds_f32 *)(Cb + s * SR * TC + jc);
            asm volatile("" : "+v"(Qs), "+v"(Cs));
            const float s2 = a.s2;
            const bool col_ok = C0 + jc < wk;
            if (col_ok) obase = (unsigned)((int64_t)s * band + (int64_t)ob * wk + C0 + jc) * 4u;
#pragma unroll
            for (int i = 0; i < SR; ++i) {
                float q[9];
#pragma unroll
                for (int dx = 0; dx < 9; ++dx) q[dx] = Qs[i * NC + dx];
                const float a3 = q[3] + q[4] + q[5];
                const float a5 = a3 + q[2] + q[6];
                const float a7 = a5 + q[1] + q[7];
                const float a9 = a7 + q[0] + q[8];
                const int ip = (i + SR - 1) % SR;
                wr.p3[i] = wr.h3[ip] + a3;
                wr.p5[i] = wr.h5[ip] + a5;
                wr.p7[i] = wr.h7[ip] + a7;
                wr.p9[i] = wr.h9[ip] + a9;
                wr.h3[i] = a3;
                wr.h5[i] = a5;
                wr.h7[i] = a7;
                wr.h9[i] = a9;
                wr.c[i] = Cs[i * TC];
                // output ring row o = i - 4: window rows o-r .. o+r as pairs
                constexpr int M = SR;
                const int o = (i + M - 4) % M;
                const float v3 = wr.p3[o] + wr.h3[(o + 1) % M];
                const float v5 = wr.p5[(o + M - 1) % M] + wr.p5[(o + 1) % M] + wr.h5[(o + 2) % M];
                const float v7 = wr.p7[(o + M - 2) % M] + wr.p7[o] + wr.p7[(o + 2) % M] + wr.h7[(o + 3) % M];
                const float v9 = wr.p9[(o + M - 3) % M] + wr.p9[(o + M - 1) % M] + wr.p9[(o + 1) % M] +
                                 wr.p9[(o + 3) % M] + wr.h9[i];
                float m = fminf(v3 * (1.f / 9.f), v5 * (1.f / 25.f));
                m = fminf(m, v7 * (1.f / 49.f));
                m = fminf(m, v9 * (1.f / 81.f));
                const float den = fmaxf(s2, m);
                const float rcp = __builtin_amdgcn_rcpf(den);
                const float c = wr.c[o];
                res[i] = c * (den > 0.f ? s2 * rcp : 0.f);
                // sensitivity dr/ds = c / m where the window mean m exceeds s2, else 0
                if (CK) sen[CK ? i : 0] = den > s2 ? c * rcp : 0.f;
            }
        } else {
#pragma unroll
            for (int i = 0; i < SR; ++i) {
                res[i] = 0.f;
                if (CK) sen[CK ? i : 0] = 0.f;
            }
            // the last CARRY ring rows become the first ones of the next step
            constexpr int N4 = CARRY * NC / 4;
            for (int e = tid - G::NW; e < 2 * N4; e += NTH - G::NW) {
                const int b = e / N4, r4 = e - (e / N4) * N4;
                float *base = ring + b * RR * NC;
                *reinterpret_cast<float4 *>(&base[4 * r4]) = *reinterpret_cast<const float4 *>(&base[NEW * NC + 4 * r4]);
            }
        }
        const unsigned row_bytes = (unsigned)wk * 4u;
#pragma unroll
        for (int i = 0; i < SR; ++i) {
            // rows before the segment's first output row or past its end (uniform)
            const bool rok = (t > 0 || i >= 2 * HALO) && ob + i < oend;
            const unsigned o = rok ? obase + (unsigned)i * row_bytes : det_bytes;
            __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(res[i]), det_rs, o, 0, 0);
            if (CK) __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(sen[CK ? i : 0]), ck_rs, o, 0, 0);
        }
        __syncthreads();
        // P: the next step's rows to LDS (over the squares); row offsets of the step after
        st.put(S, tid);
        if (tid < NEW) rmap[(t & 1) * NEW + tid] = row_of(2 * K0 + 2 * SR * (t + 2) + CARRY + tid);
        __syncthreads();
    }
}

// Forward level body: picks the staging mode of the strip (uniform across
// the workgroup) and runs the strip.
template <int TAPS, int TC, bool CK>
__device__ __forceinline__ void fwd_body(const FwdArgs &a, int tile, int plane, float *lds, const Filter &f) {
    const int C0 = (tile % a.tiles_c) * TC;
    const int mode = strip_mode(a, 2 * (C0 - HALO) - a.off_c, StripGeom<TAPS, TC>::INCQ);
    if (mode == ST_QUAD)
        fwd_strip<TAPS, TC, CK, ST_QUAD>(a, tile, plane, lds, f);
    else if (mode == ST_U8)
        fwd_strip<TAPS, TC, CK, ST_U8>(a, tile, plane, lds, f);
    else
        fwd_strip<TAPS, TC, CK, ST_F32>(a, tile, plane, lds, f);
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
// as zeros with zero_approx).  Thread t takes elements t, t + threads, ...
// of the NK x NK window in row-major order (the last slots repeat the last
// element): consecutive lanes read consecutive columns of a row, and write
// consecutive LDS words (the row stride NKS equals NK for odd NK).  The
// element offsets in a subband plane and in LDS depend only on the tile, so
// offsets() computes them once; every plane's fetch is then one load per
// element and subband.  fetch() issues a plane's loads into registers, put()
// stores them to LDS, so a caller can have the next plane's loads in flight
// while it works on the current one.  Neither branches, so the compiler can
// count the loads in flight and wait only for the ones a put needs.
template <int TAPS, int TT>
struct InvStage {
    static constexpr int NK = InvGeom<TAPS, TT>::NK, NKS = InvGeom<TAPS, TT>::NKS;
    static constexpr int NTH = inv_nt(TT), PER = (NK * NK + NTH - 1) / NTH;
    unsigned goff[PER];  // element offset within a subband plane
    int loff[PER];       // LDS offset within subband 0's rows
    float v[4][PER];
    bool za;             // approximation band read as zero

    // rmap/cmap must be in LDS (after the barrier that follows inv_maps)
    __device__ __forceinline__ void offsets(int tid, int wk, const int *rmap, const int *cmap) {
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int e = min(tid + k * NTH, NK * NK - 1);
            const int r = e / NK, c = e - (e / NK) * NK;
            goff[k] = (unsigned)(rmap[r] * wk + cmap[c]);
            loff[k] = r * NKS + c;
        }
    }
    // The zeroed approximation band is applied by put(): a select on a
    // loaded value right after fetch() would wait for that load.
    __device__ __forceinline__ void fetch(const float *__restrict__ lpp, int64_t band, bool zero_approx) {
        const PRNU_GLOBAL float *lp = gmem(lpp);
#pragma unroll
        for (int sbd = 0; sbd < 4; ++sbd)
#pragma unroll
            for (int k = 0; k < PER; ++k) v[sbd][k] = lp[sbd * band + goff[k]];
        za = zero_approx;
    }
    // fetch() as buffer loads: one descriptor per subband in scalar registers
    // and 32-bit byte offsets, for subbands of fewer than 2^29 coefficients
    __device__ __forceinline__ void fetch_buf(const float *lpp, int64_t band, bool zero_approx) {
#pragma unroll
        for (int sbd = 0; sbd < 4; ++sbd) {
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<float *>(lpp + sbd * band), 0, (int)(band * 4), 0x00020000);
#pragma unroll
            for (int k = 0; k < PER; ++k)
                v[sbd][k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, goff[k] * 4u, 0, 0));
        }
        za = zero_approx;
    }
    __device__ __forceinline__ void put(float *sb) const {
#pragma unroll
        for (int sbd = 0; sbd < 4; ++sbd)
#pragma unroll
            for (int k = 0; k < PER; ++k) sb[sbd * NK * NKS + loff[k]] = sbd == 0 && za ? 0.f : v[sbd][k];
    }
};

// Columns (axis 0): lo1/hi1[n][kc] for the 2TT output rows.
//
// Piece (kc, pp, half, v) of the column pass: output rows 4pp + 2v and
// 4pp + 2v + 1 of column kc of lo1 (half 0: from a and hl) or hi1 (half 1:
// from lh and hh), from coefficient rows 2pp + v .. 2pp + v + HT - 1.
template <int TAPS, int TT>
__device__ __forceinline__ void inv_col_piece(const float *sb, float *lo1, float *hi1, const Filter &f, int kc,
                                              int pp, int half, int v) {
    constexpr int NK = InvGeom<TAPS, TT>::NK, NKS = InvGeom<TAPS, TT>::NKS, HT = TAPS / 2;
    const int s0 = half == 0 ? 0 : 1, s1 = half == 0 ? 2 : 3;
    float p[HT], q[HT];
#pragma unroll
    for (int t = 0; t < HT; ++t) {
        const int kr = 2 * pp + v + t;
        p[t] = sb[(s0 * NK + kr) * NKS + kc];
        q[t] = sb[(s1 * NK + kr) * NKS + kc];
    }
    float *dst = half == 0 ? lo1 : hi1;
#pragma unroll
    for (int par = 0; par < 2; ++par) {
        float acc = 0.f;
#pragma unroll
        for (int i = 0; i < HT; ++i) {
            const int t = HT - 1 - i;
            acc = fmaf(f.h[2 * i + par], p[t], fmaf(f.g[2 * i + par], q[t], acc));
        }
        dst[(4 * pp + 2 * v + par) * NKS + kc] = acc;
    }
}

// Items (column kc, output row quad pp): the first rounds give every thread
// whole items (both halves and both row pairs share their loads); the
// remainder, fewer than the threads, is cut into quarter items (half, v) so
// that no wave reaches the next barrier with a whole extra item.  Every
// output sums the same products in the same order either way.
template <int TAPS, int TT>
__device__ __forceinline__ void inv_cols(int tid, const float *sb, float *lo1, float *hi1, const Filter &f) {
    constexpr int NK = InvGeom<TAPS, TT>::NK, NKS = InvGeom<TAPS, TT>::NKS, HT = TAPS / 2, NTH = inv_nt(TT);
    constexpr int ITEMS = NK * (TT / 2), FULL = ITEMS / NTH * NTH, REST = ITEMS - FULL;
    for (int it = tid; it < FULL; it += NTH) {
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
    // quarter e: item FULL + e % REST (consecutive lanes, consecutive items), piece e / REST
    for (int e = tid; e < 4 * REST; e += NTH) {
        const int qtr = e / REST, it = FULL + (e - qtr * REST);
        const int pp = it / NK, kc = it - (it / NK) * NK;
        inv_col_piece<TAPS, TT>(sb, lo1, hi1, f, kc, pp, qtr >> 1, qtr & 1);
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
// (planes [nb][C], means [nb][C][H][W]).  The intensities I of frame fr + 1
// are loaded with its subbands, one frame ahead; they and the accumulators
// go through buffer loads and stores whose out-of-image offsets read 0 and
// write nothing, so no load sits behind a per-pixel branch (a pixel outside
// the image adds W * 0 to its partial sums, which leaves them unchanged).
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
    // byte offset of each owned pixel within one intensity plane (a frame's
    // channel c for U8I), or the plane's size where the pixel lies outside
    const unsigned esz = U8I ? (unsigned)C : 4u;
    const unsigned plane_bytes = U8I ? (unsigned)(npx * C - c) : (unsigned)(npx * 4);
    unsigned ioff[ITEMS][4];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int it = tid + k * inv_nt(TT);
        const int n = it / (NO / 4), mq = it - (it / (NO / 4)) * (NO / 4);
        const int y = 2 * k0r + n - a.off_r;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int xx = 2 * k0c + 4 * mq + u - a.off_c;
            ioff[k][u] = (y >= 0 && y < H && xx >= 0 && xx < W) ? (unsigned)(y * W + xx) * esz : plane_bytes;
        }
    }
    auto i_rsrc = [&](int fr) {
        const void *base = U8I ? (const void *)(a.means8 + (int64_t)fr * npx * C + c)
                               : (const void *)(a.means + (int64_t)(fr * C + c) * npx);
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)plane_bytes, 0x00020000);
    };
    // u8 intensities stay integers: I^2 is then summed exactly in 32 bits
    using IT = typename std::conditional<U8I, unsigned, float>::type;
    auto load_i = [&](int fr, IT (&Iv)[ITEMS][4]) {
        const __amdgpu_buffer_rsrc_t rs = i_rsrc(fr);
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if constexpr (U8I)
                    Iv[k][u] = __builtin_amdgcn_raw_buffer_load_b8(rs, ioff[k][u], 0, 0);
                else
                    Iv[k][u] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, ioff[k][u], 0, 0));
            }
    };
    double sa[ITEMS][4], sbb[ITEMS][4];  // ACC_F64 partials
    float ka[ITEMS][4], kc_[ITEMS][4];   // float partial of A (+ compensation for KAHAN)
    float kb[ITEMS][4], kbc[ITEMS][4];   // ... and of B
    // u8 intensities: sum I^2 of the batch as an integer.  With at most 32
    // frames it stays below 2^24, so every accumulator mode's sum of these
    // exact squares equals it exactly (the compensation stays 0).
    unsigned iq[ITEMS][4];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            sa[k][u] = 0.0;
            sbb[k][u] = 0.0;
            ka[k][u] = kc_[k][u] = kb[k][u] = kbc[k][u] = 0.f;
            iq[k][u] = 0u;
        }
    // subband loads and intensities of frame fr + 1 are in flight while frame fr is transformed
    __syncthreads();  // maps ready
    InvStage<TAPS, TT> st;
    st.offsets(tid, a.wk, rmap, cmap);
    const int64_t band = (int64_t)a.hk * a.wk;
    // the fold's frames are below 2^28 pixels: 32-bit offsets reach every subband
    st.fetch_buf(a.lvl + (int64_t)c * 4 * band, band, a.zero_approx != 0);
    IT In[ITEMS][4];
    load_i(0, In);
    for (int fr = 0; fr < a.nb; ++fr) {
        IT Iv[ITEMS][4];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
#pragma unroll
            for (int u = 0; u < 4; ++u) Iv[k][u] = In[k][u];
        // The previous frame's column pass finished reading sb before the
        // barrier that precedes its row pass, and this frame's column pass
        // writes lo1/hi1 only after the next barrier, which every thread
        // reaches after its row pass: one barrier per hand-over suffices.
        st.put(sb);
        __syncthreads();
        if (fr + 1 < a.nb) {
            st.fetch_buf(a.lvl + (int64_t)((fr + 1) * C + c) * 4 * band, band, a.zero_approx != 0);
            load_i(fr + 1, In);
        }
        const int tf = opaque_tid();  // index arithmetic per frame, not live across the frame loop
        inv_cols<TAPS, TT>(tf, sb, lo1, hi1, f);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int it = tid + k * inv_nt(TT);
            const int n = it / (NO / 4), mq = it - (it / (NO / 4)) * (NO / 4);
            float x[4];
            inv_row_quad<TAPS, TT>(lo1, hi1, n, mq, f, x);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (U8I) iq[k][u] += Iv[k][u] * Iv[k][u];  // at most 255^2 a frame, 24-bit products
                if (ACC == PRNU_ACC_KAHAN_F32) {
                    // two-sum accumulation of W*I and I*I
                    const float I = (float)Iv[k][u];
                    const float pa = x[u] * I;
                    float t = ka[k][u] + pa;
                    float z = t - ka[k][u];
                    kc_[k][u] += (ka[k][u] - (t - z)) + (pa - z);
                    ka[k][u] = t;
                    if (!U8I) {
                        const float pb = I * I;
                        t = kb[k][u] + pb;
                        z = t - kb[k][u];
                        kbc[k][u] += (kb[k][u] - (t - z)) + (pb - z);
                        kb[k][u] = t;
                    }
                } else if (ACC == PRNU_ACC_F32) {
                    const float I = (float)Iv[k][u];
                    ka[k][u] = fmaf(x[u], I, ka[k][u]);
                    if (!U8I) kb[k][u] = fmaf(I, I, kb[k][u]);
                } else {
                    const double I = (double)Iv[k][u];
                    sa[k][u] = fma((double)x[u], I, sa[k][u]);
                    if (!U8I) sbb[k][u] = fma(I, I, sbb[k][u]);
                }
            }
        }
    }
    if constexpr (U8I) {
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                sbb[k][u] = (double)iq[k][u];
                kb[k][u] = (float)iq[k][u];
            }
    }
    // one read-modify-write of the accumulators per pixel: every load first,
    // then the sums, then the stores (out-of-image offsets read 0, store nothing)
    const unsigned ab = (unsigned)(npx * (ACC == PRNU_ACC_F64 ? 8 : 4));
    unsigned aoff[ITEMS][4];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
#pragma unroll
        for (int u = 0; u < 4; ++u)
            aoff[k][u] = ioff[k][u] == plane_bytes ? ab : ioff[k][u] / esz * (ACC == PRNU_ACC_F64 ? 8u : 4u);
    if constexpr (ACC == PRNU_ACC_F64) {
        const __amdgpu_buffer_rsrc_t ra =
            __builtin_amdgcn_make_buffer_rsrc(static_cast<double *>(a.A) + (int64_t)c * npx, 0, (int)ab, 0x00020000);
        const __amdgpu_buffer_rsrc_t rb =
            __builtin_amdgcn_make_buffer_rsrc(static_cast<double *>(a.B) + (int64_t)c * npx, 0, (int)ab, 0x00020000);
        double va[ITEMS][4], vb[ITEMS][4];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const auto la = __builtin_amdgcn_raw_buffer_load_b64(ra, aoff[k][u], 0, 0);
                const auto lb = __builtin_amdgcn_raw_buffer_load_b64(rb, aoff[k][u], 0, 0);
                __builtin_memcpy(&va[k][u], &la, 8);
                __builtin_memcpy(&vb[k][u], &lb, 8);
            }
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double na = va[k][u] + sa[k][u], nb = vb[k][u] + sbb[k][u];
                decltype(__builtin_amdgcn_raw_buffer_load_b64(ra, 0, 0, 0)) wa, wb;
                __builtin_memcpy(&wa, &na, 8);
                __builtin_memcpy(&wb, &nb, 8);
                __builtin_amdgcn_raw_buffer_store_b64(wa, ra, aoff[k][u], 0, 0);
                __builtin_amdgcn_raw_buffer_store_b64(wb, rb, aoff[k][u], 0, 0);
            }
    } else {
        // F32: A, B planes; KAHAN: value plane [0] then compensation plane [1] of each
        const int64_t cs = (int64_t)C * npx;
        float *A0 = static_cast<float *>(a.A) + (int64_t)c * npx, *B0 = static_cast<float *>(a.B) + (int64_t)c * npx;
        const __amdgpu_buffer_rsrc_t ra = __builtin_amdgcn_make_buffer_rsrc(A0, 0, (int)ab, 0x00020000);
        const __amdgpu_buffer_rsrc_t rb = __builtin_amdgcn_make_buffer_rsrc(B0, 0, (int)ab, 0x00020000);
        const __amdgpu_buffer_rsrc_t rac = __builtin_amdgcn_make_buffer_rsrc(A0 + cs, 0, (int)ab, 0x00020000);
        const __amdgpu_buffer_rsrc_t rbc = __builtin_amdgcn_make_buffer_rsrc(B0 + cs, 0, (int)ab, 0x00020000);
        float va[ITEMS][4], vb[ITEMS][4], vac[ITEMS][4], vbc[ITEMS][4];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                va[k][u] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(ra, aoff[k][u], 0, 0));
                vb[k][u] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rb, aoff[k][u], 0, 0));
                if (ACC == PRNU_ACC_KAHAN_F32) {
                    vac[k][u] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rac, aoff[k][u], 0, 0));
                    vbc[k][u] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rbc, aoff[k][u], 0, 0));
                }
            }
#pragma unroll
        for (int k = 0; k < ITEMS; ++k)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const unsigned o = aoff[k][u];
                if (ACC == PRNU_ACC_F32) {
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(va[k][u] + ka[k][u]), ra, o, 0, 0);
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(vb[k][u] + kb[k][u]), rb, o, 0, 0);
                } else {
                    float s = va[k][u], t = s + ka[k][u], z = t - s;
                    __builtin_amdgcn_raw_buffer_store_b32(
                        __float_as_uint(vac[k][u] + (kc_[k][u] + ((s - (t - z)) + (ka[k][u] - z)))), rac, o, 0, 0);
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(t), ra, o, 0, 0);
                    s = vb[k][u];
                    t = s + kb[k][u];
                    z = t - s;
                    __builtin_amdgcn_raw_buffer_store_b32(
                        __float_as_uint(vbc[k][u] + (kbc[k][u] + ((s - (t - z)) + (kb[k][u] - z)))), rbc, o, 0, 0);
                    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(t), rb, o, 0, 0);
                }
            }
    }
}

// ---------------------------------------------------------------------------
// Per-plane kernels.
template <int TAPS, int TC, bool CK>
__global__ __launch_bounds__(4 * TC) __attribute__((amdgpu_waves_per_eu(3))) void dwt_fwd_wiener(FwdArgs a,
                                                                                                Filter f) {
    __shared__ __align__(16) float lds[StripGeom<TAPS, TC>::LDS];
    int tile, plane;
    if (a.src8 && a.src8_c > 1)
        grid_tile_channels(tile, plane, a.src8_c);
    else
        grid_tile(tile, plane);
    fwd_body<TAPS, TC, CK>(a, tile, plane, lds, f);
}

template <int TAPS, int TT, int EPI>
__global__ __launch_bounds__(inv_nt(TT)) void dwt_inv(InvArgs a, Filter f) {
    __shared__ __align__(16) float lds[InvGeom<TAPS, TT>::LDS];
    int tile, plane;
    grid_tile(tile, plane);
    inv_body<TAPS, TT, EPI>(a, tile, plane, lds, f);
}

template <int TAPS, int TT, int ACC, bool U8I>
__global__ __launch_bounds__(inv_nt(TT)) __attribute__((amdgpu_waves_per_eu(4))) void dwt_inv_mle(MleArgs a, Filter f) {
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

template <int TAPS, int TC>
__global__ __launch_bounds__(4 * TC) __attribute__((amdgpu_waves_per_eu(3))) void dwt_fwd_multi(const FwdDesc *__restrict__ d, int nd,
                                                                        int total, int *ctr, Filter f) {
    __shared__ __align__(16) float lds[StripGeom<TAPS, TC>::LDS];
    __shared__ int slot;
    for (;;) {
        const int vb = next_block(ctr, &slot);
        if (vb >= total) break;
        const FwdDesc &D = d[find_desc(d, nd, vb)];
        const int local = vb - (int)D.block0;
        fwd_body<TAPS, TC, false>(D.a, local % D.tiles, local / D.tiles, lds, f);
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
    return it == g_tile.end() ? tile_default(kind) : it->second;
}

void set_tile_choice(int kind, int taps, int hk, int wk, int tt) {
    std::lock_guard<std::mutex> lk(g_tile_mu);
    g_tile[std::make_tuple(kind, taps, hk, wk)] = tile_valid(kind, tt) ? tt : tile_default(kind);
}

void fwd_layout(int taps, int tc, int hk, int wk, int64_t planes, int *strips, int *seg_rows, int *tiles) {
    strip_layout(tc, hk, wk, planes, device_cus(), tile_choice(TK_SEG, taps, hk, wk), strips, seg_rows, tiles);
}

hipError_t launch_dwt_fwd(int taps, const Filter &f, const float *src, int64_t src_stride, int src_rows,
                          int src_cols, int n_r, int n_c, int off_r, int off_c, float *out, int planes, float s2,
                          bool write_ll, hipStream_t s, float *ckpt, int64_t ckpt_stride, const unsigned char *src8,
                          int src8_c) {
    const int hk = n_r / 2, wk = n_c / 2;
    const int tc = tile_choice(TK_FWD, taps, hk, wk);
    int strips = 0, seg = 0, tiles = 0;
    fwd_layout(taps, tc, hk, wk, planes, &strips, &seg, &tiles);
    FwdArgs a{src, src_stride, src_rows, src_cols, n_r, n_c, off_r, off_c, out, s2,
              strips, write_ll ? 1 : 0, ckpt, ckpt_stride, src8, src8_c, seg};
    dim3 grid((unsigned)tiles, (unsigned)planes);
    const double bytes = (double)planes * ((src8 ? 1.0 : 4.0) * (double)src_rows * src_cols +
                                           4.0 * (write_ll ? 4.0 : 3.0) * (double)hk * wk);
    KernelTimer kt(taps == 16 ? "dwt_fwd_wiener<16>" : "dwt_fwd_wiener<8>", bytes, s,
                   (double)planes * n_r * n_c * fwd_flops_per_px(taps));
#define PRNU_FWD(TP, T_)                                                                                   \
    do {                                                                                                   \
        if (ckpt) dwt_fwd_wiener<TP, T_, true><<<grid, StripGeom<TP, T_>::NTH, 0, s>>>(a, f);              \
        else dwt_fwd_wiener<TP, T_, false><<<grid, StripGeom<TP, T_>::NTH, 0, s>>>(a, f);                 \
    } while (0)
    if (taps == 16) {
        if (tc == 32) PRNU_FWD(16, 32); else PRNU_FWD(16, 64);
    } else {
        if (tc == 32) PRNU_FWD(8, 32); else PRNU_FWD(8, 64);
    }
#undef PRNU_FWD
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
    // the fold addresses one channel plane of A or B (8 bytes a pixel) and a
    // frame (C bytes a pixel) with 32-bit buffer offsets
    if ((int64_t)H * W >= kMleMaxPixels) return hipErrorInvalidValue;
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
        if (tt == 32) dwt_fwd_multi<16, 32><<<grid, StripGeom<16, 32>::NTH, 0, s>>>(d, nd, total, ctr, f);
        else dwt_fwd_multi<16, 64><<<grid, StripGeom<16, 64>::NTH, 0, s>>>(d, nd, total, ctr, f);
    } else {
        if (tt == 32) dwt_fwd_multi<8, 32><<<grid, StripGeom<8, 32>::NTH, 0, s>>>(d, nd, total, ctr, f);
        else dwt_fwd_multi<8, 64><<<grid, StripGeom<8, 64>::NTH, 0, s>>>(d, nd, total, ctr, f);
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
        return tt == 32 ? occupancy_of(dwt_fwd_multi<16, 32>, StripGeom<16, 32>::NTH)
                        : occupancy_of(dwt_fwd_multi<16, 64>, StripGeom<16, 64>::NTH);
    return tt == 32 ? occupancy_of(dwt_fwd_multi<8, 32>, StripGeom<8, 32>::NTH)
                    : occupancy_of(dwt_fwd_multi<8, 64>, StripGeom<8, 64>::NTH);
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
