// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "prnu.h"

namespace prnu {

// ---- errors ----------------------------------------------------------------
void set_error(const char *fmt, ...);
int fail(int code, const char *fmt, ...);

// ---- optional kernel timing (see prnu_timing_enable) ----------------------
class KernelTimer {
   public:
    // bytes: what the algorithm reads once and writes once; flops: its
    // arithmetic (0 where a launch is pure data movement)
    KernelTimer(const char *name, double bytes, hipStream_t s, double flops = 0.0);
    ~KernelTimer();

   private:
    long idx_;
    hipStream_t s_;
};

// ---- filters ---------------------------------------------------------------
constexpr int kMaxTaps = 16;
// Low-pass h and quadrature-mirror high-pass g = (-1)^k h[L-1-k], rounded to
// float; passed to kernels by value so the taps live in scalar registers.
struct Filter {
    float h[kMaxTaps];
    float g[kMaxTaps];
};
// Daubechies extremal-phase low-pass, long-double spectral factorisation.
bool daubechies_lowpass(int taps, long double *h);
bool make_filter(int taps, Filter *f);
// The same filters rounded to double, for the FP64 mode of the differentiated chain.
struct Filter64 {
    double h[kMaxTaps];
    double g[kMaxTaps];
    int taps;
};
bool make_filter64(int taps, Filter64 *f);

// ---- geometry --------------------------------------------------------------
constexpr int kPadMult = 16;
inline int pad_before(int n) { return ((kPadMult - n % kPadMult) % kPadMult) / 2; }
inline int padded(int n) { return n + (kPadMult - n % kPadMult) % kPadMult; }

// Per-level pyramid buffer: [planes][4][hl][wl], subband 0 = approximation
// (later the partial reconstruction), 1 = lh, 2 = hl, 3 = hh.
inline size_t level_floats(int Hp, int Wp, int lvl) {
    return (size_t)4 * (size_t)(Hp >> lvl) * (size_t)(Wp >> lvl);
}

// ---- per-launch argument blocks (shared by the per-plane and the batched,
// work-queue launches; passed by value) --------------------------------------
struct FwdArgs {
    const float *src;
    int64_t src_stride;
    int src_rows, src_cols, n_r, n_c, off_r, off_c;
    float *out;
    float s2;
    int tiles_c;
    int write_ll;
    float *ckpt;
    int64_t ckpt_stride;
    // u8 frames [.][src_rows][src_cols][src8_c] read in place of `src` (plane
    // p = channel p % src8_c of frame p / src8_c), or null
    const unsigned char *src8;
    int src8_c;
    // forward levels run by strips: tiles_c strips of the tile width across,
    // segments of seg_rows coefficient rows down (see fwd_layout)
    int seg_rows;
};
struct InvArgs {
    const float *lvl;
    int hk, wk, zero_approx, tiles_c;
    float *out;
    int H, W, off_r, off_c;
};
// Frames of at least this many pixels are refused by the MLE fold (its
// buffer offsets into an FP64 accumulator plane are 32-bit).
constexpr int64_t kMleMaxPixels = (int64_t)1 << 28;
struct MleArgs {
    const float *lvl;
    int hk, wk, zero_approx, tiles_c, nb, C;
    const float *means;
    int H, W, off_r, off_c;
    void *A, *B;
    // u8 frames [nb][H][W][C] read in place of `means` (SDA depth 1), or null
    const unsigned char *means8;
};
// One entry of a batched launch: `blocks` virtual workgroups starting at block0.
struct FwdDesc {
    FwdArgs a;
    int tt, tiles, planes, pad;
    int64_t block0;
};
struct InvDesc {
    InvArgs a;
    int tt, tiles, planes, pad;
    int64_t block0;
};
struct MleDesc {
    MleArgs a;
    int tt, tiles, pad0, pad1;
    int64_t block0;
};
struct SdaDesc {
    const void *frames;
    int64_t npx;
    int dtype, n_frames, C, group, g0, ng, quad, bpg;
    float *means;
    int64_t block0;
};

// Tile width per kernel kind and level size: the forward level runs strips
// of 64 or 32 subband columns (64 unless prnu_autotune measured otherwise),
// the inverse and MLE levels square tiles of 32 or 16 (32 by default).
// TK_SEG is the forward strip's segment length, stored as the number of
// workgroups per CU a launch aims at (3, 6 or 12, default 6): fewer, longer
// segments pay the vertical halo and the row-filter carry less often, more
// and shorter ones fill the chip more evenly.
enum TileKind { TK_FWD = 0, TK_INV = 1, TK_MLE = 2, TK_SEG = 3 };
inline int tile_default(int kind) { return kind == TK_FWD ? 64 : kind == TK_SEG ? 6 : 32; }
inline int tile_small(int kind) { return kind == TK_FWD ? 32 : kind == TK_SEG ? 3 : 16; }
inline bool tile_valid(int kind, int tt) {
    return tt == tile_default(kind) || tt == tile_small(kind) || (kind == TK_SEG && tt == 12);
}
int tile_choice(int kind, int taps, int hk, int wk);
void set_tile_choice(int kind, int taps, int hk, int wk, int tt);
inline int tiles_for(int tt, int hk, int wk) { return ((hk + tt - 1) / tt) * ((wk + tt - 1) / tt); }
// Forward level of hk x wk coefficients over `planes` planes in strips of tc
// columns: strips per plane, rows per segment and virtual blocks per plane.
void fwd_layout(int taps, int tc, int hk, int wk, int64_t planes, int *strips, int *seg_rows, int *tiles);

// ---- kernel launchers (all enqueue on `s`, return the launch status) -------
// SDA: groups [g0, g1) of `group` frames; outputs indexed from g0.
hipError_t launch_sda(const void *frames, int64_t fstride, int dtype, int n_frames, int H, int W, int C, int group,
                      int g0, int g1, uint32_t *sums, float *means, int *counts, uint32_t *status, hipStream_t s);
// state->frames += frames, state->sda_frames += sda_frames (one thread, in stream order).
hipError_t launch_acc_state_add(prnu_acc_state *st, int64_t frames, int64_t sda_frames, hipStream_t s);

// Forward level with fused Wiener shrinkage.  src plane p at src + p*src_stride,
// stored src_rows x src_cols; the level input is the n_r x n_c plane obtained
// by symmetric padding with (off_r, off_c) samples before (level 1) or the
// plane itself (off = 0, n = stored size).  out: [planes][4][n_r/2][n_c/2].
// ckpt (nullable): per plane (stride ckpt_stride) the level's [3][n_r/2][n_c/2]
// sensitivities c/m of the detail coefficients whose window mean m exceeds s2
// (0 elsewhere), in subband order lh, hl, hh.
hipError_t launch_dwt_fwd(int taps, const Filter &f, const float *src, int64_t src_stride,
                          int src_rows, int src_cols, int n_r, int n_c, int off_r, int off_c,
                          float *out, int planes, float s2, bool write_ll, hipStream_t s,
                          float *ckpt = nullptr, int64_t ckpt_stride = 0, const unsigned char *src8 = nullptr,
                          int src8_c = 0);

enum InvEpilogue { INV_PLANE = 0, INV_RESID = 1, INV_MLE = 2 };

// Inverse level: reads lvl = [planes][4][hk][wk] (subband 0 ignored when
// zero_approx) and writes the 2hk x 2wk plane into
//   INV_PLANE: out [planes][4][2hk][2wk] subband 0,
//   INV_RESID: out [planes][H][W] cropped at (off_r, off_c).
hipError_t launch_dwt_inv(int taps, const Filter &f, const float *lvl, int hk, int wk,
                          bool zero_approx, int planes, int epi, float *out, int H, int W,
                          int off_r, int off_c, hipStream_t s);

// Inverse level 1 with the MLE epilogue: planes are [nb][C]; for every channel
// c and pixel, A[c] += sum_f W_f * I_f and B[c] += sum_f I_f^2 where I_f is
// means[f][c] ([nb][C][H][W]).
hipError_t launch_dwt_inv_mle(int taps, const Filter &f, const float *lvl, int hk, int wk,
                              bool zero_approx, int nb, int C, const float *means, int H, int W,
                              int off_r, int off_c, int acc_mode, void *A, void *B, hipStream_t s,
                              const unsigned char *means8 = nullptr);

// Batched (work-queue) launches of one tile size tt: every workgroup of a
// grid of `grid` takes virtual blocks from *ctr until `total`; *ctr must be
// zero at launch, total + grid < 2^31.  Descriptors: block0 ascending from 0,
// each covering tiles x planes (or tiles x C for the MLE) virtual blocks.
hipError_t launch_fwd_multi(int taps, int tt, const Filter &f, const FwdDesc *d, int nd, int total, int *ctr,
                            int grid, hipStream_t s);
hipError_t launch_inv_multi(int taps, int tt, const Filter &f, const InvDesc *d, int nd, int total, int *ctr,
                            int grid, hipStream_t s);
hipError_t launch_mle_multi(int taps, int tt, int acc_mode, const Filter &f, const MleDesc *d, int nd, int total,
                            int *ctr, int grid, hipStream_t s);
hipError_t launch_zero_ints(int *p, int n, hipStream_t s);
hipError_t launch_fill_pattern(float *x, int64_t n, hipStream_t s);
// Resident workgroups per CU of each batched kernel (for the persistent grid).
int fwd_multi_occupancy(int taps, int tt);
// compute units of the current device (cached per device)
int device_cus();
// Algorithmic arithmetic of a wavelet level, per pixel of the level's input
// (analysis) or output (synthesis): 2 TAPS flops per pass and direction; the
// Wiener shrinkage adds 36 per detail coefficient (3 of every 4 coefficients).
inline double fwd_flops_per_px(int taps) { return 4.0 * taps + 0.75 * 36.0; }
inline double inv_flops_per_px(int taps) { return 4.0 * taps; }
int inv_multi_occupancy(int taps, int tt);
int mle_multi_occupancy(int taps, int tt, int acc_mode);

// Batched SDA means (no sums): a 1-D grid of `total` blocks over the
// descriptors; quad = sda_quad_ok(...) for the descriptor's buffers, bpg =
// sda_blocks_per_group(quad, npx), means [ng][C][H][W] of groups g0 .. g0+ng-1.
bool sda_quad_ok(const void *frames, int64_t fstride, int dtype, int64_t npx, int C, const void *sums,
                 const void *means);
int sda_blocks_per_group(bool quad, int64_t npx);
hipError_t launch_sda_multi(const SdaDesc *d, int nd, int64_t total, hipStream_t s);

// ---- post-processing -------------------------------------------------------
// K[c] = A[c] / B[c] (0 where B = 0) as float [C][H][W].
hipError_t launch_ratio(const void *A, const void *B, int acc_mode, int64_t n, float *K,
                        hipStream_t s);
// Zero-mean per plane and optional luma.  in: [C][H][W]; out: [1][H][W] with
// luma else [C][H][W].  rowpart/colpart: double scratch of zm_scratch_doubles.
// nf frames of C planes: in [nf][C][H][W] -> out [nf][luma ? 1 : C][H][W].
size_t zm_scratch_doubles(int nf, int C, int H, int W);
hipError_t launch_zero_mean(const float *in, int nf, int C, int H, int W, bool zm, bool luma, float *out,
                            double *scratch, hipStream_t s);
// Convert planes [n][H][W] (n planes) u8/bf16/f32 interleaved frames -> luma.
hipError_t launch_luma_frames(const void *frames, int dtype, int n, int H, int W, int C,
                              float *out, hipStream_t s);

// ---- FFT -------------------------------------------------------------------
struct FftPlan {
    int n;        // length
    int nrad;     // number of passes
    int rad[16];  // radices, each in {2,3,4,5}
    int nvec;     // vectors per workgroup (power of two)
    int lvec;     // log2(nvec)
};
// columns: a plan for strided (column) vectors, which groups more vectors.
bool make_fft_plan(int n, FftPlan *p, bool columns = false);
size_t fft_twiddle_floats(int n);  // complex table of n entries, 2 floats each
hipError_t launch_twiddles(int n, float2 *tw, hipStream_t s);
// In-place 2-D complex FFT on `batch` planes [h][w] (plane stride h*w).
// dir = -1 forward, +1 inverse (unnormalised).  With rin the rows pass reads
// the real planes rin [batch][h][w] instead of data; with rout the columns
// pass stores only rscale * the real part, to rout [batch][h][w].
hipError_t launch_fft2(float2 *data, int batch, int h, int w, const FftPlan &ph,
                       const FftPlan &pw, const float2 *tw_h, const float2 *tw_w, int dir,
                       hipStream_t s, const float *rin = nullptr, float *rout = nullptr, float rscale = 1.f);

// Real rows -> half spectra of h rows x w/2+1 bins (w even, phalf planned for
// w/2), n planes of half_plane_elems(h, w/2+1, pcol) in the column-group
// layout of the column plan pcol (groups of pcol.nvec bins; see fft.hip).
// Plane p is Y[(p0+p) % ny], times mod[(p0+p) / ny] when mod is given, minus
// mean[p] when mean is given.  tw_half: table for w/2; tw_full: table for w.
hipError_t launch_rfft_rows(const float *Y, const float *mod, int ny, int p0, int n, const double *mean,
                            int h, int w, const FftPlan &phalf, const float2 *tw_half, const float2 *tw_full,
                            const FftPlan &pcol, float2 *out, hipStream_t s);
// Column transforms of half spectra S (n planes in the column-group layout
// of ph): with Px, reduce sum wgt*Px[(p0+p)/ny]*|S|^2 (DC excluded) into
// part[p][blocks]; else store |S|^2 into Pout.  Px and Pout have the same
// layout as S.
int fft_cols_power_blocks(int Mc, const FftPlan &ph);
// Elements of one half spectrum or power table in the column-group layout.
int64_t half_plane_elems(int h, int Mc, const FftPlan &ph);
hipError_t launch_fft_cols_power(const float2 *S, int n, int h, int Mc, const FftPlan &ph, const float2 *tw_h,
                                 const float *Px, int ny, int p0, float *Pout, double *part, hipStream_t s);

// ---- reductions and Wiener in the DFT domain --------------------------------
// Per-plane population variance of float planes [n][N] -> double var[n];
// scratch: reduce_scratch_doubles(n, N).
size_t reduce_scratch_doubles(int n, int64_t N);
hipError_t launch_plane_variance(const float *x, int n, int64_t N, double *var, double *scratch,
                                 hipStream_t s);
// G = F * rho with rho the Wiener residual factor of |F|/sqrt(hw); noise
// variance var[p] (per plane, device) or sigma2 >= 0 (host constant).
// Bilinear resampling of n planes [n][H][W] to [n][oh][ow] (pixel centres,
// scale = output / input size, crop offset (oy, ox) in output pixels).
hipError_t launch_resample_bilinear(const float *src, int n, int H, int W, double scale, int oy, int ox, int oh,
                                    int ow, float *out, hipStream_t s);
// Affine bilinear warp: plane k of out [n][oh][ow] samples src [k % n_src][H][W]
// at column m0 x + m1 y + m2, row m3 x + m4 y + m5 (m = affine + 6k, device).
hipError_t launch_warp_affine(const float *src, int n_src, int H, int W, const double *affine, int n, int oh, int ow,
                              float *out, hipStream_t s);
// Disjoint b x b blocks of n planes [n][H][W], block-major [k][n][b][b].
hipError_t launch_extract_blocks(const float *src, int n, int H, int W, int b, float *out, hipStream_t s);
hipError_t launch_spectral_wiener(const float2 *F, int n, int h, int w, const double *var,
                                  float sigma2, float2 *G, hipStream_t s);

// ---- PCE -------------------------------------------------------------------
// Chunk plane p (0 <= p < n) is Y[(p0+p) % ny], times mod[(p0+p) / ny] when mod
// is given.  Plain planes: mod = nullptr and ny > p0 + n.  launch_pair_stats
// skips the centred norms when nrm2 is null.
size_t pce_part_bytes(int npairs);
size_t stats_part_doubles(int n);
hipError_t launch_pair_stats(const float *Y, const float *mod, int ny, int p0, int n, int64_t N,
                             double *mean, double *nrm2, double *part, hipStream_t s);
hipError_t launch_pair_center(const float *Y, const float *mod, int ny, int p0, int n, int64_t N,
                              const double *mean, float2 *z, hipStream_t s);
// z[p] = Xs[q] * conj(Ycache ? Ycache[j] : z[p]) with q = (p0+p)/ny, j = (p0+p)%ny.
hipError_t launch_cross(const float2 *Xs, const float2 *Ycache, int ny, int p0, int n, int64_t N,
                        float2 *z, hipStream_t s);
// Reduce the n surfaces z[p] (real part = N * C) into pce/ncc/peak[p0 + p].
hipError_t launch_pce_reduce(const float2 *z, int n, int h, int w, int nbhd, int peak_mode,
                             const double *xn2, const double *yn2, bool yn2_by_j, int ny, int p0,
                             double *pce, double *ncc, int32_t *peak, void *part, hipStream_t s);

// Fixed-peak fast path: direct sums of the (2*5+1)^2 shifts around 0 plus
// sum y, sum y^2, sum xc per pair (part [n][pce_direct_blocks][124] doubles);
// the spectral energy term comes from fft_cols_power or power_dot.
int pce_direct_blocks(int h, int w);
size_t pce_direct_part_doubles(int npairs, int h, int w);
int pce_dot_blocks();
hipError_t launch_pce_direct(const float *X, const double *xmean, const float *Y, const float *mod, int ny,
                             int p0, int n, int h, int w, double *part, hipStream_t s);
// Px, Py in the column-group layout of groups of 2^lg bins.
hipError_t launch_power_dot(const float *Px, const float *Py, int ny, int p0, int n, int h, int Mc, int lg,
                            double *part, hipStream_t s);
// Doubles per (pair, block) of the direct-sum partials: 121 shifts, sum y,
// sum y^2, sum xc.
constexpr int kPceDirectStats = 124;
// The same direct sums on the matrix cores for every fingerprint of queries
// q0 .. q0+nq-1: part [(q - q0) * ny + j][nblk][124] doubles.
int pce_mfma_blocks(int nq, int ny, int h, int w);
// syy: also the sums of y^2 (the NCC's fingerprint norms); without it their
// partial slots are left unwritten.
hipError_t launch_pce_direct_mfma(const float *X, const double *xmean, const float *Y, const float *mod, int ny,
                                  int q0, int nq, int h, int w, int nblk, bool syy, double *part, hipStream_t s);
hipError_t launch_pce_finish_fixed(const double *dpart, int nblk_d, const double *spart, int nblk_s, int n,
                                   int h, int w, int nbhd, const double *xn2, int ny, int p0, double *pce,
                                   double *ncc, int32_t *peak, hipStream_t s);

// ---- adjoint -------------------------------------------------------------------
// Gradient analysis of one level: src planes (stride src_stride, stored
// src_rows x src_cols; level 1 is zero-embedded into the padded n_r x n_c
// frame at (off_r, off_c) and optionally scaled by mul (per plane) / div
// (shared)), approximation to ll_out [planes][n_r/2][n_c/2] (nullable), the
// detail bands dotted with ckpt ([3][n_r/2][n_c/2] per plane) into
// part[planes][dwt_vjp_tiles].
int dwt_vjp_tiles(int hk, int wk);
hipError_t launch_dwt_vjp(int taps, const Filter &f, const float *src, int64_t src_stride, int src_rows,
                          int src_cols, const float *mul, int64_t mul_stride, const float *div, int n_r, int n_c,
                          int off_r, int off_c, float *ll_out, const float *ckpt, int64_t ckpt_stride, int planes,
                          double *part, hipStream_t s);
hipError_t launch_vjp_finish(const double *part, int64_t n, double *out, hipStream_t s);
size_t pvjp_coef_bytes(int n);
// PCE adjoint of a chunk of n pairs; Z holds the unnormalised inverse
// transform of X^ conj(V) (N * C), V the transforms of the centred y's.
hipError_t launch_pvjp(float2 *Z, float2 *V, float2 *T1, float2 *T2, const float2 *Xs, int n, int h, int w,
                       int nbhd, int ny, int p0, const FftPlan &ph, const FftPlan &pw, const float2 *tw_h,
                       const float2 *tw_w, void *coef, const double *wts, const float *mod, double *pce, float *gX,
                       float *gY, hipStream_t s);
hipError_t launch_fill_zero(float *x, int64_t n, hipStream_t s);

// ---- FP64 mode of the differentiated chain ---------------------------------
constexpr int kRedBlocks64 = 64;  // partial sums per plane of an FP64 reduction
struct Gap64Dims {
    int ncam, m, g, d, nq, H, W, Hp, Wp, t, l, levels, taps, nbhd;
    int64_t ssz;  // checkpoint doubles per plane: 3 bands of each level
};
bool gap64_fft_length_ok(int n);
size_t gap64_workspace_bytes(const Gap64Dims &D);
// Forward and backward of the PCE gap in FP64; out (device) = loss, dL/dsigma0,
// dL/dlambda_1..4; pce_out (device, nullable) [nq][ncam].
hipError_t gap64_run(const Gap64Dims &D, const Filter64 &f, const double *theta, const float *cams,
                     const float *queries, const int *qcam, void *ws, double *out, double *pce_out, hipStream_t s);

}  // namespace prnu
