/*
 * prnu.h -- C ABI of the MI355X (gfx950) camera-fingerprint library.
 *
 * The library computes the fingerprint-extraction path of "Camera Fingerprint
 * Extraction via Spatial Domain Averaged Frames" (Taspinar, Mohanty, Memon,
 * arXiv 1909.04573):
 *
 *   spatial-domain averaged (SDA) frames            (Sec. III-B, SDA-frame mean)
 *   -> noise residual W = I - F(I), F a 4-level     (Sec. II-A, Eq. (1) and the
 *      wavelet denoiser with local Wiener shrinkage  residual definition; Sec. IV
 *                                                     names the wavelet denoiser)
 *   -> MLE fingerprint K = sum W*I / sum I^2        (Sec. III-A MLE; Sec. III-B,
 *                                                     SDA form of the MLE)
 *   -> zero-mean, luma, DFT-domain Wiener filtering
 *   -> PCE / NCC of query residuals vs fingerprints (Sec. II-A correlation step;
 *                                                     Sec. IV, PCE threshold 60)
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Array arguments are DEVICE pointers owned by the caller (row-major,
 *    planes contiguous).  The library never allocates device memory and keeps
 *    no device state between calls (a prnu_batch object owns its HIP graph);
 *    every scratch byte comes from the caller's workspace `ws` of at least the
 *    size the matching *_workspace_size call reports.  The workspace must be
 *    256-byte aligned.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  Every
 *    call only enqueues work on it; results are valid once the stream has
 *    been synchronised.  Calls on different streams with different
 *    workspaces may run concurrently.
 *  - All arguments are checked on the host before anything is enqueued; on
 *    any error nothing is enqueued and the status says why:
 *        PRNU_OK             success
 *        PRNU_E_INVAL        null pointer, bad size, bad mode or flag
 *        PRNU_E_UNSUPPORTED  valid but not implemented (e.g. FFT size with a
 *                            prime factor above 5, filter length)
 *        PRNU_E_WORKSPACE    workspace too small or misaligned
 *        PRNU_E_HIP          a HIP launch failed (the HIP error string is kept)
 *    prnu_last_error() returns a thread-local text for the last failure.
 *  - Frames are stored [n][H][W][C] (C = 1 or 3 channels, interleaved), with
 *    element type PRNU_U8, PRNU_BF16 or PRNU_F32.  Planar float data is
 *    [plane][H][W].
 *  - Readings where the paper is silent: periodised orthonormal Daubechies
 *    DWT after symmetric padding to a multiple of 16; Wiener windows 3,5,7,9
 *    with zero extension; the approximation band is kept by F, so the
 *    residual's approximation band is zero; a last SDA group with fewer than
 *    `group` frames is averaged over its own count.
 */
#ifndef PRNU_H
#define PRNU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PRNU_OK 0
#define PRNU_E_INVAL (-1)
#define PRNU_E_UNSUPPORTED (-2)
#define PRNU_E_WORKSPACE (-3)
#define PRNU_E_HIP (-4)

/* frame element types */
#define PRNU_U8 0
#define PRNU_BF16 1
#define PRNU_F32 2

/* MLE accumulator storage (A = sum W*I, B = sum I^2), see
 * prnu_fingerprint_accumulate */
#define PRNU_ACC_F64 0       /* double A[C][H][W], double B[C][H][W]          */
#define PRNU_ACC_KAHAN_F32 1 /* float A[2][C][H][W]: value plane then         */
                             /* compensation plane (value = [0] + [1]); same B */
#define PRNU_ACC_F32 2       /* float A[C][H][W], float B[C][H][W]            */

/* post-processing flags (finalize and query residuals) */
#define PRNU_ZM 1     /* per channel: subtract row means, then column means   */
#define PRNU_LUMA 2   /* C = 3: combine channels 0.299 R + 0.587 G + 0.114 B  */
#define PRNU_WIENER 4 /* DFT-domain Wiener filtering of each output plane     */

/* PCE peak location */
#define PRNU_PEAK_FIXED_00 0 /* aligned verification: peak is C(0,0)          */
#define PRNU_PEAK_ARGMAX 1   /* shift search: first maximum, row-major order   */

typedef struct prnu_denoise_params {
    float sigma0;          /* std of the noise the Wiener step assumes (grey levels) */
    int levels;            /* wavelet levels, 1..4 (padding is always to 16)          */
    int taps;              /* Daubechies filter length: 8 or 16 ("db8" = 16)          */
    float level_weight[4]; /* level l (finest = 0) uses noise variance                */
                           /* level_weight[l] * sigma0^2; all 1 for the plain method */
} prnu_denoise_params;

typedef struct prnu_pce_params {
    int peak_mode; /* PRNU_PEAK_FIXED_00 or PRNU_PEAK_ARGMAX                       */
    int nbhd;      /* odd side of the block around the peak left out of the energy */
} prnu_pce_params;

/* Text of the last error on this thread ("" if none). */
const char *prnu_last_error(void);
/* Library version string. */
const char *prnu_version(void);
/* sigma0 = 3, 4 levels, 16 taps, weights 1. */
void prnu_default_denoise_params(prnu_denoise_params *p);

/* Host-only: the Daubechies low-pass filter the kernels use, h[0..taps-1]
 * (extremal phase, sum = sqrt(2)), computed by spectral factorisation in long
 * double.  taps in {2,4,...,20}.  Enqueues nothing. */
int prnu_filter_coefficients(int taps, double *h);

/* Status bits a call ORs into a caller-zeroed device word */
#define PRNU_STATUS_NONFINITE 1u /* a BF16/F32 frame sample was NaN or +-Inf */

/* ---------------------------------------------------------------------------
 * SDA frames (Sec. III-B: the mean of d consecutive frames; the group sizes
 * n_i of the last group's shorter run).
 *
 * frames  n_frames frames of H x W x C interleaved samples of `dtype`; frame f
 *         starts at frames + f * frame_stride_bytes.  frame_stride_bytes = 0
 *         means dense (H*W*C*element size); otherwise it must be at least that
 *         and a multiple of the element size (frames that sit inside larger
 *         decoder surfaces, or every k-th frame of a buffer).
 * group   d >= 1: group i holds frames i*d .. min((i+1)*d, n_frames) - 1;
 *         g = ceil(n_frames / d) groups.
 * sums    PRNU_U8 only (else must be NULL), nullable: uint32 [g][C][H][W],
 *         exact integer sums (n_frames <= 16843009 so 255*d fits).
 * means   nullable: float [g][C][H][W] = sum / count, correctly rounded
 *         (U8: the exact integer sum divided once; BF16/F32: sum in double).
 * counts  nullable: int32 [g], the number of frames in each group.
 * status  nullable device word; PRNU_STATUS_NONFINITE is ORed in when a
 *         BF16/F32 group sum is NaN or infinite (a NaN or infinite sample;
 *         u8 frames never set it).  The caller clears it.
 * At least one of sums/means must be given.
 */
int prnu_sda_average(const void *frames, int dtype, int n_frames, int H, int W, int C,
                     int64_t frame_stride_bytes, int group, uint32_t *sums, float *means, int *counts,
                     uint32_t *status, void *stream);

/* ---------------------------------------------------------------------------
 * Noise residual W = I - F(I) of float planes (Sec. II-A; denoiser of Sec. IV).
 *
 * img    float [n_img][H][W] (grey levels), H, W >= 16.
 * resid  float [n_img][H][W] output (may not alias img).
 */
int prnu_denoise_residual_workspace_size(int n_img, int H, int W, const prnu_denoise_params *p,
                                         size_t *bytes);
int prnu_denoise_residual(const float *img, int n_img, int H, int W, const prnu_denoise_params *p,
                          float *resid, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Noise residuals without any allocation, for callers that cannot allocate
 * device memory or pass a workspace: code under HIP graph / stream capture,
 * tight serving loops, and hosts that forbid allocation.
 *
 * Same arguments, results and errors as prnu_denoise_residual minus the
 * workspace: the scratch (the wavelet pyramid of a batch of planes) is a
 * file-scope device array of PRNU_STATIC_SCRATCH_BYTES (64 MiB) that each GPU
 * the library runs on holds until the process ends; its address is looked up
 * on the first call on each device.  Planes are processed in batches that fit
 * it; PRNU_E_INVAL if the pyramid of one padded H x W plane does not (the
 * limit lies between 4000 x 3000 and 4096 x 4096 at 4 levels).  Nothing in the
 * scratch needs to start at zero: every call overwrites what it reads.
 * Every call on one GPU shares that GPU's array: calls that overlap in time on
 * one GPU (other streams or host threads) race and must be serialised by the
 * caller.  The call allocates nothing (no hipMalloc / hipFree) and only
 * enqueues kernels on `stream`.
 */
#define PRNU_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int prnu_denoise_residual_noalloc(const float *img, int n_img, int H, int W, const prnu_denoise_params *p,
                                  float *resid, void *stream);

/* ---------------------------------------------------------------------------
 * Fused SDA -> residual -> MLE accumulation (Sec. III-B: the SDA frames are
 * denoised and combined with the MLE; group = 1 is the conventional
 * per-frame estimator of Sec. III-A).
 *
 * frames   n_frames frames of H x W x C samples of `dtype`, frame f at
 *          frames + f * frame_stride_bytes (0 = dense, as prnu_sda_average);
 *          SDA groups of `group` frames are formed inside this call (the last
 *          may be shorter).  Depth-1 u8 frames are read in place when dense;
 *          strided ones are first gathered by the SDA kernel.
 * A, B     accumulators in the layout of `acc_mode` (see PRNU_ACC_*), per
 *          channel: A += sum_i W_i * I_i, B += sum_i I_i^2 over this call's SDA
 *          frames I_i.  The caller zeroes them once; calling again with more
 *          frames continues the same sums (streaming / resume).
 * state    nullable device prnu_acc_state kept beside A and B (zeroed with
 *          them): after each internal batch's MLE fold, on the same stream,
 *          `frames` and `sda_frames` grow by that batch's counts, and
 *          PRNU_STATUS_NONFINITE is ORed into `status` when a BF16/F32 frame
 *          holds a NaN or infinity.  (A, B, state) is the checkpoint of a
 *          streamed fingerprint: a run that stopped part-way shows fewer
 *          frames than were submitted.  With group > 1 a call's groups are
 *          its own: resuming mid-group is the caller's split of the frames.
 */
typedef struct prnu_acc_state {
    int64_t frames;     /* frames folded into A, B                          */
    int64_t sda_frames; /* SDA frames (groups) folded into A, B             */
    uint32_t status;    /* PRNU_STATUS_* bits                               */
    uint32_t reserved;
} prnu_acc_state;

int prnu_fingerprint_accumulate_workspace_size(int n_frames, int H, int W, int C, int group,
                                               const prnu_denoise_params *p, size_t *bytes);
int prnu_fingerprint_accumulate(const void *frames, int dtype, int n_frames, int H, int W, int C,
                                int64_t frame_stride_bytes, int group, const prnu_denoise_params *p,
                                int acc_mode, void *A, void *B, prnu_acc_state *state, void *ws,
                                size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Fingerprint finalisation: K = A / B per channel (0 where B = 0), then the
 * post-processing `flags` (PRNU_ZM, PRNU_LUMA, PRNU_WIENER) in that order.
 *
 * K         float output: [H][W] when C = 1 or PRNU_LUMA is set, else [C][H][W].
 * sigma_wf  std of the DFT-Wiener noise; < 0 uses the population std of the
 *           field being filtered.
 * PRNU_WIENER needs H and W free of prime factors above 5.
 */
int prnu_fingerprint_finalize_workspace_size(int C, int H, int W, int flags, size_t *bytes);
int prnu_fingerprint_finalize(const void *A, const void *B, int acc_mode, int C, int H, int W,
                              int flags, float sigma_wf, float *K, void *ws, size_t ws_bytes,
                              void *stream);

/* ---------------------------------------------------------------------------
 * Query residuals (Sec. II-A: the query's noise residual, to be correlated
 * with a fingerprint).  Each frame's channels are denoised, then the same
 * post-processing as prnu_fingerprint_finalize is applied.
 *
 * frames  [n][H][W][C] of `dtype`.
 * Wq      float [n][H][W] (C = 1 or PRNU_LUMA) else [n][C][H][W].
 * Iq      nullable float [n][H][W]: the frame's luma (C = 3) or plane (C = 1),
 *         the intensity that modulates the fingerprint in the matched statistic.
 */
int prnu_query_residual_workspace_size(int n, int H, int W, int C, const prnu_denoise_params *p,
                                       int flags, size_t *bytes);
int prnu_query_residual(const void *frames, int dtype, int n, int H, int W, int C,
                        const prnu_denoise_params *p, int flags, float *Wq, float *Iq, void *ws,
                        size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Block gather for the block-wise PCE protocol (Sec. IV: each fingerprint
 * and each test residual is divided into disjoint 500 x 500 blocks and
 * corresponding blocks are correlated).
 *
 * src: n planes [n][H][W] fp32 (device); out: device buffer of
 * (H/b)*(W/b)*n*b*b floats, written block-major:
 *   out[k][p][r][c] = src[p][(k / nbc)*b + r][(k % nbc)*b + c],
 *   nbc = W / b, k < (H / b) * nbc,
 * so the n planes of block k are one contiguous [n][b][b] batch for
 * prnu_pce_match.  Rows and columns past the last whole block are unused.
 * PRNU_E_INVAL for null pointers, n < 1, H or W outside [1, 32768],
 * b outside [1, min(H, W)], or more than 2^31 - 1 block-planes.  Enqueued on
 * `stream`; nothing is allocated.
 */
int prnu_extract_blocks(const float *src, int n, int H, int W, int b, float *out, void *stream);

/* Bilinear resampling for mixed-media matching (Sec. V-B: the query image is
 * resized and cropped to the geometry of the video fingerprint before its
 * PRNU is matched).
 *
 * src [n][H][W] fp32 and out [n][oh][ow] fp32, device buffers:
 *   out[p][y][x] = bilinear(src[p], (y + oy + 0.5)/scale - 0.5, (x + ox + 0.5)/scale - 0.5)
 * pixel-centre convention, sample coordinates clamped to the plane (edge
 * replication); scale = output size / input size; (oy, ox) is a crop offset
 * in output pixels.  PRNU_E_INVAL for null pointers, n outside [1, 65535],
 * sizes outside [1, 32768], a scale that is not finite and positive, or
 * negative offsets.  Enqueued on `stream`; nothing is allocated.
 */
int prnu_resample_bilinear(const float *src, int n, int H, int W, double scale, int oy, int ox, int oh, int ow,
                           float *out, void *stream);

/* ---------------------------------------------------------------------------
 * Affine bilinear warp for stabilised video (Sec. II-B: digital stabilisers
 * shift, rotate, shear or zoom each frame, so frames' sensor patterns are
 * misaligned; Sec. V-E matches stabilised videos).
 *
 * out[k][y][x] = bilinear sample of src[k % n_src] at column
 *   u = m0 x + m1 y + m2 and row v = m3 x + m4 y + m5 (pixel indices),
 * m = affine + 6 k: a DEVICE array of n * 6 doubles (one matrix per output
 * plane); u and v are computed in double and clamped to the plane (edge
 * replication).  src [n_src][H][W] fp32, out [n][oh][ow] fp32 (may not alias
 * src).  With m = (1/s, 0, (ox + 0.5)/s - 0.5, 0, 1/s, (oy + 0.5)/s - 0.5)
 * it is prnu_resample_bilinear.  PRNU_E_INVAL for null pointers, n_src < 1,
 * n outside [1, 65535], or sizes outside [1, 32768].  Enqueued on `stream`;
 * nothing is allocated.
 */
int prnu_warp_affine(const float *src, int n_src, int H, int W, const double *affine, int n, int oh, int ow,
                     float *out, void *stream);

/* ---------------------------------------------------------------------------
 * PCE / NCC matching (Sec. II-A correlation; Sec. IV uses PCE > 60).
 *
 * For every pair (q, j):  x = X[q] - mean,  y = Y'[q][j] - mean, where
 * Y'[q][j] = modulate[q] * Y[j] elementwise when `modulate` is given (the
 * query intensity times the fingerprint), else Y[j];
 * C(s) = sum_t x(t + s) y(t) (circular);  peak p per `peak_mode`;
 * energy = mean of C(s)^2 over the shifts outside the nbhd x nbhd block
 * centred on p;  pce = sign(C(p)) C(p)^2 / energy;  ncc = C(0) / (|x| |y|).
 *
 * X         float [nx][h][w];  Y float [ny][h][w];  modulate nullable [nx][h][w].
 * pce       double [nx][ny] output;  ncc nullable double [nx][ny];
 * peak      nullable int32 [nx][ny][2] (row, col) of the peak.
 * h, w > nbhd, both free of prime factors above 5 (else PRNU_E_UNSUPPORTED).
 */
int prnu_pce_match_workspace_size(int nx, int ny, int h, int w, int modulated, size_t *bytes);
int prnu_pce_match(const float *X, int nx, const float *Y, int ny, int h, int w,
                   const float *modulate, const prnu_pce_params *pp, double *pce, double *ncc,
                   int32_t *peak, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Post-processing of given planes (the chain prnu_fingerprint_finalize applies
 * after the ratio): zero-mean per plane, BT.601 luma of channel triples,
 * DFT-domain Wiener.  planes [n][C][H][W] -> out [n][C or 1][H][W] (no alias).
 * Zero-mean is linear and self-adjoint, so the same call applies its adjoint.
 */
int prnu_postprocess_workspace_size(int n, int C, int H, int W, int flags, size_t *bytes);
int prnu_postprocess(const float *planes, int n, int C, int H, int W, int flags, float sigma_wf, float *out,
                     void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Adjoint of the residual with respect to the shrinkage noise variances
 * s_l = level_weight[l] * sigma0^2 (the denoiser's parameters; Sec. II-A
 * residual, Sec. IV denoiser).  Per detail coefficient c with smallest window
 * mean m of c^2, the residual coefficient is c s / max(s, m), so
 * dr/ds = c / m where m > s and 0 elsewhere.
 *
 * prnu_denoise_residual_ckpt: as prnu_denoise_residual, and also stores those
 *   sensitivities: ckpt [n_img][prnu_denoise_ckpt_floats] float, per plane
 *   level 1's [3][Hp/2][Wp/2] (bands lh, hl, hh), then level 2, ... where
 *   Hp, Wp are H, W padded to multiples of 16.
 * prnu_denoise_residual_vjp: given dL/dW for n planes (plane p at
 *   gW + p * gW_plane_stride; stride 0 broadcasts one plane), optionally
 *   multiplied elementwise by mul[p] ([n][H][W]) and divided by div ([H][W],
 *   0 where div <= 0) -- the MLE's dK/dW_i = I_i / sum I^2 --, adds
 *   dL/ds_l summed over the planes to dLds[l] (device doubles, `levels` of them).
 */
int prnu_denoise_ckpt_floats(int H, int W, int levels, size_t *floats);
int prnu_denoise_residual_ckpt(const float *img, int n_img, int H, int W, const prnu_denoise_params *p,
                               float *resid, float *ckpt, void *ws, size_t ws_bytes, void *stream);
int prnu_denoise_residual_vjp_workspace_size(int n, int H, int W, const prnu_denoise_params *p,
                                             size_t *bytes);
int prnu_denoise_residual_vjp(const float *gW, int64_t gW_plane_stride, const float *mul, const float *div,
                              int n, int H, int W, const prnu_denoise_params *p, const float *ckpt,
                              double *dLds, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Adjoint of the fixed-peak PCE (Sec. IV statistic) for a weighted sum
 * L = sum_{q,j} weights[q][j] * PCE(X[q], Y'[q][j]) with Y' as in
 * prnu_pce_match: gX [nx][h][w] = dL/dX, gY [ny][h][w] = dL/dY (the
 * modulation folded in), both overwritten; pce (nullable) [nx][ny] receives
 * the PCE values.  weights: device doubles [nx][ny].  h, w > nbhd,
 * prime factors <= 5.
 */
int prnu_pce_vjp_workspace_size(int nx, int ny, int h, int w, size_t *bytes);
int prnu_pce_vjp(const float *X, int nx, const float *Y, int ny, int h, int w, const float *modulate,
                 int nbhd, const double *weights, double *pce, float *gX, float *gY, void *ws,
                 size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * FP64 mode of the differentiated chain (checking mode): the matched-minus-
 * unmatched fixed-peak PCE gap and its gradient with respect to
 * theta = (sigma0, lambda_1..lambda_4), s_l = lambda_l sigma0^2, every step in
 * double precision on the GPU (Sec. III-B SDA frames and MLE, Sec. II-A
 * residual and correlation, Sec. IV PCE; the same chain the FP32 entry points
 * above differentiate, with 4 wavelet levels).
 *
 * cam_frames  float [ncam][m][H][W]: each camera's frames, grouped by `group`
 *             into SDA frames (the last group may be shorter).
 * queries     float [nq][H][W]; query_cam int [nq] (device): the camera of
 *             each query (matched pair) or any other value (no match).
 * theta       HOST doubles [5], finite and >= 0.
 * out         device doubles [6]: loss = mean PCE of matched pairs - mean PCE
 *             of unmatched pairs, then dL/dsigma0, dL/dlambda_1..4.
 * pce         nullable device doubles [nq][ncam].
 * H and W need prime factors <= 5 (the DFT); nbhd odd, below H and W.
 * The kernels are plain (one thread per value, direct window sums, a
 * radix-2..5 FFT, reductions in a fixed order): results are deterministic;
 * the mode is for checking gradients at full sizes, not for speed.
 * Workspace: about (6 + 2 * 3/4) * (ncam * ceil(m / group) + nq) padded
 * planes of doubles.
 */
int prnu_pce_gap_f64_workspace_size(int ncam, int m, int nq, int H, int W, int group, int taps, int nbhd,
                                    size_t *bytes);
int prnu_pce_gap_f64(const float *cam_frames, int ncam, int m, const float *queries, int nq,
                     const int *query_cam, int H, int W, int group, int taps, int nbhd,
                     const double *theta, double *out, double *pce, void *ws, size_t ws_bytes,
                     void *stream);

/* ---------------------------------------------------------------------------
 * Batched fingerprint accumulation: many cameras of different sizes, frame
 * counts and SDA group lengths in one sequence of persistent launches (the
 * SDA -> residual -> MLE chain of prnu_fingerprint_accumulate, Sec. III-B,
 * for every camera at once).
 *
 * Each camera's SDA groups are split into jobs; jobs are packed into rounds
 * whose means and wavelet pyramids fit `round_bytes` (0 = 8 GiB), at most one
 * job per camera per round.  A round is one launch per stage over all its
 * jobs: SDA means, forward levels 1..L, inverse levels L..2, and inverse
 * level 1 with the MLE fold; the level launches are persistent work queues
 * whose workgroups take (camera, plane, tile) items from a counter.
 *
 * prnu_camera   frames [n_frames][H][W][C] of the batch's dtype; A, B that
 *               camera's accumulators in the acc_mode layout (as
 *               prnu_fingerprint_accumulate).  The A and B areas of all
 *               cameras must be pairwise disjoint.
 * prnu_batch_create  validates, packs the rounds, writes the work tables into
 *               `ws` (enqueued on `stream`, then waits for that stream), and
 *               with PRNU_BATCH_GRAPH captures the whole sequence as one HIP
 *               graph.  The cameras' buffers and `ws` must stay valid and
 *               untouched while the object lives.  With PRNU_BATCH_ZERO_ACC
 *               every launch first zeroes all A and B (with a fill kernel).
 * prnu_batch_launch  enqueues the sequence (one graph launch with
 *               PRNU_BATCH_GRAPH) on `stream`; launches of one object must not
 *               overlap.
 * prnu_batch_info_get  rounds, launches, SDA frames and denoised padded
 *               pixels of the batch.
 * prnu_fingerprint_batch  create (without graph) + launch + destroy.
 */
typedef struct prnu_camera {
    const void *frames;
    int n_frames, H, W, C, group;
    void *A, *B;
} prnu_camera;

typedef struct prnu_batch_info {
    int rounds;             /* rounds of the schedule                        */
    int launches;           /* kernel launches per prnu_batch_launch         */
    int64_t jobs;           /* (camera, run of SDA groups) jobs              */
    int64_t sda_frames;     /* SDA frames formed and denoised                */
    int64_t padded_pixels;  /* sum over SDA frames of C * Hp * Wp            */
    int64_t input_bytes;    /* frame bytes read                              */
} prnu_batch_info;

typedef struct prnu_batch prnu_batch;

#define PRNU_BATCH_ZERO_ACC 1
#define PRNU_BATCH_GRAPH 2

int prnu_batch_workspace_size(const prnu_camera *cams, int n_cams, const prnu_denoise_params *p,
                              size_t round_bytes, size_t *bytes);
int prnu_batch_create(const prnu_camera *cams, int n_cams, int dtype, const prnu_denoise_params *p, int acc_mode,
                      int flags, size_t round_bytes, void *ws, size_t ws_bytes, void *stream, prnu_batch **out);
int prnu_batch_launch(prnu_batch *b, void *stream);
int prnu_batch_info_get(const prnu_batch *b, prnu_batch_info *info);
int prnu_batch_destroy(prnu_batch *b);
int prnu_fingerprint_batch(const prnu_camera *cams, int n_cams, int dtype, const prnu_denoise_params *p,
                           int acc_mode, size_t round_bytes, void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Tile shapes of the wavelet level kernels (host state, process-wide).
 *
 * This table is the library's one piece of global state: a host-side map,
 * guarded by a mutex, from (kind, filter length, subband size) to a tile
 * width.  It holds no device memory and changes only the launch shapes,
 * never the results (every tile width computes the same values).
 *
 * A forward level with shrinkage (kind PRNU_TILE_FWD) streams strips of
 * `tile` subband columns, 64 or 32 (default 64), down the plane in steps of
 * 16 coefficient rows.  The segment of rows a workgroup walks (kind
 * PRNU_TILE_SEG, the halo's amortisation) is sized from the level and the
 * batch so that each launch holds about `tile` workgroups per CU: 3, 6 or 12
 * (default 6); longer segments recompute the 4-coefficient Wiener margin
 * and the row-filter carry at segment ends less often, shorter ones fill
 * the chip more evenly.  The Wiener margin around a strip is fixed at 4
 * coefficients by the largest (9 x 9) window.  An inverse level or inverse
 * level 1 with the MLE fold (kind PRNU_TILE_INV / _MLE) works on square
 * tiles of `tile` coefficients per side, 32 or 16 (default 32).  Choices are
 * kept per filter length and subband size hk x wk.
 * prnu_set_tile: one of the kind's values, 0 restores the default;
 *   PRNU_E_INVAL for any other value.
 * prnu_autotune: for frames of H x W x C and the denoiser `p`, times both
 *   widths of every forward level, then the three segment targets at the
 *   chosen width, inverse level 2..L and the MLE fold on synthetic planes in
 *   `ws`, as many as one fingerprint-accumulation batch holds (up to 32
 *   frames: the tile is chosen at the size it runs; events on `stream`,
 *   waits for them; not under graph capture) and keeps the fastest; `tiles`
 *   (nullable, 16 ints) receives the choices: [0..3] forward levels 1..4,
 *   [4..7] inverse levels 1..4 ([4], level 1, is the MLE fold's), [8] the
 *   MLE fold, [12..15] the forward levels' segment targets; unused entries 0.
 */
#define PRNU_TILE_FWD 0
#define PRNU_TILE_INV 1
#define PRNU_TILE_MLE 2
#define PRNU_TILE_SEG 3
int prnu_get_tile(int kind, int taps, int hk, int wk);
int prnu_set_tile(int kind, int taps, int hk, int wk, int tile);
int prnu_autotune_workspace_size(int H, int W, int C, const prnu_denoise_params *p, size_t *bytes);
int prnu_autotune(int H, int W, int C, const prnu_denoise_params *p, void *ws, size_t ws_bytes, void *stream,
                  int *tiles);

/* ---------------------------------------------------------------------------
 * Kernel timing (measurement aid, off by default).
 *
 * prnu_timing_enable(1) discards earlier records and brackets every later
 * kernel launch with a pair of HIP events on the launch's stream; (0) stops.
 * prnu_timing_report() waits for the recorded events and writes one line per
 * kernel name: "name<TAB>launches<TAB>total_ms<TAB>algorithmic_bytes<TAB>
 * algorithmic_flops", where the bytes are what the algorithm must read once
 * and write once for those launches and the flops its arithmetic (0 for pure
 * data movement).  `needed` (nullable) receives the text size including the NUL;
 * PRNU_E_INVAL if `len` is too small (the text is truncated).
 */
int prnu_timing_enable(int on);
int prnu_timing_report(char *buf, size_t len, size_t *needed);

#ifdef __cplusplus
}
#endif

#endif /* PRNU_H */
