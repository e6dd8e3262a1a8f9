// C ABI of the fingerprint library: host-side validation, workspace carving
// and the launch sequences of every entry point.  Nothing here allocates
// device memory; every buffer comes from the caller.

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <climits>

#include "host.h"
#include "internal.h"

// The Python binding views prnu_acc_state as int64 [3].
static_assert(sizeof(prnu_acc_state) == 24 && offsetof(prnu_acc_state, status) == 16, "prnu_acc_state layout");

namespace prnu {

static thread_local char g_err[512];

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

namespace {

// ---- the wavelet pyramid of a batch of planes --------------------------------
struct Pyramid {
    float *lvl[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
};

void carve_pyramid(Carver &cv, int planes, int H, int W, int levels, Pyramid *py) {
    const int Hp = padded(H), Wp = padded(W);
    for (int l = 1; l <= levels; ++l) py->lvl[l] = cv.take<float>((size_t)planes * level_floats(Hp, Wp, l));
}

int batch_planes(int n, int H, int W) {
    const int64_t px = (int64_t)padded(H) * padded(W);
    int64_t nb = kBatchPixels / px;
    if (nb < 1) nb = 1;
    if (nb > n) nb = n;
    return (int)nb;
}

// Forward levels 1..L (with shrinkage) and inverse levels L..2; the caller
// runs inverse level 1 with its epilogue.
// Sensitivity checkpoint layout per plane: level 1 [3][Hp/2][Wp/2], then level 2, ...
size_t ckpt_level_offset(int H, int W, int lvl) {
    const int Hp = padded(H), Wp = padded(W);
    size_t off = 0;
    for (int l = 1; l < lvl; ++l) off += (size_t)3 * (Hp >> l) * (Wp >> l);
    return off;
}

int run_pyramid(const Filter &f, const prnu_denoise_params *p, const float *src, int planes, int H,
                int W, const Pyramid &py, hipStream_t s, float *ckpt = nullptr, const unsigned char *src8 = nullptr,
                int src8_c = 0) {
    const int Hp = padded(H), Wp = padded(W), L = p->levels;
    const float s0 = p->sigma0 * p->sigma0;
    const int64_t cstride = (int64_t)ckpt_level_offset(H, W, L + 1);
    for (int l = 1; l <= L; ++l) {
        const float s2 = p->level_weight[l - 1] * s0;
        float *ck = ckpt ? ckpt + ckpt_level_offset(H, W, l) : nullptr;
        if (l == 1) {
            PRNU_HIP(launch_dwt_fwd(p->taps, f, src, (int64_t)H * W, H, W, Hp, Wp, pad_before(H),
                                    pad_before(W), py.lvl[1], planes, s2, L > 1, s, ck, cstride, src8, src8_c));
        } else {
            const int nr = Hp >> (l - 1), nc = Wp >> (l - 1);
            PRNU_HIP(launch_dwt_fwd(p->taps, f, py.lvl[l - 1], (int64_t)level_floats(Hp, Wp, l - 1), nr,
                                    nc, nr, nc, 0, 0, py.lvl[l], planes, s2, l < L, s, ck, cstride));
        }
    }
    for (int l = L; l >= 2; --l)
        PRNU_HIP(launch_dwt_inv(p->taps, f, py.lvl[l], Hp >> l, Wp >> l, l == L, planes, INV_PLANE,
                                py.lvl[l - 1], 0, 0, 0, 0, s));
    return PRNU_OK;
}

// ---- post-processing chain (zero-mean, luma, DFT Wiener) --------------------
struct PostWs {
    double *zm = nullptr;
    float *tmp = nullptr;
    float2 *Z = nullptr, *G = nullptr, *tw_h = nullptr, *tw_w = nullptr;
    double *var = nullptr, *red = nullptr;
};

void carve_post(Carver &cv, int nf, int C, int H, int W, int flags, PostWs *pw) {
    const int nout = nf * ((C == 3 && (flags & PRNU_LUMA)) ? 1 : C);
    pw->zm = cv.take<double>(zm_scratch_doubles(nf, C, H, W));
    if (flags & PRNU_WIENER) {
        const size_t N = (size_t)H * W;
        pw->tmp = cv.take<float>((size_t)nout * N);
        pw->Z = cv.take<float2>((size_t)nout * N);
        pw->G = cv.take<float2>((size_t)nout * N);
        pw->tw_h = cv.take<float2>((size_t)H);
        pw->tw_w = cv.take<float2>((size_t)W);
        pw->var = cv.take<double>((size_t)nout);
        pw->red = cv.take<double>(reduce_scratch_doubles(nout, (int64_t)N));
    }
}

int check_fft_dims(int H, int W, const char *fn, FftPlan *ph, FftPlan *pw) {
    if (!make_fft_plan(H, ph, true) || !make_fft_plan(W, pw))
        return fail(PRNU_E_UNSUPPORTED, "%s: DFT sizes need prime factors <= 5 and <= 5120 (got %d x %d)",
                    fn, H, W);
    return PRNU_OK;
}

// Post-processing of nf frames of C planes [nf][C][H][W] into
// out [nf][nout][H][W]; every output plane gets its own Wiener variance.
int run_post(const float *in, int nf, int C, int H, int W, int flags, float sigma_wf, float *out,
             const PostWs &pw, bool twiddles_ready, hipStream_t s) {
    const int nout = nf * ((C == 3 && (flags & PRNU_LUMA)) ? 1 : C);
    const bool wf = (flags & PRNU_WIENER) != 0;
    float *dst = wf ? pw.tmp : out;
    PRNU_HIP(launch_zero_mean(in, nf, C, H, W, (flags & PRNU_ZM) != 0, C == 3 && (flags & PRNU_LUMA), dst,
                              pw.zm, s));
    if (!wf) return PRNU_OK;
    FftPlan ph, pwl;
    PRNU_TRY(check_fft_dims(H, W, "post", &ph, &pwl));
    const int64_t N = (int64_t)H * W;
    if (!twiddles_ready) {
        PRNU_HIP(launch_twiddles(H, pw.tw_h, s));
        PRNU_HIP(launch_twiddles(W, pw.tw_w, s));
    }
    if (sigma_wf < 0.f) PRNU_HIP(launch_plane_variance(dst, nout, N, pw.var, pw.red, s));
    // the forward rows pass reads the real planes, the inverse columns pass
    // stores the real part, scaled by 1/N
    PRNU_HIP(launch_fft2(pw.Z, nout, H, W, ph, pwl, pw.tw_h, pw.tw_w, -1, s, dst));
    PRNU_HIP(launch_spectral_wiener(pw.Z, nout, H, W, pw.var, sigma_wf < 0.f ? -1.f : sigma_wf * sigma_wf,
                                    pw.G, s));
    PRNU_HIP(launch_fft2(pw.G, nout, H, W, ph, pwl, pw.tw_h, pw.tw_w, +1, s, nullptr, out,
                         (float)(1.0 / (double)N)));
    return PRNU_OK;
}

// ---- entry point plans ---------------------------------------------------
int plan_denoise(Carver &cv, int n_img, int H, int W, const prnu_denoise_params *p, Pyramid *py,
                 int *nb, int max_nb = 0) {
    *nb = batch_planes(n_img, H, W);
    if (max_nb > 0 && *nb > max_nb) *nb = max_nb;
    carve_pyramid(cv, *nb, H, W, p->levels, py);
    return PRNU_OK;
}

int frames_per_batch(int g, int H, int W, int C) {
    const int64_t px = (int64_t)C * padded(H) * padded(W);
    int64_t nb = kAccBatchPixels / px;
    if (nb < 1) nb = 1;
    if (nb > kMaxFramesPerMle) nb = kMaxFramesPerMle;
    if (nb > g) nb = g;
    return (int)nb;
}

struct AccPlan {
    int nb;
    float *means;
    Pyramid py;
};

void plan_accumulate(Carver &cv, int n_frames, int H, int W, int C, int group,
                     const prnu_denoise_params *p, AccPlan *ap) {
    const int g = (n_frames + group - 1) / group;
    ap->nb = frames_per_batch(g, H, W, C);
    ap->means = cv.take<float>((size_t)ap->nb * C * H * W);
    carve_pyramid(cv, ap->nb * C, H, W, p->levels, &ap->py);
}

struct QueryPlan {
    int nb;
    float *means, *resid;
    Pyramid py;
    PostWs post;
};

void plan_query(Carver &cv, int n, int H, int W, int C, const prnu_denoise_params *p, int flags,
                QueryPlan *qp) {
    qp->nb = frames_per_batch(n, H, W, C);
    qp->means = cv.take<float>((size_t)qp->nb * C * H * W);
    qp->resid = cv.take<float>((size_t)qp->nb * C * H * W);
    carve_pyramid(cv, qp->nb * C, H, W, p->levels, &qp->py);
    carve_post(cv, qp->nb, C, H, W, flags, &qp->post);
}

constexpr int64_t kPceChunkBytes = 512ll << 20;

struct PcePlan {
    int P;
    float2 *tw_h, *tw_w, *Xs, *Ys, *Z;
    double *xmean, *xn2, *ymean, *yn2, *spart;
    void *ppart;
    // fixed-peak fast path
    bool fast = false;
    int Mc = 0;
    float2 *tw_half = nullptr;
    float *Px = nullptr, *Py = nullptr;
    double *dpart = nullptr, *cpart = nullptr;
};

bool pce_fast_ok(int h, int w, int peak_mode, int nbhd) {
    FftPlan a, b;
    return peak_mode == PRNU_PEAK_FIXED_00 && nbhd <= 11 && (w % 2) == 0 && make_fft_plan(h, &a) &&
           make_fft_plan(w / 2, &b) && make_fft_plan(w, &b);
}

// Fingerprints per query from which the matrix-core direct sums pay off.
constexpr int kMfmaMinFingerprints = 3;
constexpr int64_t kMfmaPartDoubles = 8ll << 20;  // direct-sum partials per query chunk (64 MiB)

// Queries per chunk of the matrix-core direct sums.
int mfma_query_chunk(int nx, int ny, int nblk) {
    int64_t qc = kMfmaPartDoubles / ((int64_t)ny * nblk * kPceDirectStats);
    if (qc < 1) qc = 1;
    if (qc > nx) qc = nx;
    if (qc > 65535) qc = 65535;
    return (int)qc;
}

void plan_pce_fast(Carver &cv, int nx, int ny, int h, int w, bool modulated, PcePlan *pp) {
    const int64_t N = (int64_t)h * w;
    const int Mc = w / 2 + 1;
    const int64_t S = (int64_t)h * Mc;
    const int64_t npairs = (int64_t)nx * ny;
    int64_t P = kPceChunkBytes / (S * (int64_t)sizeof(float2));
    if (P < 1) P = 1;
    if (P > 64) P = 64;
    if (P > npairs) P = npairs;
    int64_t Pq = P;  // planes per chunk when preparing the query / fingerprint spectra
    FftPlan pc;  // the column transform's plan fixes the column-group layout of the half spectra
    make_fft_plan(h, &pc, true);
    const int64_t Sg = half_plane_elems(h, Mc, pc);
    pp->fast = true;
    pp->P = (int)P;
    pp->Mc = Mc;
    pp->tw_h = cv.take<float2>((size_t)h);
    pp->tw_w = cv.take<float2>((size_t)w);
    pp->tw_half = cv.take<float2>((size_t)(w / 2));
    pp->Px = cv.take<float>((size_t)nx * Sg);
    pp->Py = modulated ? nullptr : cv.take<float>((size_t)ny * Sg);
    pp->Z = cv.take<float2>((size_t)(P > Pq ? P : Pq) * Sg);
    pp->xmean = cv.take<double>((size_t)nx);
    pp->xn2 = cv.take<double>((size_t)nx);
    pp->ymean = cv.take<double>((size_t)ny);
    pp->yn2 = cv.take<double>((size_t)ny);
    int mx = nx > ny ? nx : ny;
    pp->spart = cv.take<double>(stats_part_doubles(mx));
    size_t dpart = pce_direct_part_doubles((int)P, h, w);
    int64_t cpairs = P;  // pairs whose energy partials are held at once
    if (ny >= kMfmaMinFingerprints) {
        const int nbm = pce_mfma_blocks(nx, ny, h, w);
        const int qc = mfma_query_chunk(nx, ny, nbm);
        const size_t m = (size_t)qc * ny * nbm * kPceDirectStats;
        if (m > dpart) dpart = m;
        if ((int64_t)qc * ny > cpairs) cpairs = (int64_t)qc * ny;  // a whole query chunk, finished at once
    }
    pp->dpart = cv.take<double>(dpart);
    FftPlan ph;
    make_fft_plan(h, &ph, true);
    const int ncb = fft_cols_power_blocks(Mc, ph);
    const int nsb = ncb > pce_dot_blocks() ? ncb : pce_dot_blocks();
    pp->cpart = cv.take<double>((size_t)cpairs * nsb);
    (void)N;
}

void plan_pce(Carver &cv, int nx, int ny, int h, int w, bool modulated, PcePlan *pp) {
    const int64_t N = (int64_t)h * w;
    const int64_t npairs = (int64_t)nx * ny;
    int64_t P = kPceChunkBytes / (N * (int64_t)sizeof(float2));
    if (P < 1) P = 1;
    if (P > 64) P = 64;
    if (P > npairs) P = npairs;
    pp->P = (int)P;
    pp->tw_h = cv.take<float2>((size_t)h);
    pp->tw_w = cv.take<float2>((size_t)w);
    pp->Xs = cv.take<float2>((size_t)nx * N);
    pp->Ys = modulated ? nullptr : cv.take<float2>((size_t)ny * N);
    pp->Z = cv.take<float2>((size_t)P * N);
    pp->xmean = cv.take<double>((size_t)nx);
    pp->xn2 = cv.take<double>((size_t)nx);
    const int ycount = modulated ? (int)P : ny;
    pp->ymean = cv.take<double>((size_t)ycount);
    pp->yn2 = cv.take<double>((size_t)ycount);
    int mx = nx > ny ? nx : ny;
    if ((int)P > mx) mx = (int)P;
    pp->spart = cv.take<double>(stats_part_doubles(mx));
    pp->ppart = cv.take<char>(pce_part_bytes((int)P));
}


struct VjpPlan {
    int nb;
    float *ll[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    double *part;
};

void plan_vjp(Carver &cv, int n, int H, int W, const prnu_denoise_params *p, VjpPlan *vp) {
    vp->nb = batch_planes(n, H, W);
    const int Hp = padded(H), Wp = padded(W);
    for (int l = 1; l < p->levels; ++l) vp->ll[l] = cv.take<float>((size_t)vp->nb * (Hp >> l) * (Wp >> l));
    vp->part = cv.take<double>((size_t)vp->nb * dwt_vjp_tiles(Hp / 2, Wp / 2));
}

struct PvjpPlan {
    int P;
    float2 *tw_h, *tw_w, *Xs, *V, *Z, *T1, *T2;
    double *xmean, *xn2, *ymean, *yn2, *spart;
    void *coef;
};

void plan_pvjp(Carver &cv, int nx, int ny, int h, int w, PvjpPlan *pl) {
    const int64_t N = (int64_t)h * w;
    const int64_t npairs = (int64_t)nx * ny;
    int64_t P = kPceChunkBytes / (4 * N * (int64_t)sizeof(float2));
    if (P < 1) P = 1;
    if (P > 64) P = 64;
    if (P > npairs) P = npairs;
    pl->P = (int)P;
    pl->tw_h = cv.take<float2>((size_t)h);
    pl->tw_w = cv.take<float2>((size_t)w);
    pl->Xs = cv.take<float2>((size_t)nx * N);
    pl->V = cv.take<float2>((size_t)P * N);
    pl->Z = cv.take<float2>((size_t)P * N);
    pl->T1 = cv.take<float2>((size_t)P * N);
    pl->T2 = cv.take<float2>((size_t)P * N);
    pl->xmean = cv.take<double>((size_t)nx);
    pl->xn2 = cv.take<double>((size_t)nx);
    pl->ymean = cv.take<double>((size_t)P);
    pl->yn2 = cv.take<double>((size_t)P);
    pl->spart = cv.take<double>(stats_part_doubles(nx > (int)P ? nx : (int)P));
    pl->coef = cv.take<char>(pvjp_coef_bytes((int)P));
}

// Fixed-peak PCE: C(0) and the shifts around it are direct sums; the total
// energy of the surface is (1/N) sum_k |X_k|^2 |Y_k|^2 (Parseval), so no
// inverse transform is needed.
int pce_fixed_fast(const float *X, int nx, const float *Y, int ny, int h, int w, const float *mod, int nbhd,
                   double *pce, double *ncc, int32_t *peak, const PcePlan &pl, hipStream_t s) {
    const int64_t N = (int64_t)h * w;
    const int Mc = pl.Mc;
    // the half-length row transforms take as many rows per workgroup as the
    // column transforms take columns (up to twice the default): their stores
    // into the column-group layout then fill whole cache lines
    FftPlan ph, phalf;
    make_fft_plan(h, &ph, true);
    make_fft_plan(w / 2, &phalf, true);
    PRNU_HIP(launch_twiddles(h, pl.tw_h, s));
    PRNU_HIP(launch_twiddles(w, pl.tw_w, s));
    PRNU_HIP(launch_twiddles(w / 2, pl.tw_half, s));
    // query statistics (the centred norms serve the NCC only) and power
    // spectra |X^|^2 of the centred queries
    PRNU_HIP(launch_pair_stats(X, nullptr, INT_MAX, 0, nx, N, pl.xmean, ncc ? pl.xn2 : nullptr, pl.spart, s));
    const int64_t S = half_plane_elems(h, Mc, ph);  // column-group layout of ph
    for (int q0 = 0; q0 < nx; q0 += pl.P) {
        const int n = nx - q0 < pl.P ? nx - q0 : pl.P;
        PRNU_HIP(launch_rfft_rows(X, nullptr, INT_MAX, q0, n, pl.xmean + q0, h, w, phalf, pl.tw_half, pl.tw_w,
                                  ph, pl.Z, s));
        PRNU_HIP(launch_fft_cols_power(pl.Z, n, h, Mc, ph, pl.tw_h, nullptr, 1, 0, pl.Px + q0 * S, nullptr, s));
    }
    if (!mod) {
        for (int j0 = 0; j0 < ny; j0 += pl.P) {
            const int n = ny - j0 < pl.P ? ny - j0 : pl.P;
            PRNU_HIP(launch_rfft_rows(Y, nullptr, INT_MAX, j0, n, nullptr, h, w, phalf, pl.tw_half, pl.tw_w,
                                      ph, pl.Z, s));
            PRNU_HIP(launch_fft_cols_power(pl.Z, n, h, Mc, ph, pl.tw_h, nullptr, 1, 0, pl.Py + j0 * S, nullptr,
                                           s));
        }
    }
    // energy partials per pair: nbs doubles each
    const int nbs = mod ? fft_cols_power_blocks(Mc, ph) : pce_dot_blocks();
    // energy of the pairs p0 .. p0+n-1 into cp [n][nbs]
    auto energy = [&](int64_t p0, int n, double *cp) -> int {
        if (mod) {
            PRNU_HIP(launch_rfft_rows(Y, mod, ny, (int)p0, n, nullptr, h, w, phalf, pl.tw_half, pl.tw_w, ph, pl.Z,
                                      s));
            PRNU_HIP(launch_fft_cols_power(pl.Z, n, h, Mc, ph, pl.tw_h, pl.Px, ny, (int)p0, nullptr, cp, s));
        } else {
            PRNU_HIP(launch_power_dot(pl.Px, pl.Py, ny, (int)p0, n, h, Mc, ph.lvec, cp, s));
        }
        return PRNU_OK;
    };
    if (ny >= kMfmaMinFingerprints) {
        // direct sums of every fingerprint of a chunk of queries on the matrix cores
        const int nbm = pce_mfma_blocks(nx, ny, h, w);
        const int qc = mfma_query_chunk(nx, ny, nbm);
        for (int q0 = 0; q0 < nx; q0 += qc) {
            const int nq = nx - q0 < qc ? nx - q0 : qc;
            PRNU_HIP(launch_pce_direct_mfma(X, pl.xmean, Y, mod, ny, q0, nq, h, w, nbm, ncc != nullptr, pl.dpart, s));
            const int64_t pa = (int64_t)q0 * ny, pb = (int64_t)(q0 + nq) * ny;
            // the energies of the chunk's pairs, P at a time, then one finish for all of them
            for (int64_t p0 = pa; p0 < pb; p0 += pl.P) {
                const int n = (int)(pb - p0 < pl.P ? pb - p0 : pl.P);
                PRNU_TRY(energy(p0, n, pl.cpart + (p0 - pa) * nbs));
            }
            PRNU_HIP(launch_pce_finish_fixed(pl.dpart, nbm, pl.cpart, nbs, (int)(pb - pa), h, w, nbhd, pl.xn2, ny,
                                             (int)pa, pce, ncc, peak, s));
        }
        return PRNU_OK;
    }
    const int64_t npairs = (int64_t)nx * ny;
    const int nbd = pce_direct_blocks(h, w);
    for (int64_t p0 = 0; p0 < npairs; p0 += pl.P) {
        const int n = (int)(npairs - p0 < pl.P ? npairs - p0 : pl.P);
        PRNU_TRY(energy(p0, n, pl.cpart));
        PRNU_HIP(launch_pce_direct(X, pl.xmean, Y, mod, ny, (int)p0, n, h, w, pl.dpart, s));
        PRNU_HIP(launch_pce_finish_fixed(pl.dpart, nbd, pl.cpart, nbs, n, h, w, nbhd, pl.xn2, ny, (int)p0, pce, ncc,
                                         peak, s));
    }
    return PRNU_OK;
}

}  // namespace
}  // namespace prnu

using namespace prnu;

extern "C" {

const char *prnu_last_error(void) { return g_err; }

const char *prnu_version(void) { return "prnu-mi355x 0.1 (gfx950)"; }

void prnu_default_denoise_params(prnu_denoise_params *p) {
    if (!p) return;
    p->sigma0 = 3.0f;
    p->levels = 4;
    p->taps = 16;
    for (int l = 0; l < 4; ++l) p->level_weight[l] = 1.0f;
}

int prnu_sda_average(const void *frames, int dtype, int n_frames, int H, int W, int C, int64_t frame_stride_bytes,
                     int group, uint32_t *sums, float *means, int *counts, uint32_t *status, void *stream) {
    const char *fn = "prnu_sda_average";
    set_error("");
    PRNU_TRY(check_frames(frames, dtype, n_frames, C, fn));
    if (H < 1 || W < 1 || H > kMaxDim || W > kMaxDim) return fail(PRNU_E_INVAL, "%s: bad H x W", fn);
    int64_t fstride;
    PRNU_TRY(check_frame_stride(frame_stride_bytes, dtype, n_frames, H, W, C, fn, &fstride));
    if (group < 1) return fail(PRNU_E_INVAL, "%s: group must be >= 1", fn);
    if (!sums && !means) return fail(PRNU_E_INVAL, "%s: need sums or means", fn);
    if (sums && dtype != PRNU_U8) return fail(PRNU_E_INVAL, "%s: integer sums need u8 frames", fn);
    if (n_frames > 16843009) return fail(PRNU_E_INVAL, "%s: too many frames for u32 sums", fn);
    const int g = (n_frames + group - 1) / group;
    PRNU_HIP(launch_sda(frames, fstride, dtype, n_frames, H, W, C, group, 0, g, sums, means, counts, status,
                        (hipStream_t)stream));
    return PRNU_OK;
}

int prnu_denoise_residual_workspace_size(int n_img, int H, int W, const prnu_denoise_params *p,
                                         size_t *bytes) {
    const char *fn = "prnu_denoise_residual_workspace_size";
    set_error("");
    if (!bytes) return fail(PRNU_E_INVAL, "%s: null output", fn);
    if (n_img < 1) return fail(PRNU_E_INVAL, "%s: n_img must be >= 1", fn);
    PRNU_TRY(check_dims(H, W, fn));
    PRNU_TRY(check_params(p, fn));
    Carver cv(nullptr);
    Pyramid py;
    int nb;
    plan_denoise(cv, n_img, H, W, p, &py, &nb);
    *bytes = cv.off;
    return PRNU_OK;
}

int prnu_denoise_residual(const float *img, int n_img, int H, int W, const prnu_denoise_params *p,
                          float *resid, void *ws, size_t ws_bytes, void *stream) {
    return denoise_run("prnu_denoise_residual", img, n_img, H, W, p, resid, nullptr, ws, ws_bytes, stream);
}

int prnu_denoise_ckpt_floats(int H, int W, int levels, size_t *floats) {
    set_error("");
    if (!floats) return fail(PRNU_E_INVAL, "prnu_denoise_ckpt_floats: null output");
    if (H < 16 || W < 16 || H > kMaxDim || W > kMaxDim || levels < 1 || levels > 4)
        return fail(PRNU_E_INVAL, "prnu_denoise_ckpt_floats: bad size or levels");
    *floats = ckpt_level_offset(H, W, levels + 1);
    return PRNU_OK;
}

int prnu_denoise_residual_ckpt(const float *img, int n_img, int H, int W, const prnu_denoise_params *p,
                               float *resid, float *ckpt, void *ws, size_t ws_bytes, void *stream) {
    if (!ckpt) return fail(PRNU_E_INVAL, "prnu_denoise_residual_ckpt: null checkpoint");
    return denoise_run("prnu_denoise_residual_ckpt", img, n_img, H, W, p, resid, ckpt, ws, ws_bytes, stream);
}

}  // extern "C"

namespace prnu {

int denoise_run(const char *fn, const float *img, int n_img, int H, int W, const prnu_denoise_params *p,
                float *resid, float *ckpt, void *ws, size_t ws_bytes, void *stream, int max_nb) {
    set_error("");
    if (!img || !resid) return fail(PRNU_E_INVAL, "%s: null pointer", fn);
    if (img == resid) return fail(PRNU_E_INVAL, "%s: resid may not alias img", fn);
    if (n_img < 1) return fail(PRNU_E_INVAL, "%s: n_img must be >= 1", fn);
    PRNU_TRY(check_dims(H, W, fn));
    PRNU_TRY(check_params(p, fn));
    Carver cv(nullptr);
    Pyramid py;
    int nb;
    plan_denoise(cv, n_img, H, W, p, &py, &nb, max_nb);
    PRNU_TRY(check_ws(cv, ws, ws_bytes, fn));
    Carver real(ws);
    plan_denoise(real, n_img, H, W, p, &py, &nb, max_nb);
    Filter f;
    make_filter(p->taps, &f);
    hipStream_t s = (hipStream_t)stream;
    const int Hp = padded(H), Wp = padded(W);
    const int64_t plane = (int64_t)H * W;
    const size_t cplane = ckpt_level_offset(H, W, p->levels + 1);
    for (int b0 = 0; b0 < n_img; b0 += nb) {
        const int n = n_img - b0 < nb ? n_img - b0 : nb;
        PRNU_TRY(run_pyramid(f, p, img + b0 * plane, n, H, W, py, s, ckpt ? ckpt + (size_t)b0 * cplane : nullptr));
        PRNU_HIP(launch_dwt_inv(p->taps, f, py.lvl[1], Hp / 2, Wp / 2, p->levels == 1, n, INV_RESID,
                                resid + b0 * plane, H, W, pad_before(H), pad_before(W), s));
    }
    return PRNU_OK;
}

int denoise_planes_fitting(int H, int W, const prnu_denoise_params *p, size_t bytes) {
    // the pyramid of nb planes, each level 256-byte aligned, must fit `bytes`
    const int Hp = padded(H), Wp = padded(W);
    size_t per = 0;
    for (int l = 1; l <= p->levels; ++l) per += level_floats(Hp, Wp, l) * sizeof(float);
    const size_t slack = (size_t)p->levels * kAlign;
    if (bytes <= slack || per > bytes - slack) return 0;
    int64_t nb = (int64_t)((bytes - slack) / per);
    if (nb > 0x7fffffff) nb = 0x7fffffff;
    for (; nb > 0; --nb) {
        Carver cv(nullptr);
        Pyramid py;
        carve_pyramid(cv, (int)nb, H, W, p->levels, &py);
        if (cv.off <= bytes) break;
    }
    return (int)nb;
}

}  // namespace prnu

extern "C" {

int prnu_fingerprint_accumulate_workspace_size(int n_frames, int H, int W, int C, int group,
                                               const prnu_denoise_params *p, size_t *bytes) {
    const char *fn = "prnu_fingerprint_accumulate_workspace_size";
    set_error("");
    if (!bytes) return fail(PRNU_E_INVAL, "%s: null output", fn);
    if (n_frames < 1 || group < 1) return fail(PRNU_E_INVAL, "%s: n_frames and group must be >= 1", fn);
    if (C != 1 && C != 3) return fail(PRNU_E_INVAL, "%s: C must be 1 or 3", fn);
    PRNU_TRY(check_dims(H, W, fn));
    PRNU_TRY(check_mle_pixels(H, W, fn));
    PRNU_TRY(check_params(p, fn));
    Carver cv(nullptr);
    AccPlan ap;
    plan_accumulate(cv, n_frames, H, W, C, group, p, &ap);
    *bytes = cv.off;
    return PRNU_OK;
}

int prnu_fingerprint_accumulate(const void *frames, int dtype, int n_frames, int H, int W, int C,
                                int64_t frame_stride_bytes, int group, const prnu_denoise_params *p, int acc_mode,
                                void *A, void *B, prnu_acc_state *state, void *ws, size_t ws_bytes, void *stream) {
    const char *fn = "prnu_fingerprint_accumulate";
    set_error("");
    PRNU_TRY(check_frames(frames, dtype, n_frames, C, fn));
    PRNU_TRY(check_dims(H, W, fn));
    PRNU_TRY(check_mle_pixels(H, W, fn));
    int64_t fstride;
    PRNU_TRY(check_frame_stride(frame_stride_bytes, dtype, n_frames, H, W, C, fn, &fstride));
    PRNU_TRY(check_params(p, fn));
    if (group < 1) return fail(PRNU_E_INVAL, "%s: group must be >= 1", fn);
    if (acc_mode != PRNU_ACC_F64 && acc_mode != PRNU_ACC_KAHAN_F32 && acc_mode != PRNU_ACC_F32)
        return fail(PRNU_E_INVAL, "%s: unknown acc_mode %d", fn, acc_mode);
    if (!A || !B) return fail(PRNU_E_INVAL, "%s: null accumulator", fn);
    if (n_frames > 16843009) return fail(PRNU_E_INVAL, "%s: too many frames", fn);
    Carver cv(nullptr);
    AccPlan ap;
    plan_accumulate(cv, n_frames, H, W, C, group, p, &ap);
    PRNU_TRY(check_ws(cv, ws, ws_bytes, fn));
    Carver real(ws);
    plan_accumulate(real, n_frames, H, W, C, group, p, &ap);
    Filter f;
    make_filter(p->taps, &f);
    hipStream_t s = (hipStream_t)stream;
    const int g = (n_frames + group - 1) / group;
    const int Hp = padded(H), Wp = padded(W);
    // SDA depth 1 on dense u8 frames: the means are the frames themselves
    // (exact in float), so the level-1 forward and the MLE fold read the
    // frames directly
    const bool direct = group == 1 && dtype == PRNU_U8 && fstride == (int64_t)H * W * C;
    uint32_t *status = state ? &state->status : nullptr;
    for (int g0 = 0; g0 < g; g0 += ap.nb) {
        const int g1 = g0 + ap.nb < g ? g0 + ap.nb : g;
        const int nb = g1 - g0;
        const unsigned char *f8 = direct ? static_cast<const unsigned char *>(frames) + (int64_t)g0 * fstride : nullptr;
        if (!direct)
            PRNU_HIP(launch_sda(frames, fstride, dtype, n_frames, H, W, C, group, g0, g1, nullptr, ap.means, nullptr,
                                status, s));
        PRNU_TRY(run_pyramid(f, p, ap.means, nb * C, H, W, ap.py, s, nullptr, f8, C));
        PRNU_HIP(launch_dwt_inv_mle(p->taps, f, ap.py.lvl[1], Hp / 2, Wp / 2, p->levels == 1, nb, C,
                                    ap.means, H, W, pad_before(H), pad_before(W), acc_mode, A, B, s, f8));
        if (state) {
            const int64_t fr = std::min<int64_t>(n_frames, (int64_t)g1 * group) - (int64_t)g0 * group;
            PRNU_HIP(launch_acc_state_add(state, fr, nb, s));
        }
    }
    return PRNU_OK;
}

int prnu_fingerprint_finalize_workspace_size(int C, int H, int W, int flags, size_t *bytes) {
    const char *fn = "prnu_fingerprint_finalize_workspace_size";
    set_error("");
    if (!bytes) return fail(PRNU_E_INVAL, "%s: null output", fn);
    if (C != 1 && C != 3) return fail(PRNU_E_INVAL, "%s: C must be 1 or 3", fn);
    if (H < 1 || W < 1 || H > kMaxDim || W > kMaxDim) return fail(PRNU_E_INVAL, "%s: bad H x W", fn);
    PRNU_TRY(check_flags(flags, fn));
    Carver cv(nullptr);
    cv.take<float>((size_t)C * H * W);
    PostWs pw;
    carve_post(cv, 1, C, H, W, flags, &pw);
    *bytes = cv.off;
    return PRNU_OK;
}

int prnu_fingerprint_finalize(const void *A, const void *B, int acc_mode, int C, int H, int W, int flags,
                              float sigma_wf, float *K, void *ws, size_t ws_bytes, void *stream) {
    const char *fn = "prnu_fingerprint_finalize";
    set_error("");
    if (!A || !B || !K) return fail(PRNU_E_INVAL, "%s: null pointer", fn);
    if (C != 1 && C != 3) return fail(PRNU_E_INVAL, "%s: C must be 1 or 3", fn);
    if (H < 1 || W < 1 || H > kMaxDim || W > kMaxDim) return fail(PRNU_E_INVAL, "%s: bad H x W", fn);
    if (acc_mode != PRNU_ACC_F64 && acc_mode != PRNU_ACC_KAHAN_F32 && acc_mode != PRNU_ACC_F32)
        return fail(PRNU_E_INVAL, "%s: unknown acc_mode %d", fn, acc_mode);
    PRNU_TRY(check_flags(flags, fn));
    if (!std::isfinite(sigma_wf)) return fail(PRNU_E_INVAL, "%s: sigma_wf must be finite", fn);
    if (flags & PRNU_WIENER) {
        FftPlan a, b;
        PRNU_TRY(check_fft_dims(H, W, fn, &a, &b));
    }
    Carver cv(nullptr);
    cv.take<float>((size_t)C * H * W);
    PostWs pw;
    carve_post(cv, 1, C, H, W, flags, &pw);
    PRNU_TRY(check_ws(cv, ws, ws_bytes, fn));
    Carver real(ws);
    float *Kc = real.take<float>((size_t)C * H * W);
    carve_post(real, 1, C, H, W, flags, &pw);
    hipStream_t s = (hipStream_t)stream;
    PRNU_HIP(launch_ratio(A, B, acc_mode, (int64_t)C * H * W, Kc, s));
    return run_post(Kc, 1, C, H, W, flags, sigma_wf, K, pw, false, s);
}

int prnu_query_residual_workspace_size(int n, int H, int W, int C, const prnu_denoise_params *p, int flags,
                                       size_t *bytes) {
    const char *fn = "prnu_query_residual_workspace_size";
    set_error("");
    if (!bytes) return fail(PRNU_E_INVAL, "%s: null output", fn);
    if (n < 1) return fail(PRNU_E_INVAL, "%s: n must be >= 1", fn);
    if (C != 1 && C != 3) return fail(PRNU_E_INVAL, "%s: C must be 1 or 3", fn);
    PRNU_TRY(check_dims(H, W, fn));
    PRNU_TRY(check_params(p, fn));
    PRNU_TRY(check_flags(flags, fn));
    Carver cv(nullptr);
    QueryPlan qp;
    plan_query(cv, n, H, W, C, p, flags, &qp);
    *bytes = cv.off;
    return PRNU_OK;
}

int prnu_query_residual(const void *frames, int dtype, int n, int H, int W, int C,
                        const prnu_denoise_params *p, int flags, float *Wq, float *Iq, void *ws,
                        size_t ws_bytes, void *stream) {
    const char *fn = "prnu_query_residual";
    set_error("");
    PRNU_TRY(check_frames(frames, dtype, n, C, fn));
    PRNU_TRY(check_dims(H, W, fn));
    PRNU_TRY(check_params(p, fn));
    PRNU_TRY(check_flags(flags, fn));
    if (!Wq) return fail(PRNU_E_INVAL, "%s: null Wq", fn);
    if (flags & PRNU_WIENER) {
        FftPlan a, b;
        PRNU_TRY(check_fft_dims(H, W, fn, &a, &b));
    }
    Carver cv(nullptr);
    QueryPlan qp;
    plan_query(cv, n, H, W, C, p, flags, &qp);
    PRNU_TRY(check_ws(cv, ws, ws_bytes, fn));
    Carver real(ws);
    plan_query(real, n, H, W, C, p, flags, &qp);
    Filter f;
    make_filter(p->taps, &f);
    hipStream_t s = (hipStream_t)stream;
    const int Hp = padded(H), Wp = padded(W);
    const int64_t plane = (int64_t)H * W;
    const int nout = (C == 3 && (flags & PRNU_LUMA)) ? 1 : C;
    bool tw_ready = false;
    for (int f0 = 0; f0 < n; f0 += qp.nb) {
        const int f1 = f0 + qp.nb < n ? f0 + qp.nb : n;
        const int nb = f1 - f0;
        PRNU_HIP(launch_sda(frames, (int64_t)H * W * C * (int64_t)elem_bytes(dtype), dtype, n, H, W, C, 1, f0, f1,
                            nullptr, qp.means, nullptr, nullptr, s));
        PRNU_TRY(run_pyramid(f, p, qp.means, nb * C, H, W, qp.py, s));
        PRNU_HIP(launch_dwt_inv(p->taps, f, qp.py.lvl[1], Hp / 2, Wp / 2, p->levels == 1, nb * C, INV_RESID,
                                qp.resid, H, W, pad_before(H), pad_before(W), s));
        PRNU_TRY(run_post(qp.resid, nb, C, H, W, flags, -1.f, Wq + (int64_t)f0 * nout * plane, qp.post,
                          tw_ready, s));
        tw_ready = (flags & PRNU_WIENER) != 0;
        if (Iq) {
            const char *fb = static_cast<const char *>(frames) + (size_t)f0 * plane * C * elem_bytes(dtype);
            PRNU_HIP(launch_luma_frames(fb, dtype, nb, H, W, C, Iq + (int64_t)f0 * plane, s));
        }
    }
    return PRNU_OK;
}

int prnu_extract_blocks(const float *src, int n, int H, int W, int b, float *out, void *stream) {
    const char *fn = "prnu_extract_blocks";
    set_error("");
    if (!src || !out) return fail(PRNU_E_INVAL, "%s: null pointer", fn);
    if (n < 1) return fail(PRNU_E_INVAL, "%s: n must be >= 1", fn);
    if (H < 1 || W < 1 || H > kMaxDim || W > kMaxDim) return fail(PRNU_E_INVAL, "%s: bad H x W", fn);
    if (b < 1 || b > H || b > W) return fail(PRNU_E_INVAL, "%s: block side must be in [1, min(H, W)]", fn);
    if ((int64_t)(H / b) * (W / b) * n > 0x7fffffff)
        return fail(PRNU_E_INVAL, "%s: too many blocks x planes", fn);
    PRNU_HIP(launch_extract_blocks(src, n, H, W, b, out, (hipStream_t)stream));
    return PRNU_OK;
}

int prnu_resample_bilinear(const float *src, int n, int H, int W, double scale, int oy, int ox, int oh, int ow,
                           float *out, void *stream) {
    const char *fn = "prnu_resample_bilinear";
    set_error("");
    if (!src || !out) return fail(PRNU_E_INVAL, "%s: null pointer", fn);
    if (n < 1 || n > 65535) return fail(PRNU_E_INVAL, "%s: n must be in [1, 65535]", fn);
    if (H < 1 || W < 1 || H > kMaxDim || W > kMaxDim) return fail(PRNU_E_INVAL, "%s: bad H x W", fn);
    if (oh < 1 || ow < 1 || oh > kMaxDim || ow > kMaxDim) return fail(PRNU_E_INVAL, "%s: bad output size", fn);
    if (!std::isfinite(scale) || scale <= 0.0) return fail(PRNU_E_INVAL, "%s: scale must be finite and > 0", fn);
    if (oy < 0 || ox < 0 || oy > kMaxDim || ox > kMaxDim) return fail(PRNU_E_INVAL, "%s: bad crop offset", fn);
    PRNU_HIP(launch_resample_bilinear(src, n, H, W, scale, oy, ox, oh, ow, out, (hipStream_t)stream));
    return PRNU_OK;
}

int prnu_warp_affine(const float *src, int n_src, int H, int W, const double *affine, int n, int oh, int ow,
                     float *out, void *stream) {
    const char *fn = "prnu_warp_affine";
    set_error("");
    if (!src || !affine || !out) return fail(PRNU_E_INVAL, "%s: null pointer", fn);
    if (n_src < 1 || n < 1 || n > 65535) return fail(PRNU_E_INVAL, "%s: need n_src >= 1 and n in [1, 65535]", fn);
    if (H < 1 || W < 1 || H > kMaxDim || W > kMaxDim) return fail(PRNU_E_INVAL, "%s: bad H x W", fn);
    if (oh < 1 || ow < 1 || oh > kMaxDim || ow > kMaxDim) return fail(PRNU_E_INVAL, "%s: bad output size", fn);
    PRNU_HIP(launch_warp_affine(src, n_src, H, W, affine, n, oh, ow, out, (hipStream_t)stream));
    return PRNU_OK;
}

int prnu_pce_match_workspace_size(int nx, int ny, int h, int w, int modulated, size_t *bytes) {
    const char *fn = "prnu_pce_match_workspace_size";
    set_error("");
    if (!bytes) return fail(PRNU_E_INVAL, "%s: null output", fn);
    if (nx < 1 || ny < 1 || h < 1 || w < 1) return fail(PRNU_E_INVAL, "%s: bad sizes", fn);
    if ((int64_t)h * w > (int64_t)INT_MAX) return fail(PRNU_E_INVAL, "%s: surface too large", fn);
    // the size covers both the shift-search path and the fixed-peak path
    Carver cv(nullptr);
    PcePlan pp;
    plan_pce(cv, nx, ny, h, w, modulated != 0, &pp);
    size_t need = cv.off;
    if (pce_fast_ok(h, w, PRNU_PEAK_FIXED_00, 11)) {
        Carver cf(nullptr);
        plan_pce_fast(cf, nx, ny, h, w, modulated != 0, &pp);
        if (cf.off > need) need = cf.off;
    }
    *bytes = need;
    return PRNU_OK;
}

int prnu_pce_match(const float *X, int nx, const float *Y, int ny, int h, int w, const float *modulate,
                   const prnu_pce_params *pp_, double *pce, double *ncc, int32_t *peak, void *ws,
                   size_t ws_bytes, void *stream) {
    const char *fn = "prnu_pce_match";
    set_error("");
    if (!X || !Y || !pce || !pp_) return fail(PRNU_E_INVAL, "%s: null pointer", fn);
    if (nx < 1 || ny < 1) return fail(PRNU_E_INVAL, "%s: nx and ny must be >= 1", fn);
    if (pp_->peak_mode != PRNU_PEAK_FIXED_00 && pp_->peak_mode != PRNU_PEAK_ARGMAX)
        return fail(PRNU_E_INVAL, "%s: unknown peak mode", fn);
    if (pp_->nbhd < 1 || !(pp_->nbhd & 1)) return fail(PRNU_E_INVAL, "%s: nbhd must be odd and >= 1", fn);
    if (h <= pp_->nbhd || w <= pp_->nbhd)
        return fail(PRNU_E_INVAL, "%s: h and w must exceed nbhd (got %d x %d, nbhd %d)", fn, h, w, pp_->nbhd);
    if ((int64_t)h * w > (int64_t)INT_MAX) return fail(PRNU_E_INVAL, "%s: surface too large", fn);
    FftPlan ph, pw;
    PRNU_TRY(check_fft_dims(h, w, fn, &ph, &pw));
    const bool modulated = modulate != nullptr;
    hipStream_t s = (hipStream_t)stream;
    const int64_t N = (int64_t)h * w;
    if (pce_fast_ok(h, w, pp_->peak_mode, pp_->nbhd)) {
        Carver cv(nullptr);
        PcePlan pl;
        plan_pce_fast(cv, nx, ny, h, w, modulated, &pl);
        PRNU_TRY(check_ws(cv, ws, ws_bytes, fn));
        Carver real(ws);
        plan_pce_fast(real, nx, ny, h, w, modulated, &pl);
        return pce_fixed_fast(X, nx, Y, ny, h, w, modulate, pp_->nbhd, pce, ncc, peak, pl, s);
    }
    Carver cv(nullptr);
    PcePlan pl;
    plan_pce(cv, nx, ny, h, w, modulated, &pl);
    PRNU_TRY(check_ws(cv, ws, ws_bytes, fn));
    Carver real(ws);
    plan_pce(real, nx, ny, h, w, modulated, &pl);
    PRNU_HIP(launch_twiddles(h, pl.tw_h, s));
    PRNU_HIP(launch_twiddles(w, pl.tw_w, s));
    // query spectra
    PRNU_HIP(launch_pair_stats(X, nullptr, INT_MAX, 0, nx, N, pl.xmean, pl.xn2, pl.spart, s));
    PRNU_HIP(launch_pair_center(X, nullptr, INT_MAX, 0, nx, N, pl.xmean, pl.Xs, s));
    PRNU_HIP(launch_fft2(pl.Xs, nx, h, w, ph, pw, pl.tw_h, pl.tw_w, -1, s));
    if (!modulated) {
        PRNU_HIP(launch_pair_stats(Y, nullptr, INT_MAX, 0, ny, N, pl.ymean, pl.yn2, pl.spart, s));
        PRNU_HIP(launch_pair_center(Y, nullptr, INT_MAX, 0, ny, N, pl.ymean, pl.Ys, s));
        PRNU_HIP(launch_fft2(pl.Ys, ny, h, w, ph, pw, pl.tw_h, pl.tw_w, -1, s));
    }
    const int64_t npairs = (int64_t)nx * ny;
    for (int64_t p0 = 0; p0 < npairs; p0 += pl.P) {
        const int n = (int)(npairs - p0 < pl.P ? npairs - p0 : pl.P);
        if (modulated) {
            PRNU_HIP(launch_pair_stats(Y, modulate, ny, (int)p0, n, N, pl.ymean, pl.yn2, pl.spart, s));
            PRNU_HIP(launch_pair_center(Y, modulate, ny, (int)p0, n, N, pl.ymean, pl.Z, s));
            PRNU_HIP(launch_fft2(pl.Z, n, h, w, ph, pw, pl.tw_h, pl.tw_w, -1, s));
            PRNU_HIP(launch_cross(pl.Xs, nullptr, ny, (int)p0, n, N, pl.Z, s));
        } else {
            PRNU_HIP(launch_cross(pl.Xs, pl.Ys, ny, (int)p0, n, N, pl.Z, s));
        }
        PRNU_HIP(launch_fft2(pl.Z, n, h, w, ph, pw, pl.tw_h, pl.tw_w, +1, s));
        PRNU_HIP(launch_pce_reduce(pl.Z, n, h, w, pp_->nbhd, pp_->peak_mode, pl.xn2, pl.yn2, !modulated, ny,
                                   (int)p0, pce, ncc, peak, pl.ppart, s));
    }
    return PRNU_OK;
}

int prnu_denoise_residual_vjp_workspace_size(int n, int H, int W, const prnu_denoise_params *p, size_t *bytes) {
    const char *fn = "prnu_denoise_residual_vjp_workspace_size";
    set_error("");
    if (!bytes) return fail(PRNU_E_INVAL, "%s: null output", fn);
    if (n < 1) return fail(PRNU_E_INVAL, "%s: n must be >= 1", fn);
    PRNU_TRY(check_dims(H, W, fn));
    PRNU_TRY(check_params(p, fn));
    Carver cv(nullptr);
    VjpPlan vp;
    plan_vjp(cv, n, H, W, p, &vp);
    *bytes = cv.off;
    return PRNU_OK;
}

int prnu_denoise_residual_vjp(const float *gW, int64_t gW_plane_stride, const float *mul, const float *div, int n,
                              int H, int W, const prnu_denoise_params *p, const float *ckpt, double *dLds, void *ws,
                              size_t ws_bytes, void *stream) {
    const char *fn = "prnu_denoise_residual_vjp";
    set_error("");
    if (!gW || !ckpt || !dLds) return fail(PRNU_E_INVAL, "%s: null pointer", fn);
    if (n < 1) return fail(PRNU_E_INVAL, "%s: n must be >= 1", fn);
    if (gW_plane_stride < 0) return fail(PRNU_E_INVAL, "%s: negative plane stride", fn);
    PRNU_TRY(check_dims(H, W, fn));
    PRNU_TRY(check_params(p, fn));
    Carver cv(nullptr);
    VjpPlan vp;
    plan_vjp(cv, n, H, W, p, &vp);
    PRNU_TRY(check_ws(cv, ws, ws_bytes, fn));
    Carver real(ws);
    plan_vjp(real, n, H, W, p, &vp);
    Filter f;
    make_filter(p->taps, &f);
    hipStream_t s = (hipStream_t)stream;
    const int Hp = padded(H), Wp = padded(W), L = p->levels;
    const int64_t plane = (int64_t)H * W;
    const int64_t cplane = (int64_t)ckpt_level_offset(H, W, L + 1);
    for (int b0 = 0; b0 < n; b0 += vp.nb) {
        const int nb = n - b0 < vp.nb ? n - b0 : vp.nb;
        for (int l = 1; l <= L; ++l) {
            const int nr = Hp >> (l - 1), nc = Wp >> (l - 1);
            const float *ck = ckpt + (int64_t)b0 * cplane + ckpt_level_offset(H, W, l);
            float *llo = l < L ? vp.ll[l] : nullptr;
            const int tiles = dwt_vjp_tiles(nr / 2, nc / 2);
            if (l == 1)
                PRNU_HIP(launch_dwt_vjp(p->taps, f, gW + b0 * gW_plane_stride, gW_plane_stride, H, W,
                                        mul ? mul + b0 * plane : nullptr, plane, div, Hp, Wp, pad_before(H),
                                        pad_before(W), llo, ck, cplane, nb, vp.part, s));
            else
                PRNU_HIP(launch_dwt_vjp(p->taps, f, vp.ll[l - 1], (int64_t)nr * nc, nr, nc, nullptr, 0, nullptr, nr,
                                        nc, 0, 0, llo, ck, cplane, nb, vp.part, s));
            PRNU_HIP(launch_vjp_finish(vp.part, (int64_t)nb * tiles, dLds + (l - 1), s));
        }
    }
    return PRNU_OK;
}

int prnu_pce_vjp_workspace_size(int nx, int ny, int h, int w, size_t *bytes) {
    const char *fn = "prnu_pce_vjp_workspace_size";
    set_error("");
    if (!bytes) return fail(PRNU_E_INVAL, "%s: null output", fn);
    if (nx < 1 || ny < 1 || h < 1 || w < 1) return fail(PRNU_E_INVAL, "%s: bad sizes", fn);
    Carver cv(nullptr);
    PvjpPlan pl;
    plan_pvjp(cv, nx, ny, h, w, &pl);
    *bytes = cv.off;
    return PRNU_OK;
}

int prnu_pce_vjp(const float *X, int nx, const float *Y, int ny, int h, int w, const float *modulate, int nbhd,
                 const double *weights, double *pce, float *gX, float *gY, void *ws, size_t ws_bytes, void *stream) {
    const char *fn = "prnu_pce_vjp";
    set_error("");
    if (!X || !Y || !weights || !gX || !gY) return fail(PRNU_E_INVAL, "%s: null pointer", fn);
    if (nx < 1 || ny < 1) return fail(PRNU_E_INVAL, "%s: nx and ny must be >= 1", fn);
    if (nbhd < 1 || !(nbhd & 1)) return fail(PRNU_E_INVAL, "%s: nbhd must be odd and >= 1", fn);
    if (h <= nbhd || w <= nbhd) return fail(PRNU_E_INVAL, "%s: h and w must exceed nbhd", fn);
    if ((int64_t)h * w > (int64_t)INT_MAX) return fail(PRNU_E_INVAL, "%s: surface too large", fn);
    FftPlan ph, pw;
    PRNU_TRY(check_fft_dims(h, w, fn, &ph, &pw));
    Carver cv(nullptr);
    PvjpPlan pl;
    plan_pvjp(cv, nx, ny, h, w, &pl);
    PRNU_TRY(check_ws(cv, ws, ws_bytes, fn));
    Carver real(ws);
    plan_pvjp(real, nx, ny, h, w, &pl);
    hipStream_t s = (hipStream_t)stream;
    const int64_t N = (int64_t)h * w;
    PRNU_HIP(launch_fill_zero(gX, (int64_t)nx * N, s));
    PRNU_HIP(launch_fill_zero(gY, (int64_t)ny * N, s));
    PRNU_HIP(launch_twiddles(h, pl.tw_h, s));
    PRNU_HIP(launch_twiddles(w, pl.tw_w, s));
    PRNU_HIP(launch_pair_stats(X, nullptr, INT_MAX, 0, nx, N, pl.xmean, pl.xn2, pl.spart, s));
    PRNU_HIP(launch_pair_center(X, nullptr, INT_MAX, 0, nx, N, pl.xmean, pl.Xs, s));
    PRNU_HIP(launch_fft2(pl.Xs, nx, h, w, ph, pw, pl.tw_h, pl.tw_w, -1, s));
    const int64_t npairs = (int64_t)nx * ny;
    for (int64_t p0 = 0; p0 < npairs; p0 += pl.P) {
        const int n = (int)(npairs - p0 < pl.P ? npairs - p0 : pl.P);
        PRNU_HIP(launch_pair_stats(Y, modulate, ny, (int)p0, n, N, pl.ymean, pl.yn2, pl.spart, s));
        PRNU_HIP(launch_pair_center(Y, modulate, ny, (int)p0, n, N, pl.ymean, pl.V, s));
        PRNU_HIP(launch_fft2(pl.V, n, h, w, ph, pw, pl.tw_h, pl.tw_w, -1, s));
        PRNU_HIP(hipMemcpyAsync(pl.Z, pl.V, (size_t)n * N * sizeof(float2), hipMemcpyDeviceToDevice, s));
        PRNU_HIP(launch_cross(pl.Xs, nullptr, ny, (int)p0, n, N, pl.Z, s));
        PRNU_HIP(launch_fft2(pl.Z, n, h, w, ph, pw, pl.tw_h, pl.tw_w, +1, s));
        PRNU_HIP(launch_pvjp(pl.Z, pl.V, pl.T1, pl.T2, pl.Xs, n, h, w, nbhd, ny, (int)p0, ph, pw, pl.tw_h, pl.tw_w,
                             pl.coef, weights, modulate, pce, gX, gY, s));
    }
    return PRNU_OK;
}

// ---- FP64 mode of the differentiated chain -----------------------------------
static int gap64_dims(int ncam, int m, int nq, int H, int W, int group, int taps, int nbhd, const char *fn,
                      prnu::Gap64Dims *D) {
    using namespace prnu;
    if (ncam < 1 || m < 1 || nq < 1) return fail(PRNU_E_INVAL, "%s: ncam, m and nq must be >= 1", fn);
    if (group < 1) return fail(PRNU_E_INVAL, "%s: group must be >= 1", fn);
    PRNU_TRY(check_dims(H, W, fn));
    if (taps != 8 && taps != 16) return fail(PRNU_E_UNSUPPORTED, "%s: taps must be 8 or 16", fn);
    if (nbhd < 1 || !(nbhd & 1) || nbhd >= H || nbhd >= W)
        return fail(PRNU_E_INVAL, "%s: nbhd must be odd, >= 1 and below H and W", fn);
    if (!gap64_fft_length_ok(H) || !gap64_fft_length_ok(W))
        return fail(PRNU_E_UNSUPPORTED, "%s: H and W need prime factors <= 5 (got %d x %d)", fn, H, W);
    D->ncam = ncam;
    D->m = m;
    D->d = group;
    D->g = (m + group - 1) / group;
    D->nq = nq;
    D->H = H;
    D->W = W;
    D->Hp = padded(H);
    D->Wp = padded(W);
    D->t = pad_before(H);
    D->l = pad_before(W);
    D->levels = 4;
    D->taps = taps;
    D->nbhd = nbhd;
    D->ssz = 0;
    for (int l = 1; l <= D->levels; ++l) D->ssz += 3 * (int64_t)(D->Hp >> l) * (D->Wp >> l);
    const int64_t planes = (int64_t)ncam * D->g + nq;
    if (planes > 65535 || planes * D->Hp * (int64_t)D->Wp > ((int64_t)1 << 31))
        return fail(PRNU_E_INVAL, "%s: at most 65535 planes and 2^31 padded pixels over all planes", fn);
    return PRNU_OK;
}

int prnu_pce_gap_f64_workspace_size(int ncam, int m, int nq, int H, int W, int group, int taps, int nbhd,
                                    size_t *bytes) {
    const char *fn = "prnu_pce_gap_f64_workspace_size";
    set_error("");
    if (!bytes) return fail(PRNU_E_INVAL, "%s: null output", fn);
    Gap64Dims D;
    PRNU_TRY(gap64_dims(ncam, m, nq, H, W, group, taps, nbhd, fn, &D));
    *bytes = gap64_workspace_bytes(D);
    return PRNU_OK;
}

int prnu_pce_gap_f64(const float *cam_frames, int ncam, int m, const float *queries, int nq, const int *query_cam,
                     int H, int W, int group, int taps, int nbhd, const double *theta, double *out, double *pce,
                     void *ws, size_t ws_bytes, void *stream) {
    const char *fn = "prnu_pce_gap_f64";
    set_error("");
    if (!cam_frames || !queries || !query_cam || !theta || !out) return fail(PRNU_E_INVAL, "%s: null pointer", fn);
    Gap64Dims D;
    PRNU_TRY(gap64_dims(ncam, m, nq, H, W, group, taps, nbhd, fn, &D));
    for (int k = 0; k < 5; ++k)
        if (!std::isfinite(theta[k]) || theta[k] < 0.0)
            return fail(PRNU_E_INVAL, "%s: theta must be finite and >= 0", fn);
    const size_t need = gap64_workspace_bytes(D);
    if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) & 255))
        return fail(PRNU_E_WORKSPACE, "%s: workspace needs %zu bytes, 256-byte aligned", fn, need);
    Filter64 f;
    if (!make_filter64(taps, &f)) return fail(PRNU_E_UNSUPPORTED, "%s: filter design failed", fn);
    PRNU_HIP(gap64_run(D, f, theta, cam_frames, queries, query_cam, ws, out, pce, (hipStream_t)stream));
    return PRNU_OK;
}

int prnu_postprocess_workspace_size(int n, int C, int H, int W, int flags, size_t *bytes) {
    const char *fn = "prnu_postprocess_workspace_size";
    set_error("");
    if (!bytes) return fail(PRNU_E_INVAL, "%s: null output", fn);
    if (n < 1 || (C != 1 && C != 3)) return fail(PRNU_E_INVAL, "%s: bad n or C", fn);
    if (H < 1 || W < 1 || H > kMaxDim || W > kMaxDim) return fail(PRNU_E_INVAL, "%s: bad H x W", fn);
    PRNU_TRY(check_flags(flags, fn));
    Carver cv(nullptr);
    PostWs pw;
    carve_post(cv, n, C, H, W, flags, &pw);
    *bytes = cv.off;
    return PRNU_OK;
}

int prnu_postprocess(const float *planes, int n, int C, int H, int W, int flags, float sigma_wf, float *out,
                     void *ws, size_t ws_bytes, void *stream) {
    const char *fn = "prnu_postprocess";
    set_error("");
    if (!planes || !out) return fail(PRNU_E_INVAL, "%s: null pointer", fn);
    if (planes == out) return fail(PRNU_E_INVAL, "%s: out may not alias planes", fn);
    if (n < 1 || (C != 1 && C != 3)) return fail(PRNU_E_INVAL, "%s: bad n or C", fn);
    if (H < 1 || W < 1 || H > kMaxDim || W > kMaxDim) return fail(PRNU_E_INVAL, "%s: bad H x W", fn);
    PRNU_TRY(check_flags(flags, fn));
    if (!std::isfinite(sigma_wf)) return fail(PRNU_E_INVAL, "%s: sigma_wf must be finite", fn);
    if (flags & PRNU_WIENER) {
        FftPlan a, b;
        PRNU_TRY(check_fft_dims(H, W, fn, &a, &b));
    }
    Carver cv(nullptr);
    PostWs pw;
    carve_post(cv, n, C, H, W, flags, &pw);
    PRNU_TRY(check_ws(cv, ws, ws_bytes, fn));
    Carver real(ws);
    carve_post(real, n, C, H, W, flags, &pw);
    return run_post(planes, n, C, H, W, flags, sigma_wf, out, pw, false, (hipStream_t)stream);
}

}  // extern "C"
