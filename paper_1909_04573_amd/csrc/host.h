// Host-side helpers shared by the entry points: status macros, workspace
// carving and argument checks.
#pragma once

#include <cmath>
#include <cstdint>

#include "internal.h"

namespace prnu {

#define PRNU_HIP(expr)                                                                       \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(PRNU_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));         \
    } while (0)

#define PRNU_TRY(expr)                  \
    do {                                \
        int rc_ = (expr);               \
        if (rc_ != PRNU_OK) return rc_; \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int64_t kBatchPixels = 48ll << 20;  // planes x padded pixels per denoise batch
// Fingerprint accumulation batches more: every batch ends in one read-modify-
// write of the accumulators, and larger level launches leave shorter tails
// (1080p RGB: 32 SDA frames, about 1.9 GB of workspace).
constexpr int64_t kAccBatchPixels = 192ll << 20;  // frames x channels x padded pixels per batch
constexpr int kMaxFramesPerMle = 32;               // SDA frames folded per accumulator update
constexpr int kMaxDim = 1 << 15;

// Bump allocator over the caller's workspace; with base == nullptr it only
// measures, so size queries and calls carve identically.
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <class T>
    T *take(size_t count) {
        off = (off + kAlign - 1) / kAlign * kAlign;
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

inline int check_ws(const Carver &cv, void *ws, size_t ws_bytes, const char *fn) {
    if (!ws) return fail(PRNU_E_WORKSPACE, "%s: null workspace", fn);
    if (reinterpret_cast<uintptr_t>(ws) % kAlign)
        return fail(PRNU_E_WORKSPACE, "%s: workspace must be %zu-byte aligned", fn, kAlign);
    if (ws_bytes < cv.off)
        return fail(PRNU_E_WORKSPACE, "%s: workspace of %zu bytes, %zu needed", fn, ws_bytes, cv.off);
    return PRNU_OK;
}

inline int check_dims(int H, int W, const char *fn) {
    if (H < 16 || W < 16 || H > kMaxDim || W > kMaxDim)
        return fail(PRNU_E_INVAL, "%s: H and W must be in [16, %d] (got %d x %d)", fn, kMaxDim, H, W);
    return PRNU_OK;
}

inline int check_frames(const void *frames, int dtype, int n, int C, const char *fn) {
    if (!frames) return fail(PRNU_E_INVAL, "%s: null frames", fn);
    if (dtype != PRNU_U8 && dtype != PRNU_BF16 && dtype != PRNU_F32)
        return fail(PRNU_E_INVAL, "%s: unknown dtype %d", fn, dtype);
    if (n < 1) return fail(PRNU_E_INVAL, "%s: need at least one frame (got %d)", fn, n);
    if (C != 1 && C != 3) return fail(PRNU_E_INVAL, "%s: C must be 1 or 3 (got %d)", fn, C);
    return PRNU_OK;
}

// MLE accumulation: a frame below 2^28 pixels (the fold's 32-bit offsets).
inline int check_mle_pixels(int H, int W, const char *fn) {
    if ((int64_t)H * W >= kMleMaxPixels)
        return fail(PRNU_E_INVAL, "%s: frames of %d x %d are too large to accumulate (limit 2^28 pixels)", fn, H, W);
    return PRNU_OK;
}

inline int check_params(const prnu_denoise_params *p, const char *fn) {
    if (!p) return fail(PRNU_E_INVAL, "%s: null denoise params", fn);
    if (!std::isfinite(p->sigma0) || p->sigma0 < 0.f)
        return fail(PRNU_E_INVAL, "%s: sigma0 must be finite and >= 0", fn);
    if (p->levels < 1 || p->levels > 4) return fail(PRNU_E_INVAL, "%s: levels must be 1..4", fn);
    if (p->taps != 8 && p->taps != 16)
        return fail(PRNU_E_UNSUPPORTED, "%s: taps must be 8 or 16 (got %d)", fn, p->taps);
    for (int l = 0; l < 4; ++l)
        if (!std::isfinite(p->level_weight[l]) || p->level_weight[l] < 0.f)
            return fail(PRNU_E_INVAL, "%s: level_weight must be finite and >= 0", fn);
    return PRNU_OK;
}

inline int check_flags(int flags, const char *fn) {
    if (flags & ~(PRNU_ZM | PRNU_LUMA | PRNU_WIENER)) return fail(PRNU_E_INVAL, "%s: unknown flags", fn);
    return PRNU_OK;
}

inline size_t elem_bytes(int dtype) { return dtype == PRNU_U8 ? 1 : dtype == PRNU_BF16 ? 2 : 4; }

// Bytes from one frame to the next: 0 asks for dense frames; otherwise at
// least a dense frame, a multiple of the sample size, and small enough that
// the last frame's offset fits in int64.  Call after check_frames.
inline int check_frame_stride(int64_t stride, int dtype, int n, int H, int W, int C, const char *fn, int64_t *out) {
    const int64_t esz = (int64_t)elem_bytes(dtype), dense = (int64_t)H * W * C * esz;
    if (stride == 0) {
        *out = dense;
        return PRNU_OK;
    }
    if (stride < dense || stride % esz != 0 || stride > INT64_MAX / n)
        return fail(PRNU_E_INVAL, "%s: frame_stride_bytes %lld must be 0 or a multiple of %lld that is >= %lld", fn,
                    (long long)stride, (long long)esz, (long long)dense);
    *out = stride;
    return PRNU_OK;
}

// Residuals of float planes in batches of at most max_nb planes (0: the
// default batch) through the workspace ws; optional sensitivity checkpoint.
int denoise_run(const char *fn, const float *img, int n_img, int H, int W, const prnu_denoise_params *p,
                float *resid, float *ckpt, void *ws, size_t ws_bytes, void *stream, int max_nb = 0);
// Planes of H x W whose wavelet pyramid (the denoise workspace) fits `bytes`.
int denoise_planes_fitting(int H, int W, const prnu_denoise_params *p, size_t bytes);

}  // namespace prnu
