// Host-side check of the C ABI under AddressSanitizer and
// UndefinedBehaviorSanitizer (test infrastructure; needs no GPU).
//
// The library's host sources (validation, workspace carving, batch round
// packing, tile table, filter design, error text) are built with the
// sanitizers on their host code; the kernels are linked as usual and never
// launched: every call below either computes on the host only (workspace
// sizes, filter coefficients, batch planning, tile table) or is rejected by
// the validation that runs before anything is enqueued.  The device pointers
// are fake addresses that no code path dereferences.
//
//   host_check [abi|batch|all]     exit status 0 when every check holds
//   host_check plant-heap|plant-ub  makes one heap over-read or one signed
//                                   overflow here, which the sanitizers must
//                                   report (shows they are active)

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "prnu.h"

namespace {

int g_checks = 0, g_failed = 0;

void expect(bool ok, const char *what, int line) {
    ++g_checks;
    if (!ok) {
        ++g_failed;
        std::fprintf(stderr, "host_check: FAILED line %d: %s (last error: %s)\n", line, what, prnu_last_error());
    }
}
#define EXPECT(cond) expect((cond), #cond, __LINE__)
#define EXPECT_RC(call, rc) expect((call) == (rc), #call " == " #rc, __LINE__)

void *fake(uintptr_t a) { return reinterpret_cast<void *>(a); }

bool error_mentions(const char *s) { return std::strstr(prnu_last_error(), s) != nullptr; }

void check_filters() {
    for (int taps = 2; taps <= 20; taps += 2) {
        std::vector<double> h(taps);
        EXPECT_RC(prnu_filter_coefficients(taps, h.data()), PRNU_OK);
        double s = 0, e = 0;
        for (double v : h) s += v, e += v * v;
        EXPECT(std::fabs(s - std::sqrt(2.0)) < 1e-13);
        EXPECT(std::fabs(e - 1.0) < 1e-13);
        // double shifts are orthogonal: sum_k h[k] h[k + 2m] = 0 for m != 0
        for (int m = 1; 2 * m < taps; ++m) {
            double o = 0;
            for (int k = 0; k + 2 * m < taps; ++k) o += h[k] * h[k + 2 * m];
            EXPECT(std::fabs(o) < 1e-13);
        }
    }
    double h[32];
    EXPECT_RC(prnu_filter_coefficients(3, h), PRNU_E_UNSUPPORTED);
    EXPECT_RC(prnu_filter_coefficients(22, h), PRNU_E_UNSUPPORTED);
    EXPECT_RC(prnu_filter_coefficients(0, h), PRNU_E_UNSUPPORTED);
    EXPECT_RC(prnu_filter_coefficients(8, nullptr), PRNU_E_INVAL);
}

void check_workspace_sizes() {
    prnu_denoise_params p;
    prnu_default_denoise_params(&p);
    size_t n = 0, n1 = 0, n8 = 0;
    const int dims[][2] = {{16, 16}, {17, 33}, {72, 104}, {1080, 1920}, {3000, 4000}, {2160, 3840}, {32768, 16}};
    for (const auto &d : dims) {
        for (int levels = 1; levels <= 4; ++levels) {
            p.levels = levels;
            EXPECT_RC(prnu_denoise_residual_workspace_size(3, d[0], d[1], &p, &n), PRNU_OK);
            EXPECT(n >= (size_t)3 * d[0] * d[1] * 4);
        }
        p.levels = 4;
        for (int C = 1; C <= 3; C += 2)
            for (int group : {1, 7, 50})
                EXPECT_RC(prnu_fingerprint_accumulate_workspace_size(400, d[0], d[1], C, group, &p, &n), PRNU_OK);
        EXPECT_RC(prnu_query_residual_workspace_size(5, d[0], d[1], 3, &p, PRNU_ZM | PRNU_LUMA, &n), PRNU_OK);
    }
    EXPECT_RC(prnu_fingerprint_accumulate_workspace_size(400, 1080, 1920, 3, 1, &p, &n1), PRNU_OK);
    EXPECT_RC(prnu_fingerprint_accumulate_workspace_size(400, 1080, 1920, 3, 50, &p, &n8), PRNU_OK);
    EXPECT(n1 == 4 * n8);
    EXPECT_RC(prnu_fingerprint_finalize_workspace_size(3, 1080, 1920, 7, &n), PRNU_OK);
    EXPECT_RC(prnu_pce_match_workspace_size(50, 4, 1080, 1920, 1, &n), PRNU_OK);
    EXPECT(n > (size_t)50 * 1080 * 1920 * 8);
    EXPECT_RC(prnu_pce_vjp_workspace_size(2, 3, 500, 500, &n), PRNU_OK);
    EXPECT_RC(prnu_denoise_residual_vjp_workspace_size(2, 200, 136, &p, &n), PRNU_OK);
    EXPECT_RC(prnu_postprocess_workspace_size(2, 3, 120, 160, 7, &n), PRNU_OK);
    EXPECT_RC(prnu_denoise_residual_workspace_size(3, 64, 64, &p, nullptr), PRNU_E_INVAL);
    EXPECT_RC(prnu_denoise_residual_workspace_size(3, 64, 64, nullptr, &n), PRNU_E_INVAL);
    size_t fl = 0;
    EXPECT_RC(prnu_denoise_ckpt_floats(1080, 1920, 4, &fl), PRNU_OK);
    EXPECT(fl > 0);
}

void check_validation() {
    prnu_denoise_params p;
    prnu_default_denoise_params(&p);
    void *fr = fake(0x100000), *out = fake(0x200000), *ws = fake(0x40000000);
    const size_t big = (size_t)1 << 30;
    float *o = static_cast<float *>(out);
    uint32_t *u = static_cast<uint32_t *>(out);
    // SDA: null frames, bad C, group 0, sums of float frames, unknown dtype, bad strides
    EXPECT_RC(prnu_sda_average(nullptr, PRNU_U8, 8, 16, 16, 1, 0, 1, u, o, nullptr, nullptr, nullptr), PRNU_E_INVAL);
    EXPECT_RC(prnu_sda_average(fr, PRNU_U8, 8, 16, 16, 2, 0, 1, nullptr, o, nullptr, nullptr, nullptr), PRNU_E_INVAL);
    EXPECT_RC(prnu_sda_average(fr, PRNU_U8, 8, 16, 16, 1, 0, 0, nullptr, o, nullptr, nullptr, nullptr), PRNU_E_INVAL);
    EXPECT_RC(prnu_sda_average(fr, PRNU_BF16, 8, 16, 16, 1, 0, 1, u, nullptr, nullptr, nullptr, nullptr),
              PRNU_E_INVAL);
    EXPECT_RC(prnu_sda_average(fr, 9, 8, 16, 16, 1, 0, 1, nullptr, o, nullptr, nullptr, nullptr), PRNU_E_INVAL);
    EXPECT_RC(prnu_sda_average(fr, PRNU_U8, 8, 16, 16, 1, 255, 1, nullptr, o, nullptr, nullptr, nullptr),
              PRNU_E_INVAL);
    EXPECT_RC(prnu_sda_average(fr, PRNU_F32, 8, 16, 16, 1, 16 * 16 * 4 + 2, 1, nullptr, o, nullptr, nullptr, nullptr),
              PRNU_E_INVAL);
    EXPECT_RC(prnu_sda_average(fr, PRNU_U8, 8, 16, 16, 1, INT64_MAX / 2, 1, nullptr, o, nullptr, nullptr, nullptr),
              PRNU_E_INVAL);
    EXPECT(error_mentions("frame_stride_bytes"));
    // residual: short side, small workspace, no planes, filter length, levels, sigma0, misaligned workspace
    EXPECT_RC(prnu_denoise_residual(static_cast<float *>(fr), 1, 15, 64, &p, o, ws, big, nullptr), PRNU_E_INVAL);
    EXPECT_RC(prnu_denoise_residual(static_cast<float *>(fr), 1, 64, 64, &p, o, ws, 16, nullptr), PRNU_E_WORKSPACE);
    EXPECT_RC(prnu_denoise_residual(static_cast<float *>(fr), 0, 64, 64, &p, o, ws, big, nullptr), PRNU_E_INVAL);
    prnu_denoise_params bad = p;
    bad.taps = 6;
    EXPECT_RC(prnu_denoise_residual(static_cast<float *>(fr), 1, 64, 64, &bad, o, ws, big, nullptr),
              PRNU_E_UNSUPPORTED);
    bad = p;
    bad.levels = 5;
    EXPECT_RC(prnu_denoise_residual(static_cast<float *>(fr), 1, 64, 64, &bad, o, ws, big, nullptr), PRNU_E_INVAL);
    bad = p;
    bad.sigma0 = NAN;
    EXPECT_RC(prnu_denoise_residual(static_cast<float *>(fr), 1, 64, 64, &bad, o, ws, big, nullptr), PRNU_E_INVAL);
    EXPECT_RC(prnu_denoise_residual(static_cast<float *>(fr), 1, 64, 64, &p, o, fake(0x40000010), big, nullptr),
              PRNU_E_WORKSPACE);
    EXPECT_RC(prnu_denoise_residual_noalloc(static_cast<float *>(fr), 1, 4096, 4096, &p, o, nullptr), PRNU_E_INVAL);
    EXPECT(error_mentions("static scratch"));
    EXPECT_RC(prnu_denoise_residual_noalloc(static_cast<float *>(fr), 1, 64, 64, &p, static_cast<float *>(fr),
                                            nullptr),
              PRNU_E_INVAL);
    // accumulate: unknown mode, null accumulator, short frame stride
    EXPECT_RC(prnu_fingerprint_accumulate(fr, PRNU_U8, 8, 64, 64, 1, 0, 1, &p, 7, out, out, nullptr, ws, big, nullptr),
              PRNU_E_INVAL);
    EXPECT_RC(prnu_fingerprint_accumulate(fr, PRNU_U8, 8, 64, 64, 1, 0, 1, &p, 0, nullptr, out, nullptr, ws, big,
                                          nullptr),
              PRNU_E_INVAL);
    EXPECT_RC(prnu_fingerprint_accumulate(fr, PRNU_U8, 8, 16384, 16384, 1, 0, 1, &p, 0, out, out, nullptr, ws, big,
                                          nullptr),
              PRNU_E_INVAL);  // 2^28 pixels: beyond the fold's 32-bit offsets
    EXPECT(error_mentions("2^28"));
    EXPECT_RC(prnu_fingerprint_accumulate(fr, PRNU_U8, 8, 64, 64, 1, 64 * 64 - 1, 1, &p, 0, out, out, nullptr, ws, big,
                                          nullptr),
              PRNU_E_INVAL);
    // finalize: DFT size with a factor 17, unknown flag
    EXPECT_RC(prnu_fingerprint_finalize(fr, fr, 0, 1, 17, 64, PRNU_WIENER, -1.f, o, ws, big, nullptr),
              PRNU_E_UNSUPPORTED);
    EXPECT_RC(prnu_fingerprint_finalize(fr, fr, 0, 1, 64, 64, 8, -1.f, o, ws, big, nullptr), PRNU_E_INVAL);
    EXPECT_RC(prnu_fingerprint_finalize(fr, fr, 0, 1, 64, 64, PRNU_ZM, INFINITY, o, ws, big, nullptr), PRNU_E_INVAL);
    // PCE: short side, factor 7, unknown peak mode
    prnu_pce_params pp = {PRNU_PEAK_FIXED_00, 11};
    const float *X = static_cast<const float *>(fr);
    double *pce = static_cast<double *>(out);
    EXPECT_RC(prnu_pce_match(X, 1, X, 1, 11, 64, nullptr, &pp, pce, nullptr, nullptr, ws, big, nullptr),
              PRNU_E_INVAL);
    EXPECT_RC(prnu_pce_match(X, 1, X, 1, 14, 64, nullptr, &pp, pce, nullptr, nullptr, ws, big, nullptr),
              PRNU_E_UNSUPPORTED);
    pp.peak_mode = 2;
    EXPECT_RC(prnu_pce_match(X, 1, X, 1, 64, 64, nullptr, &pp, pce, nullptr, nullptr, ws, big, nullptr),
              PRNU_E_INVAL);
    EXPECT(error_mentions("peak mode"));
    EXPECT_RC(prnu_query_residual(fr, PRNU_U8, 1, 64, 64, 3, &p, 16, o, nullptr, ws, big, nullptr), PRNU_E_INVAL);
    // blocks, resampling, warps
    EXPECT_RC(prnu_extract_blocks(X, 2, 64, 80, 65, o, nullptr), PRNU_E_INVAL);
    EXPECT_RC(prnu_extract_blocks(X, 2, 64, 1 << 16, 16, o, nullptr), PRNU_E_INVAL);
    EXPECT_RC(prnu_resample_bilinear(X, 1, 8, 8, NAN, 0, 0, 4, 4, o, nullptr), PRNU_E_INVAL);
    EXPECT_RC(prnu_resample_bilinear(X, 1, 8, 8, 0.5, -1, 0, 4, 4, o, nullptr), PRNU_E_INVAL);
    const double *M = static_cast<const double *>(fake(0x300000));
    EXPECT_RC(prnu_warp_affine(X, 1, 16, 16, M, 70000, 8, 8, o, nullptr), PRNU_E_INVAL);
    EXPECT_RC(prnu_warp_affine(X, 1, 16, 16, nullptr, 1, 8, 8, o, nullptr), PRNU_E_INVAL);
    // FP64 gap: sizes, DFT lengths, theta
    size_t gn = 0;
    EXPECT_RC(prnu_pce_gap_f64_workspace_size(8, 32, 64, 512, 512, 8, 16, 11, &gn), PRNU_OK);
    EXPECT(gn > (size_t)88 * 512 * 512 * 8);
    EXPECT_RC(prnu_pce_gap_f64_workspace_size(2, 8, 4, 64, 70, 4, 16, 11, &gn), PRNU_E_UNSUPPORTED);
    EXPECT_RC(prnu_pce_gap_f64_workspace_size(70000, 1, 1, 64, 64, 1, 16, 11, &gn), PRNU_E_INVAL);
    const double th_bad[5] = {3.0, 1.0, NAN, 1.0, 1.0};
    EXPECT_RC(prnu_pce_gap_f64(X, 2, 8, X, 4, static_cast<const int *>(fake(0x300000)), 64, 64, 4, 16, 11, th_bad,
                               pce, nullptr, ws, big, nullptr),
              PRNU_E_INVAL);
    // long argument values reach the error text formatting
    EXPECT_RC(prnu_sda_average(fr, PRNU_F32, 16843009, 16, 16, 3, INT64_MAX, 1, nullptr, o, nullptr, nullptr, nullptr),
              PRNU_E_INVAL);
    EXPECT(std::strlen(prnu_last_error()) > 20);
}

struct Cam {
    int n, H, W, C, d;
};

std::vector<prnu_camera> cameras(const std::vector<Cam> &spec) {
    std::vector<prnu_camera> c(spec.size());
    for (size_t i = 0; i < spec.size(); ++i) {
        // disjoint fake accumulator areas: 16 MiB apart
        c[i] = prnu_camera{fake(0x100000 + (uintptr_t)i * 0x1000), spec[i].n, spec[i].H, spec[i].W, spec[i].C,
                           spec[i].d, fake(0x10000000 + (uintptr_t)i * 0x2000000),
                           fake(0x11000000 + (uintptr_t)i * 0x2000000)};
    }
    return c;
}

void check_batch() {
    prnu_denoise_params p;
    prnu_default_denoise_params(&p);
    size_t n = 0, prev = 0;
    // many cameras of every size, depth and channel count, under shrinking round budgets
    std::vector<Cam> spec;
    const int dims[][2] = {{16, 16}, {64, 96}, {256, 256}, {720, 1280}, {1080, 1920}, {2160, 3840}, {37, 53}};
    uint32_t r = 12345;
    for (int i = 0; i < 40; ++i) {
        r = r * 1664525u + 1013904223u;
        const auto &d = dims[(r >> 8) % 7];
        spec.push_back(Cam{1 + (int)((r >> 12) % 300), d[0], d[1], (r >> 20) & 1 ? 3 : 1, 1 + (int)((r >> 22) % 60)});
    }
    std::vector<prnu_camera> cams = cameras(spec);
    for (size_t budget : {(size_t)0, (size_t)1 << 33, (size_t)1 << 31, (size_t)3 << 28}) {
        EXPECT_RC(prnu_batch_workspace_size(cams.data(), (int)cams.size(), &p, budget, &n), PRNU_OK);
        EXPECT(n > 0);
        if (budget && prev) EXPECT(n <= prev || budget > ((size_t)1 << 31));
        prev = n;
    }
    // one camera whose pyramid exceeds a tiny budget is still planned (one job per round)
    std::vector<prnu_camera> one = cameras({{3, 2160, 3840, 3, 1}});
    EXPECT_RC(prnu_batch_workspace_size(one.data(), 1, &p, 1 << 20, &n), PRNU_OK);
    // validation
    EXPECT_RC(prnu_batch_workspace_size(nullptr, 1, &p, 0, &n), PRNU_E_INVAL);
    EXPECT_RC(prnu_batch_workspace_size(cams.data(), 0, &p, 0, &n), PRNU_E_INVAL);
    std::vector<prnu_camera> bad = cameras({{10, 15, 64, 1, 1}});
    EXPECT_RC(prnu_batch_workspace_size(bad.data(), 1, &p, 0, &n), PRNU_E_INVAL);
    bad = cameras({{10, 64, 64, 2, 1}});
    EXPECT_RC(prnu_batch_workspace_size(bad.data(), 1, &p, 0, &n), PRNU_E_INVAL);
    bad = cameras({{10, 64, 64, 1, 0}});
    EXPECT_RC(prnu_batch_workspace_size(bad.data(), 1, &p, 0, &n), PRNU_E_INVAL);
    prnu_batch *h = nullptr;
    void *ws = fake(0x40000000);
    std::vector<prnu_camera> ok = cameras({{10, 64, 64, 1, 2}, {7, 32, 48, 3, 1}});
    EXPECT_RC(prnu_batch_create(ok.data(), 2, 5, &p, 0, 0, 0, ws, 1 << 30, nullptr, &h), PRNU_E_INVAL);
    EXPECT_RC(prnu_batch_create(ok.data(), 2, 0, &p, 7, 0, 0, ws, 1 << 30, nullptr, &h), PRNU_E_INVAL);
    EXPECT_RC(prnu_batch_create(ok.data(), 2, 0, &p, 0, 8, 0, ws, 1 << 30, nullptr, &h), PRNU_E_INVAL);
    EXPECT_RC(prnu_batch_create(ok.data(), 2, 0, &p, 0, 0, 0, ws, 1024, nullptr, &h), PRNU_E_WORKSPACE);
    EXPECT_RC(prnu_batch_create(ok.data(), 2, 0, &p, 0, 0, 0, fake(0x40000010), 1 << 30, nullptr, &h),
              PRNU_E_WORKSPACE);
    std::vector<prnu_camera> overlap = ok;
    overlap[1].A = static_cast<char *>(overlap[0].A) + 8;
    EXPECT_RC(prnu_batch_create(overlap.data(), 2, 0, &p, 0, 0, 0, ws, 1 << 30, nullptr, &h), PRNU_E_INVAL);
    EXPECT(error_mentions("overlap"));
    EXPECT(h == nullptr);
    EXPECT_RC(prnu_batch_launch(nullptr, nullptr), PRNU_E_INVAL);
    EXPECT_RC(prnu_batch_destroy(nullptr), PRNU_OK);
    prnu_batch_info info;
    EXPECT_RC(prnu_batch_info_get(nullptr, &info), PRNU_E_INVAL);
    // tile table: set, read back, reject, restore
    const int t0 = prnu_get_tile(0, 16, 540, 960);
    EXPECT(t0 == 64 || t0 == 32);
    EXPECT_RC(prnu_set_tile(0, 16, 540, 960, 32), PRNU_OK);
    EXPECT(prnu_get_tile(0, 16, 540, 960) == 32);
    EXPECT_RC(prnu_set_tile(0, 16, 540, 960, 48), PRNU_E_INVAL);
    EXPECT_RC(prnu_set_tile(1, 16, 540, 960, 64), PRNU_E_INVAL);
    EXPECT_RC(prnu_set_tile(0, 16, 540, 960, 0), PRNU_OK);  // back to the default
    EXPECT(prnu_get_tile(0, 16, 540, 960) == t0);
    EXPECT(prnu_get_tile(PRNU_TILE_SEG, 16, 540, 960) == 6);
    EXPECT_RC(prnu_set_tile(PRNU_TILE_SEG, 16, 540, 960, 12), PRNU_OK);
    EXPECT(prnu_get_tile(PRNU_TILE_SEG, 16, 540, 960) == 12);
    EXPECT_RC(prnu_set_tile(PRNU_TILE_SEG, 16, 540, 960, 5), PRNU_E_INVAL);
    EXPECT_RC(prnu_set_tile(PRNU_TILE_SEG, 16, 540, 960, 0), PRNU_OK);
    EXPECT_RC(prnu_set_tile(4, 16, 540, 960, 0), PRNU_E_INVAL);
    EXPECT_RC(prnu_autotune_workspace_size(1080, 1920, 1, &p, &n), PRNU_OK);
    EXPECT_RC(prnu_autotune_workspace_size(1080, 1920, 2, &p, &n), PRNU_E_INVAL);
    EXPECT_RC(prnu_autotune(1080, 1920, 1, &p, ws, 16, nullptr, nullptr), PRNU_E_WORKSPACE);
}

}  // namespace

int main(int argc, char **argv) {
    const std::string what = argc > 1 ? argv[1] : "all";
    if (what == "plant-heap") {
        volatile int *a = new int[4];
        const int v = a[argc + 2];  // one past the end
        delete[] a;
        return v;
    }
    if (what == "plant-ub") {
        volatile int big = INT32_MAX;
        return big + argc;  // signed overflow
    }
    if (what != "abi" && what != "batch" && what != "all") {
        std::fprintf(stderr, "usage: host_check [abi|batch|all]\n");
        return 2;
    }
    EXPECT(std::strlen(prnu_version()) > 0);
    if (what != "batch") {
        check_filters();
        check_workspace_sizes();
        check_validation();
    }
    if (what != "abi") check_batch();
    std::printf("host_check %s: %d checks, %d failed\n", what.c_str(), g_checks, g_failed);
    return g_failed ? 1 : 0;
}
