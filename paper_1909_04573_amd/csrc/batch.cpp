// Batched fingerprint accumulation over many cameras of uneven geometry
// (SDA -> residual -> MLE of Sec. III-B for every camera in one launch
// sequence), and the tile-shape autotuner of the wavelet level kernels.
//
// Host side only: the schedule (jobs packed into rounds under a memory
// budget), the work tables of the persistent kernels, their upload into the
// caller's workspace, and optional capture of the whole sequence as one HIP
// graph.

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "host.h"
#include "internal.h"

struct prnu_batch {
    struct Launch {
        enum Kind { ZERO_CTR, ZERO_ACC, SDA, FWD, INV, MLE } kind;
        int tt = 32;
        int nd = 0;
        int64_t total = 0;
        int grid = 0;
        const void *desc = nullptr;
        int *ctr = nullptr;
        float *fill = nullptr;
        int64_t nfill = 0;
        double bytes = 0;  // algorithmic bytes (inputs read once, outputs written once)
        double flops = 0;  // algorithmic arithmetic
    };
    std::vector<Launch> launches;
    prnu::Filter f;
    int taps = 16, acc_mode = PRNU_ACC_F64;
    hipGraphExec_t exec = nullptr;
    prnu_batch_info info{};
};

namespace prnu {
namespace {

constexpr size_t kDefaultRoundBytes = 8ull << 30;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int n_groups(const prnu_camera &c) { return (c.n_frames + c.group - 1) / c.group; }

// Means and wavelet pyramid of `ng` SDA frames of camera c (carving order of
// the round area: means, then levels 1..L, each 256-byte aligned).
size_t job_bytes(const prnu_camera &c, int levels, int ng) {
    const int Hp = padded(c.H), Wp = padded(c.W);
    size_t b = align_up((size_t)ng * c.C * c.H * c.W * sizeof(float));
    for (int l = 1; l <= levels; ++l) b += align_up((size_t)ng * c.C * level_floats(Hp, Wp, l) * sizeof(float));
    return b;
}

struct Job {
    int cam, g0, ng;
};

// Rounds of jobs: at most one job per camera per round, a camera's jobs in
// increasing group order in increasing rounds (so its accumulator updates
// keep their order), each round's jobs within `budget` bytes.  Cameras with
// the most remaining bytes are served first; a round that could take nothing
// else takes one group of its first camera even above the budget.
std::vector<std::vector<Job>> schedule(const prnu_camera *cams, int n, int levels, size_t budget,
                                       size_t *round_max) {
    std::vector<int> rem(n), next(n, 0);
    std::vector<size_t> per(n);
    for (int j = 0; j < n; ++j) {
        rem[j] = n_groups(cams[j]);
        per[j] = job_bytes(cams[j], levels, 1);
    }
    std::vector<std::vector<Job>> rounds;
    *round_max = 0;
    for (;;) {
        std::vector<int> order;
        for (int j = 0; j < n; ++j)
            if (rem[j] > 0) order.push_back(j);
        if (order.empty()) break;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return (double)rem[a] * (double)per[a] > (double)rem[b] * (double)per[b];
        });
        std::vector<Job> round;
        size_t used = 0;
        for (int j : order) {
            const size_t left = budget > used ? budget - used : 0;
            int64_t k = std::min<int64_t>(rem[j], (int64_t)(left / per[j]) + 1);
            while (k > 0 && job_bytes(cams[j], levels, (int)k) > left) --k;
            if (k == 0 && round.empty()) k = 1;
            if (k == 0) continue;
            round.push_back({j, next[j], (int)k});
            used += job_bytes(cams[j], levels, (int)k);
            next[j] += (int)k;
            rem[j] -= (int)k;
        }
        *round_max = std::max(*round_max, used);
        rounds.push_back(std::move(round));
    }
    return rounds;
}

size_t acc_bytes(const prnu_camera &c, int acc_mode) {
    const size_t px = (size_t)c.C * c.H * c.W;
    return acc_mode == PRNU_ACC_F32 ? px * 4 : px * 8;  // KAHAN_F32: two float planes
}

int check_cameras(const prnu_camera *cams, int n, const char *fn) {
    if (!cams || n < 1) return fail(PRNU_E_INVAL, "%s: need at least one camera", fn);
    for (int j = 0; j < n; ++j) {
        const prnu_camera &c = cams[j];
        if (c.n_frames < 1 || c.group < 1)
            return fail(PRNU_E_INVAL, "%s: camera %d: n_frames and group must be >= 1", fn, j);
        if (c.n_frames > 16843009) return fail(PRNU_E_INVAL, "%s: camera %d: too many frames", fn, j);
        if (c.C != 1 && c.C != 3) return fail(PRNU_E_INVAL, "%s: camera %d: C must be 1 or 3", fn, j);
        if (check_dims(c.H, c.W, fn) != PRNU_OK)
            return fail(PRNU_E_INVAL, "%s: camera %d: H and W must be in [16, %d] (got %d x %d)", fn, j, kMaxDim,
                        c.H, c.W);
        if ((int64_t)c.H * c.W >= kMleMaxPixels)
            return fail(PRNU_E_INVAL, "%s: camera %d: frames of %d x %d exceed 2^28 pixels", fn, j, c.H, c.W);
    }
    return PRNU_OK;
}

// Work tables, counters and round area inside the workspace.
struct Layout {
    std::vector<std::vector<Job>> rounds;
    size_t round_max = 0;
    size_t tables = 0;   // bytes of all work tables
    int counters = 0;    // one per work-queue launch
    size_t ctr_off = 0, round_off = 0, total = 0;
};

// Descriptor tables per round: SDA, forward levels 1..L, inverse levels L..2,
// MLE; every level stage split by tile width (the kind's default first, then
// its small one).
struct StageCount {
    int nbig = 0, nsmall = 0;
};

int stage_tt(int kind, int taps, int hk, int wk) { return tile_choice(kind, taps, hk, wk); }

void count_stage(StageCount *sc, int kind, int tt) { (tt == tile_small(kind) ? sc->nsmall : sc->nbig)++; }

Layout plan_layout(const prnu_camera *cams, int n, const prnu_denoise_params *p, size_t budget) {
    Layout L;
    L.rounds = schedule(cams, n, p->levels, budget ? budget : kDefaultRoundBytes, &L.round_max);
    const int lv = p->levels;
    for (const auto &r : L.rounds) {
        const size_t nj = r.size();
        L.tables += align_up(nj * sizeof(SdaDesc));
        // every level stage: up to two tables (one per tile size) and counters
        for (int s = 0; s < 2 * lv; ++s) {
            StageCount sc;
            for (const Job &jb : r) {
                const prnu_camera &c = cams[jb.cam];
                const int Hp = padded(c.H), Wp = padded(c.W);
                int kind, l;
                if (s < lv) {
                    kind = TK_FWD;
                    l = s + 1;
                } else if (s < 2 * lv - 1) {
                    kind = TK_INV;
                    l = lv - (s - lv);  // L .. 2
                } else {
                    kind = TK_MLE;
                    l = 1;
                }
                count_stage(&sc, kind, stage_tt(kind, p->taps, Hp >> l, Wp >> l));
            }
            const size_t dsz = s < lv ? sizeof(FwdDesc) : s < 2 * lv - 1 ? sizeof(InvDesc) : sizeof(MleDesc);
            if (sc.nbig) {
                L.tables += align_up(sc.nbig * dsz);
                ++L.counters;
            }
            if (sc.nsmall) {
                L.tables += align_up(sc.nsmall * dsz);
                ++L.counters;
            }
        }
    }
    L.ctr_off = L.tables;
    L.round_off = align_up(L.ctr_off + (size_t)L.counters * sizeof(int));
    L.total = L.round_off + L.round_max;
    return L;
}

// Builds the tables (host blob mirrored at ws) and the launch list.
int build(const prnu_camera *cams, int n, int dtype, const prnu_denoise_params *p, int acc_mode, int flags,
          const Layout &L, char *ws, std::vector<char> *blob, prnu_batch *b) {
    const int lv = p->levels, taps = p->taps;
    const float s0 = p->sigma0 * p->sigma0;
    const int ncu = device_cus();
    blob->assign(L.tables, 0);
    size_t toff = 0;
    int ci = 0;
    int *ctr = reinterpret_cast<int *>(ws + L.ctr_off);
    using Launch = prnu_batch::Launch;
    Launch zc{};
    zc.kind = Launch::ZERO_CTR;
    zc.ctr = ctr;
    zc.total = L.counters;
    b->launches.push_back(zc);
    if (flags & PRNU_BATCH_ZERO_ACC) {
        for (int j = 0; j < n; ++j) {
            Launch z{};
            z.kind = Launch::ZERO_ACC;
            z.nfill = (int64_t)(acc_bytes(cams[j], acc_mode) / sizeof(float));
            z.fill = static_cast<float *>(cams[j].A);
            b->launches.push_back(z);
            z.fill = static_cast<float *>(cams[j].B);
            b->launches.push_back(z);
        }
    }
    auto grid_for = [&](int occ, int64_t total) {
        const int64_t g = std::max<int64_t>(1, (int64_t)occ * ncu);
        return (int)std::min<int64_t>(g, total);
    };
    for (const auto &r : L.rounds) {
        const int nj = (int)r.size();
        // carve each job's means and pyramid in the round area
        std::vector<float *> means(nj);
        std::vector<std::vector<float *>> lvl(nj, std::vector<float *>(lv + 1, nullptr));
        size_t off = L.round_off;
        for (int k = 0; k < nj; ++k) {
            const prnu_camera &c = cams[r[k].cam];
            const int ng = r[k].ng, Hp = padded(c.H), Wp = padded(c.W);
            means[k] = reinterpret_cast<float *>(ws + off);
            off += align_up((size_t)ng * c.C * c.H * c.W * sizeof(float));
            for (int l = 1; l <= lv; ++l) {
                lvl[k][l] = reinterpret_cast<float *>(ws + off);
                off += align_up((size_t)ng * c.C * level_floats(Hp, Wp, l) * sizeof(float));
            }
        }
        // SDA
        {
            SdaDesc *d = reinterpret_cast<SdaDesc *>(blob->data() + toff);
            int64_t blk = 0;
            for (int k = 0; k < nj; ++k) {
                const prnu_camera &c = cams[r[k].cam];
                const int64_t npx = (int64_t)c.H * c.W;
                const bool quad = sda_quad_ok(c.frames, npx * c.C * elem_bytes(dtype), dtype, npx, c.C, nullptr, means[k]);
                d[k] = SdaDesc{c.frames, npx, dtype, c.n_frames, c.C, c.group, r[k].g0, r[k].ng, quad ? 1 : 0,
                               sda_blocks_per_group(quad, npx), means[k], blk};
                blk += (int64_t)d[k].bpg * r[k].ng;
                b->info.sda_frames += r[k].ng;
                b->info.padded_pixels += (int64_t)r[k].ng * c.C * padded(c.H) * padded(c.W);
                b->info.input_bytes += (int64_t)(std::min(c.n_frames, (r[k].g0 + r[k].ng) * c.group) -
                                                 r[k].g0 * c.group) *
                                       npx * c.C * (int64_t)elem_bytes(dtype);
            }
            if (blk > 0x7fffffff) return fail(PRNU_E_INVAL, "prnu_batch: round of %lld SDA blocks", (long long)blk);
            Launch la{};
            for (int k = 0; k < nj; ++k) {
                const prnu_camera &c = cams[r[k].cam];
                const int64_t nread = std::min(c.n_frames, (r[k].g0 + r[k].ng) * c.group) - r[k].g0 * c.group;
                la.bytes += (double)nread * c.H * c.W * c.C * elem_bytes(dtype) + 4.0 * r[k].ng * c.C * c.H * c.W;
            }
            la.kind = Launch::SDA;
            la.desc = ws + toff;
            la.nd = nj;
            la.total = blk;
            b->launches.push_back(la);
            toff += align_up(nj * sizeof(SdaDesc));
        }
        // a level stage: descriptors of one tile size, virtual blocks tile-fastest
        auto emit_stage = [&](auto make, size_t dsz, int kind_tk, int level, Launch::Kind kind) -> int {
            for (int tt : {tile_default(kind_tk), tile_small(kind_tk)}) {
                int cnt = 0;
                for (int k = 0; k < nj; ++k) {
                    const prnu_camera &c = cams[r[k].cam];
                    cnt += stage_tt(kind_tk, taps, padded(c.H) >> level, padded(c.W) >> level) == tt;
                }
                if (!cnt) continue;
                if (toff + align_up(cnt * dsz) > L.tables || ci >= L.counters)
                    return fail(PRNU_E_INVAL, "prnu_batch: tile choices changed while the batch was planned");
                char *tab = blob->data() + toff;
                int nd = 0;
                int64_t blk = 0;
                double bytes = 0, flops = 0;
                for (int k = 0; k < nj; ++k) {
                    const prnu_camera &c = cams[r[k].cam];
                    const int Hp = padded(c.H), Wp = padded(c.W);
                    const int hk = Hp >> level, wk = Wp >> level;
                    if (stage_tt(kind_tk, taps, hk, wk) != tt || nd == cnt) continue;
                    int tiles = 0;
                    const int planes = make(k, tt, tab + nd * dsz, blk, &bytes, &flops, &tiles);
                    blk += (int64_t)tiles * planes;
                    ++nd;
                }
                if (!nd) continue;
                if (blk + 65536 > 0x7fffffff)
                    return fail(PRNU_E_INVAL, "prnu_batch: level stage of %lld tiles", (long long)blk);
                Launch la{};
                la.kind = kind;
                la.tt = tt;
                la.desc = ws + toff;
                la.nd = nd;
                la.total = blk;
                la.ctr = ctr + ci++;
                la.bytes = bytes;
                la.flops = flops;
                const int occ = kind == Launch::FWD   ? fwd_multi_occupancy(taps, tt)
                                : kind == Launch::INV ? inv_multi_occupancy(taps, tt)
                                                      : mle_multi_occupancy(taps, tt, acc_mode);
                la.grid = grid_for(occ, blk);
                b->launches.push_back(la);
                toff += align_up(nd * dsz);
            }
            return PRNU_OK;
        };
        for (int l = 1; l <= lv; ++l) {
            const float s2 = p->level_weight[l - 1] * s0;
            auto mk = [&](int k, int tt, char *dst, int64_t blk0, double *bytes, double *flops, int *ntiles) {
                const prnu_camera &c = cams[r[k].cam];
                const int Hp = padded(c.H), Wp = padded(c.W);
                const int planes = r[k].ng * c.C;
                FwdDesc d{};
                int strips = 0, seg = 0, tiles = 0;
                fwd_layout(p->taps, tt, Hp >> l, Wp >> l, planes, &strips, &seg, &tiles);
                if (l == 1)
                    d.a = FwdArgs{means[k], (int64_t)c.H * c.W, c.H, c.W, Hp, Wp, pad_before(c.H), pad_before(c.W),
                                  lvl[k][1], s2, strips, lv > 1 ? 1 : 0, nullptr, 0, nullptr, 0, seg};
                else {
                    const int nr = Hp >> (l - 1), nc = Wp >> (l - 1);
                    d.a = FwdArgs{lvl[k][l - 1], (int64_t)level_floats(Hp, Wp, l - 1), nr, nc, nr, nc, 0, 0,
                                  lvl[k][l], s2, strips, l < lv ? 1 : 0, nullptr, 0, nullptr, 0, seg};
                }
                d.tt = tt;
                d.tiles = tiles;
                *ntiles = tiles;
                d.planes = planes;
                d.block0 = blk0;
                std::memcpy(dst, &d, sizeof d);
                *bytes += 4.0 * planes *
                          ((double)d.a.src_rows * d.a.src_cols + (d.a.write_ll ? 4.0 : 3.0) * (Hp >> l) * (Wp >> l));
                *flops += (double)planes * d.a.n_r * d.a.n_c * fwd_flops_per_px(taps);
                return planes;
            };
            PRNU_TRY(emit_stage(mk, sizeof(FwdDesc), TK_FWD, l, Launch::FWD));
        }
        for (int l = lv; l >= 2; --l) {
            auto mk = [&](int k, int tt, char *dst, int64_t blk0, double *bytes, double *flops, int *ntiles) {
                const prnu_camera &c = cams[r[k].cam];
                const int Hp = padded(c.H), Wp = padded(c.W);
                const int planes = r[k].ng * c.C;
                const int hk = Hp >> l, wk = Wp >> l;
                InvDesc d{};
                d.a = InvArgs{lvl[k][l], hk, wk, l == lv ? 1 : 0, (wk + tt - 1) / tt, lvl[k][l - 1], 0, 0, 0, 0};
                d.tt = tt;
                d.tiles = tiles_for(tt, hk, wk);
                *ntiles = d.tiles;
                d.planes = planes;
                d.block0 = blk0;
                std::memcpy(dst, &d, sizeof d);
                *bytes += 4.0 * planes * ((l == lv ? 3.0 : 4.0) + 4.0) * hk * wk;
                *flops += (double)planes * 4.0 * hk * wk * inv_flops_per_px(taps);
                return planes;
            };
            PRNU_TRY(emit_stage(mk, sizeof(InvDesc), TK_INV, l, Launch::INV));
        }
        {
            auto mk = [&](int k, int tt, char *dst, int64_t blk0, double *bytes, double *flops, int *ntiles) {
                const prnu_camera &c = cams[r[k].cam];
                const int Hp = padded(c.H), Wp = padded(c.W);
                const int hk = Hp >> 1, wk = Wp >> 1;
                MleDesc d{};
                d.a = MleArgs{lvl[k][1], hk, wk, lv == 1 ? 1 : 0, (wk + tt - 1) / tt, r[k].ng, c.C, means[k], c.H,
                              c.W, pad_before(c.H), pad_before(c.W), c.A, c.B};
                d.tt = tt;
                d.tiles = tiles_for(tt, hk, wk);
                *ntiles = d.tiles;
                d.block0 = blk0;
                std::memcpy(dst, &d, sizeof d);
                const double accb = acc_mode == PRNU_ACC_F32 ? 16.0 : 32.0;  // A and B, read + write
                *bytes += 4.0 * r[k].ng * c.C * ((lv == 1 ? 3.0 : 4.0) * hk * wk + (double)c.H * c.W) +
                          accb * c.C * c.H * c.W;
                *flops += (double)r[k].ng * c.C * (4.0 * hk * wk * inv_flops_per_px(taps) + 4.0 * c.H * c.W);
                return c.C;
            };
            PRNU_TRY(emit_stage(mk, sizeof(MleDesc), TK_MLE, 1, Launch::MLE));
        }
    }
    if (toff != L.tables || ci != L.counters)
        return fail(PRNU_E_INVAL, "prnu_batch: internal table size mismatch");
    b->info.rounds = (int)L.rounds.size();
    b->info.launches = (int)b->launches.size();
    for (const auto &r : L.rounds) b->info.jobs += (int64_t)r.size();
    return PRNU_OK;
}

int enqueue(const prnu_batch *b, hipStream_t s) {
    using Launch = prnu_batch::Launch;
    static const char *fwd_names[2] = {"batch_fwd_wiener<32>", "batch_fwd_wiener<64>"};
    static const char *inv_names[2] = {"batch_inv<16>", "batch_inv<32>"};
    static const char *mle_names[2] = {"batch_inv_mle<16>", "batch_inv_mle<32>"};
    for (const Launch &la : b->launches) {
        hipError_t e = hipSuccess;
        const int t32 = la.tt == 32;
        switch (la.kind) {
            case Launch::ZERO_CTR: e = launch_zero_ints(la.ctr, (int)la.total, s); break;
            case Launch::ZERO_ACC: e = launch_fill_zero(la.fill, la.nfill, s); break;
            case Launch::SDA: {
                KernelTimer kt("batch_sda", la.bytes, s);
                e = launch_sda_multi(static_cast<const SdaDesc *>(la.desc), la.nd, la.total, s);
                break;
            }
            case Launch::FWD: {
                KernelTimer kt(fwd_names[la.tt == 64], la.bytes, s, la.flops);
                e = launch_fwd_multi(b->taps, la.tt, b->f, static_cast<const FwdDesc *>(la.desc), la.nd,
                                     (int)la.total, la.ctr, la.grid, s);
                break;
            }
            case Launch::INV: {
                KernelTimer kt(inv_names[t32], la.bytes, s, la.flops);
                e = launch_inv_multi(b->taps, la.tt, b->f, static_cast<const InvDesc *>(la.desc), la.nd,
                                     (int)la.total, la.ctr, la.grid, s);
                break;
            }
            case Launch::MLE: {
                KernelTimer kt(mle_names[t32], la.bytes, s, la.flops);
                e = launch_mle_multi(b->taps, la.tt, b->acc_mode, b->f, static_cast<const MleDesc *>(la.desc), la.nd,
                                     (int)la.total, la.ctr, la.grid, s);
                break;
            }
        }
        if (e != hipSuccess) return fail(PRNU_E_HIP, "prnu_batch: launch failed: %s", hipGetErrorString(e));
    }
    return PRNU_OK;
}

// Pairwise disjointness of all accumulator areas.
int check_acc_disjoint(const prnu_camera *cams, int n, int acc_mode, const char *fn) {
    std::vector<std::pair<uintptr_t, uintptr_t>> iv;
    for (int j = 0; j < n; ++j) {
        if (!cams[j].A || !cams[j].B) return fail(PRNU_E_INVAL, "%s: camera %d: null accumulator", fn, j);
        if (!cams[j].frames) return fail(PRNU_E_INVAL, "%s: camera %d: null frames", fn, j);
        const size_t nb = acc_bytes(cams[j], acc_mode);
        for (void *p : {cams[j].A, cams[j].B}) {
            const uintptr_t a = reinterpret_cast<uintptr_t>(p);
            iv.push_back({a, a + nb});
        }
    }
    std::sort(iv.begin(), iv.end());
    for (size_t i = 1; i < iv.size(); ++i)
        if (iv[i].first < iv[i - 1].second) return fail(PRNU_E_INVAL, "%s: accumulator areas overlap", fn);
    return PRNU_OK;
}

int create_impl(const char *fn, const prnu_camera *cams, int n, int dtype, const prnu_denoise_params *p,
                int acc_mode, int flags, size_t round_bytes, void *ws, size_t ws_bytes, void *stream,
                prnu_batch **out) {
    PRNU_TRY(check_cameras(cams, n, fn));
    PRNU_TRY(check_params(p, fn));
    if (dtype != PRNU_U8 && dtype != PRNU_BF16 && dtype != PRNU_F32)
        return fail(PRNU_E_INVAL, "%s: unknown dtype %d", fn, dtype);
    if (acc_mode != PRNU_ACC_F64 && acc_mode != PRNU_ACC_KAHAN_F32 && acc_mode != PRNU_ACC_F32)
        return fail(PRNU_E_INVAL, "%s: unknown acc_mode %d", fn, acc_mode);
    if (flags & ~(PRNU_BATCH_ZERO_ACC | PRNU_BATCH_GRAPH)) return fail(PRNU_E_INVAL, "%s: unknown flags", fn);
    PRNU_TRY(check_acc_disjoint(cams, n, acc_mode, fn));
    const Layout L = plan_layout(cams, n, p, round_bytes);
    if (!ws) return fail(PRNU_E_WORKSPACE, "%s: null workspace", fn);
    if (reinterpret_cast<uintptr_t>(ws) % kAlign)
        return fail(PRNU_E_WORKSPACE, "%s: workspace must be %zu-byte aligned", fn, kAlign);
    if (ws_bytes < L.total)
        return fail(PRNU_E_WORKSPACE, "%s: workspace of %zu bytes, %zu needed", fn, ws_bytes, L.total);
    prnu_batch *b = new (std::nothrow) prnu_batch;
    if (!b) return fail(PRNU_E_INVAL, "%s: out of host memory", fn);
    b->taps = p->taps;
    b->acc_mode = acc_mode;
    make_filter(p->taps, &b->f);
    std::vector<char> blob;
    int rc = build(cams, n, dtype, p, acc_mode, flags, L, static_cast<char *>(ws), &blob, b);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (rc == PRNU_OK && !blob.empty()) {
        hipError_t e = hipMemcpyAsync(ws, blob.data(), blob.size(), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = fail(PRNU_E_HIP, "%s: table upload failed: %s", fn, hipGetErrorString(e));
    }
    if (rc == PRNU_OK && (flags & PRNU_BATCH_GRAPH)) {
        hipStream_t cs = nullptr;
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            rc = enqueue(b, cs);
            const hipError_t e2 = hipStreamEndCapture(cs, &g);
            if (rc == PRNU_OK && e2 != hipSuccess) e = e2;
        }
        if (rc == PRNU_OK && e == hipSuccess) e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (rc == PRNU_OK && e != hipSuccess)
            rc = fail(PRNU_E_HIP, "%s: graph capture failed: %s", fn, hipGetErrorString(e));
        if (g) (void)hipGraphDestroy(g);
        if (cs) (void)hipStreamDestroy(cs);
    }
    if (rc != PRNU_OK) {
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        delete b;
        return rc;
    }
    *out = b;
    return PRNU_OK;
}

// ---- autotuner -----------------------------------------------------------------
struct TunePlan {
    int nb = 1, planes = 1;
    float *means = nullptr;
    float *lvl[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    void *A = nullptr, *B = nullptr;
};

// nb SDA frames of C planes, about 16 Mi padded pixels in all.
void plan_tune(Carver &cv, int H, int W, int C, int levels, TunePlan *tp) {
    const int64_t px = (int64_t)C * padded(H) * padded(W);
    // trial launches as large as fingerprint accumulation's batches, so the
    // tile chosen is the faster one at the size it will run
    tp->nb = (int)std::max<int64_t>(1, std::min<int64_t>(kMaxFramesPerMle, kAccBatchPixels / px));
    tp->planes = tp->nb * C;
    tp->means = cv.take<float>((size_t)tp->planes * H * W);
    for (int l = 1; l <= levels; ++l)
        tp->lvl[l] = cv.take<float>((size_t)tp->planes * level_floats(padded(H), padded(W), l));
    tp->A = cv.take<double>((size_t)C * H * W);
    tp->B = cv.take<double>((size_t)C * H * W);
}

}  // namespace
}  // namespace prnu

using namespace prnu;

extern "C" {

int prnu_batch_workspace_size(const prnu_camera *cams, int n_cams, const prnu_denoise_params *p, size_t round_bytes,
                              size_t *bytes) {
    const char *fn = "prnu_batch_workspace_size";
    set_error("");
    if (!bytes) return fail(PRNU_E_INVAL, "%s: null output", fn);
    PRNU_TRY(check_cameras(cams, n_cams, fn));
    PRNU_TRY(check_params(p, fn));
    *bytes = plan_layout(cams, n_cams, p, round_bytes).total;
    return PRNU_OK;
}

int prnu_batch_create(const prnu_camera *cams, int n_cams, int dtype, const prnu_denoise_params *p, int acc_mode,
                      int flags, size_t round_bytes, void *ws, size_t ws_bytes, void *stream, prnu_batch **out) {
    const char *fn = "prnu_batch_create";
    set_error("");
    if (!out) return fail(PRNU_E_INVAL, "%s: null output", fn);
    *out = nullptr;
    return create_impl(fn, cams, n_cams, dtype, p, acc_mode, flags, round_bytes, ws, ws_bytes, stream, out);
}

int prnu_batch_launch(prnu_batch *b, void *stream) {
    set_error("");
    if (!b) return fail(PRNU_E_INVAL, "prnu_batch_launch: null batch");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (b->exec) {
        const hipError_t e = hipGraphLaunch(b->exec, s);
        if (e != hipSuccess) return fail(PRNU_E_HIP, "prnu_batch_launch: %s", hipGetErrorString(e));
        return PRNU_OK;
    }
    return enqueue(b, s);
}

int prnu_batch_info_get(const prnu_batch *b, prnu_batch_info *info) {
    set_error("");
    if (!b || !info) return fail(PRNU_E_INVAL, "prnu_batch_info_get: null argument");
    *info = b->info;
    return PRNU_OK;
}

int prnu_batch_destroy(prnu_batch *b) {
    set_error("");
    if (!b) return PRNU_OK;
    int rc = PRNU_OK;
    if (b->exec) {
        const hipError_t e = hipGraphExecDestroy(b->exec);
        if (e != hipSuccess) rc = fail(PRNU_E_HIP, "prnu_batch_destroy: %s", hipGetErrorString(e));
    }
    delete b;
    return rc;
}

int prnu_fingerprint_batch(const prnu_camera *cams, int n_cams, int dtype, const prnu_denoise_params *p,
                           int acc_mode, size_t round_bytes, void *ws, size_t ws_bytes, void *stream) {
    const char *fn = "prnu_fingerprint_batch";
    set_error("");
    prnu_batch *b = nullptr;
    PRNU_TRY(create_impl(fn, cams, n_cams, dtype, p, acc_mode, 0, round_bytes, ws, ws_bytes, stream, &b));
    const int rc = enqueue(b, static_cast<hipStream_t>(stream));
    delete b;
    return rc;
}

int prnu_get_tile(int kind, int taps, int hk, int wk) {
    if (kind < PRNU_TILE_FWD || kind > PRNU_TILE_SEG) return 0;
    return tile_choice(kind, taps, hk, wk);
}

int prnu_set_tile(int kind, int taps, int hk, int wk, int tile) {
    set_error("");
    if (kind < PRNU_TILE_FWD || kind > PRNU_TILE_SEG) return fail(PRNU_E_INVAL, "prnu_set_tile: unknown kind");
    if (taps != 8 && taps != 16) return fail(PRNU_E_UNSUPPORTED, "prnu_set_tile: taps must be 8 or 16");
    if (hk < 1 || wk < 1) return fail(PRNU_E_INVAL, "prnu_set_tile: bad subband size");
    if (tile != 0 && !tile_valid(kind, tile)) {
        if (kind == PRNU_TILE_SEG) return fail(PRNU_E_INVAL, "prnu_set_tile: segment target must be 0, 3, 6 or 12");
        return fail(PRNU_E_INVAL, "prnu_set_tile: tile must be 0, %d or %d for this kind", tile_default(kind),
                    tile_small(kind));
    }
    set_tile_choice(kind, taps, hk, wk, tile == 0 ? tile_default(kind) : tile);
    return PRNU_OK;
}

int prnu_autotune_workspace_size(int H, int W, int C, const prnu_denoise_params *p, size_t *bytes) {
    const char *fn = "prnu_autotune_workspace_size";
    set_error("");
    if (!bytes) return fail(PRNU_E_INVAL, "%s: null output", fn);
    if (C != 1 && C != 3) return fail(PRNU_E_INVAL, "%s: C must be 1 or 3", fn);
    PRNU_TRY(check_dims(H, W, fn));
    PRNU_TRY(check_params(p, fn));
    Carver cv(nullptr);
    TunePlan tp;
    plan_tune(cv, H, W, C, p->levels, &tp);
    *bytes = cv.off;
    return PRNU_OK;
}

int prnu_autotune(int H, int W, int C, const prnu_denoise_params *p, void *ws, size_t ws_bytes, void *stream,
                  int *tiles) {
    const char *fn = "prnu_autotune";
    set_error("");
    if (C != 1 && C != 3) return fail(PRNU_E_INVAL, "%s: C must be 1 or 3", fn);
    PRNU_TRY(check_dims(H, W, fn));
    PRNU_TRY(check_params(p, fn));
    Carver cv(nullptr);
    TunePlan tp;
    plan_tune(cv, H, W, C, p->levels, &tp);
    PRNU_TRY(check_ws(cv, ws, ws_bytes, fn));
    Carver real(ws);
    plan_tune(real, H, W, C, p->levels, &tp);
    hipStream_t s = static_cast<hipStream_t>(stream);
    Filter f;
    make_filter(p->taps, &f);
    const int lv = p->levels, taps = p->taps, Hp = padded(H), Wp = padded(W);
    const float s0 = p->sigma0 * p->sigma0;
    // synthetic SDA means: hashed grey levels in [40, 220]
    PRNU_HIP(launch_fill_pattern(tp.means, (int64_t)tp.planes * H * W, s));
    PRNU_HIP(launch_fill_zero(static_cast<float *>(tp.A), (int64_t)2 * C * H * W, s));
    PRNU_HIP(launch_fill_zero(static_cast<float *>(tp.B), (int64_t)2 * C * H * W, s));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PRNU_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(PRNU_E_HIP, "%s: event creation failed", fn);
    }
    int rc = PRNU_OK;
    auto fwd = [&](int l) {
        const float s2 = p->level_weight[l - 1] * s0;
        if (l == 1)
            return launch_dwt_fwd(taps, f, tp.means, (int64_t)H * W, H, W, Hp, Wp, pad_before(H), pad_before(W),
                                  tp.lvl[1], tp.planes, s2, lv > 1, s);
        const int nr = Hp >> (l - 1), nc = Wp >> (l - 1);
        return launch_dwt_fwd(taps, f, tp.lvl[l - 1], (int64_t)level_floats(Hp, Wp, l - 1), nr, nc, nr, nc, 0, 0,
                              tp.lvl[l], tp.planes, s2, l < lv, s);
    };
    auto inv = [&](int l) {
        return launch_dwt_inv(taps, f, tp.lvl[l], Hp >> l, Wp >> l, l == lv, tp.planes, INV_PLANE, tp.lvl[l - 1], 0,
                              0, 0, 0, s);
    };
    auto mle = [&](int) {
        return launch_dwt_inv_mle(taps, f, tp.lvl[1], Hp / 2, Wp / 2, lv == 1, tp.nb, C, tp.means, H, W,
                                  pad_before(H), pad_before(W), PRNU_ACC_F64, tp.A, tp.B, s);
    };
    // time `reps` launches of one stage with tile tt; the fastest of the two is kept
    auto tune = [&](int kind, int l, auto run) -> int {
        const int hk = Hp >> l, wk = Wp >> l;
        float best_ms = 0.f;
        int best = tile_default(kind);
        for (int tt : {tile_default(kind), tile_small(kind)}) {
            set_tile_choice(kind, taps, hk, wk, tt);
            if (run(l) != hipSuccess) return 0;  // warm-up
            if (hipEventRecord(e0, s) != hipSuccess) return 0;
            for (int k = 0; k < 3; ++k)
                if (run(l) != hipSuccess) return 0;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 0;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 0;
            if (tt == tile_default(kind) || ms < best_ms) {
                best_ms = ms;
                best = tt;
            }
        }
        set_tile_choice(kind, taps, hk, wk, best);
        return best;
    };
    // the forward strip's segment target, timed with the chosen width
    auto tune_seg = [&](int l) -> int {
        const int hk = Hp >> l, wk = Wp >> l;
        float best_ms = 0.f;
        int best = tile_default(TK_SEG);
        for (int k : {tile_default(TK_SEG), tile_small(TK_SEG), 12}) {
            set_tile_choice(TK_SEG, taps, hk, wk, k);
            if (fwd(l) != hipSuccess) return 0;  // warm-up
            if (hipEventRecord(e0, s) != hipSuccess) return 0;
            for (int r = 0; r < 3; ++r)
                if (fwd(l) != hipSuccess) return 0;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return 0;
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return 0;
            if (k == tile_default(TK_SEG) || ms < best_ms) {
                best_ms = ms;
                best = k;
            }
        }
        set_tile_choice(TK_SEG, taps, hk, wk, best);
        return best;
    };
    int out[16] = {0};
    // the pyramid must hold every level before the inverse stages are timed
    for (int l = 1; l <= lv && rc == PRNU_OK; ++l) {
        out[l - 1] = tune(TK_FWD, l, fwd);
        if (out[l - 1]) out[12 + l - 1] = tune_seg(l);
        if (!out[l - 1] || !out[12 + l - 1]) rc = fail(PRNU_E_HIP, "%s: forward level %d failed", fn, l);
    }
    for (int l = lv; l >= 2 && rc == PRNU_OK; --l) {
        out[4 + l - 1] = tune(TK_INV, l, inv);
        if (!out[4 + l - 1]) rc = fail(PRNU_E_HIP, "%s: inverse level %d failed", fn, l);
    }
    if (rc == PRNU_OK) {
        out[8] = tune(TK_MLE, 1, mle);
        if (!out[8]) rc = fail(PRNU_E_HIP, "%s: MLE level failed", fn);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == PRNU_OK && tiles) std::memcpy(tiles, out, sizeof out);
    return rc;
}

}  // extern "C"
