// Spatial-domain averaged frames (Sec. III-B): the mean of d consecutive frames.
//
// One thread owns 4 consecutive pixels of all C interleaved channels (4*C
// bytes of a u8 frame: one dword per channel-quad, so a wave reads a
// contiguous 256*C-byte span per frame) and walks the frames of its group,
// accumulating exact integer sums (u8) or double sums (bf16/f32).  It writes
// the de-interleaved planes: the sum (u8 only) and the correctly rounded
// float mean sum / count.  Grid: x = pixel quads, y = group.  Frame f starts
// fstride bytes after frame f - 1 (a frame's H x W x C samples are dense).
//
// Float frames: a sum that is not finite means a NaN or infinite sample in
// the group (finite floats cannot overflow a double sum of at most 2^24
// terms); such a wave ORs PRNU_STATUS_NONFINITE into *status once.

#include <hip/hip_bf16.h>

#include "internal.h"
#include "stage_dev.h"

namespace prnu {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ float bf16_to_float(uint16_t v) {
    return __uint_as_float((uint32_t)v << 16);
}

// u8 body: pixel quad block `bx` of absolute group gi, written as output group go.
template <int C>
__device__ __forceinline__ void sda_u8_body(const uint8_t *__restrict__ frames, int64_t fstride, int64_t npx,
                                            int n_frames, int group, int gi, int go, int64_t bx,
                                            uint32_t *__restrict__ sums, float *__restrict__ means) {
    const int64_t q = bx * kThreads + threadIdx.x;  // pixel quad
    if (q * 4 >= npx) return;
    const int f0 = gi * group;
    const int cnt = min(group, n_frames - f0);
    uint32_t acc[4 * C];
#pragma unroll
    for (int k = 0; k < 4 * C; ++k) acc[k] = 0;
    const PRNU_GLOBAL uint32_t *base =
        gmem(reinterpret_cast<const uint32_t *>(frames + (int64_t)f0 * fstride)) + q * C;
    const int64_t fwords = fstride / 4;  // a multiple of 4 bytes on this path
    int f = 0;
    for (; f + 4 <= cnt; f += 4) {
        uint32_t w[4][C];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k = 0; k < C; ++k) w[u][k] = __builtin_nontemporal_load(base + (f + u) * fwords + k);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k = 0; k < C; ++k)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[4 * k + b] += (w[u][k] >> (8 * b)) & 0xFFu;
    }
    for (; f < cnt; ++f) {
#pragma unroll
        for (int k = 0; k < C; ++k) {
            uint32_t w = __builtin_nontemporal_load(base + f * fwords + k);
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[4 * k + b] += (w >> (8 * b)) & 0xFFu;
        }
    }
    // byte e = 4k+b of the quad is pixel e / C, channel e % C
    const int64_t gbase = (int64_t)go * C * npx;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        uint32_t s[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) s[p] = acc[p * C + c];
        const int64_t o = gbase + (int64_t)c * npx + q * 4;
        if (sums) st4<uint32_t>(gmem(sums) + o, s[0], s[1], s[2], s[3]);
        if (means) {
            const float fc = (float)cnt;
            st4<float>(gmem(means) + o, (float)s[0] / fc, (float)s[1] / fc, (float)s[2] / fc, (float)s[3] / fc);
        }
    }
}

// Generic body: one thread per pixel, any layout / alignment / dtype.
template <int DT>
__device__ __forceinline__ void sda_generic_body(const void *__restrict__ frames, int64_t fstride, int64_t npx, int C,
                                                 int n_frames, int group, int gi, int go, int64_t bx,
                                                 uint32_t *__restrict__ sums, float *__restrict__ means,
                                                 uint32_t *__restrict__ status) {
    const int64_t p = bx * kThreads + threadIdx.x;
    if (p >= npx) return;
    const int f0 = gi * group;
    const int cnt = min(group, n_frames - f0);
    const int64_t gbase = (int64_t)go * C * npx;
    const PRNU_GLOBAL char *fb = gmem(static_cast<const char *>(frames)) + (int64_t)f0 * fstride;
    bool finite = true;
    for (int c = 0; c < C; ++c) {
        const int64_t e = p * C + c;  // sample of this pixel and channel within a frame
        if (DT == PRNU_U8) {
            uint32_t s = 0;
            for (int f = 0; f < cnt; ++f) s += reinterpret_cast<const PRNU_GLOBAL uint8_t *>(fb + f * fstride)[e];
            if (sums) gmem(sums)[gbase + (int64_t)c * npx + p] = s;
            if (means) gmem(means)[gbase + (int64_t)c * npx + p] = (float)s / (float)cnt;
        } else {
            double s = 0.0;
            for (int f = 0; f < cnt; ++f) {
                if (DT == PRNU_BF16)
                    s += (double)bf16_to_float(reinterpret_cast<const PRNU_GLOBAL uint16_t *>(fb + f * fstride)[e]);
                else
                    s += (double)reinterpret_cast<const PRNU_GLOBAL float *>(fb + f * fstride)[e];
            }
            finite = finite && __builtin_isfinite(s);
            if (means) gmem(means)[gbase + (int64_t)c * npx + p] = (float)(s / (double)cnt);
        }
    }
    if (DT != PRNU_U8 && status) {
        const uint64_t bad = __ballot(!finite);
        if (bad && __lane_id() == __ffsll((unsigned long long)bad) - 1) atomicOr(status, (uint32_t)PRNU_STATUS_NONFINITE);
    }
}

// Group sizes: the first thread of each group's first block writes counts[gi].
__device__ __forceinline__ void sda_count(int *counts, int n_frames, int group, int gi) {
    if (counts && blockIdx.x == 0 && threadIdx.x == 0) gmem(counts)[gi] = min(group, n_frames - gi * group);
}

template <int C>
__global__ __launch_bounds__(kThreads) void sda_u8_quads(const uint8_t *__restrict__ frames, int64_t fstride,
                                                         int64_t npx, int n_frames, int group, int g0,
                                                         uint32_t *__restrict__ sums, float *__restrict__ means,
                                                         int *__restrict__ counts) {
    sda_count(counts, n_frames, group, g0 + (int)blockIdx.y);
    sda_u8_body<C>(frames, fstride, npx, n_frames, group, g0 + (int)blockIdx.y, (int)blockIdx.y, blockIdx.x, sums,
                   means);
}

template <int DT>
__global__ __launch_bounds__(kThreads) void sda_generic(const void *__restrict__ frames, int64_t fstride, int64_t npx,
                                                        int C, int n_frames, int group, int g0,
                                                        uint32_t *__restrict__ sums, float *__restrict__ means,
                                                        int *__restrict__ counts, uint32_t *__restrict__ status) {
    sda_count(counts, n_frames, group, g0 + (int)blockIdx.y);
    sda_generic_body<DT>(frames, fstride, npx, C, n_frames, group, g0 + (int)blockIdx.y, (int)blockIdx.y, blockIdx.x,
                         sums, means, status);
}

// Batched SDA: block b of the 1-D grid belongs to the last descriptor with
// block0 <= b (block0 ascending, first 0); within it, block (b - block0) is
// pixel block (b - block0) % bpg of output group (b - block0) / bpg.
__global__ __launch_bounds__(kThreads) void sda_multi(const SdaDesc *__restrict__ d, int nd) {
    const int64_t vb = blockIdx.x;
    int lo = 0, hi = nd - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].block0 <= vb)
            lo = mid;
        else
            hi = mid - 1;
    }
    const SdaDesc D = d[lo];
    const int64_t local = vb - D.block0;
    const int go = (int)(local / D.bpg);
    const int64_t bx = local - (int64_t)go * D.bpg;
    if (go >= D.ng) return;
    const int gi = D.g0 + go;
    const int64_t fstride = D.npx * D.C * (D.dtype == PRNU_U8 ? 1 : D.dtype == PRNU_BF16 ? 2 : 4);
    if (D.quad) {
        const uint8_t *fr = static_cast<const uint8_t *>(D.frames);
        if (D.C == 3)
            sda_u8_body<3>(fr, fstride, D.npx, D.n_frames, D.group, gi, go, bx, nullptr, D.means);
        else
            sda_u8_body<1>(fr, fstride, D.npx, D.n_frames, D.group, gi, go, bx, nullptr, D.means);
    } else if (D.dtype == PRNU_U8) {
        sda_generic_body<PRNU_U8>(D.frames, fstride, D.npx, D.C, D.n_frames, D.group, gi, go, bx, nullptr, D.means,
                                  nullptr);
    } else if (D.dtype == PRNU_BF16) {
        sda_generic_body<PRNU_BF16>(D.frames, fstride, D.npx, D.C, D.n_frames, D.group, gi, go, bx, nullptr, D.means,
                                    nullptr);
    } else {
        sda_generic_body<PRNU_F32>(D.frames, fstride, D.npx, D.C, D.n_frames, D.group, gi, go, bx, nullptr, D.means,
                                   nullptr);
    }
}

}  // namespace

bool sda_quad_ok(const void *frames, int64_t fstride, int dtype, int64_t npx, int C, const void *sums,
                 const void *means) {
    return dtype == PRNU_U8 && (C == 1 || C == 3) && (npx % 4) == 0 && (fstride % 4) == 0 &&
           (reinterpret_cast<uintptr_t>(frames) % 4) == 0 &&
           (sums == nullptr || reinterpret_cast<uintptr_t>(sums) % 16 == 0) &&
           (means == nullptr || reinterpret_cast<uintptr_t>(means) % 16 == 0);
}

int sda_blocks_per_group(bool quad, int64_t npx) {
    return (int)(((quad ? npx / 4 : npx) + kThreads - 1) / kThreads);
}

hipError_t launch_sda_multi(const SdaDesc *d, int nd, int64_t total, hipStream_t s) {
    if (total <= 0 || nd <= 0) return hipSuccess;
    if (total > 0x7fffffff) return hipErrorInvalidValue;
    sda_multi<<<(unsigned)total, kThreads, 0, s>>>(d, nd);
    return hipGetLastError();
}

hipError_t launch_sda(const void *frames, int64_t fstride, int dtype, int n_frames, int H, int W, int C, int group,
                      int g0, int g1, uint32_t *sums, float *means, int *counts, uint32_t *status, hipStream_t s) {
    const int64_t npx = (int64_t)H * W;
    const int ng = g1 - g0;
    if (ng <= 0) return hipSuccess;
    const int64_t nread = (int64_t)min(n_frames, g1 * group) - (int64_t)g0 * group;
    const double esz = dtype == PRNU_U8 ? 1.0 : dtype == PRNU_BF16 ? 2.0 : 4.0;
    const double bytes = (double)nread * npx * C * esz +
                         (double)ng * C * npx * ((sums ? 4.0 : 0.0) + (means ? 4.0 : 0.0));
    if (sda_quad_ok(frames, fstride, dtype, npx, C, sums, means)) {
        dim3 grid((unsigned)((npx / 4 + kThreads - 1) / kThreads), (unsigned)ng);
        const uint8_t *fr = static_cast<const uint8_t *>(frames);
        KernelTimer kt(C == 1 ? "sda_u8_quads<1>" : "sda_u8_quads<3>", bytes, s);
        if (C == 1)
            sda_u8_quads<1><<<grid, kThreads, 0, s>>>(fr, fstride, npx, n_frames, group, g0, sums, means, counts);
        else
            sda_u8_quads<3><<<grid, kThreads, 0, s>>>(fr, fstride, npx, n_frames, group, g0, sums, means, counts);
    } else {
        dim3 grid((unsigned)((npx + kThreads - 1) / kThreads), (unsigned)ng);
        KernelTimer kt("sda_generic", bytes, s);
        if (dtype == PRNU_U8)
            sda_generic<PRNU_U8><<<grid, kThreads, 0, s>>>(frames, fstride, npx, C, n_frames, group, g0, sums, means,
                                                           counts, status);
        else if (dtype == PRNU_BF16)
            sda_generic<PRNU_BF16><<<grid, kThreads, 0, s>>>(frames, fstride, npx, C, n_frames, group, g0, sums,
                                                             means, counts, status);
        else
            sda_generic<PRNU_F32><<<grid, kThreads, 0, s>>>(frames, fstride, npx, C, n_frames, group, g0, sums,
                                                            means, counts, status);
    }
    return hipGetLastError();
}

// Frames-seen record of an accumulation: one thread adds this batch's counts
// after the batch's MLE fold on the same stream.
__global__ void acc_state_add(prnu_acc_state *st, int64_t frames, int64_t sda_frames) {
    if (threadIdx.x == 0) {
        gmem(&st->frames)[0] += frames;
        gmem(&st->sda_frames)[0] += sda_frames;
    }
}

hipError_t launch_acc_state_add(prnu_acc_state *st, int64_t frames, int64_t sda_frames, hipStream_t s) {
    acc_state_add<<<1, 64, 0, s>>>(st, frames, sda_frames);
    return hipGetLastError();
}

}  // namespace prnu
