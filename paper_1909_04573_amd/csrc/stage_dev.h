// Device helpers for global-memory access.
//
// staged_copy: cooperative staging of global data into LDS.  Thread `tid` of
// a group of NTH threads handles elements tid, tid + NTH, ... of `count`; it
// issues up to KB loads before storing them, so a batch of global loads is in
// flight at once instead of one load per round trip.  The load callbacks must
// not branch around their loads either: they clamp indices to valid elements
// and select zero afterwards.
#pragma once

#include <hip/hip_runtime.h>

namespace prnu {

// Global-memory views of caller pointers.  Pointers the work-queue kernels
// read from their descriptor tables would otherwise be accessed with flat
// instructions, whose completion shares a wait counter with LDS reads and so
// serialises a tile's loads behind its LDS index look-ups.
#define PRNU_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ PRNU_GLOBAL T *gmem(T *p) {
    return (PRNU_GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ const PRNU_GLOBAL T *gmem(const T *p) {
    return (const PRNU_GLOBAL T *)p;
}
// Two consecutive floats (8-byte aligned) in one load.
__device__ __forceinline__ float2 ld2(const PRNU_GLOBAL float *p) {
    typedef float v2 __attribute__((ext_vector_type(2)));
    const v2 t = *(const PRNU_GLOBAL v2 *)p;
    return make_float2(t.x, t.y);
}
// Four consecutive 32-bit values (16-byte aligned) in one store.
template <typename T>
__device__ __forceinline__ void st4(PRNU_GLOBAL T *p, T a, T b, T c, T d) {
    typedef T v4 __attribute__((ext_vector_type(4)));
    *(PRNU_GLOBAL v4 *)p = v4{a, b, c, d};
}

// Workgroups are dispatched to the XCDs (each with its own L2) round robin in
// the order of their linear index.  Renumbering them so that XCD x takes the
// x-th contiguous range of virtual blocks keeps neighbouring tiles, which
// read overlapping input halos, in the same L2.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_order(int lin, int total) {
    const int q = total / NXCD, r = total - (total / NXCD) * NXCD;
    const int x = lin % NXCD, slot = lin / NXCD;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + slot;
}
// (tile, plane) of this workgroup of a grid (tiles, planes) in that order.
__device__ __forceinline__ void grid_tile(int &tile, int &plane) {
    const int tiles = (int)gridDim.x;
    const int v = xcd_order((int)(blockIdx.x + blockIdx.y * gridDim.x), (int)(gridDim.x * gridDim.y));
    plane = v / tiles;
    tile = v - plane * tiles;
}
// Planes fastest: the planes of one tile are consecutive virtual blocks (same
// XCD, close in time), for planes that read shared inputs at the same place
// (a query's modulation and a fingerprint, each used by several pairs).
__device__ __forceinline__ void grid_plane_major(int &tile, int &plane) {
    const int planes = (int)gridDim.y;
    const int v = xcd_order((int)(blockIdx.x + blockIdx.y * gridDim.x), (int)(gridDim.x * gridDim.y));
    tile = v / planes;
    plane = v - tile * planes;
}
// The same for planes that are the C interleaved channels of frames: the C
// channels of one tile are consecutive virtual blocks (same XCD, close in
// time), so the frame bytes they share come from one L2 fill.
__device__ __forceinline__ void grid_tile_channels(int &tile, int &plane, int C) {
    const int tiles = (int)gridDim.x;
    const int v = xcd_order((int)(blockIdx.x + blockIdx.y * gridDim.x), (int)(gridDim.x * gridDim.y));
    const int frame = v / (tiles * C), r = v - frame * (tiles * C);
    tile = r / C;
    plane = frame * C + (r - tile * C);
}

template <int NTH, int KB, typename T, typename Load, typename Store>
__device__ __forceinline__ void staged_copy(int tid, int count, Load load, Store store) {
    for (int e0 = tid; e0 < count; e0 += KB * NTH) {
        T v[KB];
        // neither loads nor stores sit behind a per-lane branch (elements
        // past the end load the last one again and store it to the same
        // place): the compiler then waits for each load only where its value
        // is stored, not for every load in flight after each one
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const int e = e0 + k * NTH;
            v[k] = load(e < count ? e : count - 1);
        }
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const int e = e0 + k * NTH;
            store(e < count ? e : count - 1, v[k]);
        }
    }
}

}  // namespace prnu
