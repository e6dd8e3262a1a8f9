// Local-variance Wiener factor on an LDS tile (device helper).
//
// For a band of squared magnitudes q (zero outside the band, i.e. zero
// extension), the noise variance s2 and the centred windows w = 3, 5, 7, 9:
//     m_w  = (1/w^2) * sum of q over the w x w window
//     var  = min_w max(0, m_w - s2)
//     rho  = s2 / (var + s2)            (0 when the denominator is 0;
//                                        hardware reciprocal, <= 1 ulp)
// The caller multiplies its coefficient by rho: the noise part of it.
//
// One thread walks down one column of the tile core: every row's 3/5/7/9-wide
// horizontal sums enter a nine-row ring held in registers (static indices
// after full unrolling), and the vertical sums are re-added from the ring for
// each output row, so no running sum accumulates rounding error.
#pragma once

#include <hip/hip_runtime.h>

namespace prnu {

// load(row, col) returns q at tile position (row, col); rows r0 .. r0+NROWS+7
// and columns c .. c+8 are read; emit(row, rho, den) receives the factor of
// the coefficient at (row, c + 4) for rows r0+4 .. r0+NROWS+3, and
// den = var + s2 (the smallest window mean when it exceeds s2).
template <int NROWS, typename Load, typename Emit>
__device__ __forceinline__ void wiener_column(int r0, int c, float s2, Load load, Emit emit) {
    float h3[9], h5[9], h7[9], h9[9];
#pragma unroll
    for (int rr = 0; rr < NROWS + 8; ++rr) {
        const int row = r0 + rr;
        float q[9];
#pragma unroll
        for (int dx = 0; dx < 9; ++dx) q[dx] = load(row, c + dx);
        const float a3 = q[3] + q[4] + q[5];
        const float a5 = a3 + q[2] + q[6];
        const float a7 = a5 + q[1] + q[7];
        const float a9 = a7 + q[0] + q[8];
        h3[rr % 9] = a3;
        h5[rr % 9] = a5;
        h7[rr % 9] = a7;
        h9[rr % 9] = a9;
        if (rr >= 8) {
            float v3 = 0.f, v5 = 0.f, v7 = 0.f, v9 = 0.f;
#pragma unroll
            for (int d = -1; d <= 1; ++d) v3 += h3[(rr - 4 + d + 9) % 9];
#pragma unroll
            for (int d = -2; d <= 2; ++d) v5 += h5[(rr - 4 + d + 9) % 9];
#pragma unroll
            for (int d = -3; d <= 3; ++d) v7 += h7[(rr - 4 + d + 9) % 9];
#pragma unroll
            for (int d = -4; d <= 4; ++d) v9 += h9[(rr - 4 + d + 9) % 9];
            float est = fmaxf(0.f, v3 * (1.f / 9.f) - s2);
            est = fminf(est, fmaxf(0.f, v5 * (1.f / 25.f) - s2));
            est = fminf(est, fmaxf(0.f, v7 * (1.f / 49.f) - s2));
            est = fminf(est, fmaxf(0.f, v9 * (1.f / 81.f) - s2));
            const float den = est + s2;
            emit(row - 4, den > 0.f ? s2 * __builtin_amdgcn_rcpf(den) : 0.f, den);
        }
    }
}

}  // namespace prnu
