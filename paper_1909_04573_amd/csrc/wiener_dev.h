// Local-variance Wiener factor on an LDS tile (device helper).
//
// For a band of squared magnitudes q (zero outside the band, i.e. zero
// extension), the noise variance s2 and the centred windows w = 3, 5, 7, 9:
//     m_w  = (1/w^2) * sum of q over the w x w window
//     var  = min_w max(0, m_w - s2)
//     rho  = s2 / (var + s2) = s2 / max(s2, min_w m_w)
//                                       (0 when the denominator is 0;
//                                        hardware reciprocal, <= 1 ulp)
// The caller multiplies its coefficient by rho: the noise part of it.
//
// One thread walks down one column of the tile core: every row's 3/5/7/9-wide
// horizontal sums enter a nine-row ring held in registers (static indices
// after full unrolling), together with the sums of each row and the next, and
// the vertical sums of every output row are re-added from the ring (from
// pair sums: 14 additions for the four windows), so no running sum
// accumulates rounding error.
#pragma once

#include <hip/hip_runtime.h>

namespace prnu {

// load(row, col) returns q at tile position (row, col); rows r0 .. r0+NROWS+7
// and columns c .. c+8 are read; emit(row, rho, den) receives the factor of
// the coefficient at (row, c + 4) for rows r0+4 .. r0+NROWS+3, and
// den = max(s2, smallest window mean).
template <int NROWS, typename Load, typename Emit>
__device__ __forceinline__ void wiener_column(int r0, int c, float s2, Load load, Emit emit) {
    float h3[9], h5[9], h7[9], h9[9];  // horizontal sums of row rr (ring index rr % 9)
    float p3[9], p5[9], p7[9], p9[9];  // h(rr - 1) + h(rr), valid from rr >= 1
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
        const int i = rr % 9;
        if (rr >= 1) {
            const int ip = (rr + 8) % 9;
            p3[i] = h3[ip] + a3;
            p5[i] = h5[ip] + a5;
            p7[i] = h7[ip] + a7;
            p9[i] = h9[ip] + a9;
        }
        h3[i] = a3;
        h5[i] = a5;
        h7[i] = a7;
        h9[i] = a9;
        if (rr >= 8) {
            // output row o = rr - 4; window rows o-r .. o+r as pairs ending at o-r+1, o-r+3, ...
            const int o = rr - 4;
            const float v3 = p3[(o + 9) % 9] + h3[(o + 1) % 9];                                  // (o-1,o), o+1
            const float v5 = p5[(o - 1 + 9) % 9] + p5[(o + 1) % 9] + h5[(o + 2) % 9];            // (o-2,o-1), (o,o+1), o+2
            const float v7 = p7[(o - 2 + 9) % 9] + p7[(o + 9) % 9] + p7[(o + 2) % 9] + h7[(o + 3) % 9];
            const float v9 = p9[(o - 3 + 9) % 9] + p9[(o - 1 + 9) % 9] + p9[(o + 1) % 9] + p9[(o + 3) % 9] +
                             h9[(o + 4) % 9];
            float m = fminf(v3 * (1.f / 9.f), v5 * (1.f / 25.f));
            m = fminf(m, v7 * (1.f / 49.f));
            m = fminf(m, v9 * (1.f / 81.f));
            const float den = fmaxf(s2, m);
            emit(row - 4, den > 0.f ? s2 * __builtin_amdgcn_rcpf(den) : 0.f, den);
        }
    }
}

}  // namespace prnu
