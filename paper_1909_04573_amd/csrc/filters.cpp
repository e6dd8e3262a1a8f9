// Daubechies extremal-phase filters by spectral factorisation (host code).
//
// With y = sin^2(w/2), the squared low-pass response of the N-vanishing-moment
// Daubechies filter is cos^{2N}(w/2) P(y), P(y) = sum_{k<N} C(N-1+k, k) y^k.
// Every root y_r of P gives the reciprocal pair z, 1/z of z + 1/z = 2 - 4 y_r;
// taking the member outside the unit circle for each pair,
//     H(z) = sum_k h_k z^k  ~  (1 + z)^N prod_r (z - z_r),
// normalised to sum h = sqrt(2).  Roots of P are found with the
// Weierstrass (Durand-Kerner) iteration in complex long double, then polished
// by Newton steps on P.

#include <cmath>
#include <complex>
#include <cstring>
#include <mutex>

#include "internal.h"

namespace prnu {

using cld = std::complex<long double>;

static cld poly_eval(const long double *c, int deg, cld x) {  // c ascending
    cld acc = c[deg];
    for (int k = deg - 1; k >= 0; --k) acc = acc * x + c[k];
    return acc;
}

static cld poly_deriv(const long double *c, int deg, cld x) {
    cld acc = (long double)deg * c[deg];
    for (int k = deg - 1; k >= 1; --k) acc = acc * x + (long double)k * c[k];
    return acc;
}

bool daubechies_lowpass(int taps, long double *h) {
    if (taps < 2 || taps > 20 || (taps & 1)) return false;
    const int N = taps / 2;
    // P(y) coefficients, ascending: C(N-1+k, k)
    long double pc[16];
    for (int k = 0; k < N; ++k) {
        long double b = 1.0L;
        for (int i = 1; i <= k; ++i) b = b * (long double)(N - 1 + i) / (long double)i;
        pc[k] = b;
    }
    const int deg = N - 1;
    cld roots[16];
    if (deg > 0) {
        // Durand-Kerner on the monic polynomial
        long double mc[16];
        for (int k = 0; k <= deg; ++k) mc[k] = pc[k] / pc[deg];
        for (int i = 0; i < deg; ++i)
            roots[i] = std::pow(cld(0.4L, 0.9L), (long double)i) * 1.5L;  // distinct, off-axis
        for (int it = 0; it < 2000; ++it) {
            long double maxstep = 0.0L;
            for (int i = 0; i < deg; ++i) {
                cld num = poly_eval(mc, deg, roots[i]);
                cld den = 1.0L;
                for (int j = 0; j < deg; ++j)
                    if (j != i) den *= (roots[i] - roots[j]);
                cld step = num / den;
                roots[i] -= step;
                maxstep = std::max(maxstep, std::abs(step));
            }
            if (maxstep < 1e-30L) break;
        }
        for (int i = 0; i < deg; ++i)  // Newton polish on the original P
            for (int it = 0; it < 8; ++it) {
                cld d = poly_deriv(pc, deg, roots[i]);
                if (std::abs(d) == 0.0L) break;
                roots[i] -= poly_eval(pc, deg, roots[i]) / d;
            }
    }
    // H(z) = (1+z)^N prod (z - z_r), ascending coefficients
    cld poly[24];
    for (int k = 0; k < 24; ++k) poly[k] = 0.0L;
    poly[0] = 1.0L;
    int len = 1;
    auto mul = [&](cld a0, cld a1) {  // multiply by (a0 + a1 z)
        cld out[24];
        for (int k = 0; k <= len; ++k) out[k] = 0.0L;
        for (int k = 0; k < len; ++k) {
            out[k] += poly[k] * a0;
            out[k + 1] += poly[k] * a1;
        }
        ++len;
        for (int k = 0; k < len; ++k) poly[k] = out[k];
    };
    for (int k = 0; k < N; ++k) mul(1.0L, 1.0L);
    for (int r = 0; r < deg; ++r) {
        cld b = 2.0L - 4.0L * roots[r];
        cld disc = std::sqrt(b * b - 4.0L);
        cld z1 = (b + disc) / 2.0L, z2 = (b - disc) / 2.0L;
        cld z = std::abs(z1) > 1.0L ? z1 : z2;
        mul(-z, 1.0L);
    }
    long double s = 0.0L;
    for (int k = 0; k < taps; ++k) s += poly[k].real();
    const long double scale = std::sqrt(2.0L) / s;
    for (int k = 0; k < taps; ++k) h[k] = poly[k].real() * scale;
    return true;
}

// The root finding costs milliseconds of host time, so each filter length is
// built once per process and copied out afterwards.
bool make_filter(int taps, Filter *f) {
    if (taps != 8 && taps != 16) return false;
    static std::mutex mu;
    static Filter cache[2];
    static bool ready[2] = {false, false};
    const int slot = taps == 16;
    std::lock_guard<std::mutex> lk(mu);
    if (!ready[slot]) {
        long double h[20];
        if (!daubechies_lowpass(taps, h)) return false;
        Filter t;
        std::memset(&t, 0, sizeof(t));
        for (int k = 0; k < taps; ++k) {
            t.h[k] = (float)h[k];
            t.g[k] = (float)((k & 1 ? -1.0L : 1.0L) * h[taps - 1 - k]);
        }
        cache[slot] = t;
        ready[slot] = true;
    }
    *f = cache[slot];
    return true;
}

bool make_filter64(int taps, Filter64 *f) {
    if (taps != 8 && taps != 16) return false;
    long double h[20];
    if (!daubechies_lowpass(taps, h)) return false;
    std::memset(f, 0, sizeof(*f));
    f->taps = taps;
    for (int k = 0; k < taps; ++k) {
        f->h[k] = (double)h[k];
        f->g[k] = (double)((k & 1 ? -1.0L : 1.0L) * h[taps - 1 - k]);
    }
    return true;
}

}  // namespace prnu

extern "C" int prnu_filter_coefficients(int taps, double *h) {
    if (!h) return prnu::fail(PRNU_E_INVAL, "prnu_filter_coefficients: null output");
    long double t[20];
    if (!prnu::daubechies_lowpass(taps, t))
        return prnu::fail(PRNU_E_UNSUPPORTED, "prnu_filter_coefficients: taps must be even, 2..20");
    for (int k = 0; k < taps; ++k) h[k] = (double)t[k];
    return PRNU_OK;
}
