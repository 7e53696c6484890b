// sh_rec.h -- real harmonics of any l <= shc::kRecLmax by the normalised
// associated-Legendre recurrence (sh_rec.hip states the formulas; the
// coefficients are the generated tables of sh_rec_constants.h).  Host and device.
#pragma once

#include <hip/hip_runtime.h>

#include "sh_core.h"
#include "sh_rec_constants.h"

namespace shk {

// All (lmax+1)^2 values at the unit vector (x, y, z); store(l, m, value), and for
// m > 0 the value of +m comes just before that of -m.  keep
// masks the m = 0 rows of l > 0 at the origin, as in eval_unit.  T is double or a
// clang vector of doubles (that many points at once), or a dual number of them
// (every constant multiplies from the left).  The loops run over the
// runtime lmax; every coefficient is a table entry indexed by (l, m) alone, so
// within a wave it is one scalar load.
template <typename T, typename Store>
__host__ __device__ __forceinline__ void eval_unit_rec(T x, T y, T z, T keep, int lmax, Store&& store)
{
    using S = scalar_t<T>;     // coefficients are rounded once to the arithmetic type
    T c = T(S(1)), s = T(S(0));  // C_m + i S_m = (x + i y)^m
    for (int m = 0; m <= lmax; ++m) {
        if (m > 0) {
            const T cn = x * c - y * s;
            s = x * s + y * c;
            c = cn;
        }
        const S d = S(shc::kRecD[m]);
        T y2 = T(S(0)), y1 = T(d);  // Yb_{l-2}^m, Yb_{l-1}^m
        for (int l = m; l <= lmax; ++l) {
            T yl;
            if (l == m) {
                yl = T(d);
            } else if (l == m + 1) {
                yl = (S(shc::kRecE[m]) * d) * z;
                y2 = y1;
                y1 = yl;
            } else {
                yl = S(shc::kRecA[l][m]) * (z * y1 - S(shc::kRecB[l][m]) * y2);
                y2 = y1;
                y1 = yl;
            }
            if (m == 0) {
                store(l, 0, l > 0 ? yl * keep : yl);
            } else {
                store(l, m, yl * c);
                store(l, -m, yl * s);
            }
        }
    }
}

// Complex harmonics (Condon-Shortley phase) from the recurrence's real values, as
// complex_unit does for the explicit ones: Y_l^0 = R_l^0, and for m > 0
//     Y_l^m = (-1)^m (R_l^m + i R_l^-m) / sqrt(2),   Y_l^-m = (R_l^m - i R_l^-m) / sqrt(2);
// sink(l, m, re, im).
template <typename T, typename Sink>
__host__ __device__ __forceinline__ void complex_unit_rec(T x, T y, T z, T keep, int lmax, Sink&& sink)
{
    using S = scalar_t<T>;
    const T h = T(S(0.70710678118654752440));  // 1/sqrt(2)
    T cos_part = T(S(0));
    eval_unit_rec<T>(x, y, z, keep, lmax, [&](int l, int m, T v) {
        if (m == 0) {
            sink(l, 0, v, T(S(0)));
        } else if (m > 0) {
            cos_part = v;  // R_l^m arrives just before R_l^-m
        } else {
            const T re = h * cos_part, im = h * v;
            if (-m & 1) sink(l, -m, -re, -im);
            else sink(l, -m, re, im);
            sink(l, m, re, -im);
        }
    });
}

// Spinor harmonics (eq. spinorial) from complex_unit_rec, with the coefficient
// table of sh_rec_constants.h; sink(k, c, re, im) as for spinor_unit.
template <typename T, typename Sink>
__host__ __device__ __forceinline__ void spinor_unit_rec(T x, T y, T z, T keep, int lmax, Sink&& sink)
{
    complex_unit_rec<T>(x, y, z, keep, lmax, [&](int l, int m, T re, T im) {
        spinor_spread(l, m, re, im, [](int ll, int q) { return shc::kSpinP[ll][q]; }, sink);
    });
}

}  // namespace shk
