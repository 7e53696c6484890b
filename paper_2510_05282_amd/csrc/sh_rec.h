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
// masks the m = 0 rows of l > 0 at the origin, as in eval_unit.  T is double, float
// or a clang vector of them (that many points at once).  The loops run over the
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
                yl = S(shc::kRecE[m]) * z * d;
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

// v = sum over rows of G[row] grad_u P_row at the unit vector u = (x, y, z), for
// 0 <= lmax <= kRecLmax, where P is the off-sphere extension the recurrence
// evaluates: P_l^0 = Pb_l^0(z), P_l^m = Pb_l^m(z) C_m(x, y), P_l^-m = Pb_l^m(z) S_m(x, y)
// with C_m + i S_m = (x + i y)^m.  Its partials are
//     d(Pb C_m) = (m Pb C_{m-1}, -m Pb S_{m-1}, Pb' C_m),
//     d(Pb S_m) = (m Pb S_{m-1},  m Pb C_{m-1}, Pb' S_m),
// so per m only four sums over l are needed: a = sum G Pb and b = sum G Pb' for the
// cosine (+m) and sine (-m) rows.  Pb' follows from differentiating the recurrence:
// Pb_l' = A_l (Pb_{l-1} + z Pb_{l-1}' - B_l Pb_{l-2}').  g(row) returns G[row]; T is
// double, float or a clang vector of them.
template <typename T, typename GAt>
__host__ __device__ __forceinline__ void grad_unit_rec(T x, T y, T z, int lmax, GAt&& g, T& vx, T& vy, T& vz)
{
    using S = scalar_t<T>;
    const T zero = T(S(0));
    vx = zero;
    vy = zero;
    vz = zero;
    T c = T(S(1)), s = zero;  // C_m, S_m
    for (int m = 0; m <= lmax; ++m) {
        const T cp = c, sp = s;  // C_{m-1}, S_{m-1}
        if (m > 0) {
            c = x * cp - y * sp;
            s = x * sp + y * cp;
        }
        const S d = S(shc::kRecD[m]);
        T y1 = T(d), dy1 = zero, y2 = zero, dy2 = zero;  // Pb_{l-1}, Pb'_{l-1}, Pb_{l-2}, Pb'_{l-2}
        T ac = zero, bc = zero, as = zero, bs = zero;
        for (int l = m; l <= lmax; ++l) {
            T yl, dl;
            if (l == m) {
                yl = T(d);
                dl = zero;
            } else {
                const S a = l == m + 1 ? S(shc::kRecE[m]) : S(shc::kRecA[l][m]);
                const S b = l == m + 1 ? S(0) : S(shc::kRecB[l][m]);
                yl = a * (z * y1 - b * y2);
                dl = a * (y1 + z * dy1 - b * dy2);
                y2 = y1;
                dy2 = dy1;
                y1 = yl;
                dy1 = dl;
            }
            const T gc = g(row(l, m));
            ac += gc * yl;
            bc += gc * dl;
            if (m > 0) {
                const T gs = g(row(l, -m));
                as += gs * yl;
                bs += gs * dl;
            }
        }
        if (m == 0) {
            vz += bc;
        } else {
            const S fm = S(m);
            vx += fm * (ac * cp + as * sp);
            vy += fm * (as * cp - ac * sp);
            vz += bc * c + bs * s;
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
