// sh_rec.h -- real harmonics of any l <= shc::kRecLmax by the normalised
// associated-Legendre recurrence (sh_rec.hip states the formulas; the
// coefficients are the generated tables of sh_rec_constants.h).  Host and device.
#pragma once

#include <hip/hip_runtime.h>

#include "sh_core.h"
#include "sh_rec_constants.h"

namespace shk {

// All (lmax+1)^2 values at the unit vector (x, y, z); store(row, value).  keep
// masks the m = 0 rows of l > 0 at the origin, as in eval_unit.  T is double or a
// clang vector of doubles (that many points at once).  The loops run over the
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
            const int r0 = l * l + l;
            if (m == 0) {
                store(r0, l > 0 ? yl * keep : yl);
            } else {
                store(r0 + m, yl * c);
                store(r0 - m, yl * s);
            }
        }
    }
}

}  // namespace shk
