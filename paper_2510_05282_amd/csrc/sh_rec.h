// sh_rec.h -- real harmonics of any l by the normalised Legendre recurrence
// (see sh_rec.hip for the formulas).  Host and device.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace shk {

// All (lmax+1)^2 values at the unit vector (x, y, z); store(row, value).  keep
// masks the m = 0 rows of l > 0 at the origin, as in eval_unit.
template <typename Store>
__host__ __device__ __forceinline__ void eval_unit_rec(double x, double y, double z, double keep, int lmax,
                                                       Store&& store)
{
    double d = 0.28209479177387814347;  // 1/sqrt(4 pi)
    double c = 1.0, s = 0.0;            // C_m, S_m
    for (int m = 0; m <= lmax; ++m) {
        if (m > 0) {
            d *= sqrt(double(2 * m + 1) / double(2 * m)) * (m == 1 ? 1.41421356237309504880 : 1.0);
            const double cn = x * c - y * s;
            s = x * s + y * c;
            c = cn;
        }
        double y2 = 0.0, y1 = d;  // Yb_{l-2}^m, Yb_{l-1}^m, starting at l = m
        for (int l = m; l <= lmax; ++l) {
            double yl;
            if (l == m) {
                yl = d;
            } else if (l == m + 1) {
                yl = sqrt(double(2 * m + 3)) * z * d;
            } else {
                const double l2 = double(l) * l, m2 = double(m) * m, lm1 = double(l - 1);
                const double a = sqrt((4.0 * l2 - 1.0) / (l2 - m2));
                const double b = sqrt((lm1 * lm1 - m2) / (4.0 * lm1 * lm1 - 1.0));
                yl = a * (z * y1 - b * y2);
            }
            if (l > m) {
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
