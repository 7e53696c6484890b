// sh_proj.h -- per-point projector evaluation shared by the projector and
// serving kernels: spline lookup of R_l(r) and the product R_l(r) * R_l^m(d).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sh_core.h"

namespace shk {

struct SplineGrid {
    int n_r;
    double h, inv_h, r_max, h2_over_6;
};

// Spline value at r >= 0: interval i = floor(r/h) clamped to [0, n_r-2],
// t = r/h - i, A = 1 - t, B = t,
//     S = A y_i + B y_{i+1} + ((A^3 - A) M_i + (B^3 - B) M_{i+1}) h^2/6;
// 0 beyond r_max.
__device__ __forceinline__ double spline_eval(const double2* __restrict__ tab, const SplineGrid& g, double r)
{
    if (!(r <= g.r_max)) return r != r ? r : 0.0;  // NaN stays NaN
    const double q = r * g.inv_h;
    int i = int(q);
    i = i > g.n_r - 2 ? g.n_r - 2 : i;
    const double t = q - double(i);
    const double2 a = tab[i], b = tab[i + 1];
    const double A = 1.0 - t, B = t;
    return A * a.x + B * b.x + ((A * A * A - A) * a.y + (B * B * B - B) * b.y) * g.h2_over_6;
}

__host__ __device__ constexpr int l_of_row(int r)
{
    int l = 0;
    while ((l + 1) * (l + 1) <= r) ++l;
    return l;
}

// All projector values of one point: d = p - c, R_l(|d|) from `tab` (channel l
// at tab + l * n_r), harmonics of d; value of row f goes to out[f * stride].
template <int LMAX, typename TIO>
__device__ __forceinline__ void proj_point(const TIO* __restrict__ p, const double c[3],
                                           const double2* __restrict__ tab, const SplineGrid& g,
                                           TIO* __restrict__ out, int64_t stride)
{
    const double dx = double(p[0]) - c[0], dy = double(p[1]) - c[1], dz = double(p[2]) - c[2];
    double xb, yb, zb, keep;
    normalize(dx, dy, dz, xb, yb, zb, keep);
    const double r = sqrt(__builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz)));
    TIO R[LMAX + 1];
    static_for<0, LMAX + 1>([&](auto lc) {
        constexpr int L = decltype(lc)::value;
        R[L] = TIO(spline_eval(tab + int64_t(L) * g.n_r, g, r));
    });
    eval_unit<LMAX, TIO>(TIO(xb), TIO(yb), TIO(zb), TIO(keep), [&](int f, TIO v) {
        __builtin_nontemporal_store(R[l_of_row(f)] * v, out + int64_t(f) * stride);
    });
}

}  // namespace shk
