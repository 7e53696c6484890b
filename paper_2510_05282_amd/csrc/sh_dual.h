// sh_dual.h -- forward-mode dual numbers for the formula core.
//
// Dual<T, N> carries a value and N partial derivatives.  Running the factorised
// formulas of sh_core.h on duals gives, by the product rule applied factor by
// factor, the exact derivatives of the implemented polynomials: Z_lm and dZ_lm/dz
// from a Dual<double, 1> seeded with dz = 1, and Shat_m, Chat_m with their x and
// y partials from Dual<double, 2> seeded with dx = (1, 0), dy = (0, 1).
#pragma once

#include <hip/hip_runtime.h>

#include "sh_core.h"

namespace shk {

template <typename T, int N>
struct Dual {
    T v;
    T d[N];
    __host__ __device__ Dual() = default;
    // a constant: value c, derivatives 0
    __host__ __device__ explicit Dual(T c) : v(c)
    {
        for (int k = 0; k < N; ++k) d[k] = T(0);
    }
    // the variable number `k`: value c, derivative 1 in direction k
    static __host__ __device__ Dual var(T c, int k)
    {
        Dual r(c);
        r.d[k] = T(1);
        return r;
    }
};

template <typename T, int N> struct scalar_of<Dual<T, N>> { using type = scalar_t<T>; };

template <typename T, int N>
__host__ __device__ __forceinline__ Dual<T, N> operator+(const Dual<T, N>& a, const Dual<T, N>& b)
{
    Dual<T, N> r;
    r.v = a.v + b.v;
    for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k];
    return r;
}
template <typename T, int N>
__host__ __device__ __forceinline__ Dual<T, N> operator-(const Dual<T, N>& a, const Dual<T, N>& b)
{
    Dual<T, N> r;
    r.v = a.v - b.v;
    for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k];
    return r;
}
template <typename T, int N>
__host__ __device__ __forceinline__ Dual<T, N> operator*(const Dual<T, N>& a, const Dual<T, N>& b)
{
    Dual<T, N> r;
    r.v = a.v * b.v;
    for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
template <typename T, int N>
__host__ __device__ __forceinline__ Dual<T, N>& operator*=(Dual<T, N>& a, const Dual<T, N>& b)
{
    a = a * b;
    return a;
}
// mixed with a constant of the scalar type
template <typename T, int N>
__host__ __device__ __forceinline__ Dual<T, N> operator*(scalar_t<T> c, const Dual<T, N>& a)
{
    Dual<T, N> r;
    r.v = c * a.v;
    for (int k = 0; k < N; ++k) r.d[k] = c * a.d[k];
    return r;
}
template <typename T, int N>
__host__ __device__ __forceinline__ Dual<T, N> operator-(scalar_t<T> c, const Dual<T, N>& a)
{
    Dual<T, N> r;
    r.v = c - a.v;
    for (int k = 0; k < N; ++k) r.d[k] = -a.d[k];
    return r;
}
template <typename T, int N>
__host__ __device__ __forceinline__ Dual<T, N> operator+(scalar_t<T> c, const Dual<T, N>& a)
{
    Dual<T, N> r;
    r.v = c + a.v;
    for (int k = 0; k < N; ++k) r.d[k] = a.d[k];
    return r;
}

// Polynomial gradient contracted with an upstream gradient:
//     v = sum_{l,m} g(row(l,m)) grad_u P_lm(u)   at the unit vector u = (x, y, z),
// where g(row) returns the upstream value of a row.  Written to (vx, vy, vz).
// T is the arithmetic type of the polynomials (double or float).
template <int LMAX, typename T, typename GetG>
__host__ __device__ __forceinline__ void grad_unit(T x, T y, T z, GetG&& g, T& vx, T& vy, T& vz)
{
    using D1 = Dual<T, 1>;
    using D2 = Dual<T, 2>;
    const D1 zd = D1::var(z, 0);
    const D2 xd = D2::var(x, 0), yd = D2::var(y, 1);
    vx = T(0);
    vy = T(0);
    vz = T(0);
    static_for<0, LMAX + 1>([&](auto mc) {
        constexpr int M = decltype(mc)::value;
        if constexpr (M == 0) {
            static_for<1, LMAX + 1>([&](auto lc) {
                constexpr int L = decltype(lc)::value;
                const D1 Z = zfac<D1, L, 0>(zd);
                vz += g(row(L, 0)) * (K<scalar_t<T>>::a(L, 0) * Z.d[0]);
            });
        } else {
            const D2 S = shat<D2, M>(xd, yd);
            const D2 C = chat<D2, M>(xd, yd);
            T aS = T(0), aC = T(0), bS = T(0), bC = T(0);
            static_for<M, LMAX + 1>([&](auto lc) {
                constexpr int L = decltype(lc)::value;
                const D1 Z = zfac<D1, L, M>(zd);
                const T gs = g(row(L, -M)) * K<scalar_t<T>>::a(L, M);
                const T gc = g(row(L, M)) * K<scalar_t<T>>::b(L, M);
                aS += gs * Z.v;
                bS += gs * Z.d[0];
                aC += gc * Z.v;
                bC += gc * Z.d[0];
            });
            vx += aS * S.d[0] + aC * C.d[0];
            vy += aS * S.d[1] + aC * C.d[1];
            vz += bS * S.v + bC * C.v;
        }
    });
}

// Every value and its polynomial gradient at the unit vector u = (x, y, z):
// sink(row, P, dP/dx, dP/dy, dP/dz).  `keep` masks the rows that are nonzero at
// u = 0 besides l = 0 (as in eval_unit).
template <int LMAX, typename T, typename Sink>
__host__ __device__ __forceinline__ void eval_unit_jac(T x, T y, T z, T keep, Sink&& sink)
{
    using D1 = Dual<T, 1>;
    using D2 = Dual<T, 2>;
    const D1 zd = D1::var(z, 0);
    const D2 xd = D2::var(x, 0), yd = D2::var(y, 1);
    static_for<0, LMAX + 1>([&](auto mc) {
        constexpr int M = decltype(mc)::value;
        if constexpr (M == 0) {
            static_for<0, LMAX + 1>([&](auto lc) {
                constexpr int L = decltype(lc)::value;
                const D1 Z = zfac<D1, L, 0>(zd);
                T v = K<scalar_t<T>>::a(L, 0) * Z.v;
                if constexpr (L > 0 && L % 2 == 0) v *= keep;
                sink(row(L, 0), v, T(0), T(0), K<scalar_t<T>>::a(L, 0) * Z.d[0]);
            });
        } else {
            const D2 S = shat<D2, M>(xd, yd);
            const D2 C = chat<D2, M>(xd, yd);
            static_for<M, LMAX + 1>([&](auto lc) {
                constexpr int L = decltype(lc)::value;
                const D1 Z = zfac<D1, L, M>(zd);
                const T a = K<scalar_t<T>>::a(L, M) * Z.v, ad = K<scalar_t<T>>::a(L, M) * Z.d[0];
                const T b = K<scalar_t<T>>::b(L, M) * Z.v, bd = K<scalar_t<T>>::b(L, M) * Z.d[0];
                sink(row(L, -M), a * S.v, a * S.d[0], a * S.d[1], ad * S.v);
                sink(row(L, M), b * C.v, b * C.d[0], b * C.d[1], bd * C.v);
            });
        }
    });
}

}  // namespace shk
