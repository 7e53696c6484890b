// sh_core.h -- the per-point formula core shared by the GPU kernels.
//
// Real spherical harmonics R_l^m, l <= 9, on a unit vector (x, y, z), from the
// paper's explicit factorised Cartesian formulas (Appendix C for m <= 0,
// Appendix B for m > 0), using only adds and multiplies and the pair factor
// p(a, b) = (a - b)(a + b) (eq. rpair).  Each value is
//     R_l^-m = kA[l][m] * Z_lm(z) * Shat_m(x, y),   R_l^+m = kB[l][m] * Z_lm(z) * Chat_m(x, y)
// (sh_constants.h documents the three factors).  Z_lm is shared by +m and -m,
// so each z-polynomial is evaluated once per point rather than once per sign of m.
//
// The arithmetic type T may be a scalar (double, float) or a clang vector of
// them (double2, float4, ...): a vector evaluates that many points at once,
// lane-wise, so adjacent points of one thread share every instruction.
//
// Row of (l, m) in every output: l*l + l + m.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "sh_constants.h"

namespace shk {

constexpr int row(int l, int m) { return l * l + l + m; }
constexpr int nfun(int lmax) { return (lmax + 1) * (lmax + 1); }

template <int B, int E, typename F>
__host__ __device__ __forceinline__ void static_for(F&& f)
{
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// The hardware deals consecutive workgroups round-robin to the 8 XCDs (each with
// its own L2).  xcd_tile(b, G) is the logical workgroup of hardware workgroup b
// in a grid of G: a bijection on [0, G) under which the workgroups each XCD runs
// form one contiguous range.
constexpr int kXcds = 8;

__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t G)
{
    const uint32_t q = G / kXcds, r = G % kXcds, x = b % kXcds;
    return x * q + (x < r ? x : r) + b / kXcds;
}

// Scalar type of a (possibly vector) arithmetic type.
template <typename T> struct scalar_of { using type = T; };
template <typename S, int N> struct scalar_of<S __attribute__((ext_vector_type(N)))> { using type = S; };
template <typename T> using scalar_t = typename scalar_of<T>::type;

typedef double double2_t __attribute__((ext_vector_type(2)));
typedef float float2_t __attribute__((ext_vector_type(2)));
typedef float float4_t __attribute__((ext_vector_type(4)));

// Constants in the scalar type of the polynomials.
template <typename T> struct K;
template <> struct K<double> {
    static __host__ __device__ constexpr double zroot(int l, int m, int k) { return shc::kZRoot[l][m][k]; }
    static __host__ __device__ constexpr double a(int l, int m) { return shc::kA[l][m]; }
    static __host__ __device__ constexpr double b(int l, int m) { return shc::kB[l][m]; }
    static __host__ __device__ constexpr double tans(int m, int k) { return shc::kTanS[m][k]; }
    static __host__ __device__ constexpr double tanc(int m, int k) { return shc::kTanC[m][k]; }
};
template <> struct K<float> {
    static __host__ __device__ constexpr float zroot(int l, int m, int k) { return shc::kZRootF[l][m][k]; }
    static __host__ __device__ constexpr float a(int l, int m) { return shc::kAF[l][m]; }
    static __host__ __device__ constexpr float b(int l, int m) { return shc::kBF[l][m]; }
    static __host__ __device__ constexpr float tans(int m, int k) { return shc::kTanSF[m][k]; }
    static __host__ __device__ constexpr float tanc(int m, int k) { return shc::kTanCF[m][k]; }
};

// Pair factor p(a, b) = (a - b)(a + b), eq. rpair: kept as a product of the two
// root factors rather than a^2 - b^2.
template <typename A, typename B>
__host__ __device__ __forceinline__ auto pf(A a, B b) { return (a - b) * (a + b); }

// p(c x, y) with each root factor c x -+ y one fused multiply-add.  The library is
// compiled with contraction only where the source writes it (-ffp-contract=on),
// so a point's value is the same whether it is evaluated alone or as a lane of a
// vector of adjacent points.
// (Other arithmetic types, such as the dual numbers of the backward pass, take
// the plain product.)
template <typename T> struct fma_lanes : std::is_floating_point<T> {};
template <typename S, int N> struct fma_lanes<S __attribute__((ext_vector_type(N)))> : std::true_type {};

template <typename T>
__host__ __device__ __forceinline__ T pfs(scalar_t<T> c, T x, T y)
{
    if constexpr (fma_lanes<T>::value) {
        const T cv = T(c);
        return __builtin_elementwise_fma(cv, x, -y) * __builtin_elementwise_fma(cv, x, y);
    } else {
        return pf(c * x, y);
    }
}

// Shat_m(x, y) = y * x^[m even] * prod_{k=1}^{ceil(m/2)-1} p(tan(k pi/m) x, y).
template <typename T, int M>
__host__ __device__ __forceinline__ T shat(T x, T y)
{
    T acc = y;
    if constexpr (M % 2 == 0) acc *= x;
    static_for<0, (M + 1) / 2 - 1>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        acc *= pfs<T>(K<scalar_t<T>>::tans(M, k), x, y);
    });
    return acc;
}

// Chat_m(x, y) = x^[m odd] * prod_{k=0}^{floor(m/2)-1} p(tan((k+1/2) pi/m) x, y).
template <typename T, int M>
__host__ __device__ __forceinline__ T chat(T x, T y)
{
    T acc;
    if constexpr (M % 2 == 1) acc = x;
    static_for<0, M / 2>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        const T f = pfs<T>(K<scalar_t<T>>::tanc(M, k), x, y);
        if constexpr (k == 0 && M % 2 == 0) acc = f;
        else acc *= f;
    });
    return acc;
}

// Z_lm(z) = z^((l-m) mod 2) * prod_k p(r_k, z), r_k the positive roots of d^m P_l/dz^m.
template <typename T, int L, int M>
__host__ __device__ __forceinline__ T zfac(T z)
{
    constexpr int np = (L - M) / 2;
    constexpr bool odd = ((L - M) & 1) != 0;
    if constexpr (np == 0) {
        if constexpr (odd) return z;
        else return T(scalar_t<T>(1));
    } else {
        T acc = pf(K<scalar_t<T>>::zroot(L, M, 0), z);
        static_for<1, np>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            acc *= pf(K<scalar_t<T>>::zroot(L, M, k), z);
        });
        if constexpr (odd) acc *= z;
        return acc;
    }
}

// All (LMAX+1)^2 values at the unit vector (x, y, z); sink(row, value) receives
// each one, m-major (so each xy factor is live only while its m is processed).
// `keep` multiplies the rows that are nonzero at x = y = z = 0 besides l = 0
// (even l > 0, m = 0): 1 normally, 0 at the origin, where only l = 0 survives
// (paper, Section 2).
template <int LMAX, typename T, typename Sink>
__host__ __device__ __forceinline__ void eval_unit(T x, T y, T z, T keep, Sink&& sink)
{
    static_assert(LMAX >= 0 && LMAX <= shc::kLmax, "lmax out of range");
    using KS = K<scalar_t<T>>;
    static_for<0, LMAX + 1>([&](auto mc) {
        constexpr int M = decltype(mc)::value;
        if constexpr (M == 0) {
            static_for<0, LMAX + 1>([&](auto lc) {
                constexpr int L = decltype(lc)::value;
                T v = KS::a(L, 0) * zfac<T, L, 0>(z);
                if constexpr (L > 0 && L % 2 == 0) v *= keep;
                sink(row(L, 0), v);
            });
        } else {
            const T s = shat<T, M>(x, y);
            const T c = chat<T, M>(x, y);
            static_for<M, LMAX + 1>([&](auto lc) {
                constexpr int L = decltype(lc)::value;
                const T zf = zfac<T, L, M>(z);
                sink(row(L, -M), KS::a(L, M) * zf * s);
                sink(row(L, M), KS::b(L, M) * zf * c);
            });
        }
    });
}

// Complex harmonics Y_l^m with the Condon-Shortley phase, from the real ones
// (Section 3): Y_l^0 = R_l^0 and, for m > 0,
//     Y_l^m = (-1)^m (R_l^m + i R_l^-m) / sqrt(2),   Y_l^-m = (R_l^m - i R_l^-m) / sqrt(2).
// sink(l, m, re, im) receives each one; +m and -m are formed together as soon as
// R_l^-m and R_l^m (which eval_unit delivers back to back) are both known.
template <int LMAX, typename T, typename Sink>
__host__ __device__ __forceinline__ void complex_unit(T x, T y, T z, T keep, Sink&& sink)
{
    const T h = T(scalar_t<T>(0.70710678118654752440));  // 1/sqrt(2)
    T sin_part = T(scalar_t<T>(0));
    eval_unit<LMAX, T>(x, y, z, keep, [&](int r, T v) {
        int l = 0;
        while ((l + 1) * (l + 1) <= r) ++l;
        const int m = r - l * l - l;
        if (m == 0) {
            sink(l, 0, v, T(scalar_t<T>(0)));
        } else if (m < 0) {
            sin_part = v;  // R_l^-|m| arrives just before R_l^|m|
        } else {
            const T re = h * v, im = h * sin_part;
            if (m & 1) sink(l, m, -re, -im);
            else sink(l, m, re, im);
            sink(l, -m, re, -im);
        }
    });
}

// Spin-1/2 spinor harmonics (eq. spinorial) from the complex ones.  For orbital
// l and total j = l +- 1/2,
//     j = l + 1/2: upper =  sqrt((l + m_j + 1/2)/(2l+1)) Y_l^{m_j-1/2},
//                  lower =  sqrt((l - m_j + 1/2)/(2l+1)) Y_l^{m_j+1/2},
//     j = l - 1/2: upper = -sqrt((l - m_j + 1/2)/(2l+1)) Y_l^{m_j-1/2},
//                  lower =  sqrt((l + m_j + 1/2)/(2l+1)) Y_l^{m_j+1/2},
// with Y_l^m = 0 for |m| > l.  Each Y_l^m therefore feeds at most four
// components with fixed coefficients and is passed on as soon as it is formed.
// Spinor index k (l-major; j = l - 1/2 first; m_j ascending):
//     j = l - 1/2: k = 2l^2 + (m_j + l - 1/2),   j = l + 1/2: k = 2l^2 + 2l + (m_j + l + 1/2).
// spinor_spread passes the components fed by one Y_l^m = re + i im to
// sink(k, c, re, im) (c = 0 for the upper component); coef(l, q) = sqrt(q/(2l+1)).
// Over all m of an l, every (k, c) of that l is delivered exactly once, the
// structural zeros included.
template <typename T, typename Coef, typename Sink>
__host__ __device__ __forceinline__ void spinor_spread(int l, int m, T re, T im, Coef&& coef, Sink&& sink)
{
    using S = scalar_t<T>;
    const int base = 2 * l * l;
    // j = l + 1/2: upper of m_j = m + 1/2, lower of m_j = m - 1/2
    const T cu = T(S(coef(l, l + m + 1))), cl = T(S(coef(l, l - m + 1)));
    sink(base + 3 * l + m + 1, 0, cu * re, cu * im);
    sink(base + 3 * l + m, 1, cl * re, cl * im);
    if (m <= l - 1) {  // j = l - 1/2, upper of m_j = m + 1/2
        const T c = T(S(-coef(l, l - m)));
        sink(base + l + m, 0, c * re, c * im);
    }
    if (m >= 1 - l) {  // j = l - 1/2, lower of m_j = m - 1/2
        const T c = T(S(coef(l, l + m)));
        sink(base + l + m - 1, 1, c * re, c * im);
    }
    const T zero = T(S(0));
    if (m == l) sink(base + 4 * l + 1, 1, zero, zero);  // j = l + 1/2, m_j = l + 1/2
    if (m == -l) sink(base + 2 * l, 0, zero, zero);     // j = l + 1/2, m_j = -l - 1/2
}

// sqrt(q / (2l + 1)) for the explicit kernels, whose (l, q) are compile-time
// constants after unrolling, so the square root folds away.
struct SpinorCoef {
    __host__ __device__ double operator()(int l, int q) const { return sqrt(double(q) / double(2 * l + 1)); }
};

template <int LMAX, typename T, typename Sink>
__host__ __device__ __forceinline__ void spinor_unit(T x, T y, T z, T keep, Sink&& sink)
{
    complex_unit<LMAX, T>(x, y, z, keep,
                          [&](int l, int m, T re, T im) { spinor_spread(l, m, re, im, SpinorCoef{}, sink); });
}

// 1/sqrt(a) for a > 0: the hardware estimate (v_rsq_f64) refined by two Newton
// steps y <- y + y (1 - a y^2) / 2, each evaluated with fused multiply-adds.
__device__ __forceinline__ double rsqrt_refined(double a)
{
    double y = __builtin_amdgcn_rsq(a);
    double e = __builtin_fma(-(a * y), y, 1.0);
    y = __builtin_fma(0.5 * y, e, y);
    e = __builtin_fma(-(a * y), y, 1.0);
    y = __builtin_fma(0.5 * y, e, y);
    return y;
}

// Unit vector of (x, y, z) in double, with the near-origin guard: coordinates
// whose squares would underflow (or overflow) are first scaled by an exact power
// of two, which leaves the direction unchanged.  At exactly r = 0 the unit vector
// is returned as 0 and keep = 0.  A NaN coordinate makes every component NaN.
// rinv receives 1/r of the unscaled point (0 at the origin; it overflows to inf
// only when r itself is below the smallest normal double).
__device__ __forceinline__ void normalize(double x, double y, double z, double& xb, double& yb,
                                          double& zb, double& keep, double& rinv)
{
    const double mx = fmax(fabs(x), fmax(fabs(y), fabs(z)));
    double s = 1.0;
    if (mx < 0x1p-500 || mx > 0x1p+500) {
        s = mx < 0x1p-500 ? 0x1p+600 : 0x1p-600;
        x *= s;
        y *= s;
        z *= s;
    }
    const double r2 = __builtin_fma(x, x, __builtin_fma(y, y, z * z));
    const bool nz = r2 > 0.0;
    const double ri = nz ? rsqrt_refined(r2) : r2 * 0.0;  // 0 at the origin, NaN for NaN
    xb = x * ri;
    yb = y * ri;
    zb = z * ri;
    keep = nz ? 1.0 : 0.0;
    rinv = ri * s;
}

__device__ __forceinline__ void normalize(double x, double y, double z, double& xb, double& yb,
                                          double& zb, double& keep)
{
    double rinv;
    normalize(x, y, z, xb, yb, zb, keep, rinv);
}

}  // namespace shk
