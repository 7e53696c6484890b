// sh_proj.h -- per-point projector evaluation shared by the projector and
// serving kernels: spline lookup of R_l(r) and the product R_l(r) * R_l^m(d).
//
// Radial table layout (one table): [n_r][ch] of (y_i, M_i) -- knot i of every
// channel is adjacent, so the interval [i, i+1] of all channels of a point is
// 2 ch consecutive double2 (one 128-byte line for ch = 4) instead of ch lines
// n_r * 16 bytes apart.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sh_core.h"
#include "sh_fwd.h"
#include "sh_internal.h"

namespace shk {

struct SplineGrid {
    int n_r;
    double h, inv_h, r_max, h2_over_6;
};

// R_0 .. R_{NL-1} at r >= 0 from a table with ch >= NL channels: interval
// i = floor(r/h) clamped to [0, n_r-2], t = r/h - i, A = 1 - t, B = t,
//     S = A y_i + B y_{i+1} + ((A^3 - A) M_i + (B^3 - B) M_{i+1}) h^2/6;
// 0 beyond r_max; a NaN r gives NaN.  Split in two steps: spline_knots loads
// the pairs of knots i and i+1 (for any r: beyond r_max or NaN it reads interval 0,
// which spline_from then ignores), spline_from evaluates the cubic from them.
__host__ __device__ __forceinline__ int spline_interval(double r, const SplineGrid& g)
{
    const double q = r <= g.r_max ? r * g.inv_h : 0.0;
    const int i = int(q);
    return i > g.n_r - 2 ? g.n_r - 2 : i;
}

template <int NL, typename KN>
__host__ __device__ __forceinline__ void spline_knots(const KN* __restrict__ tab, int ch, const SplineGrid& g,
                                                      double r, KN (&a)[NL], KN (&b)[NL])
{
    const KN* k0 = tab + int64_t(spline_interval(r, g)) * ch;
    static_for<0, NL>([&](auto lc) {
        constexpr int L = decltype(lc)::value;
        a[L] = k0[L];
        b[L] = k0[ch + L];
    });
}

template <int NL, typename TIO>
__host__ __device__ __forceinline__ void spline_from(const double2 (&a)[NL], const double2 (&b)[NL],
                                                     const SplineGrid& g, double r, TIO (&R)[NL])
{
    if (!(r <= g.r_max)) {
        const double v = r != r ? r : 0.0;
        static_for<0, NL>([&](auto lc) { R[decltype(lc)::value] = TIO(v); });
        return;
    }
    const double q = r * g.inv_h;
    const double t = q - double(spline_interval(r, g));
    const double A = 1.0 - t, B = t;
    static_for<0, NL>([&](auto lc) {
        constexpr int L = decltype(lc)::value;
        R[L] = TIO(A * a[L].x + B * b[L].x + ((A * A * A - A) * a[L].y + (B * B * B - B) * b[L].y) * g.h2_over_6);
    });
}

// The same from float pairs, for the FP32 kernels: the interval i and t = r/h - i
// in FP64 (near r_max, r/h is ~n_r, and float would leave t only a few bits), the
// cubic in FP32.  Table values rounded to float and the FP32 cubic put at most a
// few 1e-7 (of max|R|) into R, well inside the FP32 tolerance.
template <int NL, typename TIO>
__host__ __device__ __forceinline__ void spline_from(const float2 (&a)[NL], const float2 (&b)[NL],
                                                     const SplineGrid& g, double r, TIO (&R)[NL])
{
    static_assert(sizeof(TIO) == 4, "float tables serve the FP32 kernels");
    if (!(r <= g.r_max)) {
        const float v = r != r ? float(r) : 0.0f;
        static_for<0, NL>([&](auto lc) { R[decltype(lc)::value] = v; });
        return;
    }
    const double q = r * g.inv_h;
    const float t = float(q - double(spline_interval(r, g)));
    const float A = 1.0f - t, B = t, h26 = float(g.h2_over_6);
    static_for<0, NL>([&](auto lc) {
        constexpr int L = decltype(lc)::value;
        R[L] = A * a[L].x + B * b[L].x + ((A * A * A - A) * a[L].y + (B * B * B - B) * b[L].y) * h26;
    });
}

// Both steps for one point, with the loads skipped beyond r_max.
template <int NL, typename TIO, typename KN>
__host__ __device__ __forceinline__ void spline_eval(const KN* __restrict__ tab, int ch, const SplineGrid& g,
                                                     double r, TIO (&R)[NL])
{
    KN a[NL], b[NL];
    if (r <= g.r_max) spline_knots<NL>(tab, ch, g, r, a, b);
    spline_from<NL, TIO>(a, b, g, r, R);
}

// Natural cubic spline on a uniform grid for one channel.  With knot spacing h
// the second derivatives solve, for k = 1 .. n_r-2,
//     M_{k-1} + 4 M_k + M_{k+1} = 6 (y_{k+1} - 2 y_k + y_{k-1}) / h^2,
// M_0 = M_{n_r-1} = 0, by forward elimination and back substitution (cc holds
// the eliminated super-diagonal).  Knot k's pair (y_k, M_k) goes to
// tc[k * stride], so the channels of a table can be interleaved.
__host__ __device__ inline void spline_solve(const double* __restrict__ yc, double2* __restrict__ tc, int64_t stride,
                                             double* __restrict__ cc, int n_r, double six_over_h2)
{
    for (int k = 0; k < n_r; ++k) tc[k * stride] = make_double2(yc[k], 0.0);
    double cprev = 0.0, dprev = 0.0;  // forward elimination over k = 1 .. n_r-2 (dp kept in .y)
    for (int k = 1; k <= n_r - 2; ++k) {
        const double rhs = six_over_h2 * (yc[k + 1] - 2.0 * yc[k] + yc[k - 1]);
        const double den = 4.0 - cprev;
        cprev = 1.0 / den;
        dprev = (rhs - dprev) / den;
        cc[k] = cprev;
        tc[k * stride].y = dprev;
    }
    for (int k = n_r - 3; k >= 1; --k) tc[k * stride].y -= cc[k] * tc[(k + 1) * stride].y;  // M_{n_r-1} = 0
}

__host__ __device__ constexpr int l_of_row(int r)
{
    int l = 0;
    while ((l + 1) * (l + 1) <= r) ++l;
    return l;
}

// All projector values of one point p (coordinates already loaded): d = p - c,
// R_l(|d|) from the table `tab` with `ch` channels, harmonics of d; the value of
// row f goes to out[f * stride].
template <int LMAX, typename TIO>
__device__ __forceinline__ void proj_point(double px, double py, double pz, const double c[3],
                                           const knot_t<TIO>* __restrict__ tab, int ch, const SplineGrid& g,
                                           TIO* __restrict__ out, int64_t stride)
{
    const double dx = px - c[0], dy = py - c[1], dz = pz - c[2];
    double xb, yb, zb, keep;
    normalize(dx, dy, dz, xb, yb, zb, keep);
    const double r = sqrt(__builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz)));
    TIO R[LMAX + 1];
    spline_eval<LMAX + 1, TIO>(tab, ch, g, r, R);
    eval_unit<LMAX, TIO>(TIO(xb), TIO(yb), TIO(zb), TIO(keep),
                         [&](int f, TIO v) { out[int64_t(f) * stride] = R[l_of_row(f)] * v; });
}

// Stores the PPL values of vector o (adjacent points) to dst[0 .. PPL-1] with the
// widest stores the alignment allows: H leading elements one by one up to a
// 16-byte boundary, 16-byte vectors, then the rest one by one (H is a
// compile-time case of the run's alignment).
template <typename TIO, int PPL, int H, typename V>
__device__ __forceinline__ void store_run_from(TIO* __restrict__ dst, V o)
{
    constexpr int UNIT = 16 / int(sizeof(TIO));
    constexpr int NVEC = H < PPL ? (PPL - H) / UNIT : 0;
    static_for<0, (H < PPL ? H : PPL)>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        dst[q] = lane<V, PPL>(o, q);
    });
    static_for<0, NVEC>([&](auto kc) {
        constexpr int i0 = H + decltype(kc)::value * UNIT;
        typename vec_of<TIO, UNIT>::type w;
        static_for<0, UNIT>([&](auto uc) {
            constexpr int u = decltype(uc)::value;
            w[u] = lane<V, PPL>(o, i0 + u);
        });
        *reinterpret_cast<typename vec_of<TIO, UNIT>::type*>(dst + i0) = w;
    });
    static_for<(H < PPL ? H : PPL) + NVEC * UNIT, PPL>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        dst[q] = lane<V, PPL>(o, q);
    });
}

// The first nvalid of the PPL values of o to dst (element-aligned).
template <typename TIO, int PPL, typename V>
__device__ __forceinline__ void store_run(TIO* __restrict__ dst, V o, int nvalid)
{
    constexpr int UNIT = 16 / int(sizeof(TIO));
    if (nvalid < PPL || PPL < UNIT) {
#pragma unroll
        for (int q = 0; q < PPL; ++q)
            if (q < nvalid) dst[q] = lane<V, PPL>(o, q);
        return;
    }
    const int a = int((reinterpret_cast<uintptr_t>(dst) / sizeof(TIO)) & (UNIT - 1));
    const int head = (UNIT - a) & (UNIT - 1);
    static_for<0, UNIT>([&](auto hc) {
        if (head == decltype(hc)::value) store_run_from<TIO, PPL, decltype(hc)::value>(dst, o);
    });
}

// The same for PPL adjacent points of one table and centre, evaluated together
// (the polynomials on PPL-wide vectors, which keeps more independent work in each
// lane): point q's coordinates are (px[q], py[q], pz[q]) and row f of point q goes
// to out[f * stride + q], for the first nvalid points only (the others are computed
// and dropped, so a tail lane runs the same code).  Each row's run of PPL values is
// written with 16-byte stores where its alignment allows (store_run).
template <int LMAX, typename TIO, int PPL>
__device__ __forceinline__ void proj_points(const double (&px)[PPL], const double (&py)[PPL], const double (&pz)[PPL],
                                            const double c[3], const knot_t<TIO>* __restrict__ tab, int ch,
                                            const SplineGrid& g, TIO* __restrict__ out, int64_t stride,
                                            int nvalid = PPL)
{
    using V = typename vec_of<TIO, PPL>::type;
    V x, y, z, k;
    TIO R[PPL][LMAX + 1];
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        const double dx = px[q] - c[0], dy = py[q] - c[1], dz = pz[q] - c[2];
        double xb, yb, zb, keep;
        normalize(dx, dy, dz, xb, yb, zb, keep);
        spline_eval<LMAX + 1, TIO>(tab, ch, g, sqrt(__builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz))), R[q]);
        lane<V, PPL>(x, q) = TIO(xb);
        lane<V, PPL>(y, q) = TIO(yb);
        lane<V, PPL>(z, q) = TIO(zb);
        lane<V, PPL>(k, q) = TIO(keep);
    }
    eval_unit<LMAX, V>(x, y, z, k, [&](int f, V v) {
        const int l = l_of_row(f);
        V r;
#pragma unroll
        for (int q = 0; q < PPL; ++q) lane<V, PPL>(r, q) = R[q][l];
        store_run<TIO, PPL>(out + int64_t(f) * stride, r * v, nvalid);
    });
}

// Lane width of the projector and serving launches.  Several adjacent points per
// lane (row stores of 16 bytes or more) raise the throughput of a launch that
// fills the GPU many times over, but lengthen each workgroup, which is what a
// launch too small to fill the GPU waits for; launches below kProjVecPoints points
// keep one point per lane.  The widths, and the LDS reservation below, were chosen
// per (dtype, lmax) on 64 x 150k-point builds from tables of lmax + 1 channels:
// FP64 four points at lmax 1, two elsewhere (lmax 0: 45% of 8 TB/s against 42%
// with four and the reservation; lmax 3: 56% against 53-54%; lmax 1: 46% against
// 44% with two; lmax 2, where proj_vec_kernel runs: 51.4-51.6% with two against
// 47.3-47.7% with four in proj_kernel, while serving keeps four there, kServePpl;
// lmax >= 4: two, +35% at lmax 6 over one, four 7-10% slower); FP32 four (+10-21% at
// lmax 3-9 over one; two or eight no faster).
template <typename TIO, int LMAX> constexpr int kProjPpl = sizeof(TIO) == 4 ? 4 : (LMAX == 1 ? 4 : 2);
constexpr int64_t kProjVecPoints = int64_t(1) << 20;

// LDS reserved (not used) by the launches with several points per lane: at most 2
// resident workgroups per CU, which keeps each row's concurrent writes in a
// smaller window (as for the forward kernel).  Measured on the same builds: +1-13%
// at FP64 lmax 1-9 and FP32 lmax >= 2; FP64 lmax 0 and FP32 lmax 0-1 run faster
// without it (the FP64 lmax 0 launch with two points per lane: 45% against 34%).
// At lmax 9, and FP64 lmax 8, more than half of the LDS: one resident workgroup per
// CU.  Measured on 64 x 150k-point builds, two runs each: FP64 lmax 9 64.1-64.3% ->
// 65.4%, FP32 60.3-60.6% -> 61.2-61.3% of 8 TB/s, FP64 lmax 8 63.5-63.7% ->
// 64.0-64.2%; FP64 lmax 7, FP32 lmax 7-8 and every lmax up to 6 slower (FP32 lmax 7
// 60.5 -> 56.9%, lmax 6 62 -> 58%); serving (its vector-lane groups), two passes
// each: closed loop 111.7-112.2k -> 113.4-114.3k req/s, Poisson p50 and p99 equal or
// lower.
template <typename TIO, int LMAX>
constexpr size_t kProjCapLds = (LMAX == 9 || (sizeof(TIO) == 8 && LMAX == 8))
                                   ? 84 * 1024
                                   : ((sizeof(TIO) == 4 ? LMAX <= 1 : LMAX == 0) ? 0 : 54 * 1024);

// Whether builds with several points per lane run proj_vec_kernel (a window of 64
// atoms held in lanes, every knot load of a lane issued before the first spline)
// instead of proj_kernel (a wave-wide search for the atom, then each point's knots
// loaded and used in turn): kProjVecKernel for builds over at most 64 atoms (the
// window is all of them), kProjVecWindow for more (the window found by a search).
// Measured on builds of 9.6M points, two runs each, fractions of 8 TB/s: over 64
// atoms (150k points each) FP32 lmax 0 / 1 / 2 / 3 / 4 47 / 44-50 / 44 / 53 / 58% ->
// 53 / 52-56 / 45 / 56-57 / 60%, FP64 lmax 2 47-48 (four points per lane) -> 51-52%
// (two), FP64 lmax 3 57 -> 58-59%, FP32 lmax 5-9 within +-0.5%, FP64 lmax 0-1 and
// 4-9 0-2% slower; over 256 / 1024 atoms FP32 lmax 0 44 /
// 36 -> 50 / 39%, lmax 1 39 / 29 -> 41 / 31%, lmax 2 38 / 31 -> 41 / 32%, FP32 lmax
// 3-4 and FP64 lmax 3 0-4% slower.
template <typename TIO, int LMAX>
constexpr bool kProjVecKernel = sizeof(TIO) == 4 ? LMAX <= 4 : (LMAX == 2 || LMAX == 3);
template <typename TIO, int LMAX>
constexpr bool kProjVecWindow = sizeof(TIO) == 4 && LMAX <= 2;

// Lane width of a launch of n points.
template <typename TIO, int LMAX> constexpr int proj_ppl(int64_t n) { return n >= kProjVecPoints ? kProjPpl<TIO, LMAX> : 1; }

// Wave-wide search over n sorted keys: the last k in [0, n) with keys[k] <= x,
// or -1 if there is none.  Every lane must be active and pass the same x; each
// round the 64 lanes probe 64 evenly spaced keys and a ballot keeps the bracket,
// so n keys take ceil(log64 n) dependent loads.  Keys that are not sorted still
// give some k in [0, n) (callers check what they use).
__device__ __forceinline__ int wave_search(const int64_t* __restrict__ keys, int n, int64_t x)
{
    const int lane = threadIdx.x & 63;
    int lo = 0, hi = n;  // the answer lies in [lo, hi)
    while (hi - lo > 1) {
        const int step = (hi - lo + 63) / 64;
        const int k = lo + lane * step;
        const bool pred = k < hi && keys[k] <= x;
        const int c = __popcll(__ballot(pred));  // lanes 0 .. c-1 probe keys <= x
        if (c == 0) return -1;
        lo += (c - 1) * step;
        hi = min(lo + step, hi);
    }
    return keys[lo] <= x ? lo : -1;
}

// The value v holds in lane k of the wave; k must be the same in every lane (one
// scalar read per 32 bits, no memory access).
template <typename T>
__device__ __forceinline__ T lane_value(T v, int k)
{
    static_assert(sizeof(T) % 4 == 0, "32-bit words");
    int w[sizeof(T) / 4];
    __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
    for (int q = 0; q < int(sizeof(T) / 4); ++q) w[q] = __builtin_amdgcn_readlane(w[q], k);
    T r;
    __builtin_memcpy(&r, w, sizeof(T));
    return r;
}

// The same for one lane (binary search): the last k in [0, n) with keys[k] <= x, or 0.
__device__ __forceinline__ int lane_search(const int64_t* __restrict__ keys, int n, int64_t x)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (keys[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

}  // namespace shk
