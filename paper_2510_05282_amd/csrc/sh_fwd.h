// sh_fwd.h -- the forward kernel template (all real Y_lm of a batch of points).
//
// Each lane evaluates PPL adjacent points at once (the formula core runs on a
// PPL-wide clang vector), so every (l, m) row gets one PPL * sizeof(T) byte
// store per lane and one contiguous 64 * PPL * sizeof(T) byte run per wave.
// Points are normalised in FP64 whatever the output type.
//
// Work distribution is XCD-aware: the hardware deals consecutive workgroups
// round-robin to the 8 XCDs, so workgroup b is remapped to the logical tile
// start(b % 8) + b / 8, giving each XCD one contiguous range of points.  The
// points that are being written at any moment then stay within a few compact
// windows of every output row, which the HBM write path rewards measurably.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sh_core.h"

namespace shk {

constexpr int kFwdBlock = 256;

template <typename S, int N> struct vec_of { typedef S type __attribute__((ext_vector_type(N))); };
template <typename S> struct vec_of<S, 1> { typedef S type; };

template <typename V, int PPL>
__device__ __forceinline__ auto& lane(V& v, int k)
{
    if constexpr (PPL == 1) return v;
    else return reinterpret_cast<scalar_t<V>*>(&v)[k];
}

// The paper's three input interfaces (Section 2): Cartesian points (normalised
// here), points already on the unit sphere, and the angles (theta, phi).
enum class In { kXyz, kUnit, kAngles };

// Unit vector (in FP64) and origin mask of point i of the input.
template <In MODE, typename TIO>
__device__ __forceinline__ void load_unit(const TIO* __restrict__ a, const TIO* __restrict__ b, uint32_t i,
                                          double& xb, double& yb, double& zb, double& kb)
{
    if constexpr (MODE == In::kXyz) {
        const TIO* p = a + 3 * size_t(i);
        normalize(double(p[0]), double(p[1]), double(p[2]), xb, yb, zb, kb);
    } else if constexpr (MODE == In::kUnit) {
        const TIO* p = a + 3 * size_t(i);
        xb = double(p[0]);
        yb = double(p[1]);
        zb = double(p[2]);
        kb = 1.0;
    } else {
        double st, ct, sp, cp;
        sincos(double(a[i]), &st, &ct);
        sincos(double(b[i]), &sp, &cp);
        xb = st * cp;
        yb = st * sp;
        zb = ct;
        kb = 1.0;
    }
}

// out is [F][ld]; the input is xyz [n][3] (kXyz, kUnit) or theta = xyz[n],
// phi = in1[n] (kAngles); n * sizeof(TIO) < 2^31 so per-row byte offsets
// fit 32 bits (the host splits larger batches).  With PPL > 1 the host
// guarantees n % PPL == 0, ld % PPL == 0 and a PPL * sizeof(TIO)-aligned out
// (a remainder of fewer than PPL points goes to a PPL = 1 launch).
template <int LMAX, typename TIO, int PPL, In MODE = In::kXyz>
__global__ __launch_bounds__(kFwdBlock) void fwd_kernel(const TIO* __restrict__ xyz, TIO* __restrict__ out,
                                                        uint32_t n, int64_t ld, const TIO* __restrict__ in1)
{
    using V = typename vec_of<TIO, PPL>::type;
    const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t t = b * kFwdBlock + threadIdx.x;  // vector index
    const uint32_t i0 = t * PPL;                     // first point of this lane
    if (i0 >= n) return;
    V x, y, z, k;
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        double xb, yb, zb, kb;
        load_unit<MODE, TIO>(xyz, in1, i0 + q, xb, yb, zb, kb);
        lane<V, PPL>(x, q) = TIO(xb);
        lane<V, PPL>(y, q) = TIO(yb);
        lane<V, PPL>(z, q) = TIO(zb);
        lane<V, PPL>(k, q) = TIO(kb);
    }
    const uint32_t boff = i0 * uint32_t(sizeof(TIO));
    eval_unit<LMAX, V>(x, y, z, k, [&](int r, V v) {
        *reinterpret_cast<V*>(reinterpret_cast<char*>(out + int64_t(r) * ld) + boff) = v;
    });
}

// Loads PPL adjacent points (from point i0) as unit vectors in V lanes; the input
// interface is chosen at run time (the same for the whole launch).
template <typename TIO, int PPL, typename V>
__device__ __forceinline__ void load_points(const TIO* __restrict__ in0, const TIO* __restrict__ in1, In mode,
                                            uint32_t i0, V& x, V& y, V& z, V& k)
{
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        double xb, yb, zb, kb;
        if (mode == In::kXyz) load_unit<In::kXyz, TIO>(in0, in1, i0 + q, xb, yb, zb, kb);
        else if (mode == In::kUnit) load_unit<In::kUnit, TIO>(in0, in1, i0 + q, xb, yb, zb, kb);
        else load_unit<In::kAngles, TIO>(in0, in1, i0 + q, xb, yb, zb, kb);
        lane<V, PPL>(x, q) = TIO(xb);
        lane<V, PPL>(y, q) = TIO(yb);
        lane<V, PPL>(z, q) = TIO(zb);
        lane<V, PPL>(k, q) = TIO(kb);
    }
}

// PPL complex values (re, im interleaved, PPL adjacent points) as one vector.
template <typename TIO, int PPL, typename V>
__device__ __forceinline__ typename vec_of<TIO, 2 * PPL>::type interleave(V re, V im)
{
    typename vec_of<TIO, 2 * PPL>::type w;
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        w[2 * q] = lane<V, PPL>(re, q);
        w[2 * q + 1] = lane<V, PPL>(im, q);
    }
    return w;
}

// Complex harmonics from the real ones (Section 3, complex_unit): out[row][i] as
// (re, im) pairs, [F][ld] complex.  Each lane evaluates PPL adjacent points and
// stores their PPL complex values of a row at once: 16 bytes per lane and row for
// FP64 with PPL = 1 and FP32 with PPL = 2.  With PPL > 1 the host guarantees
// n % PPL == 0, ld % PPL == 0 and a 16-byte aligned out.  Inputs as for fwd_kernel:
// in0 = xyz [n][3] (kXyz, kUnit) or theta[n] and in1 = phi[n] (kAngles).
template <int LMAX, typename TIO, int PPL>
__global__ __launch_bounds__(kFwdBlock) void fwd_complex_kernel(const TIO* __restrict__ in0,
                                                                TIO* __restrict__ out, uint32_t n, int64_t ld,
                                                                const TIO* __restrict__ in1, In mode)
{
    using V = typename vec_of<TIO, PPL>::type;
    using W = typename vec_of<TIO, 2 * PPL>::type;
    const uint32_t i0 = (xcd_tile(blockIdx.x, gridDim.x) * kFwdBlock + threadIdx.x) * PPL;
    if (i0 >= n) return;
    V x, y, z, k;
    load_points<TIO, PPL>(in0, in1, mode, i0, x, y, z, k);
    const uint32_t boff = i0 * uint32_t(2 * sizeof(TIO));
    complex_unit<LMAX, V>(x, y, z, k, [&](int l, int m, V re, V im) {
        *reinterpret_cast<W*>(reinterpret_cast<char*>(out + 2 * int64_t(row(l, m)) * ld) + boff) =
            interleave<TIO, PPL>(re, im);
    });
}

// Spinor harmonics (eq. spinorial): spinor_unit's values, stored as they come to
// out[(2 s + c) ld + i] as (re, im) pairs (c = 0 for the upper component), with
// the same lanes as the complex kernel.
template <int LMAX, typename TIO, int PPL>
__global__ __launch_bounds__(kFwdBlock) void fwd_spinor_kernel(const TIO* __restrict__ in0,
                                                               TIO* __restrict__ out, uint32_t n, int64_t ld,
                                                               const TIO* __restrict__ in1, In mode)
{
    using V = typename vec_of<TIO, PPL>::type;
    using W = typename vec_of<TIO, 2 * PPL>::type;
    const uint32_t i0 = (xcd_tile(blockIdx.x, gridDim.x) * kFwdBlock + threadIdx.x) * PPL;
    if (i0 >= n) return;
    V x, y, z, k;
    load_points<TIO, PPL>(in0, in1, mode, i0, x, y, z, k);
    const uint32_t boff = i0 * uint32_t(2 * sizeof(TIO));
    spinor_unit<LMAX, V>(x, y, z, k, [&](int s, int c, V re, V im) {
        *reinterpret_cast<W*>(reinterpret_cast<char*>(out + 2 * int64_t(2 * s + c) * ld) + boff) =
            interleave<TIO, PPL>(re, im);
    });
}

}  // namespace shk
