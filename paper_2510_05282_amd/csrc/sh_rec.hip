// sh_rec.hip -- real harmonics beyond l = 9 by recurrence.
//
// The explicit formulas stop at l = 9; the paper's conclusion points to
// recurrence relations for higher orders.  On the unit vector u = (x, y, z),
//     R_l^0 = Yb_l^0(z),  R_l^{+m} = Yb_l^m(z) C_m(x, y),  R_l^{-m} = Yb_l^m(z) S_m(x, y),
// with C_m + i S_m = (x + i y)^m (built by repeated complex multiplication) and
// Yb_l^m(z) = sqrt(2)^[m>0] N_lm d^m P_l/dz^m, the normalised associated Legendre
// functions with the sin^m factor moved into C_m, S_m.  They follow the stable
// normalised recurrences
//     Yb_m^m     = d_m,  d_0 = 1/sqrt(4 pi),  d_m = d_{m-1} sqrt((2m+1)/(2m)) (x sqrt(2) at m = 1),
//     Yb_{m+1}^m = sqrt(2m+3) z Yb_m^m,
//     Yb_l^m     = a_lm (z Yb_{l-1}^m - b_lm Yb_{l-2}^m),
//     a_lm = sqrt((4l^2 - 1)/(l^2 - m^2)),  b_lm = sqrt(((l-1)^2 - m^2)/(4(l-1)^2 - 1)),
// whose coefficients are generated once (gen_rec_constants.py, 50-digit mpmath),
// so the kernel does no square roots or divisions.  Same normalisation, origin
// guard and [F][ld] layout as the explicit kernels, FP64 or FP32 (normalisation
// in FP64 either way), lmax up to SH_LMAX_REC.  The launch follows the explicit
// kernel's: 16-byte row stores per lane (two FP64 or four FP32 adjacent points),
// XCD-contiguous workgroups, at most 2 resident workgroups per CU; one point per
// lane for an unaligned row stride or the remainder points.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/shmi.h"
#include "sh_core.h"
#include "sh_fwd.h"
#include "sh_internal.h"
#include "sh_rec.h"

namespace shk {

static_assert(shc::kRecLmax == SH_LMAX_REC, "recurrence tables and the public limit disagree");

constexpr int kRecBlock = 256;
constexpr int64_t kRecChunk = int64_t(1) << 28;
// Calls of at least this many points take several points per lane; smaller
// launches leave CUs idle and last one workgroup's chain of work, which the wider
// lanes lengthen, so they run one point per lane.  Kernel trace, 4k / 16k / 64k /
// 100k points, one point per lane against the wide lanes: real harmonics at lmax
// 16 FP64 25.1 / 27.3 / 33.1 / 48.5 us against 30.3 / 32.3 / 37.2 / 44.5, FP32
// 24.6 / 29.2 / 35.3 / 35.7 against 36.0 / 40.2 / 45.4 / 45.6; the backward pass at
// lmax 14 FP64 38.2 / 74.1 / 76.9 / 83.9 against 44.2 / 83.2 / 85.9 / 88.0; equal
// at 2^18 points.  The FP64 forward switches between 64k and 100k points.
// (real harmonics; the complex and spinor forms and the backward pass switch at 2^18)
template <typename TIO> constexpr int64_t kRecVecPoints = sizeof(TIO) == 8 ? int64_t(3) << 15 : int64_t(1) << 18;
constexpr int64_t kRecVecPointsCplxGrad = int64_t(1) << 18;
constexpr size_t kRecCapLds = 54 * 1024;

// TIO = double: 2 points per lane (PPL = 2); float: 4 (PPL = 4); both store 16
// bytes per lane and row.  Points are normalised in FP64 either way.
template <typename TIO, int PPL>
__global__ __launch_bounds__(kRecBlock) void rec_kernel(const TIO* __restrict__ xyz, TIO* __restrict__ out,
                                                        uint32_t n, int64_t ld, int lmax)
{
    using V = typename vec_of<TIO, PPL>::type;
    const uint32_t i0 = (xcd_tile(blockIdx.x, gridDim.x) * kRecBlock + threadIdx.x) * PPL;
    if (i0 >= n) return;
    V x, y, z, k;
    load_points<TIO, PPL>(xyz, nullptr, In::kXyz, i0, x, y, z, k);
    const uint32_t boff = i0 * uint32_t(sizeof(TIO));
    eval_unit_rec<V>(x, y, z, k, lmax, [&](int l, int m, V v) {
        *reinterpret_cast<V*>(reinterpret_cast<char*>(out + int64_t(row(l, m)) * ld) + boff) = v;
    });
}

template <typename TIO, int PPL>
static hipError_t launch_rec_one(int lmax, int64_t n, const TIO* xyz, TIO* out, int64_t ld, hipStream_t s)
{
    const unsigned grid = unsigned((n / PPL + kRecBlock - 1) / kRecBlock);
    hipLaunchKernelGGL((rec_kernel<TIO, PPL>), dim3(grid), dim3(kRecBlock), PPL > 1 ? kRecCapLds : 0, s, xyz, out,
                       uint32_t(n), ld, lmax);
    return hipGetLastError();
}

template <typename TIO>
hipError_t launch_rec(int lmax, int64_t n, const TIO* xyz, TIO* out, int64_t ld, hipStream_t s)
{
    constexpr int kVec = 16 / sizeof(TIO);
    const bool vec_ok = n >= kRecVecPoints<TIO> && ld % kVec == 0 && reinterpret_cast<uintptr_t>(out) % 16 == 0;
    for (int64_t c0 = 0; c0 < n; c0 += kRecChunk) {
        const int64_t nc = n - c0 < kRecChunk ? n - c0 : kRecChunk;
        const int64_t nmain = vec_ok ? nc - nc % kVec : 0;
        hipError_t e = hipSuccess;
        if (nmain) e = launch_rec_one<TIO, kVec>(lmax, nmain, xyz + 3 * c0, out + c0, ld, s);
        if (e == hipSuccess && nmain < nc)
            e = launch_rec_one<TIO, 1>(lmax, nc - nmain, xyz + 3 * (c0 + nmain), out + c0 + nmain, ld, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template hipError_t launch_rec<double>(int, int64_t, const double*, double*, int64_t, hipStream_t);
template hipError_t launch_rec<float>(int, int64_t, const float*, float*, int64_t, hipStream_t);

// Backward pass by recurrence: the vector-Jacobian product of sh_eval_rec,
//     g = (1/r) (v - u (u . v)),   v = sum_rows G[row] grad_u P_row(u),
// as the explicit backward kernel, with v from grad_unit_rec (the recurrence
// differentiated in z, the xy factors by their closed-form partials).  PPL
// adjacent points per lane (G read as one PPL-wide vector per row: 16 bytes in
// FP64, 8 in FP32, where four points per lane need 140 VGPRs and ran slower, and one
// point per lane reached 53% of 8 TB/s at lmax 16 against 68% with two),
// workgroups in XCD-contiguous order, no cap on resident workgroups (capping to
// 2 or 4 per CU loses 25-50% here: the kernel needs many loads in flight); the
// normalisation and 1/r in FP64.
template <typename TIO, int PPL>
__global__ __launch_bounds__(kRecBlock) void grad_rec_kernel(const TIO* __restrict__ xyz, const TIO* __restrict__ G,
                                                             TIO* __restrict__ gxyz, uint32_t n, int64_t ldg,
                                                             int lmax)
{
    using V = typename vec_of<TIO, PPL>::type;
    const uint32_t i0 = (xcd_tile(blockIdx.x, gridDim.x) * kRecBlock + threadIdx.x) * PPL;
    if (i0 >= n) return;
    double xb[PPL], yb[PPL], zb[PPL], rinv[PPL];
    V x, y, z;
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        const TIO* p = xyz + 3 * size_t(i0 + q);
        double keep;  // not needed: rinv = 0 at the origin, so the gradient is 0 there
        normalize(double(p[0]), double(p[1]), double(p[2]), xb[q], yb[q], zb[q], keep, rinv[q]);
        lane<V, PPL>(x, q) = TIO(xb[q]);
        lane<V, PPL>(y, q) = TIO(yb[q]);
        lane<V, PPL>(z, q) = TIO(zb[q]);
    }
    const uint32_t boff = i0 * uint32_t(sizeof(TIO));
    V vx, vy, vz;
    grad_unit_rec<V>(x, y, z, lmax,
                     [&](int r) {
                         return __builtin_nontemporal_load(reinterpret_cast<const V*>(
                             reinterpret_cast<const char*>(G + int64_t(r) * ldg) + boff));
                     },
                     vx, vy, vz);
    TIO* o = gxyz + 3 * size_t(i0);
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        const double gx = double(lane<V, PPL>(vx, q)), gy = double(lane<V, PPL>(vy, q)),
                     gz = double(lane<V, PPL>(vz, q));
        const double uv = xb[q] * gx + yb[q] * gy + zb[q] * gz;
        o[3 * q + 0] = TIO(rinv[q] * (gx - xb[q] * uv));
        o[3 * q + 1] = TIO(rinv[q] * (gy - yb[q] * uv));
        o[3 * q + 2] = TIO(rinv[q] * (gz - zb[q] * uv));
    }
}

// n must be a multiple of PPL (the caller sends the remainder to PPL = 1).
template <typename TIO, int PPL>
static hipError_t launch_grad_rec_one(int lmax, int64_t n, const TIO* xyz, const TIO* G, int64_t ldg, TIO* gxyz,
                                      hipStream_t s)
{
    const unsigned grid = unsigned((n / PPL + kRecBlock - 1) / kRecBlock);
    hipLaunchKernelGGL((grad_rec_kernel<TIO, PPL>), dim3(grid), dim3(kRecBlock), 0, s, xyz, G, gxyz, uint32_t(n),
                       ldg, lmax);
    return hipGetLastError();
}

template <typename TIO>
hipError_t launch_grad_rec(int lmax, int64_t n, const TIO* xyz, const TIO* G, int64_t ldg, TIO* gxyz, hipStream_t s)
{
    constexpr int kVec = 2;
    const bool vec_ok =
        n >= kRecVecPointsCplxGrad && ldg % kVec == 0 && reinterpret_cast<uintptr_t>(G) % (kVec * sizeof(TIO)) == 0;
    for (int64_t c0 = 0; c0 < n; c0 += kRecChunk) {  // kRecChunk is a multiple of kVec
        const int64_t nc = n - c0 < kRecChunk ? n - c0 : kRecChunk;
        const int64_t nmain = vec_ok ? nc - nc % kVec : 0;
        hipError_t e = hipSuccess;
        if (nmain) e = launch_grad_rec_one<TIO, kVec>(lmax, nmain, xyz + 3 * c0, G + c0, ldg, gxyz + 3 * c0, s);
        if (e == hipSuccess && nc > nmain) {
            const int64_t c1 = c0 + nmain;
            e = launch_grad_rec_one<TIO, 1>(lmax, nc - nmain, xyz + 3 * c1, G + c1, ldg, gxyz + 3 * c1, s);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template hipError_t launch_grad_rec<double>(int, int64_t, const double*, const double*, int64_t, double*,
                                            hipStream_t);
template hipError_t launch_grad_rec<float>(int, int64_t, const float*, const float*, int64_t, float*, hipStream_t);

// Complex (SPINOR = false) or spinor harmonics by recurrence, any input interface:
// the lanes and layout of fwd_complex_kernel / fwd_spinor_kernel, lmax at run time.
template <typename TIO, int PPL, bool SPINOR>
__global__ __launch_bounds__(kRecBlock) void rec_cplx_kernel(const TIO* __restrict__ in0, TIO* __restrict__ out,
                                                             uint32_t n, int64_t ld, const TIO* __restrict__ in1,
                                                             In mode, int lmax)
{
    using V = typename vec_of<TIO, PPL>::type;
    using W = typename vec_of<TIO, 2 * PPL>::type;
    const uint32_t i0 = (xcd_tile(blockIdx.x, gridDim.x) * kRecBlock + threadIdx.x) * PPL;
    if (i0 >= n) return;
    V x, y, z, k;
    load_points<TIO, PPL>(in0, in1, mode, i0, x, y, z, k);
    const uint32_t boff = i0 * uint32_t(2 * sizeof(TIO));
    auto put = [&](int64_t r, V re, V im) {
        *reinterpret_cast<W*>(reinterpret_cast<char*>(out + 2 * r * ld) + boff) = interleave<TIO, PPL>(re, im);
    };
    if constexpr (SPINOR)
        spinor_unit_rec<V>(x, y, z, k, lmax, [&](int s, int c, V re, V im) { put(2 * s + c, re, im); });
    else
        complex_unit_rec<V>(x, y, z, k, lmax, [&](int l, int m, V re, V im) { put(row(l, m), re, im); });
}

template <typename TIO, int PPL, bool SPINOR>
static hipError_t launch_rec_cplx_one(int lmax, int64_t n, In mode, const TIO* a, const TIO* b, TIO* out,
                                      int64_t ld, hipStream_t s)
{
    const unsigned grid = unsigned((n / PPL + kRecBlock - 1) / kRecBlock);
    const size_t lds = PPL * sizeof(TIO) * 2 == 16 ? kRecCapLds : 0;
    hipLaunchKernelGGL((rec_cplx_kernel<TIO, PPL, SPINOR>), dim3(grid), dim3(kRecBlock), lds, s, a, out,
                       uint32_t(n), ld, b, mode, lmax);
    return hipGetLastError();
}

template <typename TIO, bool SPINOR>
static hipError_t launch_rec_cplx(int lmax, int64_t n, int input, const TIO* in0, const TIO* in1, TIO* out,
                                  int64_t ld, hipStream_t s)
{
    constexpr int kVec = sizeof(TIO) == 4 ? 2 : 1;
    const In mode = In(input);
    const int64_t stride = mode == In::kAngles ? 1 : 3;
    const bool vec_ok = n >= kRecVecPointsCplxGrad && ld % kVec == 0 && reinterpret_cast<uintptr_t>(out) % 16 == 0;
    for (int64_t c0 = 0; c0 < n; c0 += kRecChunk) {
        const int64_t nc = n - c0 < kRecChunk ? n - c0 : kRecChunk;
        const int64_t nmain = vec_ok ? nc - nc % kVec : 0;
        auto a = [&](int64_t c) { return in0 + stride * c; };
        auto b = [&](int64_t c) { return mode == In::kAngles ? in1 + c : in1; };
        hipError_t e = hipSuccess;
        if (nmain) e = launch_rec_cplx_one<TIO, kVec, SPINOR>(lmax, nmain, mode, a(c0), b(c0), out + 2 * c0, ld, s);
        if (e == hipSuccess && nmain < nc)
            e = launch_rec_cplx_one<TIO, 1, SPINOR>(lmax, nc - nmain, mode, a(c0 + nmain), b(c0 + nmain),
                                                    out + 2 * (c0 + nmain), ld, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename TIO>
hipError_t launch_rec_complex(int lmax, int64_t n, int input, const TIO* in0, const TIO* in1, TIO* out, int64_t ld,
                              hipStream_t s)
{
    return launch_rec_cplx<TIO, false>(lmax, n, input, in0, in1, out, ld, s);
}

template <typename TIO>
hipError_t launch_rec_spinor(int lmax, int64_t n, int input, const TIO* in0, const TIO* in1, TIO* out, int64_t ld,
                             hipStream_t s)
{
    return launch_rec_cplx<TIO, true>(lmax, n, input, in0, in1, out, ld, s);
}

template hipError_t launch_rec_complex<double>(int, int64_t, int, const double*, const double*, double*, int64_t,
                                               hipStream_t);
template hipError_t launch_rec_complex<float>(int, int64_t, int, const float*, const float*, float*, int64_t,
                                              hipStream_t);
template hipError_t launch_rec_spinor<double>(int, int64_t, int, const double*, const double*, double*, int64_t,
                                              hipStream_t);
template hipError_t launch_rec_spinor<float>(int, int64_t, int, const float*, const float*, float*, int64_t,
                                             hipStream_t);

}  // namespace shk
