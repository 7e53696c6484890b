// sh_grad.hip -- backward kernel: vector-Jacobian product of the forward pass.
//
// For an upstream gradient G[F][n] the kernel returns, per point,
//     g = sum_{l,m} G_lm grad_r R_l^m(r) = (1/r) (v - u (u . v)),
//     v = sum_{l,m} G_lm grad_u P_lm(u),   u = r / |r|,
// where P_lm is the factorised polynomial the forward kernel evaluates.  Any
// smooth extension of R_l^m off the unit sphere gives the same tangential part,
// so the projection makes the result exact whatever the extension.  The polynomial
// gradients come from running the same factorised forms on dual numbers
// (grad_unit in sh_dual.h).
// One thread per point; G is read row by row (coalesced across the wave), the
// three gradient components are written per point.  Memory traffic per point:
// 3s B in (xyz) + F s B (G) + 3s B out (s = element size); this path is bound by
// reading G.  The same file holds the fused value + Jacobian kernel.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "sh_core.h"
#include "sh_dual.h"
#include "sh_internal.h"

namespace shk {

constexpr int kGradBlock = 256;
constexpr int64_t kGradChunk = int64_t(1) << 28;
// LDS reserved (not used) per workgroup of the backward kernel: at most 4 resident
// workgroups (16 waves) per CU.  Measured on MI355X: 73% of 8 TB/s against 71.8%
// uncapped (FP32: 74.1% against 71.0%).  Unlike the store-bound kernels, this
// read-bound one runs best in plain workgroup order (XCD-contiguous order: 68.6%)
// and with one point per lane: 2 adjacent points per lane (16-byte loads of G),
// or 4 in FP32, measured 0-5% slower at lmax 3, 6 and 9 with every cap and order.
constexpr size_t kGradCapLds = 40 * 1024;

// TIO is the element type of xyz, G and the result; the normalisation and 1/r
// run in FP64, the polynomials and the contraction in TIO.
template <int LMAX, typename TIO>
__global__ __launch_bounds__(kGradBlock) void grad_kernel(const TIO* __restrict__ xyz, const TIO* __restrict__ G,
                                                          TIO* __restrict__ gxyz, uint32_t n, int64_t ldg)
{
    const uint32_t i = blockIdx.x * kGradBlock + threadIdx.x;
    if (i >= n) return;
    const TIO* p = xyz + 3 * size_t(i);
    double xb, yb, zb, keep, rinv;
    normalize(double(p[0]), double(p[1]), double(p[2]), xb, yb, zb, keep, rinv);
    const uint32_t boff = i * uint32_t(sizeof(TIO));
    auto g_at = [&](int r) {
        return __builtin_nontemporal_load(
            reinterpret_cast<const TIO*>(reinterpret_cast<const char*>(G + int64_t(r) * ldg) + boff));
    };
    (void)keep;  // the origin needs no mask here: rinv = 0 there, so the gradient is 0
    TIO vx, vy, vz;
    const TIO x = TIO(xb), y = TIO(yb), z = TIO(zb);
    grad_unit<LMAX, TIO>(x, y, z, g_at, vx, vy, vz);
    const double uv = xb * double(vx) + yb * double(vy) + zb * double(vz);
    TIO* o = gxyz + 3 * size_t(i);
    o[0] = TIO(rinv * (double(vx) - xb * uv));
    o[1] = TIO(rinv * (double(vy) - yb * uv));
    o[2] = TIO(rinv * (double(vz) - zb * uv));
}

template <int LMAX, typename TIO>
static hipError_t launch_grad_l(int64_t n, const TIO* xyz, const TIO* G, int64_t ldg, TIO* gxyz, hipStream_t s)
{
    for (int64_t c0 = 0; c0 < n; c0 += kGradChunk) {
        const int64_t nc = n - c0 < kGradChunk ? n - c0 : kGradChunk;
        const unsigned grid = unsigned((nc + kGradBlock - 1) / kGradBlock);
        hipLaunchKernelGGL((grad_kernel<LMAX, TIO>), dim3(grid), dim3(kGradBlock), kGradCapLds, s, xyz + 3 * c0,
                           G + c0, gxyz + 3 * c0, uint32_t(nc), ldg);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename TIO>
hipError_t launch_grad(int lmax, int64_t n, const TIO* xyz, const TIO* G, int64_t ldg, TIO* gxyz, hipStream_t s)
{
    switch (lmax) {
    case 0: return launch_grad_l<0, TIO>(n, xyz, G, ldg, gxyz, s);
    case 1: return launch_grad_l<1, TIO>(n, xyz, G, ldg, gxyz, s);
    case 2: return launch_grad_l<2, TIO>(n, xyz, G, ldg, gxyz, s);
    case 3: return launch_grad_l<3, TIO>(n, xyz, G, ldg, gxyz, s);
    case 4: return launch_grad_l<4, TIO>(n, xyz, G, ldg, gxyz, s);
    case 5: return launch_grad_l<5, TIO>(n, xyz, G, ldg, gxyz, s);
    case 6: return launch_grad_l<6, TIO>(n, xyz, G, ldg, gxyz, s);
    case 7: return launch_grad_l<7, TIO>(n, xyz, G, ldg, gxyz, s);
    case 8: return launch_grad_l<8, TIO>(n, xyz, G, ldg, gxyz, s);
    case 9: return launch_grad_l<9, TIO>(n, xyz, G, ldg, gxyz, s);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_grad<double>(int, int64_t, const double*, const double*, int64_t, double*,
                                        hipStream_t);
template hipError_t launch_grad<float>(int, int64_t, const float*, const float*, int64_t, float*, hipStream_t);

// ---------------------------------------------------------------- fused value + Jacobian

// Values out[F][ld] and the Jacobian jac[3][F][ld] (d R_f / d x_k at
// jac[(k F + f) ld + i]) in one pass: the dual-number core gives P and grad_u P,
// which is projected with (1/r)(I - u u^T).  The launch follows the forward
// kernel's (4F + 3 doubles per point, all but 3 of them row stores): PPL = 2
// adjacent points per lane with 16-byte row stores, workgroups in XCD-contiguous
// order, at most 2 resident workgroups per CU; PPL = 1 for odd ld or a
// remainder point.
constexpr size_t kJacCapLds = 54 * 1024;

template <int LMAX, int PPL>
__global__ __launch_bounds__(kGradBlock) void jac_kernel(const double* __restrict__ xyz, double* __restrict__ out,
                                                         double* __restrict__ jac, uint32_t n, int64_t ld)
{
    constexpr int F = nfun(LMAX);
    using V = std::conditional_t<PPL == 1, double, double2_t>;
    const uint32_t i0 = (xcd_tile(blockIdx.x, gridDim.x) * kGradBlock + threadIdx.x) * PPL;
    if (i0 >= n) return;
    V x, y, z, k, ri;
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        const double* p = xyz + 3 * size_t(i0 + q);
        double xb, yb, zb, kb, rb;
        normalize(p[0], p[1], p[2], xb, yb, zb, kb, rb);
        if constexpr (PPL == 1) {
            x = xb, y = yb, z = zb, k = kb, ri = rb;
        } else {
            x[q] = xb, y[q] = yb, z[q] = zb, k[q] = kb, ri[q] = rb;
        }
    }
    const uint32_t boff = i0 * uint32_t(sizeof(double));
    auto at = [&](double* base, int64_t r) {
        return reinterpret_cast<V*>(reinterpret_cast<char*>(base + r * ld) + boff);
    };
    eval_unit_jac<LMAX, V>(x, y, z, k, [&](int f, V v, V gx, V gy, V gz) {
        const V ug = x * gx + y * gy + z * gz;
        *at(out, f) = v;
        *at(jac, f) = ri * (gx - x * ug);
        *at(jac, F + f) = ri * (gy - y * ug);
        *at(jac, 2 * F + f) = ri * (gz - z * ug);
    });
}

template <int LMAX, int PPL>
static hipError_t launch_jac_one(int64_t n, const double* xyz, double* out, double* jac, int64_t ld, hipStream_t s)
{
    const unsigned grid = unsigned((n / PPL + kGradBlock - 1) / kGradBlock);
    hipLaunchKernelGGL((jac_kernel<LMAX, PPL>), dim3(grid), dim3(kGradBlock), PPL > 1 ? kJacCapLds : 0, s, xyz, out,
                       jac, uint32_t(n), ld);
    return hipGetLastError();
}

template <int LMAX>
static hipError_t launch_jac_l(int64_t n, const double* xyz, double* out, double* jac, int64_t ld, hipStream_t s)
{
    // several points per lane from 2^18 points on (a smaller launch leaves CUs idle
    // and lasts one workgroup's chain of work, which the wider lanes lengthen: lmax
    // 6, 4k / 16k / 64k / 100k points, 7.4 / 9.2 / 16.4 / 24.4 us against 8.6 /
    // 10.6 / 16.8 / 24.9 with two points per lane)
    const bool vec_ok = n >= (int64_t(1) << 18) && ld % 2 == 0 && reinterpret_cast<uintptr_t>(out) % 16 == 0 &&
                        reinterpret_cast<uintptr_t>(jac) % 16 == 0;
    for (int64_t c0 = 0; c0 < n; c0 += kGradChunk) {
        const int64_t nc = n - c0 < kGradChunk ? n - c0 : kGradChunk;
        const int64_t nmain = vec_ok ? nc - nc % 2 : 0;
        hipError_t e = hipSuccess;
        if (nmain) e = launch_jac_one<LMAX, 2>(nmain, xyz + 3 * c0, out + c0, jac + c0, ld, s);
        if (e == hipSuccess && nmain < nc)
            e = launch_jac_one<LMAX, 1>(nc - nmain, xyz + 3 * (c0 + nmain), out + c0 + nmain, jac + c0 + nmain, ld,
                                        s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_jac(int lmax, int64_t n, const double* xyz, double* out, double* jac, int64_t ld, hipStream_t s)
{
    switch (lmax) {
    case 0: return launch_jac_l<0>(n, xyz, out, jac, ld, s);
    case 1: return launch_jac_l<1>(n, xyz, out, jac, ld, s);
    case 2: return launch_jac_l<2>(n, xyz, out, jac, ld, s);
    case 3: return launch_jac_l<3>(n, xyz, out, jac, ld, s);
    case 4: return launch_jac_l<4>(n, xyz, out, jac, ld, s);
    case 5: return launch_jac_l<5>(n, xyz, out, jac, ld, s);
    case 6: return launch_jac_l<6>(n, xyz, out, jac, ld, s);
    case 7: return launch_jac_l<7>(n, xyz, out, jac, ld, s);
    case 8: return launch_jac_l<8>(n, xyz, out, jac, ld, s);
    case 9: return launch_jac_l<9>(n, xyz, out, jac, ld, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace shk
