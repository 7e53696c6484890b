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
// 24 B in (xyz) + 8F B (G) + 24 B out; this path is bound by reading G.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sh_core.h"
#include "sh_dual.h"
#include "sh_internal.h"

namespace shk {

constexpr int kGradBlock = 256;
constexpr int64_t kGradChunk = int64_t(1) << 28;

template <int LMAX>
__global__ __launch_bounds__(kGradBlock) void grad_kernel(const double* __restrict__ xyz,
                                                          const double* __restrict__ G,
                                                          double* __restrict__ gxyz, uint32_t n,
                                                          int64_t ldg)
{
    const uint32_t i = blockIdx.x * kGradBlock + threadIdx.x;
    if (i >= n) return;
    const double* p = xyz + 3 * size_t(i);
    double xb, yb, zb, keep, rinv;
    normalize(p[0], p[1], p[2], xb, yb, zb, keep, rinv);
    const uint32_t boff = i * uint32_t(sizeof(double));
    auto g_at = [&](int r) {
        return __builtin_nontemporal_load(
            reinterpret_cast<const double*>(reinterpret_cast<const char*>(G + int64_t(r) * ldg) + boff));
    };
    (void)keep;  // the origin needs no mask here: rinv = 0 there, so the gradient is 0
    double vx, vy, vz;
    grad_unit<LMAX>(xb, yb, zb, g_at, vx, vy, vz);
    const double uv = xb * vx + yb * vy + zb * vz;
    double* o = gxyz + 3 * size_t(i);
    o[0] = rinv * (vx - xb * uv);
    o[1] = rinv * (vy - yb * uv);
    o[2] = rinv * (vz - zb * uv);
}

template <int LMAX>
static hipError_t launch_grad_l(int64_t n, const double* xyz, const double* G, int64_t ldg, double* gxyz,
                                hipStream_t s)
{
    for (int64_t c0 = 0; c0 < n; c0 += kGradChunk) {
        const int64_t nc = n - c0 < kGradChunk ? n - c0 : kGradChunk;
        const unsigned grid = unsigned((nc + kGradBlock - 1) / kGradBlock);
        hipLaunchKernelGGL((grad_kernel<LMAX>), dim3(grid), dim3(kGradBlock), 0, s, xyz + 3 * c0, G + c0,
                           gxyz + 3 * c0, uint32_t(nc), ldg);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_grad(int lmax, int64_t n, const double* xyz, const double* G, int64_t ldg, double* gxyz,
                       hipStream_t s)
{
    switch (lmax) {
    case 0: return launch_grad_l<0>(n, xyz, G, ldg, gxyz, s);
    case 1: return launch_grad_l<1>(n, xyz, G, ldg, gxyz, s);
    case 2: return launch_grad_l<2>(n, xyz, G, ldg, gxyz, s);
    case 3: return launch_grad_l<3>(n, xyz, G, ldg, gxyz, s);
    case 4: return launch_grad_l<4>(n, xyz, G, ldg, gxyz, s);
    case 5: return launch_grad_l<5>(n, xyz, G, ldg, gxyz, s);
    case 6: return launch_grad_l<6>(n, xyz, G, ldg, gxyz, s);
    case 7: return launch_grad_l<7>(n, xyz, G, ldg, gxyz, s);
    case 8: return launch_grad_l<8>(n, xyz, G, ldg, gxyz, s);
    case 9: return launch_grad_l<9>(n, xyz, G, ldg, gxyz, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace shk
