// sh_eval.hip -- forward kernels: all real Y_lm, l <= lmax, for a batch of points.
//
// One thread per point.  Each thread loads its point, normalises it in FP64
// (hardware rsqrt refined by Newton steps, with the near-origin guard), evaluates
// the factorised formulas and writes every (l, m) value to its own row of the
// [F][ld] output.  The 64 lanes of a wave hold 64 consecutive points, so each
// row store of a wave is one contiguous, line-aligned 512 B (FP64) or 256 B
// (FP32) run.  Output is written exactly once and never read back, so the stores
// are non-temporal.  The path moves 3s + F s bytes per point (s = element size)
// against a few hundred flops: it is bound by HBM stores, not by arithmetic.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sh_core.h"
#include "sh_internal.h"

namespace shk {

// Points per launch: keeps every per-row byte offset of a launch below 2^31 so
// the store address is a scalar row base plus a 32-bit per-lane offset.
constexpr int64_t kChunk = int64_t(1) << 28;
constexpr int kBlock = 256;

template <int LMAX, typename TIO>
__global__ __launch_bounds__(kBlock) void fwd_kernel(const TIO* __restrict__ xyz, TIO* __restrict__ out,
                                                     uint32_t n, int64_t ld)
{
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const TIO* p = xyz + 3 * size_t(i);
    double xb, yb, zb, keep;
    normalize(double(p[0]), double(p[1]), double(p[2]), xb, yb, zb, keep);
    const uint32_t boff = i * uint32_t(sizeof(TIO));
    eval_unit<LMAX, TIO>(TIO(xb), TIO(yb), TIO(zb), TIO(keep), [&](int r, TIO v) {
        TIO* dst = reinterpret_cast<TIO*>(reinterpret_cast<char*>(out + int64_t(r) * ld) + boff);
        __builtin_nontemporal_store(v, dst);
    });
}

template <int LMAX, typename TIO>
static hipError_t launch_fwd_l(int64_t n, const TIO* xyz, TIO* out, int64_t ld, hipStream_t s)
{
    for (int64_t c0 = 0; c0 < n; c0 += kChunk) {
        const int64_t nc = n - c0 < kChunk ? n - c0 : kChunk;
        const unsigned grid = unsigned((nc + kBlock - 1) / kBlock);
        hipLaunchKernelGGL((fwd_kernel<LMAX, TIO>), dim3(grid), dim3(kBlock), 0, s, xyz + 3 * c0, out + c0,
                           uint32_t(nc), ld);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename TIO>
hipError_t launch_fwd(int lmax, int64_t n, const TIO* xyz, TIO* out, int64_t ld, hipStream_t s)
{
    switch (lmax) {
    case 0: return launch_fwd_l<0, TIO>(n, xyz, out, ld, s);
    case 1: return launch_fwd_l<1, TIO>(n, xyz, out, ld, s);
    case 2: return launch_fwd_l<2, TIO>(n, xyz, out, ld, s);
    case 3: return launch_fwd_l<3, TIO>(n, xyz, out, ld, s);
    case 4: return launch_fwd_l<4, TIO>(n, xyz, out, ld, s);
    case 5: return launch_fwd_l<5, TIO>(n, xyz, out, ld, s);
    case 6: return launch_fwd_l<6, TIO>(n, xyz, out, ld, s);
    case 7: return launch_fwd_l<7, TIO>(n, xyz, out, ld, s);
    case 8: return launch_fwd_l<8, TIO>(n, xyz, out, ld, s);
    case 9: return launch_fwd_l<9, TIO>(n, xyz, out, ld, s);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_fwd<double>(int, int64_t, const double*, double*, int64_t, hipStream_t);
template hipError_t launch_fwd<float>(int, int64_t, const float*, float*, int64_t, hipStream_t);

}  // namespace shk
