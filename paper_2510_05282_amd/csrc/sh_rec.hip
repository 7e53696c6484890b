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
//     a_lm = sqrt((4l^2 - 1)/(l^2 - m^2)),  b_lm = sqrt(((l-1)^2 - m^2)/(4(l-1)^2 - 1)).
// Same normalisation, origin guard and [F][ld] layout as the explicit kernels;
// one point per lane, FP64, lmax up to SH_LMAX_REC.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sh_core.h"
#include "sh_internal.h"
#include "sh_rec.h"

namespace shk {

constexpr int kRecBlock = 256;
constexpr int64_t kRecChunk = int64_t(1) << 28;

__global__ __launch_bounds__(kRecBlock) void rec_kernel(const double* __restrict__ xyz, double* __restrict__ out,
                                                        uint32_t n, int64_t ld, int lmax)
{
    const uint32_t i = blockIdx.x * kRecBlock + threadIdx.x;
    if (i >= n) return;
    const double* p = xyz + 3 * size_t(i);
    double x, y, z, keep;
    normalize(p[0], p[1], p[2], x, y, z, keep);
    const uint32_t boff = i * uint32_t(sizeof(double));
    auto store = [&](int r, double v) {
        *reinterpret_cast<double*>(reinterpret_cast<char*>(out + int64_t(r) * ld) + boff) = v;
    };
    eval_unit_rec(x, y, z, keep, lmax, store);
}

hipError_t launch_rec(int lmax, int64_t n, const double* xyz, double* out, int64_t ld, hipStream_t s)
{
    for (int64_t c0 = 0; c0 < n; c0 += kRecChunk) {
        const int64_t nc = n - c0 < kRecChunk ? n - c0 : kRecChunk;
        const unsigned grid = unsigned((nc + kRecBlock - 1) / kRecBlock);
        hipLaunchKernelGGL(rec_kernel, dim3(grid), dim3(kRecBlock), 0, s, xyz + 3 * c0, out + c0, uint32_t(nc), ld,
                           lmax);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace shk
