// sh_proj.hip -- radial spline tables and the fused projector build.
//
// A projector value for atom a at grid point p is R_l(|d|) * R_l^m(d / |d|) with
// d = p - c_a (the role the harmonics play in the paper's introduction).  R_l is
// a natural cubic spline through values tabulated on a uniform radial grid; it is
// 0 beyond the table's last knot.  One pass per point computes d, r, every R_l(r)
// for l <= lmax, the harmonics, and stores their products; nothing is
// materialised in between.
//
// Device table layout of a radial handle: [n_tables][channels][n_r] of double2
// (y_i, M_i), M the spline's second derivatives, so one interval lookup reads 32
// contiguous bytes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sh_core.h"
#include "sh_internal.h"
#include "sh_proj.h"

namespace shk {

// ---------------------------------------------------------------- spline set-up

// Natural cubic spline on a uniform grid, one thread per channel.  With knot
// spacing h, the second derivatives solve, for k = 1 .. n_r-2,
//     M_{k-1} + 4 M_k + M_{k+1} = 6 (y_{k+1} - 2 y_k + y_{k-1}) / h^2,
// M_0 = M_{n_r-1} = 0; the tridiagonal system is solved by forward elimination
// and back substitution (cp holds the eliminated super-diagonal, one row per
// channel).
__global__ void spline_setup_kernel(const double* __restrict__ y, double2* __restrict__ table,
                                    double* __restrict__ cp, int n_ch, int n_r, double six_over_h2)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_ch) return;
    const double* yc = y + int64_t(c) * n_r;
    double2* tc = table + int64_t(c) * n_r;
    double* cc = cp + int64_t(c) * n_r;
    for (int k = 0; k < n_r; ++k) tc[k] = make_double2(yc[k], 0.0);
    // forward elimination over the interior unknowns k = 1 .. n_r-2 (dp in tc[k].y)
    double cprev = 0.0, dprev = 0.0;
    for (int k = 1; k <= n_r - 2; ++k) {
        const double rhs = six_over_h2 * (yc[k + 1] - 2.0 * yc[k] + yc[k - 1]);
        const double den = 4.0 - cprev;
        cprev = 1.0 / den;
        dprev = (rhs - dprev) / den;
        cc[k] = cprev;
        tc[k].y = dprev;
    }
    // back substitution; M_{n_r-1} = 0 already
    for (int k = n_r - 3; k >= 1; --k) tc[k].y -= cc[k] * tc[k + 1].y;
}

// Flat projector kernel: one thread per grid point j of the concatenated atom
// point sets; the atom is found by binary search over the CSR offsets.  A point
// whose offsets are inconsistent (outside [offsets[a], offsets[a+1]) or beyond
// n_points) is skipped, so every store stays inside out[F * n_points].
template <int LMAX, typename TIO>
__global__ __launch_bounds__(256) void proj_kernel(const TIO* __restrict__ centers,
                                                   const int64_t* __restrict__ offsets, int n_atoms,
                                                   const TIO* __restrict__ points, int64_t n_points,
                                                   const double2* __restrict__ table, int tab_ch,
                                                   int n_tables, const int32_t* __restrict__ table_of_atom,
                                                   SplineGrid g, TIO* __restrict__ out)
{
    constexpr int F = nfun(LMAX);
    const int64_t j = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (j >= n_points) return;
    int lo = 0, hi = n_atoms - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (offsets[mid] <= j) lo = mid;
        else hi = mid - 1;
    }
    const int a = lo;
    const int64_t o0 = offsets[a], o1 = offsets[a + 1];
    if (!(o0 >= 0 && o0 <= j && j < o1 && o1 <= n_points)) return;
    int t = table_of_atom ? table_of_atom[a] : a;
    t = t < 0 ? 0 : (t >= n_tables ? n_tables - 1 : t);
    const double c[3] = {double(centers[3 * a]), double(centers[3 * a + 1]), double(centers[3 * a + 2])};
    proj_point<LMAX, TIO>(points + 3 * j, c, table + int64_t(t) * tab_ch * g.n_r, g,
                          out + F * o0 + (j - o0), o1 - o0);
}

template <int LMAX, typename TIO>
static hipError_t launch_proj_l(const ProjArgs<TIO>& A, hipStream_t s)
{
    const int64_t grid = (A.n_points + 255) / 256;
    if (grid > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL((proj_kernel<LMAX, TIO>), dim3(unsigned(grid)), dim3(256), 0, s, A.centers, A.offsets,
                       A.n_atoms, A.points, A.n_points, A.table, A.tab_ch, A.n_tables, A.table_of_atom,
                       SplineGrid{A.n_r, A.h, 1.0 / A.h, A.r_max, A.h * A.h / 6.0}, A.out);
    return hipGetLastError();
}

template <typename TIO>
hipError_t launch_projectors(int lmax, const ProjArgs<TIO>& A, hipStream_t s)
{
    switch (lmax) {
    case 0: return launch_proj_l<0, TIO>(A, s);
    case 1: return launch_proj_l<1, TIO>(A, s);
    case 2: return launch_proj_l<2, TIO>(A, s);
    case 3: return launch_proj_l<3, TIO>(A, s);
    case 4: return launch_proj_l<4, TIO>(A, s);
    case 5: return launch_proj_l<5, TIO>(A, s);
    case 6: return launch_proj_l<6, TIO>(A, s);
    case 7: return launch_proj_l<7, TIO>(A, s);
    case 8: return launch_proj_l<8, TIO>(A, s);
    case 9: return launch_proj_l<9, TIO>(A, s);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_projectors<double>(int, const ProjArgs<double>&, hipStream_t);
template hipError_t launch_projectors<float>(int, const ProjArgs<float>&, hipStream_t);

hipError_t launch_spline_setup(const double* y, double2* table, double* scratch, int n_ch, int n_r, double h,
                               hipStream_t s)
{
    const int block = 64;
    hipLaunchKernelGGL(spline_setup_kernel, dim3((n_ch + block - 1) / block), dim3(block), 0, s, y, table,
                       scratch, n_ch, n_r, 6.0 / (h * h));
    return hipGetLastError();
}

}  // namespace shk
