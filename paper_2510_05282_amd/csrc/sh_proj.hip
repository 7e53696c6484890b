// sh_proj.hip -- radial spline tables and the fused projector build.
//
// A projector value for atom a at grid point p is R_l(|d|) * R_l^m(d / |d|) with
// d = p - c_a (the role the harmonics play in the paper's introduction).  R_l is
// a natural cubic spline through values tabulated on a uniform radial grid; it is
// 0 beyond the table's last knot.  One pass per point computes d, r, every R_l(r)
// for l <= lmax, the harmonics, and stores their products; nothing is
// materialised in between.
//
// Device table layout of a radial handle: [n_tables][n_r][channels] of double2
// (y_i, M_i), M the spline's second derivatives: the knots i and i+1 of all
// channels of a table are 2 * channels adjacent pairs, so one point's spline
// lookups touch one or two cache lines.
//
// Launch (measured on MI355X, 64 atoms / 0.9M points / lmax 3: 43 us -> 30 us):
// workgroups remapped so each XCD works through one contiguous range of atoms
// (their tables then stay in that XCD's L2); the atom of a wave found by one
// wave-wide search; plain stores; one point per lane, or, for builds of at least
// kProjVecPoints points, kProjPpl adjacent points per lane evaluated together.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sh_core.h"
#include "sh_internal.h"
#include "sh_proj.h"

namespace shk {

// ---------------------------------------------------------------- spline set-up

// One thread per channel c = (table t = c / ch, channel l = c % ch): values
// y[c][n_r] in, pairs to table[t][k][l] (spline_solve), scratch cp[c][n_r].
__global__ void spline_setup_kernel(const double* __restrict__ y, double2* __restrict__ table,
                                    double* __restrict__ cp, int n_ch, int ch, int n_r, double six_over_h2)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_ch) return;
    spline_solve(y + int64_t(c) * n_r, table + int64_t(c / ch) * n_r * ch + c % ch, ch, cp + int64_t(c) * n_r, n_r,
                 six_over_h2);
}

// Flat projector kernel over the concatenated atom point sets, PPL adjacent
// points per lane.  The wave's first point locates its atom by a wave-wide search
// over the CSR offsets; lanes past that atom's end search on their own.  A lane
// whose PPL points lie in one atom evaluates them together (proj_points); a lane
// that straddles an atom boundary or the end of the points takes them one by one.
// A point whose offsets are inconsistent (outside [offsets[a], offsets[a+1]) or
// beyond n_points) is skipped, so every store stays inside out[F * n_points].
template <int LMAX, typename TIO, int PPL>
__global__ __launch_bounds__(256) void proj_kernel(const TIO* __restrict__ centers,
                                                   const int64_t* __restrict__ offsets, int n_atoms,
                                                   const TIO* __restrict__ points, int64_t n_points,
                                                   const double2* __restrict__ table, int tab_ch,
                                                   int n_tables, const int32_t* __restrict__ table_of_atom,
                                                   SplineGrid g, TIO* __restrict__ out, int64_t j0)
{
    constexpr int F = nfun(LMAX);
    // first point of this wave; the launch covers points j0 .. j0 + 256 PPL gridDim.x - 1
    const int64_t w0 = j0 + (int64_t(xcd_tile(blockIdx.x, gridDim.x)) * 256 + (threadIdx.x & ~63u)) * PPL;
    if (w0 >= n_points) return;
    const int64_t j = w0 + (threadIdx.x & 63) * PPL;
    const bool live = j < n_points;
    double px[PPL], py[PPL], pz[PPL];  // in flight during the search
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        const TIO* p = points + 3 * (live && j + q < n_points ? j + q : w0);
        px[q] = double(p[0]);
        py[q] = double(p[1]);
        pz[q] = double(p[2]);
    }
    const int aw = wave_search(offsets, n_atoms, w0);
    const int64_t aw_end = aw >= 0 ? offsets[aw + 1] : -1;
    if (!live) return;
    auto table_of = [&](int a) {
        const int t = table_of_atom ? table_of_atom[a] : a;
        return table + int64_t(t < 0 ? 0 : (t >= n_tables ? n_tables - 1 : t)) * g.n_r * tab_ch;
    };
    auto center_of = [&](int a, double (&c)[3]) {
        c[0] = double(centers[3 * a]);
        c[1] = double(centers[3 * a + 1]);
        c[2] = double(centers[3 * a + 2]);
    };
    const int a = j < aw_end ? aw : lane_search(offsets, n_atoms, j);
    const int64_t o0 = offsets[a], o1 = offsets[a + 1];
    if constexpr (PPL == 1) {
        if (!(o0 >= 0 && o0 <= j && j < o1 && o1 <= n_points)) return;
        double c[3];
        center_of(a, c);
        proj_point<LMAX, TIO>(px[0], py[0], pz[0], c, table_of(a), tab_ch, g, out + F * o0 + (j - o0), o1 - o0);
    } else if (o0 >= 0 && o0 <= j && j + PPL <= o1 && o1 <= n_points) {
        double c[3];
        center_of(a, c);
        proj_points<LMAX, TIO, PPL>(px, py, pz, c, table_of(a), tab_ch, g, out + F * o0 + (j - o0), o1 - o0);
    } else {
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
            const int64_t jq = j + q;
            if (jq >= n_points) break;
            const int b = jq < aw_end ? aw : lane_search(offsets, n_atoms, jq);
            const int64_t b0 = offsets[b], b1 = offsets[b + 1];
            if (!(b0 >= 0 && b0 <= jq && jq < b1 && b1 <= n_points)) continue;
            double c[3];
            center_of(b, c);
            proj_point<LMAX, TIO>(px[q], py[q], pz[q], c, table_of(b), tab_ch, g, out + F * b0 + (jq - b0),
                                  b1 - b0);
        }
    }
}

// Points per launch: keeps each grid well inside the 32-bit work-item count of a
// dispatch (a multiple of every lane width, so only the last launch has a tail).
constexpr int64_t kProjChunk = int64_t(1) << 28;

template <int LMAX, typename TIO, int P>
static hipError_t launch_proj_p(const ProjArgs<TIO>& A, hipStream_t s)
{
    const SplineGrid g{A.n_r, A.h, 1.0 / A.h, A.r_max, A.h * A.h / 6.0};
    for (int64_t j0 = 0; j0 < A.n_points; j0 += kProjChunk) {
        const int64_t nc = A.n_points - j0 < kProjChunk ? A.n_points - j0 : kProjChunk;
        hipLaunchKernelGGL((proj_kernel<LMAX, TIO, P>), dim3(unsigned((nc + 256 * P - 1) / (256 * P))), dim3(256), 0,
                           s, A.centers, A.offsets, A.n_atoms, A.points, A.n_points, A.table, A.tab_ch, A.n_tables,
                           A.table_of_atom, g, A.out, j0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int LMAX, typename TIO>
static hipError_t launch_proj_l(const ProjArgs<TIO>& A, hipStream_t s)
{
    return A.n_points >= kProjVecPoints ? launch_proj_p<LMAX, TIO, kProjPpl<TIO>>(A, s)
                                        : launch_proj_p<LMAX, TIO, 1>(A, s);
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

hipError_t launch_spline_setup(const double* y, double2* table, double* scratch, int n_ch, int ch, int n_r,
                               double h, hipStream_t s)
{
    const int block = 64;
    hipLaunchKernelGGL(spline_setup_kernel, dim3((n_ch + block - 1) / block), dim3(block), 0, s, y, table,
                       scratch, n_ch, ch, n_r, 6.0 / (h * h));
    return hipGetLastError();
}

}  // namespace shk
