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
// kProjVecPoints points, kProjPpl adjacent points per lane evaluated together, with
// at most 2 resident workgroups per CU (kProjCapLds); those builds run
// proj_vec_kernel where kProjVecKernel or kProjVecWindow is set.
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
// points per lane.  A lane whose PPL points lie in one atom evaluates them
// together (proj_points); a lane that straddles an atom boundary or the end of
// the points takes them one by one.  A point whose offsets are inconsistent
// (outside [offsets[a], offsets[a+1]) or beyond n_points) is skipped, so every
// store stays inside out[F * n_points].
//
// Finding a point's atom: with at most 64 atoms (SMALL), lane k loads atom k's
// offsets, centre and table index while the point loads are in flight; a ballot
// over the loaded offsets gives the wave's first atom aw, whose data (and that of
// aw + 1, where a wave crosses into the next atom) every lane reads from lanes aw
// and aw + 1.  That leaves one dependent step (the spline lookup) between the
// point loads and the arithmetic.  Otherwise, and for lanes past atom aw + 1, the
// wave's atom comes from a wave-wide search and a lane's from a binary search, and
// the atom's data is loaded after it.  Measured on the 64-atom lmax 3 build (one
// point per lane): 29.6-29.8 us -> 27.6-28.0 us.  In this kernel the launches with
// several points per lane keep the search: there the preload alone cost as much as
// the shorter chain saved (-6% to +5% across lmax and dtype on 64 x 150k-point
// builds); proj_vec_kernel combines it with loading every knot of a lane at once.
struct AtomRef {
    int64_t o0, o1;  // its point range
    double c[3];
    int t;           // its table
};

template <int LMAX, typename TIO, int PPL, bool SMALL>
__global__ __launch_bounds__(256) void proj_kernel(const TIO* __restrict__ centers,
                                                   const int64_t* __restrict__ offsets, int n_atoms,
                                                   const TIO* __restrict__ points, int64_t n_points,
                                                   const knot_t<TIO>* __restrict__ table, int tab_ch,
                                                   int n_tables, const int32_t* __restrict__ table_of_atom,
                                                   SplineGrid g, TIO* __restrict__ out, int64_t j0)
{
    constexpr int F = nfun(LMAX);
    // first point of this wave; the launch covers points j0 .. j0 + 256 PPL gridDim.x - 1
    const int64_t w0 = j0 + (int64_t(xcd_tile(blockIdx.x, gridDim.x)) * 256 + (threadIdx.x & ~63u)) * PPL;
    if (w0 >= n_points) return;
    const int lane = threadIdx.x & 63;
    const int64_t j = w0 + lane * PPL;
    const bool live = j < n_points;
    double px[PPL], py[PPL], pz[PPL];
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        const TIO* p = points + 3 * (live && j + q < n_points ? j + q : w0);
        px[q] = double(p[0]);
        py[q] = double(p[1]);
        pz[q] = double(p[2]);
    }
    auto clamp_table = [&](int t) { return t < 0 ? 0 : (t >= n_tables ? n_tables - 1 : t); };
    auto load_atom = [&](int a) {
        AtomRef r;
        r.o0 = offsets[a];
        r.o1 = offsets[a + 1];
        r.c[0] = double(centers[3 * a]);
        r.c[1] = double(centers[3 * a + 1]);
        r.c[2] = double(centers[3 * a + 2]);
        r.t = clamp_table(table_of_atom ? table_of_atom[a] : a);
        return r;
    };
    AtomRef A0, A1;  // atoms aw and aw + 1 (o0 = o1 = -1 if there is none)
    A0.o0 = A0.o1 = A1.o0 = A1.o1 = -1;
    int aw;
    if constexpr (SMALL) {
        AtomRef mine{};  // atom `lane`
        if (lane < n_atoms) mine = load_atom(lane);
        const int c = __popcll(__ballot(lane < n_atoms && mine.o0 <= w0));
        aw = c - 1;
        if (aw >= 0) {
            A0 = AtomRef{lane_value(mine.o0, aw), lane_value(mine.o1, aw),
                         {lane_value(mine.c[0], aw), lane_value(mine.c[1], aw), lane_value(mine.c[2], aw)},
                         lane_value(mine.t, aw)};
        }
        if (aw + 1 < n_atoms) {
            const int b = aw + 1;
            A1 = AtomRef{lane_value(mine.o0, b), lane_value(mine.o1, b),
                         {lane_value(mine.c[0], b), lane_value(mine.c[1], b), lane_value(mine.c[2], b)},
                         lane_value(mine.t, b)};
        }
    } else {
        aw = wave_search(offsets, n_atoms, w0);
        if (aw >= 0) A0.o1 = offsets[aw + 1];  // the rest of atom aw is loaded by the lanes that need it
    }
    if (!live) return;
    // atom of point jq and its data; ok = false if jq's range is inconsistent
    auto atom_of = [&](int64_t jq, AtomRef& r) {
        if (SMALL && A0.o0 <= jq && jq < A0.o1) {
            r = A0;
        } else if (SMALL && A1.o0 <= jq && jq < A1.o1) {
            r = A1;
        } else {
            r = load_atom(jq < A0.o1 ? aw : lane_search(offsets, n_atoms, jq));
        }
        return r.o0 >= 0 && r.o0 <= jq && jq < r.o1 && r.o1 <= n_points;
    };
    AtomRef A;
    const bool ok = atom_of(j, A);
    if constexpr (PPL == 1) {
        if (!ok) return;
        proj_point<LMAX, TIO>(px[0], py[0], pz[0], A.c, table + int64_t(A.t) * g.n_r * tab_ch, tab_ch, g,
                              out + F * A.o0 + (j - A.o0), A.o1 - A.o0);
    } else if (ok && j + PPL <= A.o1) {
        proj_points<LMAX, TIO, PPL>(px, py, pz, A.c, table + int64_t(A.t) * g.n_r * tab_ch, tab_ch, g,
                                    out + F * A.o0 + (j - A.o0), A.o1 - A.o0);
    } else {
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
            const int64_t jq = j + q;
            if (jq >= n_points) break;
            AtomRef B;
            if (!atom_of(jq, B)) continue;
            proj_point<LMAX, TIO>(px[q], py[q], pz[q], B.c, table + int64_t(B.t) * g.n_r * tab_ch, tab_ch, g,
                                  out + F * B.o0 + (jq - B.o0), B.o1 - B.o0);
        }
    }
}

// The launches with several points per lane, for the (dtype, lmax) where
// kProjVecKernel (at most 64 atoms) or kProjVecWindow (more) is set: lane k loads
// the offsets, centre and table of atom a0 + k with the points (a0 = 0 for at most
// 64 atoms, as the one-point SMALL path does; otherwise the wave's atom, from one
// wave-wide search), a ballot gives the wave's
// atom and the next, and a lane then issues the knot loads of all its points before
// it evaluates any spline (spline_knots, then spline_from), so the chain per lane is
// the point loads, one wave of knot loads and the stores.  Each lane's points lie
// in one of those two atoms unless the wave crosses more than one atom boundary;
// such lanes, and lanes that straddle a boundary, take their points one by one.
// The same arithmetic as proj_kernel, so the same bits.
template <int LMAX, typename TIO, int PPL>
__global__ __launch_bounds__(256) void proj_vec_kernel(const TIO* __restrict__ centers,
                                                       const int64_t* __restrict__ offsets, int n_atoms,
                                                       const TIO* __restrict__ points, int64_t n_points,
                                                       const knot_t<TIO>* __restrict__ table, int tab_ch,
                                                       int n_tables, const int32_t* __restrict__ table_of_atom,
                                                       SplineGrid g, TIO* __restrict__ out, int64_t j0)
{
    using V = typename vec_of<TIO, PPL>::type;
    constexpr int F = nfun(LMAX);
    const int64_t w0 = j0 + (int64_t(xcd_tile(blockIdx.x, gridDim.x)) * 256 + (threadIdx.x & ~63u)) * PPL;
    if (w0 >= n_points) return;
    const int wl = threadIdx.x & 63;  // lane in the wave
    auto load_atom = [&](int a) {
        AtomRef r;
        r.o0 = offsets[a];
        r.o1 = offsets[a + 1];
        r.c[0] = double(centers[3 * a]);
        r.c[1] = double(centers[3 * a + 1]);
        r.c[2] = double(centers[3 * a + 2]);
        const int t = table_of_atom ? table_of_atom[a] : a;
        r.t = t < 0 ? 0 : (t >= n_tables ? n_tables - 1 : t);
        return r;
    };
    int a0 = 0;  // first atom of the window held in the lanes
    if (n_atoms > 64) {
        a0 = wave_search(offsets, n_atoms, w0);
        a0 = a0 < 0 ? 0 : a0;
    }
    const int nw = n_atoms - a0 < 64 ? n_atoms - a0 : 64;
    AtomRef mine{};
    if (wl < nw) mine = load_atom(a0 + wl);
    const int64_t j = w0 + wl * PPL;
    double px[PPL], py[PPL], pz[PPL];
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        const TIO* p = points + 3 * (j + q < n_points ? j + q : w0);
        px[q] = double(p[0]);
        py[q] = double(p[1]);
        pz[q] = double(p[2]);
    }
    auto atom_at = [&](int a) {
        return AtomRef{lane_value(mine.o0, a), lane_value(mine.o1, a),
                       {lane_value(mine.c[0], a), lane_value(mine.c[1], a), lane_value(mine.c[2], a)},
                       lane_value(mine.t, a)};
    };
    const int aw = __popcll(__ballot(wl < nw && mine.o0 <= w0)) - 1;  // in the window
    AtomRef A0, A1;  // atoms a0 + aw and a0 + aw + 1 (o0 = o1 = -1 if there is none)
    A0.o0 = A0.o1 = A1.o0 = A1.o1 = -1;
    if (aw >= 0) A0 = atom_at(aw);
    if (aw + 1 < nw) A1 = atom_at(aw + 1);
    if (j >= n_points) return;
    const bool in0 = A0.o0 >= 0 && A0.o0 <= j && j + PPL <= A0.o1 && A0.o1 <= n_points;
    const bool in1 = A1.o0 >= 0 && A1.o0 <= j && j + PPL <= A1.o1 && A1.o1 <= n_points;
    if (!in0 && !in1) {
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
            const int64_t jq = j + q;
            if (jq >= n_points) break;
            const AtomRef B = load_atom(lane_search(offsets, n_atoms, jq));
            if (!(B.o0 >= 0 && B.o0 <= jq && jq < B.o1 && B.o1 <= n_points)) continue;
            proj_point<LMAX, TIO>(px[q], py[q], pz[q], B.c, table + int64_t(B.t) * g.n_r * tab_ch, tab_ch, g,
                                  out + F * B.o0 + (jq - B.o0), B.o1 - B.o0);
        }
        return;
    }
    const AtomRef& A = in0 ? A0 : A1;
    const knot_t<TIO>* tab = table + int64_t(A.t) * g.n_r * tab_ch;
    knot_t<TIO> ka[PPL][LMAX + 1], kb[PPL][LMAX + 1];
    double r[PPL];
    V x, y, z, k;
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        const double dx = px[q] - A.c[0], dy = py[q] - A.c[1], dz = pz[q] - A.c[2];
        double xb, yb, zb, keep;
        normalize(dx, dy, dz, xb, yb, zb, keep);
        r[q] = sqrt(__builtin_fma(dx, dx, __builtin_fma(dy, dy, dz * dz)));
        spline_knots<LMAX + 1>(tab, tab_ch, g, r[q], ka[q], kb[q]);
        lane<V, PPL>(x, q) = TIO(xb);
        lane<V, PPL>(y, q) = TIO(yb);
        lane<V, PPL>(z, q) = TIO(zb);
        lane<V, PPL>(k, q) = TIO(keep);
    }
    TIO R[PPL][LMAX + 1];
#pragma unroll
    for (int q = 0; q < PPL; ++q) spline_from<LMAX + 1, TIO>(ka[q], kb[q], g, r[q], R[q]);
    TIO* o = out + F * A.o0 + (j - A.o0);
    const int64_t stride = A.o1 - A.o0;
    eval_unit<LMAX, V>(x, y, z, k, [&](int f, V v) {
        const int l = l_of_row(f);
        V rl;
#pragma unroll
        for (int q = 0; q < PPL; ++q) lane<V, PPL>(rl, q) = R[q][l];
        store_run<TIO, PPL>(o + int64_t(f) * stride, rl * v, PPL);
    });
}

// Points per launch: keeps each grid well inside the 32-bit work-item count of a
// dispatch (a multiple of every lane width, so only the last launch has a tail).
constexpr int64_t kProjChunk = int64_t(1) << 28;

template <int LMAX, typename TIO, int P>
static void launch_vec(const ProjArgs<TIO>& A, const SplineGrid& g, dim3 grid, size_t lds, int64_t j0, hipStream_t s)
{
    if constexpr (P > 1 && (kProjVecKernel<TIO, LMAX> || kProjVecWindow<TIO, LMAX>))
        hipLaunchKernelGGL((proj_vec_kernel<LMAX, TIO, P>), grid, dim3(256), lds, s, A.centers, A.offsets,
                           A.n_atoms, A.points, A.n_points, A.table, A.tab_ch, A.n_tables, A.table_of_atom, g,
                           A.out, j0);
}

template <int LMAX, typename TIO, int P>
static hipError_t launch_proj_p(const ProjArgs<TIO>& A, hipStream_t s)
{
    const SplineGrid g{A.n_r, A.h, 1.0 / A.h, A.r_max, A.h * A.h / 6.0};
    const size_t lds = P > 1 ? kProjCapLds<TIO, LMAX> : 0;
    for (int64_t j0 = 0; j0 < A.n_points; j0 += kProjChunk) {
        const int64_t nc = A.n_points - j0 < kProjChunk ? A.n_points - j0 : kProjChunk;
        const dim3 grid = dim3(unsigned((nc + 256 * P - 1) / (256 * P))), block = dim3(256);
        const bool vec = P > 1 && (A.n_atoms <= 64 ? kProjVecKernel<TIO, LMAX> : kProjVecWindow<TIO, LMAX>);
        if (P == 1 && A.n_atoms <= 64)
            hipLaunchKernelGGL((proj_kernel<LMAX, TIO, P, P == 1>), grid, block, 0, s, A.centers, A.offsets,
                               A.n_atoms, A.points, A.n_points, A.table, A.tab_ch, A.n_tables, A.table_of_atom, g,
                               A.out, j0);
        else if (vec)
            launch_vec<LMAX, TIO, P>(A, g, grid, lds, j0, s);
        else
            hipLaunchKernelGGL((proj_kernel<LMAX, TIO, P, false>), grid, block, lds, s, A.centers, A.offsets,
                               A.n_atoms, A.points, A.n_points, A.table, A.tab_ch, A.n_tables, A.table_of_atom, g,
                               A.out, j0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int LMAX, typename TIO>
static hipError_t launch_proj_l(const ProjArgs<TIO>& A, hipStream_t s)
{
    return A.n_points >= kProjVecPoints ? launch_proj_p<LMAX, TIO, kProjPpl<TIO, LMAX>>(A, s)
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

__global__ void narrow_tables_kernel(const double2* __restrict__ in, float2* __restrict__ out, int64_t n)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k < n) out[k] = make_float2(float(in[k].x), float(in[k].y));
}

hipError_t launch_narrow_tables(const double2* table, float2* table_f32, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(narrow_tables_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, table, table_f32, n);
    return hipGetLastError();
}

// out[row][c] = in[row][c] for c < ch_out (rows of ch_in pairs in, ch_out out)
template <typename P>
__global__ void compact_tables_kernel(const P* __restrict__ in, P* __restrict__ out, int64_t rows, int ch_in,
                                      int ch_out)
{
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= rows * ch_out) return;
    const int64_t row = k / ch_out;
    out[k] = in[row * ch_in + (k - row * ch_out)];
}

template <typename P>
hipError_t launch_compact_tables(const P* in, P* out, int64_t rows, int ch_in, int ch_out, hipStream_t s)
{
    if (rows <= 0) return hipSuccess;
    if (ch_out < 1 || ch_out > ch_in) return hipErrorInvalidValue;
    const int64_t n = rows * ch_out;
    hipLaunchKernelGGL((compact_tables_kernel<P>), dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, in, out, rows,
                       ch_in, ch_out);
    return hipGetLastError();
}

template hipError_t launch_compact_tables<double2>(const double2*, double2*, int64_t, int, int, hipStream_t);
template hipError_t launch_compact_tables<float2>(const float2*, float2*, int64_t, int, int, hipStream_t);

hipError_t launch_spline_setup(const double* y, double2* table, double* scratch, int n_ch, int ch, int n_r,
                               double h, hipStream_t s)
{
    const int block = 64;
    hipLaunchKernelGGL(spline_setup_kernel, dim3((n_ch + block - 1) / block), dim3(block), 0, s, y, table,
                       scratch, n_ch, ch, n_r, 6.0 / (h * h));
    return hipGetLastError();
}

}  // namespace shk
