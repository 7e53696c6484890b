// sh_internal.h -- launchers shared between the kernel files and the C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace shk {

// Knot pair type of the radial tables an FP64 or FP32 kernel reads.
template <typename TIO> struct Knot { using type = double2; };
template <> struct Knot<float> { using type = float2; };
template <typename TIO> using knot_t = typename Knot<TIO>::type;

// Forward values R_l^m for l <= lmax at n points xyz[n][3] into out[F][ld].
template <typename TIO>
hipError_t launch_fwd(int lmax, int64_t n, const TIO* xyz, TIO* out, int64_t ld, hipStream_t s);
// The same from unit vectors (no normalisation) and from angles theta[n], phi[n].
template <typename TIO>
hipError_t launch_fwd_unit(int lmax, int64_t n, const TIO* xyz, TIO* out, int64_t ld, hipStream_t s);
template <typename TIO>
hipError_t launch_fwd_angles(int lmax, int64_t n, const TIO* theta, const TIO* phi, TIO* out, int64_t ld,
                             hipStream_t s);
// Complex harmonics Y_l^m into out[F][ld] of (re, im) pairs (ld in complex elements).
// input: 0 = Cartesian xyz in0 [n][3], 1 = unit vectors in0 [n][3], 2 = angles
// theta = in0[n], phi = in1[n] (the values of In and of sh_input).
template <typename TIO>
hipError_t launch_fwd_complex(int lmax, int64_t n, int input, const TIO* in0, const TIO* in1, TIO* out, int64_t ld,
                              hipStream_t s);

// Vector-Jacobian product: gxyz[n][3] = sum_f G[f][i] dR_f/dx at xyz[n][3]; G is [F][ldg].
template <typename TIO>
hipError_t launch_grad(int lmax, int64_t n, const TIO* xyz, const TIO* G, int64_t ldg, TIO* gxyz, hipStream_t s);

// Spinor harmonics into out[2 (lmax+1)^2][2][ld] of (re, im) pairs; inputs as above.
template <typename TIO>
hipError_t launch_fwd_spinor(int lmax, int64_t n, int input, const TIO* in0, const TIO* in1, TIO* out, int64_t ld,
                             hipStream_t s);

// Real harmonics up to lmax <= SH_LMAX_REC by recurrence.
template <typename TIO>
hipError_t launch_rec(int lmax, int64_t n, const TIO* xyz, TIO* out, int64_t ld, hipStream_t s);
// Backward pass of launch_rec (lmax <= SH_LMAX_REC), arguments as launch_grad.
template <typename TIO>
hipError_t launch_grad_rec(int lmax, int64_t n, const TIO* xyz, const TIO* G, int64_t ldg, TIO* gxyz,
                           hipStream_t s);

// Complex and spinor harmonics by recurrence (lmax <= SH_LMAX_REC), inputs and
// layout as launch_fwd_complex / launch_fwd_spinor.
template <typename TIO>
hipError_t launch_rec_complex(int lmax, int64_t n, int input, const TIO* in0, const TIO* in1, TIO* out, int64_t ld,
                              hipStream_t s);
template <typename TIO>
hipError_t launch_rec_spinor(int lmax, int64_t n, int input, const TIO* in0, const TIO* in1, TIO* out, int64_t ld,
                             hipStream_t s);

// Values out[F][ld] and Jacobian jac[3][F][ld] in one pass (FP64).
hipError_t launch_jac(int lmax, int64_t n, const double* xyz, double* out, double* jac, int64_t ld, hipStream_t s);

// Arguments of the flat projector kernel (device pointers unless noted).
template <typename TIO>
struct ProjArgs {
    const TIO* centers;            // [n_atoms][3]
    const int64_t* offsets;        // [n_atoms+1] CSR over points
    int n_atoms;
    const TIO* points;             // [n_points][3]
    int64_t n_points;
    const knot_t<TIO>* table;      // radial handle's tables (the float copy for FP32)
    int tab_ch;                    // channels per table
    int n_tables;
    const int32_t* table_of_atom;  // [n_atoms] or null (atom a uses table a)
    int n_r;
    double h, r_max;
    TIO* out;                      // atom a's [F][n_a] block at out + F * offsets[a]
};

template <typename TIO>
hipError_t launch_projectors(int lmax, const ProjArgs<TIO>& A, hipStream_t s);

// table_f32[k] = table[k] rounded to float, k < n (device arrays).
hipError_t launch_narrow_tables(const double2* table, float2* table_f32, int64_t n, hipStream_t s);

// The first ch_out pairs of each of `rows` rows of ch_in pairs: out[rows][ch_out]
// from in[rows][ch_in] (device arrays, P = double2 or float2, 1 <= ch_out <= ch_in).
template <typename P>
hipError_t launch_compact_tables(const P* in, P* out, int64_t rows, int ch_in, int ch_out, hipStream_t s);

// Natural-spline second derivatives for n_ch = n_tables * ch channels of n_r
// values y[n_ch][n_r] (device): writes (y, M) pairs to table[n_tables][n_r][ch];
// scratch holds n_ch * n_r doubles.
hipError_t launch_spline_setup(const double* y, double2* table, double* scratch, int n_ch, int ch, int n_r,
                               double h, hipStream_t s);

}  // namespace shk
