// sh_eval.hip -- launchers of the forward kernels (all real Y_lm, l <= lmax).
//
// The kernel (sh_fwd.h) normalises each point in FP64, evaluates the factorised
// formulas and writes every (l, m) value to its row of the [F][ld] output.  The
// path moves 3s + F s bytes per point (s = element size) against a few hundred
// flops, so it is bound by HBM stores.  Launch choices, all measured on MI355X:
//  - Each lane evaluates 16 bytes' worth of adjacent points (two in FP64, four
//    in FP32) and stores 16 bytes per row: one contiguous 1 KiB run per wave and
//    row.  Outputs whose rows are not 16-byte aligned take the one-point kernel,
//    and so do calls of fewer than kFwdVecPoints points: a launch that leaves CUs
//    idle lasts as long as one workgroup's chain of work, which the wider lanes
//    lengthen (kernel trace, lmax 9, 4k / 16k / 64k / 100k points: FP64 5.4 / 6.8 /
//    10.1 / 14.0 us with one point per lane against 6.6 / 8.1 / 10.6 / 14.1 with
//    two, FP32 4.2 / 4.8 / 7.1 / 9.1 against 7.6 / 8.4 / 10.0 / 10.4 with four;
//    equal at 2^18 points, the wide lanes ahead above).
//  - Workgroups are remapped so each XCD walks one contiguous range of points.
//  - The 16-byte kernels reserve LDS they do not use, which caps the resident
//    workgroups per CU at 2 (8 waves).  Fewer points in flight keep the
//    concurrent writes of each row in a smaller window, which the HBM write path
//    turns into 3-14% more bandwidth depending on lmax; the one-point kernel
//    runs uncapped (with 4-byte stores it needs the extra waves).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sh_fwd.h"
#include "sh_internal.h"

namespace shk {

// Points per launch: keeps every per-row byte offset of a launch below 2^31 so
// the store address is a scalar row base plus a 32-bit per-lane offset.
constexpr int64_t kChunk = int64_t(1) << 28;

// Calls of at least this many points take the 16-byte lanes.
constexpr int64_t kFwdVecPoints = int64_t(1) << 18;

// LDS reserved (not used) per 256-thread workgroup of the 16-byte kernels: more
// than a third of the CU's 160 KiB, so at most 2 workgroups are resident per CU.
constexpr size_t kCapLds = 54 * 1024;

// The same for the real-harmonic kernel: FP64 at lmax >= 8 reserves more than half
// of the LDS, one resident workgroup (4 waves) per CU, fewer row streams at once.
// Measured on 2^26 points, fractions of 8 TB/s over five runs: FP64 lmax 9 67.8% ->
// 68.1-68.4%, lmax 8 68.0% -> 68.1-68.2%; lmax 7 and below and FP32 at every lmax
// equal or slower (FP64 lmax 2 74 -> 70%, FP32 lmax 2 74 -> 63%).
template <typename TIO, int LMAX>
constexpr size_t kFwdCapLds = sizeof(TIO) == 8 && LMAX >= 8 ? 84 * 1024 : kCapLds;

// Input pointers of a launch that starts at point c0.
template <In MODE, typename TIO>
struct Inputs {
    const TIO* a;
    const TIO* b;
    Inputs at(int64_t c0) const
    {
        if constexpr (MODE == In::kAngles) return {a + c0, b + c0};
        else return {a + 3 * c0, b};
    }
};

template <int LMAX, typename TIO, int PPL, In MODE>
static hipError_t launch_one(Inputs<MODE, TIO> in, TIO* out, int64_t n, int64_t ld, hipStream_t s)
{
    const int64_t nvec = n / PPL;
    const unsigned grid = unsigned((nvec + kFwdBlock - 1) / kFwdBlock);
    constexpr size_t lds = PPL > 1 ? kFwdCapLds<TIO, LMAX> : 0;
    hipLaunchKernelGGL((fwd_kernel<LMAX, TIO, PPL, MODE>), dim3(grid), dim3(kFwdBlock), lds, s,
                       in.a, out, uint32_t(n), ld, in.b);
    return hipGetLastError();
}

template <int LMAX, typename TIO, In MODE>
static hipError_t launch_fwd_l(int64_t n, Inputs<MODE, TIO> in, TIO* out, int64_t ld, hipStream_t s)
{
    constexpr int kVec = 16 / sizeof(TIO);
    const bool vec_ok = n >= kFwdVecPoints && ld % kVec == 0 &&
                        reinterpret_cast<uintptr_t>(out) % (kVec * sizeof(TIO)) == 0;
    for (int64_t c0 = 0; c0 < n; c0 += kChunk) {
        const int64_t nc = n - c0 < kChunk ? n - c0 : kChunk;
        hipError_t e;
        if (vec_ok) {
            const int64_t nmain = nc - nc % kVec;
            e = nmain ? launch_one<LMAX, TIO, kVec, MODE>(in.at(c0), out + c0, nmain, ld, s) : hipSuccess;
            if (e == hipSuccess && nmain < nc)
                e = launch_one<LMAX, TIO, 1, MODE>(in.at(c0 + nmain), out + c0 + nmain, nc - nmain, ld, s);
        } else {
            e = launch_one<LMAX, TIO, 1, MODE>(in.at(c0), out + c0, nc, ld, s);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename TIO, In MODE>
static hipError_t dispatch(int lmax, int64_t n, Inputs<MODE, TIO> in, TIO* out, int64_t ld, hipStream_t s)
{
    switch (lmax) {
    case 0: return launch_fwd_l<0, TIO, MODE>(n, in, out, ld, s);
    case 1: return launch_fwd_l<1, TIO, MODE>(n, in, out, ld, s);
    case 2: return launch_fwd_l<2, TIO, MODE>(n, in, out, ld, s);
    case 3: return launch_fwd_l<3, TIO, MODE>(n, in, out, ld, s);
    case 4: return launch_fwd_l<4, TIO, MODE>(n, in, out, ld, s);
    case 5: return launch_fwd_l<5, TIO, MODE>(n, in, out, ld, s);
    case 6: return launch_fwd_l<6, TIO, MODE>(n, in, out, ld, s);
    case 7: return launch_fwd_l<7, TIO, MODE>(n, in, out, ld, s);
    case 8: return launch_fwd_l<8, TIO, MODE>(n, in, out, ld, s);
    case 9: return launch_fwd_l<9, TIO, MODE>(n, in, out, ld, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename TIO>
hipError_t launch_fwd(int lmax, int64_t n, const TIO* xyz, TIO* out, int64_t ld, hipStream_t s)
{
    return dispatch<TIO, In::kXyz>(lmax, n, {xyz, nullptr}, out, ld, s);
}

template <typename TIO>
hipError_t launch_fwd_unit(int lmax, int64_t n, const TIO* xyz, TIO* out, int64_t ld, hipStream_t s)
{
    return dispatch<TIO, In::kUnit>(lmax, n, {xyz, nullptr}, out, ld, s);
}

template <typename TIO>
hipError_t launch_fwd_angles(int lmax, int64_t n, const TIO* theta, const TIO* phi, TIO* out, int64_t ld,
                             hipStream_t s)
{
    return dispatch<TIO, In::kAngles>(lmax, n, {theta, phi}, out, ld, s);
}

// Complex and spinor kernels: 16 bytes per lane and row (one FP64 complex, or two
// FP32 complex values of adjacent points), capped like the 16-byte real kernels.
// FP32 outputs whose rows are not 16-byte aligned, and a last odd point, take
// one point per lane.
// Inputs of a complex or spinor launch: in0 (+ in1 for angles) and their kind.
template <typename TIO>
struct AnyInputs {
    const TIO* a;
    const TIO* b;
    In mode;
    AnyInputs at(int64_t c0) const
    {
        if (mode == In::kAngles) return {a + c0, b + c0, mode};
        return {a + 3 * c0, b, mode};
    }
};

template <bool SPINOR, int LMAX, typename TIO, int PPL>
static hipError_t launch_complex_one(int64_t n, AnyInputs<TIO> in, TIO* out, int64_t ld, hipStream_t s)
{
    const auto kernel = SPINOR ? fwd_spinor_kernel<LMAX, TIO, PPL> : fwd_complex_kernel<LMAX, TIO, PPL>;
    const unsigned grid = unsigned((n / PPL + kFwdBlock - 1) / kFwdBlock);
    const size_t lds = PPL * sizeof(TIO) * 2 == 16 ? kCapLds : 0;
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(kFwdBlock), lds, s, in.a, out, uint32_t(n), ld, in.b, in.mode);
    return hipGetLastError();
}

// out holds rows of ld complex values; a launch starting at point c0 writes from
// out + 2 c0 (in TIO units).
template <bool SPINOR, int LMAX, typename TIO>
static hipError_t launch_complex_l(int64_t n, AnyInputs<TIO> in, TIO* out, int64_t ld, hipStream_t s)
{
    constexpr int kVec = sizeof(TIO) == 4 ? 2 : 1;
    // one point per lane below kFwdVecPoints, as for the real harmonics (FP32 lmax 9,
    // 4k / 16k / 64k / 100k points: 4.9 / 6.3 / 9.5 / 13.6 us against 6.3 / 7.2 /
    // 10.2 / 14.1 with two points per lane)
    const bool vec_ok = n >= kFwdVecPoints && ld % kVec == 0 && reinterpret_cast<uintptr_t>(out) % 16 == 0;
    for (int64_t c0 = 0; c0 < n; c0 += kChunk) {
        const int64_t nc = n - c0 < kChunk ? n - c0 : kChunk;
        const int64_t nmain = vec_ok ? nc - nc % kVec : 0;
        hipError_t e = hipSuccess;
        if (nmain) e = launch_complex_one<SPINOR, LMAX, TIO, kVec>(nmain, in.at(c0), out + 2 * c0, ld, s);
        if (e == hipSuccess && nmain < nc)
            e = launch_complex_one<SPINOR, LMAX, TIO, 1>(nc - nmain, in.at(c0 + nmain), out + 2 * (c0 + nmain), ld,
                                                         s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <bool SPINOR, typename TIO>
static hipError_t dispatch_complex(int lmax, int64_t n, AnyInputs<TIO> xyz, TIO* out, int64_t ld, hipStream_t s)
{
    switch (lmax) {
    case 0: return launch_complex_l<SPINOR, 0, TIO>(n, xyz, out, ld, s);
    case 1: return launch_complex_l<SPINOR, 1, TIO>(n, xyz, out, ld, s);
    case 2: return launch_complex_l<SPINOR, 2, TIO>(n, xyz, out, ld, s);
    case 3: return launch_complex_l<SPINOR, 3, TIO>(n, xyz, out, ld, s);
    case 4: return launch_complex_l<SPINOR, 4, TIO>(n, xyz, out, ld, s);
    case 5: return launch_complex_l<SPINOR, 5, TIO>(n, xyz, out, ld, s);
    case 6: return launch_complex_l<SPINOR, 6, TIO>(n, xyz, out, ld, s);
    case 7: return launch_complex_l<SPINOR, 7, TIO>(n, xyz, out, ld, s);
    case 8: return launch_complex_l<SPINOR, 8, TIO>(n, xyz, out, ld, s);
    case 9: return launch_complex_l<SPINOR, 9, TIO>(n, xyz, out, ld, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename TIO>
hipError_t launch_fwd_complex(int lmax, int64_t n, int input, const TIO* in0, const TIO* in1, TIO* out, int64_t ld,
                              hipStream_t s)
{
    return dispatch_complex<false, TIO>(lmax, n, {in0, in1, In(input)}, out, ld, s);
}

template <typename TIO>
hipError_t launch_fwd_spinor(int lmax, int64_t n, int input, const TIO* in0, const TIO* in1, TIO* out, int64_t ld,
                             hipStream_t s)
{
    return dispatch_complex<true, TIO>(lmax, n, {in0, in1, In(input)}, out, ld, s);
}

template hipError_t launch_fwd_spinor<double>(int, int64_t, int, const double*, const double*, double*, int64_t,
                                             hipStream_t);
template hipError_t launch_fwd_spinor<float>(int, int64_t, int, const float*, const float*, float*, int64_t,
                                             hipStream_t);
template hipError_t launch_fwd<double>(int, int64_t, const double*, double*, int64_t, hipStream_t);
template hipError_t launch_fwd<float>(int, int64_t, const float*, float*, int64_t, hipStream_t);
template hipError_t launch_fwd_unit<double>(int, int64_t, const double*, double*, int64_t, hipStream_t);
template hipError_t launch_fwd_unit<float>(int, int64_t, const float*, float*, int64_t, hipStream_t);
template hipError_t launch_fwd_angles<double>(int, int64_t, const double*, const double*, double*, int64_t,
                                              hipStream_t);
template hipError_t launch_fwd_angles<float>(int, int64_t, const float*, const float*, float*, int64_t,
                                             hipStream_t);
template hipError_t launch_fwd_complex<double>(int, int64_t, int, const double*, const double*, double*, int64_t,
                                             hipStream_t);
template hipError_t launch_fwd_complex<float>(int, int64_t, int, const float*, const float*, float*, int64_t,
                                             hipStream_t);

}  // namespace shk
