// sh_api.hip -- the C ABI: argument validation and dispatch to the kernels.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <memory>
#include <mutex>
#include <new>

#include "../../include/shmi.h"
#include "sh_fwd.h"
#include "sh_internal.h"
#include "sh_server.h"

// Radial tables owned by the library (opaque to C callers as `struct sh_radial`).
struct sh_radial {
    int lmax;      // channels per table - 1
    int n_tables;  // tables in this handle
    int n_r;       // knots per channel (uniform grid on [0, r_max])
    double r_max;
    double h;      // knot spacing r_max / (n_r - 1)
    double2* table;      // device, [n_tables][n_r][lmax+1] of (y, M)
    float2* table_f32;   // the same pairs rounded to float, read by the FP32 kernels
    // for L < lmax and L <= kCompactLmax: [n_tables][n_r][L+1], the first L + 1 pairs
    // of each row of table (and of table_f32); null otherwise
    double2* compact[shs::kCompactLmax + 1];
    float2* compact_f32[shs::kCompactLmax + 1];
};

namespace {

thread_local int g_last_hip = 0;

int hip_status(hipError_t e)
{
    if (e == hipSuccess) return SH_OK;
    g_last_hip = int(e);
    return SH_EHIP;
}

bool bad_lmax(int lmax) { return lmax < 0 || lmax > SH_LMAX; }

static_assert(int(shk::In::kXyz) == SH_IN_XYZ && int(shk::In::kUnit) == SH_IN_UNIT &&
                  int(shk::In::kAngles) == SH_IN_ANGLES,
              "the kernels' input kinds and sh_input must agree");

// Complex (SPINOR = false) or spinor harmonics from any input interface, by the
// explicit formulas (REC = false, lmax <= SH_LMAX) or the recurrence (REC = true,
// lmax <= SH_LMAX_REC).
template <bool SPINOR, bool REC, typename TIO>
static int eval_cplx(int lmax, int64_t n, int input, const TIO *in0, const TIO *in1, TIO *out, hipStream_t stream)
{
    if (lmax < 0 || lmax > (REC ? SH_LMAX_REC : SH_LMAX) || n < 0) return SH_EINVAL;
    if (input != SH_IN_XYZ && input != SH_IN_UNIT && input != SH_IN_ANGLES) return SH_EINVAL;
    if (n == 0) return SH_OK;
    if (!in0 || !out || (input == SH_IN_ANGLES && !in1)) return SH_EINVAL;
    if (REC)
        return hip_status(SPINOR ? shk::launch_rec_spinor<TIO>(lmax, n, input, in0, in1, out, n, stream)
                                 : shk::launch_rec_complex<TIO>(lmax, n, input, in0, in1, out, n, stream));
    return hip_status(SPINOR ? shk::launch_fwd_spinor<TIO>(lmax, n, input, in0, in1, out, n, stream)
                             : shk::launch_fwd_complex<TIO>(lmax, n, input, in0, in1, out, n, stream));
}

template <bool SPINOR, bool REC>
static int eval_cplx_any(int lmax, int64_t n, int input, int dtype, const void *in0, const void *in1, void *out,
                         hipStream_t stream)
{
    if (dtype == SH_F64)
        return eval_cplx<SPINOR, REC, double>(lmax, n, input, static_cast<const double *>(in0),
                                              static_cast<const double *>(in1), static_cast<double *>(out), stream);
    if (dtype == SH_F32)
        return eval_cplx<SPINOR, REC, float>(lmax, n, input, static_cast<const float *>(in0),
                                             static_cast<const float *>(in1), static_cast<float *>(out), stream);
    return SH_EINVAL;
}

template <typename TIO>
static int eval_unit(int lmax, int64_t n, const TIO *xyz, TIO *out, hipStream_t stream)
{
    if (bad_lmax(lmax) || n < 0) return SH_EINVAL;
    if (n == 0) return SH_OK;
    if (!xyz || !out) return SH_EINVAL;
    return hip_status(shk::launch_fwd_unit<TIO>(lmax, n, xyz, out, n, stream));
}

template <typename TIO>
static int eval_angles(int lmax, int64_t n, const TIO *theta, const TIO *phi, TIO *out, hipStream_t stream)
{
    if (bad_lmax(lmax) || n < 0) return SH_EINVAL;
    if (n == 0) return SH_OK;
    if (!theta || !phi || !out) return SH_EINVAL;
    return hip_status(shk::launch_fwd_angles<TIO>(lmax, n, theta, phi, out, n, stream));
}

template <typename TIO>
static int projectors(int lmax, int n_atoms, const TIO *centers, const int64_t *offsets, int64_t n_points,
                      const TIO *points, sh_radial_t radial, const int32_t *table_of_atom, TIO *out,
                      hipStream_t stream)
{
    if (bad_lmax(lmax) || n_atoms < 0 || n_points < 0 || !radial || radial->lmax < lmax) return SH_EINVAL;
    if (n_points == 0) return SH_OK;
    if (n_atoms == 0 || !centers || !offsets || !points || !out) return SH_EINVAL;
    if (!table_of_atom && radial->n_tables < n_atoms) return SH_EINVAL;
    // the copy with only the build's channels where the handle has one (same pairs)
    const bool cmp = lmax < radial->lmax && lmax <= shs::kCompactLmax;
    const shk::knot_t<TIO>* table;
    if constexpr (sizeof(TIO) == 8) table = cmp ? radial->compact[lmax] : radial->table;
    else table = cmp ? radial->compact_f32[lmax] : radial->table_f32;
    shk::ProjArgs<TIO> A{centers, offsets, n_atoms, points, n_points, table, cmp ? lmax + 1 : radial->lmax + 1,
                         radial->n_tables, table_of_atom, radial->n_r, radial->h, radial->r_max, out};
    return hip_status(shk::launch_projectors<TIO>(lmax, A, stream));
}

template <typename TIO>
static int grad_rec(int lmax, int64_t n, const TIO *xyz, const TIO *grad_out, TIO *grad_xyz, hipStream_t stream)
{
    if (lmax < 0 || lmax > SH_LMAX_REC || n < 0) return SH_EINVAL;
    if (n == 0) return SH_OK;
    if (!xyz || !grad_out || !grad_xyz) return SH_EINVAL;
    return hip_status(shk::launch_grad_rec<TIO>(lmax, n, xyz, grad_out, n, grad_xyz, stream));
}

// ---------------------------------------------------------------- no-allocation projectors

// Working memory of sh_projectors_noalloc, for at most SH_NOALLOC_MAX_VALUES knot
// values: the (y, M) pairs of the radial tables, their float copy and the spline
// solve's eliminated coefficients (64 MiB).  Every GPU the library runs on holds
// its own copy until the process ends; calls on one GPU share it.
constexpr size_t kNoAllocPairs = size_t(SH_NOALLOC_MAX_VALUES) * sizeof(double2);
constexpr size_t kNoAllocPairsF32 = size_t(SH_NOALLOC_MAX_VALUES) * sizeof(float2);
constexpr size_t kNoAllocCoef = size_t(SH_NOALLOC_MAX_VALUES) * sizeof(double);
static __device__ __align__(256) unsigned char scratch[kNoAllocPairs + kNoAllocPairsF32 + kNoAllocCoef];

// Device address of `scratch` on each GPU, looked up once per GPU with that GPU
// current (in host code the array's name is only a stand-in for it).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

int scratch_of_current_device(unsigned char** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_status(e);
    if (dev < 0 || dev >= kMaxDevices) return SH_EINVAL;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_status(e);
        if (!p) return hip_status(hipErrorInvalidSymbol);
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[dev]);
    return SH_OK;
}

template <typename TIO>
int projectors_noalloc(int lmax, int n_atoms, const TIO* centers, const int64_t* offsets, int64_t n_points,
                       const TIO* points, int n_tables, int n_r, double r_max, const double* values,
                       const int32_t* table_of_atom, TIO* out, hipStream_t stream)
{
    unsigned char* base = nullptr;
    const int rc = scratch_of_current_device(&base);
    if (rc != SH_OK) return rc;
    double2* pairs = reinterpret_cast<double2*>(base);
    float2* pairs_f32 = reinterpret_cast<float2*>(base + kNoAllocPairs);
    double* coef = reinterpret_cast<double*>(base + kNoAllocPairs + kNoAllocPairsF32);
    const int ch = lmax + 1;
    const int64_t nval = int64_t(n_tables) * ch * n_r;
    const double h = r_max / double(n_r - 1);
    // every entry the solve reads it writes first, so the buffer needs no clearing
    hipError_t e = shk::launch_spline_setup(values, pairs, coef, n_tables * ch, ch, n_r, h, stream);
    const shk::knot_t<TIO>* table;
    if constexpr (sizeof(TIO) == 8) {
        table = pairs;
    } else {
        if (e == hipSuccess) e = shk::launch_narrow_tables(pairs, pairs_f32, nval, stream);
        table = pairs_f32;
    }
    if (e != hipSuccess) return hip_status(e);
    shk::ProjArgs<TIO> A{centers, offsets, n_atoms, points, n_points, table, ch, n_tables, table_of_atom, n_r, h,
                         r_max, out};
    return hip_status(shk::launch_projectors<TIO>(lmax, A, stream));
}

}  // namespace

extern "C" {

const char *sh_strerror(int code)
{
    switch (code) {
    case SH_OK: return "success";
    case SH_EINVAL: return "invalid argument";
    case SH_EHIP: return "HIP runtime error";
    case SH_ENOMEM: return "out of memory";
    case SH_EBUSY: return "resource busy";
    default: return "unknown status code";
    }
}

int sh_last_hip_error(void) { return g_last_hip; }

int sh_eval_ld(int lmax, int64_t n, const void *xyz, void *out, int64_t ld, int dtype, hipStream_t stream)
{
    if (bad_lmax(lmax) || n < 0 || ld < n) return SH_EINVAL;
    if (dtype != SH_F64 && dtype != SH_F32) return SH_EINVAL;
    if (n == 0) return SH_OK;
    if (!xyz || !out) return SH_EINVAL;
    if (dtype == SH_F64)
        return hip_status(shk::launch_fwd<double>(lmax, n, static_cast<const double *>(xyz),
                                                  static_cast<double *>(out), ld, stream));
    return hip_status(shk::launch_fwd<float>(lmax, n, static_cast<const float *>(xyz),
                                             static_cast<float *>(out), ld, stream));
}

int sh_eval_unit(int lmax, int64_t n, const double *xyz, double *out, hipStream_t stream)
{
    return eval_unit<double>(lmax, n, xyz, out, stream);
}

int sh_eval_unit_f32(int lmax, int64_t n, const float *xyz, float *out, hipStream_t stream)
{
    return eval_unit<float>(lmax, n, xyz, out, stream);
}

int sh_eval_angles(int lmax, int64_t n, const double *theta, const double *phi, double *out, hipStream_t stream)
{
    return eval_angles<double>(lmax, n, theta, phi, out, stream);
}

int sh_eval_angles_f32(int lmax, int64_t n, const float *theta, const float *phi, float *out, hipStream_t stream)
{
    return eval_angles<float>(lmax, n, theta, phi, out, stream);
}

int sh_eval_complex(int lmax, int64_t n, const double *xyz, double *out, hipStream_t stream)
{
    return eval_cplx<false, false, double>(lmax, n, SH_IN_XYZ, xyz, nullptr, out, stream);
}

int sh_eval_complex_f32(int lmax, int64_t n, const float *xyz, float *out, hipStream_t stream)
{
    return eval_cplx<false, false, float>(lmax, n, SH_IN_XYZ, xyz, nullptr, out, stream);
}

int sh_eval_complex_in(int lmax, int64_t n, int input, int dtype, const void *in0, const void *in1, void *out,
                       hipStream_t stream)
{
    return eval_cplx_any<false, false>(lmax, n, input, dtype, in0, in1, out, stream);
}

int sh_eval_spinor(int lmax, int64_t n, const double *xyz, double *out, hipStream_t stream)
{
    return eval_cplx<true, false, double>(lmax, n, SH_IN_XYZ, xyz, nullptr, out, stream);
}

int sh_eval_spinor_f32(int lmax, int64_t n, const float *xyz, float *out, hipStream_t stream)
{
    return eval_cplx<true, false, float>(lmax, n, SH_IN_XYZ, xyz, nullptr, out, stream);
}

int sh_eval_spinor_in(int lmax, int64_t n, int input, int dtype, const void *in0, const void *in1, void *out,
                      hipStream_t stream)
{
    return eval_cplx_any<true, false>(lmax, n, input, dtype, in0, in1, out, stream);
}

int sh_eval_complex_rec(int lmax, int64_t n, int input, int dtype, const void *in0, const void *in1, void *out,
                        hipStream_t stream)
{
    return eval_cplx_any<false, true>(lmax, n, input, dtype, in0, in1, out, stream);
}

int sh_eval_spinor_rec(int lmax, int64_t n, int input, int dtype, const void *in0, const void *in1, void *out,
                       hipStream_t stream)
{
    return eval_cplx_any<true, true>(lmax, n, input, dtype, in0, in1, out, stream);
}

int sh_eval_rec(int lmax, int64_t n, const double *xyz, double *out, hipStream_t stream)
{
    if (lmax < 0 || lmax > SH_LMAX_REC || n < 0) return SH_EINVAL;
    if (n == 0) return SH_OK;
    if (!xyz || !out) return SH_EINVAL;
    return hip_status(shk::launch_rec<double>(lmax, n, xyz, out, n, stream));
}

int sh_eval_rec_f32(int lmax, int64_t n, const float *xyz, float *out, hipStream_t stream)
{
    if (lmax < 0 || lmax > SH_LMAX_REC || n < 0) return SH_EINVAL;
    if (n == 0) return SH_OK;
    if (!xyz || !out) return SH_EINVAL;
    return hip_status(shk::launch_rec<float>(lmax, n, xyz, out, n, stream));
}

int sh_eval(int lmax, int64_t n, const double *xyz, double *out, hipStream_t stream)
{
    return sh_eval_ld(lmax, n, xyz, out, n, SH_F64, stream);
}

int sh_eval_f32(int lmax, int64_t n, const float *xyz, float *out, hipStream_t stream)
{
    return sh_eval_ld(lmax, n, xyz, out, n, SH_F32, stream);
}

int sh_eval_grad(int lmax, int64_t n, const double *xyz, const double *grad_out, double *grad_xyz,
                 hipStream_t stream)
{
    if (bad_lmax(lmax) || n < 0) return SH_EINVAL;
    if (n == 0) return SH_OK;
    if (!xyz || !grad_out || !grad_xyz) return SH_EINVAL;
    return hip_status(shk::launch_grad<double>(lmax, n, xyz, grad_out, n, grad_xyz, stream));
}

int sh_eval_grad_f32(int lmax, int64_t n, const float *xyz, const float *grad_out, float *grad_xyz,
                     hipStream_t stream)
{
    if (bad_lmax(lmax) || n < 0) return SH_EINVAL;
    if (n == 0) return SH_OK;
    if (!xyz || !grad_out || !grad_xyz) return SH_EINVAL;
    return hip_status(shk::launch_grad<float>(lmax, n, xyz, grad_out, n, grad_xyz, stream));
}

int sh_eval_grad_rec(int lmax, int64_t n, const double *xyz, const double *grad_out, double *grad_xyz,
                     hipStream_t stream)
{
    return grad_rec<double>(lmax, n, xyz, grad_out, grad_xyz, stream);
}

int sh_eval_grad_rec_f32(int lmax, int64_t n, const float *xyz, const float *grad_out, float *grad_xyz,
                         hipStream_t stream)
{
    return grad_rec<float>(lmax, n, xyz, grad_out, grad_xyz, stream);
}

int sh_eval_jac(int lmax, int64_t n, const double *xyz, double *out, double *jac, hipStream_t stream)
{
    if (bad_lmax(lmax) || n < 0) return SH_EINVAL;
    if (n == 0) return SH_OK;
    if (!xyz || !out || !jac) return SH_EINVAL;
    return hip_status(shk::launch_jac(lmax, n, xyz, out, jac, n, stream));
}

int sh_radial_create(int lmax, int n_tables, int n_r, double r_max, const double *host_values, sh_radial_t *out)
{
    if (!out) return SH_EINVAL;
    *out = nullptr;
    if (bad_lmax(lmax) || n_tables < 1 || n_r < 2 || !(r_max > 0.0) || !isfinite(r_max) || !host_values)
        return SH_EINVAL;
    const int64_t n_ch = int64_t(n_tables) * (lmax + 1);
    const int64_t nval = n_ch * n_r;
    if (n_ch > 0x7fffffff || nval > (int64_t(1) << 34)) return SH_EINVAL;
    std::unique_ptr<sh_radial> h(new (std::nothrow) sh_radial{});
    if (!h) return SH_ENOMEM;
    h->lmax = lmax;
    h->n_tables = n_tables;
    h->n_r = n_r;
    h->r_max = r_max;
    h->h = r_max / double(n_r - 1);
    const int n_compact = lmax < shs::kCompactLmax + 1 ? lmax : shs::kCompactLmax + 1;  // L = 0 .. n_compact - 1
    const size_t rows = size_t(n_tables) * size_t(n_r);  // knot rows over all tables
    double *y = nullptr, *scratch = nullptr;
    hipStream_t st = nullptr;
    bool ok = hipMalloc(&h->table, sizeof(double2) * nval) == hipSuccess &&
              hipMalloc(&h->table_f32, sizeof(float2) * nval) == hipSuccess &&
              hipMalloc(&y, sizeof(double) * nval) == hipSuccess &&
              hipMalloc(&scratch, sizeof(double) * nval) == hipSuccess;
    for (int L = 0; ok && L < n_compact; ++L)
        ok = hipMalloc(&h->compact[L], sizeof(double2) * rows * (L + 1)) == hipSuccess &&
             hipMalloc(&h->compact_f32[L], sizeof(float2) * rows * (L + 1)) == hipSuccess;
    int rc = SH_OK;
    if (!ok) {
        (void)hipGetLastError();
        rc = SH_ENOMEM;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipMemcpyAsync(y, host_values, sizeof(double) * nval, hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = shk::launch_spline_setup(y, h->table, scratch, int(n_ch), lmax + 1, n_r, h->h, st);
        if (e == hipSuccess) e = shk::launch_narrow_tables(h->table, h->table_f32, nval, st);
        // the compact copies: the first L + 1 pairs of every knot row
        for (int L = 0; e == hipSuccess && L < n_compact; ++L) {
            e = shk::launch_compact_tables(h->table, h->compact[L], int64_t(rows), lmax + 1, L + 1, st);
            if (e == hipSuccess)
                e = shk::launch_compact_tables(h->table_f32, h->compact_f32[L], int64_t(rows), lmax + 1, L + 1, st);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        rc = hip_status(e);
    }
    if (st) (void)hipStreamDestroy(st);
    if (y) (void)hipFree(y);
    if (scratch) (void)hipFree(scratch);
    if (rc != SH_OK) {
        (void)sh_radial_destroy(h.release());
        return rc;
    }
    *out = h.release();
    return SH_OK;
}

int sh_radial_destroy(sh_radial_t radial)
{
    if (!radial) return SH_OK;
    hipError_t e = hipSuccess;
    auto release = [&](void* p) {
        if (!p) return;
        const hipError_t f = hipFree(p);
        if (e == hipSuccess) e = f;
    };
    release(radial->table);
    release(radial->table_f32);
    for (int L = 0; L <= shs::kCompactLmax; ++L) {
        release(radial->compact[L]);
        release(radial->compact_f32[L]);
    }
    delete radial;
    return hip_status(e);
}

int sh_projectors(int lmax, int n_atoms, const double *centers, const int64_t *offsets, int64_t n_points,
                  const double *points, sh_radial_t radial, const int32_t *table_of_atom, double *out,
                  hipStream_t stream)
{
    return projectors<double>(lmax, n_atoms, centers, offsets, n_points, points, radial, table_of_atom, out,
                              stream);
}

int sh_projectors_f32(int lmax, int n_atoms, const float *centers, const int64_t *offsets, int64_t n_points,
                      const float *points, sh_radial_t radial, const int32_t *table_of_atom, float *out,
                      hipStream_t stream)
{
    return projectors<float>(lmax, n_atoms, centers, offsets, n_points, points, radial, table_of_atom, out,
                             stream);
}

int sh_projectors_noalloc(int lmax, int dtype, int n_atoms, const void *centers, const int64_t *offsets,
                          int64_t n_points, const void *points, int n_tables, int n_r, double r_max,
                          const double *values, const int32_t *table_of_atom, void *out, hipStream_t stream)
{
    if (bad_lmax(lmax) || (dtype != SH_F64 && dtype != SH_F32) || n_atoms < 0 || n_points < 0 || n_tables < 1 ||
        n_r < 2 || !(r_max > 0.0) || !isfinite(r_max))
        return SH_EINVAL;
    if (int64_t(n_tables) * (lmax + 1) * n_r > SH_NOALLOC_MAX_VALUES) return SH_EINVAL;
    if (n_points == 0) return SH_OK;
    if (n_atoms == 0 || !centers || !offsets || !points || !values || !out) return SH_EINVAL;
    if (!table_of_atom && n_tables < n_atoms) return SH_EINVAL;
    if (dtype == SH_F64)
        return projectors_noalloc<double>(lmax, n_atoms, static_cast<const double *>(centers), offsets, n_points,
                                          static_cast<const double *>(points), n_tables, n_r, r_max, values,
                                          table_of_atom, static_cast<double *>(out), stream);
    return projectors_noalloc<float>(lmax, n_atoms, static_cast<const float *>(centers), offsets, n_points,
                                      static_cast<const float *>(points), n_tables, n_r, r_max, values,
                                      table_of_atom, static_cast<float *>(out), stream);
}

}  // extern "C"

namespace shs {

int radial_table(sh_radial_t radial, int table, int dtype, RadialRef* out)
{
    if (!radial || !out || table < 0 || table >= radial->n_tables || (dtype != SH_F64 && dtype != SH_F32))
        return SH_EINVAL;
    const int64_t t0 = int64_t(table) * radial->n_r * (radial->lmax + 1);
    if (dtype == SH_F64) out->tab = radial->table + t0;
    else out->tab = radial->table_f32 + t0;
    for (int L = 0; L <= kCompactLmax; ++L) {
        const int64_t c0 = int64_t(table) * radial->n_r * (L + 1);
        out->compact[L] = !radial->compact[L] ? nullptr
                          : dtype == SH_F64   ? static_cast<const void*>(radial->compact[L] + c0)
                                              : static_cast<const void*>(radial->compact_f32[L] + c0);
    }
    out->lmax = radial->lmax;
    out->n_r = radial->n_r;
    out->h = radial->h;
    out->r_max = radial->r_max;
    return SH_OK;
}

}  // namespace shs
