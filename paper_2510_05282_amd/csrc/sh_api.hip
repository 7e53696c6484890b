// sh_api.hip -- the C ABI: argument validation and dispatch to the kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/shmi.h"
#include "sh_internal.h"

namespace {

thread_local int g_last_hip = 0;

int hip_status(hipError_t e)
{
    if (e == hipSuccess) return SH_OK;
    g_last_hip = int(e);
    return SH_EHIP;
}

bool bad_lmax(int lmax) { return lmax < 0 || lmax > SH_LMAX; }

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

int sh_eval(int lmax, int64_t n, const double *xyz, double *out, hipStream_t stream)
{
    return sh_eval_ld(lmax, n, xyz, out, n, SH_F64, stream);
}

int sh_eval_f32(int lmax, int64_t n, const float *xyz, float *out, hipStream_t stream)
{
    return sh_eval_ld(lmax, n, xyz, out, n, SH_F32, stream);
}

}  // extern "C"
