/*
 * shmi.h -- C ABI of the MI355X real-spherical-harmonics library (libshmi.so).
 *
 * The library evaluates the real spherical harmonics R_l^m, 0 <= l <= lmax <= 9,
 * -l <= m <= l, of large batches of 3-D points, following the explicit
 * normalised-Cartesian method of Andrade et al., "SHarmonic" (arXiv 2510.05282):
 * each point is normalised (Section 2, eq. constraint) and the factorised
 * polynomial formulas of Appendix C (m <= 0) and Appendix B (m > 0) are evaluated.
 * The real harmonics are those of eq. real_harmomics built from the complex
 * harmonics of eq. sphericalfromlegendre (with the Condon-Shortley phase, which
 * the real form cancels).  At r = 0 only R_0^0 = 1/sqrt(4 pi) is nonzero
 * (Section 2).
 *
 * Conventions shared by every call:
 *  - Function index ("row") of (l, m): l*l + l + m.  F = (lmax+1)^2 rows.
 *  - Array pointers are DEVICE pointers (e.g. torch's data_ptr()) unless stated.
 *    The caller owns every buffer it passes; the library never frees them.
 *  - Points are [n][3] row-major (x, y, z), any length: only the direction of a
 *    point enters R_l^m.
 *  - Per-point outputs are SoA: [F][ld] row-major, value (row, i) at
 *    out[row * ld + i]; the plain calls use ld = n.
 *  - Every call is asynchronous on `stream` (0 = the null stream), returns as soon
 *    as its kernels are queued, never synchronises and never allocates device
 *    memory.  Calls on distinct streams may run concurrently from distinct
 *    threads.
 *  - n == 0 is a no-op returning SH_OK.  NaN inputs give NaN outputs; no other
 *    input values are rejected.
 *  - Return value: SH_OK or one of the SH_E* codes below; nothing is launched
 *    when the arguments are rejected.  No C++ exception crosses the ABI.
 */
#ifndef SHMI_H
#define SHMI_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SH_LMAX 9 /* highest l with explicit formulas (paper, Section 3) */

enum sh_status {
    SH_OK = 0,
    SH_EINVAL = 1, /* lmax outside [0, SH_LMAX], n < 0, a NULL pointer with n > 0, ld < n, bad dtype */
    SH_EHIP = 2,   /* the HIP runtime reported an error (sh_last_hip_error() gives it) */
    SH_ENOMEM = 3, /* the library could not allocate its own memory */
    SH_EBUSY = 4   /* a resource limit was reached; retry later */
};

enum sh_dtype { SH_F64 = 0, SH_F32 = 1 };

/* Real harmonics in double precision.
 *   xyz: [n][3] double, out: [F][n] double (F = (lmax+1)^2).
 * Points are normalised in FP64 (hardware reciprocal square root refined by
 * Newton steps; coordinates whose squares would underflow are rescaled by an
 * exact power of two first).  Max abs error against the exact value: 1e-13. */
int sh_eval(int lmax, int64_t n, const double *xyz, double *out, hipStream_t stream);

/* Single-precision twin: xyz [n][3] float, out [F][n] float.  The normalisation
 * (and the near-origin guard) still runs in FP64; the polynomials run in FP32.
 * Max abs error against the exact value at the float inputs: 5e-6. */
int sh_eval_f32(int lmax, int64_t n, const float *xyz, float *out, hipStream_t stream);

/* General form: out is [F][ld] with ld >= n (row stride in elements), and the
 * element type of xyz and out is given by dtype (SH_F64 or SH_F32). */
int sh_eval_ld(int lmax, int64_t n, const void *xyz, void *out, int64_t ld, int dtype,
               hipStream_t stream);

/* Static text for a status code (never NULL). */
const char *sh_strerror(int code);

/* The last hipError_t seen by this thread inside the library (0 if none). */
int sh_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SHMI_H */
