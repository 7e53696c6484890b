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

#define SH_LMAX 9      /* highest l with explicit formulas (paper, Section 3) */
#define SH_LMAX_REC 24 /* highest l of sh_eval_rec */

enum sh_status {
    SH_OK = 0,
    SH_EINVAL = 1, /* lmax outside [0, SH_LMAX], n < 0, a NULL pointer with n > 0, ld < n, bad dtype */
    SH_EHIP = 2,   /* the HIP runtime reported an error (sh_last_hip_error() gives it) */
    SH_ENOMEM = 3, /* the library could not allocate its own memory */
    SH_EBUSY = 4   /* a resource limit was reached; retry later */
};

enum sh_dtype { SH_F64 = 0, SH_F32 = 1 };

/* The paper's three input interfaces (Section 2), for the calls that take any:
 *   SH_IN_XYZ     in0 = Cartesian points [n][3] (normalised here, origin convention)
 *   SH_IN_UNIT    in0 = points on the unit sphere [n][3], used as given
 *   SH_IN_ANGLES  in0 = polar angle theta[n], in1 = azimuth phi[n] (radians) */
enum sh_input { SH_IN_XYZ = 0, SH_IN_UNIT = 1, SH_IN_ANGLES = 2 };

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

/* The paper's other two input interfaces (Section 2), same output layout:
 *  - sh_eval_unit: xyz [n][3] already on the unit sphere (x^2 + y^2 + z^2 = 1,
 *    eq. constraint); no normalisation is done, so other inputs give meaningless
 *    values (the formulas hold only on the sphere).  The fastest interface.
 *  - sh_eval_angles: polar angle theta[n] and azimuth phi[n] (radians); the unit
 *    vector (sin t cos p, sin t sin p, cos t) is formed in FP64. */
int sh_eval_unit(int lmax, int64_t n, const double *xyz, double *out, hipStream_t stream);
int sh_eval_unit_f32(int lmax, int64_t n, const float *xyz, float *out, hipStream_t stream);
int sh_eval_angles(int lmax, int64_t n, const double *theta, const double *phi, double *out,
                   hipStream_t stream);
int sh_eval_angles_f32(int lmax, int64_t n, const float *theta, const float *phi, float *out,
                       hipStream_t stream);

/* Beyond l = 9 the paper points to recurrence relations (Conclusion):
 * sh_eval_rec evaluates R_l^m for 0 <= lmax <= SH_LMAX_REC from the stable
 * normalised associated-Legendre recurrence in z/r and (x + i y)^m / r^m, with the
 * same normalisation, origin guard and [F][n] layout as sh_eval (double). */
int sh_eval_rec(int lmax, int64_t n, const double *xyz, double *out, hipStream_t stream);

/* Single-precision twin of sh_eval_rec (normalisation in FP64, recurrence in FP32).
 * Max abs error against the exact value at the float inputs: 5e-6 for l <= 9,
 * 1e-6 (l + 1) beyond (the recurrence accumulates rounding with l). */
int sh_eval_rec_f32(int lmax, int64_t n, const float *xyz, float *out, hipStream_t stream);

/* Complex and spinor harmonics for 0 <= lmax <= SH_LMAX_REC, built from the
 * recurrence's real harmonics exactly as sh_eval_complex_in and sh_eval_spinor_in
 * build them from the explicit ones (same arguments, input interfaces and output
 * layout).  Error bounds as sh_eval_rec (FP64) and sh_eval_rec_f32 (FP32). */
int sh_eval_complex_rec(int lmax, int64_t n, int input, int dtype, const void *in0, const void *in1, void *out,
                        hipStream_t stream);
int sh_eval_spinor_rec(int lmax, int64_t n, int input, int dtype, const void *in0, const void *in1, void *out,
                       hipStream_t stream);

/* Complex harmonics Y_l^m (eq. sphericalfromlegendre, with the Condon-Shortley
 * phase), built from the real ones (Section 3): Y_l^0 = R_l^0 and, for m > 0,
 *   Y_l^m = (-1)^m (R_l^m + i R_l^-m) / sqrt(2),   Y_l^-m = (R_l^m - i R_l^-m) / sqrt(2)
 * (so that Y_l^-m = (-1)^m conj(Y_l^m), eq. conjm).  out is [F][n] complex values
 * stored as (re, im) pairs, i.e. 2 F n doubles (floats for the _f32 twin); row of
 * (l, m) as elsewhere. */
int sh_eval_complex(int lmax, int64_t n, const double *xyz, double *out, hipStream_t stream);
int sh_eval_complex_f32(int lmax, int64_t n, const float *xyz, float *out, hipStream_t stream);

/* Complex harmonics from any input interface (enum sh_input) in dtype SH_F64 or
 * SH_F32 (inputs and output alike); same output as sh_eval_complex.  SH_EINVAL
 * also for an unknown input or dtype, or in1 NULL with SH_IN_ANGLES. */
int sh_eval_complex_in(int lmax, int64_t n, int input, int dtype, const void *in0, const void *in1, void *out,
                       hipStream_t stream);

/* Spinor harmonics for spin 1/2 (eq. spinorial), built from the complex ones as
 * in Section 3: for orbital l and total j = l + 1/2 (l >= 0) or j = l - 1/2
 * (l >= 1), with m_j = -j .. j,
 *   j = l + 1/2:  upper =  sqrt((l + m_j + 1/2)/(2l+1)) Y_l^{m_j-1/2},
 *                 lower =  sqrt((l - m_j + 1/2)/(2l+1)) Y_l^{m_j+1/2},
 *   j = l - 1/2:  upper = -sqrt((l - m_j + 1/2)/(2l+1)) Y_l^{m_j-1/2},
 *                 lower =  sqrt((l + m_j + 1/2)/(2l+1)) Y_l^{m_j+1/2},
 * with Y_l^m = 0 for |m| > l.  Spinors are numbered l-major, j = l - 1/2 before
 * j = l + 1/2, m_j ascending: k = 2l^2 + (m_j + l - 1/2) for j = l - 1/2 and
 * k = 2l^2 + 2l + (m_j + l + 1/2) for j = l + 1/2, so there are 2 (lmax+1)^2 of
 * them.  out is [2 (lmax+1)^2][2][n] complex values, (re, im) pairs, component
 * 0 the upper (spin-up) one: 4 (lmax+1)^2 n complex values in all.  Arguments,
 * validation and origin convention as sh_eval_complex. */
int sh_eval_spinor(int lmax, int64_t n, const double *xyz, double *out, hipStream_t stream);
int sh_eval_spinor_f32(int lmax, int64_t n, const float *xyz, float *out, hipStream_t stream);

/* Spinor harmonics from any input interface, as sh_eval_complex_in. */
int sh_eval_spinor_in(int lmax, int64_t n, int input, int dtype, const void *in0, const void *in1, void *out,
                      hipStream_t stream);

/* Backward pass of sh_eval (vector-Jacobian product), for forces:
 *   grad_xyz[i][k] = sum_{row} grad_out[row][i] * d R_row(x_i) / d x_{i,k}
 * with xyz [n][3], grad_out [F][n] and grad_xyz [n][3], all double.  The
 * derivative is that of the unit-vector formulas composed with the
 * normalisation u = x / |x|: (1/r) (I - u u^T) grad_u.  At r = 0 the gradient
 * is defined as 0.  grad_xyz is overwritten (not accumulated). */
int sh_eval_grad(int lmax, int64_t n, const double *xyz, const double *grad_out, double *grad_xyz,
                 hipStream_t stream);

/* Single-precision twin of sh_eval_grad: float xyz, grad_out and grad_xyz; the
 * normalisation and 1/r in FP64, the polynomial gradients and the contraction
 * over rows in FP32. */
int sh_eval_grad_f32(int lmax, int64_t n, const float *xyz, const float *grad_out, float *grad_xyz,
                     hipStream_t stream);

/* Backward pass of sh_eval_rec / sh_eval_rec_f32 for 0 <= lmax <= SH_LMAX_REC:
 * arguments, convention and origin as sh_eval_grad (sh_eval_grad_f32), with
 * grad_out [(lmax+1)^2][n].  The gradient differentiates the recurrence in z and
 * the xy factors in closed form; per point |error|_inf <= 1e-12 (1 + |g|_inf) in
 * FP64 and 5e-6 (lmax + 1) (1 + |g|_inf) in FP32 (2e-5 for lmax <= 9). */
int sh_eval_grad_rec(int lmax, int64_t n, const double *xyz, const double *grad_out, double *grad_xyz,
                     hipStream_t stream);
int sh_eval_grad_rec_f32(int lmax, int64_t n, const float *xyz, const float *grad_out, float *grad_xyz,
                         hipStream_t stream);

/* Values and their Cartesian Jacobian in one pass, for forces:
 *   out [F][n]      R_row(x_i)
 *   jac [3][F][n]   d R_row(x_i) / d x_{i,k} at jac[(k * F + row) * n + i]
 * (double).  Same derivative convention as sh_eval_grad; 0 at the origin. */
int sh_eval_jac(int lmax, int64_t n, const double *xyz, double *out, double *jac, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Projector build.  The paper's motivating use (Section 1): the angular part of
 * pseudopotential / PAW projectors on a real-space grid.  For atom a with centre
 * c_a and grid points p_j, the projector value is
 *     out_a[row(l,m)][j] = R_l(|d_j|) * R_l^m(d_j / |d_j|),   d_j = p_j - c_a,
 * where the radial function R_l is a natural cubic spline through values on a
 * uniform radial grid and is 0 beyond the grid's last knot r_max.
 */
typedef struct sh_radial *sh_radial_t;

/* Radial tables: host_values is a HOST array [n_tables][lmax+1][n_r] of R_l at
 * the knots r_i = i * r_max / (n_r - 1).  The library copies them to the device
 * and solves the natural-spline second derivatives there (on a private stream;
 * the call returns when the tables are ready).  The handle owns device memory
 * until sh_radial_destroy: the (y, M) pairs in double, 16 bytes per knot and
 * channel, and a float copy of them for the FP32 kernels, 8 bytes more.  SH_EINVAL
 * for lmax outside [0, 9], n_tables < 1,
 * n_r < 2, r_max not positive and finite, or NULL pointers; SH_ENOMEM when the
 * device allocation fails. */
int sh_radial_create(int lmax, int n_tables, int n_r, double r_max, const double *host_values,
                     sh_radial_t *out);

/* Frees a handle (NULL is a no-op).  No call using it may still be running. */
int sh_radial_destroy(sh_radial_t radial);

/* Projector arrays for n_atoms atoms whose grid points are concatenated:
 *   centers        [n_atoms][3]        device
 *   offsets        [n_atoms + 1] int64 device, CSR: atom a owns points
 *                  offsets[a] .. offsets[a+1]-1; offsets[0] = 0,
 *                  offsets[n_atoms] = n_points, nondecreasing
 *   n_points       host value, the total number of points
 *   points         [n_points][3]       device, absolute coordinates (periodic
 *                  images already unwrapped by the caller)
 *   radial         tables with lmax(radial) >= lmax
 *   table_of_atom  [n_atoms] int32 device: table used by atom a (clamped to
 *                  [0, n_tables-1]); NULL means atom a uses table a
 *   out            [F * n_points] device: atom a's block [F][n_a] starts at
 *                  out + F * offsets[a] (row stride n_a = its point count)
 * Device-side arrays are not validated by the host; a point whose offsets are
 * inconsistent is skipped (nothing is written for it), so no store leaves out. */
int sh_projectors(int lmax, int n_atoms, const double *centers, const int64_t *offsets, int64_t n_points,
                  const double *points, sh_radial_t radial, const int32_t *table_of_atom, double *out,
                  hipStream_t stream);

/* Single-precision twin: float centers, points and out.  d = p - c, |d|, the
 * normalisation and the spline's interval run in FP64; the spline's cubic (from
 * float copies of the tables the handle keeps), the harmonics and the product in
 * FP32.  Same 5e-6 bound as sh_eval_f32 (times max(1, max|R_l|)). */
int sh_projectors_f32(int lmax, int n_atoms, const float *centers, const int64_t *offsets, int64_t n_points,
                      const float *points, sh_radial_t radial, const int32_t *table_of_atom, float *out,
                      hipStream_t stream);

/* ---------------------------------------------------------------------------
 * For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation: the projector
 * build of sh_projectors / sh_projectors_f32 with the radial functions given as
 * their knot values instead of a handle, allocating nothing.
 *   dtype          SH_F64 or SH_F32: the type of centers, points and out
 *   n_tables, n_r, r_max, values
 *                  DEVICE array [n_tables][lmax+1][n_r] of double: R_l at the
 *                  knots r_i = i r_max / (n_r - 1) (the layout sh_radial_create
 *                  takes, with lmax + 1 channels per table)
 *   other arguments as sh_projectors (centers, offsets, points, table_of_atom
 *                  and out DEVICE; table_of_atom NULL means atom a uses table a).
 * The natural-spline set-up of sh_radial_create runs on `stream` before the
 * build, with its working arrays (the tables' (y, M) pairs, their float copy and
 * the solve's coefficients) in a buffer the library keeps in static device memory:
 * 64 MiB on every GPU it runs on, held until the process ends.  The results are
 * the same, bit for bit, as sh_radial_create of the same values followed by
 * sh_projectors (or _f32).  SH_EINVAL, with nothing launched, for the argument
 * errors of sh_projectors and sh_radial_create and when n_tables (lmax + 1) n_r
 * exceeds SH_NOALLOC_MAX_VALUES.  Calls that overlap on one GPU (concurrent
 * streams or threads) share that buffer and race; order them on one stream.  The
 * buffer keeps the last call's contents, which no call relies on. */
#define SH_NOALLOC_MAX_VALUES (1 << 21)
int sh_projectors_noalloc(int lmax, int dtype, int n_atoms, const void *centers, const int64_t *offsets,
                          int64_t n_points, const void *points, int n_tables, int n_r, double r_max,
                          const double *values, const int32_t *table_of_atom, void *out, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of projector requests of uneven lmax, point
 * count and dtype.  Atoms (device point sets with a centre and a radial table)
 * are registered once and stay on the device.  Each request asks for the
 * projectors of one atom up to some lmax.  A scheduler thread admits pending
 * requests in arrival order while their output fits in an HBM budget (carved
 * from one device allocation made at creation), packs all admitted requests into
 * one batch and launches it on a free stream slot (one kernel per (dtype, lmax)
 * group of the batch; the small groups of a batch may share one), so requests
 * that arrive while others run are admitted as memory and slots free up and their
 * work overlaps on the device.  Results stay on the device until released.
 * Within a batch the launches run smallest output first and each request
 * completes when its launch does.  A request's latency is measured from
 * sh_server_submit to the host seeing its launch complete.  Creation also runs
 * every serving kernel once on an empty request, so that no first launch (which
 * is slow) falls in the middle of serving.  Every function is thread-safe.
 */
typedef struct sh_server *sh_server_t;

#define SH_REQ_AUTORELEASE 1 /* free the output as soon as it is complete (no result) */

enum sh_req_state {
    SH_REQ_PENDING = 0,  /* waiting for budget */
    SH_REQ_QUEUED = 1,   /* admitted, output allocated, not yet launched */
    SH_REQ_RUNNING = 2,  /* in a launched batch */
    SH_REQ_DONE = 3,     /* result available */
    SH_REQ_FAILED = 4,   /* its batch failed, or the server shut down first */
    SH_REQ_RELEASED = 5  /* output returned to the budget */
};

typedef struct {
    int64_t submitted, completed, failed;
    int64_t deferred; /* admitted requests that had waited while the budget was full */
    int64_t batches;
    int64_t points_done;
    uint64_t bytes_in_use, peak_bytes;  /* output bytes admitted (arena) */
    double first_submit_s, last_done_s; /* seconds since creation; -1 before the first submit */
    double scheduler_cpu_s;             /* CPU time used by the scheduler thread (-1 if unknown) */
} sh_server_stats_t;

/* A server with an HBM budget of budget_bytes (allocated now), at most
 * max_pending requests waiting for admission (more: SH_EBUSY) and n_slots
 * batches in flight (1..16, one stream each). */
int sh_server_create(uint64_t budget_bytes, int max_pending, int n_slots, sh_server_t *out);

/* The same scheduler with a simulated executor that computes nothing: a launch
 * takes launch_seconds of host time (0 to 10), a batch completes after its output
 * bytes at bytes_per_second, and every fail_every-th launch (0: never) fails.
 * For testing the scheduling logic without a GPU; results are not readable
 * (their addresses are arena offsets). */
int sh_server_create_simulated(uint64_t budget_bytes, int max_pending, int n_slots, double bytes_per_second,
                               int fail_every, double launch_seconds, sh_server_t *out);

/* Refuses new work, fails what was not launched, waits for running batches,
 * then frees everything (NULL is a no-op). */
int sh_server_destroy(sh_server_t srv);

/* Registers an atom: n points [n][3] of dtype (device, owned by the caller and
 * kept valid while the server may use them), centre (host, 3 doubles), table
 * `table` of `radial` (NULL only for simulated servers).  SH_EINVAL if n is not
 * positive or exceeds 256 * (2^24 - 1) (a batch is one dispatch, whose grid of
 * 256-point tiles must stay below 2^32 work-items). */
int sh_server_add_atom(sh_server_t srv, int dtype, int64_t n, const void *points, const double *center,
                       sh_radial_t radial, int table, int *atom_id);

/* Enqueues "projectors of atom_id up to lmax" (output [F][n] of the atom's
 * dtype).  SH_EBUSY when max_pending requests already wait; SH_EINVAL when the
 * output could never fit the budget or lmax exceeds the atom's table. */
int sh_server_submit(sh_server_t srv, int atom_id, int lmax, int flags, int64_t *ticket);

/* Current state (enum sh_req_state) of a request. */
int sh_server_poll(sh_server_t srv, int64_t ticket, int *state);

/* Waits up to timeout_s seconds for DONE/FAILED/RELEASED; SH_EBUSY on timeout. */
int sh_server_wait(sh_server_t srv, int64_t ticket, double timeout_s, int *state);

/* Device address of a DONE request's [F][n] output (valid until released).
 * SH_EBUSY while the request has not finished. */
int sh_server_result(sh_server_t srv, int64_t ticket, void **out);

/* Returns a finished request's output to the budget (SH_EBUSY if not finished).
 * The server may hand that memory to the next request's kernel as soon as this
 * returns, on its own streams: GPU work of the caller that reads the output must
 * have completed before the call (synchronise the stream it was queued on). */
int sh_server_release(sh_server_t srv, int64_t ticket);

/* Waits until nothing is pending, queued or running; SH_EBUSY on timeout. */
int sh_server_drain(sh_server_t srv, double timeout_s);

int sh_server_stats(sh_server_t srv, sh_server_stats_t *out);

/* Copies up to cap completed-request latencies (ms, completion order) into
 * out_ms (may be NULL) and returns how many there are (negative on error). */
int64_t sh_server_latencies(sh_server_t srv, double *out_ms, int64_t cap);

/* Static text for a status code (never NULL). */
const char *sh_strerror(int code);

/* The last hipError_t seen by this thread inside the library (0 if none). */
int sh_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SHMI_H */
