// Test-only: host build of the GPU formula core (sh_core.h), so the factorised
// formulas and their constants can be checked on the CPU against the oracle.
// Inputs are unit vectors; the kernels' FP64 normalisation is not part of this.
// Also the radial spline (sh_proj.h) in the device table layout.
#include <vector>

#include "../../paper_2510_05282_amd/csrc/sh_core.h"

template <int LMAX, typename T>
static void run(long n, const T *u, T *out)
{
    for (long i = 0; i < n; ++i)
        shk::eval_unit<LMAX, T>(u[3 * i], u[3 * i + 1], u[3 * i + 2], T(1),
                                [&](int r, T v) { out[r * n + i] = v; });
}

extern "C" void core_eval9_f64(long n, const double *u, double *out) { run<9, double>(n, u, out); }
extern "C" void core_eval9_f32(long n, const float *u, float *out) { run<9, float>(n, u, out); }
extern "C" void core_eval3_f64(long n, const double *u, double *out) { run<3, double>(n, u, out); }

#include "../../paper_2510_05282_amd/csrc/sh_dual.h"

// Tangential gradient at unit vectors u (r = 1): g = v - u (u . v).
template <int LMAX>
static void grad(long n, const double *u, const double *G, double *out)
{
    for (long i = 0; i < n; ++i) {
        double vx, vy, vz;
        shk::grad_unit<LMAX>(u[3 * i], u[3 * i + 1], u[3 * i + 2],
                             [&](int r) { return G[r * n + i]; }, vx, vy, vz);
        const double uv = u[3 * i] * vx + u[3 * i + 1] * vy + u[3 * i + 2] * vz;
        out[3 * i] = vx - u[3 * i] * uv;
        out[3 * i + 1] = vy - u[3 * i + 1] * uv;
        out[3 * i + 2] = vz - u[3 * i + 2] * uv;
    }
}

extern "C" void core_grad9(long n, const double *u, const double *G, double *out) { grad<9>(n, u, G, out); }
extern "C" void core_grad6(long n, const double *u, const double *G, double *out) { grad<6>(n, u, G, out); }

// FP32 gradient core at float unit vectors.
extern "C" void core_grad9_f32(long n, const float *u, const float *G, float *out)
{
    for (long i = 0; i < n; ++i) {
        float vx, vy, vz;
        shk::grad_unit<9>(u[3 * i], u[3 * i + 1], u[3 * i + 2], [&](int r) { return G[r * n + i]; }, vx, vy, vz);
        const float uv = u[3 * i] * vx + u[3 * i + 1] * vy + u[3 * i + 2] * vz;
        out[3 * i] = vx - u[3 * i] * uv;
        out[3 * i + 1] = vy - u[3 * i + 1] * uv;
        out[3 * i + 2] = vz - u[3 * i + 2] * uv;
    }
}

// Values and projected Jacobian at unit vectors (r = 1): val[F][n], jac[3][F][n].
extern "C" void core_jac9(long n, const double *u, double *val, double *jac)
{
    const int F = 100;
    for (long i = 0; i < n; ++i) {
        const double x = u[3 * i], y = u[3 * i + 1], z = u[3 * i + 2];
        shk::eval_unit_jac<9, double>(x, y, z, 1.0, [&](int f, double v, double gx, double gy, double gz) {
            const double ug = x * gx + y * gy + z * gz;
            val[f * n + i] = v;
            jac[(0 * F + f) * n + i] = gx - x * ug;
            jac[(1 * F + f) * n + i] = gy - y * ug;
            jac[(2 * F + f) * n + i] = gz - z * ug;
        });
    }
}

#include "../../paper_2510_05282_amd/csrc/sh_rec.h"

// Recurrence core at unit vectors: out[(lmax+1)^2][n].
extern "C" void core_rec(long n, const double *u, int lmax, double *out)
{
    for (long i = 0; i < n; ++i)
        shk::eval_unit_rec<double>(u[3 * i], u[3 * i + 1], u[3 * i + 2], 1.0, lmax,
                                   [&](int l, int m, double v) { out[shk::row(l, m) * n + i] = v; });
}

// Complex and spinor cores at unit vectors: (re, im) pairs, out[rows][n][2] with
// rows = (lmax+1)^2 complex values, or 2 (lmax+1)^2 spinors x 2 components.
// Every entry of `out` must be written once: the caller fills it with NaN first.
extern "C" void core_complex9(long n, const double *u, double *out)
{
    for (long i = 0; i < n; ++i)
        shk::complex_unit<9, double>(u[3 * i], u[3 * i + 1], u[3 * i + 2], 1.0,
                                     [&](int l, int m, double re, double im) {
                                         double *o = out + 2 * (long(shk::row(l, m)) * n + i);
                                         o[0] = re;
                                         o[1] = im;
                                     });
}

template <int LMAX>
static void spinor(long n, const double *u, double *out, int *count)
{
    for (long i = 0; i < n; ++i)
        shk::spinor_unit<LMAX, double>(u[3 * i], u[3 * i + 1], u[3 * i + 2], 1.0,
                                       [&](int k, int c, double re, double im) {
                                           const long e = (long(2 * k + c) * n + i);
                                           out[2 * e] = re;
                                           out[2 * e + 1] = im;
                                           count[e] += 1;
                                       });
}

extern "C" void core_spinor(long n, const double *u, int lmax, double *out, int *count)
{
    switch (lmax) {
    case 0: spinor<0>(n, u, out, count); break;
    case 1: spinor<1>(n, u, out, count); break;
    case 4: spinor<4>(n, u, out, count); break;
    case 9: spinor<9>(n, u, out, count); break;
    default: break;
    }
}

#include "../../paper_2510_05282_amd/csrc/sh_proj.h"

// Radial tables in the device layout: y[n_tables][4][n_r] -> interleaved
// [n_tables][n_r][4] (y, M) by spline_solve, then R_0..R_3 of table t at r[k]:
// out[k][4].
// With f32 != 0 the pairs are rounded to float and evaluated by the FP32 lookup
// the FP32 kernels use.
extern "C" void core_spline4(int n_tables, int n_r, double r_max, const double *y, int t, long n, const double *r,
                             double *out, int f32)
{
    const int ch = 4;
    const double h = r_max / double(n_r - 1);
    std::vector<double2> tab(size_t(n_tables) * n_r * ch);
    std::vector<double> cc(n_r);
    for (int c = 0; c < n_tables * ch; ++c)
        shk::spline_solve(y + long(c) * n_r, tab.data() + long(c / ch) * n_r * ch + c % ch, ch, cc.data(), n_r,
                          6.0 / (h * h));
    std::vector<float2> tabf(tab.size());
    for (size_t k = 0; k < tab.size(); ++k) tabf[k] = make_float2(float(tab[k].x), float(tab[k].y));
    const shk::SplineGrid g{n_r, h, 1.0 / h, r_max, h * h / 6.0};
    for (long k = 0; k < n; ++k) {
        if (f32) {
            float R[4];
            shk::spline_eval<4, float>(tabf.data() + long(t) * n_r * ch, ch, g, r[k], R);
            for (int l = 0; l < 4; ++l) out[4 * k + l] = R[l];
        } else {
            double R[4];
            shk::spline_eval<4, double>(tab.data() + long(t) * n_r * ch, ch, g, r[k], R);
            for (int l = 0; l < 4; ++l) out[4 * k + l] = R[l];
        }
    }
}

// FP32 recurrence core at float unit vectors: out[(lmax+1)^2][n].
extern "C" void core_rec_f32(long n, const float *u, int lmax, float *out)
{
    for (long i = 0; i < n; ++i)
        shk::eval_unit_rec<float>(u[3 * i], u[3 * i + 1], u[3 * i + 2], 1.0f, lmax,
                                  [&](int l, int m, float v) { out[shk::row(l, m) * n + i] = v; });
}

// Complex and spinor harmonics by recurrence at unit vectors (any lmax <= 24):
// complex out[F][n][2]; spinor out[S][2][n][2] with a write count per entry.
extern "C" void core_complex_rec(long n, const double *u, int lmax, double *out)
{
    for (long i = 0; i < n; ++i)
        shk::complex_unit_rec<double>(u[3 * i], u[3 * i + 1], u[3 * i + 2], 1.0, lmax,
                                      [&](int l, int m, double re, double im) {
                                          double *o = out + 2 * (long(shk::row(l, m)) * n + i);
                                          o[0] = re;
                                          o[1] = im;
                                      });
}

extern "C" void core_spinor_rec(long n, const double *u, int lmax, double *out, int *count)
{
    for (long i = 0; i < n; ++i)
        shk::spinor_unit_rec<double>(u[3 * i], u[3 * i + 1], u[3 * i + 2], 1.0, lmax,
                                     [&](int k, int c, double re, double im) {
                                         const long e = long(2 * k + c) * n + i;
                                         out[2 * e] = re;
                                         out[2 * e + 1] = im;
                                         count[e] += 1;
                                     });
}

// Backward by recurrence at unit vectors (r = 1): out[n][3] = (I - u u^T) v.
template <typename T>
static void grad_rec(long n, const T *u, int lmax, const T *G, T *out)
{
    for (long i = 0; i < n; ++i) {
        T v[3];
        shk::grad_unit_rec<T>(u[3 * i], u[3 * i + 1], u[3 * i + 2], lmax,
                              [&](int r) { return G[long(r) * n + i]; }, v[0], v[1], v[2]);
        const T uv = u[3 * i] * v[0] + u[3 * i + 1] * v[1] + u[3 * i + 2] * v[2];
        for (int q = 0; q < 3; ++q) out[3 * i + q] = v[q] - u[3 * i + q] * uv;
    }
}

extern "C" void core_grad_rec(long n, const double *u, int lmax, const double *G, double *out)
{
    grad_rec<double>(n, u, lmax, G, out);
}

extern "C" void core_grad_rec_f32(long n, const float *u, int lmax, const float *G, float *out)
{
    grad_rec<float>(n, u, lmax, G, out);
}
