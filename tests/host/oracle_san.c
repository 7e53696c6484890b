/* oracle_san.c -- calls every entry point of the C oracle on small inputs that
 * include its special cases (the origin, poles, a NaN point, points beyond the
 * radial cutoff, empty atoms), for the address and undefined-behaviour sanitizer
 * build.  The values themselves are pinned by the Python tests; this checks
 * memory safety and prints OK with a few closed-form values. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef long double ld;
int orc_eval_xyz(int lmax, int64_t n, const double *xyz, ld *out);
int orc_eval_xyz_f32(int lmax, int64_t n, const float *xyz, ld *out);
int orc_eval_angles(int lmax, int64_t n, const ld *theta, const ld *phi, ld *out);
int orc_eval_complex_xyz(int lmax, int64_t n, const double *xyz, ld *re, ld *im);
int orc_eval_complex_angles(int lmax, int64_t n, const ld *theta, const ld *phi, ld *re, ld *im);
int orc_jacobian_xyz(int lmax, int64_t n, const double *xyz, ld *jac);
int orc_grad_xyz(int lmax, int64_t n, const double *xyz, const double *G, ld *gxyz);
int orc_spline_setup(int n_r, double r_max, const double *y, ld *M);
int orc_spline_eval(int n_r, double r_max, const double *y, const ld *M, int64_t n, const ld *r, ld *out);
int orc_projectors(int lmax, int n_atoms, const double *centers, const int64_t *offsets, const double *points,
                   const int *table_of_atom, int n_r, double r_max, const double *tables, const ld *Ms, ld *out);
int orc_lmax_limit(void);

int main(void)
{
    const double pts[] = {0, 0, 0,  0, 0, 2,  0, 0, -1,  1, 0, 0,  0.3, -0.4, 0.5,  NAN, 1, 1,  1e-200, 0, 0};
    const int n = 7, L = orc_lmax_limit();
    const int F = (L + 1) * (L + 1);
    ld *out = calloc((size_t)F * n, sizeof(ld)), *re = calloc((size_t)F * n, sizeof(ld)),
       *im = calloc((size_t)F * n, sizeof(ld)), *jac = calloc((size_t)3 * F * n, sizeof(ld)),
       *g = calloc((size_t)3 * n, sizeof(ld));
    double *G = calloc((size_t)F * n, sizeof(double));
    float p32[21];
    for (int k = 0; k < 21; ++k) p32[k] = (float)pts[k];
    for (int k = 0; k < F * n; ++k) G[k] = sin(0.1 * k);
    int rc = 0;
    rc |= orc_eval_xyz(L, n, pts, out);
    const ld y00 = out[0];
    rc |= orc_eval_xyz_f32(9, n, p32, out);
    ld th[3] = {0.0L, 1.0L, 3.141592653589793L}, ph[3] = {0.0L, 2.0L, -1.0L};
    rc |= orc_eval_angles(L, 3, th, ph, out);
    rc |= orc_eval_complex_xyz(L, n, pts, re, im);
    rc |= orc_eval_complex_angles(L, 3, th, ph, re, im);
    rc |= orc_jacobian_xyz(9, n, pts, jac);
    rc |= orc_grad_xyz(L, n, pts, G, g);
    /* spline on 50 knots and evaluation inside, at the ends and beyond r_max */
    double y[50];
    ld M[50], r[5] = {0.0L, 0.37L, 1.5L, 2.0L, 2.5L}, s[5];
    for (int k = 0; k < 50; ++k) y[k] = cos(0.1 * k);
    rc |= orc_spline_setup(50, 2.0, y, M);
    rc |= orc_spline_eval(50, 2.0, y, M, 5, r, s);
    /* projectors: three atoms, the middle one empty, a shared table */
    const double cen[] = {0, 0, 0,  5, 5, 5,  1, 1, 1};
    const int64_t off[] = {0, 4, 4, n};
    double tabs[2 * 4 * 50];
    ld Ms[2 * 4 * 50];
    for (int k = 0; k < 2 * 4 * 50; ++k) tabs[k] = cos(0.05 * k);
    for (int c = 0; c < 2 * 4; ++c) rc |= orc_spline_setup(50, 2.0, tabs + 50 * c, Ms + 50 * c);
    const int toa[] = {1, 0, 1};
    ld *pr = calloc((size_t)16 * n, sizeof(ld));
    rc |= orc_projectors(3, 3, cen, off, pts, toa, 50, 2.0, tabs, Ms, pr);
    printf("R_0^0 at the origin %.18Lf (1/sqrt(4 pi) = %.18f), spline at 0: %.6Lf (y0 %.6f)\n", y00,
           1.0 / sqrt(4 * 3.14159265358979323846), s[0], y[0]);
    free(out); free(re); free(im); free(jac); free(g); free(G); free(pr);
    if (rc) {
        printf("FAILED rc=%d\n", rc);
        return 1;
    }
    printf("OK\n");
    return 0;
}
