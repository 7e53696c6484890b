// Test-only: host build of the GPU formula core (sh_core.h), so the factorised
// formulas and their constants can be checked on the CPU against the oracle.
// Inputs are unit vectors; the kernels' FP64 normalisation is not part of this.
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
