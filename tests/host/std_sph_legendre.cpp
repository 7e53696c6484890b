// Test-only: the C++17 standard library's std::sph_legendre(l, m, theta), which
// is Y_l^m(theta, 0) with the Condon-Shortley phase, for a batch of angles.
// An independent library routine that pins the oracle's Legendre functions.
#include <cmath>

extern "C" void std_sph_legendre(int lmax, long n, const double *theta, double *out)
{
    for (int l = 0; l <= lmax; ++l)
        for (int m = 0; m <= l; ++m)
            for (long i = 0; i < n; ++i)
                out[((long)(l * (l + 1) / 2 + m)) * n + i] =
                    std::sph_legendre((unsigned)l, (unsigned)m, theta[i]);
}
