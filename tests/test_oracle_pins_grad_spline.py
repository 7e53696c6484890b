"""Pins of the oracle's gradient, radial spline and projector build."""
from __future__ import annotations

import math

import mpmath as mp
import numpy as np

from paper_2510_05282_amd import workloads

LD = np.longdouble
PI_LD = LD("3.14159265358979323846264338327950288")


def _grid_points(n, seed, r_lo=1.0, r_hi=3.0):
    """Random points rounded to multiples of 2^-20 so that +-k 2^-16 steps are exact."""
    p = workloads.isotropic_points(n, r_lo, r_hi, seed=seed)
    return np.round(p * 2.0**20) / 2.0**20


def test_jacobian_vs_central_differences(orc):
    """Fourth-order central differences of the oracle's forward values (steps are
    exact in double; sums in long double) against the analytic Jacobian."""
    lmax = 9
    pts = _grid_points(40, seed=21)
    J = orc.jacobian_xyz(lmax, pts)
    h = 2.0**-16
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        f = {s: orc.eval_xyz(lmax, pts + s * e) for s in (-2, -1, 1, 2)}
        fd = (-f[2] + 8 * f[1] - 8 * f[-1] + f[-2]) / (12 * LD(h))
        assert np.abs(fd - J[k]).max() <= 1e-12


def test_gradient_sum_rule_and_euler(orc):
    """r^2 sum_m |grad R_l^m|^2 = l(l+1)(2l+1)/(4 pi) and r . grad R = 0."""
    pts = np.concatenate([workloads.isotropic_points(500, 0.1, 5, seed=22),
                          np.array([[0, 0, 2.0], [0, 0, -1.0], [1e-9, 0, 1], [3.0, 0, 0]])])
    J = orc.jacobian_xyz(9, pts)
    r2 = (pts.astype(LD) ** 2).sum(1)
    for l in range(10):
        sl = slice(l * l, (l + 1) * (l + 1))
        s = r2 * (J[:, sl] ** 2).sum(axis=(0, 1))
        ref = LD(l * (l + 1) * (2 * l + 1)) / (4 * PI_LD)
        assert (np.abs(s - ref)).max() <= 1e-16 * max(1.0, float(ref))
    euler = (J * pts.T.astype(LD)[:, None, :]).sum(0)
    assert np.abs(euler).max() <= 1e-16


def test_jacobian_brute_force_mpmath(orc):
    """mpmath numerical differentiation (40 digits) of the definition: the real
    harmonic from mpmath's complex Y (eq. real_harmomics) of the Cartesian point."""
    mp.mp.dps = 40

    def real_y(l, m, x, y, z):
        r = mp.sqrt(x * x + y * y + z * z)
        th, ph = mp.acos(z / r), mp.atan2(y, x)
        if m == 0:
            return mp.re(mp.spherharm(l, 0, th, ph))
        if m < 0:
            return mp.re(1j / mp.sqrt(2) * (mp.spherharm(l, m, th, ph)
                                            - (-1) ** m * mp.spherharm(l, -m, th, ph)))
        return mp.re(1 / mp.sqrt(2) * (mp.spherharm(l, -m, th, ph)
                                       + (-1) ** m * mp.spherharm(l, m, th, ph)))

    pts = np.array([[0.3, -1.1, 0.7], [-1.5, 0.25, -0.4]])
    J = orc.jacobian_xyz(6, pts)
    for i, (x, y, z) in enumerate(pts):
        X, Y, Z = mp.mpf(x), mp.mpf(y), mp.mpf(z)
        for l in (1, 4, 6):
            for m in range(-l, l + 1):
                row = l * l + l + m
                d = [mp.diff(lambda t: real_y(l, m, t, Y, Z), X),
                     mp.diff(lambda t: real_y(l, m, X, t, Z), Y),
                     mp.diff(lambda t: real_y(l, m, X, Y, t), Z)]
                for k in range(3):
                    assert abs(float(d[k]) - float(J[k, row, i])) <= 1e-16 * (1 + abs(float(d[k])))


def test_gradient_contraction_and_origin(orc):
    pts = np.concatenate([workloads.isotropic_points(50, 0.5, 5, seed=23), np.zeros((1, 3))])
    G = np.random.default_rng(24).standard_normal((49, pts.shape[0]))
    g = orc.grad_xyz(6, pts, G)
    J = orc.jacobian_xyz(6, pts)
    ref = np.einsum("fi,kfi->ik", G.astype(LD), J)
    assert np.abs(g - ref).max() <= 1e-16
    assert np.all(g[-1] == 0)


# ---------------------------------------------------------------- spline


def test_spline_interpolates_knots_and_linear(orc):
    y = np.random.default_rng(25).standard_normal(50)
    M = orc.spline_setup(y, 3.0)
    r = np.arange(50, dtype=LD) * (LD(3.0) / LD(49))  # knots, formed in long double
    assert np.abs(orc.spline_eval(y, M, 3.0, r) - y.astype(LD)).max() <= 1e-16
    lin = 0.7 - 1.3 * np.linspace(0, 3.0, 50)
    Ml = orc.spline_setup(lin, 3.0)
    assert np.abs(Ml).max() <= 1e-12  # rounding noise of the y values over h^2
    rr = np.random.default_rng(26).uniform(0, 3.0, 1000).astype(LD)
    assert np.abs(orc.spline_eval(lin, Ml, 3.0, rr) - (LD(0.7) - LD(1.3) * rr)).max() <= 1e-15
    assert np.all(orc.spline_eval(y, M, 3.0, np.array([3.0000001, 10.0])) == 0)


def test_spline_matches_scipy_natural(orc):
    """Library routine: scipy's natural cubic spline through the same knots."""
    from scipy.interpolate import CubicSpline
    rng = np.random.default_rng(27)
    tab = workloads.radial_table(rng, 3, n_r=2000, r_max=3.0)
    knots = np.linspace(0, 3.0, 2000)
    rr = rng.uniform(0, 3.0, 5000)
    for l in range(4):
        M = orc.spline_setup(tab[l], 3.0)
        ref = CubicSpline(knots, tab[l], bc_type="natural")(rr)
        got = orc.spline_eval(tab[l], M, 3.0, rr).astype(np.float64)
        assert np.abs(got - ref).max() <= 1e-13


# ---------------------------------------------------------------- projector


def test_projector_unit_radial_reduces_to_eval(orc):
    """R_l = 1 everywhere: the projector is the plain harmonic of p - c."""
    A = workloads.atom_spheres(seed=3, n_atoms=3, box=20.0, radius=1.0, h=0.25, lmax=3, n_r=64)
    ones = np.ones_like(A.tables)
    out = orc.projectors(3, A.centers, A.offsets, A.points, ones, A.r_max)
    for a in range(3):
        j0, j1 = A.offsets[a], A.offsets[a + 1]
        d = A.points[j0:j1] - A.centers[a]
        ref = orc.eval_xyz(3, d)
        got = out[16 * j0:16 * j1].reshape(16, j1 - j0)
        assert np.abs(got - ref).max() <= 1e-18


def test_projector_brute_force(orc):
    """A few projector values from scipy's natural spline times the real harmonic
    built from mpmath's complex Y (eq. real_harmomics)."""
    from scipy.interpolate import CubicSpline
    mp.mp.dps = 30
    A = workloads.atom_spheres(seed=4, n_atoms=2, box=20.0, radius=3.0, h=0.5, lmax=3, n_r=2000)
    out = orc.projectors(3, A.centers, A.offsets, A.points, A.tables, A.r_max)
    knots = np.linspace(0, A.r_max, A.tables.shape[2])
    rng = np.random.default_rng(5)
    for a in range(2):
        j0, j1 = int(A.offsets[a]), int(A.offsets[a + 1])
        na = j1 - j0
        block = out[16 * j0:16 * j1].reshape(16, na)
        for j in rng.integers(0, na, 5):
            d = A.points[j0 + j] - A.centers[a]
            r = math.sqrt(float((d * d).sum()))
            X, Y, Z = (mp.mpf(float(v)) for v in d)
            th, ph = mp.acos(Z / mp.sqrt(X * X + Y * Y + Z * Z)), mp.atan2(Y, X)
            for l in range(4):
                R = CubicSpline(knots, A.tables[a, l], bc_type="natural")(r)
                for m in range(-l, l + 1):
                    if m == 0:
                        yv = mp.re(mp.spherharm(l, 0, th, ph))
                    elif m < 0:
                        yv = mp.re(1j / mp.sqrt(2) * (mp.spherharm(l, m, th, ph)
                                                      - (-1) ** m * mp.spherharm(l, -m, th, ph)))
                    else:
                        yv = mp.re(1 / mp.sqrt(2) * (mp.spherharm(l, -m, th, ph)
                                                     + (-1) ** m * mp.spherharm(l, m, th, ph)))
                    assert abs(float(block[l * l + l + m, j]) - R * float(yv)) <= 1e-13


def test_gradient_high_l_sum_rule_euler_and_differences(orc):
    """The oracle's Jacobian up to l = 24 (beyond the explicit formulas): the sum
    rule r^2 sum_m |grad R_l^m|^2 = l(l+1)(2l+1)/(4 pi), Euler's relation, and
    fourth-order central differences of its own forward values."""
    lmax = 24
    pts = np.concatenate([workloads.isotropic_points(200, 0.5, 3, seed=28), np.array([[0, 0, 2.0], [1e-7, 0, 1]])])
    J = orc.jacobian_xyz(lmax, pts)
    r2 = (pts.astype(LD) ** 2).sum(1)
    for l in range(lmax + 1):
        sl = slice(l * l, (l + 1) * (l + 1))
        s = r2 * (J[:, sl] ** 2).sum(axis=(0, 1))
        ref = LD(l * (l + 1) * (2 * l + 1)) / (4 * PI_LD)
        assert np.abs(s - ref).max() <= 1e-15 * max(1.0, float(ref)), l
    assert np.abs((J * pts.T.astype(LD)[:, None, :]).sum(0)).max() <= 1e-15
    h = 2.0**-18
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        f = {s: orc.eval_xyz(lmax, pts + s * e) for s in (-2, -1, 1, 2)}
        fd = (-f[2] + 8 * f[1] - 8 * f[-1] + f[-2]) / (12 * LD(h))
        assert np.abs(fd - J[k]).max() <= 1e-9
