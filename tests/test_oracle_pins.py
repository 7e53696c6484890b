"""Pins of the CPU oracle against values the paper and the mathematics fix.

Nothing here compares the oracle with itself: each check uses printed values,
closed forms, invariants, library routines or arbitrary-precision brute force.
"""
from __future__ import annotations

import math
import os

import mpmath as mp
import numpy as np
import pytest

from paper_2510_05282_amd import workloads
from tests import appc_forms

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
LD = np.longdouble
PI_LD = LD("3.14159265358979323846264338327950288")


def _row(l, m):
    return l * l + l + m


def _mpf(v):
    """Exact conversion of a long double to mpmath (as a sum of two doubles)."""
    hi = float(v)
    lo = float(LD(v) - LD(hi))
    return mp.mpf(hi) + mp.mpf(lo)


def _load_table(name):
    vals = {}
    for ln in open(os.path.join(GOLDEN, name)):
        ln = ln.strip()
        if not ln or ln.startswith("#"):
            continue
        parts = ln.split()
        l, m = int(parts[0]), int(parts[1])
        vals[(l, m)] = [float(v) for v in parts[2:]]
    return vals


# Appendix D: points of Tables ref1 and ref2 (the second with the decimal point of
# phi restored, see tests/golden/appD_table_ref2.txt)
APPD = {
    "appD_table_ref1.txt": ("2.12160245947564796", "-1.82732370250979703"),
    "appD_table_ref2.txt": ("1.69050041976591414", "0.758228122208986166"),
}


@pytest.mark.parametrize("name", sorted(APPD))
def test_appendix_d_reference_values(orc, name):
    """Appendix D tables: 2 x 100 printed FP64 values (reading: first value column
    is R_l^{+m}, second is R_l^{-m})."""
    th, ph = APPD[name]
    Y = orc.eval_angles(9, [LD(th)], [LD(ph)])[:, 0]
    vals = _load_table(name)
    assert len(vals) == 55
    worst = 0.0
    for (l, m), v in vals.items():
        if m == 0:
            worst = max(worst, abs(float(Y[_row(l, 0)]) - v[0]))
        else:
            worst = max(worst, abs(float(Y[_row(l, m)]) - v[0]))
            worst = max(worst, abs(float(Y[_row(l, -m)]) - v[1]))
    assert worst <= 1e-15, worst


def test_appendix_d_readings_are_needed(orc):
    """The columns as labelled, or phi as printed in Table ref2, do not match."""
    vals = _load_table("appD_table_ref1.txt")
    Y = orc.eval_angles(9, [LD(APPD["appD_table_ref1.txt"][0])],
                        [LD(APPD["appD_table_ref1.txt"][1])])[:, 0]
    as_labelled = max(abs(float(Y[_row(l, -m)]) - v[0]) for (l, m), v in vals.items() if m > 0)
    assert as_labelled > 0.1
    vals2 = _load_table("appD_table_ref2.txt")
    Y2 = orc.eval_angles(9, [LD("1.69050041976591414")], [LD("7.58228122208986166")])[:, 0]
    printed_phi = max(abs(float(Y2[_row(l, m)]) - v[0]) for (l, m), v in vals2.items())
    assert printed_phi > 0.1


def _mp_real_ylm(l, m, theta, phi):
    """Real harmonic from the complex one (mpmath.spherharm, which carries the
    Condon-Shortley phase) by the paper's eq. real_harmomics, literally."""
    if m == 0:
        return mp.re(mp.spherharm(l, 0, theta, phi))
    if m < 0:
        v = 1j / mp.sqrt(2) * (mp.spherharm(l, m, theta, phi)
                               - (-1) ** m * mp.spherharm(l, -m, theta, phi))
    else:
        v = 1 / mp.sqrt(2) * (mp.spherharm(l, -m, theta, phi)
                              + (-1) ** m * mp.spherharm(l, m, theta, phi))
    assert abs(mp.im(v)) < mp.mpf(10) ** (-30)
    return mp.re(v)


def _mp_angles(x, y, z):
    r = mp.sqrt(x * x + y * y + z * z)
    return mp.acos(z / r), mp.atan2(y, x)


def test_definition_brute_force_mpmath(orc):
    """Cartesian oracle vs eq. real_harmomics over mpmath's complex Y at 40 digits,
    on random points and points close to the poles and axes."""
    mp.mp.dps = 40
    pts = np.concatenate([workloads.isotropic_points(24, 0.1, 5.0, seed=7),
                          np.array([[1e-7, 2e-7, 1.0], [3e-9, -1e-9, -2.0], [1.0, 0.0, 0.0],
                                    [0.0, -3.0, 0.0], [0.5, 0.5, 1e-12], [-2.0, 1.0, -0.5]])])
    Y = orc.eval_xyz(9, pts)
    worst = 0.0
    for i, (x, y, z) in enumerate(pts):
        th, ph = _mp_angles(mp.mpf(x), mp.mpf(y), mp.mpf(z))
        for l in range(10):
            for m in range(-l, l + 1):
                ref = _mp_real_ylm(l, m, th, ph)
                worst = max(worst, abs(float(_mpf(Y[_row(l, m), i]) - ref)))
    assert worst <= 2e-17, worst


def test_library_routine_scipy(orc):
    """scipy.special.sph_harm_y (complex, Condon-Shortley phase) through
    eq. real_harmomics, in double precision."""
    from scipy.special import sph_harm_y
    pts = workloads.isotropic_points(500, 0.1, 5.0, seed=3)
    x, y, z = pts.T
    th = np.arccos(z / np.sqrt((pts * pts).sum(1)))
    ph = np.arctan2(y, x)
    Y = orc.eval_xyz(9, pts).astype(np.float64)
    for l in range(10):
        for m in range(-l, l + 1):
            if m == 0:
                ref = sph_harm_y(l, 0, th, ph).real
            elif m < 0:
                ref = (1j / math.sqrt(2) * (sph_harm_y(l, m, th, ph)
                                            - (-1) ** m * sph_harm_y(l, -m, th, ph))).real
            else:
                ref = (1 / math.sqrt(2) * (sph_harm_y(l, -m, th, ph)
                                           + (-1) ** m * sph_harm_y(l, m, th, ph))).real
            assert np.abs(Y[_row(l, m)] - ref).max() <= 5e-14, (l, m)


def test_appendix_c_forms_match_definition(orc):
    """Every Appendix C formula (with the three corrected readings), and every m>0
    value from Appendix B rotations, against the oracle at 40-digit precision."""
    mp.mp.dps = 40
    F = appc_forms.forms()
    pts = workloads.isotropic_points(30, 0.5, 2.0, seed=11)
    Y = orc.eval_xyz(9, pts)
    for i, (x, y, z) in enumerate(pts):
        X, Yv, Z = mp.mpf(x), mp.mpf(y), mp.mpf(z)
        r = mp.sqrt(X * X + Yv * Yv + Z * Z)
        xb, yb, zb = X / r, Yv / r, Z / r
        for key, f in F.items():
            if len(key) == 3 and key[2] == "printed":
                continue
            l, m = key[0], key[1]
            err = abs(f(xb, yb, zb) - _mpf(Y[_row(l, m), i]))
            assert err <= 2e-17, (key, float(err))
        for l in range(1, 10):
            for m in range(1, l + 1):
                v = appc_forms.positive_m(l, m, xb, yb, zb)
                err = abs(v - _mpf(Y[_row(l, m), i]))
                assert err <= 2e-17, ((l, m), float(err))


def test_appendix_c_garbled_forms_are_garbled(orc):
    """The three printed forms that the corrected readings replace are wrong."""
    mp.mp.dps = 40
    F = appc_forms.forms()
    pts = workloads.isotropic_points(5, 0.5, 2.0, seed=12)
    Y = orc.eval_xyz(9, pts)
    for key in [(5, 0, "printed"), (8, -1, "printed"), (9, -7, "printed")]:
        errs = []
        for i, (x, y, z) in enumerate(pts):
            X, Yv, Z = mp.mpf(x), mp.mpf(y), mp.mpf(z)
            r = mp.sqrt(X * X + Yv * Yv + Z * Z)
            errs.append(abs(F[key](X / r, Yv / r, Z / r) - _mpf(Y[_row(key[0], key[1]), i])))
        assert max(errs) > 1e-3, key


def test_poles_and_origin(orc):
    """At +-z only m = 0 survives: R_l^0(+-z) = (+-1)^l sqrt((2l+1)/(4 pi)).
    At r = 0 only l = 0 is nonzero (paper, Section 2)."""
    pts = np.array([[0, 0, 2.5], [0, 0, -0.1], [0, 0, 1e-200], [0, 0, 0.0]], dtype=np.float64)
    Y = orc.eval_xyz(9, pts)
    for l in range(10):
        for m in range(-l, l + 1):
            for i, sgn in enumerate([1, -1, 1]):
                ref = sgn ** l * np.sqrt(LD(2 * l + 1) / (4 * PI_LD)) if m == 0 else LD(0)
                assert abs(Y[_row(l, m), i] - ref) <= 1e-18
            ref0 = 1 / np.sqrt(4 * PI_LD) if l == 0 else LD(0)
            assert abs(Y[_row(l, m), 3] - ref0) <= 1e-19


def _dfact(n):
    return 1 if n <= 0 else n * _dfact(n - 2)


def test_equator_axes_closed_form(orc):
    """On the +-x and +-y axes: P~_l^m(0) = 0 for odd l+m, else
    (-1)^((l-m)/2) (l+m-1)!!/(l-m)!!, and cos(m phi), sin(m phi) in {0, +-1}."""
    axes = {(1, 0, 0): 0.0, (0, 1, 0): math.pi / 2, (-1, 0, 0): math.pi, (0, -1, 0): -math.pi / 2}
    pts = np.array([[3 * a for a in k] for k in axes], dtype=np.float64)
    Y = orc.eval_xyz(9, pts)
    for i, phi in enumerate(axes.values()):
        for l in range(10):
            for m in range(0, l + 1):
                P = 0.0 if (l + m) % 2 else (-1) ** ((l - m) // 2) * _dfact(l + m - 1) / _dfact(l - m)
                N = np.sqrt(LD(2 * l + 1) / (4 * PI_LD) * LD(math.factorial(l - m))
                            / LD(math.factorial(l + m)))
                c = round(math.cos(m * phi))
                s = round(math.sin(m * phi))
                if m == 0:
                    assert abs(Y[_row(l, 0), i] - N * P) <= 1e-18
                else:
                    assert abs(Y[_row(l, m), i] - np.sqrt(LD(2)) * N * P * c) <= 1e-18
                    assert abs(Y[_row(l, -m), i] - np.sqrt(LD(2)) * N * P * s) <= 1e-18


def test_addition_theorem(orc):
    """sum_m (R_l^m)^2 = (2l+1)/(4 pi) for every l and every direction."""
    sp = workloads.special_points()
    pts = np.concatenate([workloads.isotropic_points(2000, 0.01, 10, seed=5),
                          sp[(sp * sp).sum(1) > 0]])
    Y = orc.eval_xyz(9, pts)
    for l in range(10):
        s = (Y[l * l:(l + 1) * (l + 1)] ** 2).sum(axis=0)
        ref = LD(2 * l + 1) / (4 * PI_LD)
        assert (np.abs(s - ref) / ref).max() <= 1e-17


def test_orthonormality_exact_quadrature(orc):
    """Gauss-Legendre (10 nodes in cos theta) x 19 uniform phi integrates every
    product R_l^m R_l'^m' with l, l' <= 9 exactly; the Gram matrix is I."""
    xg, wg = np.polynomial.legendre.leggauss(10)
    nphi = 19
    phis = 2 * np.pi * np.arange(nphi) / nphi
    th = np.repeat(np.arccos(xg), nphi)
    ph = np.tile(phis, 10)
    w = np.repeat(wg, nphi) * (2 * np.pi / nphi)
    Y = orc.eval_angles(9, th.astype(LD), ph.astype(LD)).astype(np.float64)
    G = (Y * w) @ Y.T
    assert np.abs(G - np.eye(100)).max() <= 1e-14


def test_parity_and_mirror(orc):
    """R(-u) = (-1)^l R(u); y -> -y flips the sign of m < 0 terms only."""
    pts = workloads.isotropic_points(300, 0.1, 5, seed=9)
    Y = orc.eval_xyz(9, pts)
    Yn = orc.eval_xyz(9, -pts)
    mirror = pts * np.array([1, -1, 1])
    Ym = orc.eval_xyz(9, mirror)
    for l in range(10):
        for m in range(-l, l + 1):
            assert np.abs(Yn[_row(l, m)] - (-1) ** l * Y[_row(l, m)]).max() <= 1e-17
            sgn = -1 if m < 0 else 1
            assert np.abs(Ym[_row(l, m)] - sgn * Y[_row(l, m)]).max() <= 1e-17


def test_scale_invariance_and_f32_widening(orc):
    """Only the direction matters; float32 inputs are widened exactly."""
    pts = workloads.isotropic_points(200, 0.1, 5, seed=4)
    Y1 = orc.eval_xyz(9, pts)
    Y2 = orc.eval_xyz(9, pts * 1024.0)
    assert np.abs(Y1 - Y2).max() <= 1e-17
    p32 = pts.astype(np.float32)
    assert np.array_equal(orc.eval_xyz(9, p32), orc.eval_xyz(9, p32.astype(np.float64)))


def test_complex_harmonics_mpmath_and_scipy(orc):
    """Complex Y_l^m from the definition: mpmath spherharm (40 digits) and scipy
    sph_harm_y, both carrying the Condon-Shortley phase."""
    from scipy.special import sph_harm_y
    mp.mp.dps = 40
    pts = np.concatenate([workloads.isotropic_points(12, 0.1, 5.0, seed=51),
                          np.array([[1e-8, 0, 1.0], [0.0, -2.0, 0.0]])])
    re, im = orc.eval_complex_xyz(9, pts)
    for i, (x, y, z) in enumerate(pts):
        th, ph = _mp_angles(mp.mpf(x), mp.mpf(y), mp.mpf(z))
        for l in range(10):
            for m in range(-l, l + 1):
                ref = mp.spherharm(l, m, th, ph)
                r = _row(l, m)
                assert abs(_mpf(re[r, i]) - mp.re(ref)) <= 2e-17
                assert abs(_mpf(im[r, i]) - mp.im(ref)) <= 2e-17
    big = workloads.isotropic_points(500, 0.1, 5.0, seed=52)
    re, im = orc.eval_complex_xyz(9, big)
    th = np.arccos(big[:, 2] / np.sqrt((big * big).sum(1)))
    ph = np.arctan2(big[:, 1], big[:, 0])
    for l in range(10):
        for m in range(-l, l + 1):
            ref = sph_harm_y(l, m, th, ph)
            r = _row(l, m)
            assert np.abs(re[r].astype(np.float64) - ref.real).max() <= 5e-14
            assert np.abs(im[r].astype(np.float64) - ref.imag).max() <= 5e-14


def test_complex_from_real_reading(orc):
    """Y_l^m = (-1)^m (R_l^m + i R_l^-m) / sqrt(2) for m > 0; the relation as
    printed in Section 3 (without 1/sqrt(2)) does not hold."""
    pts = workloads.isotropic_points(200, 0.1, 5.0, seed=53)
    R = orc.eval_xyz(9, pts)
    re, im = orc.eval_complex_xyz(9, pts)
    h = 1 / np.sqrt(LD(2))
    worst = LD(0)
    for l in range(10):
        assert np.abs(re[_row(l, 0)] - R[_row(l, 0)]).max() <= 1e-18
        for m in range(1, l + 1):
            s = (-1) ** m
            worst = max(worst, np.abs(re[_row(l, m)] - s * h * R[_row(l, m)]).max())
            worst = max(worst, np.abs(im[_row(l, m)] - s * h * R[_row(l, -m)]).max())
            printed = np.abs(re[_row(l, m)] - s * R[_row(l, m)]).max()
            assert printed > 1e-3
    assert worst <= 1e-18


def test_high_l_mpmath_addition_and_quadrature(orc):
    """Beyond l = 9 (the recurrence interface goes to l = 24): mpmath at 40 digits
    for l = 12, 17, 24, the addition theorem for every l <= 24, and exact
    Gauss-Legendre x uniform-phi orthonormality up to l = 24."""
    mp.mp.dps = 40
    L = 24
    pts = np.concatenate([workloads.isotropic_points(6, 0.1, 5.0, seed=81),
                          np.array([[1e-8, 2e-8, 1.0], [0.0, -3.0, 1e-9]])])
    Y = orc.eval_xyz(L, pts)
    for i, (x, y, z) in enumerate(pts):
        th, ph = _mp_angles(mp.mpf(x), mp.mpf(y), mp.mpf(z))
        for l in (12, 17, 24):
            for m in range(-l, l + 1, 5):
                ref = _mp_real_ylm(l, m, th, ph)
                assert abs(_mpf(Y[_row(l, m), i]) - ref) <= 1e-16, (l, m)
    big = workloads.isotropic_points(500, 0.1, 5, seed=82)
    Yb = orc.eval_xyz(L, big)
    for l in range(L + 1):
        s = (Yb[l * l:(l + 1) * (l + 1)] ** 2).sum(axis=0)
        ref = LD(2 * l + 1) / (4 * PI_LD)
        assert (np.abs(s - ref) / ref).max() <= 1e-16
    xg, wg = np.polynomial.legendre.leggauss(L + 1)
    nphi = 2 * L + 1
    phis = 2 * np.pi * np.arange(nphi) / nphi
    th = np.repeat(np.arccos(xg), nphi)
    ph = np.tile(phis, L + 1)
    w = np.repeat(wg, nphi) * (2 * np.pi / nphi)
    Yq = orc.eval_angles(L, th.astype(LD), ph.astype(LD)).astype(np.float64)
    G = (Yq * w) @ Yq.T
    assert np.abs(G - np.eye((L + 1) ** 2)).max() <= 1e-13


def test_spinor_harmonics_closed_forms(orc):
    """Spinor harmonics (eq. spinorial): for every j the sum over m_j of |Omega|^2
    is (2j+1)/(4 pi) at every direction; they are orthonormal under exact
    quadrature; l = 0 gives pure spin up/down Y_0^0."""
    lmax = 4
    pts = workloads.isotropic_points(300, 0.1, 5, seed=91)
    re, im = orc.eval_spinor_xyz(lmax, pts)
    for l in range(lmax + 1):
        for kappa in (-1, 1):
            if kappa < 0 and l == 0:
                continue
            j2 = 2 * l + kappa
            ks = [orc.spinor_index(l, kappa, mj2) for mj2 in range(-j2, j2 + 1, 2)]
            tot = (re[ks] ** 2 + im[ks] ** 2).sum(axis=(0, 1))
            ref = LD(j2 + 1) / (4 * PI_LD)
            assert (np.abs(tot - ref) / ref).max() <= 1e-17
    y00 = 1 / np.sqrt(4 * PI_LD)
    up, dn = orc.spinor_index(0, 1, 1), orc.spinor_index(0, 1, -1)
    assert np.abs(re[up, 0] - y00).max() <= 1e-18 and np.all(re[up, 1] == 0)
    assert np.abs(re[dn, 1] - y00).max() <= 1e-18 and np.all(re[dn, 0] == 0)
    # orthonormality: Gauss-Legendre in cos(theta) x uniform phi, exact for l <= 4
    xg, wg = np.polynomial.legendre.leggauss(lmax + 2)
    nphi = 2 * lmax + 3
    th = np.repeat(np.arccos(xg), nphi)
    ph = np.tile(2 * np.pi * np.arange(nphi) / nphi, lmax + 2)
    w = np.repeat(wg, nphi) * (2 * np.pi / nphi)
    q = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)
    r2, i2 = orc.eval_spinor_xyz(lmax, q)
    Z = (r2 + 1j * i2).astype(np.complex128).reshape(r2.shape[0], -1)  # [spinor][2 n]
    W = np.tile(w, 2)
    G = (Z.conj() * W) @ Z.T
    assert np.abs(G - np.eye(r2.shape[0])).max() <= 1e-13


def _spinor_cx(orc, lmax, theta, phi):
    re, im = orc.eval_spinor_angles(lmax, np.asarray(theta, dtype=LD), np.asarray(phi, dtype=LD))
    return re + 1j * im  # [spinor][2][n] complex long double


def test_spinor_labels_are_angular_momentum_eigenstates(orc):
    """The (l, j, m_j) label of every spinor of the oracle, pinned by the angular
    momentum algebra rather than by eq. spinorial itself: with L_z = -i d/dphi and
    L_+- = e^{+-i phi} (+-d/dtheta + i cot(theta) d/dphi) (Condon-Shortley
    convention) applied by 4th-order central differences,
        J_z Omega = (L_z + sigma_z / 2) Omega = m_j Omega,
        (sigma . L) Omega = (j(j+1) - l(l+1) - 3/4) Omega = l (j = l + 1/2), -(l+1) (j = l - 1/2),
    where (sigma . L) Omega = (L_z up + L_- down, -L_z down + L_+ up).  A reversed
    m_j order, swapped j = l +- 1/2 blocks or a wrong relative sign between the two
    components fails one of them."""
    lmax = 4
    rng = np.random.default_rng(93)
    th = rng.uniform(0.3, 2.8, 24).astype(LD)
    ph = rng.uniform(0.0, 2 * np.pi, 24).astype(LD)
    h = LD("1e-3")
    O = _spinor_cx(orc, lmax, th, ph)

    def d4(f, a, b):  # 4th-order central difference in the angle selected by (a, b)
        return (-f(2 * a, 2 * b) + 8 * f(a, b) - 8 * f(-a, -b) + f(-2 * a, -2 * b)) / (12 * h)

    dth = d4(lambda a, b: _spinor_cx(orc, lmax, th + a, ph + b), h, LD(0))
    dph = d4(lambda a, b: _spinor_cx(orc, lmax, th + a, ph + b), LD(0), h)
    cot = np.cos(th) / np.sin(th)
    Lz = -1j * dph
    Lp = np.exp(1j * ph) * (dth + 1j * cot * dph)
    Lm = np.exp(-1j * ph) * (-dth + 1j * cot * dph)
    up, dn = 0, 1
    checked = 0
    for l in range(lmax + 1):
        for kappa in (-1, 1):
            if kappa < 0 and l == 0:
                continue
            j2 = 2 * l + kappa
            so = l if kappa > 0 else -(l + 1)
            for mj2 in range(-j2, j2 + 1, 2):
                k = orc.spinor_index(l, kappa, mj2)
                jz = np.stack([Lz[k, up] + O[k, up] / 2, Lz[k, dn] - O[k, dn] / 2])
                sl = np.stack([Lz[k, up] + Lm[k, dn], -Lz[k, dn] + Lp[k, up]])
                scale = 1 + np.abs(O[k]).max()
                assert np.abs(jz - LD(mj2) / 2 * O[k]).max() <= 1e-9 * scale, (l, kappa, mj2)
                assert np.abs(sl - so * O[k]).max() <= 1e-9 * scale, (l, kappa, mj2)
                checked += 1
    assert checked == 2 * (lmax + 1) ** 2


def test_spinor_azimuthal_rotation_and_mpmath(orc):
    """phi -> phi + alpha multiplies the upper component of Omega_{j m_j} by
    e^{i (m_j - 1/2) alpha} and the lower by e^{i (m_j + 1/2) alpha}; and every
    spinor for l = 1 .. 4 equals eq. spinorial composed from mpmath's spherharm at
    40 digits (j = l + 1/2: upper +sqrt(l + m_j + 1/2), lower sqrt(l - m_j + 1/2);
    j = l - 1/2: upper -sqrt(l - m_j + 1/2), lower sqrt(l + m_j + 1/2); all over
    sqrt(2l + 1), upper with Y_l^{m_j - 1/2}, lower with Y_l^{m_j + 1/2})."""
    lmax = 4
    rng = np.random.default_rng(94)
    th = rng.uniform(0.05, 3.09, 12).astype(LD)
    ph = rng.uniform(0.0, 2 * np.pi, 12).astype(LD)
    alpha = LD("0.7345")
    O = _spinor_cx(orc, lmax, th, ph)
    R = _spinor_cx(orc, lmax, th, ph + alpha)
    mp.mp.dps = 40
    for l in range(1, lmax + 1):
        for kappa in (-1, 1):
            j2 = 2 * l + kappa
            for mj2 in range(-j2, j2 + 1, 2):
                k = orc.spinor_index(l, kappa, mj2)
                for c, shift in ((0, -1), (1, 1)):
                    ph_fac = np.exp(1j * alpha * LD(mj2 + shift) / 2)
                    assert np.abs(R[k, c] - ph_fac * O[k, c]).max() <= 1e-15, (l, kappa, mj2, c)
                for i in range(th.size):
                    t, f = _mpf(th[i]), _mpf(ph[i])

                    def Y(m):
                        return mp.mpc(0) if abs(m) > l else mp.spherharm(l, m, t, f)

                    mu, ml = (mj2 - 1) // 2, (mj2 + 1) // 2
                    if kappa > 0:
                        cu, cl = mp.sqrt(mp.mpf(2 * l + mj2 + 1) / 2), mp.sqrt(mp.mpf(2 * l - mj2 + 1) / 2)
                    else:
                        cu, cl = -mp.sqrt(mp.mpf(2 * l - mj2 + 1) / 2), mp.sqrt(mp.mpf(2 * l + mj2 + 1) / 2)
                    den = mp.sqrt(2 * l + 1)
                    for c, ref in ((0, cu * Y(mu) / den), (1, cl * Y(ml) / den)):
                        got = O[k, c, i]
                        err = abs(mp.mpc(_mpf(got.real), _mpf(got.imag)) - ref)
                        assert err <= 1e-17, (l, kappa, mj2, c, float(err))


def test_library_routine_std_sph_legendre(orc, tmp_path):
    """libstdc++'s std::sph_legendre(l, m, theta) = Y_l^m(theta, 0), Condon-Shortley
    phase included, so R_l^0 = Y_l^0 and R_l^{+-m} = sqrt(2) (-1)^m Y_l^m(theta, 0)
    {cos, sin}(m phi) (eq. real_harmomics)."""
    import ctypes
    import shutil
    import subprocess
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    so = str(tmp_path / "std_sph_legendre.so")
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "host", "std_sph_legendre.cpp")
    subprocess.check_call([gxx, "-O2", "-std=c++17", "-fPIC", "-shared", src, "-o", so])
    L = ctypes.CDLL(so)
    L.std_sph_legendre.argtypes = [ctypes.c_int, ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p]
    th = np.concatenate([np.arccos(np.random.default_rng(53).uniform(-1, 1, 2000)), [0.0, np.pi, np.pi / 2]])
    ph = np.random.default_rng(54).uniform(-np.pi, np.pi, th.shape[0])
    leg = np.empty((55, th.shape[0]))
    L.std_sph_legendre(9, th.shape[0], th.ctypes.data, leg.ctypes.data)
    got = orc.eval_angles(9, th.astype(LD), ph.astype(LD)).astype(np.float64)
    for l in range(10):
        for m in range(0, l + 1):
            y = leg[l * (l + 1) // 2 + m]
            if m == 0:
                assert np.abs(got[_row(l, 0)] - y).max() <= 1e-14
            else:
                s = math.sqrt(2.0) * (-1) ** m
                assert np.abs(got[_row(l, m)] - s * y * np.cos(m * ph)).max() <= 1e-14
                assert np.abs(got[_row(l, -m)] - s * y * np.sin(m * ph)).max() <= 1e-14


def test_complex_from_angles_mpmath(orc):
    """The angular entry of the complex oracle against mpmath's spherharm, which
    takes (theta, phi) directly; poles and azimuths in every quadrant included."""
    mp.mp.dps = 40
    rng = np.random.default_rng(55)
    th = np.concatenate([np.arccos(rng.uniform(-1, 1, 10)), [0.0, np.pi, 1e-9, np.pi / 2]])
    ph = np.concatenate([rng.uniform(-np.pi, np.pi, 10), [0.3, -2.5, 3.0, -0.7]])
    re, im = orc.eval_complex_angles(9, th.astype(LD), ph.astype(LD))
    for i in range(th.shape[0]):
        t, p = _mpf(LD(th[i])), _mpf(LD(ph[i]))
        for l in range(10):
            for m in range(-l, l + 1):
                ref = mp.spherharm(l, m, t, p)
                r = _row(l, m)
                assert abs(_mpf(re[r, i]) - mp.re(ref)) <= 2e-17
                assert abs(_mpf(im[r, i]) - mp.im(ref)) <= 2e-17


def test_maxerr_helper_matches_stored_values(orc):
    """The comparison helper for whole outputs (oracle.eval_xyz_maxerr) reports per
    l the largest deviation of a given array from eval_xyz's values: zero-level for
    eval_xyz's own values rounded to double (at most half an ulp), the planted
    error in the l it was planted in, +inf for a NaN, and it honours padded rows."""
    pts = workloads.points_plain_eval(seed=7, n_random=3000)
    ref = orc.eval_xyz(9, pts)
    wide = np.zeros((100, pts.shape[0] + 5))
    wide[:, :pts.shape[0]] = ref.astype(np.float64)
    e0 = orc.eval_xyz_maxerr(9, pts, wide)
    half_ulp = np.abs(ref).astype(np.float64).max(axis=1) * 2.0 ** -53
    assert np.all(e0 <= np.array([half_ulp[l * l:(l + 1) ** 2].max() for l in range(10)]) * 1.0001)
    wide[50, 11] += 3e-11  # row 50: l = 7
    e1 = orc.eval_xyz_maxerr(9, pts, wide)
    assert abs(e1[7] - 3e-11) < 1e-14 and np.all(np.delete(e1, 7) == np.delete(e0, 7))
    wide[2, 0] = np.nan  # row 2: l = 1
    assert np.isinf(orc.eval_xyz_maxerr(9, pts, wide)[1])
