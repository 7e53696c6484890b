#!/usr/bin/env python3
"""Writes sh_constants.h: the constants of the factorised real-harmonic formulas
used by the GPU kernels.  Run from anywhere; it rewrites the header next to itself.

Every explicit formula of the paper (Appendix C, and the m > 0 values of
Appendix B) has the shape

    R_l^{-m} = A_lm * Z_lm(z) * Shat_m(x, y)      (m > 0; m = 0 uses A_l0 * Z_l0)
    R_l^{+m} = B_lm * Z_lm(z) * Chat_m(x, y)

on the unit sphere, with the pair factor p(a, b) = (a - b)(a + b) (eq. rpair):

* Z_lm(z) = z^((l-m) mod 2) * prod_k p(r_k, z), where the r_k are the positive
  roots of d^m P_l / dz^m.  The paper's closed-form roots (Gauss-Legendre nodes,
  roots of P_l', ...) and its printed high-precision roots are exactly these; its
  Horner-form entries are the same polynomials written unfactorised.
* Shat_m(x, y) = y * x^[m even] * prod_k p(tan(k pi/m) x, y), k = 1..ceil(m/2)-1:
  the factors of Im (x + i y)^m, one linear factor per zero line phi = k pi/m.
* Chat_m(x, y) = x^[m odd] * prod_k p(tan((k+1/2) pi/m) x, y), k = 0..floor(m/2)-1:
  the factors of Re (x + i y)^m.  Appendix B obtains R_l^{+m} by rotating the
  (x, y) pair of the m < 0 formula by pi/(2m) (up to a sign); a rotation leaves
  Z_lm unchanged and maps the zero lines of sin(m phi) onto those of cos(m phi),
  so the rotated xy factor is Chat_m up to a constant, which B_lm absorbs.

The prefactors follow from the leading coefficient of d^m P_l/dz^m,
(2l)! / (2^l l! (l-m)!), the normalisation N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)
of eq. sphericalfromlegendre, sqrt(2) for m != 0 (eq. real_harmomics with the
Condon-Shortley phase cancelled), (-1)^(number of pairs) from z^2 - r^2 = -p(r, z),
and the leading coefficients of Shat_m and Chat_m against Im/Re (x+iy)^m.

Everything is computed with mpmath at 50 digits and rounded once to double and
once to float.
"""
from __future__ import annotations

import os

import mpmath as mp
import sympy as sp

LMAX = 9
mp.mp.dps = 50


def zroots(l: int, m: int):
    """Positive roots of d^m P_l/dz^m (ascending) and its leading coefficient."""
    z = sp.symbols("z")
    q = sp.Poly(sp.diff(sp.legendre(l, z), z, m), z)
    lead = q.LC()
    e = (l - m) % 2
    # q = lead * z^e * w-polynomial in w = z^2
    coeffs = q.all_coeffs()  # highest first
    # drop the z^e factor and keep every second coefficient
    if e:
        assert coeffs[-1] == 0
        coeffs = coeffs[:-1]
    wcoef = coeffs[::2]
    assert all(c == 0 for c in coeffs[1::2])
    npairs = (l - m) // 2
    if npairs == 0:
        return [], lead
    ws = mp.polyroots([mp.mpf(sp.Rational(c).p) / mp.mpf(sp.Rational(c).q) for c in wcoef],
                      maxsteps=200, extraprec=200)
    ws = sorted(mp.re(w) for w in ws)
    for w in ws:
        assert 0 < w < 1
    return [mp.sqrt(w) for w in ws], lead


def nlm(l, m):
    return mp.sqrt(mp.mpf(2 * l + 1) / (4 * mp.pi) * mp.factorial(l - m) / mp.factorial(l + m))


def s_tans(m):
    return [mp.tan(k * mp.pi / m) for k in range(1, (m + 1) // 2)]


def c_tans(m):
    return [mp.tan((k + mp.mpf(1) / 2) * mp.pi / m) for k in range(m // 2)]


def s_scale(m):
    """Im (x+iy)^m = s_m * Shat_m: compare the coefficients of x^(m-1) y."""
    prod = mp.mpf(1)
    for t in s_tans(m):
        prod *= t * t
    return m / prod


def c_scale(m):
    """Re (x+iy)^m = c_m * Chat_m: compare the coefficients of x^m."""
    prod = mp.mpf(1)
    for t in c_tans(m):
        prod *= t * t
    return 1 / prod


def build():
    A = [[mp.mpf(0)] * (LMAX + 1) for _ in range(LMAX + 1)]
    B = [[mp.mpf(0)] * (LMAX + 1) for _ in range(LMAX + 1)]
    R = [[[] for _ in range(LMAX + 1)] for _ in range(LMAX + 1)]
    for l in range(LMAX + 1):
        for m in range(l + 1):
            roots, lead = zroots(l, m)
            lead = mp.mpf(sp.Rational(lead).p) / mp.mpf(sp.Rational(lead).q)
            sign = (-1) ** len(roots)
            base = nlm(l, m) * lead * sign
            R[l][m] = roots
            if m == 0:
                A[l][m] = base
                B[l][m] = mp.mpf(0)
            else:
                A[l][m] = mp.sqrt(2) * base * s_scale(m)
                B[l][m] = mp.sqrt(2) * base * c_scale(m)
    return A, B, R


def fmt_d(v) -> str:
    return mp.nstr(v, 17, min_fixed=0, max_fixed=0, strip_zeros=False) if v != 0 else "0.0"


def fmt_f(v) -> str:
    """Nearest float (24-bit significand) of the 50-digit value, written exactly."""
    if v == 0:
        return "0.0f"
    with mp.workprec(24):
        f = +v
    return repr(float(f)) + "f"


def emit(path: str):
    A, B, R = build()
    L = LMAX + 1

    def table3(rows, f):
        out = []
        for l in range(L):
            inner = []
            for m in range(L):
                rs = list(rows[l][m]) + [mp.mpf(0)] * (4 - len(rows[l][m])) if m <= l else [mp.mpf(0)] * 4
                inner.append("{" + ", ".join(f(v) for v in rs) + "}")
            out.append("  {" + ", ".join(inner) + "}")
        return "{\n" + ",\n".join(out) + "\n}"

    def table2(rows, f):
        out = []
        for l in range(L):
            out.append("  {" + ", ".join(f(rows[l][m]) if m <= l else f(mp.mpf(0))
                                         for m in range(L)) + "}")
        return "{\n" + ",\n".join(out) + "\n}"

    def tans(fn, f):
        out = []
        for m in range(L):
            ts = fn(m) if m > 0 else []
            ts = list(ts) + [mp.mpf(0)] * (4 - len(ts))
            out.append("  {" + ", ".join(f(t) for t in ts) + "}")
        return "{\n" + ",\n".join(out) + "\n}"

    body = f"""// Generated by gen_sh_constants.py -- do not edit by hand.
//
// Constants of the factorised real spherical harmonics for l <= {LMAX}
// (paper Appendix C for m <= 0, Appendix B for m > 0), on the unit sphere:
//   R_l^-m = kA[l][m] * Z_lm(z) * Shat_m(x, y)     (m = 0: kA[l][0] * Z_l0(z))
//   R_l^+m = kB[l][m] * Z_lm(z) * Chat_m(x, y)
//   Z_lm(z)  = z^((l-m)&1) * prod_k p(kZRoot[l][m][k], z),  k < (l-m)/2
//   Shat_m   = y * x^[m even] * prod_k p(kTanS[m][k] * x, y), k < ceil(m/2)-1
//   Chat_m   = x^[m odd]      * prod_k p(kTanC[m][k] * x, y), k < floor(m/2)
//   p(a, b)  = (a - b) * (a + b)                            (eq. rpair)
// kZRoot[l][m] are the positive roots of d^m P_l/dz^m, kTanS[m][k] = tan(k pi/m),
// kTanC[m][k] = tan((k+1/2) pi/m).  Values rounded once from 50-digit mpmath.
#pragma once

namespace shc {{

constexpr int kLmax = {LMAX};

constexpr double kZRoot[{L}][{L}][4] = {table3(R, fmt_d)};

constexpr float kZRootF[{L}][{L}][4] = {table3(R, fmt_f)};

constexpr double kA[{L}][{L}] = {table2(A, fmt_d)};

constexpr double kB[{L}][{L}] = {table2(B, fmt_d)};

constexpr float kAF[{L}][{L}] = {table2(A, fmt_f)};

constexpr float kBF[{L}][{L}] = {table2(B, fmt_f)};

constexpr double kTanS[{L}][4] = {tans(s_tans, fmt_d)};

constexpr double kTanC[{L}][4] = {tans(c_tans, fmt_d)};

constexpr float kTanSF[{L}][4] = {tans(s_tans, fmt_f)};

constexpr float kTanCF[{L}][4] = {tans(c_tans, fmt_f)};

}}  // namespace shc
"""
    with open(path, "w") as fh:
        fh.write(body)


if __name__ == "__main__":
    emit(os.path.join(os.path.dirname(os.path.abspath(__file__)), "sh_constants.h"))
