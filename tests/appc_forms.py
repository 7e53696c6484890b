"""The paper's explicit factorised formulas (Appendix C) for R_l^m, m <= 0, l <= 9,
restated in mpmath, plus the Appendix B rotations that give m > 0.

Used only by tests, as a second, Cartesian route to the real harmonics that is
independent of the oracle's Legendre recurrence.  Three printed forms are garbled
in the paper; the readings used here are:

* R_5^0: the division by 3 sits outside the square root, i.e. the roots are
  sqrt(5 -+ 2 sqrt(10/7)) / 3 (these are the positive Gauss-Legendre nodes of P_5);
* R_8^-1, rooted form: the prefactor is -2145/64 (the Horner form is printed right);
* R_9^-7, polynomial form: the factor y-bar is missing (the rooted form is right).

Where the paper prints two forms of one harmonic, both are listed (the second
under a "/rooted" key) so that each is checked on its own.  Literal printed forms
of the garbled entries are kept under "/printed" keys for the reading tests.
"""
from __future__ import annotations

import mpmath as mp


def p(a, b):
    """Pair factor (a - b)(a + b) (paper eq. rpair)."""
    return (a - b) * (a + b)


def _forms():
    s = mp.sqrt
    pi = mp.pi
    F = {}
    F[(0, 0)] = lambda x, y, z: 1 / s(4 * pi)
    # l = 1
    F[(1, -1)] = lambda x, y, z: s(3 / (4 * pi)) * y
    F[(1, 0)] = lambda x, y, z: s(3 / (4 * pi)) * z
    # l = 2
    F[(2, -2)] = lambda x, y, z: s(15 / pi) / 2 * x * y
    F[(2, -1)] = lambda x, y, z: s(15 / pi) / 2 * y * z
    F[(2, 0)] = lambda x, y, z: s(5 / pi) / 4 * p(s(3) * z, 1)
    # l = 3
    F[(3, -3)] = lambda x, y, z: s(70 / pi) / 8 * y * p(s(3) * x, y)
    F[(3, -2)] = lambda x, y, z: s(105 / pi) / 2 * x * y * z
    F[(3, -1)] = lambda x, y, z: s(42 / pi) / 8 * y * p(s(5) * z, 1)
    F[(3, 0)] = lambda x, y, z: s(7 / pi) / 4 * p(s(5) * z, s(3)) * z
    # l = 4
    F[(4, -4)] = lambda x, y, z: mp.mpf(3) / 4 * s(35 / pi) * x * y * p(x, y)
    F[(4, -3)] = lambda x, y, z: mp.mpf(3) / 8 * s(70 / pi) * y * p(s(3) * x, y) * z
    F[(4, -2)] = lambda x, y, z: mp.mpf(3) / 4 * s(5 / pi) * x * y * p(s(7) * z, 1)
    F[(4, -1)] = lambda x, y, z: mp.mpf(3) / 8 * s(10 / pi) * y * z * p(s(7) * z, s(3))
    F[(4, 0)] = lambda x, y, z: (mp.mpf(105) / 16 * s(1 / pi)
                                 * p(s((3 + 2 * s(mp.mpf(6) / 5)) / 7), z)
                                 * p(s((3 - 2 * s(mp.mpf(6) / 5)) / 7), z))
    # l = 5
    F[(5, -5)] = lambda x, y, z: (mp.mpf(30) / 64 * s(154 / pi) * y
                                  * p(s(1 - 2 / s(5)) * y, x) * p(s(1 + 2 / s(5)) * y, x))
    F[(5, -4)] = lambda x, y, z: mp.mpf(3) / 4 * s(385 / pi) * p(x, y) * y * z * x
    F[(5, -3)] = lambda x, y, z: s(770 / pi) / 32 * y * p(y, s(3) * x) * p(1, 3 * z)
    F[(5, -2)] = lambda x, y, z: s(1155 / pi) / 4 * x * y * p(s(3) * z, 1) * z
    F[(5, -1)] = lambda x, y, z: (mp.mpf(21) / 16 * s(165 / pi) * y
                                  * p(s((7 - 2 * s(7)) / 21), z) * p(s((7 + 2 * s(7)) / 21), z))
    F[(5, 0)] = lambda x, y, z: (mp.mpf(63) / 16 * s(11 / pi) * z
                                 * p(s(5 - 2 * s(mp.mpf(10) / 7)) / 3, z)
                                 * p(s(5 + 2 * s(mp.mpf(10) / 7)) / 3, z))
    F[(5, 0, "printed")] = lambda x, y, z: (mp.mpf(63) / 16 * s(11 / pi) * z
                                            * p(s((5 - 2 * s(mp.mpf(10) / 7)) / 3), z)
                                            * p(s((5 + 2 * s(mp.mpf(10) / 7)) / 3), z))
    # l = 6
    F[(6, -6)] = lambda x, y, z: s(6006 / pi) / 32 * x * y * p(x, s(3) * y) * p(s(3) * x, y)
    F[(6, -5)] = lambda x, y, z: (mp.mpf(3) / 32 * s(2002 / pi) * y * z
                                  * p(s(5 - 2 * s(5)) * x, y) * p(s(5 + 2 * s(5)) * x, y))
    F[(6, -4)] = lambda x, y, z: mp.mpf(3) / 8 * s(91 / pi) * x * y * p(x, y) * p(s(11) * z, 1)
    F[(6, -3)] = lambda x, y, z: (s(2730 / pi) / 32 * y * z * p(s(3) * x, y)
                                  * p(s(11) * z, s(3)))
    F[(6, -2)] = lambda x, y, z: (mp.mpf(33) / 32 * s(2730 / pi) * x * y
                                  * p(s((3 - 4 / s(3)) / 11), z) * p(s((3 + 4 / s(3)) / 11), z))
    F[(6, -1)] = lambda x, y, z: (mp.mpf(33) / 16 * s(273 / pi) * y * z
                                  * p(s((15 - 2 * s(15)) / 33), z) * p(s((15 + 2 * s(15)) / 33), z))
    F[(6, 0)] = lambda x, y, z: s(13 / pi) / 32 * (z * z * ((231 * z * z - 315) * z * z + 105) - 5)
    # l = 7
    t7 = [mp.mpf("0.481574618807528644332162353056970575219"),
          mp.mpf("1.253960337662703837570910978336464443221"),
          mp.mpf("4.381286267534823072404689085032695444150")]
    poly7 = lambda x, y: 7 * x**6 - 35 * x**4 * y**2 + 21 * x**2 * y**4 - y**6  # noqa: E731
    F[(7, -7)] = lambda x, y, z: mp.mpf(3) / 64 * s(715 / pi) * y * poly7(x, y)
    F[(7, -7, "rooted")] = lambda x, y, z: (mp.mpf(3) / 64 * s(715 / pi) * y * p(t7[0] * x, y)
                                            * p(t7[1] * x, y) * p(t7[2] * x, y))
    F[(7, -6)] = lambda x, y, z: (mp.mpf(3) / 32 * s(10010 / pi) * x * y * z
                                  * p(x, s(3) * y) * p(s(3) * x, y))
    F[(7, -5)] = lambda x, y, z: (mp.mpf(3) / 64 * s(385 / pi) * y * p(s(13) * z, 1)
                                  * p(s(5 - 2 * s(5)) * x, y) * p(s(5 + 2 * s(5)) * x, y))
    F[(7, -4)] = lambda x, y, z: (mp.mpf(3) / 8 * s(385 / pi) * x * y * z * p(x, y)
                                  * p(s(13) * z, s(3)))
    F[(7, -3)] = lambda x, y, z: (mp.mpf(429) / 64 * s(35 / pi) * y * p(s(3) * x, y)
                                  * p(s((33 - 2 * s(165)) / 143), z)
                                  * p(s((33 + 2 * s(165)) / 143), z))
    F[(7, -2)] = lambda x, y, z: (mp.mpf(429) / 32 * s(70 / pi) * x * y * z
                                  * p(s((55 - 4 * s(55)) / 143), z)
                                  * p(s((55 + 4 * s(55)) / 143), z))
    F[(7, -1)] = lambda x, y, z: (s(105 / pi) / 64 * y
                                  * (z * z * ((429 * z * z - 495) * z * z + 135) - 5))
    F[(7, 0)] = lambda x, y, z: (s(15 / pi) / 32 * z
                                 * (-35 + z * z * (315 + z * z * (-693 + 429 * z * z))))
    # l = 8
    F[(8, -8)] = lambda x, y, z: (mp.mpf(12) / 128 * s(12155 / pi) * x * y * p(x, y)
                                  * p((1 + s(2)) * x, y) * p((1 - s(2)) * x, y))
    F[(8, -7)] = lambda x, y, z: mp.mpf(3) / 64 * s(12155 / pi) * y * z * poly7(x, y)
    F[(8, -7, "rooted")] = lambda x, y, z: (mp.mpf(3) / 64 * s(12155 / pi) * y * z
                                            * p(t7[0] * x, y) * p(t7[1] * x, y)
                                            * p(t7[2] * x, y))
    F[(8, -6)] = lambda x, y, z: (s(14586 / pi) / 64 * x * y * p(x, s(3) * y) * p(s(3) * x, y)
                                  * p(s(15) * z, 1))
    F[(8, -5)] = lambda x, y, z: (mp.mpf(3) / 64 * s(17017 / pi) * y * z * p(s(5) * z, 1)
                                  * p(s(5 + 2 * s(5)) * x, y) * p(s(5 - 2 * s(5)) * x, y))
    F[(8, -4)] = lambda x, y, z: (mp.mpf(195) / 32 * s(1309 / pi) * x * y * p(x, y)
                                  * p(s((13 - 2 * s(26)) / 65), z)
                                  * p(s((13 + 2 * s(26)) / 65), z))
    F[(8, -3)] = lambda x, y, z: (mp.mpf(39) / 64 * s(19635 / pi) * y * z * p(s(3) * x, y)
                                  * p(s((1 - 2 / s(13)) / 3), z) * p(s((1 + 2 / s(13)) / 3), z))
    F[(8, -2)] = lambda x, y, z: (mp.mpf(3) / 64 * s(1190 / pi) * x * y
                                  * (z * z * ((143 * z * z - 143) * z * z + 33) - 1))
    F[(8, -1)] = lambda x, y, z: (mp.mpf(3) / 64 * s(17 / pi) * y * z
                                  * (z * z * ((715 * z * z - 1001) * z * z + 385) - 35))
    r81 = [mp.mpf("0.36311746382617815871075206870865921"),
           mp.mpf("0.67718627951073775344588542709134245"),
           mp.mpf("0.89975799541146015731234524441833796")]
    F[(8, -1, "rooted")] = lambda x, y, z: (-mp.mpf(2145) / 64 * s(17 / pi) * y * z
                                            * p(r81[0], z) * p(r81[1], z) * p(r81[2], z))
    F[(8, -1, "printed")] = lambda x, y, z: (mp.mpf(2145) / 64 * s(17 / pi) * y * z
                                             * p(r81[0], z) * p(r81[1], z) * p(r81[2], z))
    F[(8, 0)] = lambda x, y, z: (s(17 / pi) / 256
                                 * ((z * z * ((6435 * z * z - 12012) * z * z + 6930) - 1260) * z * z
                                    + 35))
    # l = 9
    t9 = [mp.mpf("0.363970234266202361351047882776834043890"),
          mp.mpf("0.839099631177280011763127298123181364687"),
          mp.mpf("5.671281819617709530994418439863964421625")]
    F[(9, -9)] = lambda x, y, z: (s(461890 / pi) / 512 * y * p(s(3) * x, y)
                                  * (3 * x**6 - 27 * x**4 * y**2 + 33 * x**2 * y**4 - y**6))
    F[(9, -9, "rooted")] = lambda x, y, z: (s(461890 / pi) / 512 * y * p(y, s(3) * x)
                                            * p(y, t9[0] * x) * p(y, t9[1] * x) * p(y, t9[2] * x))
    F[(9, -8)] = lambda x, y, z: (mp.mpf(3) / 32 * s(230945 / pi) * x * y * z * p(x, y)
                                  * p((1 + s(2)) * x, y) * p((1 - s(2)) * x, y))
    F[(9, -7)] = lambda x, y, z: (-mp.mpf(3) / 512 * s(27170 / pi) * p(1, s(17) * z) * y
                                  * poly7(x, y))
    F[(9, -7, "printed")] = lambda x, y, z: (-mp.mpf(3) / 512 * s(27170 / pi) * p(1, s(17) * z)
                                             * poly7(x, y))
    F[(9, -7, "rooted")] = lambda x, y, z: (mp.mpf(3) / 512 * s(27170 / pi) * y
                                            * p(1, s(17) * z) * p(y, t7[0] * x)
                                            * p(y, t7[1] * x) * p(y, t7[2] * x))
    F[(9, -6)] = lambda x, y, z: (s(81510 / pi) / 64 * x * y * z * p(x, s(3) * y)
                                  * p(s(3) * x, y) * p(s(17) * z, s(3)))
    F[(9, -5)] = lambda x, y, z: (mp.mpf(255) / 256 * s(5434 / pi) * y
                                  * p(s(5 - 2 * s(5)) * x, y) * p(s(5 + 2 * s(5)) * x, y)
                                  * p(s((15 - 2 * s(35)) / 85), z)
                                  * p(s((15 + 2 * s(35)) / 85), z))
    F[(9, -4)] = lambda x, y, z: (mp.mpf(51) / 32 * s(95095 / pi) * x * y * z * p(x, y)
                                  * p(s((5 - 2 * s(2)) / 17), z) * p(s((5 + 2 * s(2)) / 17), z))
    F[(9, -3)] = lambda x, y, z: (s(43890 / pi) / 256 * y * p(s(3) * x, y)
                                  * (z * z * ((221 * z * z - 195) * z * z + 39) - 1))
    F[(9, -2)] = lambda x, y, z: (-mp.mpf(3) / 64 * s(2090 / pi) * x * y * z
                                  * ((z * z * (273 - 221 * z * z) - 91) * z * z + 7))
    F[(9, -1)] = lambda x, y, z: (mp.mpf(3) / 256 * s(95 / pi) * y
                                  * ((z * z * ((2431 * z * z - 4004) * z * z + 2002) - 308) * z * z
                                     + 7))
    r91 = [mp.mpf("0.16527895766638702462621976595817353"),
           mp.mpf("0.47792494981044449566117509273125800"),
           mp.mpf("0.73877386510550507500310617485983073"),
           mp.mpf("0.91953390816645881382893266082233813")]
    F[(9, -1, "rooted")] = lambda x, y, z: (mp.mpf(7293) / 256 * s(95 / pi) * y
                                            * p(r91[0], z) * p(r91[1], z) * p(r91[2], z)
                                            * p(r91[3], z))
    F[(9, 0)] = lambda x, y, z: (s(19 / pi) / 256 * z
                                 * ((z * z * ((12155 * z * z - 25740) * z * z + 18018) - 4620)
                                    * z * z + 315))
    r90 = [mp.mpf("0.32425342340380892903853801464333661"),
           mp.mpf("0.61337143270059039730870203934147418"),
           mp.mpf("0.83603110732663579429942978806973488"),
           mp.mpf("0.96816023950762608983557620290367287")]
    F[(9, 0, "rooted")] = lambda x, y, z: (mp.mpf(12155) / 256 * s(19 / pi) * z
                                           * p(r90[0], z) * p(r90[1], z) * p(r90[2], z)
                                           * p(r90[3], z))
    return F


FORMS = None


def forms():
    global FORMS
    if FORMS is None:
        FORMS = _forms()
    return FORMS


def positive_m(l: int, m: int, x, y, z):
    """R_l^m for m > 0 from the m < 0 formula by the Appendix B rotations:
    odd m: pi/2 rotation with sign (-1)^n, m = 2n+1 (eq. rsymm90);
    m = 2(2n+1): pi/4 rotation with sign (-1)^n (eq. rsymm45);
    other m (4, 8): rotation of the (x, y) pair by pi/(2m) (eq. rsymm)."""
    f = forms()[(l, -m)]
    if m % 2 == 1:
        n = (m - 1) // 2
        return (-1) ** n * f(-y, x, z)
    if (m // 2) % 2 == 1:
        n = (m // 2 - 1) // 2
        h = 1 / mp.sqrt(2)
        return (-1) ** n * f((x - y) * h, (x + y) * h, z)
    a = mp.pi / (2 * m)
    return f(mp.cos(a) * x - mp.sin(a) * y, mp.sin(a) * x + mp.cos(a) * y, z)
