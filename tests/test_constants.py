"""The generated constants of the GPU formulas (csrc/sh_constants.h) against the
roots and tangents the paper prints in Appendix C (closed forms and 35-39 digit
numerical roots)."""
from __future__ import annotations

import math
import os
import re

import numpy as np
import pytest

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2510_05282_amd", "csrc", "sh_constants.h")


def _array(name):
    text = open(HDR).read()
    m = re.search(r"constexpr (?:double|float) " + name + r"\[[^=]*=\s*(\{.*?\});", text, re.S)
    assert m, name
    nums = [float(v.rstrip("f")) for v in re.findall(r"-?\d+\.\d+(?:e-?\d+)?f?", m.group(1))]
    return np.array(nums)


@pytest.fixture(scope="module")
def roots():
    return _array("kZRoot").reshape(10, 10, 4)


def _close(a, b, rel=2e-16):
    assert abs(a - b) <= rel * abs(b), (a, b)


def test_printed_numerical_roots(roots):
    # R_8^-1 (rooted form), R_9^-1, R_9^0: roots of d^m P_l / dz^m
    for got, want in [
        (roots[8, 1, :3], ["0.36311746382617815871075206870865921", "0.67718627951073775344588542709134245",
                           "0.89975799541146015731234524441833796"]),
        (roots[9, 1, :4], ["0.16527895766638702462621976595817353", "0.47792494981044449566117509273125800",
                           "0.73877386510550507500310617485983073", "0.91953390816645881382893266082233813"]),
        (roots[9, 0, :4], ["0.32425342340380892903853801464333661", "0.61337143270059039730870203934147418",
                           "0.83603110732663579429942978806973488", "0.96816023950762608983557620290367287"]),
    ]:
        for g, w in zip(got, want):
            _close(g, float(w))


def test_closed_form_roots(roots):
    s = math.sqrt
    cases = {
        (2, 0): [1 / s(3)], (3, 0): [s(3 / 5)], (3, 1): [1 / s(5)],
        (4, 0): [s((3 - 2 * s(6 / 5)) / 7), s((3 + 2 * s(6 / 5)) / 7)],
        (4, 1): [s(3 / 7)], (4, 2): [1 / s(7)],
        (5, 0): [s(5 - 2 * s(10 / 7)) / 3, s(5 + 2 * s(10 / 7)) / 3],  # reading: /3 outside the root
        (5, 1): [s((7 - 2 * s(7)) / 21), s((7 + 2 * s(7)) / 21)],
        (5, 3): [1 / 3],
        (6, 2): [s((3 - 4 / s(3)) / 11), s((3 + 4 / s(3)) / 11)],
        (6, 1): [s((15 - 2 * s(15)) / 33), s((15 + 2 * s(15)) / 33)],
        (6, 3): [s(3 / 11)], (6, 4): [1 / s(11)],
        (7, 3): [s((33 - 2 * s(165)) / 143), s((33 + 2 * s(165)) / 143)],
        (7, 2): [s((55 - 4 * s(55)) / 143), s((55 + 4 * s(55)) / 143)],
        (7, 4): [s(3 / 13)], (7, 5): [1 / s(13)],
        (8, 4): [s((13 - 2 * s(26)) / 65), s((13 + 2 * s(26)) / 65)],
        (8, 3): [s((1 - 2 / s(13)) / 3), s((1 + 2 / s(13)) / 3)],
        (8, 5): [1 / s(5)], (8, 6): [1 / s(15)],
        (9, 5): [s((15 - 2 * s(35)) / 85), s((15 + 2 * s(35)) / 85)],
        (9, 4): [s((5 - 2 * s(2)) / 17), s((5 + 2 * s(2)) / 17)],
        (9, 6): [s(3 / 17)], (9, 7): [1 / s(17)],
    }
    for (l, m), want in cases.items():
        for g, w in zip(roots[l, m, : len(want)], want):
            _close(g, w, rel=1e-15)


def test_tangents_of_the_xy_factors():
    ts = _array("kTanS").reshape(10, 4)
    tc = _array("kTanC").reshape(10, 4)
    printed7 = ["0.481574618807528644332162353056970575219", "1.253960337662703837570910978336464443221",
                "4.381286267534823072404689085032695444150"]
    for g, w in zip(ts[7, :3], printed7):
        _close(g, float(w))
    printed9 = ["0.363970234266202361351047882776834043890", "0.839099631177280011763127298123181364687",
                math.sqrt(3), "5.671281819617709530994418439863964421625"]
    for g, w in zip(ts[9, :4], printed9):
        _close(g, float(w), rel=3e-16)
    _close(ts[3, 0], math.sqrt(3))
    _close(ts[5, 0], math.sqrt(5 - 2 * math.sqrt(5)), rel=1e-15)
    _close(ts[5, 1], math.sqrt(5 + 2 * math.sqrt(5)), rel=1e-15)
    _close(tc[4, 0], math.sqrt(2) - 1, rel=1e-15)  # cos(4 phi) zero lines: tan(pi/8), tan(3pi/8)
    _close(tc[4, 1], math.sqrt(2) + 1, rel=1e-15)
