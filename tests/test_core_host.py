"""CPU checks of the GPU formula core (sh_core.h built for the host) and of its
generated constants, against the oracle.  No GPU is involved: this catches a
wrong constant or factor before any kernel runs."""
from __future__ import annotations

import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2510_05282_amd import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LD = np.longdouble


@pytest.fixture(scope="module")
def core(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    so = str(tmp_path_factory.mktemp("core") / "core_check.so")
    subprocess.check_call([hipcc, "-x", "hip", "--cuda-host-only", "-O2", "-std=c++17", "-fPIC",
                           "-shared", os.path.join(ROOT, "tests", "host", "core_check.hip"),
                           "-o", so], stderr=subprocess.DEVNULL)
    L = ctypes.CDLL(so)
    for fn in ("core_eval9_f64", "core_eval9_f32", "core_eval3_f64"):
        getattr(L, fn).argtypes = [ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p]
    return L


def _units(pts, dtype):
    p = pts.astype(LD)
    r = np.sqrt((p * p).sum(1, keepdims=True))
    return np.ascontiguousarray((p / r).astype(dtype))


def _run(core, fn, u, F, dtype):
    out = np.empty((F, u.shape[0]), dtype=dtype)
    getattr(core, fn)(u.shape[0], u.ctypes.data, out.ctypes.data)
    return out


def _pts():
    sp = workloads.special_points()
    sp = sp[(sp * sp).sum(1) > 0]
    near_pole = np.array([[1e-12, 3e-12, 1.0], [-2e-8, 1e-8, -1.0], [1e-5, 0.0, 1.0]])
    return np.concatenate([workloads.isotropic_points(20000, 0.1, 5.0, seed=31), sp, near_pole])


def test_core_fp64_matches_oracle(core, orc):
    u = _units(_pts(), np.float64)
    got = _run(core, "core_eval9_f64", u, 100, np.float64)
    ref = orc.eval_xyz(9, u)
    err = np.abs(got.astype(LD) - ref).max(axis=1)
    assert err.max() <= 1e-13, err.max()
    # the explicit forms are as accurate as the paper reports (about 1e-14 at l = 9)
    assert err.max() <= 3e-14


def test_core_lower_lmax_is_a_prefix(core):
    u = _units(_pts()[:500], np.float64)
    a = _run(core, "core_eval9_f64", u, 100, np.float64)
    b = _run(core, "core_eval3_f64", u, 16, np.float64)
    assert np.array_equal(a[:16], b)


def test_core_fp32_matches_oracle(core, orc):
    u = _units(_pts(), np.float32)
    got = _run(core, "core_eval9_f32", u, 100, np.float32)
    ref = orc.eval_xyz(9, u)  # at the float unit vectors, widened exactly
    err = np.abs(got.astype(LD) - ref).max(axis=1)
    assert err.max() <= 5e-6, err.max()


@pytest.mark.parametrize("lmax,fn", [(9, "core_grad9"), (6, "core_grad6")])
def test_core_gradient_matches_oracle(core, orc, lmax, fn):
    """Dual-number gradient of the factorised forms, projected on the tangent
    plane, against the oracle's analytic gradient (unit points, r = 1)."""
    getattr(core, fn).argtypes = [ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    u = _units(_pts(), np.float64)
    F = (lmax + 1) ** 2
    G = np.random.default_rng(41).standard_normal((F, u.shape[0]))
    out = np.empty((u.shape[0], 3))
    getattr(core, fn)(u.shape[0], u.ctypes.data, G.ctypes.data, out.ctypes.data)
    ref = orc.grad_xyz(lmax, u, G)
    scale = 1 + np.abs(ref).max(axis=1, keepdims=True)
    err = (np.abs(out.astype(LD) - ref) / scale).max()
    assert err <= 1e-12, err


def test_core_gradient_fp32(core, orc):
    core.core_grad9_f32.argtypes = [ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    u = _units(_pts(), np.float32)
    G = np.random.default_rng(42).standard_normal((100, u.shape[0])).astype(np.float32)
    out = np.empty((u.shape[0], 3), dtype=np.float32)
    core.core_grad9_f32(u.shape[0], u.ctypes.data, G.ctypes.data, out.ctypes.data)
    ref = orc.grad_xyz(9, u.astype(np.float64), G.astype(np.float64))
    scale = 1 + np.abs(ref).max(axis=1, keepdims=True)
    err = (np.abs(out.astype(LD) - ref) / scale).max()
    assert err <= 2e-5, err


def test_core_values_and_jacobian(core, orc):
    core.core_jac9.argtypes = [ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    u = _units(_pts()[:5000], np.float64)
    n = u.shape[0]
    val = np.empty((100, n))
    jac = np.empty((3, 100, n))
    core.core_jac9(n, u.ctypes.data, val.ctypes.data, jac.ctypes.data)
    assert np.abs(val.astype(LD) - orc.eval_xyz(9, u)).max() <= 3e-14
    J = orc.jacobian_xyz(9, u)
    assert np.abs(jac.astype(LD) - J).max() <= 1e-12 * (1 + float(np.abs(J).max()))


@pytest.mark.parametrize("lmax", [0, 1, 9, 16, 24])
def test_core_recurrence(core, orc, lmax):
    core.core_rec.argtypes = [ctypes.c_long, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    u = _units(_pts()[:20000], np.float64)
    F = (lmax + 1) ** 2
    out = np.empty((F, u.shape[0]))
    core.core_rec(u.shape[0], u.ctypes.data, lmax, out.ctypes.data)
    err = np.abs(out.astype(LD) - orc.eval_xyz(lmax, u)).max()
    assert err <= 1e-13, err


def test_core_complex(core, orc):
    core.core_complex9.argtypes = [ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p]
    u = _units(_pts()[:20000], np.float64)
    out = np.full((100, u.shape[0], 2), np.nan)
    core.core_complex9(u.shape[0], u.ctypes.data, out.ctypes.data)
    re, im = orc.eval_complex_xyz(9, u)
    assert np.abs(out[..., 0].astype(LD) - re).max() <= 1e-13
    assert np.abs(out[..., 1].astype(LD) - im).max() <= 1e-13


@pytest.mark.parametrize("lmax", [0, 1, 4, 9])
def test_core_spinor(core, orc, lmax):
    """Spinor core: every (spinor, component) written exactly once, values equal
    to the oracle's composition of eq. spinorial."""
    core.core_spinor.argtypes = [ctypes.c_long, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                 ctypes.c_void_p]
    u = _units(_pts()[:5000], np.float64)
    S = 2 * (lmax + 1) ** 2
    out = np.full((S, 2, u.shape[0], 2), np.nan)
    count = np.zeros((S, 2, u.shape[0]), dtype=np.int32)
    core.core_spinor(u.shape[0], u.ctypes.data, lmax, out.ctypes.data, count.ctypes.data)
    assert (count == 1).all()
    re, im = orc.eval_spinor_xyz(lmax, u)
    assert np.abs(out[..., 0].astype(LD) - re).max() <= 1e-13
    assert np.abs(out[..., 1].astype(LD) - im).max() <= 1e-13


def test_core_spline_interleaved_tables(core, orc):
    """The device spline (solve and lookup in the channel-interleaved table layout)
    against the oracle's natural spline, every channel of several tables: FP64
    within 1e-13, and the FP32 lookup from float-rounded pairs within 5e-7 (the
    tables are scaled to max|R_l| = 1)."""
    core.core_spline4.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_int,
                                  ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    rng = np.random.default_rng(12)
    n_tables, n_r, r_max = 3, 257, 3.0
    y = np.stack([workloads.radial_table(rng, 3, n_r, r_max) for _ in range(n_tables)])
    y = np.ascontiguousarray(y)
    knots = np.linspace(0.0, r_max, n_r)
    r = np.concatenate([rng.uniform(0, r_max, 4000), knots, [r_max, r_max * (1 + 1e-12), 4.0, 0.0]])
    for t in range(n_tables):
        out = np.empty((r.shape[0], 4))
        core.core_spline4(n_tables, n_r, r_max, y.ctypes.data, t, r.shape[0], r.ctypes.data, out.ctypes.data, 0)
        out32 = np.empty((r.shape[0], 4))
        core.core_spline4(n_tables, n_r, r_max, y.ctypes.data, t, r.shape[0], r.ctypes.data, out32.ctypes.data, 1)
        for l in range(4):
            M = orc.spline_setup(y[t, l], r_max)
            ref = orc.spline_eval(y[t, l], M, r_max, r)
            assert np.abs(out[:, l].astype(LD) - ref).max() <= 1e-13, (t, l)
            assert np.abs(out32[:, l].astype(LD) - ref).max() <= 5e-7, (t, l)


@pytest.mark.parametrize("lmax", [9, 24])
def test_core_recurrence_fp32(core, orc, lmax):
    """FP32 recurrence core at float unit vectors: per-l error <= 5e-6 up to l = 9
    and 1e-6 (l + 1) beyond, against the oracle at the same float vectors."""
    core.core_rec_f32.argtypes = [ctypes.c_long, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    u = _units(_pts()[:20000], np.float32)
    F = (lmax + 1) ** 2
    out = np.empty((F, u.shape[0]), dtype=np.float32)
    core.core_rec_f32(u.shape[0], u.ctypes.data, lmax, out.ctypes.data)
    err = np.abs(out.astype(LD) - orc.eval_xyz(lmax, u)).max(axis=1)
    for l in range(lmax + 1):
        assert err[l * l:(l + 1) * (l + 1)].max() <= (5e-6 if l <= 9 else 1e-6 * (l + 1)), l


@pytest.mark.parametrize("lmax", [0, 9, 17, 24])
def test_core_complex_and_spinor_by_recurrence(core, orc, lmax):
    """Complex and spinor harmonics built on the recurrence core, against the
    oracle's complex definition and its eq. spinorial composition; every spinor
    entry written exactly once."""
    core.core_complex_rec.argtypes = [ctypes.c_long, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    core.core_spinor_rec.argtypes = [ctypes.c_long, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_void_p]
    u = _units(_pts()[:3000], np.float64)
    n, F, S = u.shape[0], (lmax + 1) ** 2, 2 * (lmax + 1) ** 2
    out = np.full((F, n, 2), np.nan)
    core.core_complex_rec(n, u.ctypes.data, lmax, out.ctypes.data)
    re, im = orc.eval_complex_xyz(lmax, u)
    assert np.abs(out[..., 0].astype(LD) - re).max() <= 1e-13
    assert np.abs(out[..., 1].astype(LD) - im).max() <= 1e-13
    sp = np.full((S, 2, n, 2), np.nan)
    count = np.zeros((S, 2, n), dtype=np.int32)
    core.core_spinor_rec(n, u.ctypes.data, lmax, sp.ctypes.data, count.ctypes.data)
    assert (count == 1).all()
    sre, sim = orc.eval_spinor_xyz(lmax, u)
    assert np.abs(sp[..., 0].astype(LD) - sre).max() <= 1e-13
    assert np.abs(sp[..., 1].astype(LD) - sim).max() <= 1e-13


@pytest.mark.parametrize("lmax", [9, 24])
def test_core_gradient_by_recurrence(core, orc, lmax):
    """Recurrence on dual numbers: the contracted gradient at unit vectors against
    the oracle, |dg|_inf <= 1e-12 (1 + |g|_inf) (FP64) and 2e-5 / 5e-6 (lmax + 1) (FP32)."""
    for fn in ("core_grad_rec", "core_grad_rec_f32"):
        getattr(core, fn).argtypes = [ctypes.c_long, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                      ctypes.c_void_p]
    u = _units(_pts()[:3000], np.float64)
    F = (lmax + 1) ** 2
    G = np.random.default_rng(lmax).standard_normal((F, u.shape[0]))
    out = np.empty((u.shape[0], 3))
    core.core_grad_rec(u.shape[0], u.ctypes.data, lmax, G.ctypes.data, out.ctypes.data)
    ref = orc.grad_xyz(lmax, u, G)
    scale = 1 + np.abs(ref.astype(np.float64)).max(axis=1)
    assert (np.abs(out.astype(LD) - ref).max(axis=1) / scale).max() <= 1e-12
    u32, G32 = u.astype(np.float32), G.astype(np.float32)
    out32 = np.empty((u.shape[0], 3), dtype=np.float32)
    core.core_grad_rec_f32(u.shape[0], u32.ctypes.data, lmax, G32.ctypes.data, out32.ctypes.data)
    ref32 = orc.grad_xyz(lmax, u32.astype(np.float64), G32.astype(np.float64))
    scale32 = 1 + np.abs(ref32.astype(np.float64)).max(axis=1)
    tol = 2e-5 if lmax <= 9 else 5e-6 * (lmax + 1)
    assert (np.abs(out32.astype(LD) - ref32).max(axis=1) / scale32).max() <= tol
