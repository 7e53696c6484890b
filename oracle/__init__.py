"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Python access (ctypes) to ``sh_oracle.c``, the plain long-double reference for the
real spherical harmonics, their Cartesian gradient, the natural cubic radial spline
and the projector build.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the GPU library never does.

Every result is returned as ``numpy.longdouble`` so that callers round to double
exactly once, at the comparison.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sh_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

LD = np.longdouble
if np.finfo(LD).nmant < 63:  # pragma: no cover - x86-64 always has 80-bit long double
    raise RuntimeError("the oracle needs x87 extended precision long double")


def build(force: bool = True) -> str:
    """Compile the oracle shared library with gcc (OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        i64, i32, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        L.orc_eval_xyz.argtypes = [i32, i64, vp, vp]
        L.orc_eval_xyz_f32.argtypes = [i32, i64, vp, vp]
        L.orc_eval_xyz_maxerr.argtypes = [i32, i64, vp, vp, i64, vp]
        L.orc_eval_angles.argtypes = [i32, i64, vp, vp, vp]
        L.orc_jacobian_xyz.argtypes = [i32, i64, vp, vp]
        L.orc_grad_xyz.argtypes = [i32, i64, vp, vp, vp]
        L.orc_spline_setup.argtypes = [i32, ctypes.c_double, vp, vp]
        L.orc_spline_eval.argtypes = [i32, ctypes.c_double, vp, vp, i64, vp, vp]
        L.orc_projectors.argtypes = [i32, i32, vp, vp, vp, vp, i32, ctypes.c_double, vp, vp, vp]
        L.orc_num_threads.restype = i32
        L.orc_eval_complex_xyz.argtypes = [i32, i64, vp, vp, vp]
        L.orc_eval_complex_angles.argtypes = [i32, i64, vp, vp, vp, vp]
        _lib = L
    return _lib


def num_threads() -> int:
    """OpenMP threads the oracle's batch loops use."""
    return int(lib().orc_num_threads())


def set_num_threads(k: int) -> None:
    """Use k OpenMP threads in later batch calls."""
    lib().orc_set_num_threads(int(k))


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (code {rc})")


def nfun(lmax: int) -> int:
    return (lmax + 1) * (lmax + 1)


def row(l: int, m: int) -> int:
    """Flat index of (l, m): l-major, m ascending from -l to l."""
    return l * l + l + m


def eval_xyz_maxerr(lmax: int, xyz, got) -> np.ndarray:
    """Largest |got[row][i] - R_row(xyz_i)| per l over all points, for outputs too
    large to hold in long double; got is a [F][>= n] float64 array (rows may be
    longer than n).  Returns float64 [lmax + 1]."""
    a = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1, 3))
    g = np.asarray(got)
    if g.dtype != np.float64 or g.ndim != 2 or g.shape[0] != nfun(lmax) or g.shape[1] < a.shape[0] \
            or g.strides[1] != 8:
        raise ValueError("got must be a float64 [F][>= n] array with contiguous rows")
    err = np.zeros(lmax + 1)
    _check(lib().orc_eval_xyz_maxerr(lmax, a.shape[0], _p(a), ctypes.c_void_p(g.ctypes.data),
                                     ctypes.c_int64(g.strides[0] // 8), _p(err)), "eval_xyz_maxerr")
    return err


def eval_xyz(lmax: int, xyz) -> np.ndarray:
    """Real harmonics R_l^m at Cartesian points; returns [F][n] long double.

    float32 inputs are widened exactly (the FP32 error reference); anything else
    is converted to float64 first."""
    xyz = np.asarray(xyz)
    if xyz.dtype == np.float32:
        a = np.ascontiguousarray(xyz.reshape(-1, 3))
        out = np.empty((nfun(lmax), a.shape[0]), dtype=LD)
        _check(lib().orc_eval_xyz_f32(lmax, a.shape[0], _p(a), _p(out)), "eval_xyz_f32")
        return out
    a = np.ascontiguousarray(xyz.reshape(-1, 3), dtype=np.float64)
    out = np.empty((nfun(lmax), a.shape[0]), dtype=LD)
    _check(lib().orc_eval_xyz(lmax, a.shape[0], _p(a), _p(out)), "eval_xyz")
    return out


def eval_complex_xyz(lmax: int, xyz):
    """Complex harmonics Y_l^m at Cartesian points; returns (re, im), each [F][n]
    long double."""
    a = np.ascontiguousarray(np.asarray(xyz).reshape(-1, 3), dtype=np.float64)
    re = np.empty((nfun(lmax), a.shape[0]), dtype=LD)
    im = np.empty_like(re)
    _check(lib().orc_eval_complex_xyz(lmax, a.shape[0], _p(a), _p(re), _p(im)), "eval_complex_xyz")
    return re, im


def eval_complex_angles(lmax: int, theta, phi):
    """Complex harmonics at polar angle theta and azimuth phi; returns (re, im),
    each [F][n] long double."""
    t = np.ascontiguousarray(np.atleast_1d(theta), dtype=LD)
    f = np.ascontiguousarray(np.atleast_1d(phi), dtype=LD)
    assert t.shape == f.shape
    re = np.empty((nfun(lmax), t.shape[0]), dtype=LD)
    im = np.empty_like(re)
    _check(lib().orc_eval_complex_angles(lmax, t.shape[0], _p(t), _p(f), _p(re), _p(im)), "eval_complex_angles")
    return re, im


def spinor_index(l: int, kappa: int, twice_mj: int) -> int:
    """Index of the spinor harmonic with orbital l, j = l + kappa/2 (kappa = +1 or -1)
    and m_j = twice_mj / 2: l-major, j = l - 1/2 before j = l + 1/2, m_j ascending."""
    base = 2 * l * l
    if kappa < 0:
        return base + (twice_mj + 2 * l - 1) // 2
    return base + 2 * l + (twice_mj + 2 * l + 1) // 2


def eval_spinor_xyz(lmax: int, xyz):
    """Spinor harmonics (paper eq. spinorial) from the complex definition, for
    l <= lmax: returns (re, im), each [2 (lmax+1)^2][2][n] long double, component 0
    the upper (spin up) one.  For j = l + 1/2 and j = l - 1/2 (l >= 1):
        upper = +- sqrt(l +- m_j + 1/2) Y_l^{m_j - 1/2} / sqrt(2l + 1)
        lower =    sqrt(l -+ m_j + 1/2) Y_l^{m_j + 1/2} / sqrt(2l + 1)
    with Y_l^m = 0 for |m| > l."""
    return _spinor_from_complex(lmax, *eval_complex_xyz(lmax, xyz))


def eval_spinor_angles(lmax: int, theta, phi):
    """Spinor harmonics at polar angle theta and azimuth phi, as eval_spinor_xyz."""
    return _spinor_from_complex(lmax, *eval_complex_angles(lmax, theta, phi))


def _spinor_from_complex(lmax: int, re_y, im_y):
    """eq. spinorial applied to the complex harmonics re_y + i im_y [F][n]."""
    n = re_y.shape[1]
    ns = 2 * (lmax + 1) ** 2
    re = np.zeros((ns, 2, n), dtype=LD)
    im = np.zeros((ns, 2, n), dtype=LD)

    def y(l, m2):  # m2 = 2m (odd m_j +- 1/2 -> integer m)
        m = m2 // 2
        if abs(m) > l:
            return np.zeros(n, dtype=LD), np.zeros(n, dtype=LD)
        return re_y[l * l + l + m], im_y[l * l + l + m]

    for l in range(lmax + 1):
        den = np.sqrt(LD(2 * l + 1))
        for kappa in (-1, 1):
            if kappa < 0 and l == 0:
                continue
            j2 = 2 * l + kappa
            for mj2 in range(-j2, j2 + 1, 2):
                k = spinor_index(l, kappa, mj2)
                ur, ui = y(l, mj2 - 1)
                lr, li = y(l, mj2 + 1)
                if kappa > 0:
                    cu = np.sqrt(LD(2 * l + mj2 + 1) / 2) / den
                    cl = np.sqrt(LD(2 * l - mj2 + 1) / 2) / den
                else:
                    cu = -np.sqrt(LD(2 * l - mj2 + 1) / 2) / den
                    cl = np.sqrt(LD(2 * l + mj2 + 1) / 2) / den
                re[k, 0], im[k, 0] = cu * ur, cu * ui
                re[k, 1], im[k, 1] = cl * lr, cl * li
    return re, im


def eval_angles(lmax: int, theta, phi) -> np.ndarray:
    """Real harmonics at polar angle theta and azimuth phi; returns [F][n] long double."""
    t = np.ascontiguousarray(np.atleast_1d(theta), dtype=LD)
    f = np.ascontiguousarray(np.atleast_1d(phi), dtype=LD)
    assert t.shape == f.shape
    out = np.empty((nfun(lmax), t.shape[0]), dtype=LD)
    _check(lib().orc_eval_angles(lmax, t.shape[0], _p(t), _p(f), _p(out)), "eval_angles")
    return out


def jacobian_xyz(lmax: int, xyz) -> np.ndarray:
    """d R_l^m / d x_k; returns [3][F][n] long double."""
    a = np.ascontiguousarray(np.asarray(xyz).reshape(-1, 3), dtype=np.float64)
    out = np.empty((3, nfun(lmax), a.shape[0]), dtype=LD)
    _check(lib().orc_jacobian_xyz(lmax, a.shape[0], _p(a), _p(out)), "jacobian_xyz")
    return out


def grad_xyz(lmax: int, xyz, G) -> np.ndarray:
    """sum_f G[f][i] dR_f/dx_k at point i; returns [n][3] long double."""
    a = np.ascontiguousarray(np.asarray(xyz).reshape(-1, 3), dtype=np.float64)
    g = np.ascontiguousarray(G, dtype=np.float64)
    assert g.shape == (nfun(lmax), a.shape[0])
    out = np.empty((a.shape[0], 3), dtype=LD)
    _check(lib().orc_grad_xyz(lmax, a.shape[0], _p(a), _p(g), _p(out)), "grad_xyz")
    return out


def spline_setup(y, r_max: float) -> np.ndarray:
    """Second derivatives M of the natural cubic spline through y on the uniform
    grid [0, r_max]; returns long double [n_r]."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    M = np.empty(y.shape[0], dtype=LD)
    _check(lib().orc_spline_setup(y.shape[0], float(r_max), _p(y), _p(M)), "spline_setup")
    return M


def spline_eval(y, M, r_max: float, r) -> np.ndarray:
    y = np.ascontiguousarray(y, dtype=np.float64)
    M = np.ascontiguousarray(M, dtype=LD)
    rr = np.ascontiguousarray(np.atleast_1d(r), dtype=LD)
    out = np.empty(rr.shape[0], dtype=LD)
    _check(lib().orc_spline_eval(y.shape[0], float(r_max), _p(y), _p(M), rr.shape[0],
                                 _p(rr), _p(out)), "spline_eval")
    return out


def projectors(lmax: int, centers, offsets, points, tables, r_max: float,
               table_of_atom=None) -> np.ndarray:
    """Projector arrays for every atom, concatenated: atom a's [F][n_a] block
    starts at flat offset F*offsets[a].  ``tables`` is [n_tables][lmax+1][n_r]
    radial values on the uniform grid [0, r_max]; ``table_of_atom[a]`` picks the
    table of atom a (default: table a)."""
    c = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 3)
    n_atoms = c.shape[0]
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    p = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
    t = np.ascontiguousarray(tables, dtype=np.float64)
    assert t.ndim == 3 and t.shape[1] == lmax + 1
    n_r = t.shape[2]
    if table_of_atom is None:
        table_of_atom = np.arange(n_atoms)
    toa = np.ascontiguousarray(table_of_atom, dtype=np.int32)
    assert off.shape == (n_atoms + 1,) and p.shape[0] == off[-1]
    Ms = np.empty(t.shape, dtype=LD)
    for k in range(t.shape[0]):
        for l in range(lmax + 1):
            Ms[k, l] = spline_setup(t[k, l], r_max)
    out = np.empty(nfun(lmax) * int(off[-1]), dtype=LD)
    _check(lib().orc_projectors(lmax, n_atoms, _p(c), _p(off), _p(p), _p(toa), n_r,
                                float(r_max), _p(t), _p(Ms), _p(out)), "projectors")
    return out
