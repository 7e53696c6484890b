"""MI355X real spherical harmonics (l <= 9) after arXiv 2510.05282 ("SHarmonic").

Python binding of libshmi.so.  The functions carry the names of the C ABI
(include/shmi.h) and only marshal arguments: they check tensor devices, dtypes
and shapes, allocate outputs with torch when none is given, and pass raw device
pointers and the current HIP stream to the library.  Every value is computed by
the library's HIP kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import ShError, check, lib

SH_LMAX = 9
SH_LMAX_REC = 24
SH_F64 = 0
SH_F32 = 1

__all__ = ["SH_F32", "SH_F64", "SH_LMAX", "SH_LMAX_REC", "Radial", "ShError", "SphericalHarmonics", "nfun", "row", "sh_eval",
           "sh_eval_angles", "sh_eval_angles_f32", "sh_eval_complex", "sh_eval_complex_f32",
           "sh_eval_spinor", "sh_eval_spinor_f32", "spinor_index", "sh_eval_complex_unit",
           "sh_eval_complex_angles", "sh_eval_spinor_unit", "sh_eval_spinor_angles",
           "SH_IN_XYZ", "SH_IN_UNIT", "SH_IN_ANGLES", "sh_eval_complex_rec", "sh_eval_spinor_rec",
           "sh_eval_f32", "sh_eval_grad", "sh_eval_grad_f32", "sh_eval_grad_rec", "sh_eval_grad_rec_f32",
           "sh_eval_jac", "sh_eval_ld",
           "sh_eval_rec", "sh_eval_rec_f32", "sh_eval_unit", "sh_eval_unit_f32",
           "sh_projectors", "sh_projectors_f32", "sh_projectors_noalloc", "sh_radial_create", "sh_radial_destroy",
           "sh_strerror", "spherical_harmonics"]


def nfun(lmax: int) -> int:
    """Number of (l, m) rows for l <= lmax."""
    return (lmax + 1) * (lmax + 1)


def row(l: int, m: int) -> int:
    """Row of (l, m) in every output: l*l + l + m."""
    return l * l + l + m


def _stream(dev: torch.device, stream) -> int:
    s = torch.cuda.current_stream(dev) if stream is None else stream
    return int(s.cuda_stream)


def _points(xyz: torch.Tensor, dtype: torch.dtype) -> int:
    if not isinstance(xyz, torch.Tensor) or not xyz.is_cuda:
        raise TypeError("xyz must be a CUDA (HIP) tensor")
    if xyz.dtype != dtype:
        raise TypeError(f"xyz must be {dtype}, got {xyz.dtype}")
    if xyz.dim() != 2 or xyz.shape[1] != 3 or not xyz.is_contiguous():
        raise ValueError("xyz must be a contiguous [n, 3] tensor")
    return xyz.shape[0]


def _dtype_code(dtype: torch.dtype) -> int:
    if dtype == torch.float64:
        return SH_F64
    if dtype == torch.float32:
        return SH_F32
    raise TypeError("only float64 and float32 are supported")


def sh_eval_ld(lmax: int, xyz: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
    """R_l^m for l <= lmax into ``out``, a [F, n] view whose rows may be padded
    (out.stride(0) = ld >= n, out.stride(1) = 1).  dtype is taken from xyz."""
    code = _dtype_code(xyz.dtype)
    n = _points(xyz, xyz.dtype)
    F = nfun(lmax)
    if out.dtype != xyz.dtype or out.device != xyz.device:
        raise TypeError("out must match xyz in dtype and device")
    if out.dim() != 2 or out.shape[0] != F or out.shape[1] != n or (n > 1 and out.stride(1) != 1):
        raise ValueError(f"out must be a [{F}, {n}] view with unit column stride")
    ld = out.stride(0) if F > 1 else max(n, 1)
    with torch.cuda.device(xyz.device):
        check("sh_eval_ld", lib().sh_eval_ld(lmax, n, xyz.data_ptr(), out.data_ptr(), ld, code,
                                             _stream(xyz.device, stream)))
    return out


def _eval(fn: str, dtype: torch.dtype, lmax: int, xyz: torch.Tensor, out, stream) -> torch.Tensor:
    n = _points(xyz, dtype)
    F = nfun(lmax)
    if out is None:
        out = torch.empty((F, n), dtype=dtype, device=xyz.device)
    elif (out.dtype != dtype or out.device != xyz.device or tuple(out.shape) != (F, n)
          or not out.is_contiguous()):
        raise ValueError(f"out must be a contiguous [{F}, {n}] {dtype} tensor on {xyz.device}")
    with torch.cuda.device(xyz.device):
        check(fn, getattr(lib(), fn)(lmax, n, xyz.data_ptr(), out.data_ptr(),
                                     _stream(xyz.device, stream)))
    return out


def sh_eval(lmax: int, xyz: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Real harmonics R_l^m, l <= lmax, of float64 points xyz [n, 3] -> [F, n] float64."""
    return _eval("sh_eval", torch.float64, lmax, xyz, out, stream)


def sh_eval_f32(lmax: int, xyz: torch.Tensor, out: torch.Tensor | None = None,
                stream=None) -> torch.Tensor:
    """Single-precision twin of sh_eval (normalisation still in FP64)."""
    return _eval("sh_eval_f32", torch.float32, lmax, xyz, out, stream)


def sh_eval_rec(lmax: int, xyz: torch.Tensor, out: torch.Tensor | None = None, stream=None):
    """Real harmonics for lmax <= 24 by recurrence (float64), layout as sh_eval."""
    return _eval("sh_eval_rec", torch.float64, lmax, xyz, out, stream)


def sh_eval_rec_f32(lmax: int, xyz: torch.Tensor, out: torch.Tensor | None = None, stream=None):
    """Single-precision twin of sh_eval_rec (normalisation in FP64)."""
    return _eval("sh_eval_rec_f32", torch.float32, lmax, xyz, out, stream)


def sh_eval_unit(lmax: int, xyz: torch.Tensor, out: torch.Tensor | None = None, stream=None):
    """Like sh_eval for points already on the unit sphere (no normalisation)."""
    return _eval("sh_eval_unit", torch.float64, lmax, xyz, out, stream)


def sh_eval_unit_f32(lmax: int, xyz: torch.Tensor, out: torch.Tensor | None = None, stream=None):
    return _eval("sh_eval_unit_f32", torch.float32, lmax, xyz, out, stream)


def _angles(fn, dtype, lmax, theta, phi, out, stream):
    for name, t in (("theta", theta), ("phi", phi)):
        if not t.is_cuda or t.dtype != dtype or t.dim() != 1 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous 1-D {dtype} CUDA tensor")
    n = theta.shape[0]
    if phi.shape[0] != n:
        raise ValueError("theta and phi must have the same length")
    F = nfun(lmax)
    if out is None:
        out = torch.empty((F, n), dtype=dtype, device=theta.device)
    elif out.dtype != dtype or tuple(out.shape) != (F, n) or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous [{F}, {n}] {dtype} tensor")
    with torch.cuda.device(theta.device):
        check(fn, getattr(lib(), fn)(lmax, n, theta.data_ptr(), phi.data_ptr(), out.data_ptr(),
                                     _stream(theta.device, stream)))
    return out


def sh_eval_angles(lmax: int, theta: torch.Tensor, phi: torch.Tensor, out=None, stream=None):
    """Real harmonics at polar angles theta[n] and azimuths phi[n] (float64)."""
    return _angles("sh_eval_angles", torch.float64, lmax, theta, phi, out, stream)


def sh_eval_angles_f32(lmax: int, theta: torch.Tensor, phi: torch.Tensor, out=None, stream=None):
    return _angles("sh_eval_angles_f32", torch.float32, lmax, theta, phi, out, stream)


def _complex(fn, dtype, ctype, lmax, xyz, out, stream):
    n = _points(xyz, dtype)
    F = nfun(lmax)
    if out is None:
        out = torch.empty((F, n), dtype=ctype, device=xyz.device)
    elif out.dtype != ctype or tuple(out.shape) != (F, n) or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous [{F}, {n}] {ctype} tensor")
    with torch.cuda.device(xyz.device):
        check(fn, getattr(lib(), fn)(lmax, n, xyz.data_ptr(), out.data_ptr(), _stream(xyz.device, stream)))
    return out


def sh_eval_complex(lmax: int, xyz: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    """Complex harmonics Y_l^m [F, n] (complex128) of float64 points."""
    return _complex("sh_eval_complex", torch.float64, torch.complex128, lmax, xyz, out, stream)


def sh_eval_complex_f32(lmax: int, xyz: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    """Complex harmonics [F, n] (complex64) of float32 points."""
    return _complex("sh_eval_complex_f32", torch.float32, torch.complex64, lmax, xyz, out, stream)


def spinor_index(l: int, twice_j: int, twice_mj: int) -> int:
    """Row of the spinor harmonic (l, j = twice_j/2, m_j = twice_mj/2) in the
    output of sh_eval_spinor: l-major, j = l - 1/2 before j = l + 1/2, m_j ascending."""
    if twice_j == 2 * l + 1:
        return 2 * l * l + 2 * l + (twice_mj + 2 * l + 1) // 2
    if twice_j == 2 * l - 1 and l >= 1:
        return 2 * l * l + (twice_mj + 2 * l - 1) // 2
    raise ValueError(f"no spinor harmonic with l={l}, 2j={twice_j}")


def _spinor(fn, dtype, ctype, lmax, xyz, out, stream):
    n = _points(xyz, dtype)
    S = 2 * (lmax + 1) ** 2
    if out is None:
        out = torch.empty((S, 2, n), dtype=ctype, device=xyz.device)
    elif out.dtype != ctype or tuple(out.shape) != (S, 2, n) or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous [{S}, 2, {n}] {ctype} tensor")
    with torch.cuda.device(xyz.device):
        check(fn, getattr(lib(), fn)(lmax, n, xyz.data_ptr(), out.data_ptr(), _stream(xyz.device, stream)))
    return out


def sh_eval_spinor(lmax: int, xyz: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    """Spin-1/2 spinor harmonics [2 (lmax+1)^2, 2, n] (complex128) of float64 points;
    the middle index is the spin component (0 = up)."""
    return _spinor("sh_eval_spinor", torch.float64, torch.complex128, lmax, xyz, out, stream)


def sh_eval_spinor_f32(lmax: int, xyz: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    """Spinor harmonics [2 (lmax+1)^2, 2, n] (complex64) of float32 points."""
    return _spinor("sh_eval_spinor_f32", torch.float32, torch.complex64, lmax, xyz, out, stream)


SH_IN_XYZ, SH_IN_UNIT, SH_IN_ANGLES = 0, 1, 2


def _cplx_in(fn: str, spinor: bool, lmax: int, input_kind: int, a: torch.Tensor, b, out, stream):
    """Complex (spinor=False) or spinor harmonics through the any-input entry points;
    the dtype (float64 -> complex128, float32 -> complex64) is taken from ``a``."""
    code = _dtype_code(a.dtype)
    if input_kind == SH_IN_ANGLES:
        if not (a.is_cuda and isinstance(b, torch.Tensor) and b.is_cuda and a.dim() == 1 and b.shape == a.shape
                and b.dtype == a.dtype and a.is_contiguous() and b.is_contiguous()):
            raise ValueError("theta and phi must be contiguous 1-D CUDA tensors of one shape and dtype")
        n = a.shape[0]
    else:
        n = _points(a, a.dtype)
    ctype = torch.complex128 if a.dtype == torch.float64 else torch.complex64
    shape = (2 * (lmax + 1) ** 2, 2, n) if spinor else (nfun(lmax), n)
    if out is None:
        out = torch.empty(shape, dtype=ctype, device=a.device)
    elif out.dtype != ctype or tuple(out.shape) != shape or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous {list(shape)} {ctype} tensor")
    with torch.cuda.device(a.device):
        check(fn, getattr(lib(), fn)(lmax, n, input_kind, code, a.data_ptr(),
                                     b.data_ptr() if input_kind == SH_IN_ANGLES else None, out.data_ptr(),
                                     _stream(a.device, stream)))
    return out


def sh_eval_complex_rec(lmax: int, a: torch.Tensor, b: torch.Tensor | None = None, input_kind: int = SH_IN_XYZ,
                        out=None, stream=None) -> torch.Tensor:
    """Complex harmonics for lmax <= 24 by recurrence; a = xyz or unit vectors [n, 3],
    or a = theta and b = phi with input_kind = SH_IN_ANGLES."""
    return _cplx_in("sh_eval_complex_rec", False, lmax, input_kind, a, b, out, stream)


def sh_eval_spinor_rec(lmax: int, a: torch.Tensor, b: torch.Tensor | None = None, input_kind: int = SH_IN_XYZ,
                       out=None, stream=None) -> torch.Tensor:
    """Spinor harmonics for lmax <= 24 by recurrence; inputs as sh_eval_complex_rec."""
    return _cplx_in("sh_eval_spinor_rec", True, lmax, input_kind, a, b, out, stream)


def sh_eval_complex_unit(lmax: int, u: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    """Complex harmonics of points already on the unit sphere (float64 or float32)."""
    return _cplx_in("sh_eval_complex_in", False, lmax, SH_IN_UNIT, u, None, out, stream)


def sh_eval_complex_angles(lmax: int, theta: torch.Tensor, phi: torch.Tensor, out=None, stream=None):
    """Complex harmonics at polar angles theta and azimuths phi (float64 or float32)."""
    return _cplx_in("sh_eval_complex_in", False, lmax, SH_IN_ANGLES, theta, phi, out, stream)


def sh_eval_spinor_unit(lmax: int, u: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    """Spinor harmonics of points already on the unit sphere."""
    return _cplx_in("sh_eval_spinor_in", True, lmax, SH_IN_UNIT, u, None, out, stream)


def sh_eval_spinor_angles(lmax: int, theta: torch.Tensor, phi: torch.Tensor, out=None, stream=None):
    """Spinor harmonics at polar angles theta and azimuths phi."""
    return _cplx_in("sh_eval_spinor_in", True, lmax, SH_IN_ANGLES, theta, phi, out, stream)


def _grad(fn: str, dtype, lmax, xyz, grad_out, grad_xyz, stream):
    n = _points(xyz, dtype)
    F = nfun(lmax)
    if (grad_out.dtype != dtype or grad_out.device != xyz.device
            or tuple(grad_out.shape) != (F, n) or not grad_out.is_contiguous()):
        raise ValueError(f"grad_out must be a contiguous [{F}, {n}] {dtype} tensor on {xyz.device}")
    if grad_xyz is None:
        grad_xyz = torch.empty((n, 3), dtype=dtype, device=xyz.device)
    elif (grad_xyz.dtype != dtype or grad_xyz.device != xyz.device
          or tuple(grad_xyz.shape) != (n, 3) or not grad_xyz.is_contiguous()):
        raise ValueError(f"grad_xyz must be a contiguous [{n}, 3] {dtype} tensor on {xyz.device}")
    with torch.cuda.device(xyz.device):
        check(fn, getattr(lib(), fn)(lmax, n, xyz.data_ptr(), grad_out.data_ptr(), grad_xyz.data_ptr(),
                                     _stream(xyz.device, stream)))
    return grad_xyz


def sh_eval_grad(lmax: int, xyz: torch.Tensor, grad_out: torch.Tensor,
                 grad_xyz: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Backward of sh_eval: grad_xyz[i, k] = sum_f grad_out[f, i] dR_f(x_i)/dx_{i,k}.
    xyz [n, 3] and grad_out [F, n] float64 -> [n, 3] float64."""
    return _grad("sh_eval_grad", torch.float64, lmax, xyz, grad_out, grad_xyz, stream)


def sh_eval_grad_f32(lmax: int, xyz: torch.Tensor, grad_out: torch.Tensor,
                     grad_xyz: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Single-precision twin of sh_eval_grad (normalisation and 1/r in FP64)."""
    return _grad("sh_eval_grad_f32", torch.float32, lmax, xyz, grad_out, grad_xyz, stream)


def sh_eval_jac(lmax: int, xyz: torch.Tensor, out: torch.Tensor | None = None,
                jac: torch.Tensor | None = None, stream=None):
    """Values [F, n] and Jacobian [3, F, n] (jac[k, f, i] = dR_f(x_i)/dx_{i,k}) in one pass."""
    n = _points(xyz, torch.float64)
    F = nfun(lmax)
    if out is None:
        out = torch.empty((F, n), dtype=torch.float64, device=xyz.device)
    if jac is None:
        jac = torch.empty((3, F, n), dtype=torch.float64, device=xyz.device)
    for name, t, shape in (("out", out, (F, n)), ("jac", jac, (3, F, n))):
        if (t.dtype != torch.float64 or t.device != xyz.device or tuple(t.shape) != shape
                or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {list(shape)} float64 tensor on {xyz.device}")
    with torch.cuda.device(xyz.device):
        check("sh_eval_jac", lib().sh_eval_jac(lmax, n, xyz.data_ptr(), out.data_ptr(), jac.data_ptr(),
                                               _stream(xyz.device, stream)))
    return out, jac


def sh_eval_grad_rec(lmax: int, xyz: torch.Tensor, grad_out: torch.Tensor, grad_xyz=None, stream=None):
    """Backward pass of sh_eval_rec (lmax <= 24, float64)."""
    return _grad("sh_eval_grad_rec", torch.float64, lmax, xyz, grad_out, grad_xyz, stream)


def sh_eval_grad_rec_f32(lmax: int, xyz: torch.Tensor, grad_out: torch.Tensor, grad_xyz=None, stream=None):
    """Backward pass of sh_eval_rec_f32 (lmax <= 24, float32)."""
    return _grad("sh_eval_grad_rec_f32", torch.float32, lmax, xyz, grad_out, grad_xyz, stream)


class SphericalHarmonics(torch.autograd.Function):
    """R_l^m(xyz) for l <= lmax as a differentiable op: forward is sh_eval
    (sh_eval_f32 for float32 points), the gradient with respect to the points is
    sh_eval_grad (sh_eval_grad_f32); for 9 < lmax <= 24 the recurrence entries
    sh_eval_rec(_f32) and sh_eval_grad_rec(_f32)."""

    @staticmethod
    def forward(ctx, xyz: torch.Tensor, lmax: int) -> torch.Tensor:
        xyz = xyz.contiguous()
        ctx.lmax = lmax
        ctx.save_for_backward(xyz)
        f64 = xyz.dtype == torch.float64
        if lmax > SH_LMAX:
            return sh_eval_rec(lmax, xyz) if f64 else sh_eval_rec_f32(lmax, xyz)
        return sh_eval(lmax, xyz) if f64 else sh_eval_f32(lmax, xyz)

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        (xyz,) = ctx.saved_tensors
        g = grad_out.contiguous()
        f64 = xyz.dtype == torch.float64
        if ctx.lmax > SH_LMAX:
            return (sh_eval_grad_rec if f64 else sh_eval_grad_rec_f32)(ctx.lmax, xyz, g), None
        return (sh_eval_grad if f64 else sh_eval_grad_f32)(ctx.lmax, xyz, g), None


def spherical_harmonics(xyz: torch.Tensor, lmax: int) -> torch.Tensor:
    """Differentiable real harmonics [F, n] of float64 or float32 points [n, 3],
    lmax <= 24 (explicit formulas up to 9, the recurrence beyond)."""
    return SphericalHarmonics.apply(xyz, lmax)


class Radial:
    """Device radial tables (a C `sh_radial_t` handle).  values: host array
    [n_tables][lmax+1][n_r] of R_l at the knots i * r_max / (n_r - 1)."""

    def __init__(self, values, r_max: float):
        v = np.ascontiguousarray(values, dtype=np.float64)
        if v.ndim == 2:
            v = v[None]
        if v.ndim != 3:
            raise ValueError("values must be [n_tables][lmax+1][n_r]")
        self.n_tables, ch, self.n_r = v.shape
        self.lmax = ch - 1
        self.r_max = float(r_max)
        h = ctypes.c_void_p()
        check("sh_radial_create", lib().sh_radial_create(self.lmax, self.n_tables, self.n_r, self.r_max,
                                                        v.ctypes.data, ctypes.byref(h)))
        self.handle = h

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and self.handle.value:
            check("sh_radial_destroy", lib().sh_radial_destroy(self.handle))
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sh_radial_create(values, r_max: float) -> Radial:
    return Radial(values, r_max)


def sh_radial_destroy(radial: Radial) -> None:
    radial.close()


def _projectors(fn: str, dtype, lmax, centers, offsets, points, radial, table_of_atom, out, stream):
    for name, t in (("centers", centers), ("points", points)):
        if not t.is_cuda or t.dtype != dtype or t.dim() != 2 or t.shape[1] != 3 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous [*, 3] {dtype} CUDA tensor")
    n_atoms = centers.shape[0]
    if (offsets.dtype != torch.int64 or not offsets.is_cuda or tuple(offsets.shape) != (n_atoms + 1,)
            or not offsets.is_contiguous()):
        raise ValueError(f"offsets must be a contiguous int64 CUDA tensor of {n_atoms + 1} entries")
    n_points = points.shape[0]
    F = nfun(lmax)
    if out is None:
        out = torch.empty(F * n_points, dtype=dtype, device=points.device)
    elif out.dtype != dtype or out.numel() != F * n_points or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous {dtype} tensor of {F * n_points} elements")
    toa = 0
    if table_of_atom is not None:
        if (table_of_atom.dtype != torch.int32 or not table_of_atom.is_cuda
                or tuple(table_of_atom.shape) != (n_atoms,) or not table_of_atom.is_contiguous()):
            raise ValueError("table_of_atom must be a contiguous int32 CUDA tensor of n_atoms entries")
        toa = table_of_atom.data_ptr()
    with torch.cuda.device(points.device):
        check(fn, getattr(lib(), fn)(lmax, n_atoms, centers.data_ptr(), offsets.data_ptr(), n_points,
                                     points.data_ptr(), radial.handle, toa or None, out.data_ptr(),
                                     _stream(points.device, stream)))
    return out


def sh_projectors(lmax: int, centers: torch.Tensor, offsets: torch.Tensor, points: torch.Tensor,
                  radial: Radial, table_of_atom: torch.Tensor | None = None,
                  out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Projectors R_l(|p - c_a|) R_l^m(p - c_a) for every atom (float64); returns the
    flat output in which atom a's [F][n_a] block starts at F * offsets[a]."""
    return _projectors("sh_projectors", torch.float64, lmax, centers, offsets, points, radial,
                       table_of_atom, out, stream)


def sh_projectors_f32(lmax: int, centers: torch.Tensor, offsets: torch.Tensor, points: torch.Tensor,
                      radial: Radial, table_of_atom: torch.Tensor | None = None,
                      out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Single-precision twin of sh_projectors (float32 centers, points, output)."""
    return _projectors("sh_projectors_f32", torch.float32, lmax, centers, offsets, points, radial,
                       table_of_atom, out, stream)


def sh_projectors_noalloc(lmax: int, centers: torch.Tensor, offsets: torch.Tensor, points: torch.Tensor,
                          values: torch.Tensor, r_max: float, table_of_atom: torch.Tensor | None = None,
                          out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """The projector build from radial knot values (a float64 CUDA tensor
    [n_tables, lmax + 1, n_r] on the uniform grid over [0, r_max]) instead of a
    Radial handle; the library allocates nothing (its working arrays live in a
    static device buffer).  centers, points and out are float64 or float32 (the
    dtype of points); pass `out` to keep the call free of allocation here too."""
    dtype = points.dtype
    if dtype not in (torch.float64, torch.float32):
        raise TypeError("points must be float64 or float32")
    if (not values.is_cuda or values.dtype != torch.float64 or values.dim() != 3 or values.shape[1] != lmax + 1
            or not values.is_contiguous()):
        raise ValueError(f"values must be a contiguous float64 CUDA tensor [n_tables, {lmax + 1}, n_r]")
    for name, t in (("centers", centers), ("points", points)):
        if not t.is_cuda or t.dtype != dtype or t.dim() != 2 or t.shape[1] != 3 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous [*, 3] {dtype} CUDA tensor")
    n_atoms = centers.shape[0]
    if (offsets.dtype != torch.int64 or not offsets.is_cuda or tuple(offsets.shape) != (n_atoms + 1,)
            or not offsets.is_contiguous()):
        raise ValueError(f"offsets must be a contiguous int64 CUDA tensor of {n_atoms + 1} entries")
    n_points = points.shape[0]
    F = nfun(lmax)
    if out is None:
        out = torch.empty(F * n_points, dtype=dtype, device=points.device)
    elif out.dtype != dtype or out.numel() != F * n_points or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous {dtype} tensor of {F * n_points} elements")
    toa = 0
    if table_of_atom is not None:
        if (table_of_atom.dtype != torch.int32 or not table_of_atom.is_cuda
                or tuple(table_of_atom.shape) != (n_atoms,) or not table_of_atom.is_contiguous()):
            raise ValueError("table_of_atom must be a contiguous int32 CUDA tensor of n_atoms entries")
        toa = table_of_atom.data_ptr()
    code = SH_F64 if dtype == torch.float64 else SH_F32
    with torch.cuda.device(points.device):
        check("sh_projectors_noalloc",
              lib().sh_projectors_noalloc(lmax, code, n_atoms, centers.data_ptr(), offsets.data_ptr(), n_points,
                                          points.data_ptr(), values.shape[0], values.shape[2], float(r_max),
                                          values.data_ptr(), toa or None, out.data_ptr(),
                                          _stream(points.device, stream)))
    return out


def sh_strerror(code: int) -> str:
    return lib().sh_strerror(code).decode()
