"""MI355X real spherical harmonics (l <= 9) after arXiv 2510.05282 ("SHarmonic").

Python binding of libshmi.so.  The functions carry the names of the C ABI
(include/shmi.h) and only marshal arguments: they check tensor devices, dtypes
and shapes, allocate outputs with torch when none is given, and pass raw device
pointers and the current HIP stream to the library.  Every value is computed by
the library's HIP kernels.
"""
from __future__ import annotations

import torch

from ._lib import ShError, check, lib

SH_LMAX = 9
SH_F64 = 0
SH_F32 = 1

__all__ = ["SH_LMAX", "ShError", "nfun", "row", "sh_eval", "sh_eval_f32", "sh_eval_ld",
           "sh_strerror"]


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


def sh_strerror(code: int) -> str:
    return lib().sh_strerror(code).decode()
