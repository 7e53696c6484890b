"""Loader of libshmi.so (ctypes).

torch is imported first on purpose: it loads its own HIP runtime
(libamdhip64.so.7), and the dynamic linker then binds libshmi.so to that same
runtime, so device pointers and stream handles from torch are valid in the
library.  There is no fallback: without the built library every call fails.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (must precede the CDLL load, see above)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libshmi.so")

_lib = None


class ServerStats(ctypes.Structure):
    """Mirror of sh_server_stats_t."""
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("deferred", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("points_done", ctypes.c_int64),
                ("bytes_in_use", ctypes.c_uint64), ("peak_bytes", ctypes.c_uint64),
                ("first_submit_s", ctypes.c_double), ("last_done_s", ctypes.c_double),
                ("scheduler_cpu_s", ctypes.c_double)]


class ShError(RuntimeError):
    """A libshmi call returned a nonzero status."""

    def __init__(self, fn: str, code: int, hip: int = 0):
        self.code = code
        self.hip = hip
        msg = f"{fn} failed: {lib().sh_strerror(code).decode()} (status {code})"
        if hip:
            msg += f", hipError {hip}"
        super().__init__(msg)


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2510_05282_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    i32, i64, vp = ctypes.c_int, ctypes.c_int64, ctypes.c_void_p
    L.sh_eval.argtypes = [i32, i64, vp, vp, vp]
    L.sh_eval.restype = i32
    L.sh_eval_f32.argtypes = [i32, i64, vp, vp, vp]
    L.sh_eval_f32.restype = i32
    L.sh_eval_ld.argtypes = [i32, i64, vp, vp, i64, i32, vp]
    L.sh_eval_ld.restype = i32
    for fn in ("sh_eval_unit", "sh_eval_unit_f32", "sh_eval_complex", "sh_eval_complex_f32", "sh_eval_rec", "sh_eval_rec_f32",
               "sh_eval_spinor", "sh_eval_spinor_f32"):
        getattr(L, fn).argtypes = [i32, i64, vp, vp, vp]
        getattr(L, fn).restype = i32
    for fn in ("sh_eval_complex_in", "sh_eval_spinor_in", "sh_eval_complex_rec", "sh_eval_spinor_rec"):
        getattr(L, fn).argtypes = [i32, i64, i32, i32, vp, vp, vp, vp]
        getattr(L, fn).restype = i32
    for fn in ("sh_eval_angles", "sh_eval_angles_f32"):
        getattr(L, fn).argtypes = [i32, i64, vp, vp, vp, vp]
        getattr(L, fn).restype = i32
    L.sh_eval_grad.argtypes = [i32, i64, vp, vp, vp, vp]
    L.sh_eval_grad.restype = i32
    L.sh_eval_grad_f32.argtypes = [i32, i64, vp, vp, vp, vp]
    L.sh_eval_grad_f32.restype = i32
    L.sh_eval_jac.argtypes = [i32, i64, vp, vp, vp, vp]
    for fn in ("sh_eval_grad_rec", "sh_eval_grad_rec_f32"):
        getattr(L, fn).argtypes = [i32, i64, vp, vp, vp, vp]
        getattr(L, fn).restype = i32
    L.sh_eval_jac.restype = i32
    L.sh_radial_create.argtypes = [i32, i32, i32, ctypes.c_double, vp, ctypes.POINTER(vp)]
    L.sh_radial_create.restype = i32
    L.sh_radial_destroy.argtypes = [vp]
    L.sh_radial_destroy.restype = i32
    L.sh_projectors.argtypes = [i32, i32, vp, vp, i64, vp, vp, vp, vp, vp]
    L.sh_projectors.restype = i32
    L.sh_projectors_f32.argtypes = [i32, i32, vp, vp, i64, vp, vp, vp, vp, vp]
    L.sh_projectors_f32.restype = i32
    L.sh_projectors_noalloc.argtypes = [i32, i32, i32, vp, vp, i64, vp, i32, i32, ctypes.c_double, vp, vp, vp, vp]
    L.sh_projectors_noalloc.restype = i32
    u64, f64 = ctypes.c_uint64, ctypes.c_double
    L.sh_server_create.argtypes = [u64, i32, i32, ctypes.POINTER(vp)]
    L.sh_server_create_simulated.argtypes = [u64, i32, i32, f64, i32, f64, ctypes.POINTER(vp)]
    L.sh_server_destroy.argtypes = [vp]
    L.sh_server_add_atom.argtypes = [vp, i32, i64, vp, ctypes.POINTER(f64), vp, i32,
                                     ctypes.POINTER(i32)]
    L.sh_server_submit.argtypes = [vp, i32, i32, i32, ctypes.POINTER(i64)]
    L.sh_server_poll.argtypes = [vp, i64, ctypes.POINTER(i32)]
    L.sh_server_wait.argtypes = [vp, i64, f64, ctypes.POINTER(i32)]
    L.sh_server_result.argtypes = [vp, i64, ctypes.POINTER(vp)]
    L.sh_server_release.argtypes = [vp, i64]
    L.sh_server_drain.argtypes = [vp, f64]
    L.sh_server_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    L.sh_server_latencies.argtypes = [vp, vp, i64]
    L.sh_server_latencies.restype = i64
    for fn in ("sh_server_create", "sh_server_create_simulated", "sh_server_destroy", "sh_server_add_atom",
               "sh_server_submit", "sh_server_poll", "sh_server_wait", "sh_server_result",
               "sh_server_release", "sh_server_drain", "sh_server_stats"):
        getattr(L, fn).restype = i32
    L.sh_strerror.argtypes = [i32]
    L.sh_strerror.restype = ctypes.c_char_p
    L.sh_last_hip_error.argtypes = []
    L.sh_last_hip_error.restype = i32
    _lib = L
    return _lib


def check(fn: str, rc: int) -> None:
    if rc != 0:
        raise ShError(fn, rc, lib().sh_last_hip_error() if rc == 2 else 0)
