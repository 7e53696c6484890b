"""Python binding of the projector server (sh_server_* in include/shmi.h)."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import ServerStats, check, lib

SH_F64, SH_F32 = 0, 1
SH_REQ_AUTORELEASE = 1
PENDING, QUEUED, RUNNING, DONE, FAILED, RELEASED = range(6)


class Server:
    """Continuous-batching projector server.  `simulated=True` uses the
    executor that computes nothing (scheduling tests without a GPU)."""

    def __init__(self, budget_bytes: int, max_pending: int = 1 << 16, n_slots: int = 3,
                 simulated: bool = False, sim_bytes_per_s: float = 5e12, sim_fail_every: int = 0,
                 sim_launch_s: float = 0.0):
        h = ctypes.c_void_p()
        if simulated:
            check("sh_server_create_simulated",
                  lib().sh_server_create_simulated(int(budget_bytes), max_pending, n_slots,
                                                   float(sim_bytes_per_s), sim_fail_every,
                                                   float(sim_launch_s), ctypes.byref(h)))
        else:
            check("sh_server_create", lib().sh_server_create(int(budget_bytes), max_pending, n_slots,
                                                             ctypes.byref(h)))
        self.handle = h
        self._keep = []  # tensors whose memory registered atoms point into

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().sh_server_destroy(self.handle)
        self.handle = None
        self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_atom(self, points, center, radial=None, table: int = 0, dtype: int | None = None,
                 n: int | None = None) -> int:
        """Registers an atom.  points: a contiguous [n, 3] CUDA tensor (float64 or
        float32), kept alive by the server object; or, for a simulated server, any
        nonzero integer address with explicit n and dtype."""
        if isinstance(points, torch.Tensor):
            if not points.is_cuda or points.dim() != 2 or points.shape[1] != 3 or not points.is_contiguous():
                raise ValueError("points must be a contiguous [n, 3] CUDA tensor")
            dtype = SH_F64 if points.dtype == torch.float64 else SH_F32
            if points.dtype not in (torch.float64, torch.float32):
                raise TypeError("points must be float64 or float32")
            n, ptr = points.shape[0], points.data_ptr()
            self._keep.append(points)
        else:
            ptr = int(points)
        c = (ctypes.c_double * 3)(*[float(v) for v in np.asarray(center).ravel()[:3]])
        aid = ctypes.c_int()
        check("sh_server_add_atom", lib().sh_server_add_atom(self.handle, dtype, int(n), ptr, c,
                                                             radial.handle if radial is not None else None,
                                                             table, ctypes.byref(aid)))
        if radial is not None:
            self._keep.append(radial)
        return aid.value

    def submit(self, atom: int, lmax: int, flags: int = 0) -> int:
        """Returns a ticket; raises ShError (status 4, SH_EBUSY) on back-pressure."""
        t = ctypes.c_int64()
        check("sh_server_submit", lib().sh_server_submit(self.handle, atom, lmax, flags, ctypes.byref(t)))
        return t.value

    def try_submit(self, atom: int, lmax: int, flags: int = 0) -> tuple[int, int]:
        """(status, ticket) without raising."""
        t = ctypes.c_int64(-1)
        rc = lib().sh_server_submit(self.handle, atom, lmax, flags, ctypes.byref(t))
        return rc, t.value

    def poll(self, ticket: int) -> int:
        s = ctypes.c_int()
        check("sh_server_poll", lib().sh_server_poll(self.handle, ticket, ctypes.byref(s)))
        return s.value

    def wait(self, ticket: int, timeout_s: float = 60.0) -> int:
        s = ctypes.c_int()
        check("sh_server_wait", lib().sh_server_wait(self.handle, ticket, timeout_s, ctypes.byref(s)))
        return s.value

    def result_ptr(self, ticket: int) -> int:
        p = ctypes.c_void_p()
        check("sh_server_result", lib().sh_server_result(self.handle, ticket, ctypes.byref(p)))
        return p.value or 0

    def result(self, ticket: int, lmax: int, n: int, dtype: torch.dtype) -> torch.Tensor:
        """The finished request's [F, n] output as a tensor that aliases the
        server's memory (valid until release; clone() it to keep it)."""
        F = (lmax + 1) ** 2
        typestr = "<f8" if dtype == torch.float64 else "<f4"
        return torch.as_tensor(_DeviceArray(self.result_ptr(ticket), (F, n), typestr), device="cuda")

    def release(self, ticket: int) -> None:
        """Returns a finished request's output memory to the server, which may give
        it to the next request's kernel at once: the work already queued on the
        current torch stream (a clone() of the result, say) is waited for first."""
        if torch.cuda.is_available() and torch.cuda.is_initialized():
            torch.cuda.current_stream().synchronize()
        check("sh_server_release", lib().sh_server_release(self.handle, ticket))

    def drain(self, timeout_s: float = 600.0) -> None:
        check("sh_server_drain", lib().sh_server_drain(self.handle, timeout_s))

    def stats(self) -> dict:
        s = ServerStats()
        check("sh_server_stats", lib().sh_server_stats(self.handle, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in ServerStats._fields_}

    def latencies_ms(self) -> np.ndarray:
        n = lib().sh_server_latencies(self.handle, None, 0)
        out = np.empty(max(n, 0), dtype=np.float64)
        if n > 0:
            lib().sh_server_latencies(self.handle, out.ctypes.data, n)
        return out


class _DeviceArray:
    """Describes server-owned device memory to torch (no copy)."""

    def __init__(self, ptr: int, shape: tuple, typestr: str):
        self.__cuda_array_interface__ = {"shape": shape, "typestr": typestr, "data": (ptr, False),
                                         "strides": None, "version": 3}
