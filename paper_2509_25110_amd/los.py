"""ctypes binding of liblos.so (C ABI in include/los.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of liblos.so.  PyTorch is used for device memory and streams: tensors
are passed by ``data_ptr()`` and the stream is the caller's current
``torch.cuda`` stream.  Importing this module raises if the library has not
been built (``python -m paper_2509_25110_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblos.so")

LOS_OK = 0
LOS_ERR_INVALID = 1
LOS_ERR_HIP = 2
LOS_ERR_OOM = 3
LOS_ERR_UNSUPPORTED = 4
LOS_ERR_NUMERIC = 5

LOS_FP64 = 0
LOS_FP32 = 1
LOS_BF16X3 = 2

_STATUS = {1: "LOS_ERR_INVALID", 2: "LOS_ERR_HIP", 3: "LOS_ERR_OOM", 4: "LOS_ERR_UNSUPPORTED",
           5: "LOS_ERR_NUMERIC"}

# every symbol include/los.h declares
EXPORTS = ("los_last_error", "los_version", "los_ctx_create", "los_ctx_destroy",
           "los_bessel_table", "los_project", "cl_integrate")


class LosError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_STATUS.get(code, "?"), code, msg))
        self.code = code


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load liblos.so and declare its signatures (no GPU call is made)."""
    if not os.path.exists(path):
        raise ImportError("liblos.so not built at %s; run python -m paper_2509_25110_amd.build" % path)
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.los_last_error.restype = ctypes.c_char_p
    lib.los_last_error.argtypes = []
    lib.los_version.restype = ctypes.c_char_p
    lib.los_version.argtypes = []
    lib.los_ctx_create.restype = ctypes.c_int
    lib.los_ctx_create.argtypes = [ctypes.POINTER(vp)]
    lib.los_ctx_destroy.restype = None
    lib.los_ctx_destroy.argtypes = [vp]
    lib.los_bessel_table.restype = ctypes.c_int
    lib.los_bessel_table.argtypes = [vp, vp, i64, i32, i32, vp, vp]
    lib.los_project.restype = ctypes.c_int
    lib.los_project.argtypes = [vp, i32, i32, i64, i64, dbl, vp, vp, vp, vp, i32, i32, vp, vp]
    lib.cl_integrate.restype = ctypes.c_int
    lib.cl_integrate.argtypes = [vp, vp, i32, i32, i32, i64, vp, vp,
                                 ctypes.POINTER(ctypes.c_int32), i32, vp, vp]
    return lib


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


def _check(rc: int):
    if rc != LOS_OK:
        raise LosError(rc, lib().los_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _need(t: torch.Tensor, dtype, numel: int, name: str):
    if t.dtype != dtype:
        raise ValueError("%s must be %s (got %s)" % (name, dtype, t.dtype))
    if t.numel() != numel:
        raise ValueError("%s must have %d elements (got %d)" % (name, numel, t.numel()))


class Context:
    """A los_ctx (device workspace owner) bound to the current device."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(lib().los_ctx_create(ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            lib().los_ctx_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- entry points (same names as the C ABI) ----

    def los_bessel_table(self, x: torch.Tensor, lmin: int, lmax: int,
                         out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        nx = x.numel()
        if out is None:
            out = torch.empty((lmax - lmin + 1, nx), dtype=torch.float64, device=x.device)
        _need(x, torch.float64, nx, "x")
        _need(out, torch.float64, (lmax - lmin + 1) * nx, "out")
        _check(lib().los_bessel_table(self._h, _ptr(x), nx, lmin, lmax, _ptr(out), _stream(stream)))
        return out

    def los_project(self, lmin: int, lmax: int, k: torch.Tensor, tau: torch.Tensor, tau0: float,
                    w_tau: torch.Tensor, S: torch.Tensor, prec: int = LOS_FP64,
                    delta: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        nsrc, nk, ntau = S.shape
        nl = lmax - lmin + 1
        want = torch.float64 if prec == LOS_FP64 else torch.float32
        if S.dtype != want:
            raise ValueError("S must be %s for precision %d (got %s)" % (want, prec, S.dtype))
        if delta is None:
            delta = torch.empty((nk, nl, nsrc), dtype=S.dtype, device=S.device)
        _need(k, torch.float64, nk, "k")
        _need(tau, torch.float64, ntau, "tau")
        _need(w_tau, torch.float64, ntau, "w_tau")
        _need(delta, S.dtype, nk * nl * nsrc, "delta")
        _check(lib().los_project(self._h, lmin, lmax, nk, ntau, float(tau0), _ptr(k), _ptr(tau),
                                 _ptr(w_tau), _ptr(S), nsrc, prec, _ptr(delta), _stream(stream)))
        return delta

    def cl_integrate(self, delta: torch.Tensor, w_lnk: torch.Tensor, Pk: torch.Tensor,
                     pairs: Sequence[Tuple[int, int]], cl: Optional[torch.Tensor] = None,
                     stream=None) -> torch.Tensor:
        nk, nl, nsrc = delta.shape
        prec = LOS_FP64 if delta.dtype == torch.float64 else LOS_FP32
        flat = [int(v) for p in pairs for v in p]
        npairs = len(flat) // 2
        arr = (ctypes.c_int32 * len(flat))(*flat)
        if cl is None:
            cl = torch.empty((npairs, nl), dtype=torch.float64, device=delta.device)
        _need(w_lnk, torch.float64, nk, "w_lnk")
        _need(Pk, torch.float64, nk, "Pk")
        _need(cl, torch.float64, npairs * nl, "cl")
        _check(lib().cl_integrate(self._h, _ptr(delta), prec, nsrc, nl, nk, _ptr(w_lnk), _ptr(Pk),
                                  arr, npairs, _ptr(cl), _stream(stream)))
        return cl


def version() -> str:
    return lib().los_version().decode()
