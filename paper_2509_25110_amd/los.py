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
           "los_bessel_table", "los_project", "los_project_kernels", "los_project_tensor",
           "cl_integrate", "cl_integrate_noalloc",
           "los_spline_sources", "los_interp_sources", "los_project_lsample", "los_cl_interp",
           "los_batch_create",
           "los_batch_columns", "los_batch_info", "los_batch_solve", "los_batch_solve_timed",
           "los_batch_destroy",
           "emu_create", "emu_destroy", "emu_nparams", "emu_get_params", "emu_set_params",
           "emu_get_pca", "emu_set_pca", "emu_forward", "emu_loss_grad", "emu_fit", "emu_train",
           "emu_infer", "emu_infer_spectra", "emu_merge", "emu_merge_spectrum", "emu_save",
           "emu_load")


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
    lib.los_ctx_create.argtypes = [ctypes.POINTER(vp), ctypes.c_char_p]
    lib.los_ctx_destroy.restype = None
    lib.los_ctx_destroy.argtypes = [vp]
    lib.los_bessel_table.restype = ctypes.c_int
    lib.los_bessel_table.argtypes = [vp, vp, i64, i32, i32, vp, vp]
    lib.los_project.restype = ctypes.c_int
    lib.los_project.argtypes = [vp, i32, i32, i64, i64, dbl, vp, vp, vp, vp, i32, i32, vp, vp]
    lib.los_project_kernels.restype = ctypes.c_int
    lib.los_project_kernels.argtypes = [vp, i32, i32, i64, i64, dbl, vp, vp, vp, vp, i32,
                                        ctypes.c_uint32, i32, vp, vp]
    lib.los_project_tensor.restype = ctypes.c_int
    lib.los_project_tensor.argtypes = [vp, i32, i32, i64, i64, dbl, vp, vp, vp, vp, vp, vp]
    lib.cl_integrate.restype = ctypes.c_int
    lib.cl_integrate.argtypes = [vp, vp, i32, i32, i32, i64, vp, vp,
                                 ctypes.POINTER(ctypes.c_int32), i32, vp, vp]
    lib.cl_integrate_noalloc.restype = ctypes.c_int
    lib.cl_integrate_noalloc.argtypes = [vp, vp, i32, i32, i32, i64, vp, vp,
                                         ctypes.POINTER(ctypes.c_int32), i32, vp, vp]
    lib.los_project_lsample.restype = ctypes.c_int
    lib.los_project_lsample.argtypes = [vp, i32, i32, ctypes.POINTER(ctypes.c_int32), i32, i64,
                                        i64, dbl, vp, vp, vp, vp, i32, ctypes.c_uint32, vp, vp]
    lib.los_cl_interp.restype = ctypes.c_int
    lib.los_cl_interp.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int32), i32, vp, i32, i32, vp,
                                  vp]
    lib.los_spline_sources.restype = ctypes.c_int
    lib.los_spline_sources.argtypes = [vp, i32, i64, i64, vp, vp, vp, vp]
    lib.los_interp_sources.restype = ctypes.c_int
    lib.los_interp_sources.argtypes = [vp, i32, i64, i64, vp, vp, vp, i64, vp, i32, vp, vp]
    lib.los_batch_create.restype = ctypes.c_int
    lib.los_batch_create.argtypes = [vp, i32, i32, vp, vp, vp, i64, i64, vp, i32, i32,
                                     ctypes.POINTER(vp)]
    lib.los_batch_columns.restype = ctypes.c_int
    lib.los_batch_columns.argtypes = [vp, vp, ctypes.POINTER(i64)]
    lib.los_batch_info.restype = ctypes.c_int
    lib.los_batch_info.argtypes = [vp, vp]
    lib.los_batch_solve.restype = ctypes.c_int
    lib.los_batch_solve.argtypes = [vp, dbl, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.los_batch_solve_timed.restype = ctypes.c_int
    lib.los_batch_solve_timed.argtypes = [vp, dbl, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.los_batch_destroy.restype = None
    lib.los_batch_destroy.argtypes = [vp]
    u64 = ctypes.c_uint64
    sig = {
        "emu_create": [vp, i32, i32, i32, i32, i32, i32, u64, ctypes.POINTER(vp)],
        "emu_nparams": [vp, ctypes.POINTER(i64)],
        "emu_get_params": [vp, i32, vp],
        "emu_set_params": [vp, i32, vp],
        "emu_get_pca": [vp, vp, vp, vp, vp, vp, vp],
        "emu_set_pca": [vp, vp, vp, vp, vp, vp, vp],
        "emu_forward": [vp, i32, vp, i64, vp, vp],
        "emu_loss_grad": [vp, i32, vp, vp, i64, vp, vp, vp],
        "emu_fit": [vp, i32, vp, vp, i64, i32, i32, dbl, vp, vp],
        "emu_train": [vp, vp, vp, vp, vp, i64, i32, i32, dbl, vp, vp],
        "emu_infer": [vp, vp, i64, vp, vp, vp, dbl, vp],
        "emu_infer_spectra": [vp, vp, i64, vp, vp, vp, dbl, vp],
        "emu_merge": [vp, vp, i64, vp, vp, i64, vp, vp, vp],
        "emu_merge_spectrum": [vp, i32, vp, i64, vp, vp, i64, vp, vp, vp],
        "emu_save": [vp, ctypes.c_char_p, vp],
        "emu_load": [vp, ctypes.c_char_p, ctypes.POINTER(vp)],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.restype = ctypes.c_int
        fn.argtypes = args
    lib.emu_destroy.restype = None
    lib.emu_destroy.argtypes = [vp]
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
    """A los_ctx (device workspace owner) bound to the current device; tune_cache (a file
    path) keeps the batch autotuner's choices across processes."""

    def __init__(self, tune_cache: Optional[str] = None):
        h = ctypes.c_void_p()
        _check(lib().los_ctx_create(ctypes.byref(h),
                                    os.fsencode(tune_cache) if tune_cache else None))
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

    def los_project_kernels(self, lmin: int, lmax: int, k: torch.Tensor, tau: torch.Tensor,
                            tau0: float, w_tau: torch.Tensor, S: torch.Tensor, kernel_mask: int,
                            prec: int = LOS_FP64, delta: Optional[torch.Tensor] = None,
                            stream=None) -> torch.Tensor:
        """los_project with the E-mode kernel eps_l for the sources set in kernel_mask."""
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
        _check(lib().los_project_kernels(self._h, lmin, lmax, nk, ntau, float(tau0), _ptr(k),
                                         _ptr(tau), _ptr(w_tau), _ptr(S), nsrc, int(kernel_mask),
                                         prec, _ptr(delta), _stream(stream)))
        return delta

    def los_project_tensor(self, lmin: int, lmax: int, k: torch.Tensor, tau: torch.Tensor,
                           tau0: float, w_tau: torch.Tensor, S: torch.Tensor,
                           delta: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """Tensor-mode projection: S is [2, nk, ntau] (S_T, S_P) float64; returns delta
        [nk, nl, 3] float64 (T, E, B)."""
        two, nk, ntau = S.shape
        if two != 2:
            raise ValueError("S must be [2, nk, ntau] (S_T, S_P)")
        nl = lmax - lmin + 1
        if delta is None:
            delta = torch.empty((nk, nl, 3), dtype=torch.float64, device=S.device)
        _need(S, torch.float64, 2 * nk * ntau, "S")
        _need(k, torch.float64, nk, "k")
        _need(tau, torch.float64, ntau, "tau")
        _need(w_tau, torch.float64, ntau, "w_tau")
        _need(delta, torch.float64, nk * nl * 3, "delta")
        _check(lib().los_project_tensor(self._h, lmin, lmax, nk, ntau, float(tau0), _ptr(k),
                                        _ptr(tau), _ptr(w_tau), _ptr(S), _ptr(delta),
                                        _stream(stream)))
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


    def cl_integrate_noalloc(self, delta: torch.Tensor, w_lnk: torch.Tensor, Pk: torch.Tensor,
                             pairs: Sequence[Tuple[int, int]], cl: torch.Tensor,
                             stream=None) -> torch.Tensor:
        """cl_integrate into a caller-supplied `cl`, with the library's fixed device scratch
        (no allocation by the library)."""
        nk, nl, nsrc = delta.shape
        prec = LOS_FP64 if delta.dtype == torch.float64 else LOS_FP32
        flat = [int(v) for p in pairs for v in p]
        npairs = len(flat) // 2
        arr = (ctypes.c_int32 * len(flat))(*flat)
        _need(w_lnk, torch.float64, nk, "w_lnk")
        _need(Pk, torch.float64, nk, "Pk")
        _need(cl, torch.float64, npairs * nl, "cl")
        _check(lib().cl_integrate_noalloc(self._h, _ptr(delta), prec, nsrc, nl, nk, _ptr(w_lnk),
                                          _ptr(Pk), arr, npairs, _ptr(cl), _stream(stream)))
        return cl

    def los_project_lsample(self, lmin: int, lmax: int, ls, k: torch.Tensor, tau: torch.Tensor,
                            tau0: float, w_tau: torch.Tensor, S: torch.Tensor, kernel_mask: int = 0,
                            delta: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """FP64 projection at the sampled multipoles ls (host list): delta[nk, len(ls), nsrc]."""
        nsrc, nk, ntau = S.shape
        lsl = [int(v) for v in ls]
        arr = (ctypes.c_int32 * len(lsl))(*lsl)
        if delta is None:
            delta = torch.empty((nk, len(lsl), nsrc), dtype=torch.float64, device=S.device)
        _need(S, torch.float64, nsrc * nk * ntau, "S")
        _need(k, torch.float64, nk, "k")
        _need(tau, torch.float64, ntau, "tau")
        _need(w_tau, torch.float64, ntau, "w_tau")
        _need(delta, torch.float64, nk * len(lsl) * nsrc, "delta")
        _check(lib().los_project_lsample(self._h, lmin, lmax, arr, len(lsl), nk, ntau, float(tau0),
                                         _ptr(k), _ptr(tau), _ptr(w_tau), _ptr(S), nsrc,
                                         int(kernel_mask), _ptr(delta), _stream(stream)))
        return delta

    def los_cl_interp(self, ls, cls: torch.Tensor, lmin: int, lmax: int,
                      cl: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """C_l at every l in [lmin, lmax] from cls[npairs, len(ls)] at the sampled ls."""
        lsl = [int(v) for v in ls]
        arr = (ctypes.c_int32 * len(lsl))(*lsl)
        npairs = cls.numel() // max(len(lsl), 1)
        nl = lmax - lmin + 1
        if cl is None:
            cl = torch.empty((npairs, nl), dtype=torch.float64, device=cls.device)
        _need(cls, torch.float64, npairs * len(lsl), "cls")
        _need(cl, torch.float64, npairs * nl, "cl")
        _check(lib().los_cl_interp(self._h, npairs, arr, len(lsl), _ptr(cls), lmin, lmax, _ptr(cl),
                                   _stream(stream)))
        return cl

    def los_spline_sources(self, q: torch.Tensor, Sc: torch.Tensor,
                           M: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """Natural-spline second derivatives in k of Sc[nsrc, nkc, ntau] on the knots q."""
        nsrc, nkc, ntau = Sc.shape
        if M is None:
            M = torch.empty_like(Sc)
        _need(q, torch.float64, nkc, "q")
        _need(Sc, torch.float64, nsrc * nkc * ntau, "Sc")
        _need(M, torch.float64, nsrc * nkc * ntau, "M")
        _check(lib().los_spline_sources(self._h, nsrc, nkc, ntau, _ptr(q), _ptr(Sc), _ptr(M),
                                        _stream(stream)))
        return M

    def los_interp_sources(self, q: torch.Tensor, Sc: torch.Tensor, M: torch.Tensor,
                           k: torch.Tensor, out_prec: int = LOS_FP64,
                           S: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """S[nsrc, nk, ntau]: the spline through Sc (second derivatives M) at k."""
        nsrc, nkc, ntau = Sc.shape
        nk = k.numel()
        dt = torch.float64 if out_prec == LOS_FP64 else torch.float32
        if S is None:
            S = torch.empty((nsrc, nk, ntau), dtype=dt, device=Sc.device)
        _need(q, torch.float64, nkc, "q")
        _need(Sc, torch.float64, nsrc * nkc * ntau, "Sc")
        _need(M, torch.float64, nsrc * nkc * ntau, "M")
        _need(k, torch.float64, nk, "k")
        _need(S, dt, nsrc * nk * ntau, "S")
        _check(lib().los_interp_sources(self._h, nsrc, nkc, ntau, _ptr(q), _ptr(Sc), _ptr(M), nk,
                                        _ptr(k), out_prec, _ptr(S), _stream(stream)))
        return S

    def los_batch_create(self, lmax, koff, k_index, nk_master: int, ntau: int,
                         pairs: Sequence[Tuple[int, int]], prec: int = LOS_BF16X3,
                         nsrc: int = 3) -> "Batch":
        """Plan a batch (host arrays); see Batch."""
        return Batch(self, lmax, koff, k_index, nk_master, ntau, pairs, prec, nsrc)


class Emulator:
    """A los_emu (entry points emu_*): ensemble MLP emulator of the 4 spectra."""

    def __init__(self, ctx: Context, nparam: int, nl: int, ncomp: int = 96, width: int = 512,
                 depth: int = 4, members: int = 4, seed: int = 1, _handle=None):
        if _handle is None:
            h = ctypes.c_void_p()
            _check(lib().emu_create(ctx.handle, nparam, nl, ncomp, width, depth, members, seed,
                                    ctypes.byref(h)))
        else:
            h = _handle
        self._h = h
        self.nparam, self.nl, self.ncomp, self.members = nparam, nl, ncomp, members
        self.width, self.depth, self.seed = width, depth, seed
        self.nout = 4 * ncomp
        n = ctypes.c_int64()
        _check(lib().emu_nparams(h, ctypes.byref(n)))
        self.nparams = int(n.value)

    def emu_get_params(self, member: int):
        import numpy as np
        out = np.empty(self.nparams, dtype=np.float32)
        _check(lib().emu_get_params(self._h, member, out.ctypes.data))
        return out

    def emu_set_params(self, member: int, theta):
        import numpy as np
        t = np.ascontiguousarray(theta, dtype=np.float32)
        if t.size != self.nparams:
            raise ValueError("expected %d parameters" % self.nparams)
        _check(lib().emu_set_params(self._h, member, t.ctypes.data))

    def emu_get_pca(self):
        import numpy as np
        lo = np.empty(self.nparam); hi = np.empty(self.nparam)
        mean = np.empty((4, self.nl)); basis = np.empty((4, self.nl, self.ncomp))
        sigma = np.empty((4, self.ncomp)); t = np.empty(self.nl)
        _check(lib().emu_get_pca(self._h, lo.ctypes.data, hi.ctypes.data, mean.ctypes.data,
                                 basis.ctypes.data, sigma.ctypes.data, t.ctypes.data))
        return dict(lo=lo, hi=hi, mean=mean, basis=basis, sigma=sigma, te_scale=t)

    def emu_set_pca(self, lo, hi, mean, basis, sigma, te_scale):
        import numpy as np
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (lo, hi, mean, basis, sigma,
                                                                    te_scale)]
        _check(lib().emu_set_pca(self._h, *[a.ctypes.data for a in arrs]))

    def emu_forward(self, member: int, u: torch.Tensor, out: Optional[torch.Tensor] = None,
                    stream=None) -> torch.Tensor:
        n = u.shape[0]
        _need(u, torch.float32, n * self.nparam, "u")
        if out is None:
            out = torch.empty((n, self.nout), dtype=torch.float32, device=u.device)
        _check(lib().emu_forward(self._h, member, _ptr(u), n, _ptr(out), _stream(stream)))
        return out

    def emu_loss_grad(self, member: int, u: torch.Tensor, z: torch.Tensor, stream=None):
        n = u.shape[0]
        _need(u, torch.float32, n * self.nparam, "u")
        _need(z, torch.float32, n * self.nout, "z")
        loss = torch.empty(1, dtype=torch.float32, device=u.device)
        grad = torch.empty(self.nparams, dtype=torch.float32, device=u.device)
        _check(lib().emu_loss_grad(self._h, member, _ptr(u), _ptr(z), n, _ptr(loss), _ptr(grad),
                                   _stream(stream)))
        return loss, grad

    def emu_fit(self, member: int, u: torch.Tensor, z: torch.Tensor, epochs: int, batch: int,
                lr: float, stream=None):
        import numpy as np
        n = u.shape[0]
        _need(u, torch.float32, n * self.nparam, "u")
        _need(z, torch.float32, n * self.nout, "z")
        hist = np.zeros(epochs, dtype=np.float32)
        _check(lib().emu_fit(self._h, member, _ptr(u), _ptr(z), n, epochs, batch, float(lr),
                             hist.ctypes.data, _stream(stream)))
        return hist

    def emu_train(self, params: torch.Tensor, lo, hi, cl: torch.Tensor, epochs: int = 200,
                  batch: int = 256, lr: float = 1e-3, stream=None):
        import numpy as np
        n = params.shape[0]
        _need(params, torch.float64, n * self.nparam, "params")
        _need(cl, torch.float64, n * 4 * self.nl, "cl")
        lo = np.ascontiguousarray(lo, dtype=np.float64)
        hi = np.ascontiguousarray(hi, dtype=np.float64)
        hist = np.zeros(self.members * epochs, dtype=np.float32)
        _check(lib().emu_train(self._h, _ptr(params), lo.ctypes.data, hi.ctypes.data, _ptr(cl), n,
                               epochs, batch, float(lr), hist.ctypes.data, _stream(stream)))
        return hist.reshape(self.members, epochs)

    def emu_infer(self, params: torch.Tensor, threshold: float = 1e-3, cl=None, stream=None):
        n = params.shape[0]
        _need(params, torch.float64, n * self.nparam, "params")
        if cl is None:
            cl = torch.empty((n, 4, self.nl), dtype=torch.float64, device=params.device)
        err = torch.empty(n, dtype=torch.float32, device=params.device)
        flag = torch.empty(n, dtype=torch.uint8, device=params.device)
        _check(lib().emu_infer(self._h, _ptr(params), n, _ptr(cl), _ptr(err), _ptr(flag),
                               float(threshold), _stream(stream)))
        return cl, err, flag

    def emu_infer_spectra(self, params: torch.Tensor, threshold: float = 1e-3, cl=None,
                          stream=None):
        """emu_infer with the error estimate and the fallback flag per spectrum:
        (cl [n, 4, nl], err4 [n, 4] float32, flag4 [n, 4] uint8)."""
        n = params.shape[0]
        _need(params, torch.float64, n * self.nparam, "params")
        if cl is None:
            cl = torch.empty((n, 4, self.nl), dtype=torch.float64, device=params.device)
        err4 = torch.empty((n, 4), dtype=torch.float32, device=params.device)
        flag4 = torch.empty((n, 4), dtype=torch.uint8, device=params.device)
        _check(lib().emu_infer_spectra(self._h, _ptr(params), n, _ptr(cl), _ptr(err4),
                                       _ptr(flag4), float(threshold), _stream(stream)))
        return cl, err4, flag4

    def emu_merge_spectrum(self, spectrum: int, rows, cl_solved: torch.Tensor, cl: torch.Tensor,
                           err4=None, flag4=None, stream=None):
        """Replace spectrum `spectrum` (0 TT, 1 EE, 2 TE, 3 PP) of rows `rows` (host ints) by
        re-solved values cl_solved [len(rows), nl] (float64, device); their err4 and flag4 of
        that spectrum become 0."""
        import numpy as np
        r = np.ascontiguousarray(rows, dtype=np.int64)
        n = cl.shape[0]
        _need(cl, torch.float64, n * 4 * self.nl, "cl")
        if r.size:
            _need(cl_solved, torch.float64, r.size * self.nl, "cl_solved")
        if err4 is not None:
            _need(err4, torch.float32, 4 * n, "err4")
        if flag4 is not None:
            _need(flag4, torch.uint8, 4 * n, "flag4")
        _check(lib().emu_merge_spectrum(self._h, int(spectrum), r.ctypes.data, r.size,
                                        _ptr(cl_solved) if r.size else None, _ptr(cl), n,
                                        _ptr(err4), _ptr(flag4), _stream(stream)))
        return cl

    def emu_merge(self, rows, cl_solved: torch.Tensor, cl: torch.Tensor, err=None, flag=None,
                  stream=None):
        """Replace rows `rows` (host ints) of an emu_infer result by re-solved spectra
        cl_solved [len(rows), 4, nl] (float64, device); their err and flag become 0."""
        import numpy as np
        r = np.ascontiguousarray(rows, dtype=np.int64)
        n = cl.shape[0]
        _need(cl, torch.float64, n * 4 * self.nl, "cl")
        if r.size:
            _need(cl_solved, torch.float64, r.size * 4 * self.nl, "cl_solved")
        if err is not None:
            _need(err, torch.float32, n, "err")
        if flag is not None:
            _need(flag, torch.uint8, n, "flag")
        _check(lib().emu_merge(self._h, r.ctypes.data, r.size, _ptr(cl_solved) if r.size else None,
                               _ptr(cl), n, _ptr(err), _ptr(flag), _stream(stream)))
        return cl

    def emu_save(self, path: str, stream=None):
        _check(lib().emu_save(self._h, os.fsencode(path), _stream(stream)))

    @classmethod
    def emu_load(cls, ctx: Context, path: str) -> "Emulator":
        """An emulator created from a file written by emu_save; its shape is read from the
        file."""
        import struct
        h = ctypes.c_void_p()
        _check(lib().emu_load(ctx.handle, os.fsencode(path), ctypes.byref(h)))
        with open(path, "rb") as f:
            head = f.read(64)  # the header: magic, version, 6 shape ints, pad, seed, ...
        np_, nl, ncomp, width, depth, members = struct.unpack("<6i", head[12:36])
        seed = struct.unpack("<Q", head[40:48])[0]
        return cls(ctx, np_, nl, ncomp, width, depth, members, seed, _handle=h)

    def emu_destroy(self):
        if self._h is not None and self._h.value:
            lib().emu_destroy(self._h)
        self._h = None

    close = emu_destroy

    def __del__(self):
        try:
            self.emu_destroy()
        except Exception:
            pass


class Batch:
    """A los_batch plan: models on a shared master k grid (entry points los_batch_*)."""

    def __init__(self, ctx: Context, lmax, koff, k_index, nk_master: int, ntau: int,
                 pairs: Sequence[Tuple[int, int]], prec: int, nsrc: int):
        import numpy as np
        self._lmax = np.ascontiguousarray(lmax, dtype=np.int32)
        self._koff = np.ascontiguousarray(koff, dtype=np.int64)
        self._kidx = np.ascontiguousarray(k_index, dtype=np.int64)
        flat = np.ascontiguousarray([int(v) for p in pairs for v in p], dtype=np.int32)
        self.nmodels = int(self._lmax.size)
        self.npairs = int(flat.size // 2)
        self.nsrc = nsrc
        self.ntau = int(ntau)
        self.lmax_max = int(self._lmax.max())
        h = ctypes.c_void_p()
        _check(lib().los_batch_create(ctx.handle, self.nmodels, nsrc, self._lmax.ctypes.data,
                                      self._koff.ctypes.data, self._kidx.ctypes.data,
                                      int(nk_master), int(ntau), flat.ctypes.data, self.npairs,
                                      prec, ctypes.byref(h)))
        self._h = h

    def los_batch_columns(self):
        """(col, ncols): packed column of source 0 of every (model, j), and the column count."""
        import numpy as np
        col = np.zeros(int(self._koff[-1]), dtype=np.int64)
        n = ctypes.c_int64()
        _check(lib().los_batch_columns(self._h, col.ctypes.data, ctypes.byref(n)))
        return col, int(n.value)

    def los_batch_info(self) -> dict:
        import numpy as np
        info = np.zeros(10, dtype=np.int32)
        _check(lib().los_batch_info(self._h, info.ctypes.data))
        keys = ("tile_mb", "tile_nc", "rows_per_chunk", "chunks", "rows", "lmax", "tuned",
                "graph", "fused", "fused_shape")
        return {k: int(v) for k, v in zip(keys, info)}

    def los_batch_solve(self, tau0: float, k_master: torch.Tensor, tau: torch.Tensor,
                        w_tau: torch.Tensor, S_packed: torch.Tensor, w_lnk: torch.Tensor,
                        Pk: torch.Tensor, cl: Optional[torch.Tensor] = None,
                        stream=None) -> torch.Tensor:
        npos = int(self._koff[-1])
        if cl is None:
            cl = torch.empty((self.nmodels, self.npairs, self.lmax_max - 1), dtype=torch.float64,
                             device=S_packed.device)
        _need(tau, torch.float64, self.ntau, "tau")
        _need(w_tau, torch.float64, self.ntau, "w_tau")
        _need(w_lnk, torch.float64, npos, "w_lnk")
        _need(Pk, torch.float64, npos, "Pk")
        _need(cl, torch.float64, self.nmodels * self.npairs * (self.lmax_max - 1), "cl")
        if S_packed.dtype != torch.float32 or S_packed.numel() % self.ntau:
            raise ValueError("S_packed must be float32 [ncols, ntau]")
        if k_master.dtype != torch.float64:
            raise ValueError("k_master must be float64")
        _check(lib().los_batch_solve(self._h, float(tau0), _ptr(k_master), _ptr(tau), _ptr(w_tau),
                                     _ptr(S_packed), _ptr(w_lnk), _ptr(Pk), _ptr(cl),
                                     _stream(stream)))
        return cl

    def los_batch_solve_timed(self, tau0: float, k_master: torch.Tensor, tau: torch.Tensor,
                              w_tau: torch.Tensor, S_packed: torch.Tensor, w_lnk: torch.Tensor,
                              Pk: torch.Tensor, cl: torch.Tensor, stream=None) -> dict:
        """Eager instrumented solve into `cl`; returns the summed device milliseconds and launch
        counts of the Bessel, product and C_l kernels."""
        import numpy as np
        npos = int(self._koff[-1])
        _need(w_lnk, torch.float64, npos, "w_lnk")
        _need(Pk, torch.float64, npos, "Pk")
        _need(cl, torch.float64, self.nmodels * self.npairs * (self.lmax_max - 1), "cl")
        if S_packed.dtype != torch.float32 or S_packed.numel() % self.ntau:
            raise ValueError("S_packed must be float32 [ncols, ntau]")
        ms = np.zeros(3, dtype=np.float64)
        n = np.zeros(3, dtype=np.int32)
        _check(lib().los_batch_solve_timed(self._h, float(tau0), _ptr(k_master), _ptr(tau),
                                           _ptr(w_tau), _ptr(S_packed), _ptr(w_lnk), _ptr(Pk),
                                           _ptr(cl), ms.ctypes.data, n.ctypes.data,
                                           _stream(stream)))
        return {"bessel_ms": float(ms[0]), "product_ms": float(ms[1]), "cl_ms": float(ms[2]),
                "launches": int(n[1])}

    def los_batch_destroy(self):
        if self._h is not None and self._h.value:
            lib().los_batch_destroy(self._h)
        self._h = None

    close = los_batch_destroy

    def __del__(self):
        try:
            self.los_batch_destroy()
        except Exception:
            pass


def version() -> str:
    return lib().los_version().decode()
