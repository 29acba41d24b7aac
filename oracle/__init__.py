"""Plain FP64 CPU oracle for the line-of-sight projection (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never does, and the two
share no code: the arithmetic lives in ``los_oracle.c`` (plain C, IEEE double,
OpenMP over k), which this module compiles on demand with gcc and calls
through ctypes.

Functions follow the gCAMB paper, Sec. 2.1 Eq. 1-3 (C_l and the LOS transfer
integrals) and Sec. 3.2 / Algorithm 1 (loop over k, then l, then tau):

* :func:`sph_jl`        -- j_l(x), l = 0..lmax (spherical Bessel kernel, flat space)
* :func:`bessel_table`  -- j_l(x_i) as an [l - lmin][i] table
* :func:`eps_l`         -- the E-mode kernel sqrt((l+2)!/(l-2)!) j_l(x)/x^2 (Eq. 3)
* :func:`project`       -- Delta^X_l(k_i) = sum_n w_n S_X(k_i, tau_n) K_l(k_i (tau0 - tau_n)),
                           K = j_l, or eps_l for the sources selected by a mask
* :func:`cl`            -- C^XY_l = 4 pi sum_i w_i P(k_i) Delta^X_l(k_i) Delta^Y_l(k_i)
* :func:`tensor_kernels` -- the tensor-mode kernels K^T, K^E, K^B of the line-of-sight method
* :func:`project_tensor` -- the tensor transfer functions Delta^T, Delta^E, Delta^B
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "los_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liblos_oracle.so")
_lock = threading.Lock()
_lib = None

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_int32_p = ctypes.POINTER(ctypes.c_int32)


_SHA_PATH = _LIB_PATH + ".src-sha256"


def _src_sha() -> str:
    import hashlib
    with open(_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def build(force: bool = False) -> str:
    """Compile ``los_oracle.c`` into ``liblos_oracle.so`` (gcc -O2 -fopenmp, no fast-math).
    Without ``force`` the library is rebuilt only when it is missing or was built from other
    source text (a hash kept beside it; file times are not used, since copies reorder them)."""
    sha = _src_sha()
    stale = not os.path.exists(_LIB_PATH) or not os.path.exists(_SHA_PATH)
    if not stale:
        with open(_SHA_PATH) as f:
            stale = f.read().strip() != sha
    if force or stale:
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-fno-fast-math",
               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
        with open(_SHA_PATH, "w") as f:
            f.write(sha + "\n")
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            lib.oracle_sph_jl.argtypes = [ctypes.c_int32, ctypes.c_double, _c_double_p]
            lib.oracle_bessel_table.argtypes = [_c_double_p, ctypes.c_int64, ctypes.c_int32,
                                                ctypes.c_int32, _c_double_p]
            lib.oracle_project.argtypes = [
                ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                _c_double_p, _c_double_p, _c_double_p, _c_double_p, ctypes.c_int32,
                _c_double_p, _c_double_p]
            lib.oracle_project_kernels.argtypes = [
                ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                _c_double_p, _c_double_p, _c_double_p, _c_double_p, ctypes.c_int32,
                ctypes.c_uint32, _c_double_p, _c_double_p]
            lib.oracle_eps_l.argtypes = [ctypes.c_int32, ctypes.c_double, _c_double_p,
                                         _c_double_p]
            lib.oracle_cl.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, _c_double_p,
                                      _c_double_p, _c_double_p, _c_int32_p, ctypes.c_int32,
                                      _c_double_p]
            lib.oracle_num_threads.argtypes = []
            lib.oracle_tensor_kernels.argtypes = [ctypes.c_int32, ctypes.c_double, _c_double_p,
                                                  _c_double_p, _c_double_p, _c_double_p]
            lib.oracle_project_tensor.argtypes = [
                ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                _c_double_p, _c_double_p, _c_double_p, _c_double_p, _c_double_p, _c_double_p]
            for f in (lib.oracle_sph_jl, lib.oracle_bessel_table, lib.oracle_project,
                      lib.oracle_project_kernels, lib.oracle_eps_l, lib.oracle_cl,
                      lib.oracle_num_threads, lib.oracle_tensor_kernels,
                      lib.oracle_project_tensor):
                f.restype = ctypes.c_int
            _lib = lib
    return _lib


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_c_double_p)


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle %s failed with status %d" % (what, rc))


def num_threads() -> int:
    """OpenMP threads the oracle uses (``OMP_NUM_THREADS`` or all cores)."""
    return int(_load().oracle_num_threads())


def sph_jl(lmax: int, x: float) -> np.ndarray:
    """j_l(x) for l = 0..lmax in FP64."""
    out = np.empty(lmax + 1, dtype=np.float64)
    _check(_load().oracle_sph_jl(int(lmax), float(x), out.ctypes.data_as(_c_double_p)), "sph_jl")
    return out


def bessel_table(x, lmin: int, lmax: int) -> np.ndarray:
    """out[l - lmin, i] = j_l(x[i])."""
    x, xp = _f64(x)
    out = np.empty((lmax - lmin + 1, x.size), dtype=np.float64)
    _check(_load().oracle_bessel_table(xp, x.size, int(lmin), int(lmax),
                                       out.ctypes.data_as(_c_double_p)), "bessel_table")
    return out


def eps_l(lmax, x) -> np.ndarray:
    """E-mode kernel eps_l(x) = sqrt((l+2)!/(l-2)!) j_l(x) / x^2 for l = 0..lmax (Sec. 2.1,
    Eq. 3); 0 for l < 2; the x -> 0 limit is sqrt(24)/15 at l = 2 and 0 above."""
    jl = np.empty(lmax + 1)
    out = np.empty(lmax + 1)
    _check(_load().oracle_eps_l(int(lmax), float(x), jl.ctypes.data_as(_c_double_p),
                                out.ctypes.data_as(_c_double_p)), "eps_l")
    return out


def project(lmin, lmax, k, tau, tau0, w_tau, S, with_abs=False, k_range=None, eps_mask=0):
    """LOS projection (Eq. 2-3).

    ``S`` is [nsrc, nk, ntau]; returns delta [nk, nl, nsrc] (and the absolute
    sum ``A`` of the same shape if ``with_abs``).  ``k_range=(a, b)`` computes
    only rows a..b-1 and returns arrays of b - a rows (each row depends only on
    its own k and S row, so this equals slicing the full result).  Sources whose
    bit is set in ``eps_mask`` use the E-mode kernel eps_l instead of j_l.
    """
    S = np.asarray(S)
    k = np.asarray(k)
    if k_range is not None:
        a, b = k_range
        k = k[a:b]
        S = S[:, a:b, :]
    k, kp = _f64(k)
    tau, tp = _f64(tau)
    w_tau, wp = _f64(w_tau)
    S, sp = _f64(S)
    nsrc, nk, ntau = S.shape
    assert nk == k.size and ntau == tau.size == w_tau.size
    nl = lmax - lmin + 1
    delta = np.empty((nk, nl, nsrc))
    absd = np.empty((nk, nl, nsrc)) if with_abs else None
    rc = _load().oracle_project_kernels(
        int(lmin), int(lmax), nk, ntau, float(tau0), kp, tp, wp, sp, nsrc, int(eps_mask),
        delta.ctypes.data_as(_c_double_p),
        absd.ctypes.data_as(_c_double_p) if with_abs else None)
    _check(rc, "project")
    return (delta, absd) if with_abs else delta


def cl(delta, w_lnk, Pk, pairs) -> np.ndarray:
    """C_l (Eq. 1): returns [npairs, nl] with cl[p, l] = 4 pi sum_k w P delta[k,l,a] delta[k,l,b]."""
    delta, dp = _f64(delta)
    nk, nl, nsrc = delta.shape
    w_lnk, wp = _f64(w_lnk)
    Pk, pp = _f64(Pk)
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    out = np.empty((pr.shape[0], nl), dtype=np.float64)
    rc = _load().oracle_cl(nl, nk, nsrc, dp, wp, pp, pr.ctypes.data_as(_c_int32_p), pr.shape[0],
                           out.ctypes.data_as(_c_double_p))
    _check(rc, "cl")
    return out


def tensor_kernels(lmax, x):
    """Tensor-mode kernels at one x for l = 0..lmax: (K^T, K^E, K^B) with
    K^T = sqrt((l+2)!/(l-2)!) j_l/x^2, K^E = -j_l + j_l'' + 2 j_l/x^2 + 4 j_l'/x,
    K^B = 2 j_l' + 4 j_l/x (the published tensor line-of-sight kernels of the method the
    paper cites in Sec. 2.1); 0 for l < 2."""
    jl, kt, ke, kb = (np.empty(lmax + 1) for _ in range(4))
    _check(_load().oracle_tensor_kernels(int(lmax), float(x), jl.ctypes.data_as(_c_double_p),
                                         kt.ctypes.data_as(_c_double_p),
                                         ke.ctypes.data_as(_c_double_p),
                                         kb.ctypes.data_as(_c_double_p)), "tensor_kernels")
    return kt, ke, kb


def project_tensor(lmin, lmax, k, tau, tau0, w_tau, S, with_abs=False, k_range=None):
    """Tensor transfer functions: ``S`` is [2, nk, ntau] (S_T, S_P); returns delta
    [nk, nl, 3] with the T, E and B transfer functions (and, if ``with_abs``, the scale
    sum_n |w S| times the absolute sum of each kernel's terms, same shape).  lmin >= 2."""
    S = np.asarray(S)
    k = np.asarray(k)
    if k_range is not None:
        a, b = k_range
        k = k[a:b]
        S = S[:, a:b, :]
    k, kp = _f64(k)
    tau, tp = _f64(tau)
    w_tau, wp = _f64(w_tau)
    S, sp = _f64(S)
    nsrc, nk, ntau = S.shape
    assert nsrc == 2 and nk == k.size and ntau == tau.size == w_tau.size
    nl = lmax - lmin + 1
    delta = np.empty((nk, nl, 3))
    absd = np.empty((nk, nl, 3)) if with_abs else None
    rc = _load().oracle_project_tensor(
        int(lmin), int(lmax), nk, ntau, float(tau0), kp, tp, wp, sp,
        delta.ctypes.data_as(_c_double_p),
        absd.ctypes.data_as(_c_double_p) if with_abs else None)
    _check(rc, "project_tensor")
    return (delta, absd) if with_abs else delta
