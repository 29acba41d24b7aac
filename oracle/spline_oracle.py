"""Plain FP64 oracle for the source interpolation step (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module; the GPU library never does.

The gCAMB paper (Sec. 3.2, the calling sequence of SourceToTransfers) names an
InterpolateSources step that prepares the source data on the integration grid
before the line-of-sight integrals, without fixing the scheme.  The reading
taken here: the sources are known on a coarse wavenumber grid q_0 < ... <
q_{N-1} (the grid the perturbation equations are evolved on) at the same tau
nodes as the projection, and each source at each tau node is carried to the
projection's k grid by the natural cubic spline in k through those N values.

Natural cubic spline (the textbook definition): on [q_j, q_{j+1}] with
h_j = q_{j+1} - q_j, A = (q_{j+1} - k) / h_j, B = 1 - A,

    s(k) = A y_j + B y_{j+1} + ((A^3 - A) M_j + (B^3 - B) M_{j+1}) h_j^2 / 6

where the second derivatives M solve, for j = 1 .. N-2,

    h_{j-1}/6 M_{j-1} + (h_{j-1} + h_j)/3 M_j + h_j/6 M_{j+1}
        = (y_{j+1} - y_j)/h_j - (y_j - y_{j-1})/h_{j-1},

with M_0 = M_{N-1} = 0 (continuity of s'' at the knots and zero curvature at
the ends).  N = 2 gives the straight line.  A k outside [q_0, q_{N-1}] takes
the cubic of the end interval.

The tridiagonal system is solved by a library banded solver (LAPACK through
scipy), one right-hand side per (source, tau node) column.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_banded


def second_derivatives(q, Sc) -> np.ndarray:
    """M[s, j, n]: the natural-spline second derivatives in k of Sc[s, :, n]
    on the knots q (strictly increasing, N = len(q) >= 2)."""
    q = np.asarray(q, dtype=np.float64)
    Sc = np.asarray(Sc, dtype=np.float64)
    nsrc, N, ntau = Sc.shape
    if q.shape != (N,) or N < 2:
        raise ValueError("need q[N] with N >= 2 matching Sc[:, N, :]")
    h = np.diff(q)
    if np.any(h <= 0):
        raise ValueError("q must be strictly increasing")
    M = np.zeros_like(Sc)
    if N == 2:
        return M
    n = N - 2  # interior knots j = 1 .. N-2
    ab = np.zeros((3, n))
    ab[0, 1:] = h[1:n] / 6.0          # super-diagonal: h_j / 6 multiplies M_{j+1}
    ab[1, :] = (h[:n] + h[1:]) / 3.0  # diagonal: (h_{j-1} + h_j) / 3
    ab[2, :-1] = h[1:n] / 6.0         # sub-diagonal: h_{j-1} / 6 multiplies M_{j-1}
    # right-hand side for every column at once: [n, nsrc * ntau]
    Y = Sc.transpose(1, 0, 2).reshape(N, -1)
    rhs = (Y[2:] - Y[1:-1]) / h[1:, None] - (Y[1:-1] - Y[:-2]) / h[:-1, None]
    Mi = solve_banded((1, 1), ab, rhs)
    M[:, 1:-1, :] = Mi.reshape(n, nsrc, ntau).transpose(1, 0, 2)
    return M


def interval(q, k) -> np.ndarray:
    """j with q_j <= k < q_{j+1}, clamped to 0 .. N-2 (end cubics outside the knots)."""
    q = np.asarray(q, dtype=np.float64)
    j = np.searchsorted(q, np.asarray(k, dtype=np.float64), side="right") - 1
    return np.clip(j, 0, q.size - 2)


def evaluate(q, Sc, M, k) -> np.ndarray:
    """S[s, i, n] = s(k_i) for the spline through Sc[s, :, n] with second derivatives M."""
    q = np.asarray(q, dtype=np.float64)
    Sc = np.asarray(Sc, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    k = np.asarray(k, dtype=np.float64)
    j = interval(q, k)
    h = q[j + 1] - q[j]
    A = (q[j + 1] - k) / h
    B = (k - q[j]) / h
    cA = (A ** 3 - A) * h * h / 6.0
    cB = (B ** 3 - B) * h * h / 6.0
    return (A[None, :, None] * Sc[:, j, :] + B[None, :, None] * Sc[:, j + 1, :]
            + cA[None, :, None] * M[:, j, :] + cB[None, :, None] * M[:, j + 1, :])


def interp_cl(ls, cls, lmin, lmax) -> np.ndarray:
    """C_l at every l in [lmin, lmax] from cls[npairs, len(ls)] at the sampled multipoles ls
    (the output l-sampling of the gCAMB paper, Sec. 3.1, read as the natural cubic spline
    in l of D_l = l (l + 1) C_l through the sampled points, divided back by l (l + 1))."""
    ls = np.asarray(ls, dtype=np.float64)
    cls = np.atleast_2d(np.asarray(cls, dtype=np.float64))
    if ls[0] != lmin or ls[-1] != lmax:
        raise ValueError("the sampled multipoles must include lmin and lmax")
    ell = np.arange(lmin, lmax + 1, dtype=np.float64)
    if ls.size == 1:
        return cls.copy()
    D = cls * (ls * (ls + 1.0))[None, :]
    Dall = interpolate(ls, D[:, :, None], ell)[:, :, 0]
    return Dall / (ell * (ell + 1.0))[None, :]


def interpolate(q, Sc, k) -> np.ndarray:
    """Sources on the projection grid: evaluate(q, Sc, second_derivatives(q, Sc), k)."""
    return evaluate(q, Sc, second_derivatives(q, Sc), k)
