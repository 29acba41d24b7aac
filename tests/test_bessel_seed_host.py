"""The Bessel seed functions the kernels use (bessel_dev.hpp), built for the host from the
same source (liblos_hostcheck.so), against 30-digit mpmath values of j_l(x) =
sqrt(pi/(2x)) J_{l+1/2}(x):

* debye_j: Debye's expansion of J_nu(nu sech a) (DLMF 10.19.3) with the u_k of DLMF
  10.41.10-11, at and above the band edge l = ltop(x) = floor(x + 14.2 x^(1/3) + 9.5),
  where the kernels start their descending runs;
* node_top_pair: the (unweighted) pair (j_R, j_{R+1}) at a node's top row R for every branch
  (Debye seed for 64 <= x < lmax + 1, upward recurrence for x >= lmax + 1, Miller's
  recurrence normalised by the upward value below 64), with R the top row of the 16-row
  block holding min(cut(x), lmax), for both band cuts: the FP64 one ltop(x) and the MFMA
  paths' ltop_mfma(x) = floor(x + 9 x^(1/3) + 4) (the seed still starts at ltop and runs
  down to R);
* the MFMA band cut drops no value above 1.2e-12 of the largest |j_l(x)| over l.
Bound 1e-13: relative for the Debye values themselves (their own error is about |eta| ~ 60
ulps of e^eta); for the pair at R relative to the largest |j_l| over the rows lmin..R+1 the
sweep covers (a Miller pair at the band edge carries the seed's error there, which the
descending sweep then damps; a pair reached by a run near the turning point or by the
upward recurrence carries the run's rounding)."""
import ctypes
import math
import os

import numpy as np
import pytest
from scipy.special import spherical_jn

mpmath = pytest.importorskip("mpmath")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2509_25110_amd", "liblos_hostcheck.so")


@pytest.fixture(scope="module")
def hc():
    if not os.path.exists(LIB):
        from paper_2509_25110_amd import build
        build.build_hostcheck(verbose=False)
    lib = ctypes.CDLL(LIB)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.los_hostcheck_debye_j.argtypes = [i64, vp, vp, vp]
    lib.los_hostcheck_node_top_pair.argtypes = [i64, vp, i32, i32, i32, vp, vp, vp]
    return lib


def jl_mp(l, x):
    mpmath.mp.dps = 30
    x = mpmath.mpf(x)
    return mpmath.sqrt(mpmath.pi / (2 * x)) * mpmath.besselj(l + mpmath.mpf(1) / 2, x,
                                                             maxterms=10 ** 6)


def ltop(x):
    return int(math.floor(x + 14.2 * np.cbrt(x) + 9.5))


def ltop_mfma(x):
    return int(math.floor(x + 9.0 * np.cbrt(x) + 4.0))


def debye(hc, ls, xs):
    ls = np.ascontiguousarray(ls, dtype=np.int32)
    xs = np.ascontiguousarray(xs, dtype=np.float64)
    out = np.empty(xs.size)
    hc.los_hostcheck_debye_j(xs.size, ls.ctypes.data, xs.ctypes.data, out.ctypes.data)
    return out


def test_debye_at_and_above_band_edge(hc):
    xs, ls = [], []
    for x in (64.0, 99.5, 250.0, 777.7, 1500.0, 3333.3, 5000.0):
        for dl in (0, 1, 7, 16):
            xs.append(x)
            ls.append(ltop(x) + dl)
    got = debye(hc, ls, xs)
    worst = 0.0
    for l, x, g in zip(ls, xs, got):
        ref = jl_mp(l, x)
        err = float(abs(g / ref - 1))
        worst = max(worst, err)
        assert err <= 1e-13, (l, x, err)
    print("debye_j worst relative error %.2e" % worst)


def test_debye_series_branch_boundary(hc):
    """Both ways of forming eta (the series for s = sqrt(1 - (x/nu)^2) <= 0.7, logs above)
    around the switch, s = 0.7 at nu = x / sqrt(0.51)."""
    xs, ls = [], []
    for x in (200.0, 350.0):
        lc = int(x / math.sqrt(0.51) - 0.5)
        for l in (lc - 1, lc, lc + 1, lc + 2):
            if l >= ltop(x):
                xs.append(x)
                ls.append(l)
    got = debye(hc, ls, xs)
    for l, x, g in zip(ls, xs, got):
        assert abs(g / jl_mp(l, x) - 1) <= 1e-13, (l, x)


@pytest.mark.parametrize("mfma", [0, 1], ids=["fp64_cut", "mfma_cut"])
@pytest.mark.parametrize("lmin,lmax", [(2, 2500), (2, 300), (37, 1000), (1, 64)])
def test_node_top_pair_branches(hc, lmin, lmax, mfma):
    xs = np.array([0.5, 3.0, 20.0, 63.9, 64.0, 200.0, 0.8 * lmax, lmax - 30.0, lmax - 0.5,
                   lmax + 1.0, lmax + 1.5, 1.7 * lmax + 3.3], dtype=np.float64)
    xs = xs[xs > 0]
    n = xs.size
    cur, nxt = np.empty(n), np.empty(n)
    R = np.empty(n, dtype=np.int32)
    hc.los_hostcheck_node_top_pair(n, xs.ctypes.data, lmin, lmax, mfma, cur.ctypes.data,
                                   nxt.ctypes.data, R.ctypes.data)
    cut = ltop_mfma if mfma else ltop
    for i, x in enumerate(xs):
        rc = min(cut(x), lmax) if math.floor(x) < lmax + 1 else lmax
        want_R = lmin + (rc - lmin) // 16 * 16 + 15 if rc >= lmin else -1
        assert R[i] == want_R, (x, R[i], want_R)
        if want_R < 0:
            continue
        # the rows the sweep will cover: the bound is relative to their largest |j_l|
        scale = float(np.max(np.abs(spherical_jn(np.arange(lmin, want_R + 2), x))))
        # an upward run that ends past the turning point (x < R + 1 <= lmax + 16) has taken up
        # to 15 unstable steps in rows that are swept but never stored; the error it leaves
        # there is damped on the way back down
        tol = 1e-11 if (math.floor(x) >= lmax + 1 and want_R + 1 > x) else 1e-13
        for got, l in ((cur[i], want_R), (nxt[i], want_R + 1)):
            ref = jl_mp(l, x)
            sc = scale * tol / 1e-13
            assert abs(got - ref) <= 1e-13 * float(sc), (lmin, lmax, x, l, got, float(ref))


def test_mfma_band_cut_tail():
    """Above ltop_mfma(x) no |j_l(x)| exceeds 1.2e-12 of the largest over l (scipy's
    spherical_jn, accurate to a few ulps of the peak here), and the cut is below ltop."""
    worst = 0.0
    for x in (0.3, 1.0, 5.0, 20.0, 63.9, 64.0, 100.0, 300.0, 1000.0, 3000.0, 6000.0, 14000.0):
        ls = np.arange(0, int(x + 20 * np.cbrt(x) + 40))
        j = spherical_jn(ls, x)
        peak = float(np.max(np.abs(j)))
        tail = float(np.max(np.abs(j[ltop_mfma(x) + 1:]))) / peak
        worst = max(worst, tail)
        assert tail <= 1.2e-12, (x, tail)
        assert ltop_mfma(x) <= ltop(x)
    print("largest dropped |j_l| / peak: %.2e" % worst)
