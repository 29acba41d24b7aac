"""Pins for the oracle's spherical Bessel functions j_l(x).

The oracle's kernel is the flat-space radial function of the LOS integrals
(paper Sec. 2.1, below Eq. 3).  None of these checks retype the oracle: they
compare it with closed forms (DLMF 10.49.3), with mpmath at 40 digits, with
scipy, and its two branches (upward from sin/cos, Miller with the sum rule)
against each other.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy.special import spherical_jn

import oracle


def series(l, x, terms=30):
    """Power series j_l(x) = x^l / (2l+1)!! sum_k (-x^2/2)^k / (k! (2l+3)(2l+5)...(2l+2k+1))."""
    df = 1.0
    for m in range(1, 2 * l + 2, 2):
        df *= m
    term, acc = 1.0, 1.0
    for k in range(1, terms):
        term *= -(x * x / 2.0) / (k * (2 * l + 2 * k + 1))
        acc += term
    return x**l / df * acc


def closed_forms(x):
    if x < 1.0:  # the closed forms cancel badly for small x
        return tuple(series(l, x) for l in range(3))
    s, c = math.sin(x), math.cos(x)
    j0 = s / x
    j1 = s / x**2 - c / x
    j2 = (3.0 / x**2 - 1.0) * s / x - 3.0 * c / x**2
    return j0, j1, j2


def mp_jl(l, x):
    mp.mp.dps = 40
    x = mp.mpf(x)
    return float(mp.sqrt(mp.pi / (2 * x)) * mp.besselj(l + mp.mpf(1) / 2, x, maxprec=60000,
                                                       maxterms=10**6))


@pytest.mark.parametrize("x", [0.05, 0.7, 1.9, 3.14159, 6.5, 11.0, 40.3, 250.0, 1999.5])
@pytest.mark.parametrize("lmax", [2, 60, 3000])
def test_closed_forms_both_branches(x, lmax):
    """j_0, j_1, j_2 from the closed forms, whichever branch lmax/x selects."""
    j = oracle.sph_jl(lmax, x)
    ref = closed_forms(x)
    scale = max(abs(v) for v in ref)
    for l in range(min(3, lmax + 1)):
        assert abs(j[l] - ref[l]) <= 2e-14 * scale + 1e-15 * abs(ref[l]), (l, j[l], ref[l])


def test_x_zero_and_tiny():
    j = oracle.sph_jl(10, 0.0)
    assert j[0] == 1.0 and np.all(j[1:] == 0.0)
    j = oracle.sph_jl(10, 1e-200)
    assert j[0] == 1.0 and abs(j[1] - 1e-200 / 3) < 1e-214 and np.all(j[3:] == 0.0)
    with pytest.raises(ValueError):
        oracle.sph_jl(10, -1.0)


@pytest.mark.parametrize("x,lmax", [
    (0.37, 60), (2.5, 80), (17.3, 200), (123.4, 400), (777.7, 1200),
    (2499.3, 2500), (2500.9, 2500), (4321.1, 2500), (6999.7, 2500), (13999.9, 5000),
    (4990.2, 5000)])
def test_mpmath_normwise_and_tail(x, lmax):
    """Against 40-digit mpmath on l samples through the turning point.

    Normwise: |err| <= 3e-13 max|j| over the samples; in the evanescent tail
    (l > x + 2 x^(1/3)), where j_l has no zeros, also relative 1e-11.
    """
    t = int(x)
    ls = {0, 1, 2, 3, 7, lmax // 3, lmax // 2, max(t - 40, 0), max(t - 5, 0), t, t + 1, t + 3,
          t + 10, t + 25, t + 60, lmax}
    ls = sorted(l for l in ls if 0 <= l <= lmax)
    j = oracle.sph_jl(lmax, x)
    ref = np.array([mp_jl(l, x) for l in ls])
    got = j[ls]
    env = np.max(np.abs(ref))
    assert np.max(np.abs(got - ref)) <= 3e-13 * env, list(zip(ls, got, ref))
    tail = np.array([l > x + 2 * x ** (1 / 3) and abs(r) > 1e-280 for l, r in zip(ls, ref)])
    if tail.any():
        rel = np.abs(got[tail] / ref[tail] - 1)
        assert np.max(rel) <= 1e-11, rel


def test_branches_agree():
    """Upward (sin/cos) and Miller (sum-rule) branches agree where both apply."""
    for x in [5.5, 33.3, 300.7, 1234.5, 3999.9]:
        lo = int(x) - 1                     # x >= lo + 1: upward branch
        up = oracle.sph_jl(lo, x)
        mil = oracle.sph_jl(int(x) + 300, x)  # x < lmax + 1: Miller branch
        env = np.max(np.abs(mil))
        assert np.max(np.abs(up - mil[: lo + 1])) <= 5e-13 * env, x


def test_scipy_sweep():
    """Broad sweep against scipy.special.spherical_jn, normwise per x."""
    rng = np.random.default_rng(7)
    for x in np.concatenate([rng.uniform(0.01, 10, 8), rng.uniform(10, 3000, 12)]):
        lmax = int(rng.integers(5, 1500))
        j = oracle.sph_jl(lmax, x)
        ref = spherical_jn(np.arange(lmax + 1), x)
        env = np.max(np.abs(ref))
        assert np.max(np.abs(j - ref)) <= 1e-11 * env, (x, lmax)


def test_sum_rule_and_recurrence_residual():
    """sum (2l+1) j_l^2 = 1 once lmax is far above x; three-term recurrence holds."""
    for x in [0.9, 12.0, 480.0, 2600.0]:
        lmax = int(x + 40 * max(x, 1) ** (1 / 3) + 50)
        j = oracle.sph_jl(lmax, x)
        l = np.arange(lmax + 1)
        assert abs(np.sum((2 * l + 1) * j * j) - 1.0) < 1e-13
        res = (2 * l[1:-1] + 1) / x * j[1:-1] - j[:-2] - j[2:]
        assert np.max(np.abs(res)) <= 1e-12 * np.max(np.abs(j)) * max(1.0, (2 * lmax + 1) / x)


def test_table_layout():
    x = np.array([0.0, 0.5, 3.0, 150.0, 900.0])
    t = oracle.bessel_table(x, 2, 40)
    assert t.shape == (39, 5)
    for i, xi in enumerate(x):
        np.testing.assert_array_equal(t[:, i], oracle.sph_jl(40, xi)[2:])
