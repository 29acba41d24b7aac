"""Pins of the oracle's E-mode kernel eps_l(x) = sqrt((l+2)!/(l-2)!) j_l(x) / x^2
(gCAMB paper Sec. 2.1, Eq. 3 and the text below it) against values fixed
independently of it: 40-digit mpmath, the small-x series of j_l, the
closed-form j_2, and the delta-source identity of the projection."""
import math

import numpy as np
import pytest

import oracle

mpmath = pytest.importorskip("mpmath")


def eps_mp(l, x):
    mpmath.mp.dps = 40
    x = mpmath.mpf(x)
    jl = mpmath.sqrt(mpmath.pi / (2 * x)) * mpmath.besselj(l + mpmath.mpf(1) / 2, x,
                                                           maxterms=10 ** 6)
    pref = mpmath.sqrt(mpmath.factorial(l + 2) / mpmath.factorial(l - 2))
    return pref * jl / x ** 2


@pytest.mark.parametrize("x", [1e-3, 0.5, 3.0, 50.0, 700.0, 1500.5])
def test_eps_vs_mpmath(x):
    ls = [2, 3, 4, 10, 60, 100, 400, 1000, 1600]
    lmax = max(ls)
    got = oracle.eps_l(lmax, x)
    ref = {l: float(eps_mp(l, x)) for l in ls}
    peak = max(abs(v) for v in ref.values())
    for l in ls:
        err = abs(got[l] - ref[l])
        # relative where the value is not in the evanescent tail, else against the peak
        assert err <= 1e-12 * max(abs(ref[l]), 1e-9 * peak), (l, x, got[l], ref[l])
    assert got[0] == 0.0 and got[1] == 0.0


def test_eps_small_x_limit_and_series():
    e0 = oracle.eps_l(5, 0.0)
    assert e0[2] == math.sqrt(24.0) / 15.0 and np.all(e0[3:] == 0.0)
    x = 1e-4
    e = oracle.eps_l(5, x)
    # j_2(x)/x^2 = (1/15)(1 - x^2/14 + ...), j_3(x)/x^2 = (x/105)(1 - x^2/18 + ...)
    assert abs(e[2] - math.sqrt(24.0) * (1 / 15) * (1 - x * x / 14)) < 1e-15
    ref3 = math.sqrt(120.0) * x / 105 * (1 - x * x / 18)
    assert abs(e[3] - ref3) < 1e-13 * ref3


def test_eps_closed_form_l2():
    for x in (1.0, 7.3, 42.0, 333.0):
        j2 = (3 / x ** 3 - 1 / x) * math.sin(x) - 3 * math.cos(x) / x ** 2
        ref = math.sqrt(24.0) * j2 / x ** 2
        got = oracle.eps_l(2, x)[2]
        assert abs(got - ref) <= 1e-13 * max(abs(ref), math.sqrt(24.0) / x ** 3)


def test_emode_delta_source_identity_and_mask_zero():
    """S = 1/w at one node n*: Delta^E_l(k) = eps_l(k chi*) exactly; mask 0 gives the j_l
    projection."""
    rng = np.random.default_rng(8)
    ntau, nk, lmax = 40, 5, 30
    tau = np.linspace(0, 14000.0, ntau)
    w = np.full(ntau, 14000.0 / (ntau - 1))
    k = np.exp(np.linspace(np.log(1e-4), np.log(2e-3), nk))
    S = np.zeros((2, nk, ntau))
    S[:, :, 7] = 1.0 / w[7]
    d = oracle.project(2, lmax, k, tau, 14000.0, w, S, eps_mask=0b10)
    for i in range(nk):
        x = k[i] * (14000.0 - tau[7])
        np.testing.assert_allclose(d[i, :, 1], oracle.eps_l(lmax, x)[2:], rtol=1e-14, atol=0)
        np.testing.assert_allclose(d[i, :, 0], oracle.sph_jl(lmax, x)[2:], rtol=1e-14, atol=0)
    S2 = rng.normal(size=(2, nk, ntau))
    np.testing.assert_array_equal(oracle.project(2, lmax, k, tau, 14000.0, w, S2, eps_mask=0),
                                  oracle.project(2, lmax, k, tau, 14000.0, w, S2))


def test_emode_x_zero_node():
    """The node at tau = tau0 (x = 0) adds w S sqrt(24)/15 to l = 2 and nothing above."""
    tau = np.array([0.0, 7000.0, 14000.0])
    w = np.array([1.0, 2.0, 3.0])
    k = np.array([1e-3])
    S = np.zeros((1, 1, 3))
    S[0, 0, 2] = 5.0
    d = oracle.project(2, 6, k, tau, 14000.0, w, S, eps_mask=1)
    assert d[0, 0, 0] == 3.0 * 5.0 * math.sqrt(24.0) / 15.0
    assert np.all(d[0, 1:, 0] == 0.0)
