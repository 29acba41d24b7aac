"""Pins of the oracle's tensor-mode line-of-sight kernels (the tensor counterpart of
Eq. 2-3 that the gCAMB paper, Sec. 2.1, says arises for tensor perturbations and B modes;
kernels as published for the line-of-sight method it cites):
  K^T_l = sqrt((l+2)!/(l-2)!) j_l / x^2,  K^E_l = -j_l + j_l'' + 2 j_l/x^2 + 4 j_l'/x,
  K^B_l = 2 j_l' + 4 j_l/x,
against values fixed independently of the oracle: 40-digit mpmath (j_l from the Bessel
function of half-integer order, its derivatives by numerical differentiation at that
precision), the small-x power series, the large-x asymptotic form, brute-force mpmath sums
of the discrete projection, and the delta-source identity."""
import math

import numpy as np
import pytest

import oracle

mpmath = pytest.importorskip("mpmath")


def kernels_mp(l, x):
    """(K^T, K^E, K^B, term scale of E, term scale of B) at 40 digits."""
    mpmath.mp.dps = 40
    x = mpmath.mpf(x)
    half = mpmath.mpf(1) / 2

    def j(t):
        return mpmath.sqrt(mpmath.pi / (2 * t)) * mpmath.besselj(l + half, t, maxterms=10 ** 6)

    j0 = j(x)
    j1 = mpmath.diff(j, x, 1)
    j2 = mpmath.diff(j, x, 2)
    pref = mpmath.sqrt(mpmath.factorial(l + 2) / mpmath.factorial(l - 2))
    kt = pref * j0 / x ** 2
    ke = -j0 + j2 + 2 * j0 / x ** 2 + 4 * j1 / x
    kb = 2 * j1 + 4 * j0 / x
    se = abs(j0) + abs(j2) + abs(2 * j0 / x ** 2) + abs(4 * j1 / x)
    sb = abs(2 * j1) + abs(4 * j0 / x)
    return float(kt), float(ke), float(kb), float(se), float(sb)


@pytest.mark.parametrize("x", [1e-2, 0.7, 4.0, 45.0, 310.0, 1203.7])
def test_tensor_kernels_vs_mpmath(x):
    ls = [2, 3, 5, 20, 90, 300, 1000, 1500]
    lmax = max(ls)
    kt, ke, kb = oracle.tensor_kernels(lmax, x)
    ref = {l: kernels_mp(l, x) for l in ls}
    peak = [max(abs(v[i]) for v in ref.values()) for i in range(3)]
    for l in ls:
        rt, re, rb, se, sb = ref[l]
        # relative to the kernel's own term scale where it is not in the evanescent tail,
        # else against the largest value over l
        assert abs(kt[l] - rt) <= 1e-12 * max(abs(rt), 1e-9 * peak[0]), (l, x, kt[l], rt)
        assert abs(ke[l] - re) <= 1e-12 * max(se, 1e-9 * peak[1]), (l, x, ke[l], re)
        assert abs(kb[l] - rb) <= 1e-12 * max(sb, 1e-9 * peak[2]), (l, x, kb[l], rb)
    for arr in (kt, ke, kb):
        assert arr[0] == 0.0 and arr[1] == 0.0


def test_tensor_small_x_series():
    """Power series of j_l: j_2 = x^2/15 - x^4/210 + ..., j_3 = x^3/105 - ...; so
    K^E_2 = 4/5 - (22/105) x^2, K^B_2 = 8x/15 - 2x^3/35 + 16x^5/7560, K^T_2 = sqrt(24)(1/15 - x^2/210),
    K^E_3 = 4x/21 + O(x^3), K^B_3 = 2x^2/21 + O(x^4); at x = 0 the limits 4/5, 0, sqrt(24)/15
    at l = 2 and 0 above."""
    kt, ke, kb = oracle.tensor_kernels(6, 0.0)
    assert kt[2] == math.sqrt(24.0) / 15.0 and ke[2] == 0.8 and kb[2] == 0.0
    assert np.all(kt[3:] == 0.0) and np.all(ke[3:] == 0.0) and np.all(kb[3:] == 0.0)
    x = 1e-3
    kt, ke, kb = oracle.tensor_kernels(6, x)
    assert abs(ke[2] - (0.8 - 22.0 / 105.0 * x * x + (1 / 210 + 56 / 7560) * x ** 4)) < 2e-16
    assert abs(kb[2] - (8 * x / 15 - 2 * x ** 3 / 35 + 16 * x ** 5 / 7560)) < 1e-15 * x
    assert abs(kt[2] - math.sqrt(24.0) * (1 / 15 - x * x / 210)) < 1e-14
    assert abs(ke[3] - 4 * x / 21) < 1e-5 * 4 * x / 21
    assert abs(kb[3] - 2 * x * x / 21) < 1e-5 * 2 * x * x / 21


def test_tensor_large_x_asymptotics():
    """For x >> l^2: j_l ~ sin(x - l pi/2)/x and j_l'' ~ -j_l, so K^E ~ -2 sin(x - l pi/2)/x and
    K^B ~ 2 cos(x - l pi/2)/x, with corrections O(l^2/x^2) relative."""
    x = 2.0e5 + 0.37
    kt, ke, kb = oracle.tensor_kernels(4, x)
    for l in (2, 3, 4):
        ph = x - l * math.pi / 2
        assert abs(ke[l] + 2 * math.sin(ph) / x) < 1e-4 * 2 / x
        assert abs(kb[l] - 2 * math.cos(ph) / x) < 1e-4 * 2 / x


def _grid(nk, ntau, kmax, seed):
    rng = np.random.default_rng(seed)
    tau0 = 14000.0
    tau = np.sort(np.concatenate([[0.0, tau0], rng.uniform(0, tau0, ntau - 2)]))
    w = np.empty(ntau)
    w[1:-1] = 0.5 * (tau[2:] - tau[:-2])
    w[0], w[-1] = 0.5 * (tau[1] - tau[0]), 0.5 * (tau[-1] - tau[-2])
    k = np.exp(np.linspace(np.log(1e-4), np.log(kmax), nk))
    S = rng.normal(size=(2, nk, ntau))
    return tau0, tau, w, k, S


def test_project_tensor_brute_force_mpmath():
    """The discrete sums Delta^X_l(k_i) = sum_n w_n S_X K^X_l(k_i chi_n) on a 4 x 9 grid
    (including the x = 0 node) evaluated term by term in 40-digit mpmath."""
    tau0, tau, w, k, S = _grid(4, 9, 0.05, 3)
    lmin, lmax = 2, 40
    d, A = oracle.project_tensor(lmin, lmax, k, tau, tau0, w, S, with_abs=True)
    for i in range(k.size):
        for l in (2, 3, 7, 25, 40):
            acc = [mpmath.mpf(0)] * 3
            for n in range(tau.size):
                x = k[i] * (tau0 - tau[n])
                if x == 0.0:
                    kt, ke, kb = (math.sqrt(24.0) / 15, 0.8, 0.0) if l == 2 else (0.0, 0.0, 0.0)
                else:
                    kt, ke, kb = kernels_mp(l, x)[:3]
                acc[0] += mpmath.mpf(w[n] * S[0, i, n]) * kt
                acc[1] += mpmath.mpf(w[n] * S[1, i, n]) * ke
                acc[2] += mpmath.mpf(w[n] * S[1, i, n]) * kb
            for c in range(3):
                ref = float(acc[c])
                assert abs(d[i, l - lmin, c] - ref) <= 1e-12 * A[i, l - lmin, c] + 1e-300, \
                    (i, l, c, d[i, l - lmin, c], ref)


def test_project_tensor_delta_source_and_layout():
    """S = 1/w at one node n*: Delta^T_l = K^T_l(k chi*) from S_T alone, Delta^E and Delta^B
    from S_P alone; linear in S."""
    tau0, tau, w, k, _ = _grid(5, 30, 0.01, 4)
    n = 11
    lmax = 60
    for src in (0, 1):
        S = np.zeros((2, k.size, tau.size))
        S[src, :, n] = 1.0 / w[n]
        d = oracle.project_tensor(2, lmax, k, tau, tau0, w, S)
        for i in range(k.size):
            kt, ke, kb = oracle.tensor_kernels(lmax, k[i] * (tau0 - tau[n]))
            if src == 0:
                np.testing.assert_allclose(d[i, :, 0], kt[2:], rtol=1e-14, atol=0)
                assert np.all(d[i, :, 1:] == 0.0)
            else:
                assert np.all(d[i, :, 0] == 0.0)
                np.testing.assert_allclose(d[i, :, 1], ke[2:], rtol=1e-14, atol=0)
                np.testing.assert_allclose(d[i, :, 2], kb[2:], rtol=1e-14, atol=0)
    rng = np.random.default_rng(5)
    S1, S2 = rng.normal(size=(2, 2, k.size, tau.size))
    d1, A1 = oracle.project_tensor(2, lmax, k, tau, tau0, w, S1, with_abs=True)
    d2, A2 = oracle.project_tensor(2, lmax, k, tau, tau0, w, S2, with_abs=True)
    d12 = oracle.project_tensor(2, lmax, k, tau, tau0, w, 2.0 * S1 - 3.0 * S2)
    assert np.all(np.abs(d12 - (2 * d1 - 3 * d2)) <= 1e-13 * (2 * A1 + 3 * A2))


def test_project_tensor_rejects_lmin_below_2():
    tau0, tau, w, k, S = _grid(2, 5, 0.01, 6)
    with pytest.raises(ValueError):
        oracle.project_tensor(1, 10, k, tau, tau0, w, S)
