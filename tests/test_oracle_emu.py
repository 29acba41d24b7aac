"""Pins of the emulator oracle (oracle/emu_oracle.py) against facts fixed
independently of it: published generator outputs, identities of GELU, central
finite differences, Adam's closed-form first step, the Eckart-Young truncation
error of PCA, library routines for SVD and medians."""
import math
import statistics

import numpy as np

from oracle import emu_oracle as eo


def test_splitmix64_reference_outputs():
    # SplitMix64 seeded with 0: the first outputs quoted with the generator's reference code
    s, a = eo.splitmix64(0)
    s, b = eo.splitmix64(s)
    s, c = eo.splitmix64(s)
    assert (a, b, c) == (0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F)


def test_gelu_identities():
    x = np.linspace(-6, 6, 101)
    assert eo.gelu(np.array([0.0]))[0] == 0.0
    np.testing.assert_allclose(eo.gelu(x) - eo.gelu(-x), x, atol=1e-15)       # x Phi(x) + x Phi(-x) - x ... = x
    np.testing.assert_allclose(eo.gelu(np.array([40.0])), [40.0], rtol=0, atol=0)
    h = 1e-6
    fd = (eo.gelu(x + h) - eo.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(eo.gelu_grad(x), fd, atol=1e-9)
    # GELU(1) = Phi(1) with the standard normal CDF
    assert abs(eo.gelu(np.array([1.0]))[0] - 0.5 * (1 + math.erf(1 / math.sqrt(2)))) < 1e-16


def test_mlp_gradient_vs_finite_differences():
    rng = np.random.default_rng(3)
    sizes = eo.layer_sizes(5, 7, 3, 4)
    theta = rng.normal(size=eo.n_params(sizes)) * 0.5
    u = rng.uniform(-1, 1, size=(6, 5))
    tgt = rng.normal(size=(6, 4))
    loss, g = eo.loss_and_grad(theta, sizes, u, tgt)
    h = 1e-6
    idx = rng.choice(theta.size, 40, replace=False)
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        lp, _ = eo.loss_and_grad(tp, sizes, u, tgt)
        lm, _ = eo.loss_and_grad(tm, sizes, u, tgt)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, g[i])


def test_linear_net_gradient_closed_form():
    """No hidden layer: out = u W^T + b, so d loss / dW = 2/(n m) (out - t)^T u."""
    rng = np.random.default_rng(4)
    sizes = [3, 2]
    theta = rng.normal(size=eo.n_params(sizes))
    u = rng.normal(size=(5, 3))
    t = rng.normal(size=(5, 2))
    W = theta[:6].reshape(2, 3)
    b = theta[6:]
    d = u @ W.T + b - t
    _, g = eo.loss_and_grad(theta, sizes, u, t)
    np.testing.assert_allclose(g[:6], (2.0 / 10) * (d.T @ u).ravel(), rtol=1e-14)
    np.testing.assert_allclose(g[6:], (2.0 / 10) * d.sum(axis=0), rtol=1e-14)


def test_adam_first_step_closed_form():
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    th, m, v = eo.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    # bias correction makes m_hat = g and v_hat = g^2 at t = 1
    np.testing.assert_allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-15)


def test_adam_constant_gradient_three_steps():
    """With the same gradient at every step, m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so
    the bias-corrected moments are exactly g and g^2 at every t and each step moves theta by
    -lr g / (|g| + eps).  A wrong correction exponent at t >= 2 breaks this."""
    g = np.array([3.0, -0.5, 2.0 ** -10, 7.25])
    th, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    for t in (1, 2, 3):
        th, m, v = eo.adam_step(th, g, m, v, t, lr=0.01)
        np.testing.assert_allclose(m, (1 - 0.9 ** t) * g, rtol=1e-15)
        np.testing.assert_allclose(v, (1 - 0.999 ** t) * g * g, rtol=1e-12)
        np.testing.assert_allclose(th, -0.01 * t * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_adam_two_steps_hand_computed():
    """Adam (Kingma and Ba, Algorithm 1) for one parameter, gradients 1 then -2, lr 0.1,
    carried out in exact rational arithmetic for the moments and their bias corrections (the
    oracle's FP64 evaluation agrees to rounding; a wrong bias-correction power moves theta by
    more than 1e-2):
      t=1: m = 1/10, v = 1/1000, mhat = 1, vhat = 1;
      t=2: m = -11/100, v = 4999/1000000, mhat = -11/19, vhat = 4999/1999."""
    from fractions import Fraction as F
    b1, b2 = F(9, 10), F(999, 1000)
    m1, v1 = (1 - b1) * 1, (1 - b2) * 1
    m2, v2 = b1 * m1 + (1 - b1) * (-2), b2 * v1 + (1 - b2) * 4
    assert (m2, v2) == (F(-11, 100), F(4999, 1000000))
    mh2, vh2 = m2 / (1 - b1 ** 2), v2 / (1 - b2 ** 2)
    assert (mh2, vh2) == (F(-11, 19), F(4999, 1999))
    th1 = -0.1 * 1.0 / (1.0 + 1e-8)
    th2 = th1 - 0.1 * float(mh2) / (np.sqrt(float(vh2)) + 1e-8)
    th, m, v = eo.adam_step(np.zeros(1), np.array([1.0]), np.zeros(1), np.zeros(1), 1, lr=0.1)
    assert abs(th[0] - th1) <= 1e-16
    th, m, v = eo.adam_step(th, np.array([-2.0]), m, v, 2, lr=0.1)
    assert abs(m[0] - float(m2)) <= 1e-15 and abs(v[0] - float(v2)) <= 1e-15
    assert abs(th[0] - th2) <= 1e-13, (th[0], th2)
    # the third step with gradient 0.5 continues the same recursion
    m3, v3 = b1 * m2 + (1 - b1) * F(1, 2), b2 * v2 + (1 - b2) * F(1, 4)
    th3 = th2 - 0.1 * float(m3 / (1 - b1 ** 3)) / (np.sqrt(float(v3 / (1 - b2 ** 3))) + 1e-8)
    th, m, v = eo.adam_step(th, np.array([0.5]), m, v, 3, lr=0.1)
    assert abs(th[0] - th3) <= 1e-13, (th[0], th3)


def test_pca_truncation_floor_and_svd():
    rng = np.random.default_rng(5)
    n, nl, k = 300, 40, 6
    basis = np.linalg.qr(rng.normal(size=(nl, nl)))[0]
    spec = np.exp(-0.4 * np.arange(nl))
    y = (rng.normal(size=(n, nl)) * spec) @ basis.T + 3.0
    y = np.stack([y, 2 * y, -y, y + 1], axis=1)
    mu, V, w = eo.pca_fit(y, k)
    floor = eo.pca_floor(w, k)
    for s in range(4):
        X = y[:, s] - mu[s]
        rec = X @ V[s] @ V[s].T
        mse = np.mean(np.sum((X - rec) ** 2, axis=1))
        assert abs(mse - floor[s]) <= 1e-10 * max(floor[s], 1e-300) + 1e-13
        # same subspace as the top right singular vectors of the centred data
        Us, Ss, Vt = np.linalg.svd(X, full_matrices=False)
        P1 = V[s] @ V[s].T
        P2 = Vt[:k].T @ Vt[:k]
        assert np.max(np.abs(P1 - P2)) < 1e-9
        np.testing.assert_allclose(w[s][:k], Ss[:k] ** 2 / n, rtol=1e-10)
        # the per-spectrum target scale makes the scaled coefficients' total variance 1
        z = (X @ V[s]) / eo.target_scale(w, k)[s]
        assert abs(np.sum(np.mean(z * z, axis=0)) - 1.0) < 1e-12


def test_te_scale_is_lower_median_and_transform_roundtrip():
    rng = np.random.default_rng(6)
    te = rng.normal(size=(7, 5))
    t = eo.te_scale(te)
    for l in range(5):
        assert t[l] == statistics.median_low(list(np.abs(te[:, l])))
    z = np.zeros((4, 2))
    z[3, 1] = 2.0
    np.testing.assert_array_equal(eo.te_scale(z), [1.0, 1.0])    # zero median -> 1
    cl = np.stack([np.exp(rng.normal(size=(7, 5))), np.exp(rng.normal(size=(7, 5))), te,
                   np.exp(rng.normal(size=(7, 5)))], axis=1)
    back = eo.inverse_transform(eo.transform(cl, t), t)
    np.testing.assert_allclose(back, cl, rtol=1e-13)


def test_ensemble_error_closed_form():
    rng = np.random.default_rng(7)
    c = np.exp(rng.normal(size=(3, 4, 9)))
    c[:, 2] = rng.normal(size=(3, 9)) * 0.1
    same = np.stack([c, c])
    mean, err = eo.ensemble_stats(same)
    np.testing.assert_array_equal(mean, c)
    assert np.all(err == 0)
    d = 1e-3
    mean, err = eo.ensemble_stats(np.stack([c, c * (1 + d)]))
    # auto spectra: |c - c (1 + d/2)| / (c (1 + d/2)) = (d/2) / (1 + d/2); TE is scaled by
    # sqrt(TT EE) and is small here, so the auto spectra set the maximum
    np.testing.assert_allclose(err, (d / 2) / (1 + d / 2), rtol=1e-12)
