"""Plain FP64 CPU oracle of the C_l emulator (test infrastructure only).

Only the test suite and bench.py's cpu_baseline leg may use this module; the
GPU library never does and shares no code with it.

The emulator replaces the solve of Eq. 1-3 (gCAMB paper, Sec. 2.1) for a
parameter vector by a learned map; the paper itself motivates fast repeated
solves (Sec. 1, parameter-space sampling) but gives no emulator, so every
definition below is this project's and is written out plainly:

* inputs  u = 2 (p - lo) / (hi - lo) - 1 for the 5 source parameters;
* targets per spectrum s (TT, EE, TE, PP) over l = 2..lmax:
  y = log C for TT, EE, PP and y = asinh(C_TE / t_l) for TE, with t_l the
  lower median over the training set of |C_TE(l)| (1 where that median is 0:
  then every |C_TE(l)| below the median is 0 and asinh(0 / t) = 0 for any t);
* PCA per spectrum: mean mu_s, basis V_s = top ncomp eigenvectors of the
  covariance of y_s, coefficients c = (y - mu) V, scaled targets
  z = c / sigma_s with one scale per spectrum, sigma_s = sqrt of the summed
  variance of the kept components (see :func:`target_scale`);
* MLP: h_0 = u, h_{i+1} = GELU(h_i W_i^T + b_i) for the hidden layers,
  output h_d W_d^T + b_d; GELU(x) = x (1 + erf(x / sqrt 2)) / 2;
* loss: mean over batch and outputs of (out - z)^2;
* Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias correction;
* ensemble of E members: prediction = mean over members of C_l; error
  estimate = max over spectra, l and members of |C_e - C_mean| / scale with
  scale |C_mean| (TT, EE, PP) or sqrt(C_mean,TT C_mean,EE) (TE).

Flat parameter layout of one member: for each layer, W (out x in,
row-major) then b (out).
"""
from __future__ import annotations

import math

import numpy as np

SQRT1_2 = 1.0 / math.sqrt(2.0)
MASK64 = (1 << 64) - 1


# ---------------------------------------------------------------- generator

def splitmix64(state: int):
    """One step of SplitMix64 (Steele, Lea, Flood 2014): returns (new_state, output)."""
    state = (state + 0x9E3779B97F4A7C15) & MASK64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return state, z ^ (z >> 31)


# ---------------------------------------------------------------- MLP

def gelu(x):
    from scipy.special import erf
    return 0.5 * x * (1.0 + erf(x * SQRT1_2))


def gelu_grad(x):
    from scipy.special import erf
    return 0.5 * (1.0 + erf(x * SQRT1_2)) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def layer_sizes(nin, width, depth, nout):
    return [nin] + [width] * depth + [nout]


def unflatten(theta, sizes):
    """Split a flat parameter vector into [(W, b)] per layer."""
    out, o = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        W = theta[o:o + a * b].reshape(b, a)
        o += a * b
        bias = theta[o:o + b]
        o += b
        out.append((W, bias))
    assert o == theta.size
    return out


def n_params(sizes):
    return sum(a * b + b for a, b in zip(sizes[:-1], sizes[1:]))


def forward(theta, sizes, u):
    """Returns (output, [pre-activations], [activations]) for inputs u [n, nin]."""
    layers = unflatten(np.asarray(theta, dtype=np.float64), sizes)
    h = np.asarray(u, dtype=np.float64)
    acts, pres = [h], []
    for i, (W, b) in enumerate(layers):
        z = h @ W.T + b
        pres.append(z)
        h = gelu(z) if i < len(layers) - 1 else z
        acts.append(h)
    return h, pres, acts


def loss_and_grad(theta, sizes, u, target):
    """MSE loss over batch and outputs, and its gradient with respect to theta (backprop)."""
    out, pres, acts = forward(theta, sizes, u)
    n, m = out.shape
    diff = out - target
    loss = float(np.mean(diff * diff))
    layers = unflatten(np.asarray(theta, dtype=np.float64), sizes)
    g = 2.0 * diff / (n * m)             # d loss / d output
    grads = []
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        if i < len(layers) - 1:
            g = g * gelu_grad(pres[i])
        grads.append((g.T @ acts[i], g.sum(axis=0)))
        g = g @ W
    flat = []
    for gW, gb in reversed(grads):
        flat.append(gW.ravel())
        flat.append(gb)
    return loss, np.concatenate(flat)


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


# ---------------------------------------------------------------- targets and PCA

def te_scale(cl_te):
    """Lower median over samples (axis 0) of |C_TE|, per l; 1 where it is 0."""
    a = np.sort(np.abs(cl_te), axis=0)
    t = a[(a.shape[0] - 1) // 2].copy()
    t[t == 0] = 1.0
    return t


def transform(cl, t):
    """cl [n, 4, nl] (TT, EE, TE, PP) -> y [n, 4, nl]."""
    y = np.empty_like(cl, dtype=np.float64)
    y[:, 0] = np.log(cl[:, 0])
    y[:, 1] = np.log(cl[:, 1])
    y[:, 2] = np.arcsinh(cl[:, 2] / t)
    y[:, 3] = np.log(cl[:, 3])
    return y


def inverse_transform(y, t):
    cl = np.empty_like(y)
    cl[:, 0] = np.exp(y[:, 0])
    cl[:, 1] = np.exp(y[:, 1])
    cl[:, 2] = t * np.sinh(y[:, 2])
    cl[:, 3] = np.exp(y[:, 3])
    return cl


def pca_fit(y, ncomp):
    """Per spectrum: mean, top-ncomp eigenvectors of the covariance (columns, by decreasing
    eigenvalue), all eigenvalues (descending).  y [n, nspec, nl]."""
    n = y.shape[0]
    means, bases, evals = [], [], []
    for s in range(y.shape[1]):
        mu = y[:, s].mean(axis=0)
        X = y[:, s] - mu
        C = X.T @ X / n
        w, V = np.linalg.eigh(C)
        order = np.argsort(w)[::-1]
        means.append(mu)
        bases.append(V[:, order[:ncomp]])
        evals.append(w[order])
    return np.stack(means), np.stack(bases), np.stack(evals)


def target_scale(evals, ncomp):
    """sigma_s = sqrt(sum of the top ncomp covariance eigenvalues) per spectrum: the coefficient
    c_j has variance lambda_j, so z = c / sigma_s has total variance 1 per spectrum."""
    return np.sqrt(evals[:, :ncomp].sum(axis=1))


def pca_floor(evals, ncomp):
    """Mean squared reconstruction error per sample of the best rank-ncomp projection:
    the sum of the discarded covariance eigenvalues."""
    return evals[:, ncomp:].sum(axis=1)


def ensemble_stats(cls):
    """cls [E, n, 4, nl] -> (mean [n, 4, nl], error estimate [n])."""
    mean = cls.mean(axis=0)
    scale = np.abs(mean).copy()
    scale[:, 2] = np.sqrt(mean[:, 0] * mean[:, 1])
    dev = np.abs(cls - mean[None]) / scale[None]
    return mean, dev.max(axis=(0, 2, 3))
