"""GPU parity of the tensor-mode projection (los_project_tensor) against the CPU oracle,
through the C ABI.

The oracle (oracle.project_tensor) evaluates the published tensor kernels
  K^T_l = sqrt((l+2)!/(l-2)!) j_l / x^2,  K^E_l = -j_l + j_l'' + 2 j_l/x^2 + 4 j_l'/x,
  K^B_l = 2 j_l' + 4 j_l/x
from j_l and its derivatives at every node; the GPU sweeps the columns S_P, S_P/x, S_P/x^2,
S_T/x^2 over the rows lmin-1 .. lmax and combines neighbouring rows (j_l' and j_l'' written
through j_{l-1} and j_l).  Different formulas, so agreement checks both.

Bound, normwise per (l, output) as for the scalar FP64 path (the 1e-10 target):
  max_k |Delta - Delta_ref| <= 1e-10 * max_k scale,
scale = the oracle's absolute term sums plus the absolute sums of the terms the GPU combines
(E: 2|P0_l| + 2|P1_{l-1}| + l(l-1)|P2_l|; B: 2|P0_{l-1}| + 2(l-1)|P1_l|, with
P_p,m = sum_n |w S_P j_m / x^p|, from the oracle's plain projection).  Either formula's
rounding error is a small multiple of its own term sums, so their difference is bounded by
their sum.  C_l: 1e-10 relative elementwise for TT, EE, BB and TE relative to sqrt(TT EE).
"""
import os

import numpy as np
import pytest

import oracle
from paper_2509_25110_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN_T2 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "t2_cl_oracle.txt")
TOL = 1e-10


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def ctx(torch_dev):
    from paper_2509_25110_amd import los
    c = los.Context()
    yield c
    c.close()


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_tensor(torch, ctx, wl, cl=True):
    d = ctx.los_project_tensor(wl.lmin, wl.lmax, dev(torch, wl.k), dev(torch, wl.tau), wl.tau0,
                               dev(torch, wl.w_tau), dev(torch, wl.S))
    c = ctx.cl_integrate(d, dev(torch, wl.w_lnk), dev(torch, wl.Pk), wl.pairs) if cl else None
    torch.cuda.synchronize()
    return d.cpu().numpy(), (c.cpu().numpy() if cl else None)


def gpu_term_scale(wl, rows=None):
    """Absolute term sums of the GPU's row combination (see the module docstring)."""
    k = wl.k if rows is None else wl.k[rows]
    S = wl.S if rows is None else wl.S[:, rows, :]
    x = k[:, None] * (wl.tau0 - wl.tau)[None, :]
    with np.errstate(divide="ignore"):
        ix = np.where(x > 0, 1.0 / np.where(x > 0, x, 1.0), 0.0)
    Sx = np.stack([S[1], S[1] * ix, S[1] * ix * ix])
    _, A = oracle.project(wl.lmin - 1, wl.lmax, k, wl.tau, wl.tau0, wl.w_tau, Sx, with_abs=True)
    l = np.arange(wl.lmin, wl.lmax + 1, dtype=np.float64)[None, :]
    hi, lo = A[:, 1:, :], A[:, :-1, :]
    sE = 2 * hi[..., 0] + 2 * lo[..., 1] + l * (l - 1) * hi[..., 2]
    sB = 2 * lo[..., 0] + 2 * (l - 1) * hi[..., 1]
    return sE, sB


def normwise_err(d, ref, Aor, sE, sB):
    scale = Aor.copy()
    scale[..., 1] += sE
    scale[..., 2] += sB
    top = np.maximum(np.max(scale, axis=0, keepdims=True), 1e-300)
    return float(np.max(np.abs(d - ref) / top))


def cl_err(c, cref, pairs):
    worst = 0.0
    for p, (a, b) in enumerate(pairs):
        if a == b:
            rel = np.abs(c[p] / cref[p] - 1)
        else:
            rel = np.abs(c[p] - cref[p]) / np.sqrt(cref[pairs.index((a, a))] *
                                                    cref[pairs.index((b, b))])
        worst = max(worst, float(np.max(rel)))
    return worst


SMALL = [
    dict(lmax=40, nk=12, kmax=0.02, ntau=200),                # one block of rows
    dict(lmax=150, nk=9, kmax=0.05, ntau=700),                # ragged l and tau
    dict(lmax=333, nk=16, kmax=3000.0 / 14000, ntau=1500),    # several blocks, x >> lmax at high k
    dict(lmax=61, nk=7, kmax=6e-3, ntau=64),                  # small x only
    dict(lmax=90, nk=5, kmax=0.2, ntau=190, kmin=0.01),       # x >> lmax for most nodes
]


@pytest.mark.parametrize("cfg", SMALL, ids=[str(i) for i in range(len(SMALL))])
def test_tensor_small_vs_oracle(torch_dev, ctx, cfg):
    wl = inputs.tensor_workload(**cfg)
    d, c = run_tensor(torch_dev, ctx, wl)
    assert np.all(np.isfinite(d)) and np.all(np.isfinite(c))
    ref, Aor = oracle.project_tensor(wl.lmin, wl.lmax, wl.k, wl.tau, wl.tau0, wl.w_tau, wl.S,
                                     with_abs=True)
    sE, sB = gpu_term_scale(wl)
    err = normwise_err(d, ref, Aor, sE, sB)
    cref = oracle.cl(ref, wl.w_lnk, wl.Pk, wl.pairs)
    cerr = cl_err(c, cref, list(wl.pairs))
    print("tensor %s: delta normwise %.2e, C_l rel %.2e" % (cfg, err, cerr))
    assert err <= TOL, err
    assert cerr <= TOL, cerr


def test_tensor_lmin_above_2(torch_dev, ctx):
    """lmin > 2: the rows start at lmin - 1 inside the sweep; no limit terms."""
    wl = inputs.tensor_workload(lmax=120, nk=6, kmax=0.05, ntau=400)
    full, _ = run_tensor(torch_dev, ctx, wl, cl=False)
    for lmin in (3, 17, 18, 37, 120):
        wl.lmin = lmin
        d, _ = run_tensor(torch_dev, ctx, wl, cl=False)
        ref, Aor = oracle.project_tensor(lmin, wl.lmax, wl.k, wl.tau, wl.tau0, wl.w_tau, wl.S,
                                         with_abs=True)
        sE, sB = gpu_term_scale(wl)
        assert normwise_err(d, ref, Aor, sE, sB) <= TOL, lmin
        # the same rows as the lmin = 2 run (blocks start elsewhere, so equal to rounding)
        np.testing.assert_allclose(d, full[:, lmin - 2:, :], rtol=0,
                                   atol=1e-12 * np.max(np.abs(full)))


def test_tensor_x_zero_limits(torch_dev, ctx):
    """A single node at tau = tau0 (x = 0 for every k) with the others weighted 0: the
    transfer functions are the kernels' limits, K^T_2 = sqrt(24)/15, K^E_2 = 4/5, all else 0."""
    wl = inputs.tensor_workload(lmax=20, nk=3, kmax=0.02, ntau=64)
    w = np.zeros_like(wl.w_tau)
    w[-1] = 1.0
    wl.w_tau = w
    S = np.zeros_like(wl.S)
    S[0, :, -1] = 2.0
    S[1, :, -1] = 3.0
    wl.S = S
    d, _ = run_tensor(torch_dev, ctx, wl, cl=False)
    want = np.zeros_like(d)
    want[:, 0, 0] = 2.0 * np.sqrt(24.0) / 15.0
    want[:, 0, 1] = 3.0 * 0.8
    np.testing.assert_allclose(d, want, rtol=1e-15, atol=1e-300)


def test_tensor_delta_source(torch_dev, ctx):
    """One node n* with S = 1/w: Delta_l(k) equals the kernel at x = k chi_{n*} (the oracle's
    tensor_kernels, evaluated pointwise)."""
    wl = inputs.tensor_workload(lmax=200, nk=8, kmax=0.1, ntau=300)
    ns = 123
    S = np.zeros_like(wl.S)
    S[:, :, ns] = 1.0 / wl.w_tau[ns]
    wl.S = S
    d, _ = run_tensor(torch_dev, ctx, wl, cl=False)
    chi = wl.tau0 - wl.tau[ns]
    for i in range(wl.nk):
        kt, ke, kb = oracle.tensor_kernels(wl.lmax, wl.k[i] * chi)
        want = np.stack([kt[2:], ke[2:], kb[2:]], axis=1)
        scale = np.max(np.abs(want), axis=0, keepdims=True) + 1e-300
        assert np.max(np.abs(d[i] - want) / scale) <= 1e-11, i


def test_tensor_deterministic(torch_dev, ctx):
    wl = inputs.tensor_workload(lmax=300, nk=10, kmax=0.1, ntau=900)
    a, ca = run_tensor(torch_dev, ctx, wl)
    b, cb = run_tensor(torch_dev, ctx, wl)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(ca, cb)


def test_tensor_argument_errors(torch_dev, ctx):
    from paper_2509_25110_amd import los
    wl = inputs.tensor_workload(lmax=20, nk=3, ntau=64)
    with pytest.raises(ValueError):   # S must be [2, nk, ntau]
        ctx.los_project_tensor(2, 20, dev(torch_dev, wl.k), dev(torch_dev, wl.tau), wl.tau0,
                               dev(torch_dev, wl.w_tau), dev(torch_dev, wl.S[:1]))
    with pytest.raises(los.LosError):  # lmin < 2
        ctx.los_project_tensor(1, 20, dev(torch_dev, wl.k), dev(torch_dev, wl.tau), wl.tau0,
                               dev(torch_dev, wl.w_tau), dev(torch_dev, wl.S))


def test_t2_full_size(torch_dev, ctx):
    """The tensor workload at the paper's tensor settings (l = 2..1500, k up to 3000/tau0,
    2000 log-k, 3000 tau) in the launch configuration bench.py times: every C_l within 1e-10
    of the oracle (golden file written by make_golden.py T2), and sampled k rows of Delta
    normwise within 1e-10."""
    wl = inputs.tensor_workload()
    d, c = run_tensor(torch_dev, ctx, wl)
    gold = np.loadtxt(GOLDEN_T2)
    assert gold.shape[0] == wl.nl
    cerr = cl_err(c, gold[:, 1:].T, list(wl.pairs))
    rows = np.array([0, 1, 500, 1000, 1501, 1750, 1998, 1999])
    ref, Aor = oracle.project_tensor(wl.lmin, wl.lmax, wl.k[rows], wl.tau, wl.tau0, wl.w_tau,
                                     wl.S[:, rows, :], with_abs=True)
    sE, sB = gpu_term_scale(wl, rows)
    err = normwise_err(d[rows], ref, Aor, sE, sB)
    print("T2: C_l rel err %.3e, delta normwise (sampled rows) %.3e" % (cerr, err))
    assert cerr <= TOL, cerr
    assert err <= TOL, err
