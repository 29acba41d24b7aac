"""GPU parity of the source interpolation in k (the InterpolateSources step of the
gCAMB paper, Sec. 3.2, read as the natural cubic spline in k at each tau node):
los_spline_sources (second derivatives) and los_interp_sources (evaluation)
against the oracle (oracle/spline_oracle.py), and the chain spline ->
interpolation -> projection against the oracle's chain.

Bounds.  The spline matrix is strictly diagonally dominant (off-diagonal sum
half the diagonal), so its condition number is at most 3 and a backward-stable
solve in FP64 differs from another by a few ulps of max|M| per column: M is
checked normwise per column at 1e-13.  The evaluation is a 4-term sum with
weights bounded by 1 + h^2 |M| terms: checked at 1e-14 of the column's
max(|y|, h^2 |M|) scale; FP32 output at half an FP32 ulp plus that."""
import numpy as np
import pytest

import oracle
from oracle import spline_oracle as so
from paper_2509_25110_amd import inputs

pytestmark = pytest.mark.gpu


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


def knots(rng, N):
    return np.cumsum(rng.uniform(0.05, 1.0, N)) + 0.3


def check_M(got, ref):
    scale = np.maximum(np.abs(ref).max(axis=1, keepdims=True), 1e-300)
    err = float(np.max(np.abs(got - ref) / scale))
    assert err <= 1e-13, err
    # natural ends are exactly zero
    assert np.all(got[:, 0, :] == 0.0) and np.all(got[:, -1, :] == 0.0)


@pytest.mark.parametrize("N,nsrc,ntau", [
    (2, 2, 9),        # straight lines: M = 0, no system
    (3, 1, 5),        # one unknown
    (17, 2, 33),      # 15 unknowns: one partial segment
    (18, 1, 64),      # 16 unknowns: exactly one segment
    (19, 3, 7),       # 17: a second segment with one row; ragged column groups
    (40, 3, 50),
    (514, 2, 40),     # 32 segments, 16 columns per workgroup
    (1026, 1, 20),    # 64 segments, 8 columns per workgroup
    (1027, 2, 13),    # 65 segments, 4 columns per workgroup
    (4098, 1, 9),     # 256 segments, 2 columns
    (8194, 1, 5),     # 512 segments, 1 column
    (8211, 1, 4),     # 513 segments (last one partial), 1 column, 576 threads
    (16386, 1, 3),    # 1024 segments (the maximum), 1 column, 1024 threads
])
def test_second_derivatives_parity(torch_dev, ctx, N, nsrc, ntau):
    torch = torch_dev
    rng = np.random.default_rng(N * 7 + ntau)
    q = knots(rng, N)
    Sc = rng.normal(size=(nsrc, N, ntau))
    M = ctx.los_spline_sources(dev(torch, q), dev(torch, Sc))
    torch.cuda.synchronize()
    check_M(M.cpu().numpy(), so.second_derivatives(q, Sc))


def test_second_derivatives_log_grid_reuse(torch_dev, ctx):
    """Log-spaced knots over 3.7 decades (the workload's grid shape), then a second
    call on a smaller grid reusing the context's tables."""
    torch = torch_dev
    wl = inputs.config("C1")
    cs = inputs.coarse_sources(wl, inputs.COARSE_NK["C1"])
    M = ctx.los_spline_sources(dev(torch, cs.q), dev(torch, cs.Sc))
    torch.cuda.synchronize()
    check_M(M.cpu().numpy(), so.second_derivatives(cs.q, cs.Sc))
    rng = np.random.default_rng(5)
    q = knots(rng, 21)
    Sc = rng.normal(size=(2, 21, 11))
    M2 = ctx.los_spline_sources(dev(torch, q), dev(torch, Sc))
    torch.cuda.synchronize()
    check_M(M2.cpu().numpy(), so.second_derivatives(q, Sc))


def eval_scale(q, Sc, M, k):
    j = so.interval(q, k)
    h = q[j + 1] - q[j]
    y = np.maximum(np.abs(Sc[:, j, :]), np.abs(Sc[:, j + 1, :]))
    m = np.maximum(np.abs(M[:, j, :]), np.abs(M[:, j + 1, :])) * (h * h)[None, :, None]
    return np.maximum(y, m) + 1e-300


@pytest.mark.parametrize("out_prec", [0, 1])
def test_interp_parity(torch_dev, ctx, out_prec):
    torch = torch_dev
    rng = np.random.default_rng(11 + out_prec)
    N, nsrc, ntau = 57, 3, 301
    q = knots(rng, N)
    Sc = rng.normal(size=(nsrc, N, ntau))
    M = so.second_derivatives(q, Sc)
    # inside, at every knot, and outside at both ends (end cubics)
    k = np.sort(np.concatenate([rng.uniform(q[0], q[-1], 200), q,
                                [q[0] - 0.2, q[0] - 1e-9, q[-1] + 1e-9, q[-1] + 0.3]]))
    S = ctx.los_interp_sources(dev(torch, q), dev(torch, Sc), dev(torch, M), dev(torch, k),
                               out_prec=out_prec)
    torch.cuda.synchronize()
    got = S.cpu().numpy().astype(np.float64)
    ref = so.evaluate(q, Sc, M, k)
    scale = eval_scale(q, Sc, M, k)
    err = np.abs(got - ref) / scale
    if out_prec == 0:
        assert float(err.max()) <= 1e-14, float(err.max())
    else:
        assert np.all(np.abs(got - ref) <= 2.0 ** -24 * np.abs(ref) + 1e-14 * scale)
    # at the knots the spline reproduces the data
    at = np.searchsorted(k, q)
    assert np.allclose(got[:, at, :], Sc, rtol=0, atol=(1e-14 if out_prec == 0 else 1e-7) * 4)


def test_chain_c2_full_size_sampled(torch_dev, ctx):
    """The C2 workload with its sources given on 1000 coarse knots: GPU spline ->
    GPU interpolation onto the 4000 LOS k -> GPU FP64 projection, against the oracle's
    spline, interpolation and projection on sampled k rows (the launch shapes are the
    full-size ones)."""
    torch = torch_dev
    wl = inputs.config("C2")
    cs = inputs.coarse_sources(wl, inputs.COARSE_NK["C2"])
    q_d, Sc_d = dev(torch, cs.q), dev(torch, cs.Sc)
    M_d = ctx.los_spline_sources(q_d, Sc_d)
    S_d = ctx.los_interp_sources(q_d, Sc_d, M_d, dev(torch, wl.k))
    d = ctx.los_project(wl.lmin, wl.lmax, dev(torch, wl.k), dev(torch, wl.tau), wl.tau0,
                        dev(torch, wl.w_tau), S_d)
    torch.cuda.synchronize()
    M_ref = so.second_derivatives(cs.q, cs.Sc)
    check_M(M_d.cpu().numpy(), M_ref)
    rows = np.array([0, 1, 7, 999, 2000, 3333, wl.nk - 2, wl.nk - 1])
    S_ref = so.evaluate(cs.q, cs.Sc, M_ref, wl.k[rows])
    S_got = S_d[:, torch.from_numpy(rows).cuda(), :].cpu().numpy()
    err = np.abs(S_got - S_ref) / eval_scale(cs.q, cs.Sc, M_ref, wl.k[rows])
    assert float(err.max()) <= 1e-14, float(err.max())
    pick = rows[[0, 4, 7]]
    ref, A = oracle.project(wl.lmin, wl.lmax, wl.k[pick], wl.tau, wl.tau0, wl.w_tau,
                            so.evaluate(cs.q, cs.Sc, M_ref, wl.k[pick]), with_abs=True)
    got = d[torch.from_numpy(pick).cuda()].cpu().numpy()
    scale = np.maximum(A.max(axis=0, keepdims=True), 1e-300)
    assert float(np.max(np.abs(got - ref) / scale)) <= 1e-10
