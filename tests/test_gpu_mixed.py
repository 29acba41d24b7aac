"""GPU parity of the mixed-precision projection (LOS_FP32, LOS_BF16X3) against
the CPU oracle, through the C ABI.

The oracle gets the same float32 source values the GPU gets (S rounded to FP32,
then widened), so only the path's own arithmetic is tested.  Bounds:
  * Delta normwise, per (l, source): max_k |Delta - Delta_ref| <= eps * max_k A
    with A = sum_n |w_n S j_l| and
      FP32:   eps = (ntau + 2) 2^-24   (J rounded to FP32, FP32 accumulation)
      BF16X3: eps = 3 2^-16 + (ntau + 2) 2^-24   (split-product error on top);
  * C_l: 1e-4 relative elementwise (TE relative to sqrt(TT EE)), the accuracy
    the mixed path is specified to keep, on the full-size workload.  On the
    small grids some C_l are ill-conditioned (coarse tau sampling of a fast
    oscillation leaves |Delta| far below A), so there the bound is
    max(1e-4 |C_ref|, 2.2 eps CA) with CA = 4 pi sum_i w_i P_i A_a A_b, the
    first-order propagation of the normwise Delta bound; each run reports the
    plain relative error as well.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2509_25110_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN_C3 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_cl_oracle.txt")
PRECS = {"fp32": 1, "bf16x3": 2}


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


def run_mixed(torch, ctx, wl, prec):
    S32 = np.ascontiguousarray(wl.S.astype(np.float32))
    d = ctx.los_project(wl.lmin, wl.lmax, dev(torch, wl.k), dev(torch, wl.tau), wl.tau0,
                        dev(torch, wl.w_tau), dev(torch, S32), prec=prec)
    c = ctx.cl_integrate(d, dev(torch, wl.w_lnk), dev(torch, wl.Pk), wl.pairs)
    torch.cuda.synchronize()
    return d.cpu().numpy().astype(np.float64), c.cpu().numpy(), S32.astype(np.float64)


def eps_for(prec, ntau):
    e = (ntau + 2) * 2.0 ** -24
    return e + 3 * 2.0 ** -16 if prec == 2 else e


def cl_rel_err(c, cref, pairs):
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
    dict(lmax=61, nk=12, kmax=0.02, ntau=300, nsrc=3),             # ragged l blocks
    dict(lmax=130, nk=10, kmax=0.03, ntau=700, nsrc=1),            # ragged tau blocks
    dict(lmax=200, nk=9, kmax=0.05, ntau=1000, nsrc=2),
    dict(lmax=90, nk=7, kmax=0.2, ntau=190, nsrc=3, kmin=0.01),    # x >> lmax for most nodes
    dict(lmax=333, nk=16, kmax=0.1, ntau=2500, nsrc=3),
    dict(lmax=60, nk=5, kmax=6e-3, ntau=64, nsrc=3),               # small x only
]


@pytest.mark.parametrize("prec", list(PRECS), ids=list(PRECS))
@pytest.mark.parametrize("cfg", SMALL, ids=[str(i) for i in range(len(SMALL))])
def test_mixed_small_vs_oracle(torch_dev, ctx, cfg, prec):
    p = PRECS[prec]
    wl = inputs.small(**cfg)
    d, c, S64 = run_mixed(torch_dev, ctx, wl, p)
    assert np.all(np.isfinite(d)) and np.all(np.isfinite(c))
    ref, A = oracle.project(wl.lmin, wl.lmax, wl.k, wl.tau, wl.tau0, wl.w_tau, S64, with_abs=True)
    scale = np.maximum(np.max(A, axis=0, keepdims=True), 1e-300)
    err = float(np.max(np.abs(d - ref) / scale))
    assert err <= eps_for(p, wl.ntau), (prec, err)
    cref = oracle.cl(ref, wl.w_lnk, wl.Pk, wl.pairs)
    cerr = cl_rel_err(c, cref, list(wl.pairs))
    CA = oracle.cl(A, wl.w_lnk, wl.Pk, wl.pairs)
    bound = np.maximum(1e-4 * np.abs(cref), 2.2 * eps_for(p, wl.ntau) * CA)
    worst = float(np.max(np.abs(c - cref) / bound))
    print("mixed %s cfg %s: delta normwise %.2e, C_l rel %.2e, C_l err / bound %.2e"
          % (prec, cfg, err, cerr, worst))
    assert worst <= 1.0, (prec, worst, cerr)


@pytest.mark.parametrize("mb,nc", [(1, 1), (2, 1), (2, 2), (4, 4), (16, 8)])
def test_mixed_tiles_agree(torch_dev, ctx, mb, nc, monkeypatch):
    """Table pipeline: every compiled tile shape, including the LDS-staged 256 x 128 kernel,
    gives the same Delta (bitwise: the tau order of the accumulation does not depend on the
    tile)."""
    monkeypatch.setenv("LOS_MIXED_FUSED", "0")
    wl = inputs.small(lmax=150, nk=6, kmax=0.05, ntau=700, nsrc=3)
    base, _, _ = run_mixed(torch_dev, ctx, wl, 2)
    monkeypatch.setenv("LOS_GEMM_MB", str(mb))
    monkeypatch.setenv("LOS_GEMM_NC", str(nc))
    d, _, _ = run_mixed(torch_dev, ctx, wl, 2)
    np.testing.assert_array_equal(d, base)


FUSED_CASES = [
    dict(lmax=150, nk=6, kmax=0.05, ntau=700, nsrc=3),
    dict(lmax=61, nk=12, kmax=0.02, ntau=300, nsrc=3),              # ragged l, one tile
    dict(lmax=333, nk=9, kmax=0.1, ntau=2500, nsrc=3),              # several l tiles, 40 chunks
    dict(lmax=90, nk=7, kmax=0.2, ntau=190, nsrc=1, kmin=0.01),     # x >> lmax, ragged tau
    dict(lmax=600, nk=4, kmax=0.06, ntau=1003, nsrc=2),             # ntau not a multiple of 4
]


@pytest.mark.parametrize("prec", list(PRECS), ids=list(PRECS))
@pytest.mark.parametrize("shape", [4, 5, 0, 1, 2, 3])
@pytest.mark.parametrize("cfg", FUSED_CASES, ids=[str(i) for i in range(len(FUSED_CASES))])
def test_mixed_fused_matches_tables(torch_dev, ctx, cfg, shape, prec, monkeypatch):
    """The default pipeline (Bessel tiles regenerated in LDS from seeds every 32 multipoles)
    gives bitwise the Delta of the table pipeline (whole FP32 tables, fragment product): the
    same recurrence cadence and the same accumulation order, for every tile shape."""
    p = PRECS[prec]
    wl = inputs.small(**cfg)
    monkeypatch.setenv("LOS_MIXED_FUSED", "0")
    monkeypatch.setenv("LOS_GEMM_MB", "2")
    monkeypatch.setenv("LOS_GEMM_NC", "1")
    base, _, _ = run_mixed(torch_dev, ctx, wl, p)
    monkeypatch.delenv("LOS_MIXED_FUSED")
    monkeypatch.setenv("LOS_FUSED_SHAPE", str(shape))
    d, _, _ = run_mixed(torch_dev, ctx, wl, p)
    np.testing.assert_array_equal(d, base)


def test_mixed_chunked_workspace(torch_dev, ctx, monkeypatch):
    """A workspace that holds one k row at a time gives the same result."""
    wl = inputs.small(lmax=120, nk=9, kmax=0.04, ntau=500, nsrc=3)
    base, _, _ = run_mixed(torch_dev, ctx, wl, 1)
    monkeypatch.setenv("LOS_JTAB_MIB", "1")
    d, _, _ = run_mixed(torch_dev, ctx, wl, 1)
    np.testing.assert_array_equal(d, base)


def test_mixed_edge_cases(torch_dev, ctx):
    for lmin, lmax, nk, ntau in [(2, 2, 1, 5), (37, 37, 3, 129), (2, 9, 4, 64), (150, 160, 3, 200),
                                 (2, 40, 2, 31)]:
        wl = inputs.small(lmax=lmax, nk=nk, kmax=0.05, ntau=ntau, nsrc=3)
        wl.lmin = lmin
        for p in (1, 2):
            d, _, S64 = run_mixed(torch_dev, ctx, wl, p)
            ref, A = oracle.project(wl.lmin, wl.lmax, wl.k, wl.tau, wl.tau0, wl.w_tau, S64,
                                    with_abs=True)
            scale = np.maximum(np.max(A, axis=0, keepdims=True), 1e-300)
            assert np.max(np.abs(d - ref) / scale) <= eps_for(p, wl.ntau), (lmin, lmax, p)


def test_mixed_dtype_checked(torch_dev, ctx):
    wl = inputs.small(lmax=20, nk=3, ntau=64, nsrc=1)
    with pytest.raises(ValueError):
        ctx.los_project(wl.lmin, wl.lmax, dev(torch_dev, wl.k), dev(torch_dev, wl.tau), wl.tau0,
                        dev(torch_dev, wl.w_tau), dev(torch_dev, wl.S), prec=1)


@pytest.mark.parametrize("prec", list(PRECS), ids=list(PRECS))
def test_c3_full_size_sampled(torch_dev, ctx, prec):
    """The mixed-precision workload (C3: l = 2..5000, 8000 k, 4000 tau, T/E/lensing) in the
    launch configuration bench.py times: every sampled C_l within 1e-4 of the FP64 oracle."""
    wl = inputs.config("C3")
    _, c, _ = run_mixed(torch_dev, ctx, wl, PRECS[prec])
    assert np.all(np.isfinite(c))
    gold = np.loadtxt(GOLDEN_C3)
    ls = gold[:, 0].astype(int) - wl.lmin
    cref = gold[:, 1:].T
    err = cl_rel_err(c[:, ls], cref, list(wl.pairs))
    print("C3 %s: max C_l rel err vs oracle %.3e" % (prec, err))
    assert err <= 1e-4, (prec, err)
