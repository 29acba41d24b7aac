"""GPU parity of the E-mode kernel eps_l = sqrt((l+2)!/(l-2)!) j_l(x)/x^2 (gCAMB
paper Sec. 2.1, Eq. 3) in the FP64 projection (los_project_kernels) against the
oracle's projection with the same kernel mask.  Bounds as for the j_l path:
Delta normwise 1e-10 (A = sum_n |w S eps_l|), C_l 1e-10 relative."""
import numpy as np
import pytest

import oracle
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


def run(torch, ctx, wl, mask, S=None):
    S = wl.S if S is None else S
    d = ctx.los_project_kernels(wl.lmin, wl.lmax, dev(torch, wl.k), dev(torch, wl.tau), wl.tau0,
                                dev(torch, wl.w_tau), dev(torch, S), mask)
    c = ctx.cl_integrate(d, dev(torch, wl.w_lnk), dev(torch, wl.Pk), wl.pairs)
    torch.cuda.synchronize()
    return d.cpu().numpy(), c.cpu().numpy()


def check(torch, ctx, wl, mask, S=None, tol=1e-10):
    S = wl.S if S is None else S
    d, c = run(torch, ctx, wl, mask, S)
    ref, A = oracle.project(wl.lmin, wl.lmax, wl.k, wl.tau, wl.tau0, wl.w_tau, S, with_abs=True,
                            eps_mask=mask)
    scale = np.maximum(np.max(A, axis=0, keepdims=True), 1e-300)
    err = float(np.max(np.abs(d - ref) / scale))
    assert err <= tol, ("delta normwise", err)
    cref = oracle.cl(ref, wl.w_lnk, wl.Pk, wl.pairs)
    for p, (a, b) in enumerate(wl.pairs):
        if a == b:
            rel = np.abs(c[p] / cref[p] - 1)
        else:
            rel = np.abs(c[p] - cref[p]) / np.sqrt(cref[wl.pairs.index((a, a))] *
                                                  cref[wl.pairs.index((b, b))])
        assert np.max(rel) <= tol, ("C_l", p, float(np.max(rel)))
    return d


SMALL = [
    dict(lmax=61, nk=12, kmax=0.02, ntau=300),
    dict(lmax=200, nk=9, kmax=0.05, ntau=1000),
    dict(lmax=90, nk=7, kmax=0.2, ntau=190, kmin=0.01),
    dict(lmax=333, nk=16, kmax=0.1, ntau=2500),
    dict(lmax=60, nk=5, kmax=6e-3, ntau=64),
]


@pytest.mark.parametrize("cfg", SMALL, ids=[str(i) for i in range(len(SMALL))])
def test_emode_small_vs_oracle(torch_dev, ctx, cfg):
    """T and lensing on j_l, E on eps_l (mask 0b010)."""
    check(torch_dev, ctx, inputs.small(nsrc=3, **cfg), 0b010)


def test_emode_every_source_and_x_zero_node(torch_dev, ctx):
    """All sources on eps_l with random, non-separable sources that are non-zero at tau = tau0
    (x = 0 there): the l = 2 limit w S sqrt(24)/15 is included."""
    wl = inputs.small(lmax=120, nk=10, kmax=0.04, ntau=400, nsrc=3)
    rng = np.random.default_rng(31)
    S = rng.normal(size=wl.S.shape)
    assert wl.tau[-1] == wl.tau0
    check(torch_dev, ctx, wl, 0b111, S=S)
    wl2 = inputs.small(lmax=40, nk=4, kmax=1e-3, ntau=64, nsrc=3)
    check(torch_dev, ctx, wl2, 0b101, S=rng.normal(size=wl2.S.shape))


def test_emode_mask_zero_equals_los_project(torch_dev, ctx):
    torch = torch_dev
    wl = inputs.small(lmax=150, nk=8, kmax=0.05, ntau=600, nsrc=3)
    d0, _ = run(torch, ctx, wl, 0)
    d1 = ctx.los_project(wl.lmin, wl.lmax, dev(torch, wl.k), dev(torch, wl.tau), wl.tau0,
                         dev(torch, wl.w_tau), dev(torch, wl.S)).cpu().numpy()
    np.testing.assert_array_equal(d0, d1)


def test_emode_errors(torch_dev, ctx, monkeypatch):
    torch = torch_dev
    from paper_2509_25110_amd import los
    wl = inputs.small(lmax=20, nk=3, ntau=64, nsrc=2)
    args = (wl.lmin, wl.lmax, dev(torch, wl.k), dev(torch, wl.tau), wl.tau0, dev(torch, wl.w_tau))
    with pytest.raises(los.LosError) as e:
        ctx.los_project_kernels(*args, dev(torch, wl.S), 0b100)          # source 2 of 2
    assert e.value.code == los.LOS_ERR_INVALID
    with pytest.raises(los.LosError) as e:
        ctx.los_project_kernels(*args, dev(torch, wl.S.astype(np.float32)), 0b10, prec=2)
    assert e.value.code == los.LOS_ERR_UNSUPPORTED
    monkeypatch.setenv("LOS_PROJ_SCHEME", "0")
    with pytest.raises(los.LosError) as e:
        ctx.los_project_kernels(*args, dev(torch, wl.S), 0b10)
    assert e.value.code == los.LOS_ERR_UNSUPPORTED


def test_emode_c2_full_size_sampled_rows(torch_dev, ctx):
    """The C2 workload with the E source on eps_l: sampled k rows against the oracle, per
    (l, source) normwise 1e-10 of the sampled rows' absolute sums."""
    torch = torch_dev
    wl = inputs.config("C2")
    d, c = run(torch, ctx, wl, 0b010)
    assert np.all(np.isfinite(d)) and np.all(np.isfinite(c))
    rows = [0, 900, 2100, 3000, 3600, 3999]
    refs, As = [], []
    for r in rows:
        ref, A = oracle.project(wl.lmin, wl.lmax, wl.k, wl.tau, wl.tau0, wl.w_tau, wl.S,
                                with_abs=True, k_range=(r, r + 1), eps_mask=0b010)
        refs.append(ref[0])
        As.append(A[0])
    scale = np.maximum(np.max(np.stack(As), axis=0), 1e-300)
    for r, ref in zip(rows, refs):
        assert np.max(np.abs(d[r] - ref) / scale) <= 1e-10, r
