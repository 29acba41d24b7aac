"""GPU parity of the FP64 projection across the launch shapes its chooser picks
(waves per workgroup, slots per lane, 8- or 2-block ring of partial sums) as
ntau grows to the 8192 limit, for 1 and 3 sources, against the oracle on a
few k rows (bounds as for the plain FP64 path: Delta normwise 1e-10)."""
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


@pytest.mark.parametrize("ntau", [200, 600, 3000, 4000, 7000, 8192])
@pytest.mark.parametrize("nsrc", [1, 3])
def test_shapes_parity(torch_dev, ctx, ntau, nsrc):
    torch = torch_dev
    wl = inputs.small(lmax=150, nk=6, kmax=0.03, ntau=ntau, nsrc=nsrc)
    dv = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    d = ctx.los_project(wl.lmin, wl.lmax, dv(wl.k), dv(wl.tau), wl.tau0, dv(wl.w_tau), dv(wl.S))
    torch.cuda.synchronize()
    ref, A = oracle.project(wl.lmin, wl.lmax, wl.k, wl.tau, wl.tau0, wl.w_tau, wl.S,
                            with_abs=True)
    scale = np.maximum(A.max(axis=0, keepdims=True), 1e-300)
    err = float(np.max(np.abs(d.cpu().numpy() - ref) / scale))
    assert err <= 1e-10, err
