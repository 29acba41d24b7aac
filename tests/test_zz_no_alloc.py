"""cl_integrate_noalloc (the C_l reduction with the library's fixed device scratch, no
allocation) against cl_integrate (context workspace), through the C ABI: bitwise equal
results on two calls in a row, the second with a smaller input, and a clear error for a
request beyond the fixed scratch."""
import numpy as np
import pytest

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


def case(torch, seed, nk, nl, nsrc, dtype):
    rng = np.random.default_rng(seed)
    delta = torch.from_numpy(rng.standard_normal((nk, nl, nsrc))).to(dtype).cuda()
    k = inputs.log_k_grid(nk, 1e-4, 0.5)
    w = torch.from_numpy(inputs.trapezoid_weights(np.log(k))).cuda()
    P = torch.from_numpy(inputs.primordial(k, 2.1e-9, 0.965)).cuda()
    return delta, w, P


def test_noalloc_matches_cl_integrate_twice(torch_dev, ctx):
    torch = torch_dev
    # first call: the C2 shape (4000 k, l = 2..2500, T/E/lensing, TT/EE/TE/PP), FP64
    d, w, P = case(torch, 1, 4000, 2499, 3, torch.float64)
    pairs = [(0, 0), (1, 1), (0, 1), (2, 2)]
    ref = ctx.cl_integrate(d, w, P, pairs)
    out = torch.full_like(ref, float("nan"))
    ctx.cl_integrate_noalloc(d, w, P, pairs, cl=out)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), ref.cpu().numpy())
    # second call, smaller: FP32 transfer functions, 2 sources, 2 pairs, fewer k and l
    d2, w2, P2 = case(torch, 2, 300, 177, 2, torch.float32)
    pairs2 = [(0, 0), (0, 1)]
    ref2 = ctx.cl_integrate(d2, w2, P2, pairs2)
    out2 = torch.full_like(ref2, float("nan"))
    ctx.cl_integrate_noalloc(d2, w2, P2, pairs2, cl=out2)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out2.cpu().numpy(), ref2.cpu().numpy())
    # and the FP64 oracle-free check that the value is the plain sum (first-order bound)
    dd = d2.double().cpu().numpy()
    want = 4 * np.pi * np.einsum("k,kl,kl->l", (w2 * P2).cpu().numpy(), dd[:, :, 0], dd[:, :, 1])
    np.testing.assert_allclose(out2.cpu().numpy()[1], want, rtol=1e-12,
                               atol=1e-13 * np.max(np.abs(want)))


def test_noalloc_rejects_beyond_scratch(torch_dev, ctx):
    from paper_2509_25110_amd import los
    torch = torch_dev
    # 16 pairs at nl = 16000 need about 35 MB of partial sums, beyond the fixed 16 MiB
    d = torch.zeros((20, 16000, 4), dtype=torch.float32, device="cuda")
    w = torch.ones(20, dtype=torch.float64, device="cuda")
    pairs = [(a, b) for a in range(4) for b in range(4)]
    cl = torch.empty((16, 16000), dtype=torch.float64, device="cuda")
    with pytest.raises(los.LosError, match="scratch"):
        ctx.cl_integrate_noalloc(d, w, w, pairs, cl=cl)
