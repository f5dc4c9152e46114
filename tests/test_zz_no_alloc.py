"""The allocation-free misfit entry point (eth_misfit_noalloc) against the
handle-based eth_misfit it mirrors: same kernels, same reduction order, so J
and dJ/dx agree bit for bit.  Two calls in a row, the second on a smaller
input, so the second reads partial sums the first left in the shared array
only where it writes them itself."""
import pytest
import torch

pytestmark = pytest.mark.gpu


def _inputs(n, batch, seed):
    g = torch.Generator().manual_seed(seed)
    N = 2 * (2 * n + 1) ** 2 + (n + 1) ** 2 + n * n
    x = torch.rand((batch, N), generator=g, dtype=torch.float64) * 2 - 1
    t = torch.rand((batch, N), generator=g, dtype=torch.float64) * 2 - 1
    return x.cuda(), t.cuda()


def _check_pair(n, batch, seed, domain):
    from paper_2303_10233_amd import eth
    x, t = _inputs(n, batch, seed)
    P = eth.Problem(n, domain=domain, max_batch=batch, device="cuda:0")
    try:
        J_ref, g_ref = P.misfit(x, t, grad=True)
    finally:
        torch.cuda.synchronize()
        P.close()
    J = torch.full((batch,), float("nan"), dtype=torch.float64, device="cuda:0")
    g = torch.full_like(x, float("nan"))
    eth.misfit_noalloc(x, t, n, domain=domain, J=J, out_grad=g)
    torch.cuda.synchronize()
    assert torch.equal(J, J_ref), (n, batch, (J - J_ref).abs().max().item())
    assert torch.equal(g, g_ref), (n, batch)
    # J is the plain quadratic form of the gradient it returns
    N = x.shape[1]
    nv2 = 2 * (2 * n + 1) ** 2
    e = (x - t)[:, :nv2]
    q = 0.5 * (e * g[:, :nv2]).sum(dim=1)
    assert torch.allclose(J, q, rtol=1e-12, atol=0), (J, q)
    assert torch.all(g[:, nv2:N] == 0)


def test_noalloc_misfit_matches_handle_misfit_twice():
    print("no-alloc misfit: n=96 batch=3, then n=20 batch=1", flush=True)
    _check_pair(96, 3, 11, (0.0, 1.0, 0.0, 1.0))
    _check_pair(20, 1, 12, (-1.0, 1.0, -1.0, 1.0))


def test_noalloc_misfit_rejects_oversize():
    from paper_2303_10233_amd import eth
    n = 2048
    N = 2 * (2 * n + 1) ** 2 + (n + 1) ** 2 + n * n
    x = torch.zeros((2, N), dtype=torch.float64, device="cuda:0")
    with pytest.raises(eth.EthError) as ei:
        eth.misfit_noalloc(x, x, n, grad=False)
    assert ei.value.status == eth.EINVAL
    assert "scratch" in str(ei.value)
    # one right-hand side of the same size fits
    J, _ = eth.misfit_noalloc(x[:1], x[:1], n, grad=False)
    torch.cuda.synchronize()
    assert float(J) == 0.0
