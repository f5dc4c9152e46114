"""Ragged batches (several Stokes cavities of different sizes solved together
on their own streams): each result equals the standalone solve of the same
problem bit for bit (same kernels, deterministic reductions), and the
smallest agrees with the oracle's direct solution."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle.assemble import Mesh, System, lid_dirichlet  # noqa: E402
from oracle.direct import direct_solve, rel_err  # noqa: E402
from paper_2303_10233_amd import eth  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    eth.load_library()


@pytest.mark.parametrize("prec,graph", [(eth.FP64, True), (eth.MIXED, True), (eth.FP64, False), (eth.FP64, 2),
                                        (eth.MIXED, 2)])
def test_ragged_equals_standalone(prec, graph):
    sizes = [8, 12, 16, 24, 32, 48, 64]
    print(f"[ragged] sizes={sizes} prec={prec} graph={graph}", flush=True)
    R = eth.RaggedBatch(sizes, precision=prec)
    bs = R.assemble_rhs()
    # an FP32 preconditioner is symmetric only to FP32 rounding: ask mixed
    # precision for the configured 1e-6, FP64 for 1e-10
    rtol = 1e-10 if prec == eth.FP64 else 1e-6
    xs, infos = R.solve(bs, rtol=rtol, maxit=2000, use_graph=graph, true_residual=True)
    torch.cuda.synchronize()
    if graph == 2:   # a second solve replays the joint graph captured by the first
        xs, infos = R.solve(bs, rtol=rtol, maxit=2000, use_graph=graph, true_residual=True, out=xs)
        torch.cuda.synchronize()
    for n, b, x, info in zip(sizes, bs, xs, infos):
        assert info["status"] == 0
        P = eth.Problem(n, precision=prec)
        xr, ir = P.solve(P.assemble_rhs(), rtol=rtol, maxit=2000, use_graph=graph)
        assert ir[0]["iterations"] == info["iterations"]
        assert torch.equal(x, xr)
        assert info["rel_residual_true"] < 100 * rtol
    m = Mesh(8)
    s = System(m)
    xd = direct_solve(s, s.rhs(None, lid_dirichlet(m)))
    assert rel_err(xs[0].cpu().numpy(), xd) < (1e-8 if prec == eth.FP64 else 1e-4)
    R.close()


def test_ragged_paper_sizes_converge():
    """The ragged cavity set n_i = 32 + 16 (i mod 15), i < 32, mixed precision."""
    sizes = [32 + 16 * (i % 15) for i in range(32)]
    R = eth.RaggedBatch(sizes, precision=eth.MIXED)
    bs = R.assemble_rhs()
    xs, infos = R.solve(bs, rtol=1e-6, maxit=2000)
    its = [i["iterations"] for i in infos]
    print(f"  iterations {its}", flush=True)
    assert all(i["status"] == 0 for i in infos)
    R.close()
