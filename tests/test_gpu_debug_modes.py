"""Debug mode ETH_DEBUG_NAN_FILL=1: every workspace starts as NaN instead of
whatever the allocator returned.  A solve that reads only what it wrote gives
bit for bit the result of the default mode."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2303_10233_amd import eth  # noqa: E402
from paper_2303_10233_amd.workloads import recirculating_wind  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    eth.load_library()


def _stokes(prec):
    P = eth.Problem(64, precision=prec, max_batch=2)
    b = P.assemble_rhs(batch=2)
    x, info = P.solve(b, rtol=1e-8, maxit=500, use_graph=True)
    out = (x.clone(), [i["iterations"] for i in info])
    P.close()
    return out


def _oseen(schur):
    n = 32
    w = torch.as_tensor(recirculating_wind(n), dtype=torch.float64, device="cuda:0")
    P = eth.Problem(n, domain=(-1.0, 1.0, -1.0, 1.0), nu=0.01, kind=eth.OSEEN, wind=w, oseen_schur=schur)
    b = P.assemble_rhs()
    method = eth.TWO_STAGE if schur == 0 else eth.FGMRES
    x, info = P.solve(b, rtol=1e-8, maxit=400, method=method, raise_on_error=False)
    out = (x.clone(), [info[0]["iterations"]])
    P.close()
    return out


def _step(prec):
    """Flow over a step, m = 8: Stokes start and two Picard steps (M_1 and
    two-stage solves, every workspace of the sparse path)."""
    P = eth.StepProblem(8, precision=prec)
    x, infos = P.picard(2, rtol=1e-8, maxit=800)
    out = (x.clone(), [i["iterations"] for i in infos])
    P.close()
    return out


@pytest.mark.parametrize("case", ["stokes_mixed", "stokes_fp64", "oseen_two_stage", "oseen_lsc", "step_mixed",
                                  "step_fp64"])
def test_nan_filled_workspaces_change_nothing(case, monkeypatch):
    print(f"[nan fill] {case}", flush=True)
    run = {"stokes_mixed": lambda: _stokes(eth.MIXED), "stokes_fp64": lambda: _stokes(eth.FP64),
           "oseen_two_stage": lambda: _oseen(0), "oseen_lsc": lambda: _oseen(2),
           "step_mixed": lambda: _step(eth.MIXED), "step_fp64": lambda: _step(eth.FP64)}[case]
    x0, it0 = run()
    monkeypatch.setenv("ETH_DEBUG_NAN_FILL", "1")
    x1, it1 = run()
    assert it0 == it1
    assert bool(torch.isfinite(x1).all())
    assert torch.equal(x0, x1)


@pytest.mark.parametrize("prec", [eth.MIXED, eth.FP64])
def test_delta_finished_in_the_v_update_changes_nothing(prec, monkeypatch):
    """The MINRES delta reduction finished inside the v update gives the
    iterates of the separate finishing launch bit for bit."""
    out = []
    for fold in ("1", "0"):
        monkeypatch.setenv("ETH_DEBUG_FOLD_DELTA", fold)
        out.append(_stokes(prec))
    assert out[0][1] == out[1][1]
    assert torch.equal(out[0][0], out[1][0])


@pytest.mark.parametrize("prec", [eth.MIXED, eth.FP64])
@pytest.mark.parametrize("graph", [True, False])
def test_wx_update_folded_into_the_next_v_update_changes_nothing(prec, graph, monkeypatch):
    """The MINRES w/x update made by the next iteration's v update (and by a
    closing launch at the end of each run of iterations) gives the iterates
    of its own launch bit for bit, eagerly and graph-replayed, with two
    right-hand sides that stop at different iterations (the gated iterations
    after the first one stops must make its last update exactly once)."""
    from paper_2303_10233_amd.workloads import uniform_vector
    print(f"[fold wx] prec={prec} graph={graph}", flush=True)
    out = []
    for fold in ("1", "0"):
        monkeypatch.setenv("ETH_DEBUG_FOLD_WX", fold)
        P = eth.Problem(64, precision=prec, max_batch=2)
        b = P.empty(2)
        b[0] = P.assemble_rhs()
        y = torch.as_tensor(uniform_vector(P.N, 11), dtype=torch.float64, device="cuda:0")
        b[1] = P.apply_operator(y)
        x, info = P.solve(b, rtol=1e-8, maxit=500, use_graph=graph)
        out.append((x.clone(), [i["iterations"] for i in info], [i["status"] for i in info]))
        P.close()
    assert out[0][2] == [eth.OK, eth.OK]
    assert out[0][1][0] != out[0][1][1]
    assert out[0][1] == out[1][1]
    assert torch.equal(out[0][0], out[1][0])
