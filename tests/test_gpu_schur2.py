"""GPU parity of the comparison Schur blocks (Sec. 3.1 two-field PCD M_2,
Sec. 3.2 least-squares commutator M_3) against the oracle, and their
convergence behaviour on the device.

The oracle uses the GPU's pieces: the damped-Jacobi F multigrid, ten
Chebyshev-Jacobi steps for Q_1, and the pressure Laplacian's pseudo-inverse
(CG on the GPU to 1e-12, the bordered direct solve in the oracle)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import oracle.precond as opc  # noqa: E402
from oracle.assemble import Mesh, System, lid_dirichlet  # noqa: E402
from oracle.direct import direct_solve, rel_err  # noqa: E402
from oracle.schur2 import OseenM2, OseenM3  # noqa: E402
from paper_2303_10233_amd import eth  # noqa: E402
from paper_2303_10233_amd.workloads import recirculating_wind, uniform_vector  # noqa: E402

DEV = "cuda:0"


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    eth.load_library()


def _setup(n, nu, schur, prec=eth.FP64):
    m = Mesh(n, -1, 1, -1, 1)
    w = recirculating_wind(n)
    s = System(m, nu=nu, wind=w)
    P = eth.Problem(n, domain=(-1.0, 1.0, -1.0, 1.0), nu=nu, kind=eth.OSEEN, wind=_t(w), precision=prec,
                    oseen_schur=schur, schur_cg_tol=1e-12)
    return m, s, P


@pytest.mark.parametrize("n,schur,prec,tol", [(16, 1, eth.FP64, 1e-9), (32, 1, eth.FP64, 1e-9),
                                              (16, 2, eth.FP64, 1e-9), (32, 2, eth.FP64, 1e-9),
                                              (32, 1, eth.MIXED, 2e-4), (32, 2, eth.MIXED, 2e-4)])
def test_schur_blocks_match_oracle(n, schur, prec, tol):
    print(f"[schur2] n={n} schur={schur} prec={prec}", flush=True)
    m, s, P = _setup(n, 0.01, schur, prec)
    r = uniform_vector(m.N, 500 + n)
    r[: 2 * m.nv][s.vel_bnd] = 0.0
    z = _np(P.apply_preconditioner(_t(r)))
    vel, _ = opc.oseen_velocity_gmg(s)
    cls = OseenM2 if schur == 1 else OseenM3
    pre = cls(s, velocity_solve=vel, q1_steps=10)
    zref = s.to_full(pre(s.to_interior(r)))
    o = 2 * m.nv
    ep, eu = rel_err(z[o:], zref[o:]), rel_err(z[:o], zref[:o])
    print(f"  pressure {ep:.2e} velocity {eu:.2e}", flush=True)
    assert ep < tol and eu < tol
    P.close()


def test_fgmres_with_m2_stagnates_and_m3_converges():
    """Cavity nu = 1/100 on 32^2, FGMRES(50) from zero: M_2 starts faster than
    M_1 and then stagnates (Sec. 3.1), M_3 converges (Sec. 3.2, Q2-Q1*)."""
    n = 32
    hist = {}
    for schur in (0, 1, 2):
        m, s, P = _setup(n, 0.01, schur)
        b = P.assemble_rhs()
        x, info = P.solve(b, rtol=1e-8, maxit=250, method=eth.FGMRES, raise_on_error=False, history_len=300)
        hist[schur] = (np.array(info[0]["history"]), info[0])
        print(f"  schur={schur}: status={info[0]['status']} its={info[0]['iterations']} "
              f"true={info[0]['rel_residual_true']:.2e}", flush=True)
        if schur == 2:
            xd = direct_solve(s, s.rhs(None, lid_dirichlet(m)))
            assert rel_err(_np(x), xd) < 1e-5
        P.close()
    h0, h1, h2 = hist[0][0], hist[1][0], hist[2][0]
    assert h1[20] < 0.5 * h0[20]
    assert hist[1][1]["status"] == eth.WMAXIT and h1[-1] > 1e-3
    assert hist[2][1]["status"] == 0 and hist[2][1]["iterations"] <= 100
