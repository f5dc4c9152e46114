"""GPU parity of the Oseen operator (eq:oseen-system) through the C ABI
against the CPU oracle: K x, K^T x and the lifted RHS with the recirculating
wind, on seeded inputs.  FP64 applies agree to rounding (1e-13 relative; the
GPU integrates N(w) with 3x3 Gauss points, the oracle with 5x5, both exact for
a Q2 wind)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle.assemble import Mesh, System, lid_dirichlet  # noqa: E402
from oracle.direct import rel_err  # noqa: E402
from paper_2303_10233_amd import eth  # noqa: E402
from paper_2303_10233_amd.workloads import (gaussian_bumps, recirculating_wind,  # noqa: E402
                                            uniform_vector)

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


def _problem(n, nu, wind, **kw):
    return eth.Problem(n, domain=(-1.0, 1.0, -1.0, 1.0), nu=nu, kind=eth.OSEEN, wind=_t(wind),
                       mq=eth.MQ_DIAG, **kw)


@pytest.mark.parametrize("n", [2, 5, 16, 33, 64])
@pytest.mark.parametrize("transpose", [False, True])
def test_oseen_apply_matches_oracle(n, transpose):
    print(f"[oseen apply] n={n} transpose={transpose}", flush=True)
    m = Mesh(n, -1, 1, -1, 1)
    w = recirculating_wind(n)
    nu = 0.01
    s = System(m, nu=nu, wind=w)
    P = _problem(n, nu, w, max_batch=2, velocity=eth.VEL_EXACT if n <= 32 else eth.VEL_GMG)
    xs = [uniform_vector(m.N, 500 + n + k) for k in range(2)]
    X = torch.stack([_t(x) for x in xs])
    Y = _np(P.apply_operator(X, transpose=transpose))
    for k in range(2):
        ref = s.apply_full(xs[k], transpose=transpose)
        assert rel_err(Y[k], ref) < 1e-13


def test_oseen_general_wind_matches_oracle():
    """A wind that is not divergence free and not tangential (random nodal
    values): N is then not skew, so this separates N from N^T."""
    n = 12
    m = Mesh(n, -1, 1, -1, 1)
    w = uniform_vector(2 * m.nv, 77)
    s = System(m, nu=0.3, wind=w)
    P = _problem(n, 0.3, w)
    x = uniform_vector(m.N, 78)
    for tr in (False, True):
        y = _np(P.apply_operator(_t(x), transpose=tr))
        assert rel_err(y, s.apply_full(x, transpose=tr)) < 1e-13


def test_oseen_transpose_pair():
    n = 20
    m = Mesh(n, -1, 1, -1, 1)
    w = uniform_vector(2 * m.nv, 5)
    P = _problem(n, 0.05, w)
    s = System(m)
    x, y = uniform_vector(m.N, 1), uniform_vector(m.N, 2)
    Kx = _np(P.apply_operator(_t(x)))
    KTy = _np(P.apply_operator(_t(y), transpose=True))
    a = s.to_interior(Kx) @ s.to_interior(y)
    b = s.to_interior(x) @ s.to_interior(KTy)
    assert abs(a - b) <= 1e-13 * (abs(a) + abs(b))


@pytest.mark.parametrize("n", [4, 33])
def test_oseen_lift_matches_oracle(n):
    m = Mesh(n, -1, 1, -1, 1)
    w = recirculating_wind(n)
    nu = 0.02
    s = System(m, nu=nu, wind=w)
    P = _problem(n, nu, w)
    f = gaussian_bumps(n, 4000, -1, 1, -1, 1)
    b = _np(P.assemble_rhs(_t(f)))
    assert rel_err(b, s.rhs(f, lid_dirichlet(m))) < 1e-13
    b0 = _np(P.assemble_rhs(None))
    assert rel_err(b0, s.rhs(None, lid_dirichlet(m))) < 1e-13
