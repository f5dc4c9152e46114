"""GPU parity of the discrete adjoint (K^T lambda = dJ/dx) and the gradients
dJ/df = M_v lambda~ and dJ/dnu = -lambda_u^T (A u)_I through the C ABI,
against the oracle's adjoint (itself pinned by central finite differences),
and of the autograd Functions against central differences of GPU solves.

J = 1/2 ||u - u_t||^2 in L2 (M_v-weighted over all velocity nodes); u_t is
the solution under the bump forcing of seed 5000 and the gradient is taken
at f0 = 0.5 * bumps(seed 4999) (at f = 0 the Stokes velocity does not depend
on nu and dJ/dnu would vanish)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle.assemble import Mesh, System, lid_dirichlet  # noqa: E402
from oracle.direct import BorderedLU, adjoint_gradients, misfit, rel_err  # noqa: E402
from paper_2303_10233_amd import eth  # noqa: E402
from paper_2303_10233_amd.workloads import gaussian_bumps, recirculating_wind  # noqa: E402

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


def _case(oseen, n, prec=eth.FP64, max_batch=1):
    if oseen:
        m = Mesh(n, -1, 1, -1, 1)
        w = recirculating_wind(n)
        nu = 0.01
        dom = (-1.0, 1.0, -1.0, 1.0)
        P = eth.Problem(n, domain=dom, nu=nu, kind=eth.OSEEN, wind=_t(w), precision=prec,
                        max_batch=max_batch)
    else:
        m = Mesh(n)
        w = None
        nu = 1.0
        dom = (0.0, 1.0, 0.0, 1.0)
        P = eth.Problem(n, domain=dom, nu=nu, precision=prec, max_batch=max_batch)
    s = System(m, nu=nu, wind=w)
    ft = gaussian_bumps(n, 5000, *dom)
    f0 = 0.5 * gaussian_bumps(n, 4999, *dom)
    return m, s, P, ft, f0


@pytest.mark.parametrize("oseen", [False, True])
def test_adjoint_gradients_match_oracle(oseen):
    n = 16
    print(f"[adjoint] oseen={oseen} n={n}", flush=True)
    m, s, P, ft, f0 = _case(oseen, n)
    lu = BorderedLU(s)
    uB = lid_dirichlet(m)
    xt_ref = lu.solve(s.rhs(ft, uB))
    x_ref = lu.solve(s.rhs(f0, uB))
    lam_ref, dJdf_ref, dJdnu_ref = adjoint_gradients(s, x_ref, xt_ref, lu=lu)
    # GPU: forward, misfit, adjoint, gradients
    xt, _ = P.solve(P.assemble_rhs(_t(ft)), rtol=1e-12, maxit=3000)
    x, info = P.solve(P.assemble_rhs(_t(f0)), rtol=1e-12, maxit=3000)
    assert info[0]["status"] == 0
    J, g = P.misfit(x, xt)
    assert abs(float(J) - misfit(s, x_ref, xt_ref)) <= 1e-9 * misfit(s, x_ref, xt_ref)
    o = 2 * m.nv
    gh = _np(g)
    assert np.abs(gh[o:]).max() == 0.0
    assert rel_err(gh[:o], s.Mv @ (x_ref[:o] - xt_ref[:o])) < 1e-9
    lam, ainfo = P.solve_adjoint(g, rtol=1e-12, maxit=3000)
    assert ainfo[0]["status"] == 0
    lh = _np(lam)
    assert np.abs(lh[:o][s.vel_bnd]).max() == 0.0
    assert rel_err(lh[:o], lam_ref[:o]) < 1e-9
    dJdf = _np(P.grad_forcing(lam))
    assert rel_err(dJdf, dJdf_ref) < 1e-9
    dJdnu = float(P.grad_viscosity(lam, x))
    assert abs(dJdnu - dJdnu_ref) <= 1e-8 * abs(dJdnu_ref)


def test_adjoint_pressure_part_of_g_is_projected():
    """A constant added to the pressure blocks of g lies in null(K) = null(K^T):
    the adjoint must not change."""
    m, s, P, ft, f0 = _case(False, 12)
    rng = np.random.default_rng(3)
    g = rng.uniform(-1, 1, m.N)
    g2 = g.copy()
    g2[2 * m.nv: 2 * m.nv + m.nk] += 3.0
    g2[2 * m.nv + m.nk:] -= 1.5
    l1, _ = P.solve_adjoint(_t(g), rtol=1e-12, maxit=3000)
    l2, _ = P.solve_adjoint(_t(g2), rtol=1e-12, maxit=3000)
    assert rel_err(_np(l2), _np(l1)) < 1e-10


@pytest.mark.parametrize("oseen", [False, True])
def test_autograd_matches_central_differences(oseen):
    n = 16
    print(f"[autograd FD] oseen={oseen}", flush=True)
    m, s, P, ft, f0 = _case(oseen, n)
    xt = eth.FlowSolve.apply(_t(ft), torch.tensor(P.nu, dtype=torch.float64), P, 1e-12, 3000).detach()
    f = _t(f0).requires_grad_(True)
    nu = torch.tensor(P.nu, dtype=torch.float64, requires_grad=True)
    x = eth.FlowSolve.apply(f, nu, P, 1e-12, 3000)
    J = eth.l2_misfit(x, xt, P)
    J.backward()
    gf = _np(f.grad)
    gnu = float(nu.grad)

    def Jof(fv, nuv):
        if nuv == P.nu:
            Q = P
        else:
            Q = _case_nu(oseen, n, nuv)
        xx, _ = Q.solve(Q.assemble_rhs(_t(fv)), rtol=1e-12, maxit=3000)
        return float(Q.misfit(xx, xt, grad=False)[0])

    eps = 1e-6
    rng = np.random.default_rng(1)
    idx = rng.choice(np.flatnonzero(np.abs(gf) > 1e-3 * np.abs(gf).max()), 6, replace=False)
    for i in idx:
        e = np.zeros(2 * m.nv)
        e[i] = eps
        fd = (Jof(f0 + e, P.nu) - Jof(f0 - e, P.nu)) / (2 * eps)
        assert abs(fd - gf[i]) <= 2e-5 * np.abs(gf).max()
    fdnu = (Jof(f0, P.nu * (1 + eps)) - Jof(f0, P.nu * (1 - eps))) / (2 * eps * P.nu)
    assert abs(fdnu - gnu) <= 1e-4 * abs(gnu)


def _case_nu(oseen, n, nu):
    if oseen:
        w = recirculating_wind(n)
        return eth.Problem(n, domain=(-1.0, 1.0, -1.0, 1.0), nu=nu, kind=eth.OSEEN, wind=_t(w))
    return eth.Problem(n, nu=nu)


def _misfit_grads(P, n, dom, seeds):
    """dJ/dx = [M_v (u - u_t); 0] for targets u_t from the bump seeds, at the
    solution for f0 = 0.5 * bumps(4999) (smooth adjoint right-hand sides)."""
    x, _ = P.solve(P.assemble_rhs(_t(0.5 * gaussian_bumps(n, 4999, *dom))), rtol=1e-12, maxit=3000)
    G = []
    for sd in seeds:
        xt, _ = P.solve(P.assemble_rhs(_t(gaussian_bumps(n, sd, *dom))), rtol=1e-12, maxit=3000)
        G.append(P.misfit(x, xt)[1])
    return torch.stack(G)


@pytest.mark.parametrize("oseen", [False, True])
def test_batched_adjoint_equals_single(oseen):
    n = 32
    m, s, P, ft, f0 = _case(oseen, n, max_batch=2)
    dom = (-1.0, 1.0, -1.0, 1.0) if oseen else (0.0, 1.0, 0.0, 1.0)
    G = _misfit_grads(P, n, dom, (5000, 5001))
    # a constant on the pressure blocks (in null(K^T)) must not matter
    G[1, 2 * m.nv:] += 0.25
    L, info = P.solve_adjoint(G, rtol=1e-10, maxit=4000)
    print(f"  iterations {[i['iterations'] for i in info]}", flush=True)
    assert all(i["status"] == 0 for i in info)
    Lh = _np(L)
    Gh = _np(G)
    for k in range(2):
        l1, _ = P.solve_adjoint(G[k].clone(), rtol=1e-10, maxit=4000)
        assert rel_err(Lh[k], _np(l1)) < 1e-7
    # residual of the transposed system on the projected g
    o = 2 * m.nv
    for k in range(2):
        gk = Gh[k].copy()
        gk[: o][s.vel_bnd] = 0.0
        gk[o: o + m.nk] -= gk[o: o + m.nk].mean()
        gk[o + m.nk:] -= gk[o + m.nk:].mean()
        r = s.to_interior(gk) - s.K.T @ s.to_interior(Lh[k])
        # FGMRES stops on this residual; MINRES on its P^{-1}-norm estimate
        bound = 1.05e-10 if oseen else 1e-8
        assert np.linalg.norm(r) <= bound * np.linalg.norm(s.to_interior(gk))


def test_oseen_adjoint_mixed_n64():
    n = 64
    m, s, P, ft, f0 = _case(True, n, prec=eth.MIXED)
    _, _, P64, _, _ = _case(True, n)
    g = _misfit_grads(P64, n, (-1.0, 1.0, -1.0, 1.0), (5000,))[0]
    lm, im = P.solve_adjoint(g, rtol=1e-9, maxit=3000)
    ld, idd = P64.solve_adjoint(g, rtol=1e-9, maxit=3000)
    print(f"  adjoint iterations mixed {im[0]['iterations']} fp64 {idd[0]['iterations']}", flush=True)
    assert im[0]["status"] == 0 and idd[0]["status"] == 0
    o = 2 * m.nv
    assert rel_err(_np(lm)[:o], _np(ld)[:o]) < 1e-6
