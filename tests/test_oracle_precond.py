"""Pins of the oracle's preconditioner pieces (Sec. 2.2-2.3 pressure-mass
solves, geometric multigrid, Sec. 3.1 PCD and the two-stage algorithm)
against dense linear algebra, closed forms and the identities the paper states."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.assemble import Mesh, System, frame_null_vector, lid_dirichlet, \
    recirculating_wind, laplacian
from oracle.direct import direct_solve, canonicalize, rel_err
from oracle.krylov import minres
from oracle import precond as pc


def _dense_op(f, n):
    return np.column_stack([f(e) for e in np.eye(n)])


@pytest.mark.parametrize("n", [2, 4])
def test_mq_bordered_solve_is_pseudo_inverse(n):
    m = Mesh(n)
    s = System(m)
    op = pc.MQExact(m, s.MQ)
    r = np.random.default_rng(n).standard_normal(m.np_)
    np.testing.assert_allclose(op(r), np.linalg.pinv(s.MQ.toarray()) @ r, atol=1e-11)


def test_mq_diag_bordered():
    m = Mesh(5)
    s = System(m)
    op = pc.MQDiag(m, s.MQ)
    D = np.diag(s.MQ.diagonal())
    k = frame_null_vector(m)
    Kb = np.block([[D, k[:, None]], [k[None, :], np.zeros((1, 1))]])
    r = np.random.default_rng(1).standard_normal(m.np_)
    z = op(r)
    np.testing.assert_allclose(z, np.linalg.solve(Kb, np.append(r, 0))[:-1], atol=1e-12)
    Z = _dense_op(op, m.np_)
    assert np.abs(Z - Z.T).max() < 1e-12 * np.abs(Z).max()
    assert abs(k @ z) < 1e-12 * np.linalg.norm(z)


def test_multicolour_sgs_equals_triangular_splitting():
    """One symmetric sweep from zero applies M_SGS^{-1} with
    M_SGS = (D+L) D^{-1} (D+U) in the colour order (D+L lower part)."""
    m = Mesh(4)
    s = System(m)
    M = s.MQ.toarray()
    col = pc.mq_colours(m)
    perm = np.argsort(col, kind="stable")
    Mp = M[np.ix_(perm, perm)]
    D = np.diag(np.diag(Mp))
    L = np.tril(Mp, -1)
    U = np.triu(Mp, 1)
    r = np.random.default_rng(3).standard_normal(m.np_)
    y = sla.solve_triangular(D + L, r[perm], lower=True)
    z = sla.solve_triangular(D + U, D @ y, lower=False)
    expect = np.empty_like(z)
    expect[perm] = z
    got = pc.multicolour_sgs(s.MQ, col, r, np.zeros(m.np_))
    np.testing.assert_allclose(got, expect, atol=1e-11)
    # colours are independent sets of the M_Q graph
    for c in range(5):
        idx = np.flatnonzero(col == c)
        sub = M[np.ix_(idx, idx)]
        assert np.abs(sub - np.diag(np.diag(sub))).max() == 0.0


@pytest.mark.parametrize("n", [4, 8])
def test_sgs_spectrum_in_unit_interval(n):
    """SGS for a symmetric positive semi-definite matrix: eigenvalues of
    M_SGS^{-1} M_Q lie in [0, 1] (Sec. 2.3)."""
    m = Mesh(n)
    ev = pc.sgs_spectrum(m, System(m).MQ)
    assert ev[0] > -1e-12 and ev[-1] < 1 + 1e-10
    assert abs(ev[-1] - 1) < 1e-8          # the top eigenvalue is attained
    assert np.sum(np.abs(ev) < 1e-10) == 1  # only k is annihilated


def test_chebyshev_residual_polynomial_closed_form():
    """For A = diag(lam), M = I, the Chebyshev error after m steps is
    T_m((theta - lam)/delta) / T_m(theta/delta) times the initial error."""
    lam = np.linspace(0.1, 1.0, 25)
    lo, hi = 0.1, 1.0
    theta, delta = (hi + lo) / 2, (hi - lo) / 2
    x_true = np.random.default_rng(4).standard_normal(lam.size)
    r = lam * x_true
    for steps in (1, 2, 5, 9):
        x = pc.chebyshev(lambda v: lam * v, lambda v: v, r, np.zeros_like(r), lo, hi, steps)
        T = np.polynomial.chebyshev.Chebyshev.basis(steps)
        expect = T((theta - lam) / delta) / T(theta / delta) * x_true
        np.testing.assert_allclose(x_true - x, expect, atol=1e-12)


def test_cheb_sgs_operator_symmetric_psd_null_k_and_converges():
    m = Mesh(4)
    s = System(m)
    ev = pc.sgs_spectrum(m, s.MQ)
    lo = ev[1]
    op = pc.MQChebSGS(m, s.MQ, lo=lo, steps=20)
    Z = _dense_op(op, m.np_)
    assert np.abs(Z - Z.T).max() < 1e-10 * np.abs(Z).max()
    w = np.linalg.eigvalsh(0.5 * (Z + Z.T))
    assert w[0] > -1e-10 * w[-1] and np.sum(w < 1e-10 * w[-1]) == 1
    k = frame_null_vector(m)
    assert np.abs(Z @ k).max() < 1e-10 * np.abs(Z).max()
    # with the exact interval and many steps it approaches M_Q^+
    op60 = pc.MQChebSGS(m, s.MQ, lo=lo, steps=60)
    r = np.random.default_rng(5).standard_normal(m.np_)
    np.testing.assert_allclose(op60(r), np.linalg.pinv(s.MQ.toarray()) @ r, rtol=1e-6, atol=1e-6 * np.abs(np.linalg.pinv(s.MQ.toarray()) @ r).max())


def test_gmg_vcycle_symmetric_convergent_and_exact_on_one_level():
    m = Mesh(16)
    g = pc.GMG(m, laplacian, coarse_n=4)
    n = g.A[0].shape[0]
    V = _dense_op(lambda v: g.vcycle(0, v), n)
    assert np.abs(V - V.T).max() < 1e-10 * np.abs(V).max()
    A = g.A[0].toarray()
    E = np.eye(n) - V @ A
    rho = max(abs(np.linalg.eigvals(E)))
    assert rho < 0.25, rho
    g1 = pc.GMG(Mesh(4), laplacian, coarse_n=4)
    r = np.random.default_rng(6).standard_normal(g1.A[0].shape[0])
    np.testing.assert_allclose(g1.vcycle(0, r), np.linalg.solve(g1.A[0].toarray(), r), atol=1e-12)


def test_pcd_pressure_laplacian_null_space_constants():
    m = Mesh(6, -1, 1, -1, 1)
    s = System(m, nu=0.01, wind=recirculating_wind(m))
    P = pc.PCDStage1(s)
    Ap = P.Ap.toarray()
    ev, V = np.linalg.eigh(Ap)
    assert np.sum(ev < 1e-12 * ev[-1]) == 1
    assert np.abs(Ap @ np.ones(m.nk)).max() < 1e-13
    # F_1 annihilates constants for an enclosed wind (w.n = 0)
    assert np.abs(P.F1 @ np.ones(m.nk)).max() < 1e-13


@pytest.mark.parametrize("nu", [1 / 20, 1 / 100])
def test_two_stage_reaches_direct_solution_and_residual_identity(nu):
    m = Mesh(8, -1, 1, -1, 1)
    s = System(m, nu=nu, wind=recirculating_wind(m))
    b = s.rhs(None, lid_dirichlet(m))
    xd = direct_solve(s, b)
    eta, c = 1e-10, 10.0
    x, info = pc.two_stage(s, b, eta=eta, c=c)
    assert rel_err(canonicalize(x, m), xd) < 1e-7
    # pr.residualbound: ||z*||^2 = ||r*||^2 + ||r_1*||^2 + ||g_0 - B_0 u_1*||^2
    # with ||r*||^2 + ||r_1*||^2 <= c^2 eta^2 ||b||^2
    zs = info["z_star"]
    nI = s.nI
    r_red = zs[: nI + m.nk]
    r0 = zs[nI + m.nk:]
    bint = s.to_interior(b)
    u1 = info["x_stage1"][:nI]
    np.testing.assert_allclose(r0, bint[nI + m.nk:] - s.BI[m.nk:] @ u1, atol=1e-13)
    assert np.linalg.norm(r_red) <= c * eta * info["bnorm"] * (1 + 1e-6)
    lhs = np.linalg.norm(zs) ** 2
    assert lhs <= (c * eta * info["bnorm"]) ** 2 + np.linalg.norm(r0) ** 2 + 1e-30
    # the transition jump: the stage-I result violates eta once B_0 u is counted
    assert np.linalg.norm(zs) > eta * info["bnorm"]


def test_m1_preconditioned_gmres_converges():
    m = Mesh(8, -1, 1, -1, 1)
    s = System(m, nu=0.05, wind=recirculating_wind(m))
    b = s.rhs(None, lid_dirichlet(m))
    from oracle.krylov import fgmres
    x, info = fgmres(lambda v: s.K @ v, s.to_interior(b), pc.OseenM1(s), tol=1e-10,
                     restart=50, maxit=500)
    assert info["converged"]
    xf = canonicalize(s.to_full(x, b[: 2 * m.nv]), m)
    assert rel_err(xf, direct_solve(s, b)) < 1e-7
