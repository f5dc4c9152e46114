"""Pins of the oracle's Krylov solvers: MINRES of alg:minres and restarted
flexible GMRES, against exact solutions, the ideal-preconditioner spectrum of
Sec. 2 and the optimality properties that define the methods."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle.assemble import Mesh, System, lid_dirichlet
from oracle.direct import direct_solve, canonicalize, rel_err
from oracle.krylov import minres, fgmres, KrylovBreakdown
from oracle.precond import StokesBlockDiag


def _sym_indefinite(n, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.concatenate([rng.uniform(0.5, 3, n // 2), -rng.uniform(0.5, 3, n - n // 2)])
    return (Q * ev) @ Q.T


def test_minres_solves_nonsingular_indefinite():
    A = _sym_indefinite(40, 1)
    rng = np.random.default_rng(2)
    L = rng.standard_normal((40, 40))
    P = L @ L.T + 40 * np.eye(40)
    b = rng.standard_normal(40)
    x, info = minres(lambda v: A @ v, b, lambda v: np.linalg.solve(P, v), tol=1e-13, maxit=200)
    assert info["converged"]
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-10)


def test_minres_eta_is_preconditioned_residual_norm():
    """|eta_j| of alg:minres equals ||b - A x_j||_{P^{-1}} at every step."""
    A = _sym_indefinite(30, 3)
    rng = np.random.default_rng(4)
    d = rng.uniform(0.5, 2.0, 30)
    b = rng.standard_normal(30)
    hist = []
    for k in range(1, 15):
        x, info = minres(lambda v: A @ v, b, lambda v: v / d, tol=0.0, maxit=k)
        r = b - A @ x
        hist.append((np.sqrt(r @ (r / d)), info["eta"][-1] * info["gamma"][0]))
    for true, eta in hist:
        assert abs(true - eta) <= 1e-10 * max(true, 1e-30) + 1e-13
    # monotone non-increasing residual (minimal residual property)
    vals = [h[0] for h in hist]
    assert all(vals[i + 1] <= vals[i] * (1 + 1e-12) for i in range(len(vals) - 1))


def test_minres_matches_scipy_minres_solution():
    A = _sym_indefinite(50, 5)
    b = np.random.default_rng(6).standard_normal(50)
    x, _ = minres(lambda v: A @ v, b, lambda v: v, tol=1e-12, maxit=500)
    xs, _ = spla.minres(A, b, rtol=1e-13, maxiter=500)
    np.testing.assert_allclose(x, xs, rtol=1e-7, atol=1e-9)


def test_minres_breakdown_for_indefinite_preconditioner():
    A = _sym_indefinite(10, 7)
    b = np.ones(10)
    with pytest.raises(KrylovBreakdown):
        minres(lambda v: A @ v, b, lambda v: -v, tol=1e-10, maxit=20)


def test_ideal_preconditioner_three_steps():
    """With P = diag(A, S^+), S = B A^{-1} B^T, the preconditioned Stokes
    matrix has eigenvalues only 0, 1 and (1 +- sqrt 5)/2 (Sec. 2), so MINRES
    converges in three iterations (one more allowed for rounding)."""
    m = Mesh(4)
    s = System(m)
    A = s.AI.toarray()
    B = s.BI.toarray()
    S = B @ np.linalg.solve(A, B.T)
    Sp = np.linalg.pinv(S, rcond=1e-10)
    nI = s.nI
    prec = lambda v: np.concatenate([np.linalg.solve(A, v[:nI]), Sp @ v[nI:]])
    b = s.to_interior(s.rhs(None, lid_dirichlet(m)))
    x, info = minres(lambda v: s.K @ v, b, prec, tol=1e-10, maxit=10)
    assert info["converged"] and info["iterations"] <= 4
    # eigenvalues of P^{-1} K on the range are 1 and (1 +- sqrt5)/2
    Pd = np.zeros_like(s.K.toarray())
    Pd[:nI, :nI] = np.linalg.inv(A)
    Pd[nI:, nI:] = Sp
    ev = np.linalg.eigvals(Pd @ s.K.toarray()).real
    targets = _golden_spectrum()
    dist = np.abs(ev[:, None] - targets[None, :])
    assert dist.min(axis=1).max() < 1e-8          # every eigenvalue is a printed one
    assert (dist.min(axis=0) < 1e-8).all()         # and every printed one occurs


def _golden_spectrum():
    """The eigenvalues the paper prints for the ideal block preconditioner
    (tests/golden/ideal_block_preconditioner_spectrum.txt, Sec. 2)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "ideal_block_preconditioner_spectrum.txt")
    vals = []
    with open(path) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                value, expr = line.split()
                exact = {"0": 0.0, "1": 1.0, "(1-sqrt(5))/2": (1 - 5 ** 0.5) / 2,
                         "(1+sqrt(5))/2": (1 + 5 ** 0.5) / 2}[expr]
                assert abs(float(value) - exact) < 1e-15
                vals.append(float(value))
    return np.array(vals)


def test_minres_p1_reaches_direct_solution():
    m = Mesh(8)
    s = System(m, nu=0.5)
    b = s.rhs(None, lid_dirichlet(m))
    xd = direct_solve(s, b)
    P = StokesBlockDiag(s, "exact", "exact")
    x, info = minres(lambda v: s.K @ v, s.to_interior(b), P, tol=1e-13, maxit=300)
    xf = canonicalize(s.to_full(x, b[: 2 * m.nv]), m)
    assert rel_err(xf, xd) < 1e-10


@pytest.mark.slow
def test_minres_p1_mesh_independent():
    """Tables 1 and 3: with exact blocks the MINRES count does not grow
    with refinement (our element/domain differ, so only the pattern is
    checked)."""
    its = []
    for n in (8, 16, 32, 64):
        m = Mesh(n)
        s = System(m)
        b = s.to_interior(s.rhs(None, lid_dirichlet(m)))
        P = StokesBlockDiag(s, "exact", "exact")
        _, info = minres(lambda v: s.K @ v, b, P, tol=1e-8, maxit=300)
        its.append(info["iterations"])
    assert max(its) - min(its) <= 4, its


def test_fgmres_solves_and_is_minimal():
    rng = np.random.default_rng(8)
    n = 40
    A = rng.standard_normal((n, n)) + 8 * np.eye(n)
    b = rng.standard_normal(n)
    x, info = fgmres(lambda v: A @ v, b, lambda v: v, tol=1e-13, restart=50, maxit=200)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-11)
    # residual after k unrestarted steps equals min over the Krylov space
    for k in (3, 7):
        xk, ik = fgmres(lambda v: A @ v, b, lambda v: v, tol=0.0, restart=k, maxit=k)
        Kry = np.column_stack([np.linalg.matrix_power(A, i) @ b for i in range(k)])
        Qk, _ = np.linalg.qr(Kry)
        AK = A @ Qk
        y, *_ = np.linalg.lstsq(AK, b, rcond=None)
        best = np.linalg.norm(b - AK @ y)
        assert abs(np.linalg.norm(b - A @ xk) - best) < 1e-10 * np.linalg.norm(b)
        assert abs(ik["residuals"][-1] - best) < 1e-10 * np.linalg.norm(b)


def test_fgmres_restart_and_flexible():
    rng = np.random.default_rng(9)
    n = 60
    A = rng.standard_normal((n, n)) + 10 * np.eye(n)
    b = rng.standard_normal(n)
    D = np.diag(A).copy()
    x, info = fgmres(lambda v: A @ v, b, lambda v: v / D, tol=1e-12, restart=5, maxit=400)
    assert info["converged"]
    assert np.linalg.norm(b - A @ x) <= 1e-12 * np.linalg.norm(b) * 1.01
