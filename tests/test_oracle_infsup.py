"""Pins of the inf-sup oracle (Sec. 2.4, eq:inf-sup_eig) and of its EST-MINRES
estimate: the dense generalised eigenvalue against the eigenvalues of the
preconditioned saddle-point matrix (eq:spec_q), the harmonic Ritz values
against exact eigenvalues when the Krylov space is invariant, and the
EST-MINRES estimate of exactly preconditioned MINRES against the dense value."""
import numpy as np
import pytest

from oracle.assemble import Mesh, System, lid_dirichlet
from oracle.infsup import est_minres, harmonic_ritz, infsup_dense
from oracle.krylov import minres
from oracle.precond import StokesBlockDiag


def test_harmonic_ritz_of_an_invariant_space_are_eigenvalues():
    rng = np.random.default_rng(2)
    k = 7
    delta = rng.uniform(-2, 2, k)
    gamma = np.concatenate([[1.0], rng.uniform(0.2, 1.0, k - 1), [0.0]])   # beta = 0
    T = np.diag(delta) + np.diag(gamma[1:k], 1) + np.diag(gamma[1:k], -1)
    assert np.allclose(harmonic_ritz(delta, gamma), np.sort(np.linalg.eigvalsh(T)), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n", [2, 4])
def test_dense_infsup_matches_preconditioned_spectrum(n):
    """gamma^2 = theta (theta - 1) for the negative eigenvalue theta of
    diag(A, M_Q^+)^{-1} K closest to zero (eigenvalues of the non-symmetric
    product, computed without the Schur complement)."""
    m = Mesh(n)
    s = System(m)
    K = s.K.toarray()
    nI = s.nI
    MQ = s.MQ.toarray()
    # rows of diag(A, M_Q^+)^{-1}-preconditioned K: [A^{-1} K_u; M_Q^+ K_p]
    PK = np.vstack([np.linalg.solve(K[:nI, :nI], K[:nI, :]), np.linalg.pinv(MQ) @ K[nI:, :]])
    lam = np.linalg.eigvals(PK)
    lam = np.real(lam[np.abs(np.imag(lam)) < 1e-8])
    neg = lam[lam < -1e-8]
    th = neg.max()
    assert abs(th * (th - 1.0) - infsup_dense(s)) < 1e-9


@pytest.mark.parametrize("n,random_rhs", [(2, True), (4, False), (8, False)])
def test_est_minres_with_exact_blocks_gives_the_dense_value(n, random_rhs):
    m = Mesh(n)
    s = System(m)
    b = s.to_interior(s.rhs(None, lid_dirichlet(m)))
    if random_rhs:
        b = np.random.default_rng(0).uniform(-1, 1, b.size)
        nI = s.nI
        b[nI:nI + m.nk] -= b[nI:nI + m.nk].mean()
        b[nI + m.nk:] -= b[nI + m.nk:].mean()
    _, info = minres(lambda v: s.K @ v, b, StokesBlockDiag(s, "exact", "exact"), tol=1e-12, maxit=500)
    g2, th = est_minres(info["delta"], info["gamma"])
    ref = infsup_dense(s)
    assert th < 0
    assert abs(g2 - ref) <= 1e-8 * ref
