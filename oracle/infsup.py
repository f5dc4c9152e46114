"""Oracle for the inf-sup constant of the discrete Stokes problem (Sec. 2.4,
eq:inf-sup_eig) and its EST-MINRES estimate.

Test infrastructure (imported only by tests/, smoke() and the CPU baseline).

* `infsup_dense`: gamma^2 = the smallest nonzero eigenvalue of
  B A^{-1} B^T p = sigma M_Q p restricted to p orthogonal to the frame null
  vector k (eq:pressure_null_vector), where M_Q is nonsingular; the enclosed
  flow hydrostatic pressure gives sigma = 0 and is skipped.  Dense, small n.
* `harmonic_ritz` / `est_minres`: with the block preconditioner diag(A, M_Q)
  the eigenvalues of the preconditioned saddle-point matrix are 1 and
  (1 +- sqrt(1 + 4 sigma))/2 (eq:spec_q), so a negative eigenvalue theta
  gives sigma = theta (theta - 1).  EST-MINRES takes theta from the harmonic
  Ritz values of the Lanczos process inside MINRES (the delta_j / gamma_j of
  alg:minres): with T_k = tridiag(gamma_{j+1}, delta_j, gamma_{j+1}) and
  beta = gamma_{k+1}, the harmonic Ritz values satisfy
  (T_k^2 + beta^2 e_k e_k^T) y = theta T_k y; the negative one closest to zero
  estimates the eigenvalue that belongs to gamma^2.
"""
import numpy as np
import scipy.linalg as sla

from .assemble import frame_null_vector


def infsup_dense(system):
    """gamma^2 by the dense generalised eigenproblem on k^perp (small n)."""
    s = system
    nI = s.nI
    K = s.K.toarray()
    Au = K[:nI, :nI]
    B = K[nI:, :nI]
    S = B @ np.linalg.solve(Au, B.T)
    MQ = s.MQ.toarray()
    k = frame_null_vector(s.mesh)
    # orthonormal basis of k^perp
    Q, _ = np.linalg.qr(np.column_stack([k, np.eye(len(k))]))
    Z = Q[:, 1:]
    sig = sla.eigh(Z.T @ S @ Z, Z.T @ MQ @ Z, eigvals_only=True)
    scale = max(abs(sig).max(), 1.0)
    pos = sig[sig > 1e-10 * scale]
    return float(pos.min())


def harmonic_ritz(delta, gamma):
    """Harmonic Ritz values after k = len(delta) Lanczos steps; gamma holds
    gamma_1 .. gamma_{k+1} as recorded by oracle.krylov.minres."""
    k = len(delta)
    T = np.diag(np.asarray(delta, dtype=np.float64))
    if k > 1:
        off = np.asarray(gamma[1:k], dtype=np.float64)
        T += np.diag(off, 1) + np.diag(off, -1)
    G = T @ T
    G[k - 1, k - 1] += float(gamma[k]) ** 2
    mu = sla.eigh(T, G, eigvals_only=True)          # mu = 1 / theta
    mu = mu[np.abs(mu) > 0]
    return np.sort(1.0 / mu)


def est_minres(delta, gamma):
    """(gamma^2 estimate, theta) from the negative harmonic Ritz value closest
    to zero, or (None, None) if there is none yet."""
    theta = harmonic_ritz(delta, gamma)
    neg = theta[theta < 0]
    if neg.size == 0:
        return None, None
    t = float(neg.max())
    return t * (t - 1.0), t
