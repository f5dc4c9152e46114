"""Krylov solvers written out from the paper.

Test infrastructure (see the package docstring).

minres  -- preconditioned MINRES (the method of alg:minres, Sec. 2.1, after
           eq:anull) derived here from its two ingredients: the preconditioned
           Lanczos process, which builds a P-orthonormal basis q_1 .. q_k of the
           Krylov space together with the tridiagonal matrix T_k of the
           preconditioned operator in that basis, and the minimisation of
           || beta_1 e_1 - T_k y || over y by a QR factorisation of the
           (k+1) x k extended tridiagonal matrix, updated one Givens rotation
           per step.  Stopping rule of Sec. 2.4: the residual in the P^{-1}
           norm relative to its initial value.
fgmres  -- restarted GMRES with right (flexible) preconditioning, modified
           Gram-Schmidt Arnoldi and Givens rotations (Sec. 3: GMRES monitored by
           the Euclidean residual norm of eq:residual-norm).
"""
import math

import numpy as np


class KrylovBreakdown(RuntimeError):
    pass


class _Lanczos:
    """Preconditioned Lanczos for a symmetric operator A and a symmetric
    positive semi-definite preconditioner P (given as its action r -> P^{-1} r
    on consistent vectors, the singular case of Sec. 2.2 included).

    It keeps the residual-space vectors u_k = P q_k beta-scaled (u_k = beta_k
    P q_k), so that q_k = P^{-1} u_k / beta_k needs one preconditioner
    application per step.  Each step returns the diagonal entry alpha_k =
    q_k^T A q_k and the next off-diagonal entry beta_{k+1} of T_k."""

    def __init__(self, apply, precond, r0):
        self.apply, self.precond = apply, precond
        self.u_old = np.zeros_like(r0)
        self.u = r0
        self.pu = precond(r0)
        self.beta_old = 0.0
        self.beta = self._norm(self.u, self.pu, scale=None)

    @staticmethod
    def _norm(u, pu, scale):
        b2 = float(u @ pu)
        if scale is not None and -1e-14 * scale < b2 < 0:
            b2 = 0.0                       # rounding around an exact zero
        if b2 < 0 or not math.isfinite(b2):
            raise KrylovBreakdown("P is not positive semi-definite (u^T P^{-1} u < 0)")
        return math.sqrt(b2)

    def step(self):
        """Returns (q_k, alpha_k, beta_{k+1})."""
        q = self.pu / self.beta
        Aq = self.apply(q)
        alpha = float(Aq @ q)
        # three-term recurrence in the residual space; the u_{k-1} term is
        # absent at k = 1 (beta_0 = 0, u_0 = 0)
        u_new = Aq - (alpha / self.beta) * self.u
        if self.beta_old > 0.0:
            u_new -= (self.beta / self.beta_old) * self.u_old
        pu_new = self.precond(u_new)
        beta_new = self._norm(u_new, pu_new, scale=abs(alpha) * self.beta)
        self.u_old, self.u, self.pu = self.u, u_new, pu_new
        self.beta_old, self.beta = self.beta, beta_new
        return q, alpha, beta_new


class _TridiagonalQR:
    """QR factorisation of the extended tridiagonal matrix of the Lanczos
    process, one column at a time.  Column k has beta_k above the diagonal,
    alpha_k on it and beta_{k+1} below; the two previous rotations act on it,
    then a new rotation annihilates beta_{k+1}.  The R factor has three
    diagonals (rho on the diagonal, then sigma and tau above it), and the
    transformed right-hand side beta_1 e_1 gives the least-squares step t_k
    and the residual norm |phi|."""

    def __init__(self, beta1):
        self.rot = [(1.0, 0.0), (1.0, 0.0)]     # rotations k-2, k-1 as (cos, sin)
        self.phi = beta1

    def add_column(self, beta_k, alpha_k, beta_next):
        (c2, s2), (c1, s1) = self.rot
        tau = s2 * beta_k                       # row k-2
        t = c2 * beta_k
        sigma = c1 * t + s1 * alpha_k           # row k-1
        diag = -s1 * t + c1 * alpha_k           # row k before the new rotation
        rho = math.hypot(diag, beta_next)
        c, s = diag / rho, beta_next / rho
        self.rot = [(c1, s1), (c, s)]
        step = c * self.phi
        self.phi = -s * self.phi
        return rho, sigma, tau, step


def minres(apply, b, precond, tol=1e-8, maxit=1000, x0=None, record=False):
    """Preconditioned MINRES (alg:minres).

    apply(v) -> A v, precond(v) -> z with P z = v (P symmetric positive
    semi-definite; the singular case of Sec. 2.2 is allowed for consistent b).
    x_k = x_0 + Q_k y_k minimises the P^{-1}-norm of the residual over the
    Krylov space; with R_k the QR factor of the Lanczos matrix, the search
    directions d_k = (q_k - sigma_k d_{k-1} - tau_k d_{k-2}) / rho_k are the
    columns of Q_k R_k^{-1}, so x_k = x_{k-1} + t_k d_k.  Stops when
    |phi_k| / beta_1 <= tol, the relative P^{-1}-norm residual (reading of the
    algorithm's convergence test).  Returns (x, info) with info =
    dict(iterations, eta (history of |phi|/beta_1), gamma (the beta_k),
    delta (the alpha_k), converged).
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    lz = _Lanczos(apply, precond, b - apply(x))
    beta1 = lz.beta
    info = dict(iterations=0, eta=[1.0], gamma=[beta1], delta=[], converged=False)
    if beta1 == 0.0:
        info["converged"] = True
        return x, info
    qr = _TridiagonalQR(beta1)
    d_old = np.zeros_like(b)        # d_{k-2}
    d = np.zeros_like(b)            # d_{k-1}
    for k in range(1, maxit + 1):
        beta_k = lz.beta
        q, alpha, beta_next = lz.step()
        rho, sigma, tau, step = qr.add_column(beta_k if k > 1 else 0.0, alpha, beta_next)
        d_new = (q - sigma * d - tau * d_old) / rho
        x = x + step * d_new
        d_old, d = d, d_new
        info["iterations"] = k
        info["eta"].append(abs(qr.phi) / beta1)
        info["gamma"].append(beta_next)
        info["delta"].append(alpha)
        if abs(qr.phi) / beta1 <= tol or beta_next == 0.0:
            info["converged"] = True
            break
    return x, info


def _givens(a, b):
    if b == 0.0:
        return 1.0, 0.0
    r = math.hypot(a, b)
    return a / r, b / r


def fgmres(apply, b, precond, tol=1e-6, maxit=1000, restart=50, x0=None,
           atol=None):
    """Restarted flexible GMRES, right preconditioned.

    Minimises ||b - A x||_2 over x0 + span{Z}, Z_j = precond(V_j).  Stops when
    the residual norm is <= atol (default tol * ||b||).  Returns (x, info) with
    info = dict(iterations, residuals (absolute, one per Arnoldi step plus the
    initial one), converged).
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    target = tol * np.linalg.norm(b) if atol is None else atol
    r = b - apply(x)
    beta = np.linalg.norm(r)
    info = dict(iterations=0, residuals=[beta], converged=beta <= target)
    total = 0
    while not info["converged"] and total < maxit:
        m = min(restart, maxit - total)
        V = np.zeros((m + 1, b.size))
        Z = np.zeros((m, b.size))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = precond(V[j])
            w = apply(Z[j])
            for i in range(j + 1):                       # modified Gram-Schmidt
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):                           # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            total += 1
            info["residuals"].append(abs(g[j + 1]))
            if abs(g[j + 1]) <= target or H[j, j] == 0.0:
                break
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k]) if k > 0 else np.zeros(0)
        x = x + Z[:k].T @ y
        r = b - apply(x)
        beta = np.linalg.norm(r)
        info["converged"] = beta <= target * (1 + 1e-8) or abs(g[k]) <= target
        if beta == 0.0:
            info["converged"] = True
    info["iterations"] = total
    info["final_residual"] = float(np.linalg.norm(b - apply(x)))
    return x, info
