"""Krylov solvers written out from the paper.

Test infrastructure (see the package docstring).

minres  -- preconditioned MINRES exactly in the order of alg:minres (Sec. 2.1,
           after eq:anull), with the stopping rule of Sec. 2.4 (relative
           reduction of the preconditioned residual norm |eta_j| / gamma_1).
fgmres  -- restarted GMRES with right (flexible) preconditioning, modified
           Gram-Schmidt Arnoldi and Givens rotations (Sec. 3: GMRES monitored by
           the Euclidean residual norm of eq:residual-norm).
"""
import math

import numpy as np


class KrylovBreakdown(RuntimeError):
    pass


def minres(apply, b, precond, tol=1e-8, maxit=1000, x0=None, record=False):
    """Preconditioned MINRES (alg:minres).

    apply(v) -> A v, precond(v) -> z with P z = v (P symmetric positive
    semi-definite; the singular case of Sec. 2.2 is allowed for consistent b).
    Reading of the paper's first step: at j = 1 the term (gamma_1/gamma_0) v_0 is
    taken to be zero (gamma_0 = 0, v_0 = 0).
    Stops when |eta| / gamma_1 <= tol, i.e. the P^{-1}-norm of the residual has
    been reduced by tol.  Returns (x, info) with info = dict(iterations,
    eta (history of |eta|/gamma_1), gamma, delta, converged).
    """
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    v_prev = np.zeros_like(b)
    w_prev = np.zeros_like(b)          # w^(j-1)
    w_cur = np.zeros_like(b)           # w^(j)
    v = b - apply(x)                   # v^(1)
    z = precond(v)
    g2 = float(z @ v)
    if g2 < 0 or not math.isfinite(g2):
        raise KrylovBreakdown("preconditioner is not positive semi-definite")
    gamma = math.sqrt(g2)              # gamma_1
    gamma_prev = 0.0
    info = dict(iterations=0, eta=[1.0], gamma=[gamma], delta=[], converged=False)
    if gamma == 0.0:
        info["converged"] = True
        return x, info
    eta = gamma
    gamma1 = gamma
    s_prev, s_cur = 0.0, 0.0           # s_{j-1}, s_j
    c_prev, c_cur = 1.0, 1.0           # c_{j-1}, c_j
    for j in range(1, maxit + 1):
        z = z / gamma                                   # z^(j) normalised
        Az = apply(z)
        delta = float(Az @ z)
        v_next = Az - (delta / gamma) * v
        if j > 1:
            v_next -= (gamma / gamma_prev) * v_prev
        z_next = precond(v_next)
        g2 = float(z_next @ v_next)
        if g2 < 0 and g2 > -1e-14 * abs(delta) * gamma1:
            g2 = 0.0
        if g2 < 0 or not math.isfinite(g2):
            raise KrylovBreakdown("gamma^2 < 0: preconditioner not positive semi-definite")
        gamma_next = math.sqrt(g2)
        a0 = c_cur * delta - c_prev * s_cur * gamma
        a1 = math.sqrt(a0 * a0 + gamma_next * gamma_next)
        a2 = s_cur * delta + c_prev * c_cur * gamma
        a3 = s_prev * gamma
        c_next = a0 / a1
        s_next = gamma_next / a1
        w_next = (z - a3 * w_prev - a2 * w_cur) / a1
        x = x + (c_next * eta) * w_next
        eta = -s_next * eta
        # shift the recurrences
        v_prev, v = v, v_next
        w_prev, w_cur = w_cur, w_next
        gamma_prev, gamma = gamma, gamma_next
        s_prev, s_cur = s_cur, s_next
        c_prev, c_cur = c_cur, c_next
        z = z_next
        info["iterations"] = j
        info["eta"].append(abs(eta) / gamma1)
        info["gamma"].append(gamma)
        info["delta"].append(delta)
        if abs(eta) / gamma1 <= tol:
            info["converged"] = True
            break
        if gamma == 0.0:
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
