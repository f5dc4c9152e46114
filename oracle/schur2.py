"""The comparison preconditioners of Sec. 3.1 and Sec. 3.2 for the Oseen
system: the two-field PCD approximation M_2 (eq:twofield-pcd,
eq:nse-precon-ref) and the least-squares commutator M_3 (eq:lsc-definition,
eq:nse-precon-lsc), with exact pieces (sparse direct solves).

Test infrastructure: plain, slow, FP64; imported only by tests and the
benchmark's CPU leg.  Shares nothing with the HIP path.

Readings (where the text is garbled or refers to a book):
* F_0 as printed, a sum of element integrals of gradients of indicator
  functions, vanishes identically; the text says the operator comes from
  the pressure jumps across interior element edges.  Read as the
  cell-centred finite-volume operator of -nu Lap + w . grad on the
  elements: diffusion nu sum_e (|e| / d_e) [p]_e [q]_e (d_e the distance of
  the two centroids, |e|/d_e = 1 on squares), convection by upwind edge
  fluxes F_e = int_e w . n (exact for the Q2 wind by Simpson's rule): row T
  collects F_e times the upstream value over the edges of T.  No boundary
  terms (w . n = 0 on an enclosed-flow boundary).  With div w = 0 the rows
  sum to zero, so F_0 1 = 0 like F_1 1 = 0.
* LSC: H = D^{-1/2} M D^{-1/2} with the boundary scaling D of the cited
  book; here D = I (H = M = diag of the velocity mass matrix on the interior
  nodes), so M_3 is the unscaled least-squares commutator.  Parity unpinned
  as a preconditioner design beyond its definition (no printed values).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assemble import q1_mass, q1_convection_diffusion
from .precond import OseenM1


def edge_fluxes(mesh, wind):
    """(Fx, Fy): Fx[ey, i] = int over the vertical edge x = x0 + i h of
    element row ey of w . e_x (i = 0..n), Fy[j, ex] likewise for horizontal
    edges with w . e_y.  The nodal Q2 wind restricted to an edge is the
    quadratic through its three nodes, so Simpson's rule is exact."""
    n, nq, h = mesh.n, mesh.nq, mesh.h
    wx = wind[: mesh.nv].reshape(nq, nq)     # [J, I]
    wy = wind[mesh.nv:].reshape(nq, nq)
    Fx = np.empty((n, n + 1))
    for ey in range(n):
        J0 = 2 * ey
        col = lambda I: (wx[J0, I] + 4 * wx[J0 + 1, I] + wx[J0 + 2, I]) * h / 6.0
        Fx[ey] = [col(2 * i) for i in range(n + 1)]
    Fy = np.empty((n + 1, n))
    for j in range(n + 1):
        J = 2 * j
        Fy[j] = [(wy[J, 2 * ex] + 4 * wy[J, 2 * ex + 1] + wy[J, 2 * ex + 2]) * h / 6.0 for ex in range(n)]
    return Fx, Fy


def p0_convection_diffusion(mesh, wind, nu):
    """F_0 on the n^2 elements (index ey*n + ex), see the module docstring."""
    n = mesh.n
    Fx, Fy = edge_fluxes(mesh, wind)
    rows, cols, vals = [], [], []

    def add(i, j, v):
        rows.append(i)
        cols.append(j)
        vals.append(v)
    for ey in range(n):
        for ex in range(n):
            T = ey * n + ex
            # (neighbour, outward flux from T) over the four edges
            nbs = []
            if ex > 0:
                nbs.append((T - 1, -Fx[ey, ex]))
            if ex < n - 1:
                nbs.append((T + 1, Fx[ey, ex + 1]))
            if ey > 0:
                nbs.append((T - n, -Fy[ey, ex]))
            if ey < n - 1:
                nbs.append((T + n, Fy[ey + 1, ex]))
            for U, out in nbs:
                add(T, T, nu)              # diffusion: |e| / d_e = 1
                add(T, U, -nu)
                if out > 0:                # outflow: upstream value is p_T
                    add(T, T, out)
                else:                      # inflow: upstream value is p_U
                    add(T, U, out)
    return sp.coo_matrix((vals, (rows, cols)), shape=(n * n, n * n)).tocsr()


class _PressureLaplacianPinv:
    """(B M^{-1} B^T)^+ on the two-field pressure space, M = diag of the
    velocity mass matrix on the interior nodes: a bordered direct solve with
    the enclosed-flow null space span{[1_{n_k}; 0], [0; 1_{n_0}]} of B^T."""

    def __init__(self, system):
        s = system
        m = s.mesh
        mv = s.Mv.diagonal()[s.vI]
        self.Minv = 1.0 / mv
        self.L = (s.BI @ sp.diags(self.Minv) @ s.BI.T).tocsr()
        Z = np.zeros((m.np_, 2))
        Z[: m.nk, 0] = 1.0
        Z[m.nk:, 1] = 1.0
        Kb = sp.bmat([[self.L, sp.csr_matrix(Z)], [sp.csr_matrix(Z.T), None]]).tocsc()
        self.lu = spla.splu(Kb)
        self.np_ = m.np_

    def __call__(self, r):
        return self.lu.solve(np.concatenate([r, [0.0, 0.0]]))[: self.np_]


class PressureLaplacianCG:
    """(B M^{-1} B^T)^+ b by conjugate gradients on the range of the singular
    pressure Laplacian (the GPU's inexact solve): b is projected onto the
    complement of the null space (block means removed); from x = 0 the plain
    CG recurrence (residual r, direction p, rho = r.r, step rho / p.Lp,
    direction update with rho_new / rho) runs until
    r.r <= tol^2 b.b or maxit steps; x is projected at the end."""

    def __init__(self, system, tol=1e-10, maxit=2000):
        s = system
        m = s.mesh
        mv = s.Mv.diagonal()[s.vI]
        self.Minv = 1.0 / mv
        self.L = (s.BI @ sp.diags(self.Minv) @ s.BI.T).tocsr()
        self.nk = m.nk
        self.tol, self.maxit = tol, maxit
        self.iterations = 0

    def project(self, v):
        v = np.array(v, dtype=np.float64, copy=True)
        v[: self.nk] -= v[: self.nk].mean()
        v[self.nk:] -= v[self.nk:].mean()
        return v

    def __call__(self, b):
        b = self.project(b)
        x = np.zeros_like(b)
        r = b.copy()
        p = r.copy()
        rho = float(r @ r)
        stop = self.tol * self.tol * rho
        it = 0
        while rho > stop and it < self.maxit:
            q = self.L @ p
            pq = float(p @ q)
            if not pq > 0.0:
                break
            alpha = rho / pq
            x = x + alpha * p
            r = r - alpha * q
            rn = float(r @ r)
            p = r + (rn / rho) * p
            rho = rn
            it += 1
        self.iterations = it
        return self.project(x)


class OseenM2:
    """M_2 = [[F, B^T], [0, -M_S]] with the two-field PCD approximation
    M_S = diag(Q_1, Q_0) diag(F_1, F_0)^{-1} B M^{-1} B^T (eq:twofield-pcd),
    right preconditioner: z_p = -M_S^{-1} r_p with
    M_S^{-1} = (B M^{-1} B^T)^+ diag(F_1, F_0) diag(Q_1, Q_0)^{-1} (only
    applications of F_1 and F_0 are needed), z_u = F^{-1}(r_u - B^T z_p)."""

    def __init__(self, system, velocity_solve=None, q1_steps=None, lp=None):
        """velocity_solve: F^{-1} (default exact); q1_steps: None for an exact
        Q_1 solve, else that many Chebyshev-Jacobi steps on [1/4, 9/4] (the
        PCD's Q_1 solve); lp: the pressure-Laplacian pseudo-inverse (default
        the bordered direct solve, or a PressureLaplacianCG)."""
        s = self.s = system
        m = s.mesh
        self.nI = s.nI
        self.vel = velocity_solve or spla.splu(s.FI.tocsc()).solve
        self.Q1 = q1_mass(m).tocsc()
        self.q1_lu = spla.splu(self.Q1)
        self.q1_steps = q1_steps
        self.F1 = q1_convection_diffusion(m, s.wind, s.nu)
        self.F0 = p0_convection_diffusion(m, s.wind, s.nu)
        self.q0 = m.h * m.h
        self.Lp = lp or _PressureLaplacianPinv(s)
        self.Minv = 1.0 / s.Mv.diagonal()[s.vI]
        self.nk = m.nk

    def q1_inv(self, r):
        if self.q1_steps is None:
            return self.q1_lu.solve(r)
        from .precond import chebyshev
        dinv = 1.0 / self.Q1.diagonal()
        return chebyshev(lambda v: self.Q1 @ v, lambda v: dinv * v, r, np.zeros_like(r), 0.25, 2.25,
                         self.q1_steps)

    def schur_inv(self, rp):
        a = self.F1 @ self.q1_inv(rp[: self.nk])
        b = self.F0 @ (rp[self.nk:] / self.q0)
        return self.Lp(np.concatenate([a, b]))

    def __call__(self, r):
        zp = -self.schur_inv(r[self.nI:])
        zu = self.vel(r[: self.nI] - self.s.BI.T @ zp)
        return np.concatenate([zu, zp])


class OseenM3(OseenM2):
    """M_3 = [[F, B^T], [0, -M_S]] with the least-squares commutator
    M_S = (B H^{-1} B^T)(B M^{-1} F H^{-1} B^T)^{-1}(B M^{-1} B^T), H = M
    (eq:lsc-definition with D = I): M_S^{-1} = (B M^{-1} B^T)^+
    (B M^{-1} F M^{-1} B^T) (B M^{-1} B^T)^+."""

    def schur_inv(self, rp):
        t = self.Lp(rp)
        mi = self.Minv
        t = self.s.BI @ (mi * (self.s.FI @ (mi * (self.s.BI.T @ t))))
        return self.Lp(t)


def m1(system, velocity_solve=None):
    """M_1 of eq:nse-precon-ref with exact pieces (for comparisons)."""
    return OseenM1(system, velocity_solve=velocity_solve)
