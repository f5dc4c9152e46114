"""Block preconditioners for the enriched Taylor-Hood systems, written plainly
from the paper's definitions with sparse matrices.

Test infrastructure (see the package docstring).

Stokes, eq:stokes_pre with viscosity nu:  P = diag(nu*A~, M~_Q / nu), where the
pressure block is applied through the bordered (Lagrange-multiplier) system
[[M_S, k], [k^T, 0]] of Sec. 2.2 so that every output is orthogonal to the
frame null vector k.
  * exact   : M_S = M_Q  -> z = M_Q^+ r (bordered SuperLU)        (P_1, Sec. 2.4)
  * diag    : M_S = diag(M_Q) -> bordered diagonal solve           (Sec. 2.3)
  * cheb_sgs: m steps of Chebyshev semi-iteration based on symmetric
              Gauss-Seidel for M_Q (Sec. 2.3, P_2 of Sec. 2.4), on k-orthogonal
              input, output projected onto k^perp.
Velocity block: exact (SuperLU) or one geometric-multigrid V-cycle.

Oseen, eq:nse-precon-diag (block upper triangular, right preconditioning):
  * M_1 = [[F, B^T], [0, -M_Q/nu]]   (eq:nse-precon-ref)
  * stage-I PCD on the reduced Taylor-Hood system (eq:reduced-system) with
    the Schur approximation of eq:discrete-commutator1x:
        B_1 F^{-1} B_1^T ~ Q_1 F_1^{-1} A_p,  A_p = B_1 M^{-1} B_1^T,
    M = diag of the velocity mass matrix, so M_S^{-1} = A_p^+ F_1 Q_1^{-1}.
  * two_stage(): Step I / Step II of Sec. 3.1.

Multicolour ordering (the GPU-friendly reading of "symmetric Gauss-Seidel"):
Q1 node (c, d) has colour (c mod 2) + 2 (d mod 2), every element pressure has
colour 4; a symmetric sweep visits colours 0,1,2,3,4 then 3,2,1,0.
"""
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assemble import Mesh, laplacian, frame_null_vector, q1_mass, \
    q1_convection_diffusion, velocity_mass, pressure_mass
from .krylov import fgmres


# -- pressure-mass solves ------------------------------------------------------

class MQExact:
    """z = M_Q^+ r via the bordered system [[M_Q, k], [k^T, 0]] (Sec. 2.2)."""

    def __init__(self, mesh, MQ):
        k = frame_null_vector(mesh)[:, None]
        Kb = sp.bmat([[MQ, sp.csr_matrix(k)], [sp.csr_matrix(k.T), None]]).tocsc()
        self.lu = spla.splu(Kb)
        self.n = MQ.shape[0]

    def __call__(self, r):
        return self.lu.solve(np.concatenate([r, [0.0]]))[: self.n]


class MQDiag:
    """Bordered solve with M_S = diag(M_Q):  z = D^{-1}(r - lam k), k^T z = 0,
    i.e. lam = k^T D^{-1} r / k^T D^{-1} k (Sec. 2.2 with the diagonal
    approximation of Sec. 2.3)."""

    def __init__(self, mesh, MQ):
        self.dinv = 1.0 / MQ.diagonal()
        self.k = frame_null_vector(mesh)
        self.kDk = float(self.k @ (self.dinv * self.k))

    def __call__(self, r):
        y = self.dinv * r
        lam = float(self.k @ y) / self.kDk
        return y - lam * (self.dinv * self.k)


def mq_colours(mesh):
    """Colour (0..4) of every pressure frame coefficient."""
    n = mesh.n
    c = np.arange(mesh.nk) % (n + 1)
    d = np.arange(mesh.nk) // (n + 1)
    return np.concatenate([(c % 2) + 2 * (d % 2), np.full(mesh.n0, 4)])


def multicolour_sgs(M, colours, r, x):
    """One symmetric multicolour Gauss-Seidel sweep for M x = r from x:
    forward over colours 0..4, backward over 3..0 (colour 4 is diagonal within
    itself, so a repeated update of it would change nothing)."""
    x = np.array(x, dtype=np.float64, copy=True)
    dinv = 1.0 / M.diagonal()
    ncol = int(colours.max()) + 1
    order = list(range(ncol)) + list(range(ncol - 2, -1, -1))
    for col in order:
        idx = np.flatnonzero(colours == col)
        res = r[idx] - M[idx] @ x
        x[idx] += dinv[idx] * res
    return x


def chebyshev(apply_A, apply_Minv, r, x0, lo, hi, steps):
    """Chebyshev semi-iteration for A x = r preconditioned by M (eigenvalues
    of M^{-1}A assumed in [lo, hi]), `steps` applications of M^{-1}, standard
    three-term recurrence:
        theta = (hi+lo)/2, delta = (hi-lo)/2, sigma = theta/delta
        d_0 = M^{-1} r_0 / theta,  rho_0 = 1/sigma
        rho_k = 1 / (2 sigma - rho_{k-1}),
        d_k = rho_k rho_{k-1} d_{k-1} + (2 rho_k / delta) M^{-1} r_k
        x_{k+1} = x_k + d_k
    """
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma = theta / delta
    x = np.array(x0, dtype=np.float64, copy=True)
    res = r - apply_A(x)
    d = apply_Minv(res) / theta
    rho = 1.0 / sigma
    x = x + d
    for _ in range(1, steps):
        res = r - apply_A(x)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * apply_Minv(res)
        rho = rho_new
        x = x + d
    return x


class MQChebSGS:
    """`steps` Chebyshev steps based on multicolour SGS for M_Q, eigenvalue
    interval [lo, hi] of M_SGS^{-1} M_Q (hi = 1 for SGS on a symmetric positive
    semi-definite matrix), applied as  z = P q(M_SGS^{-1} M_Q) M_SGS^{-1} P r with
    P the Euclidean projector onto k^perp (symmetric positive semi-definite,
    null space span{k})."""

    def __init__(self, mesh, MQ, lo, hi=1.0, steps=20):
        self.M = MQ.tocsr()
        self.col = mq_colours(mesh)
        self.k = frame_null_vector(mesh)
        self.kk = float(self.k @ self.k)
        self.lo, self.hi, self.steps = lo, hi, steps

    def project(self, v):
        return v - (float(self.k @ v) / self.kk) * self.k

    def sgs_inv(self, r):
        return multicolour_sgs(self.M, self.col, r, np.zeros_like(r))

    def __call__(self, r):
        r = self.project(r)
        z = chebyshev(lambda v: self.M @ v, self.sgs_inv, r, np.zeros_like(r),
                      self.lo, self.hi, self.steps)
        return self.project(z)


def sgs_spectrum(mesh, MQ):
    """Dense eigenvalues of M_SGS^{-1} M_Q (small meshes only)."""
    M = MQ.toarray()
    col = mq_colours(mesh)
    n = M.shape[0]
    Minv = np.zeros_like(M)
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        Minv[:, i] = multicolour_sgs(MQ.tocsr(), col, e, np.zeros(n))
    ev = np.linalg.eigvals(Minv @ M)
    return np.sort(ev.real)


# -- geometric multigrid for the scalar Q2 Laplacian / conv-diff --------------

def gmg_levels(n, coarse_n=4):
    """Mesh sizes of the hierarchy: halve while n is even and n > coarse_n."""
    ns = [n]
    while ns[-1] % 2 == 0 and ns[-1] > coarse_n:
        ns.append(ns[-1] // 2)
    return ns


def q2_prolongation(fine, coarse):
    """Interpolation of Q2 functions of the coarse mesh at the fine Q2 nodes
    (the natural embedding of nested Q2 spaces), all nodes x all nodes."""
    Xf, Yf = fine.q2_coords()
    H = coarse.h
    ex = np.minimum(np.floor((Xf - coarse.x0) / H + 1e-12).astype(int), coarse.n - 1)
    ey = np.minimum(np.floor((Yf - coarse.y0) / H + 1e-12).astype(int), coarse.n - 1)
    xi = (Xf - coarse.x0) / H - ex
    et = (Yf - coarse.y0) / H - ey
    from .fem import q2_1d
    vx, _ = q2_1d(xi)
    vy, _ = q2_1d(et)
    rows, cols, vals = [], [], []
    for j in range(3):
        for i in range(3):
            w = vx[i] * vy[j]
            cidx = (2 * ey + j) * coarse.nq + (2 * ex + i)
            nz = np.abs(w) > 1e-15
            rows.append(np.flatnonzero(nz))
            cols.append(cidx[nz])
            vals.append(w[nz])
    P = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(fine.nv, coarse.nv)).tocsr()
    P.sum_duplicates()
    return P


def lambda_max_dinv(A):
    """Largest eigenvalue of D^{-1} A for symmetric positive definite A
    (dense for small A, else ARPACK on D^{-1/2} A D^{-1/2} from a fixed start
    vector, to about ten significant digits)."""
    d = 1.0 / np.sqrt(A.diagonal())
    S = sp.diags(d) @ A @ sp.diags(d)
    if S.shape[0] <= 400:
        return float(np.linalg.eigvalsh(S.toarray())[-1])
    return float(spla.eigsh(S, k=1, which="LA", return_eigenvectors=False, tol=1e-8,
                            ncv=40, v0=np.ones(S.shape[0]))[0])


class GMG:
    """One V-cycle for the interior scalar operator of `make_op(mesh)` applied
    to both velocity components (the velocity block of eq:stokes_pre).

    Levels by gmg_levels(); level operators re-discretised on each mesh (equal
    to the Galerkin products for nested Q2 spaces with exact integration);
    exact solve on the coarsest level; pre/post smoothing by a Chebyshev
    polynomial of the given degree in D^{-1}A with interval
    [lo_frac*lam, hi_frac*lam] where lam = lambda_max(D^{-1}A) on that level
    (given, or computed exactly).  Parity unpinned as a whole (the method is a
    preconditioner design of this implementation, the paper uses AMG); pinned
    by the Galerkin identity, symmetry and convergence-rate tests.
    """

    def __init__(self, mesh, make_op, degree=2, lo_frac=0.3, hi_frac=1.1,
                 coarse_n=4, lambdas=None):
        self.ns = gmg_levels(mesh.n, coarse_n)
        self.meshes = [Mesh(k, mesh.x0, mesh.x1, mesh.y0, mesh.y1) for k in self.ns]
        self.A, self.I, self.P = [], [], []
        for lvl, m in enumerate(self.meshes):
            bnd = m.boundary_q2()
            I = np.flatnonzero(~bnd)
            Af = make_op(m)
            self.A.append(Af[I][:, I].tocsr())
            self.I.append(I)
        for lvl in range(len(self.meshes) - 1):
            Pf = q2_prolongation(self.meshes[lvl], self.meshes[lvl + 1])
            self.P.append(Pf[self.I[lvl]][:, self.I[lvl + 1]].tocsr())
        self.dinv = [1.0 / A.diagonal() for A in self.A]
        if lambdas is None:
            lambdas = [lambda_max_dinv(A) for A in self.A[:-1]]
        self.lam = list(lambdas)
        self.degree, self.lo_frac, self.hi_frac = degree, lo_frac, hi_frac
        self.coarse_lu = spla.splu(self.A[-1].tocsc())

    def smooth(self, lvl, r, x):
        A, dinv, lam = self.A[lvl], self.dinv[lvl], self.lam[lvl]
        return chebyshev(lambda v: A @ v, lambda v: dinv * v, r, x,
                         self.lo_frac * lam, self.hi_frac * lam, self.degree)

    def vcycle(self, lvl, r):
        if lvl == len(self.A) - 1:
            return self.coarse_lu.solve(r)
        x = self.smooth(lvl, r, np.zeros_like(r))
        rc = self.P[lvl].T @ (r - self.A[lvl] @ x)
        x = x + self.P[lvl] @ self.vcycle(lvl + 1, rc)
        return self.smooth(lvl, r, x)

    def __call__(self, r_int):
        """r_int: interior velocity vector [u_x interior; u_y interior]."""
        m = self.A[0].shape[0]
        return np.concatenate([self.vcycle(0, r_int[:m]), self.vcycle(0, r_int[m:])])


def stokes_gmg(system, **kw):
    """GMG for nu*A (the Stokes velocity block)."""
    nu = system.nu
    g = GMG(system.mesh, laplacian, **kw)
    return lambda r: g(r) / nu, g


# -- block preconditioners -------------------------------------------------------

class StokesBlockDiag:
    """eq:stokes_pre with viscosity nu on the interior layout [u_I; p]:
    z_u = (nu A~)^{-1} r_u,  z_p = nu * M~_S^{+} r_p."""

    def __init__(self, system, velocity="exact", mq="exact", mq_lo=None,
                 mq_steps=20, gmg_kw=None, schur_kw=None):
        s = system
        self.s = s
        self.nI = s.nI
        if velocity == "exact":
            lu = spla.splu((s.nu * s.AI).tocsc())
            self.vel = lu.solve
        elif velocity == "gmg":
            self.vel, self.gmg = stokes_gmg(s, **(gmg_kw or {}))
        else:
            raise ValueError(velocity)
        if mq == "exact":
            self.mq = MQExact(s.mesh, s.MQ)
        elif mq == "diag":
            self.mq = MQDiag(s.mesh, s.MQ)
        elif mq == "cheb_sgs":
            self.mq = MQChebSGS(s.mesh, s.MQ, lo=mq_lo, steps=mq_steps)
        elif mq == "schur_gmg":
            self.mq = MQSchurGMG(s.mesh, s.MQ, **(schur_kw or {}))
        else:
            raise ValueError(mq)

    def __call__(self, r):
        return np.concatenate([self.vel(r[: self.nI]), self.s.nu * self.mq(r[self.nI:])])


class OseenM1:
    """M_1 = [[F~, B^T], [0, -M_Q/nu]] (eq:nse-precon-ref), right
    preconditioner:  z_p = -nu M_Q^+ r_p,  z_u = F~^{-1}(r_u - B^T z_p)."""

    def __init__(self, system, velocity_solve=None, mq=None):
        s = self.s = system
        self.nI = s.nI
        self.vel = velocity_solve or spla.splu(s.FI.tocsc()).solve
        self.mq = mq or MQExact(s.mesh, s.MQ)

    def __call__(self, r):
        zp = -self.s.nu * self.mq(r[self.nI:])
        zu = self.vel(r[: self.nI] - self.s.BI.T @ zp)
        return np.concatenate([zu, zp])


class PCDStage1:
    """Stage-I preconditioner on the reduced system [F B_1^T; B_1 0]
    (eq:reduced-system) with M_S = Q_1 F_1^{-1} A_p (eq:discrete-commutator1x):
        z_p = -A_p^+ F_1 Q_1^{-1} r_p,  z_u = F~^{-1}(r_u - B_1^T z_p).
    A_p = B_1 diag(M_v)^{-1} B_1^T over interior velocity nodes (singular,
    null space = constants; A_p^+ by a bordered solve).  F_1 and Q_1 carry no
    boundary conditions."""

    def __init__(self, system, velocity_solve=None):
        s = self.s = system
        m = s.mesh
        self.nI = s.nI
        self.B1 = s.BI[: m.nk].tocsr()
        self.vel = velocity_solve or spla.splu(s.FI.tocsc()).solve
        self.Q1 = q1_mass(m)
        self.F1 = q1_convection_diffusion(m, s.wind, s.nu)
        mv = s.Mv.diagonal()[s.vI]
        self.Ap = (self.B1 @ sp.diags(1.0 / mv) @ self.B1.T).tocsr()
        one = np.ones((m.nk, 1))
        Kb = sp.bmat([[self.Ap, sp.csr_matrix(one)], [sp.csr_matrix(one.T), None]]).tocsc()
        self.ap_lu = spla.splu(Kb)
        self.q1_lu = spla.splu(self.Q1.tocsc())

    def ap_pinv(self, r):
        return self.ap_lu.solve(np.concatenate([r, [0.0]]))[:-1]

    def schur_inv(self, rp):
        return self.ap_pinv(self.F1 @ self.q1_lu.solve(rp))

    def __call__(self, r):
        zp = -self.schur_inv(r[self.nI:])
        zu = self.vel(r[: self.nI] - self.B1.T @ zp)
        return np.concatenate([zu, zp])


def two_stage(system, b_full, eta=1e-6, c=10.0, restart=50, maxit=2000,
              stage1_prec=None, stage2_prec=None):
    """The two-stage PCD algorithm of Sec. 3.1.

    Step I:  FGMRES on the reduced system [F B_1^T; B_1 0][u; q_1] = [f; g_1]
             preconditioned by PCD, stopped when the reduced residual is
             <= c*eta*||b|| (||b|| = norm of the full lifted interior RHS, the
             initial residual for a zero initial vector).
    Step II: FGMRES on the full system with M_1 from [u_1*; q_1*; 0],
             stopped at eta*||b||.
    Returns (x_full (not canonicalised), info).
    """
    s = system
    m = s.mesh
    nI = s.nI
    b = s.to_interior(b_full)
    bnorm = float(np.linalg.norm(b))
    Kred = s.K[: nI + m.nk][:, : nI + m.nk].tocsr()
    bred = b[: nI + m.nk]
    P1 = stage1_prec or PCDStage1(s)
    x1, info1 = fgmres(lambda v: Kred @ v, bred, P1, restart=restart, maxit=maxit,
                       atol=c * eta * bnorm)
    x0 = np.concatenate([x1, np.zeros(m.n0)])
    z_star = b - s.K @ x0
    P2 = stage2_prec or OseenM1(s)
    x, info2 = fgmres(lambda v: s.K @ v, b, P2, restart=restart, maxit=maxit,
                      atol=eta * bnorm, x0=x0)
    info = dict(stage1=info1, stage2=info2, bnorm=bnorm, z_star=z_star, x_stage1=x0,
                iterations=info1["iterations"] + info2["iterations"])
    return s.to_full(x, u_boundary=b_full[: 2 * m.nv]), info


# -- inexact Oseen preconditioner pieces ---------------------------------------
# The GPU path replaces the exact solves of M_1 and PCD by the iterations
# below; the oracle implements the same algorithms so that preconditioner
# applications can be compared directly.

def inject_q2(field_fine, fine, coarse):
    """Nodal values of a Q2 field at the coarse Q2 nodes (a subset of the fine
    nodes): injection, component by component (layout [x | y])."""
    r = fine.n // coarse.n
    nc = coarse.nq
    idx = (np.arange(nc)[:, None] * r * fine.nq + np.arange(nc)[None, :] * r).reshape(-1)
    return np.concatenate([field_fine[: fine.nv][idx], field_fine[fine.nv:][idx]])


def wind_speed_max(wind, mesh):
    """max over the Q2 nodes of the Euclidean length of the nodal wind."""
    return float(np.sqrt(wind[: mesh.nv] ** 2 + wind[mesh.nv:] ** 2).max())


def level_viscosity(nu, h, wmax, peclet_max=None):
    """Viscosity of a multigrid level of element side h.  With peclet_max
    given, the level operator is nu_l A + N with
        nu_l = max(nu, wmax * h / (2 * peclet_max)),
    so that its element Peclet number wmax * h / (2 nu_l) is at most
    peclet_max: where the unstabilised Galerkin operator is convection
    dominated, the cycle approximates the inverse of a more diffusive
    operator (the paper's experiments have mesh Peclet numbers of order one
    and say nothing about this regime; see the V-cycle docstrings)."""
    if peclet_max is None:
        return nu
    return max(nu, wmax * h / (2.0 * peclet_max))


def oseen_level_operator(fine_mesh, wind, nu, peclet_max=None):
    """make_op for the GMG of F = nu A + N(w): on every level the wind is the
    injection of the finest-level nodal wind and the viscosity is
    level_viscosity(nu, h_l, max |w|, peclet_max) (nu itself when
    peclet_max is None)."""
    from .assemble import convection
    wmax = wind_speed_max(wind, fine_mesh)

    def make(mesh):
        w = wind if mesh.n == fine_mesh.n else inject_q2(wind, fine_mesh, mesh)
        nul = level_viscosity(nu, mesh.h, wmax, peclet_max)
        return nul * laplacian(mesh) + convection(mesh, w)
    return make


class GMGJacobi(GMG):
    """V(nu1, nu2) cycle with damped Jacobi smoothing x <- x + omega D^{-1}(r - A x)
    (suitable for the nonsymmetric convection-diffusion block F); exact solve on
    the coarsest level.  Parity unpinned as a whole (a design of this
    implementation; the paper uses AMG); pinned by contraction on the Oseen
    operator and by the two-stage solve reaching the direct solution."""

    def __init__(self, mesh, make_op, omega=0.7, sweeps=2, coarse_n=32):
        self.omega, self.sweeps = omega, sweeps
        super().__init__(mesh, make_op, coarse_n=coarse_n, lambdas=[1.0] * 32)

    def smooth(self, lvl, r, x):
        A, dinv = self.A[lvl], self.dinv[lvl]
        for _ in range(self.sweeps):
            x = x + self.omega * dinv * (r - A @ x)
        return x


def q1_prolongation(fine, coarse):
    """Bilinear interpolation of coarse Q1 functions at the fine Q1 nodes."""
    r = fine.n // coarse.n
    assert r == 2
    nf, nc = fine.n + 1, coarse.n + 1

    def p1(nf_, nc_):
        P = np.zeros((nf_, nc_))
        for i in range(nf_):
            if i % 2 == 0:
                P[i, i // 2] = 1.0
            else:
                P[i, i // 2] = P[i, i // 2 + 1] = 0.5
        return sp.csr_matrix(P)
    P1 = p1(nf, nc)
    return sp.kron(P1, P1).tocsr()   # y index outer, x index inner


def pressure_laplacian_Ap(mesh):
    """A_p = B_1 diag(M_v)^{-1} B_1^T over the interior velocity nodes
    (eq:discrete-commutator1x, with M the diagonal of the velocity mass)."""
    from .assemble import System
    s = System(mesh)
    B1 = s.BI[: mesh.nk]
    mv = s.Mv.diagonal()[s.vI]
    return (B1 @ sp.diags(1.0 / mv) @ B1.T).tocsr()


class ApGMG:
    """A_p^+ r by one V(deg, deg) cycle of a Q1 geometric multigrid with
    Chebyshev-Jacobi smoothing ([lo_frac, hi_frac] * lambda_max(D^{-1}A_p)),
    bilinear transfers, re-discretised A_p on every level and the bordered
    (pseudo-inverse) solve on the coarsest level; input and output are
    projected onto the mean-zero vectors (A_p is singular with the constants).
    Parity unpinned as a whole (design choices the paper leaves open); pinned
    by exactness on one level and contraction."""

    def __init__(self, mesh, coarse_n=4, degree=2, lo_frac=0.3, hi_frac=1.1, lambdas=None):
        self.ns = gmg_levels(mesh.n, coarse_n)
        self.meshes = [Mesh(k, mesh.x0, mesh.x1, mesh.y0, mesh.y1) for k in self.ns]
        self.A = [pressure_laplacian_Ap(m) for m in self.meshes]
        self.P = [q1_prolongation(self.meshes[l], self.meshes[l + 1]) for l in range(len(self.ns) - 1)]
        self.dinv = [1.0 / A.diagonal() for A in self.A]
        if lambdas is None:
            lambdas = [lambda_max_dinv(A) for A in self.A[:-1]]
        self.lam = list(lambdas)
        self.degree, self.lo_frac, self.hi_frac = degree, lo_frac, hi_frac
        Ac = self.A[-1]
        one = np.ones((Ac.shape[0], 1))
        self.coarse = spla.splu(sp.bmat([[Ac, sp.csr_matrix(one)], [sp.csr_matrix(one.T), None]]).tocsc())

    def smooth(self, lvl, r, x):
        A, dinv, lam = self.A[lvl], self.dinv[lvl], self.lam[lvl]
        return chebyshev(lambda v: A @ v, lambda v: dinv * v, r, x,
                         self.lo_frac * lam, self.hi_frac * lam, self.degree)

    def vcycle(self, lvl, r):
        if lvl == len(self.A) - 1:
            return self.coarse.solve(np.concatenate([r, [0.0]]))[:-1]
        x = self.smooth(lvl, r, np.zeros_like(r))
        rc = self.P[lvl].T @ (r - self.A[lvl] @ x)
        x = x + self.P[lvl] @ self.vcycle(lvl + 1, rc)
        return self.smooth(lvl, r, x)

    def __call__(self, r):
        r = r - r.mean()
        z = self.vcycle(0, r)
        return z - z.mean()


class PCDStage1Inexact(PCDStage1):
    """Stage-I PCD with the GPU's inexact pieces: F^{-1} by GMGJacobi,
    Q_1^{-1} by `q1_steps` Chebyshev-Jacobi steps on Wathen's interval
    [1/4, 9/4], A_p^+ by ApGMG.  Parity unpinned as an operator (its pieces'
    multigrids are); pinned by the two-stage solve reaching the direct
    solution."""

    def __init__(self, system, velocity_solve, q1_steps=10, ap_kw=None):
        super().__init__(system, velocity_solve=velocity_solve)
        self.q1_steps = q1_steps
        self.q1_dinv = 1.0 / self.Q1.diagonal()
        self.apgmg = ApGMG(system.mesh, **(ap_kw or {}))

    def q1_inv(self, r):
        return chebyshev(lambda v: self.Q1 @ v, lambda v: self.q1_dinv * v, r, np.zeros_like(r),
                         0.25, 2.25, self.q1_steps)

    def schur_inv(self, rp):
        return self.apgmg(self.F1 @ self.q1_inv(rp))


def oseen_velocity_gmg(system, omega=0.7, sweeps=2, coarse_n=32, peclet_max=None):
    """F^{-1} approximation for both velocity components of an Oseen system:
    one GMGJacobi cycle per component; with peclet_max the level operators
    carry the viscosity of level_viscosity (the finest included), which keeps
    damped Jacobi a smoother where the Galerkin F is convection dominated
    (at element Peclet numbers of 8 and more the unmodified cycle amplifies
    the error and preconditions nothing).  Pinned as a whole operator
    against the dense V-cycle formula."""
    g = GMGJacobi(system.mesh,
                  oseen_level_operator(system.mesh, system.wind, system.nu, peclet_max),
                  omega=omega, sweeps=sweeps, coarse_n=coarse_n)
    m = g.A[0].shape[0]
    return (lambda r: np.concatenate([g.vcycle(0, r[:m]), g.vcycle(0, r[m:])])), g


# -- mesh-independent pressure-mass solve by P0 elimination (Sec. 2.3 variant) --

def schur_Sk(mesh):
    """S_k = Q_k - R^T Q_0^{-1} R: the Q1 block of M_Q after eliminating the
    P0 block (Q_0 = h^2 I).  Symmetric positive semi-definite with null space
    the constants (M_Q k = 0); pT S_k p is the squared L2 distance of the Q1
    function p from its element means."""
    M = pressure_mass(mesh).tocsr()
    nk = mesh.nk
    Qk = M[:nk, :nk]
    R = M[nk:, :nk]
    q0 = M[nk:, nk:].diagonal()
    return (Qk - R.T @ sp.diags(1.0 / q0) @ R).tocsr()


class Q1GMG:
    """One V(deg, deg) cycle of a Q1 geometric multigrid for a symmetric
    positive semi-definite operator whose null space is the constants (input
    and output projected onto mean-zero vectors): Chebyshev-Jacobi smoothing
    on [lo_frac, hi_frac] * lambda_max(D^{-1} A_l), bilinear transfers and a
    bordered solve on the coarsest level.  ops[l] is the level-l operator.
    Parity unpinned as a whole; pinned by mesh-independent contraction on S_k."""

    def __init__(self, meshes, ops, degree=2, lo_frac=0.3, hi_frac=1.1, lambdas=None):
        self.meshes, self.A = meshes, ops
        self.P = [q1_prolongation(meshes[l], meshes[l + 1]) for l in range(len(meshes) - 1)]
        self.dinv = [1.0 / A.diagonal() for A in self.A]
        if lambdas is None:
            lambdas = [lambda_max_dinv(A) for A in self.A[:-1]]
        self.lam = list(lambdas)
        self.degree, self.lo_frac, self.hi_frac = degree, lo_frac, hi_frac
        Ac = self.A[-1]
        one = np.ones((Ac.shape[0], 1))
        self.coarse = spla.splu(sp.bmat([[Ac, sp.csr_matrix(one)], [sp.csr_matrix(one.T), None]]).tocsc())

    def smooth(self, lvl, r, x):
        A, dinv, lam = self.A[lvl], self.dinv[lvl], self.lam[lvl]
        return chebyshev(lambda v: A @ v, lambda v: dinv * v, r, x,
                         self.lo_frac * lam, self.hi_frac * lam, self.degree)

    def vcycle(self, lvl, r):
        if lvl == len(self.A) - 1:
            return self.coarse.solve(np.concatenate([r, [0.0]]))[:-1]
        x = self.smooth(lvl, r, np.zeros_like(r))
        rc = self.P[lvl].T @ (r - self.A[lvl] @ x)
        x = x + self.P[lvl] @ self.vcycle(lvl + 1, rc)
        return self.smooth(lvl, r, x)

    def __call__(self, r):
        r = r - r.mean()
        z = self.vcycle(0, r)
        return z - z.mean()


class MQSchurGMG:
    """M_Q^+ approximated through the block factorisation of M_Q by its P0
    block (Q_0 = h^2 I):
        z_k = B (r_k - R^T Q_0^{-1} r_0),   z_0 = Q_0^{-1} (r_0 - R z_k),
    B one Q1GMG cycle for S_k (schur_Sk) whose coarse operators are the
    re-discretised S_k scaled by (h / h_l)^2 (S_k behaves like h^2 times a
    Laplacian, so this matches the Galerkin coarse operator on smooth modes),
    input and output projected onto k^perp as in MQChebSGS.  Symmetric
    positive semi-definite; mesh-independent where the Chebyshev-SGS solve
    is not.  Pinned by: the elimination with an exact S_k^+ equals the
    bordered M_Q^+ solve; pT S_k p is the distance of p from its element
    means; the V-cycle contracts at an h-independent rate.  The multigrid
    itself is a design of this implementation (the paper only names the
    P0 elimination), so its exact output has no value to be pinned to."""

    def __init__(self, mesh, MQ, coarse_n=4, degree=2, lo_frac=0.3, hi_frac=1.1, lambdas=None):
        M = MQ.tocsr()
        nk = mesh.nk
        self.nk = nk
        self.R = M[nk:, :nk].tocsr()
        self.q0inv = 1.0 / M[nk:, nk:].diagonal()
        self.k = frame_null_vector(mesh)
        self.kk = float(self.k @ self.k)
        ns = gmg_levels(mesh.n, coarse_n)
        meshes = [Mesh(k, mesh.x0, mesh.x1, mesh.y0, mesh.y1) for k in ns]
        ops = [schur_Sk(m) * (mesh.h / m.h) ** 2 for m in meshes]
        self.gmg = Q1GMG(meshes, ops, degree, lo_frac, hi_frac, lambdas)

    def project(self, v):
        return v - (float(self.k @ v) / self.kk) * self.k

    def __call__(self, r):
        r = self.project(r)
        rk, r0 = r[: self.nk], r[self.nk:]
        zk = self.gmg(rk - self.R.T @ (self.q0inv * r0))
        z0 = self.q0inv * (r0 - self.R @ zk)
        return self.project(np.concatenate([zk, z0]))
