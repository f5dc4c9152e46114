"""Flow over a step (Sec. 3, the inflow-outflow example): the L-shaped domain
D = [-1, 0) x [0, 1]  union  [0, L] x [-1, 1]  (L = 5 in the paper), fixed
walls, the parabolic inflow u_x = 4 y (1 - y) on x = -1 and the natural
(do-nothing) outflow condition on x = L, discretised with the enriched
Taylor-Hood element Q2 - (Q1 + P0) on squares of side h = 1/m.

Test infrastructure (see the package docstring).

The mesh object has the interface of `assemble.Mesh` that the generic
assembly uses (element connectivity, Dirichlet mask, sizes), so the global
matrices, `assemble.System`, the M_1 preconditioner, FGMRES and the
two-stage driver apply unchanged.  What differs from the enclosed cavity:

* numbering: the nodes of the bounding box [-1, L] x [-1, 1] that belong to
  the closure of some element, counted row by row (y outer, x inner); the same
  for the Q1 nodes and for the elements (the P0 coefficients);
* Dirichlet rows: every boundary velocity node except those of the outflow
  segment x = L, -1 < y < 1, whose velocity values are unknowns;
* null space: with an outflow boundary the pressure function p_1 + p_0 is
  unique, so null(K) is spanned by [0; k] alone, k = [1_{n_k}; -1_{n_0}] (the
  one-dimensional null space of the text); the canonical representative has
  element pressures of mean zero;
* A_p = B_1 diag(M_v)^{-1} B_1^T is nonsingular (B_1^T 1 is nonzero through
  the outflow), so the PCD uses A_p^{-1} itself;
* F_1 with natural boundary conditions annihilates the constants (its
  diffusion and convection rows sum to zero) while A_p does not, so
  Q_1 F_1^{-1} A_p cannot stand for the nonsingular B_1 F^{-1} B_1^T.  The
  PCD literature the paper cites for these matrices (Sec. 3.1) closes this
  with a Robin condition on the inflow boundary: F_1 gains
  -int_{inflow} (w . n) psi_j psi_i ds, which for the inflow x = -1 (outward
  normal -e_x) is int w_x psi_j psi_i dy.

A "channel" variant (the strip [-1, L] x [0, 1], same inflow and outflow)
has Poiseuille flow u = (4 y (1 - y), 0), p = 8 nu (L - x) as exact solution of
Stokes and of Oseen with that wind; both are in the discrete spaces, which
pins the assembly, the outflow condition and the pressure level.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .assemble import System, frame_null_vector, q1_mass, q1_convection_diffusion, laplacian, \
    convection
from .fem import gauss01, q1_1d, q2_1d
from .krylov import fgmres
from .precond import chebyshev, lambda_max_dinv, level_viscosity, wind_speed_max, MQExact, MQDiag


def _touching(I, nmax, half):
    """Element indices along one axis that touch grid line I (half = True:
    the Q2 half grid, where odd lines lie inside one element)."""
    if half:
        return (I // 2 - 1, I // 2) if I % 2 == 0 else ((I - 1) // 2,)
    return (I - 1, I)


class StepMesh:
    """Square elements of side 1/m on the step (or channel) domain."""

    def __init__(self, m, L=5, channel=False):
        if m < 1 or L < 1:
            raise ValueError("m and L must be >= 1")
        self.m, self.L, self.channel = int(m), int(L), bool(channel)
        self.n = self.m                       # elements per unit length (level size)
        self.h = 1.0 / m
        self.x0 = -1.0
        self.y0 = 0.0 if channel else -1.0
        self.ex = (1 + L) * m                 # elements of the bounding box along x
        self.ey = m if channel else 2 * m     # ... along y
        act = np.ones((self.ey, self.ex), dtype=bool)
        if not channel:
            act[:m, :m] = False               # the step: x < 0, y < 0
        self.elem_active = act

        def node_flags(nx, ny, half):
            active = np.zeros((ny, nx), dtype=bool)
            inside = np.ones((ny, nx), dtype=bool)
            for J in range(ny):
                ty = _touching(J, self.ey, half)
                for I in range(nx):
                    tx = _touching(I, self.ex, half)
                    any_ = False
                    all_ = True
                    for b in ty:
                        for a in tx:
                            ok = 0 <= a < self.ex and 0 <= b < self.ey and act[b, a]
                            any_ = any_ or ok
                            all_ = all_ and ok
                    active[J, I] = any_
                    inside[J, I] = all_
            return active, inside

        self.nqx, self.nqy = 2 * self.ex + 1, 2 * self.ey + 1
        q2_act, q2_in = node_flags(self.nqx, self.nqy, True)
        q1_act, _ = node_flags(self.ex + 1, self.ey + 1, False)
        self.q2_active, self.q1_active = q2_act, q1_act
        self.q2_index = np.full(q2_act.shape, -1, dtype=np.int64)
        self.q2_index[q2_act] = np.arange(int(q2_act.sum()))
        self.q1_index = np.full(q1_act.shape, -1, dtype=np.int64)
        self.q1_index[q1_act] = np.arange(int(q1_act.sum()))
        self.el_index = np.full(act.shape, -1, dtype=np.int64)
        self.el_index[act] = np.arange(int(act.sum()))
        J, I = np.nonzero(q2_act)             # row-major order = compact order
        self.q2_IJ = (I, J)
        outflow = (I == self.nqx - 1) & (J > 0) & (J < self.nqy - 1)
        self._boundary = (~q2_in[J, I]) & ~outflow
        self._outflow = outflow
        self.nv = int(q2_act.sum())
        self.nk = int(q1_act.sum())
        self.n0 = int(act.sum())
        self.np_ = self.nk + self.n0
        self.N = 2 * self.nv + self.np_

    # -- interface of assemble.Mesh ----------------------------------------
    def q2_coords(self):
        I, J = self.q2_IJ
        return self.x0 + I * (self.h / 2), self.y0 + J * (self.h / 2)

    def q1_coords(self):
        J, I = np.nonzero(self.q1_active)
        return self.x0 + I * self.h, self.y0 + J * self.h

    def centroids(self):
        J, I = np.nonzero(self.elem_active)
        return self.x0 + (I + 0.5) * self.h, self.y0 + (J + 0.5) * self.h

    def element_dofs(self):
        """(vel9, q1_4, p0) compact indices of every element, in element order."""
        ey, ex = np.nonzero(self.elem_active)
        vel = np.empty((ex.size, 9), dtype=np.int64)
        for j in range(3):
            for i in range(3):
                vel[:, 3 * j + i] = self.q2_index[2 * ey + j, 2 * ex + i]
        q1 = np.empty((ex.size, 4), dtype=np.int64)
        for b in range(2):
            for a in range(2):
                q1[:, 2 * b + a] = self.q1_index[ey + b, ex + a]
        p0 = self.el_index[ey, ex]
        assert (vel >= 0).all() and (q1 >= 0).all()
        return vel, q1, p0

    def boundary_q2(self):
        """Dirichlet mask over the velocity nodes (walls and inflow)."""
        return self._boundary.copy()

    def outflow_q2(self):
        """Velocity nodes of the open outflow segment (natural condition)."""
        return self._outflow.copy()


def inflow_dirichlet(mesh):
    """Full velocity vector (2 n_v) with u_x = 4 y (1 - y) on x = -1 and zero
    on every other Dirichlet node."""
    X, Y = mesh.q2_coords()
    ux = np.where((np.abs(X - mesh.x0) < 1e-12) & mesh.boundary_q2(), 4.0 * Y * (1.0 - Y), 0.0)
    return np.concatenate([ux, np.zeros(mesh.nv)])


def poiseuille(mesh, nu):
    """Exact channel solution on the full layout: u = (4y(1-y), 0), p_1 at the
    Q1 nodes = 8 nu (L - x), p_0 = 0."""
    X, Y = mesh.q2_coords()
    Xk, _ = mesh.q1_coords()
    return np.concatenate([4.0 * Y * (1.0 - Y), np.zeros(mesh.nv), 8.0 * nu * (mesh.L - Xk),
                           np.zeros(mesh.n0)])


# -- direct solve (one-dimensional null space) ---------------------------------

def null_vector_interior(system):
    """[0_u; k] on the interior layout."""
    return np.concatenate([np.zeros(system.nI), frame_null_vector(system.mesh)])


def canonicalize(x_full, mesh):
    """Shift along k so that the element pressures have mean zero."""
    x = np.array(x_full, dtype=np.float64, copy=True)
    o = 2 * mesh.nv
    c = x[o + mesh.nk:].mean()
    x[o: o + mesh.nk] += c
    x[o + mesh.nk:] -= c
    return x


class StepLU:
    """LU factors of [[K, z], [z^T, 0]] with z = [0; k]; solve() returns the
    solution of K x = b with k^T p = 0 (then canonicalised)."""

    def __init__(self, system):
        self.system = system
        z = null_vector_interior(system)[:, None]
        Kb = sp.bmat([[system.K, sp.csr_matrix(z)], [sp.csr_matrix(z.T), None]]).tocsc()
        self.lu = spla.splu(Kb)
        self.n = system.K.shape[0]

    def solve(self, b_full, trans=False):
        s = self.system
        sol = self.lu.solve(np.concatenate([s.to_interior(b_full), [0.0]]), trans="T" if trans else "N")
        x = s.to_full(sol[: self.n], u_boundary=None if trans else b_full[: 2 * s.mesh.nv])
        return canonicalize(x, s.mesh)


def direct_solve(system, b_full):
    return StepLU(system).solve(b_full)


def stokes_start(mesh, nu):
    S = System(mesh, nu=nu)
    return direct_solve(S, S.rhs(None, inflow_dirichlet(mesh)))


def picard(mesh, nu, steps, x0=None):
    """[u^(0), ..., u^(steps)]: u^(0) the Stokes solution, then Oseen solves
    whose wind is the whole nodal velocity of the previous iterate."""
    uD = inflow_dirichlet(mesh)
    x = stokes_start(mesh, nu) if x0 is None else np.array(x0, float)
    out = [x]
    for _ in range(steps):
        S = System(mesh, nu=nu, wind=x[: 2 * mesh.nv])
        x = direct_solve(S, S.rhs(None, uD))
        out.append(x)
    return out


def line_fluxes(mesh, x_full):
    """Volume flux int u_x dy through every vertical element line x = x0 + i h
    (i = 0..ex), by Simpson's rule on each element edge (exact for the
    quadratic trace of u_x along the edge)."""
    ux = np.zeros((mesh.nqy, mesh.nqx))
    I, J = mesh.q2_IJ
    ux[J, I] = x_full[: mesh.nv]
    out = []
    for i in range(mesh.ex + 1):
        Ic = 2 * i
        f = 0.0
        for b in range(mesh.ey):
            # the edge belongs to the domain when an element on either side is active
            left = i - 1 >= 0 and mesh.elem_active[b, i - 1]
            right = i < mesh.ex and mesh.elem_active[b, i]
            if left or right:
                f += mesh.h / 6.0 * (ux[2 * b, Ic] + 4.0 * ux[2 * b + 1, Ic] + ux[2 * b + 2, Ic])
        out.append(f)
    return np.array(out)


# -- multigrid hierarchy on step meshes ----------------------------------------

def step_levels(m, coarse_m=4):
    """Element counts per unit length: halve while even and above coarse_m."""
    ms = [m]
    while ms[-1] % 2 == 0 and ms[-1] > coarse_m:
        ms.append(ms[-1] // 2)
    return ms


def _locate(mesh_c, X, Y):
    """An active coarse element containing each point, and the local coordinates."""
    H = mesh_c.h
    gx = (X - mesh_c.x0) / H
    gy = (Y - mesh_c.y0) / H
    ex = np.full(X.shape, -1, dtype=np.int64)
    ey = np.full(X.shape, -1, dtype=np.int64)
    for dx in (0, -1):
        for dy in (0, -1):
            cx = np.floor(gx + 1e-12).astype(np.int64) + dx
            cy = np.floor(gy + 1e-12).astype(np.int64) + dy
            ok = (cx >= 0) & (cx < mesh_c.ex) & (cy >= 0) & (cy < mesh_c.ey)
            ok[ok] = mesh_c.elem_active[cy[ok], cx[ok]]
            # a corner or edge point belongs to the closure of the candidate
            ok &= (gx >= cx - 1e-12) & (gx <= cx + 1 + 1e-12) & (gy >= cy - 1e-12) & (gy <= cy + 1 + 1e-12)
            take = ok & (ex < 0)
            ex[take] = cx[take]
            ey[take] = cy[take]
    assert (ex >= 0).all(), "point outside the coarse domain"
    return ex, ey, gx - ex, gy - ey


def q2_prolongation(fine, coarse):
    """Values of coarse Q2 functions at the fine Q2 nodes (nv_f x nv_c)."""
    X, Y = fine.q2_coords()
    ex, ey, xi, et = _locate(coarse, X, Y)
    vx, _ = q2_1d(xi)
    vy, _ = q2_1d(et)
    rows, cols, vals = [], [], []
    for j in range(3):
        for i in range(3):
            w = vx[i] * vy[j]
            c = coarse.q2_index[2 * ey + j, 2 * ex + i]
            nz = np.abs(w) > 1e-15
            rows.append(np.flatnonzero(nz))
            cols.append(c[nz])
            vals.append(w[nz])
    P = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(fine.nv, coarse.nv)).tocsr()
    P.sum_duplicates()
    return P


def q1_prolongation(fine, coarse):
    """Values of coarse Q1 functions at the fine Q1 nodes (nk_f x nk_c)."""
    X, Y = fine.q1_coords()
    ex, ey, xi, et = _locate(coarse, X, Y)
    vx, _ = q1_1d(xi)
    vy, _ = q1_1d(et)
    rows, cols, vals = [], [], []
    for b in range(2):
        for a in range(2):
            w = vx[a] * vy[b]
            c = coarse.q1_index[ey + b, ex + a]
            nz = np.abs(w) > 1e-15
            rows.append(np.flatnonzero(nz))
            cols.append(c[nz])
            vals.append(w[nz])
    P = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(fine.nk, coarse.nk)).tocsr()
    P.sum_duplicates()
    return P


def inject_q2(field, fine, coarse):
    """Nodal values of a Q2 field (layout [x | y]) at the coarse nodes, which
    are fine nodes."""
    I, J = coarse.q2_IJ
    idx = fine.q2_index[2 * J, 2 * I]
    return np.concatenate([field[: fine.nv][idx], field[fine.nv:][idx]])


class LevelCycle:
    """One V(nu, nu) cycle over given interior level operators A_l, transfers
    P_l (fine x coarse; restriction P_l^T) and an exact coarsest solve.
    smoother 'jacobi': nu damped-Jacobi steps x <- x + omega D^{-1}(r - A x);
    smoother 'chebyshev': the Chebyshev polynomial of degree nu in D^{-1}A on
    [lo_frac, hi_frac] * lambda_l."""

    def __init__(self, A, P, smoother="jacobi", sweeps=2, omega=0.7, lambdas=None, lo_frac=0.3,
                 hi_frac=1.1):
        self.A = [a.tocsr() for a in A]
        self.P = [p.tocsr() for p in P]
        self.dinv = [1.0 / a.diagonal() for a in self.A]
        self.smoother, self.sweeps, self.omega = smoother, sweeps, omega
        if smoother == "chebyshev" and lambdas is None:
            lambdas = [lambda_max_dinv(a) for a in self.A[:-1]]
        self.lam = lambdas
        self.lo_frac, self.hi_frac = lo_frac, hi_frac
        self.coarse = spla.splu(self.A[-1].tocsc())

    def smooth(self, lvl, r, x):
        A, dinv = self.A[lvl], self.dinv[lvl]
        if self.smoother == "jacobi":
            for _ in range(self.sweeps):
                x = x + self.omega * dinv * (r - A @ x)
            return x
        lam = self.lam[lvl]
        return chebyshev(lambda v: A @ v, lambda v: dinv * v, r, x, self.lo_frac * lam,
                         self.hi_frac * lam, self.sweeps)

    def vcycle(self, lvl, r):
        if lvl == len(self.A) - 1:
            return self.coarse.solve(r)
        x = self.smooth(lvl, r, np.zeros_like(r))
        rc = self.P[lvl].T @ (r - self.A[lvl] @ x)
        x = x + self.P[lvl] @ self.vcycle(lvl + 1, rc)
        return self.smooth(lvl, r, x)


def velocity_gmg(system, coarse_m=4, omega=0.7, sweeps=2, peclet_max=None):
    """F^{-1} (both components) by one damped-Jacobi V(2,2) cycle on the step
    hierarchy: level operators re-discretised with the injected wind and the
    viscosity of `level_viscosity`; returns (apply, cycle)."""
    mesh = system.mesh
    meshes = [StepMesh(k, mesh.L, mesh.channel) for k in step_levels(mesh.m, coarse_m)]
    wmax = wind_speed_max(system.wind, mesh) if system.wind is not None else 0.0
    A, P, free = [], [], []
    w = system.wind
    for lvl, ml in enumerate(meshes):
        if lvl > 0 and w is not None:
            w = inject_q2(w, meshes[lvl - 1], ml)
        nul = level_viscosity(system.nu, ml.h, wmax, peclet_max) if w is not None else system.nu
        F = nul * laplacian(ml)
        if w is not None:
            F = F + convection(ml, w)
        I = np.flatnonzero(~ml.boundary_q2())
        A.append(F[I][:, I])
        free.append(I)
    for lvl in range(len(meshes) - 1):
        Pf = q2_prolongation(meshes[lvl], meshes[lvl + 1])
        P.append(Pf[free[lvl]][:, free[lvl + 1]])
    cyc = LevelCycle(A, P, "jacobi", sweeps=sweeps, omega=omega)
    cyc.meshes = meshes
    m0 = A[0].shape[0]
    return (lambda r: np.concatenate([cyc.vcycle(0, r[:m0]), cyc.vcycle(0, r[m0:])])), cyc


def pressure_laplacian(mesh):
    """A_p = B_1 diag(M_v)^{-1} B_1^T over the free velocity nodes."""
    s = System(mesh)
    B1 = s.BI[: mesh.nk]
    mv = s.Mv.diagonal()[s.vI]
    return (B1 @ sp.diags(1.0 / mv) @ B1.T).tocsr()


def ap_gmg(mesh, coarse_m=4, degree=2, lambdas=None):
    """A_p^{-1} by one Chebyshev-Jacobi V(2,2) cycle over re-discretised
    A_p on the step hierarchy with bilinear transfers."""
    meshes = [StepMesh(k, mesh.L, mesh.channel) for k in step_levels(mesh.m, coarse_m)]
    A = [pressure_laplacian(ml) for ml in meshes]
    P = [q1_prolongation(meshes[l], meshes[l + 1]) for l in range(len(meshes) - 1)]
    cyc = LevelCycle(A, P, "chebyshev", sweeps=degree, lambdas=lambdas)
    cyc.meshes = meshes
    return cyc


def f1_inflow_term(mesh, wind):
    """The inflow boundary term of F_1: int_{x=-1} w_x psi_j psi_i dy over the
    inflow element edges, Q1 basis along the edge, Q2 trace of the wind
    (5-point Gauss, exact)."""
    xq, wq = gauss01(5)
    v1, _ = q1_1d(xq)
    v2, _ = q2_1d(xq)
    rows, cols, vals = [], [], []
    for b in range(mesh.ey):
        if not mesh.elem_active[b, 0]:
            continue
        kk = (mesh.q1_index[b, 0], mesh.q1_index[b + 1, 0])
        wx = sum(wind[mesh.q2_index[2 * b + j, 0]] * v2[j] for j in range(3))
        for a in range(2):
            for c in range(2):
                rows.append(kk[a])
                cols.append(kk[c])
                vals.append(mesh.h * np.sum(wq * wx * v1[a] * v1[c]))
    return sp.coo_matrix((vals, (rows, cols)), shape=(mesh.nk, mesh.nk)).tocsr()


def step_f1(system, robin=True):
    """F_1 of Sec. 3.1 on the step, with the inflow term when robin."""
    F1 = q1_convection_diffusion(system.mesh, system.wind, system.nu)
    if robin:
        F1 = F1 + f1_inflow_term(system.mesh, system.wind)
    return F1.tocsr()


class PCDStage1:
    """Stage-I preconditioner on the reduced system (Sec. 3.1) for the step:
        z_p = -A_p^{-1} F_1 Q_1^{-1} r_p,   z_u = F~^{-1}(r_u - B_1^T z_p),
    F_1 with the inflow term (step_f1) unless robin is False,
    exact pieces by default (A_p is nonsingular here); `inexact` replaces
    Q_1^{-1} by q1_steps Chebyshev-Jacobi steps on [1/4, 9/4] and A_p^{-1} by
    one cycle of ap_gmg."""

    def __init__(self, system, velocity_solve=None, inexact=False, q1_steps=10, ap_kw=None, robin=True):
        s = self.s = system
        m = s.mesh
        self.nI = s.nI
        self.B1 = s.BI[: m.nk].tocsr()
        self.vel = velocity_solve or spla.splu(s.FI.tocsc()).solve
        self.Q1 = q1_mass(m)
        self.F1 = step_f1(s, robin)
        self.Ap = pressure_laplacian(m)
        self.inexact = inexact
        if inexact:
            self.q1_steps = q1_steps
            self.q1_dinv = 1.0 / self.Q1.diagonal()
            self.apc = ap_gmg(m, **(ap_kw or {}))
        else:
            self.ap_lu = spla.splu(self.Ap.tocsc())
            self.q1_lu = spla.splu(self.Q1.tocsc())

    def schur_inv(self, rp):
        if self.inexact:
            q = chebyshev(lambda v: self.Q1 @ v, lambda v: self.q1_dinv * v, rp, np.zeros_like(rp),
                          0.25, 2.25, self.q1_steps)
            return self.apc.vcycle(0, self.F1 @ q)
        return self.ap_lu.solve(self.F1 @ self.q1_lu.solve(rp))

    def __call__(self, r):
        zp = -self.schur_inv(r[self.nI:])
        zu = self.vel(r[: self.nI] - self.B1.T @ zp)
        return np.concatenate([zu, zp])


def two_stage(system, b_full, eta=1e-6, c=10.0, restart=50, maxit=2000, stage1_prec=None,
              stage2_prec=None):
    """Step I / Step II of Sec. 3.1 on the step (the enclosed-flow driver of
    `precond.two_stage` with the step's PCD and M_1); returns the
    canonicalised full-layout solution and the info dictionary."""
    from .precond import two_stage as _two_stage, OseenM1
    s = system
    P1 = stage1_prec or PCDStage1(s)
    P2 = stage2_prec or OseenM1(s)
    x, info = _two_stage(s, b_full, eta=eta, c=c, restart=restart, maxit=maxit, stage1_prec=P1,
                         stage2_prec=P2)
    return canonicalize(x, s.mesh), info


def mq_colours(mesh):
    """Colour of every pressure frame coefficient: Q1 node (I, J) has
    (I mod 2) + 2 (J mod 2), every element 4 (the enclosed-flow colouring on
    the grid indices of the bounding box)."""
    J, I = np.nonzero(mesh.q1_active)
    return np.concatenate([(I % 2) + 2 * (J % 2), np.full(mesh.n0, 4)])


class MQChebSGS:
    """`steps` Chebyshev steps based on multicolour SGS for M_Q on [lo, 1],
    input and output projected onto k^perp (Sec. 2.3)."""

    def __init__(self, system, lo=None, steps=20):
        from .precond import multicolour_sgs
        mesh = system.mesh
        self._sgs = multicolour_sgs
        self.M = system.MQ.tocsr()
        self.col = mq_colours(mesh)
        self.k = frame_null_vector(mesh)
        self.kk = float(self.k @ self.k)
        self.lo = lo if lo is not None else min(0.01, 0.4 / (mesh.m * (1 + mesh.L)))
        self.steps = steps

    def project(self, v):
        return v - (float(self.k @ v) / self.kk) * self.k

    def __call__(self, r):
        r = self.project(r)
        z = chebyshev(lambda v: self.M @ v, lambda v: self._sgs(self.M, self.col, v, np.zeros_like(v)), r,
                      np.zeros_like(r), self.lo, 1.0, self.steps)
        return self.project(z)


def mq_diag(system):
    """diag(M_Q) with the k-bordered correction (the diagonal option of Sec. 2.3)."""
    return MQDiag(system.mesh, system.MQ)


def mq_exact(system):
    return MQExact(system.mesh, system.MQ)


__all__ = ["StepMesh", "inflow_dirichlet", "poiseuille", "StepLU", "direct_solve", "canonicalize",
           "stokes_start", "picard", "line_fluxes", "step_levels", "q2_prolongation", "q1_prolongation",
           "inject_q2", "LevelCycle", "velocity_gmg", "pressure_laplacian", "ap_gmg", "PCDStage1",
           "two_stage", "mq_diag", "mq_exact", "fgmres", "f1_inflow_term", "step_f1", "mq_colours",
           "MQChebSGS"]
