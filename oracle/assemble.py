"""Global assembly of the enriched Taylor-Hood Stokes / Oseen matrices on a
uniform n x n mesh of square Q2 elements (Sec. 2, eq:saddle_point; Sec. 3,
eq:oseen-system), Dirichlet data and the lifted right-hand side.

Test infrastructure (see the package docstring).

Global layout of a full vector (length N = 2(2n+1)^2 + (n+1)^2 + n^2):
    [ u_x on all (2n+1)^2 Q2 nodes | u_y on all Q2 nodes |
      p_k on the (n+1)^2 Q1 nodes  | p_0 on the n^2 elements ]
Node (I, J) of a (m x m) grid has index J*m + I (x fastest).  The pressure
part is the frame of eq:eth_spec: first the Q1 Lagrange coefficients, then the
element indicator coefficients, so the frame null vector of
eq:pressure_null_vector is k = [1_{n_k}; -1_{n_0}].
"""
import numpy as np
import scipy.sparse as sp

from .fem import element_matrices


class Mesh:
    """Uniform mesh of n x n square elements on [x0,x1] x [y0,y1]."""

    def __init__(self, n, x0=0.0, x1=1.0, y0=0.0, y1=1.0):
        if n < 1:
            raise ValueError("n must be >= 1")
        if abs((x1 - x0) - (y1 - y0)) > 1e-14 * abs(x1 - x0):
            raise ValueError("square domain required (square elements)")
        self.n = n
        self.x0, self.x1, self.y0, self.y1 = x0, x1, y0, y1
        self.h = (x1 - x0) / n
        self.nq = 2 * n + 1            # Q2 nodes per side
        self.nv = self.nq ** 2         # Q2 nodes per velocity component
        self.nk = (n + 1) ** 2         # Q1 pressure nodes
        self.n0 = n * n                # P0 pressures (elements)
        self.np_ = self.nk + self.n0
        self.N = 2 * self.nv + self.np_

    # -- coordinates -------------------------------------------------------
    def q2_coords(self):
        t = np.arange(self.nq) * (self.h / 2)
        X, Y = np.meshgrid(self.x0 + t, self.y0 + t, indexing="xy")
        return X.reshape(-1), Y.reshape(-1)

    def q1_coords(self):
        t = np.arange(self.n + 1) * self.h
        X, Y = np.meshgrid(self.x0 + t, self.y0 + t, indexing="xy")
        return X.reshape(-1), Y.reshape(-1)

    def centroids(self):
        t = (np.arange(self.n) + 0.5) * self.h
        X, Y = np.meshgrid(self.x0 + t, self.y0 + t, indexing="xy")
        return X.reshape(-1), Y.reshape(-1)

    # -- element connectivity ---------------------------------------------
    def element_dofs(self):
        """(vel9, q1_4, p0) global node indices of every element."""
        n, nq = self.n, self.nq
        ey, ex = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        ex = ex.reshape(-1)
        ey = ey.reshape(-1)
        vel = np.empty((n * n, 9), dtype=np.int64)
        for j in range(3):
            for i in range(3):
                vel[:, 3 * j + i] = (2 * ey + j) * nq + (2 * ex + i)
        q1 = np.empty((n * n, 4), dtype=np.int64)
        for b in range(2):
            for a in range(2):
                q1[:, 2 * b + a] = (ey + b) * (n + 1) + (ex + a)
        p0 = ey * n + ex
        return vel, q1, p0

    def boundary_q2(self):
        """Boolean mask over the Q2 nodes of one component: True on the boundary."""
        I = np.arange(self.nv) % self.nq
        J = np.arange(self.nv) // self.nq
        return (I == 0) | (J == 0) | (I == self.nq - 1) | (J == self.nq - 1)


def _scatter(rows, cols, vals, shape):
    return sp.coo_matrix((vals.reshape(-1), (rows.reshape(-1), cols.reshape(-1))),
                         shape=shape).tocsr()


def _square(mesh, Ael, dofs=None):
    vel = mesh.element_dofs()[0] if dofs is None else dofs
    ne = vel.shape[0]
    rows = np.broadcast_to(vel[:, :, None], (ne, 9, 9))
    cols = np.broadcast_to(vel[:, None, :], (ne, 9, 9))
    vals = np.broadcast_to(Ael, (ne, 9, 9)) if Ael.ndim == 2 else Ael
    return _scatter(rows, cols, vals, (mesh.nv, mesh.nv))


def laplacian(mesh):
    """Scalar Q2 stiffness matrix int grad phi_i . grad phi_j (all nodes)."""
    return _square(mesh, element_matrices(mesh.h)["A"])


def velocity_mass(mesh):
    """Scalar Q2 mass matrix int phi_i phi_j (all nodes)."""
    return _square(mesh, element_matrices(mesh.h)["M"])


def convection(mesh, wind):
    """Scalar Q2 convection matrix N_ij = int (w . grad phi_j) phi_i, where the
    wind w is the Q2 field with nodal values wind = [w_x (nv); w_y (nv)]
    (the discrete wind w_h of eq:generic-conv-diff)."""
    E = element_matrices(mesh.h)
    vel = mesh.element_dofs()[0]
    wx = wind[: mesh.nv][vel]           # (ne, 9)
    wy = wind[mesh.nv:][vel]
    Nel = np.einsum("ijm,em->eij", E["Cx"], wx) + np.einsum("ijm,em->eij", E["Cy"], wy)
    return _square(mesh, Nel)


def divergence(mesh):
    """B (n_p x 2 n_v): rows [Q1 nodes; elements], columns [u_x; u_y] on all
    Q2 nodes, B = -int q div u (b(u,p) of eq:stokes_fe)."""
    E = element_matrices(mesh.h)
    vel, q1, p0 = mesh.element_dofs()
    ne = vel.shape[0]
    blocks = []
    for comp, (k1, k0) in enumerate((("B1x", "B0x"), ("B1y", "B0y"))):
        r1 = np.broadcast_to(q1[:, :, None], (ne, 4, 9))
        c1 = np.broadcast_to(vel[:, None, :], (ne, 4, 9))
        B1 = _scatter(r1, c1, np.broadcast_to(E[k1], (ne, 4, 9)), (mesh.nk, mesh.nv))
        r0 = np.broadcast_to(p0[:, None], (ne, 9))
        B0 = _scatter(r0, vel, np.broadcast_to(E[k0], (ne, 9)), (mesh.n0, mesh.nv))
        blocks.append(sp.vstack([B1, B0]))
    return sp.hstack(blocks).tocsr()


def pressure_mass(mesh):
    """M_Q = [[Q_k, R^T], [R, Q_0]] of the frame (Sec. 2.3), n_p x n_p."""
    E = element_matrices(mesh.h)
    _, q1, p0 = mesh.element_dofs()
    ne = q1.shape[0]
    Qk = _scatter(np.broadcast_to(q1[:, :, None], (ne, 4, 4)),
                  np.broadcast_to(q1[:, None, :], (ne, 4, 4)),
                  np.broadcast_to(E["Qk"], (ne, 4, 4)), (mesh.nk, mesh.nk))
    R = _scatter(np.broadcast_to(p0[:, None], (ne, 4)), q1,
                 np.broadcast_to(E["R"], (ne, 4)), (mesh.n0, mesh.nk))
    Q0 = sp.identity(mesh.n0, format="csr") * E["Q0"]
    return sp.bmat([[Qk, R.T], [R, Q0]]).tocsr()


def q1_mass(mesh):
    """Q_1 = int psi_i psi_j over the Q1 pressure nodes (Sec. 3.1)."""
    M = pressure_mass(mesh)
    return M[: mesh.nk, : mesh.nk].tocsr()


def q1_convection_diffusion(mesh, wind, nu):
    """F_1 = nu int grad psi_j . grad psi_i + int (w_h . grad psi_j) psi_i on
    the Q1 pressure nodes with natural boundary conditions (Sec. 3.1)."""
    E = element_matrices(mesh.h)
    vel, q1, _ = mesh.element_dofs()
    ne = q1.shape[0]
    wx = wind[: mesh.nv][vel]
    wy = wind[mesh.nv:][vel]
    Fel = nu * E["Kp"][None] + np.einsum("abm,em->eab", E["Cpx"], wx) + \
        np.einsum("abm,em->eab", E["Cpy"], wy)
    return _scatter(np.broadcast_to(q1[:, :, None], (ne, 4, 4)),
                    np.broadcast_to(q1[:, None, :], (ne, 4, 4)), Fel, (mesh.nk, mesh.nk))


def frame_null_vector(mesh):
    """k = [1_{n_k}; -1_{n_0}] (eq:pressure_null_vector)."""
    return np.concatenate([np.ones(mesh.nk), -np.ones(mesh.n0)])


# -- boundary data -----------------------------------------------------------

def lid_dirichlet(mesh, lid_u=1.0, corner_mode=0):
    """Full-length velocity vector (2 n_v) holding the Dirichlet data of a
    driven cavity: u = (lid_u, 0) on the top wall y = y1, zero elsewhere.
    corner_mode 0 ("watertight") sets the two top corners to zero,
    corner_mode 1 ("leaky") gives them the lid value, corner_mode 2
    ("regularised", the enclosed-flow example of Sec. 3 on [-1, 1]^2) uses
    u_x = lid_u (1 - xi^4) with xi the top-wall coordinate mapped to [-1, 1]."""
    nq = mesh.nq
    ux = np.zeros(mesh.nv)
    top = (nq - 1) * nq + np.arange(nq)
    if corner_mode == 2:
        X, _ = mesh.q2_coords()
        xi = 2.0 * (X.ravel()[top] - mesh.x0) / (mesh.x1 - mesh.x0) - 1.0
        ux[top] = lid_u * (1.0 - xi ** 4)
        return np.concatenate([ux, np.zeros(mesh.nv)])
    ux[top] = lid_u
    if corner_mode == 0:
        ux[top[0]] = 0.0
        ux[top[-1]] = 0.0
    return np.concatenate([ux, np.zeros(mesh.nv)])


def recirculating_wind(mesh):
    """Nodal Q2 values of w = (2y(1-x^2), -2x(1-y^2)) (exactly representable in
    Q2, divergence free, w.n = 0 on the boundary of [-1,1]^2)."""
    X, Y = mesh.q2_coords()
    return np.concatenate([2 * Y * (1 - X ** 2), -2 * X * (1 - Y ** 2)])


class System:
    """The discrete Stokes (wind None) or Oseen problem on one mesh.

    Velocity block F = nu*A + N(w) acting on each component; B as in
    eq:saddle_point.  Boundary velocity values are Dirichlet data; the linear
    system of eq:saddle_point / eq:oseen-system is the one on the interior
    velocity nodes and all pressure frame coefficients.
    """

    def __init__(self, mesh, nu=1.0, wind=None):
        self.mesh = mesh
        self.nu = float(nu)
        self.wind = None if wind is None else np.asarray(wind, dtype=np.float64)
        A = laplacian(mesh)
        F = nu * A
        if self.wind is not None:
            F = F + convection(mesh, self.wind)
        self.A_s = A.tocsr()                        # scalar Laplacian
        self.F_s = F.tocsr()                        # scalar conv-diff (= nu A for Stokes)
        self.Fv = sp.block_diag([self.F_s, self.F_s]).tocsr()
        self.Av = sp.block_diag([A, A]).tocsr()
        self.Mv = sp.block_diag([velocity_mass(mesh)] * 2).tocsr()
        self.B = divergence(mesh)
        self.MQ = pressure_mass(mesh)
        bnd = mesh.boundary_q2()
        self.vel_bnd = np.concatenate([bnd, bnd])
        self.vI = np.flatnonzero(~self.vel_bnd)     # interior velocity indices
        self.vB = np.flatnonzero(self.vel_bnd)
        self.nI = self.vI.size
        # interior system on [u_I; p]
        FI = self.Fv[self.vI][:, self.vI]
        BI = self.B[:, self.vI]
        self.K = sp.bmat([[FI, BI.T], [BI, None]]).tocsr()
        self.FI, self.BI = FI.tocsr(), BI.tocsr()
        self.AI = self.Av[self.vI][:, self.vI].tocsr()

    # -- layout maps -------------------------------------------------------
    def to_interior(self, x_full):
        m = self.mesh
        return np.concatenate([x_full[: 2 * m.nv][self.vI], x_full[2 * m.nv:]])

    def to_full(self, x_int, u_boundary=None):
        m = self.mesh
        x = np.zeros(m.N)
        if u_boundary is not None:
            x[self.vB] = u_boundary[self.vB]
        x[self.vI] = x_int[: self.nI]
        x[2 * m.nv:] = x_int[self.nI:]
        return x

    # -- interface semantics -------------------------------------------------
    def apply_full(self, x_full, transpose=False):
        """y = K x on the full layout: boundary entries of x are ignored and
        boundary rows of y are zero (so the Stokes operator stays symmetric)."""
        K = self.K.T if transpose else self.K
        return self.to_full(K @ self.to_interior(x_full))

    def rhs(self, f_nodal=None, u_dirichlet=None):
        """Lifted right-hand side on the full layout.

        Interior velocity rows: (M_v f_h)_I - F_IB u_B; pressure rows: -B_B u_B;
        boundary velocity rows: the Dirichlet values u_B themselves."""
        m = self.mesh
        uB = np.zeros(2 * m.nv) if u_dirichlet is None else np.asarray(u_dirichlet, float)
        uB = np.where(self.vel_bnd, uB, 0.0)
        fu = np.zeros(2 * m.nv) if f_nodal is None else self.Mv @ np.asarray(f_nodal, float)
        bu = fu - self.Fv @ uB
        bp = -(self.B @ uB)
        b = np.zeros(m.N)
        b[: 2 * m.nv] = np.where(self.vel_bnd, uB, bu)
        b[2 * m.nv:] = bp
        return b
