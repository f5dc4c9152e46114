"""Direct solution of the enriched Taylor-Hood systems, canonicalisation of the
pressure frame, and adjoint gradients.

Test infrastructure (see the package docstring).

The discrete solution of eq:stokes_fe / eq:oseen-system is unique in the
velocity; the pressure frame vector is unique only up to the null space of
B^T.  For enclosed flow that null space is spanned by [1_{n_k}; 0] and
[0; 1_{n_0}] (a constant vertex pressure and a constant element pressure; the
frame null vector k of eq:pressure_null_vector is their difference).  The
oracle borders the system with both vectors, which returns the canonical
representative with sum(p_k) = sum(p_0) = 0.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def pressure_null_basis(mesh, n_int_vel):
    """Columns [0_u; 1_{n_k}; 0] and [0_u; 0; 1_{n_0}] on the interior layout."""
    Z = np.zeros((n_int_vel + mesh.np_, 2))
    Z[n_int_vel: n_int_vel + mesh.nk, 0] = 1.0
    Z[n_int_vel + mesh.nk:, 1] = 1.0
    return Z


class BorderedLU:
    """LU factors of [[K, Z], [Z^T, 0]] with Z the enclosed-flow pressure
    null basis; solve() returns the canonical solution of K x = b and the two
    Lagrange multipliers (zero for a consistent b)."""

    def __init__(self, system):
        self.system = system
        m = system.mesh
        Z = pressure_null_basis(m, system.nI)
        self.Z = Z
        Kb = sp.bmat([[system.K, sp.csr_matrix(Z)], [sp.csr_matrix(Z.T), None]]).tocsc()
        self.lu = spla.splu(Kb)
        self.n = system.K.shape[0]

    def solve_interior(self, b_int, trans=False):
        rhs = np.concatenate([b_int, np.zeros(2)])
        sol = self.lu.solve(rhs, trans="T" if trans else "N")
        return sol[: self.n], sol[self.n:]

    def solve(self, b_full, trans=False):
        """Full-layout solve: boundary rows of b carry the Dirichlet data."""
        s = self.system
        x_int, _ = self.solve_interior(s.to_interior(b_full), trans=trans)
        return s.to_full(x_int, u_boundary=b_full[: 2 * s.mesh.nv] if not trans else None)


def canonicalize(x_full, mesh):
    """Remove the means of the Q1 and P0 pressure blocks (the enclosed-flow
    canonical representative of the pressure frame vector)."""
    x = np.array(x_full, dtype=np.float64, copy=True)
    o = 2 * mesh.nv
    x[o: o + mesh.nk] -= x[o: o + mesh.nk].mean()
    x[o + mesh.nk:] -= x[o + mesh.nk:].mean()
    return x


def direct_solve(system, b_full):
    """Canonical full-layout solution of the lifted system."""
    return canonicalize(BorderedLU(system).solve(b_full), system.mesh)


def rel_err(x, y):
    """Relative 2-norm difference ||x - y|| / ||y||."""
    d = np.linalg.norm(np.asarray(x) - np.asarray(y))
    return d / max(np.linalg.norm(y), 1e-300)


# -- adjoint ---------------------------------------------------------------

def misfit(system, x_full, u_target_full):
    """J = 1/2 (u - u_t)^T M_v (u - u_t) over all velocity nodes."""
    m = system.mesh
    e = x_full[: 2 * m.nv] - u_target_full[: 2 * m.nv]
    return 0.5 * float(e @ (system.Mv @ e))


def adjoint_gradients(system, x_full, u_target_full, lu=None):
    """Discrete adjoint of J(u(f, nu)) for the lifted system.

    lambda solves K^T lambda = dJ/dx on the interior layout (dJ/dx =
    [M_v (u - u_t)]_I, zero pressure part); then, with lambda zero-extended to
    the boundary velocity nodes,
      dJ/df  = M_v lambda_u                      (all nodal forces)
      dJ/dnu = -lambda_u^T (A u_full)_I          (b depends on nu via -nu A_IB u_B,
                                                  K via nu A_II).
    Returns (lambda_full, dJdf, dJdnu).
    """
    m = system.mesh
    lu = lu if lu is not None else BorderedLU(system)
    e = x_full[: 2 * m.nv] - u_target_full[: 2 * m.nv]
    g = np.zeros(m.N)
    g[: 2 * m.nv] = system.Mv @ e
    g_int = system.to_interior(g)
    lam_int, _ = lu.solve_interior(g_int, trans=True)
    lam = system.to_full(lam_int)
    lam_u = lam[: 2 * m.nv]
    dJdf = system.Mv @ lam_u
    Au = system.Av @ x_full[: 2 * m.nv]
    dJdnu = -float(lam_u[system.vI] @ Au[system.vI])
    return lam, dJdf, dJdnu
