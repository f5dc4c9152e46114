"""Basis functions, quadrature and element matrices of the enriched Taylor-Hood
element Q2 - (Q1 + P0) on square elements (Sec. 2.1: eq:eth_pressure_space,
eq:eth_spec, eq:function_basis; bilinear forms of eq:stokes_fe).

Test infrastructure (see the package docstring).  Everything here is computed by
Gauss-Legendre quadrature from the Lagrange basis definitions; no closed-form
element tables are used, so the closed forms elsewhere can be checked against it.

Conventions
-----------
* Reference element [0,1]^2, physical element of side h: x = x_e + h*xi.
* 1-D Q2 nodes at xi = 0, 1/2, 1; 1-D Q1 nodes at xi = 0, 1.
* 2-D local index: Q2 node (i, j) -> 3*j + i, Q1 node (a, b) -> 2*b + a
  (x index fastest), matching the global row-major, x-fastest numbering.
"""
import numpy as np


def gauss01(m):
    """m-point Gauss-Legendre rule on [0, 1] (exact for degree 2m-1)."""
    x, w = np.polynomial.legendre.leggauss(m)
    return 0.5 * (x + 1.0), 0.5 * w


def q2_1d(xi):
    """1-D quadratic Lagrange basis on nodes 0, 1/2, 1 and its derivative."""
    xi = np.asarray(xi, dtype=np.float64)
    v = np.stack([(1 - xi) * (1 - 2 * xi), 4 * xi * (1 - xi), xi * (2 * xi - 1)])
    d = np.stack([4 * xi - 3, 4 - 8 * xi, 4 * xi - 1])
    return v, d


def q1_1d(xi):
    """1-D linear Lagrange basis on nodes 0, 1 and its derivative."""
    xi = np.asarray(xi, dtype=np.float64)
    v = np.stack([1 - xi, xi])
    d = np.stack([-np.ones_like(xi), np.ones_like(xi)])
    return v, d


def _tensor(vx, vy):
    """2-D tensor basis values at a tensor grid of points.

    vx: (nbx, nqx) values in x, vy: (nby, nqy) values in y.
    Returns array (nby*nbx, nqy*nqx) with local index b*nbx + a (x fastest)
    and point index qy*nqx + qx.
    """
    out = np.einsum("bq,ap->baqp", vy, vx)
    nb, na, nqy, nqx = out.shape
    return out.reshape(nb * na, nqy * nqx)


class ReferenceElement:
    """Values and derivatives of the 2-D bases at an m x m Gauss grid."""

    def __init__(self, m=5):
        xi, w = gauss01(m)
        self.w = np.einsum("q,p->qp", w, w).reshape(-1)
        v2, d2 = q2_1d(xi)
        v1, d1 = q1_1d(xi)
        # Q2 (9 functions): value, d/dxi, d/deta
        self.phi = _tensor(v2, v2)
        self.phi_x = _tensor(d2, v2)
        self.phi_y = _tensor(v2, d2)
        # Q1 (4 functions)
        self.psi = _tensor(v1, v1)
        self.psi_x = _tensor(d1, v1)
        self.psi_y = _tensor(v1, d1)


def element_matrices(h, m=5):
    """Element matrices of every bilinear form used by the method.

    Returned dictionary (element of side h):
      A    (9,9)  int grad phi_i . grad phi_j          (velocity Laplacian)
      M    (9,9)  int phi_i phi_j                      (velocity mass)
      B1x  (4,9)  -int psi_a d/dx phi_j                (Q1 rows of B, x part)
      B1y  (4,9)  -int psi_a d/dy phi_j
      B0x  (9,)   -int_T d/dx phi_j                    (P0 row of B)
      B0y  (9,)
      Qk   (4,4)  int psi_a psi_b                      (Q1 mass)
      R    (4,)   int_T psi_a                          (P0 x Q1 cross mass)
      Q0   float  |T|                                  (P0 mass)
      Kp   (4,4)  int grad psi_a . grad psi_b          (Q1 Laplacian)
      Cx, Cy (9,9,9)  convection tensors: N_T[i,j] = sum_m Cx[i,j,m] wx_m + Cy[i,j,m] wy_m
                  where N_T[i,j] = int (w . grad phi_j) phi_i and w = sum_m w_m phi_m
      Cpx, Cpy (4,4,9)  the same for Q1 test/trial functions and a Q2 wind
    The sign of B follows b(u, p) = -int p div u (eq:stokes_fe).
    """
    r = ReferenceElement(m)
    W = r.w
    h2 = h * h
    out = {}
    out["A"] = np.einsum("q,iq,jq->ij", W, r.phi_x, r.phi_x) + np.einsum(
        "q,iq,jq->ij", W, r.phi_y, r.phi_y)
    out["M"] = h2 * np.einsum("q,iq,jq->ij", W, r.phi, r.phi)
    out["B1x"] = -h * np.einsum("q,aq,jq->aj", W, r.psi, r.phi_x)
    out["B1y"] = -h * np.einsum("q,aq,jq->aj", W, r.psi, r.phi_y)
    out["B0x"] = -h * np.einsum("q,jq->j", W, r.phi_x)
    out["B0y"] = -h * np.einsum("q,jq->j", W, r.phi_y)
    out["Qk"] = h2 * np.einsum("q,aq,bq->ab", W, r.psi, r.psi)
    out["R"] = h2 * np.einsum("q,aq->a", W, r.psi)
    out["Q0"] = h2 * float(np.sum(W))
    out["Kp"] = np.einsum("q,aq,bq->ab", W, r.psi_x, r.psi_x) + np.einsum(
        "q,aq,bq->ab", W, r.psi_y, r.psi_y)
    out["Cx"] = h * np.einsum("q,iq,jq,mq->ijm", W, r.phi, r.phi_x, r.phi)
    out["Cy"] = h * np.einsum("q,iq,jq,mq->ijm", W, r.phi, r.phi_y, r.phi)
    out["Cpx"] = h * np.einsum("q,aq,bq,mq->abm", W, r.psi, r.psi_x, r.phi)
    out["Cpy"] = h * np.einsum("q,aq,bq,mq->abm", W, r.psi, r.psi_y, r.phi)
    return out


def eval_q2_field(nodal9, xi, eta):
    """Evaluate a Q2 element field (9 local nodal values) at (xi, eta)."""
    vx, _ = q2_1d(np.atleast_1d(xi))
    vy, _ = q2_1d(np.atleast_1d(eta))
    basis = np.einsum("bq,aq->baq", vy, vx).reshape(9, -1)
    return nodal9 @ basis
