"""Pins of the oracle's pressure convection-diffusion pieces (Sec. 3.1: the
matrices Q_1 and F_1 behind eq:discrete-commutator1x) and of the diagonal
pressure-mass approximation (Sec. 2.3), against values fixed by the
mathematics rather than by the oracle's own formulas:

* element tensors of F_1 against exact 1-D tables (rational numbers from the
  Lagrange bases, integrated by hand);
* F_1 applied to the linear and bilinear functions, with constant and with the
  recirculating wind, against nodal values worked out by integration by parts
  (these fix the viscosity scaling, the sign of the convection term and which
  factor carries the derivative);
* the Galerkin identity P^T F_h P = F_H for the Q2 and Q1 convection-diffusion
  operators with the recirculating wind (nested spaces, exact quadrature);
* the spectrum of diag(M_Q)^{-1} M_Q by brute force (largest eigenvalue 13/4,
  smallest nonzero one proportional to h^2);
* the sign of the PCD Schur approximation: (A_p^+ F_1 Q_1^{-1})(B_1 F^{-1} B_1^T)
  has its spectrum on mean-zero vectors in one box of the right half-plane
  for every mesh, while the same product with the convection term transposed
  leaves it."""
import numpy as np
import pytest
import scipy.linalg

from oracle import precond as pc
from oracle.assemble import (Mesh, System, convection, frame_null_vector, laplacian,
                             q1_convection_diffusion, q1_mass, recirculating_wind)
from oracle.fem import element_matrices

H = 0.3
# int_0^1 psi_a psi_b phi_m and int_0^1 psi_a psi_b' phi_m on the reference
# interval (psi: Q1 basis 1 - x, x; phi: Q2 basis on 0, 1/2, 1), exact rationals
T1M = np.array([[[9, 12, -1], [1, 8, 1]], [[1, 8, 1], [-1, 12, 9]]]) / 60.0
T1C = np.array([[[-1, -2, 0], [1, 2, 0]], [[0, -2, -1], [0, 2, 1]]]) / 6.0
KP1 = np.array([[1.0, -1.0], [-1.0, 1.0]]) / H       # Q1 stiffness, width H
MP1 = np.array([[2.0, 1.0], [1.0, 2.0]]) * H / 6.0   # Q1 mass, width H


def test_q1_element_tensors_match_exact_tables():
    E = element_matrices(H)
    # local Q1 index 2*b + a and Q2 index 3*j + i, x index fastest
    np.testing.assert_allclose(E["Kp"], np.kron(MP1, KP1) + np.kron(KP1, MP1), atol=1e-13)
    Cpx = np.einsum("abm,cdn->cadbnm", T1C, H * T1M).reshape(4, 4, 9)
    Cpy = np.einsum("abm,cdn->acbdmn", T1C, H * T1M).reshape(4, 4, 9)
    np.testing.assert_allclose(E["Cpx"], Cpx, atol=1e-14)
    np.testing.assert_allclose(E["Cpy"], Cpy, atol=1e-14)
    # summing the Q2 index reproduces the constant-wind Q1 convection
    np.testing.assert_allclose(T1M.sum(axis=2), MP1 / H, atol=1e-15)


def _q1_grid(m):
    I = np.arange(m.nk) % (m.n + 1)
    J = np.arange(m.nk) // (m.n + 1)
    X, Y = m.q1_coords()
    return I, J, X, Y


def _area_weights(m):
    """int psi_i over the domain: h^2 halved once per boundary direction."""
    I, J, _, _ = _q1_grid(m)
    wx = np.where((I == 0) | (I == m.n), 0.5, 1.0)
    wy = np.where((J == 0) | (J == m.n), 0.5, 1.0)
    return m.h * m.h * wx * wy


def _edge_flux(m, along_x):
    """int_boundary psi_i n_x ds (along_x) or n_y ds: +-h on the right/left
    (top/bottom) wall, +-h/2 at its corners, 0 elsewhere."""
    I, J, _, _ = _q1_grid(m)
    a, b = (I, J) if along_x else (J, I)
    w = np.where((b == 0) | (b == m.n), 0.5, 1.0) * m.h
    return np.where(a == m.n, w, 0.0) - np.where(a == 0, w, 0.0)


@pytest.mark.parametrize("n", [3, 6])
def test_f1_on_linear_and_bilinear_functions_constant_wind(n):
    """Constant wind (a, b): F_1 x = nu * int_boundary psi n_x + a * int psi,
    F_1 y likewise; at interior nodes F_1 (xy) = (a y_i + b x_i) h^2 (the
    Laplacian term vanishes by parts, the linear integrand is symmetric over the
    node's support)."""
    m = Mesh(n, -0.5, 1.0, 0.2, 1.7)
    a, b, nu = 1.3, -0.6, 0.07
    w = np.concatenate([np.full(m.nv, a), np.full(m.nv, b)])
    F1 = q1_convection_diffusion(m, w, nu)
    I, J, X, Y = _q1_grid(m)
    area = _area_weights(m)
    np.testing.assert_allclose(F1 @ X, nu * _edge_flux(m, True) + a * area, atol=1e-13)
    np.testing.assert_allclose(F1 @ Y, nu * _edge_flux(m, False) + b * area, atol=1e-13)
    inner = (I > 0) & (I < n) & (J > 0) & (J < n)
    np.testing.assert_allclose((F1 @ (X * Y))[inner], ((a * Y + b * X) * m.h ** 2)[inner],
                               atol=1e-13)
    # constants are annihilated only by the convection-diffusion operator with
    # no net boundary flux: here nu * 0 + (w . grad 1) = 0 as well
    assert np.abs(F1 @ np.ones(m.nk)).max() < 1e-13


@pytest.mark.parametrize("n", [4, 8])
def test_f1_recirculating_wind_on_linear_functions(n):
    """w = (2y(1-x^2), -2x(1-y^2)) on [-1,1]^2, interior nodes: F_1 x =
    int w_x psi_i = 2 y_i h * (h (1 - x_i^2) - h^3/6) and F_1 y = -2 x_i h *
    (h (1 - y_i^2) - h^3/6) (the diffusion term vanishes for linear
    functions away from the boundary)."""
    m = Mesh(n, -1.0, 1.0, -1.0, 1.0)
    F1 = q1_convection_diffusion(m, recirculating_wind(m), 0.01)
    I, J, X, Y = _q1_grid(m)
    h = m.h
    inner = (I > 0) & (I < n) & (J > 0) & (J < n)
    ex = 2 * Y * h * (h * (1 - X ** 2) - h ** 3 / 6)
    ey = -2 * X * h * (h * (1 - Y ** 2) - h ** 3 / 6)
    np.testing.assert_allclose((F1 @ X)[inner], ex[inner], atol=1e-14)
    np.testing.assert_allclose((F1 @ Y)[inner], ey[inner], atol=1e-14)


def test_galerkin_identity_convection_diffusion_recirculating_wind():
    """Nested Q2 (and Q1) spaces with the wind exactly representable on both
    meshes and exact quadrature: P^T F_h P = F_H for F = nu A + N(w) and for
    F_1.  The multigrid for F and the PCD's coarse pieces rely on it."""
    fine, coarse = Mesh(8, -1, 1, -1, 1), Mesh(4, -1, 1, -1, 1)
    nu = 0.013
    Ff = nu * laplacian(fine) + convection(fine, recirculating_wind(fine))
    Fc = nu * laplacian(coarse) + convection(coarse, recirculating_wind(coarse))
    P = pc.q2_prolongation(fine, coarse)
    D = (P.T @ Ff @ P - Fc).toarray()
    assert np.abs(D).max() < 1e-13 * np.abs(Fc.toarray()).max()
    P1 = pc.q1_prolongation(fine, coarse)
    F1f = q1_convection_diffusion(fine, recirculating_wind(fine), nu)
    F1c = q1_convection_diffusion(coarse, recirculating_wind(coarse), nu)
    D1 = (P1.T @ F1f @ P1 - F1c).toarray()
    assert np.abs(D1).max() < 1e-13 * np.abs(F1c.toarray()).max()
    Q1f, Q1c = q1_mass(fine), q1_mass(coarse)
    assert np.abs((P1.T @ Q1f @ P1 - Q1c).toarray()).max() < 1e-15


@pytest.mark.parametrize("n", [4, 8, 16])
def test_diag_mq_spectrum(n):
    """diag(M_Q)^{-1} M_Q (the C1 pressure block, Sec. 2.3): one zero
    eigenvalue (k), largest 13/4 on every mesh, smallest nonzero one
    O(h^2): lambda_min * n^2 in [0.55, 0.6] for n = 4, 8, 16 (so MINRES counts
    with it grow like 1/h).  The bordered diagonal solve z = D^{-1}(r - lam k),
    k^T z = 0, preconditions M_Q on k^perp with the spectrum of the projected
    pencil (P M P, P D P), P the Euclidean projector onto k^perp."""
    m = Mesh(n)
    s = System(m)
    M = s.MQ.toarray()
    ds = 1.0 / np.sqrt(np.diag(M))
    ev = np.linalg.eigvalsh(ds[:, None] * M * ds[None, :])
    assert abs(ev[0]) < 1e-13 and ev[1] > 1e-6
    assert abs(ev[-1] - 3.25) < 1e-12
    assert 0.55 < ev[1] * n * n < 0.6, ev[1] * n * n
    op = pc.MQDiag(m, s.MQ)
    Z = np.column_stack([op(e) for e in np.eye(m.np_)])
    k = frame_null_vector(m)
    U = np.linalg.svd(np.eye(m.np_) - np.outer(k, k) / (k @ k))[0][:, : m.np_ - 1]
    mu = np.sort(np.linalg.eigvals(U.T @ Z @ M @ U).real)
    pencil = scipy.linalg.eigh(U.T @ M @ U, U.T @ np.diag(np.diag(M)) @ U, eigvals_only=True)
    np.testing.assert_allclose(mu, pencil, rtol=1e-9, atol=1e-12)
    assert mu[0] > 0 and mu[-1] <= 3.25 + 1e-12


def _pcd_spectrum(m, nu, transpose_convection=False):
    s = System(m, nu=nu, wind=recirculating_wind(m))
    P = pc.PCDStage1(s)
    B1 = P.B1.toarray()
    S = B1 @ np.linalg.solve(s.FI.toarray(), B1.T)
    F1 = P.F1.toarray()
    if transpose_convection:
        F1 = F1.T
    T = np.linalg.pinv(P.Ap.toarray()) @ F1 @ np.linalg.solve(P.Q1.toarray(), S)
    nk = m.nk
    U = np.linalg.svd(np.eye(nk) - 1.0 / nk)[0][:, : nk - 1]
    return np.linalg.eigvals(U.T @ T @ U)


def test_pcd_schur_approximation_sign_and_mesh_independence():
    """The stage-I PCD approximates B_1 F^{-1} B_1^T by Q_1 F_1^{-1} A_p
    (eq:discrete-commutator1x), so A_p^+ F_1 Q_1^{-1} S is close to the
    identity in a mesh-independent way: on n = 4, 8, 16 (nu = 1/10,
    recirculating wind) its eigenvalues on mean-zero vectors have real parts
    in [0.15, 1] and imaginary parts below 2.  With the convection term of
    F_1 transposed (a sign error for this skew wind) real parts go negative."""
    for n in (4, 8, 16):
        m = Mesh(n, -1, 1, -1, 1)
        ev = _pcd_spectrum(m, 0.1)
        assert ev.real.min() > 0.15 and ev.real.max() < 1.0, (n, ev.real.min(), ev.real.max())
        assert np.abs(ev.imag).max() < 2.0
    bad = _pcd_spectrum(Mesh(8, -1, 1, -1, 1), 0.1, transpose_convection=True)
    assert bad.real.min() < -0.3
