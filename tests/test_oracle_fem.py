"""Pins of the oracle's discretisation against closed forms and exact
solutions fixed by the mathematics (Sec. 2.1 eq:eth_pressure_space,
eq:stokes_fe; prop:Qnull, rem:Bnull; Sec. 3 enclosed-flow null space)."""
import numpy as np
import pytest

from oracle.assemble import (Mesh, System, frame_null_vector, lid_dirichlet,
                             recirculating_wind, convection, laplacian, q1_mass)
from oracle.direct import direct_solve, canonicalize, BorderedLU
from oracle.fem import element_matrices
from oracle.precond import q2_prolongation, gmg_levels

H = 0.3
# 1-D closed forms for an element of width h (hand-derived from the Lagrange
# bases on nodes 0, h/2, h and 0, h)
K1 = np.array([[7, -8, 1], [-8, 16, -8], [1, -8, 7]]) / (3 * H)
M1 = np.array([[4, 2, -1], [2, 16, 2], [-1, 2, 4]]) * H / 30
C1 = np.array([[-1 / 2, 2 / 3, -1 / 6], [-2 / 3, 0, 2 / 3], [1 / 6, -2 / 3, 1 / 2]])
G1 = np.array([[-5 / 6, 2 / 3, 1 / 6], [-1 / 6, -2 / 3, 5 / 6]])
MPQ = H * np.array([[1 / 6, 1 / 3, 0], [0, 1 / 3, 1 / 6]])
G0 = np.array([-1.0, 0.0, 1.0])
M0 = H * np.array([1 / 6, 2 / 3, 1 / 6])
MP = H / 6 * np.array([[2, 1], [1, 2]])


def test_element_matrices_match_closed_forms():
    E = element_matrices(H)
    # local index 3*j + i with i the x index -> np.kron(y_factor, x_factor)
    np.testing.assert_allclose(E["A"], np.kron(M1, K1) + np.kron(K1, M1), atol=1e-13)
    np.testing.assert_allclose(E["M"], np.kron(M1, M1), atol=1e-14)
    np.testing.assert_allclose(E["B1x"], -np.kron(MPQ, G1), atol=1e-14)
    np.testing.assert_allclose(E["B1y"], -np.kron(G1, MPQ), atol=1e-14)
    np.testing.assert_allclose(E["B0x"], -np.kron(M0, G0), atol=1e-14)
    np.testing.assert_allclose(E["B0y"], -np.kron(G0, M0), atol=1e-14)
    np.testing.assert_allclose(E["Qk"], np.kron(MP, MP), atol=1e-14)
    np.testing.assert_allclose(E["R"], np.full(4, H * H / 4), atol=1e-14)
    assert abs(E["Q0"] - H * H) < 1e-14
    # constant wind (1, 0): N_T = int phi_i d/dx phi_j = kron(M1, C1)
    wx = np.ones(9)
    Nx = np.einsum("ijm,m->ij", E["Cx"], wx)
    np.testing.assert_allclose(Nx, np.kron(M1, C1 * 1.0), atol=1e-14)


def _manufactured(n, nu, wind=None, second=False):
    m = Mesh(n, -0.5, 1.5, 0.25, 2.25)
    X, Y = m.q2_coords()
    if not second:
        ux, uy = X ** 2 + Y ** 2, -2 * X * Y
        dpx, dpy = 2.0, -1.0
        lap = (4.0, 0.0)
        grad = ((2 * X, 2 * Y), (-2 * Y, -2 * X))    # (d/dx, d/dy) of ux, uy
    else:
        ux, uy = Y ** 2, X ** 2
        dpx, dpy = 1.0, 1.0
        lap = (2.0, 2.0)
        grad = ((0 * X, 2 * Y), (2 * X, 0 * Y))
    fx = -nu * lap[0] + dpx + np.zeros_like(X)
    fy = -nu * lap[1] + dpy + np.zeros_like(X)
    if wind is not None:
        wx, wy = wind
        fx = fx + wx * grad[0][0] + wy * grad[0][1]
        fy = fy + wx * grad[1][0] + wy * grad[1][1]
        wvec = np.concatenate([np.full(m.nv, wx), np.full(m.nv, wy)])
    else:
        wvec = None
    s = System(m, nu=nu, wind=wvec)
    u = np.concatenate([ux, uy])
    x = direct_solve(s, s.rhs(np.concatenate([fx, fy]), u))
    Xk, Yk = m.q1_coords()
    pk = dpx * Xk + dpy * Yk
    return m, x, u, pk - pk.mean()


@pytest.mark.parametrize("n", [2, 3, 8])
@pytest.mark.parametrize("second", [False, True])
def test_manufactured_stokes_exact(n, second):
    """u in Q2, p in Q1, constant f: the Galerkin solution is the interpolant."""
    m, x, u, pk = _manufactured(n, 0.7, second=second)
    o = 2 * m.nv
    assert np.abs(x[:o] - u).max() < 1e-11
    assert np.abs(x[o:o + m.nk] - pk).max() < 1e-10
    assert np.abs(x[o + m.nk:]).max() < 1e-10


@pytest.mark.parametrize("n", [2, 5])
def test_manufactured_oseen_constant_wind_exact(n):
    m, x, u, pk = _manufactured(n, 0.05, wind=(1.0, 0.5))
    o = 2 * m.nv
    assert np.abs(x[:o] - u).max() < 1e-11
    assert np.abs(x[o:o + m.nk] - pk).max() < 1e-9


@pytest.mark.parametrize("n", [2, 4])
def test_pressure_mass_null_space_is_k(n):
    """prop:Qnull by brute force."""
    m = Mesh(n)
    s = System(m)
    ev, V = np.linalg.eigh(s.MQ.toarray())
    small = ev < 1e-12 * ev[-1]
    assert small.sum() == 1
    k = frame_null_vector(m)
    cos = abs(V[:, small][:, 0] @ k) / np.linalg.norm(k)
    assert cos > 1 - 1e-12


@pytest.mark.parametrize("n", [2, 3, 4])
def test_enclosed_flow_null_space_dimension_two(n):
    """rem:Bnull and the 2-D enclosed-flow null space (Sec. 3 cavity example):
    null(B^T) over interior velocities is span{[1;0], [0;1]} and the saddle
    point matrix has the same null space."""
    m = Mesh(n)
    s = System(m)
    BT = s.BI.T.toarray()
    U, sv, Vt = np.linalg.svd(BT)
    null = Vt[sv.size:] if sv.size < BT.shape[1] else None
    rank = int(np.sum(sv > 1e-12 * sv[0]))
    assert BT.shape[1] - rank == 2
    basis = Vt[rank:].T
    e1 = np.concatenate([np.ones(m.nk), np.zeros(m.n0)])
    e0 = np.concatenate([np.zeros(m.nk), np.ones(m.n0)])
    for e in (e1, e0):
        proj = basis @ (basis.T @ e)
        assert np.linalg.norm(proj - e) < 1e-10 * np.linalg.norm(e)
    svK = np.linalg.svd(s.K.toarray(), compute_uv=False)
    assert int(np.sum(svK < 1e-12 * svK[0])) == 2


def test_null_vector_identities_elementwise():
    m = Mesh(7, -1, 1, -1, 1)
    s = System(m)
    k = frame_null_vector(m)
    assert np.abs(s.MQ @ k).max() < 1e-15
    assert np.abs(s.B.T @ k).max() < 1e-15


@pytest.mark.parametrize("corner_mode", [0, 1])
def test_elementwise_mass_conservation(corner_mode):
    """The P0 enrichment gives zero mean divergence on every element
    (Sec. 2.1); plain Taylor-Hood (Q1 pressure only) does not."""
    m = Mesh(16)
    s = System(m)
    uB = lid_dirichlet(m, 1.0, corner_mode)
    x = direct_solve(s, s.rhs(None, uB))
    u = x[: 2 * m.nv]
    div_T = -(s.B[m.nk:] @ u)             # int_T div u_h per element
    assert np.abs(div_T).max() < 1e-10 * np.abs(u).max()
    # contrast: Taylor-Hood Q2-Q1 on the same mesh
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    B1 = s.BI[: m.nk]
    KTH = sp.bmat([[s.FI, B1.T], [B1, None]]).tocsr()
    one = np.zeros((KTH.shape[0], 1))
    one[s.nI:, 0] = 1
    Kb = sp.bmat([[KTH, sp.csr_matrix(one)], [sp.csr_matrix(one.T), None]]).tocsc()
    b = s.rhs(None, uB)
    bth = np.concatenate([b[: 2 * m.nv][s.vI], b[2 * m.nv: 2 * m.nv + m.nk], [0]])
    xth = spla.spsolve(Kb, bth)
    uth = uB.copy()
    uth[s.vI] = xth[: s.nI]
    div_th = -(s.B[m.nk:] @ uth)
    assert np.abs(div_th).max() > 1e-5


def test_convection_skew_for_recirculating_wind():
    """For the divergence-free wind with w.n = 0 (exact in Q2, exactly
    integrated) N is skew-symmetric, so F(w)^T = F(-w)."""
    m = Mesh(6, -1, 1, -1, 1)
    w = recirculating_wind(m)
    N = convection(m, w).toarray()
    assert np.abs(N + N.T).max() < 1e-13 * np.abs(N).max()
    sp_ = System(m, nu=0.01, wind=w)
    sm = System(m, nu=0.01, wind=-w)
    assert np.abs((sp_.K.T - sm.K).toarray()).max() < 1e-13


def test_galerkin_identity_q2():
    """P^T A_h P = A_H for nested Q2 spaces with exact integration."""
    fine, coarse = Mesh(8), Mesh(4)
    P = q2_prolongation(fine, coarse)
    Ah, AH = laplacian(fine), laplacian(coarse)
    assert abs(P.T @ Ah @ P - AH).max() < 1e-13
    # prolongation reproduces a Q2 function exactly
    X, Y = coarse.q2_coords()
    Xf, Yf = fine.q2_coords()
    f = lambda x, y: x * x * y - 3 * x * y * y + 2 * y
    assert np.abs(P @ f(X, Y) - f(Xf, Yf)).max() < 1e-13
    assert gmg_levels(256) == [256, 128, 64, 32, 16, 8, 4]
    assert gmg_levels(48) == [48, 24, 12, 6, 3]


@pytest.mark.parametrize("n", [4, 8, 16])
def test_q1_mass_jacobi_interval(n):
    """Wathen's bound for bilinear mass matrices: diag(Q)^{-1} Q has its
    eigenvalues in [1/4, 9/4], independently of h."""
    Q = q1_mass(Mesh(n)).toarray()
    d = 1 / np.sqrt(np.diag(Q))
    ev = np.linalg.eigvalsh(d[:, None] * Q * d[None, :])
    assert ev[0] >= 0.25 - 1e-12 and ev[-1] <= 2.25 + 1e-12
