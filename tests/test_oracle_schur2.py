"""Pins of the comparison preconditioners of Sec. 3.1 (two-field PCD, M_2)
and Sec. 3.2 (least-squares commutator, M_3) in the oracle (oracle/schur2.py).

* F_0 (the jump-based P0 convection-diffusion operator): with no wind it is
  nu times the element-adjacency graph Laplacian; on linear and quadratic
  element functions with a constant wind it reproduces the element integrals
  of -nu Lap p + w . grad p at interior elements; its rows sum to zero for
  the divergence-free recirculating wind; the edge fluxes equal the exact
  integrals of w . n.
* The pressure Laplacian B M^{-1} B^T has exactly the two enclosed-flow null
  vectors; its CG pseudo-inverse equals the bordered direct one.
* M_S^{-1} of M_2 and of M_3 maps into the complement of the null space of
  B F^{-1} B^T (the paper notes that M_S and B F^{-1} B^T share it).
* Convergence as the paper describes it: M_1 about 50 GMRES iterations per
  decade; M_2 a fast first phase then stagnation, whose onset is delayed on
  the finer mesh; M_3 converging for Q2-Q1* on squares (footnote of Sec. 3.2).
"""
import numpy as np
import pytest

from oracle.assemble import Mesh, System, lid_dirichlet, recirculating_wind
from oracle.krylov import fgmres
from oracle.schur2 import (OseenM2, OseenM3, PressureLaplacianCG, _PressureLaplacianPinv, edge_fluxes, m1,
                           p0_convection_diffusion)


def test_f0_without_wind_is_the_graph_laplacian():
    m = Mesh(2)
    F0 = p0_convection_diffusion(m, np.zeros(2 * m.nv), 0.3).toarray()
    L = np.array([[2, -1, -1, 0], [-1, 2, 0, -1], [-1, 0, 2, -1], [0, -1, -1, 2]], float)
    assert np.allclose(F0, 0.3 * L, atol=1e-15)


@pytest.mark.parametrize("a,c", [(1.0, 0.5), (-0.7, 0.2)])
def test_f0_on_linear_and_quadratic_functions(a, c):
    """Interior elements, constant wind (a, c): F_0 applied to the element
    values of p equals int_T (-nu Lap p + w . grad p): exact for linear p
    (upwind differences of a linear function), and the diffusion part exact
    for quadratics (second differences)."""
    n, nu = 8, 0.05
    m = Mesh(n)
    X, Y = m.q2_coords()
    wind = np.concatenate([np.full(m.nv, a), np.full(m.nv, c)])
    F0 = p0_convection_diffusion(m, wind, nu)
    cx, cy = m.centroids()
    h = m.h
    inner = ((cx > h) & (cx < 1 - h) & (cy > h) & (cy < 1 - h))
    p = 2 * cx - 3 * cy                       # linear: Lap p = 0, w . grad p = 2a - 3c
    assert np.allclose((F0 @ p)[inner], (2 * a - 3 * c) * h * h, atol=1e-13)
    q = cx ** 2 + cy ** 2                     # diffusion of a quadratic: -nu Lap q = -4 nu
    D0 = p0_convection_diffusion(m, np.zeros(2 * m.nv), nu)
    assert np.allclose((D0 @ q)[inner], -4 * nu * h * h, atol=1e-13)


def test_f0_rows_sum_to_zero_and_fluxes_are_exact():
    n = 8
    m = Mesh(n, -1, 1, -1, 1)
    w = recirculating_wind(m)
    F0 = p0_convection_diffusion(m, w, 0.01)
    assert np.abs(F0 @ np.ones(m.n0)).max() < 1e-14
    # int over x = xi, y in [y0, y0 + h] of 2y(1 - x^2) = (1 - xi^2)((y0 + h)^2 - y0^2)
    Fx, Fy = edge_fluxes(m, w)
    h = m.h
    for ey in range(n):
        y0 = -1 + ey * h
        for i in range(n + 1):
            xi = -1 + i * h
            assert abs(Fx[ey, i] - (1 - xi ** 2) * ((y0 + h) ** 2 - y0 ** 2)) < 1e-14
    for j in range(n + 1):
        yj = -1 + j * h
        for ex in range(n):
            x0 = -1 + ex * h
            assert abs(Fy[j, ex] - (-(1 - yj ** 2) * ((x0 + h) ** 2 - x0 ** 2))) < 1e-14


def test_pressure_laplacian_null_space_and_cg():
    m = Mesh(4, -1, 1, -1, 1)
    s = System(m, nu=0.01, wind=recirculating_wind(m))
    d = _PressureLaplacianPinv(s)
    ev = np.linalg.eigvalsh(d.L.toarray())
    assert np.sum(ev < 1e-12 * ev[-1]) == 2
    m = Mesh(16, -1, 1, -1, 1)
    s = System(m, nu=0.01, wind=recirculating_wind(m))
    cg = PressureLaplacianCG(s, tol=1e-13)
    d = _PressureLaplacianPinv(s)
    b = np.random.default_rng(3).standard_normal(m.np_)
    x = cg(b)
    xd = d(cg.project(b))
    assert np.linalg.norm(x - xd) < 1e-11 * np.linalg.norm(xd)
    assert abs(x[: m.nk].sum()) < 1e-10 and abs(x[m.nk:].sum()) < 1e-10


@pytest.mark.parametrize("cls", [OseenM2, OseenM3])
def test_schur_approximations_keep_the_null_space(cls):
    m = Mesh(8, -1, 1, -1, 1)
    s = System(m, nu=0.02, wind=recirculating_wind(m))
    P = cls(s)
    z = P.schur_inv(np.random.default_rng(1).standard_normal(m.np_))
    for v in (np.r_[np.ones(m.nk), np.zeros(m.n0)], np.r_[np.zeros(m.nk), np.ones(m.n0)]):
        assert abs(z @ v) < 1e-10 * np.linalg.norm(z) * np.linalg.norm(v)


def _history(n, make):
    m = Mesh(n, -1, 1, -1, 1)
    s = System(m, nu=0.01, wind=recirculating_wind(m))
    b = s.to_interior(s.rhs(None, lid_dirichlet(m)))
    _, info = fgmres(lambda v: s.K @ v, b, make(s), tol=1e-8, maxit=250, restart=50)
    return np.array(info["residuals"]) / np.linalg.norm(b), info


def test_two_field_pcd_stagnates_and_lsc_converges():
    """Cavity, nu = 1/100, exact pieces, GMRES(50).  Measured: M_1 1.0 ->
    2.3e-3 in 400 iterations on 32^2; M_2 1.0 -> 0.043 in 20, then 3.1e-3
    after 400 (stagnation from ~0.1 at 16^2, ~0.03 at 32^2); M_3 1e-8 in 51
    iterations at 16^2 and 36 at 32^2."""
    r2 = {}
    for n in (16, 32):
        r1, _ = _history(n, m1)
        assert r1[100] > 1e-2 and r1[250] > 1e-3      # ~ 50 iterations per decade or slower
        r = r2[n] = _history(n, OseenM2)[0]
        assert r[20] < 0.5 * r1[20]                    # fast first phase
        assert r[250] > 1e-3                           # then stagnation
        assert r[250] > 0.02 * r[40]                   # less than two decades in 210 iterations
    assert r2[32][30] < r2[16][30]                     # onset delayed on the finer mesh
    for n in (16, 32):
        r3, info = _history(n, OseenM3)
        assert info["converged"] and info["iterations"] <= 80
