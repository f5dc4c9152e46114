"""Pins of the pressure-mass solve by elimination of the P0 block (Sec. 2.3
variant, oracle.precond.schur_Sk / MQSchurGMG / Q1GMG)."""
import numpy as np
import pytest

from oracle.assemble import Mesh, System
from oracle.fem import gauss01
from oracle.precond import MQExact, MQSchurGMG, Q1GMG, gmg_levels, q1_prolongation, schur_Sk


def _distance_from_element_means(mesh, p):
    """sum_T int_T (p_h - mean_T p_h)^2 by tensor Gauss quadrature of the
    bilinear p_h (independent of the assembled matrices)."""
    xg, wg = gauss01(3)
    h = mesh.h
    n = mesh.n
    P = p.reshape(n + 1, n + 1)
    tot = 0.0
    for ey in range(n):
        for ex in range(n):
            v = np.empty((3, 3))
            for j, t in enumerate(xg):
                for i, s in enumerate(xg):
                    v[j, i] = (P[ey, ex] * (1 - s) * (1 - t) + P[ey, ex + 1] * s * (1 - t) +
                               P[ey + 1, ex] * (1 - s) * t + P[ey + 1, ex + 1] * s * t)
            W = np.outer(wg, wg)
            mean = float((W * v).sum())
            tot += h * h * float((W * (v - mean) ** 2).sum())
    return tot


@pytest.mark.parametrize("n", [2, 5])
def test_schur_quadratic_form_is_distance_from_element_means(n):
    m = Mesh(n, 0.0, 2.0, 0.0, 2.0)
    S = schur_Sk(m)
    p = np.random.default_rng(n).uniform(-1, 1, m.nk)
    assert abs(p @ (S @ p) - _distance_from_element_means(m, p)) < 1e-12 * max(1.0, p @ p)
    assert np.abs(S @ np.ones(m.nk)).max() < 1e-14


def test_schur_element_form():
    """On one element S_k = (h^2/144) [[7,-1,-5,-1],...] in counter-clockwise
    vertex order (eigenvalues 0, 4, 12, 12 times h^2/144)."""
    m = Mesh(1, 0.0, 3.0, 0.0, 3.0)
    S = schur_Sk(m).toarray()
    h2 = m.h ** 2
    ccw = [0, 1, 3, 2]           # (0,0), (1,0), (1,1), (0,1) in the x-fastest node order
    ref = np.array([[7, -1, -5, -1], [-1, 7, -1, -5], [-5, -1, 7, -1], [-1, -5, -1, 7]]) * h2 / 144
    assert np.allclose(S[np.ix_(ccw, ccw)], ref, atol=1e-14)


def test_elimination_with_exact_schur_solve_is_the_pseudo_inverse():
    """With S_k^+ exact the block elimination gives M_Q^+ r (compared with the
    bordered exact solve) for a consistent right-hand side."""
    n = 4
    m = Mesh(n)
    s = System(m)
    Q = MQSchurGMG(m, s.MQ)
    S = schur_Sk(m).toarray()
    Sp = np.linalg.pinv(S)
    Q.gmg = lambda r: Sp @ (r - r.mean())
    r = np.random.default_rng(1).uniform(-1, 1, m.nk + m.n0)
    assert np.allclose(Q(r), MQExact(m, s.MQ)(Q.project(r)), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("n", [32, 64])
def test_schur_multigrid_contracts_mesh_independently(n):
    """The V-cycle as a stationary iteration for S_k x = b (mean-zero b)
    reduces the residual by an h-independent factor per cycle."""
    m = Mesh(n)
    ns = gmg_levels(n, 4)
    meshes = [Mesh(k) for k in ns]
    ops = [schur_Sk(mm) * (m.h / mm.h) ** 2 for mm in meshes]
    G = Q1GMG(meshes, ops)
    S = ops[0]
    b = np.random.default_rng(3).uniform(-1, 1, m.nk)
    b -= b.mean()
    x = np.zeros_like(b)
    errs = []
    for _ in range(6):
        x = x + G(b - S @ x)
        errs.append(np.linalg.norm(b - S @ x))
    rate = (errs[-1] / errs[1]) ** (1 / 4)
    assert rate < 0.35
