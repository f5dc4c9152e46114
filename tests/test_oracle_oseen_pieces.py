"""Pins of the oracle's inexact Oseen preconditioner pieces (the algorithms
the GPU path implements): transfers reproduce the functions they must,
the multigrid cycles are convergent stationary iterations, the Q1 mass
Chebyshev solve converges to Q_1^{-1}, and the two-stage PCD algorithm with
these pieces reaches the direct solution."""
import numpy as np
import pytest

from oracle.assemble import Mesh, System, lid_dirichlet, recirculating_wind, q1_mass
from oracle.direct import direct_solve, canonicalize, rel_err
from oracle import precond as pc


def test_q1_prolongation_reproduces_bilinear():
    fine, coarse = Mesh(8, -1, 1, -1, 1), Mesh(4, -1, 1, -1, 1)
    P = pc.q1_prolongation(fine, coarse)
    f = lambda x, y: 1.5 + 2 * x - y + 0.7 * x * y
    Xc, Yc = coarse.q1_coords()
    Xf, Yf = fine.q1_coords()
    assert np.abs(P @ f(Xc, Yc) - f(Xf, Yf)).max() < 1e-14


def test_injection_of_a_q2_field():
    fine, coarse = Mesh(16, -1, 1, -1, 1), Mesh(4, -1, 1, -1, 1)
    assert np.abs(pc.inject_q2(recirculating_wind(fine), fine, coarse) - recirculating_wind(coarse)).max() == 0.0


def _contraction(apply_inv, A, its=12, seed=0):
    e = np.random.default_rng(seed).standard_normal(A.shape[0])
    e -= e.mean() if A.shape[0] else 0
    nrm = [np.linalg.norm(e)]
    for _ in range(its):
        e = e - apply_inv(A @ e)
        nrm.append(np.linalg.norm(e))
    return (nrm[-1] / nrm[-5]) ** 0.25


def test_oseen_velocity_gmg_contracts():
    m = Mesh(64, -1, 1, -1, 1)
    s = System(m, nu=1 / 100, wind=recirculating_wind(m))
    _, g = pc.oseen_velocity_gmg(s)
    assert g.ns == [64, 32]
    assert _contraction(lambda r: g.vcycle(0, r), g.A[0]) < 0.5


def test_ap_gmg_contracts_and_is_exact_on_one_level():
    m = Mesh(32)
    g = pc.ApGMG(m)
    A = g.A[0]
    rho = _contraction(lambda r: g(r), A)
    assert rho < 0.3, rho
    # mean-zero output, A_p annihilates constants
    r = np.random.default_rng(2).standard_normal(A.shape[0])
    assert abs(g(r).mean()) < 1e-14
    g4 = pc.ApGMG(Mesh(4))
    r4 = np.random.default_rng(3).standard_normal(g4.A[0].shape[0])
    r4 -= r4.mean()
    np.testing.assert_allclose(g4(r4), np.linalg.pinv(g4.A[0].toarray()) @ r4, atol=1e-11)


def test_q1_chebyshev_converges_to_inverse():
    m = Mesh(16, -1, 1, -1, 1)
    s = System(m, nu=0.01, wind=recirculating_wind(m))
    vs, _ = pc.oseen_velocity_gmg(s, coarse_n=8)
    P = pc.PCDStage1Inexact(s, vs, q1_steps=40)
    r = np.random.default_rng(4).standard_normal(m.nk)
    ref = np.linalg.solve(q1_mass(m).toarray(), r)
    assert rel_err(P.q1_inv(r), ref) < 1e-10


def test_two_stage_with_inexact_pieces_reaches_direct_solution():
    # cell Peclet |w| h / (2 nu) = 1.25 on the finest level (Jacobi smoothing
    # of the unstabilised Galerkin F needs it to be O(1))
    n = 32
    m = Mesh(n, -1, 1, -1, 1)
    s = System(m, nu=1 / 20, wind=recirculating_wind(m))
    b = s.rhs(None, lid_dirichlet(m))
    vs, _ = pc.oseen_velocity_gmg(s, coarse_n=16)
    mq = pc.MQChebSGS(m, s.MQ, lo=0.01, steps=20)
    x, info = pc.two_stage(s, b, eta=1e-10, c=10.0, stage1_prec=pc.PCDStage1Inexact(s, vs),
                           stage2_prec=pc.OseenM1(s, velocity_solve=vs, mq=mq))
    assert info["stage2"]["converged"]
    assert rel_err(canonicalize(x, m), direct_solve(s, b)) < 1e-7
