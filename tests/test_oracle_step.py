"""Pins of the step-domain oracle (Sec. 3, the inflow-outflow example)
against facts fixed by the mathematics rather than by the oracle itself:

* Poiseuille flow u = (4y(1-y), 0), p = 8 nu (L - x) solves Stokes, and
  Oseen with that wind, in the channel with the natural outflow condition;
  it lies in Q2 x Q1, so the discrete solution equals it to rounding (a
  wrong sign of B, a missing viscosity, a Dirichlet outflow or a shifted
  pressure level all break it);
* the P0 rows of B make every element conserve mass, so the volume flux
  through every vertical grid line equals the inflow flux 2/3 (a dropped or
  mis-signed P0 block, a wrong wall condition or a wrong node numbering
  breaks it);
* null(K) is exactly span{[0; k]} with an outflow boundary (dense rank);
* nested Q2 and Q1 spaces: the Galerkin products of the transfers reproduce
  the coarse Laplacian and Q1 mass;
* the inflow term of F_1 sums to the inflow flux, and without it stage I
  stalls while with it it converges (the reading of the PCD boundary
  treatment)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.assemble import System, laplacian, q1_mass, frame_null_vector
from oracle.precond import OseenM1
from oracle.step import (StepMesh, inflow_dirichlet, poiseuille, direct_solve, stokes_start, picard,
                         line_fluxes, q2_prolongation, q1_prolongation, step_levels, velocity_gmg,
                         PCDStage1, two_stage, MQChebSGS, f1_inflow_term, step_f1, pressure_laplacian)

NU = 1.0 / 50


@pytest.mark.parametrize("m", [1, 2, 4])
@pytest.mark.parametrize("oseen", [False, True])
def test_channel_reproduces_poiseuille_flow(m, oseen):
    M = StepMesh(m, channel=True)
    ex = poiseuille(M, NU)
    S = System(M, nu=NU, wind=ex[: 2 * M.nv] if oseen else None)
    x = direct_solve(S, S.rhs(None, inflow_dirichlet(M)))
    assert np.abs(x - ex).max() < 1e-12


@pytest.mark.parametrize("m", [2, 4])
def test_step_fluxes_equal_the_inflow_flux_on_every_line(m):
    M = StepMesh(m)
    x = stokes_start(M, NU)
    f = line_fluxes(M, x)
    assert np.abs(f - 2.0 / 3.0).max() < 1e-13
    # an Oseen step with that wind conserves mass as well
    S = System(M, nu=NU, wind=x[: 2 * M.nv])
    y = direct_solve(S, S.rhs(None, inflow_dirichlet(M)))
    assert np.abs(line_fluxes(M, y) - 2.0 / 3.0).max() < 1e-13
    # and the velocity differs from the Stokes one (the convection is there)
    assert np.abs(y[: 2 * M.nv] - x[: 2 * M.nv]).max() > 1e-3


def test_null_space_is_one_dimensional():
    M = StepMesh(2)
    S = System(M, nu=NU)
    K = S.K.toarray()
    s = np.linalg.svd(K, compute_uv=False)
    assert s[-1] < 1e-12 * s[0] and s[-2] > 1e-8 * s[0]
    z = np.concatenate([np.zeros(S.nI), frame_null_vector(M)])
    assert np.abs(K @ z).max() < 1e-13


def test_mesh_counts():
    # the step at m: the (12m+1)(4m+1) half-grid nodes of the bounding box
    # minus the 2m x 2m with x < 0 and y < 0 (the closed step corner region
    # touches no element); Q1 likewise with m x m
    for m in (1, 2, 3, 4):
        M = StepMesh(m)
        assert M.nv == (12 * m + 1) * (4 * m + 1) - 4 * m * m
        assert M.nk == (6 * m + 1) * (2 * m + 1) - m * m
        assert M.n0 == 11 * m * m
        # Dirichlet: everything on the boundary but the 4m - 1 open outflow nodes
        assert M.outflow_q2().sum() == 4 * m - 1


def test_galerkin_identities_of_the_transfers():
    f, c = StepMesh(4), StepMesh(2)
    P = q2_prolongation(f, c)
    If = np.flatnonzero(~f.boundary_q2())
    Ic = np.flatnonzero(~c.boundary_q2())
    Pi = P[If][:, Ic]
    Af = laplacian(f)[If][:, If]
    Ac = laplacian(c)[Ic][:, Ic]
    assert abs(Pi.T @ Af @ Pi - Ac).max() < 1e-12
    Pq = q1_prolongation(f, c)
    assert abs(Pq.T @ q1_mass(f) @ Pq - q1_mass(c)).max() < 1e-15
    # interpolation reproduces quadratics / bilinears exactly
    X, Y = f.q2_coords()
    Xc, Yc = c.q2_coords()
    g = lambda x, y: 1 + x - 2 * y + x * y + 0.5 * x * x - y * y
    assert np.abs(P @ g(Xc, Yc) - g(X, Y)).max() < 1e-13
    assert step_levels(16, 4) == [16, 8, 4] and step_levels(12, 4) == [12, 6, 3]


def test_inflow_term_of_f1_sums_to_the_inflow_flux():
    M = StepMesh(4)
    x = stokes_start(M, NU)
    T = f1_inflow_term(M, x[: 2 * M.nv])
    assert abs(T.sum() - 2.0 / 3.0) < 1e-13
    S = System(M, nu=NU, wind=x[: 2 * M.nv])
    F1 = step_f1(S, robin=False)
    assert np.abs(F1 @ np.ones(M.nk)).max() < 1e-13      # natural F_1 annihilates constants
    assert np.abs(pressure_laplacian(M) @ np.ones(M.nk)).max() > 1e-3   # A_p does not


def test_stage1_needs_the_inflow_term():
    M = StepMesh(4)
    x = stokes_start(M, NU)
    S = System(M, nu=NU, wind=x[: 2 * M.nv])
    b = S.rhs(None, inflow_dirichlet(M))
    _, info = two_stage(S, b, eta=1e-6, stage1_prec=PCDStage1(S, robin=True), maxit=300)
    assert info["stage1"]["iterations"] <= 40
    _, info = two_stage(S, b, eta=1e-6, stage1_prec=PCDStage1(S, robin=False), maxit=300)
    assert info["stage1"]["iterations"] >= 200


def test_two_stage_with_inexact_pieces_reaches_the_direct_solution():
    M = StepMesh(8)
    x = picard(M, NU, 1)[-1]
    S = System(M, nu=NU, wind=x[: 2 * M.nv])
    b = S.rhs(None, inflow_dirichlet(M))
    xd = direct_solve(S, b)
    vel, cyc = velocity_gmg(S)
    assert [mm.m for mm in cyc.meshes] == [8, 4]
    P1 = PCDStage1(S, velocity_solve=vel, inexact=True)
    P2 = OseenM1(S, velocity_solve=vel, mq=MQChebSGS(S))
    y, info = two_stage(S, b, eta=1e-10, stage1_prec=P1, stage2_prec=P2, maxit=800)
    assert np.linalg.norm(y - xd) / np.linalg.norm(xd) < 1e-8
    assert info["stage1"]["iterations"] < 60
