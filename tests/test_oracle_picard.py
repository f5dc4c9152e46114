"""Pins of the Picard oracle (oracle/picard.py) and the regularised lid.

* the regularised lid equals lid_u (1 - xi^4) at the top nodes and zero on the
  other walls (closed form);
* at a low Reynolds number the fixed-point map contracts and its limit makes
  the discrete steady Navier-Stokes residual vanish, with the wind evaluated
  at the full velocity of the limit itself (so a wind that drops the
  Dirichlet values, or one taken from another vector, fails);
* convection is quadratic in the velocity: for a lid speed eps the Picard
  iterate differs from the Stokes solution by O(eps^2) relative to eps;
* a zero lid keeps every iterate zero.
"""
import numpy as np
import pytest

from oracle.assemble import Mesh, System, lid_dirichlet
from oracle.picard import ns_residual, picard, stokes_start


def test_regularised_lid_closed_form():
    m = Mesh(8, -1.0, 1.0, -1.0, 1.0)
    uD = lid_dirichlet(m, 0.7, corner_mode=2)
    X, Y = m.q2_coords()
    top = np.isclose(Y, 1.0)
    assert np.allclose(uD[: m.nv][top], 0.7 * (1.0 - X[top] ** 4), rtol=0, atol=1e-15)
    assert np.all(uD[: m.nv][~top] == 0.0)
    assert np.all(uD[m.nv:] == 0.0)
    # on another square the wall coordinate is mapped to [-1, 1]
    m2 = Mesh(4, 0.0, 2.0, 0.0, 2.0)
    u2 = lid_dirichlet(m2, 1.0, corner_mode=2)
    X2, Y2 = m2.q2_coords()
    t2 = np.isclose(Y2, 2.0)
    assert np.allclose(u2[: m2.nv][t2], 1.0 - (X2[t2] - 1.0) ** 4, atol=1e-15)


def test_picard_converges_to_a_navier_stokes_root():
    m = Mesh(4, -1.0, 1.0, -1.0, 1.0)
    nu = 0.5
    xs = picard(m, nu, 25)
    d = [np.linalg.norm(xs[k + 1][: 2 * m.nv] - xs[k][: 2 * m.nv]) for k in range(len(xs) - 1)]
    assert d[-1] < 1e-13 * np.linalg.norm(xs[-1][: 2 * m.nv])
    assert all(d[k + 1] < 0.5 * d[k] for k in range(6))
    uD = lid_dirichlet(m, 1.0, 2)
    b = System(m, nu=nu).rhs(None, uD)
    r = ns_residual(m, nu, xs[-1], uD)
    assert np.linalg.norm(r) < 1e-11 * np.linalg.norm(b)
    # the same vector with the Dirichlet values left out of the wind is no root
    x_bad = xs[-1].copy()
    x_bad[: 2 * m.nv][System(m).vel_bnd] = 0.0
    S = System(m, nu=nu, wind=x_bad[: 2 * m.nv])
    r_bad = S.apply_full(xs[-1]) - S.rhs(None, uD)
    r_bad[: 2 * m.nv][S.vel_bnd] = 0.0
    assert np.linalg.norm(r_bad) > 1e-4 * np.linalg.norm(b)
    # the Stokes start is no root either (the flow convects)
    assert np.linalg.norm(ns_residual(m, nu, xs[0], uD)) > 1e-3 * np.linalg.norm(b)


def test_convection_is_quadratic_in_the_lid_speed():
    m = Mesh(4, -1.0, 1.0, -1.0, 1.0)
    ratios = []
    for eps in (1e-2, 1e-3):
        xs = picard(m, 0.01, 1, lid_u=eps)
        du = np.linalg.norm(xs[1][: 2 * m.nv] - xs[0][: 2 * m.nv]) / eps
        ratios.append(du / eps)
    assert ratios[0] > 0
    assert ratios[1] == pytest.approx(ratios[0], rel=0.05)


def test_zero_lid_stays_zero():
    m = Mesh(4, -1.0, 1.0, -1.0, 1.0)
    xs = picard(m, 0.01, 3, lid_u=0.0)
    assert all(np.all(x == 0.0) for x in xs)


def test_stokes_start_velocity_independent_of_viscosity():
    m = Mesh(4, -1.0, 1.0, -1.0, 1.0)
    a = stokes_start(m, 1.0)
    b = stokes_start(m, 0.01)
    o = 2 * m.nv
    assert np.allclose(a[:o], b[:o], atol=1e-12)
    assert np.allclose(0.01 * a[o:], b[o:], atol=1e-12)
