"""Pins of the oracle's discrete adjoint gradients by central finite
differences (J is quadratic in the forcing, so the FD is exact up to
rounding; in the viscosity it is smooth)."""
import numpy as np
import pytest

from oracle.assemble import Mesh, System, lid_dirichlet, recirculating_wind
from oracle.direct import BorderedLU, misfit, adjoint_gradients
from paper_2303_10233_amd.workloads import gaussian_bumps


def _setup(oseen, n=4):
    if oseen:
        m = Mesh(n, -1, 1, -1, 1)
        w = recirculating_wind(m)
        nu = 1 / 100
        ft = gaussian_bumps(n, 5000, -1, 1, -1, 1)
    else:
        m = Mesh(n)
        w = None
        nu = 1.0
        ft = gaussian_bumps(n, 5000)
    uB = lid_dirichlet(m)
    return m, w, nu, ft, uB


def _J(m, w, nu, f, uB, ut):
    s = System(m, nu=nu, wind=w)
    x = BorderedLU(s).solve(s.rhs(f, uB))
    return misfit(s, x, ut)


@pytest.mark.parametrize("oseen", [False, True])
def test_adjoint_gradients_match_central_fd(oseen):
    m, w, nu, ft, uB = _setup(oseen)
    s = System(m, nu=nu, wind=w)
    ut = BorderedLU(s).solve(s.rhs(ft, uB))
    # evaluation point: a second bump forcing (at f = 0 the Stokes velocity
    # does not depend on nu, so dJ/dnu would vanish identically)
    f0 = 0.5 * gaussian_bumps(m.n, 4999, m.x0, m.x1, m.y0, m.y1)
    x = BorderedLU(s).solve(s.rhs(f0, uB))
    _, dJdf, dJdnu = adjoint_gradients(s, x, ut)
    eps = 1e-6
    rng = np.random.default_rng(0)
    idx = rng.choice(2 * m.nv, 24, replace=False)
    for i in idx:
        e = np.zeros(2 * m.nv)
        e[i] = eps
        fd = (_J(m, w, nu, f0 + e, uB, ut) - _J(m, w, nu, f0 - e, uB, ut)) / (2 * eps)
        assert abs(fd - dJdf[i]) <= 1e-7 * np.abs(dJdf).max() + 1e-12
    fdnu = (_J(m, w, nu * (1 + eps), f0, uB, ut) - _J(m, w, nu * (1 - eps), f0, uB, ut)) / (2 * eps * nu)
    assert abs(fdnu - dJdnu) <= 1e-6 * abs(dJdnu)
