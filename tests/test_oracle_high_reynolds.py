"""The two-stage method itself at nu = 1/1000 (Sec. 3 Oseen problem, Sec.
3.1 two-stage algorithm) on the unstabilised Galerkin discretisation, with
exact pieces (direct F, Q_1 and A_p solves in PCD; direct F and bordered M_Q
solves in M_1), restarted GMRES(50): the record behind the statement that
these meshes need more than 4096 iterations per stage, whatever the
preconditioner's inexact pieces do.

Measured with the env-gated test below (ETH_LONG_ORACLE=1; about 40 min per
mesh on one core):
  64^2  (element Peclet 31):   stage I 4096 its -> 2.55e-5 (target 1e-5),
                               stage II 4096 its -> 2.41e-5 (target 1e-6);
  128^2 (element Peclet 15.6): stage I reaches 1e-5 after 2376 its,
                               stage II 4096 its -> 7.8e-6, flat at ~1e-5.
The quick test keeps the qualitative record in the regular suite: at
nu = 1/100 the same exact pieces converge in a few dozen iterations per
stage, at nu = 1/1000 stage I is still above 1e-2 after 150."""
import os

import numpy as np
import pytest

from oracle.assemble import Mesh, System, lid_dirichlet, recirculating_wind
from oracle.precond import two_stage


def _run(n, nu, maxit):
    m = Mesh(n, -1, 1, -1, 1)
    s = System(m, nu=nu, wind=recirculating_wind(m))
    b = s.rhs(None, lid_dirichlet(m, 1.0, 0))
    _, info = two_stage(s, b, eta=1e-6, c=10.0, restart=50, maxit=maxit)
    bn = info["bnorm"]
    r1 = np.array(info["stage1"]["residuals"]) / bn
    r2 = np.array(info["stage2"]["residuals"]) / bn
    return info, r1, r2


def test_exact_pieces_stall_at_high_reynolds_but_not_at_re_200():
    info, r1, r2 = _run(64, 1e-2, 400)
    assert info["stage1"]["converged"] and info["stage2"]["converged"]
    assert info["iterations"] < 150
    info, r1, r2 = _run(64, 1e-3, 150)
    assert not info["stage1"]["converged"]
    assert r1[-1] > 1e-2
    assert not info["stage2"]["converged"]


@pytest.mark.slow
@pytest.mark.skipif(os.environ.get("ETH_LONG_ORACLE") != "1",
                    reason="about 40 min per mesh; set ETH_LONG_ORACLE=1")
@pytest.mark.parametrize("n", [64, 128])
def test_exact_pieces_need_more_than_4096_iterations(n):
    maxit = int(os.environ.get("ETH_LONG_ORACLE_MAXIT", "4096"))
    info, r1, r2 = _run(n, 1e-3, maxit)
    print(f"n={n}: stage I {len(r1) - 1} its -> {r1[-1]:.3e}; stage II {len(r2) - 1} its -> {r2[-1]:.3e}")
    assert not info["stage2"]["converged"]
