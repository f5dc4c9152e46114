"""Oracle for the Picard (fixed-point) linearisation of the steady
Navier-Stokes equations that produces the Oseen systems of Sec. 3.

Test infrastructure (imported only by tests/, smoke() and the CPU baseline).

The Oseen operator of eq:oseen-system has F = nu A + N(w_h), where the wind
w_h is the velocity of the most recent nonlinear iterate (the text after
eq:generic-conv-diff).  The enclosed-flow example of Sec. 3 takes the system
that results after five such fixed-point steps started from the Stokes
solution with the same boundary data.  Every step here is an exact (sparse
direct) solve:

    u^(0) = Stokes solution,   u^(k) = Oseen solve with wind w = u^(k-1),

where the wind is the full nodal Q2 velocity of the iterate, Dirichlet values
included.  `ns_residual` is the discrete steady Navier-Stokes residual
R(x) = K(u) x - b(u) with the wind equal to the velocity of x itself: zero at
a fixed point of the iteration.
"""
import numpy as np

from .assemble import System, lid_dirichlet
from .direct import direct_solve


def stokes_start(mesh, nu, lid_u=1.0, corner_mode=2, f_nodal=None):
    """u^(0): the Stokes solution with the cavity boundary data."""
    uD = lid_dirichlet(mesh, lid_u, corner_mode)
    S = System(mesh, nu=nu)
    return direct_solve(S, S.rhs(f_nodal, uD))


def picard_step(mesh, nu, x, uD, f_nodal=None):
    """One fixed-point step: wind = the velocity of x (all 2 n_v nodal values)."""
    S = System(mesh, nu=nu, wind=x[: 2 * mesh.nv])
    return direct_solve(S, S.rhs(f_nodal, uD))


def picard(mesh, nu, steps, lid_u=1.0, corner_mode=2, f_nodal=None, x0=None):
    """[u^(0), u^(1), ..., u^(steps)] as full-layout vectors (pressure
    canonicalised); x0 replaces the Stokes start when given."""
    uD = lid_dirichlet(mesh, lid_u, corner_mode)
    x = stokes_start(mesh, nu, lid_u, corner_mode, f_nodal) if x0 is None else np.array(x0, float)
    out = [x]
    for _ in range(steps):
        x = picard_step(mesh, nu, x, uD, f_nodal)
        out.append(x)
    return out


def ns_residual(mesh, nu, x, uD, f_nodal=None):
    """R(x) on the interior velocity and pressure rows (boundary rows zero)."""
    S = System(mesh, nu=nu, wind=x[: 2 * mesh.nv])
    r = S.apply_full(x) - S.rhs(f_nodal, uD)
    r[: 2 * mesh.nv][S.vel_bnd] = 0.0
    return r
