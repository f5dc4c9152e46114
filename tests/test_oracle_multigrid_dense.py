"""Pins of the oracle's multigrid cycles as whole operators.

Each cycle of the oracle is written recursively (smooth, restrict the
residual, recurse, prolongate, smooth).  Here the same cycle is rebuilt on
small meshes from dense matrices with the textbook formula for one V-cycle
started from zero,

    B_l = M_l + (I - M_l A_l) C_l (I - A_l M_l) + (I - M_l A_l) M_l,
    C_l = P_l B_{l+1} P_l^T,       B_coarsest = A_coarsest^{-1} (or A^+),

where M_l is the smoother's approximate inverse after the given number of
steps from zero: for a polynomial smoother with error polynomial p (p(0) = 1)
in X = D^{-1} A, M = q(X) D^{-1} with q(t) = (1 - p(t)) / t, evaluated here
from the polynomial's power-basis coefficients.  The Chebyshev error
polynomial is T_d((theta - t)/delta) / T_d(theta/delta) on [lo, hi]
(theta, delta the centre and half width); damped Jacobi with weight w and s
sweeps has p(t) = (1 - w t)^s.  Where the hierarchy is re-discretised, the
coarse operators of the formula are the Galerkin products P^T A P, so the test
also checks that re-discretisation equals Galerkin coarsening.

A dropped smoothing step, a wrong transfer, a missing coarse correction or a
mis-scaled coarse operator changes B by O(1), far above the 1e-10 bound."""
import numpy as np
import numpy.polynomial.chebyshev as C
import numpy.polynomial.polynomial as Pn
import pytest

from oracle import precond as pc
from oracle.assemble import Mesh, System, frame_null_vector, laplacian, recirculating_wind


def _cheb_error_poly(lo, hi, d):
    """Power-basis coefficients of T_d((theta - t)/delta) / T_d(theta/delta)."""
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    Td = C.cheb2poly([0] * d + [1])                     # T_d in power basis of s
    # substitute s = (theta - t)/delta
    s_of_t = np.array([theta / delta, -1.0 / delta])
    out = np.zeros(1)
    power = np.ones(1)
    for c in Td:
        out = Pn.polyadd(out, c * power)
        power = Pn.polymul(power, s_of_t)
    return out / Pn.polyval(0.0, out)


def _jacobi_error_poly(w, s):
    return Pn.polypow([1.0, -w], s)


def _smoother_inverse(A, p):
    """M = q(X) D^{-1}, X = D^{-1} A, q = (1 - p)/t."""
    q = -np.asarray(p[1:], dtype=np.float64)            # (1 - p(t)) / t
    dinv = 1.0 / np.diag(A)
    X = dinv[:, None] * A
    Q = np.zeros_like(A)
    for c in q[::-1]:                                   # Horner
        Q = Q @ X + c * np.eye(A.shape[0])
    return Q * dinv[None, :]


def _vcycle_dense(As, Ps, Ms, coarse_inv):
    B = coarse_inv
    for l in range(len(As) - 2, -1, -1):
        A, M = As[l], Ms[l]
        I = np.eye(A.shape[0])
        Cl = Ps[l] @ B @ Ps[l].T
        B = M + (I - M @ A) @ Cl @ (I - A @ M) + (I - M @ A) @ M
    return B


def _columns(op, n):
    return np.column_stack([op(e) for e in np.eye(n)])


def _galerkin_hierarchy(A0, Ps):
    As = [A0]
    for P in Ps:
        As.append(P.T @ As[-1] @ P)
    return As


@pytest.mark.parametrize("degree", [1, 2, 3])
def test_stokes_gmg_is_the_chebyshev_vcycle(degree):
    m = Mesh(16)
    g = pc.GMG(m, laplacian, coarse_n=4, degree=degree)
    assert g.ns == [16, 8, 4]
    Ps = [P.toarray() for P in g.P]
    As = _galerkin_hierarchy(g.A[0].toarray(), Ps)
    for l in range(1, len(As)):
        assert np.abs(As[l] - g.A[l].toarray()).max() < 1e-12 * np.abs(As[l]).max()
    Ms = [_smoother_inverse(As[l], _cheb_error_poly(g.lo_frac * g.lam[l], g.hi_frac * g.lam[l], degree))
          for l in range(len(As) - 1)]
    B = _vcycle_dense(As, Ps, Ms, np.linalg.inv(As[-1]))
    V = _columns(lambda v: g.vcycle(0, v), As[0].shape[0])
    assert np.abs(V - B).max() < 1e-10 * np.abs(B).max()


def test_oseen_velocity_multigrid_is_the_damped_jacobi_vcycle():
    m = Mesh(16, -1, 1, -1, 1)
    s = System(m, nu=1 / 20, wind=recirculating_wind(m))
    _, g = pc.oseen_velocity_gmg(s, coarse_n=4, omega=0.7, sweeps=2)
    assert g.ns == [16, 8, 4]
    Ps = [P.toarray() for P in g.P]
    As = _galerkin_hierarchy(g.A[0].toarray(), Ps)
    for l in range(1, len(As)):
        # injected wind = the coarse interpolant of this Q2 wind: Galerkin
        assert np.abs(As[l] - g.A[l].toarray()).max() < 1e-12 * np.abs(As[l]).max()
    Ms = [_smoother_inverse(As[l], _jacobi_error_poly(0.7, 2)) for l in range(len(As) - 1)]
    B = _vcycle_dense(As, Ps, Ms, np.linalg.inv(As[-1]))
    V = _columns(lambda v: g.vcycle(0, v), As[0].shape[0])
    assert np.abs(V - B).max() < 1e-10 * np.abs(B).max()


def _singular_cycle_dense(g):
    """Q1 cycles for operators whose null space is the constants: the level
    operators are the cycle's own (A_p and S_k are re-discretised by design,
    not Galerkin); the coarsest solve is the pseudo-inverse; input and output
    are projected onto mean-zero vectors."""
    As = [A.toarray() for A in g.A]
    Ps = [P.toarray() for P in g.P]
    Ms = [_smoother_inverse(As[l], _cheb_error_poly(g.lo_frac * g.lam[l], g.hi_frac * g.lam[l], g.degree))
          for l in range(len(As) - 1)]
    B = _vcycle_dense(As, Ps, Ms, np.linalg.pinv(As[-1]))
    n = As[0].shape[0]
    Pi = np.eye(n) - 1.0 / n
    return Pi @ B @ Pi


def test_pressure_laplacian_multigrid_is_the_chebyshev_vcycle():
    g = pc.ApGMG(Mesh(16, -1, 1, -1, 1), coarse_n=4)
    assert g.ns == [16, 8, 4]
    B = _singular_cycle_dense(g)
    V = _columns(g, g.A[0].shape[0])
    assert np.abs(V - B).max() < 1e-10 * np.abs(B).max()


def test_schur_multigrid_and_p0_elimination_are_the_block_factorisation():
    """MQSchurGMG: z_k = G (r_k - R^T Q_0^{-1} r_0), z_0 = Q_0^{-1}(r_0 - R z_k)
    with G the dense Q1 cycle for S_k, both ends projected onto k^perp."""
    m = Mesh(16)
    s = System(m)
    op = pc.MQSchurGMG(m, s.MQ, coarse_n=4)
    G = _singular_cycle_dense(op.gmg)
    M = s.MQ.toarray()
    nk = m.nk
    R = M[nk:, :nk]
    Q0i = np.diag(1.0 / np.diag(M[nk:, nk:]))
    T = np.block([[G, -G @ R.T @ Q0i],
                  [-Q0i @ R @ G, Q0i + Q0i @ R @ G @ R.T @ Q0i]])
    k = frame_null_vector(m)
    Pk = np.eye(m.np_) - np.outer(k, k) / (k @ k)
    ref = Pk @ T @ Pk
    Z = _columns(op, m.np_)
    assert np.abs(Z - ref).max() < 1e-10 * np.abs(ref).max()


def test_dense_formula_detects_a_dropped_post_smoothing():
    """The formula is sharp enough to tell the cycle from a variant without
    post-smoothing (a plausible slip in a recursive cycle)."""
    m = Mesh(8)
    g = pc.GMG(m, laplacian, coarse_n=4)
    Ps = [P.toarray() for P in g.P]
    As = _galerkin_hierarchy(g.A[0].toarray(), Ps)
    Ms = [_smoother_inverse(As[0], _cheb_error_poly(0.3 * g.lam[0], 1.1 * g.lam[0], 2))]
    B = _vcycle_dense(As, Ps, Ms, np.linalg.inv(As[-1]))

    def pre_only(r):
        x = g.smooth(0, r, np.zeros_like(r))
        return x + g.P[0] @ g.coarse_lu.solve(g.P[0].T @ (r - g.A[0] @ x))
    V = _columns(pre_only, As[0].shape[0])
    assert np.abs(V - B).max() > 1e-3 * np.abs(B).max()


def test_stabilised_oseen_multigrid_is_the_damped_jacobi_vcycle():
    """With a Peclet cap the level operators are nu_l A_l + N_l with A_l, N_l
    the Galerkin products of the finest Laplacian and convection and
    nu_l = max(nu, max|w| h_l / (2 peclet_max)); the cycle is the textbook
    damped-Jacobi V-cycle on those operators."""
    from oracle.assemble import convection
    m = Mesh(16, -1, 1, -1, 1)
    w = recirculating_wind(m)
    s = System(m, nu=1e-3, wind=w)
    _, g = pc.oseen_velocity_gmg(s, coarse_n=4, omega=0.7, sweeps=2, peclet_max=4.0)
    assert g.ns == [16, 8, 4]
    I0 = g.I[0]
    A = laplacian(m).toarray()[np.ix_(I0, I0)]
    N = convection(m, w).toarray()[np.ix_(I0, I0)]
    Ps = [P.toarray() for P in g.P]
    wmax = 2.0                                   # max |w| of the recirculating wind on [-1,1]^2
    assert abs(pc.wind_speed_max(w, m) - wmax) < 1e-12
    As = []
    for l, k in enumerate(g.ns):
        h = 2.0 / k
        nul = max(1e-3, wmax * h / 8.0)
        assert nul == pc.level_viscosity(1e-3, h, wmax, 4.0)
        As.append(nul * A + N)
        assert np.abs(As[l] - g.A[l].toarray()).max() < 1e-12 * np.abs(As[l]).max()
        if l + 1 < len(g.ns):
            A = Ps[l].T @ A @ Ps[l]
            N = Ps[l].T @ N @ Ps[l]
    Ms = [_smoother_inverse(As[l], _jacobi_error_poly(0.7, 2)) for l in range(len(As) - 1)]
    B = _vcycle_dense(As, Ps, Ms, np.linalg.inv(As[-1]))
    V = _columns(lambda v: g.vcycle(0, v), As[0].shape[0])
    assert np.abs(V - B).max() < 1e-10 * np.abs(B).max()


def test_stabilised_cycle_contracts_where_the_plain_cycle_diverges():
    """nu = 1/1000 on 16^2 (element Peclet number 125): the plain damped-Jacobi
    cycle amplifies the error by orders of magnitude, the Peclet-capped one is
    a contraction for its own finest operator and leaves the spectrum of the
    preconditioned F in the right half-plane (GMRES on F B converges)."""
    m = Mesh(16, -1, 1, -1, 1)
    s = System(m, nu=1e-3, wind=recirculating_wind(m))
    I0 = np.flatnonzero(~m.boundary_q2())
    F = s.F_s[I0][:, I0].toarray()
    E = np.eye(F.shape[0])
    _, gp = pc.oseen_velocity_gmg(s, coarse_n=4)
    Bp = _columns(lambda v: gp.vcycle(0, v), F.shape[0])
    assert np.abs(np.linalg.eigvals(E - Bp @ F)).max() > 10.0
    _, gs = pc.oseen_velocity_gmg(s, coarse_n=4, peclet_max=4.0)
    Bs = _columns(lambda v: gs.vcycle(0, v), F.shape[0])
    Fs = gs.A[0].toarray()
    assert np.abs(np.linalg.eigvals(E - Bs @ Fs)).max() < 0.8
    assert np.linalg.eigvals(F @ Bs).real.min() > 0.0
