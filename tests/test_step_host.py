"""The library's host assembly for the step domain (eth_step_host_layout,
eth_step_host_matrix: no GPU involved) against the oracle's: numbering,
Dirichlet set, K, M_Q, Q_1, F_1 with its inflow term, A_p, both
prolongations and the lifted right-hand side, on the step and the channel,
with a random wind (so that every convection coefficient matters)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle.assemble import System, q1_mass
from oracle.step import (StepMesh, inflow_dirichlet, step_f1, pressure_laplacian, q2_prolongation,
                         q1_prolongation)
from paper_2303_10233_amd.workloads import uniform_vector

eth = pytest.importorskip("paper_2303_10233_amd.eth")

NU = 0.02


def _mat(m, which, channel, wind):
    p, c, v, shape = eth.step_host_matrix(m, which, 5, channel, NU, wind)
    return sp.csr_matrix((v, c, p), shape=shape)


@pytest.mark.parametrize("channel", [False, True])
@pytest.mark.parametrize("m", [2, 4])
def test_host_assembly_matches_the_oracle(m, channel):
    M = StepMesh(m, channel=channel)
    lay = eth.step_host_layout(m, 5, channel)
    I, J = M.q2_IJ
    assert (lay["nv"], lay["nk"], lay["n0"], lay["N"]) == (M.nv, M.nk, M.n0, M.N)
    assert (lay["q2_ij"][:, 0] == I).all() and (lay["q2_ij"][:, 1] == J).all()
    Jk, Ik = np.nonzero(M.q1_active)
    assert (lay["q1_ij"][:, 0] == Ik).all() and (lay["q1_ij"][:, 1] == Jk).all()
    assert (lay["dirichlet"] == M.boundary_q2()).all()
    w = np.random.default_rng(m + 10 * channel).standard_normal(2 * M.nv)
    S = System(M, nu=NU, wind=w)
    # K on the full layout: the oracle's interior operator, Dirichlet rows and columns empty
    keep = np.concatenate([S.vI, np.arange(2 * M.nv, M.N)])
    Kref = np.zeros((M.N, M.N))
    Kref[np.ix_(keep, keep)] = S.K.toarray()
    K = _mat(m, eth.STEP_K, channel, w)
    assert np.abs(K.toarray() - Kref).max() < 1e-13
    assert abs(_mat(m, eth.STEP_MQ, channel, w) - S.MQ).max() < 1e-15
    assert abs(_mat(m, eth.STEP_Q1, channel, w) - q1_mass(M)).max() < 1e-15
    assert abs(_mat(m, eth.STEP_F1, channel, w) - step_f1(S)).max() < 1e-13
    assert abs(_mat(m, eth.STEP_AP, channel, w) - pressure_laplacian(M)).max() < 1e-12
    Mc = StepMesh(m // 2, channel=channel)
    P = q2_prolongation(M, Mc).toarray()
    P *= (~M.boundary_q2())[:, None] * (~Mc.boundary_q2())[None, :]
    assert np.abs(_mat(m, eth.STEP_P, channel, w).toarray() - P).max() == 0.0
    assert abs(_mat(m, eth.STEP_PQ, channel, w) - q1_prolongation(M, Mc)).max() == 0.0
    b = _mat(m, eth.STEP_RHS, channel, w).toarray().ravel()
    assert np.abs(b - S.rhs(None, inflow_dirichlet(M))).max() < 1e-13


def test_host_calls_reject_bad_sizes():
    with pytest.raises(eth.EthError):
        eth.step_host_layout(0)
    with pytest.raises(eth.EthError):
        eth.step_host_matrix(3, eth.STEP_P)      # odd m has no coarser level


def test_threaded_host_assembly_does_not_depend_on_the_thread_count(monkeypatch):
    """F and K are filled row by row on several host threads, each row
    summing its elements in ascending order: one thread and eight give the
    same matrices bit for bit (m = 32, 45 569 velocity nodes, enough rows for
    the threaded fill)."""
    M = StepMesh(32)
    w = uniform_vector(2 * M.nv, 3)
    out = []
    for nt in ("1", "8"):
        monkeypatch.setenv("ETH_HOST_THREADS", nt)
        out.append([eth.step_host_matrix(32, k, nu=1.0 / 50, wind=w) for k in (eth.STEP_K, eth.STEP_RHS)])
    for a, b in zip(out[0], out[1]):
        for x, y in zip(a[:3], b[:3]):
            assert np.array_equal(x, y)
