"""The pressure-mass rows of the flow over a step as the GPU's bounding-box
sweep forms them (Sec. 2.3 and Sec. 3, the inflow-outflow example), checked
on the CPU against the oracle's assembled M_Q: a Q1 node's row follows from
which of its four elements are present (the corner below the inflow channel
is absent), an element's row is h^2 on itself and h^2/4 at its vertices.
Small meshes of the step and of the channel, every row compared."""
import numpy as np
import pytest

from oracle.assemble import pressure_mass
from oracle.step import StepMesh


def _present(M, e, f):
    return 0 <= e < M.ex and 0 <= f < M.ey and bool(M.elem_active[f, e])


def _q1_row(M, c, d):
    """The row of Q1 node (c, d) from the presence bits of its elements
    SW, SE, NW, NE: {(kind, i, j): value} over Q1 nodes and elements."""
    h2 = M.h * M.h
    sw, se = _present(M, c - 1, d - 1), _present(M, c, d - 1)
    nw, ne = _present(M, c - 1, d), _present(M, c, d)
    P = sw + se + nw + ne
    w = {(0, 0): 4 * P,
         (0, -1): 2 * (sw + se), (0, 1): 2 * (nw + ne),
         (-1, 0): 2 * (sw + nw), (1, 0): 2 * (se + ne),
         (-1, -1): sw, (1, -1): se, (-1, 1): nw, (1, 1): ne}
    row = {}
    for (a, b), v in w.items():
        if v:
            row[("q", c + a, d + b)] = h2 / 36.0 * v
    for (e, f), p in (((c - 1, d - 1), sw), ((c, d - 1), se), ((c - 1, d), nw), ((c, d), ne)):
        if p:
            row[("e", e, f)] = h2 / 4.0
    return P, row


def _index(M, key):
    kind, i, j = key
    if kind == "q":
        return int(M.q1_index[j, i])
    return M.nk + int(M.el_index[j, i])


@pytest.mark.parametrize("m,channel", [(1, False), (2, False), (3, False), (2, True), (3, True)])
def test_presence_bit_rows_equal_the_assembled_pressure_mass(m, channel):
    M = StepMesh(m, channel=channel)
    A = pressure_mass(M).toarray()
    h2 = M.h * M.h
    seen = np.zeros(A.shape[0], dtype=bool)
    for d in range(M.ey + 1):
        for c in range(M.ex + 1):
            P, row = _q1_row(M, c, d)
            # a node touching no present element is absent from the mesh
            assert (P > 0) == bool(M.q1_active[d, c])
            if P == 0:
                continue
            k = int(M.q1_index[d, c])
            expect = np.zeros(A.shape[1])
            for key, v in row.items():
                j = _index(M, key)
                assert j >= 0, key
                expect[j] += v
            assert np.abs(A[k] - expect).max() <= 1e-15 * h2
            # the update's scale 9 / (h^2 P) is the inverse diagonal
            assert A[k, k] == pytest.approx(h2 * P / 9.0, rel=1e-15)
            seen[k] = True
    for f in range(M.ey):
        for e in range(M.ex):
            if not _present(M, e, f):
                assert M.el_index[f, e] < 0
                continue
            k = M.nk + int(M.el_index[f, e])
            expect = np.zeros(A.shape[1])
            expect[k] = h2
            for c, d in ((e, f), (e + 1, f), (e, f + 1), (e + 1, f + 1)):
                expect[int(M.q1_index[d, c])] = h2 / 4.0
            assert np.abs(A[k] - expect).max() <= 1e-15 * h2
            seen[k] = True
    assert seen.all()


def test_absent_corner_is_the_box_corner():
    """The absent elements of the step are exactly e < m, f < m of the
    bounding box (the corner the GPU masks by two bounds); the re-entrant
    corner node has three present elements."""
    m = 3
    M = StepMesh(m)
    for f in range(M.ey):
        for e in range(M.ex):
            assert bool(M.elem_active[f, e]) == (not (e < m and f < m))
    P, _ = _q1_row(M, m, m)
    assert P == 3
    assert StepMesh(m, channel=True).elem_active.all()
