"""Pins of the oracle's boundary (d-1)-simplex mass and weighted mass (the
Neumann / Robin terms of the remark after the weighted-mass algorithm of
Section 4.1), on the boundary facets of the unit square and cube.

The boundary mass integrates products of P1 traces exactly, so the total is
the perimeter / surface area, x^T M x is the boundary integral of x^2, and
with an affine weight w the weighted matrix integrates w u v exactly; the
reference segment and triangle give the textbook matrices.
"""
import numpy as np
import pytest

import oracle
from helpers import floored_err, to_scipy
from paper_1401_3301_amd import meshgen as mg


def _mesh(d):
    return mg.jittered_square(6, 0.2, seed=111) if d == 2 else mg.kuhn_cube(4, 0.15, seed=112,
                                                                           perm_seed=113)


def _M(m, w=None):
    f = mg.boundary_facets(m)
    rp, ci, v, av = oracle.boundary_mass(m.q, f, w)
    return to_scipy(rp, ci, v, m.nq), f


def test_facet_counts():
    assert mg.boundary_facets(_mesh(2)).shape == (2, 4 * 6)
    assert mg.boundary_facets(_mesh(3)).shape == (3, 6 * 2 * 16)


@pytest.mark.parametrize("d", [2, 3])
def test_total_and_second_moment(d):
    m = _mesh(d)
    M, _ = _M(m)
    one = np.ones(m.nq)
    assert abs(one @ (M @ one) - (4.0 if d == 2 else 6.0)) < 1e-13
    # int over the boundary of x^2: square 1/3 + 1/3 + 1 + 0, cube 4 * 1/3 + 1 + 0
    x = m.q[0]
    assert abs(x @ (M @ x) - (5.0 / 3.0 if d == 2 else 7.0 / 3.0)) < 1e-13
    # interior vertices have empty rows
    inner = mg.interior_mask(d, m.n)
    assert M[inner].nnz == 0


@pytest.mark.parametrize("d", [2, 3])
def test_weighted_with_affine_weight(d):
    m = _mesh(d)
    w = 1.5 + 0.5 * m.q[0] - 0.25 * m.q[1]
    Mw, _ = _M(m, w)
    one = np.ones(m.nq)
    # int over the boundary of w: by symmetry of the faces, w at the centre times the area
    area = 4.0 if d == 2 else 6.0
    assert abs(one @ (Mw @ one) - (1.5 + 0.25 - 0.125) * area) < 1e-13
    # w = 1 gives the plain mass
    M1, _ = _M(m, np.ones(m.nq))
    M0, _ = _M(m)
    assert abs(M1 - M0).max() < 1e-15


def test_reference_simplices():
    # segment (0,0)-(2,0) inside R^2 and triangle of area 1/2 in the plane x + y + z = 1
    q = np.array([[0.0, 2.0], [0.0, 0.0]])
    rp, ci, v, _ = oracle.boundary_mass(q, np.array([[0], [1]], np.int32))
    np.testing.assert_allclose(to_scipy(rp, ci, v, 2).toarray(), 2.0 * np.array([[2, 1], [1, 2]]) / 6,
                               rtol=1e-15)
    q3 = np.array([[1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0]])
    rp, ci, v, _ = oracle.boundary_mass(q3, np.array([[0], [1], [2]], np.int32))
    area = np.sqrt(3.0) / 2.0
    np.testing.assert_allclose(to_scipy(rp, ci, v, 3).toarray(),
                               area * (1 + np.eye(3)) / 12.0, rtol=1e-14)


def test_errors():
    m = _mesh(2)
    f = mg.boundary_facets(m)
    bad = f.copy()
    bad[1, 0] = bad[0, 0]
    with pytest.raises(oracle.OracleError) as e:
        oracle.boundary_mass(m.q, bad)
    assert e.value.name == "ERR_INDEX"
    q = m.q.copy()
    q[:, f[1, 0]] = q[:, f[0, 0]]
    with pytest.raises(oracle.OracleError) as e:
        oracle.boundary_mass(q, f)
    assert e.value.name == "ERR_DEGENERATE"
