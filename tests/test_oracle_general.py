"""Pins of the oracle's general second-order operator (the PDE of the
introduction, constant coefficients, weak form).

P1 functions are in the discrete space, so for u, v affine the bilinear form
v^T K u is exactly int A grad u . grad v - int u b . grad v + int (c . grad u) v
+ int a0 u v, a closed form on the unit square / cube; special coefficient
choices reduce to the stiffness and mass matrices; b = c alone gives an
antisymmetric matrix.
"""
import numpy as np
import pytest

import oracle
from helpers import floored_err, to_scipy
from paper_1401_3301_amd import meshgen as mg


def _mesh(d):
    return mg.jittered_square(6, 0.2, seed=91) if d == 2 else mg.kuhn_cube(3, 0.15, seed=92,
                                                                          perm_seed=93)


def _K(m, coef):
    rp, ci, v, av = oracle.assemble_general(m.q, m.me, coef)
    return to_scipy(rp, ci, v, m.nq), (rp, ci, v, av)


@pytest.mark.parametrize("d", [2, 3])
def test_reduces_to_stiffness_and_mass(d):
    m = _mesh(d)
    _, (rp, ci, v, _) = _K(m, oracle.general_coef(d, A=np.eye(d)))
    rs, cs, vs, avs = oracle.assemble(m.q, m.me, "STIFF")
    assert np.array_equal(rp, rs) and np.array_equal(ci, cs)
    assert floored_err(v, vs, avs) < 1e-14
    _, (rp, ci, v, _) = _K(m, oracle.general_coef(d, a0=1.0))
    rm, cm, vm, avm = oracle.assemble(m.q, m.me, "MASS")
    assert floored_err(v, vm, avm) < 1e-14


@pytest.mark.parametrize("d", [2, 3])
def test_bilinear_form_on_affine_functions(d):
    m = _mesh(d)
    x = m.q
    one = np.ones(m.nq)
    rng = np.random.default_rng(94 + d)
    A = rng.uniform(-1, 1, (d, d))
    b = rng.uniform(-1, 1, d)
    c = rng.uniform(-1, 1, d)
    a0 = 0.7
    K, _ = _K(m, oracle.general_coef(d, A, b, c, a0))
    # u = x_0, v = x_1 on the unit square / cube (integrals: 1/2 for x_i, 1/4 for x_0 x_1)
    u, v = x[0], x[1]
    want = A[1, 0] - b[1] * 0.5 + c[0] * 0.5 + a0 * 0.25
    assert abs(v @ (K @ u) - want) < 1e-13
    # u = 1, v = x_0: only the b and reaction terms
    want = -b[0] + a0 * 0.5
    assert abs(x[0] @ (K @ one) - want) < 1e-13
    # u = x_1, v = 1: c and reaction
    want = c[1] + a0 * 0.5
    assert abs(one @ (K @ x[1]) - want) < 1e-13


@pytest.mark.parametrize("d", [2, 3])
def test_skew_part(d):
    m = _mesh(d)
    b = np.array([0.3, -1.1, 0.6])[:d]
    K, _ = _K(m, oracle.general_coef(d, b=b, c=b))
    assert abs(K + K.T).max() <= 1e-15 * abs(K).max()
    # without b and reaction, constants are in the kernel: K 1 = 0
    K2, _ = _K(m, oracle.general_coef(d, A=np.array([[2.0, 0.5, 0], [-0.3, 1.0, 0.2],
                                                     [0.1, 0, 1.5]])[:d, :d],
                                      c=np.array([1.0, 2.0, -1.0])[:d]))
    assert np.abs(K2 @ np.ones(m.nq)).max() < 1e-13 * abs(K2).max()


def test_rows_variant():
    m = _mesh(2)
    coef = oracle.general_coef(2, np.array([[1, 0.2], [0.1, 2]]), [0.5, -0.2], [0.1, 0.3], 0.4)
    rp, ci, v, av = oracle.assemble_general(m.q, m.me, coef)
    rows = np.array([3, 0, m.nq - 1])
    rr, cr, vr, ar = oracle.assemble_general(m.q, m.me, coef, rows=rows)
    for s, r in enumerate(rows):
        assert np.array_equal(cr[rr[s]:rr[s + 1]], ci[rp[r]:rp[r + 1]])
        assert np.array_equal(vr[rr[s]:rr[s + 1]], v[rp[r]:rp[r + 1]])
