"""Pins of the oracle's elasticity with nodal (P1) Lame fields (Section 5.1).

For P1 fields lambda_h, mu_h the element matrix is |K|/(d+1) (lambda^s Q-term +
mu^s S-term), which integrates the P1 interpolants exactly.  With fields that
are affine in x (so P1-exact) the strain energy of simple displacement fields
is a closed-form integral over the unit square / cube; constant fields give
the constant-coefficient operator; rigid motions are in the kernel.
"""
import numpy as np
import pytest

import oracle
from helpers import floored_err, to_scipy
from paper_1401_3301_amd import meshgen as mg


def _mesh(d):
    return mg.jittered_square(7, 0.2, seed=71) if d == 2 else mg.kuhn_cube(4, 0.15, seed=72,
                                                                          perm_seed=73)


def _K(m, lam, mu):
    rp, ci, v, av = oracle.assemble_lame(m.q, m.me, lam, mu)
    return to_scipy(rp, ci, v, m.d * m.nq), (rp, ci, v, av)


def _vec(m, f):
    """Interleaved dof vector (r = d*i + l) of a vector field f(q) -> (d, nq)."""
    return np.ascontiguousarray(f(m.q).T).ravel()


@pytest.mark.parametrize("d", [2, 3])
def test_constant_fields_give_the_constant_operator(d):
    m = _mesh(d)
    _, (rp, ci, v, _) = _K(m, np.full(m.nq, 1.0), np.full(m.nq, 0.5))
    rp2, ci2, v2, av2 = oracle.assemble(m.q, m.me, "ELAS", lam=1.0, mu=0.5)
    assert np.array_equal(rp, rp2) and np.array_equal(ci, ci2)
    assert floored_err(v, v2, av2) < 1e-15


@pytest.mark.parametrize("d", [2, 3])
def test_energies_with_affine_fields(d):
    m = _mesh(d)
    x = m.q
    a0, a = 1.3, np.array([0.4, -0.7, 0.25])[:d]
    b0, b = 0.8, np.array([-0.3, 0.5, 0.2])[:d]
    lam = a0 + a @ x
    mu = b0 + b @ x
    K, _ = _K(m, lam, mu)
    c = np.full(d, 0.5)                       # centroid of the unit square / cube
    int_lam, int_mu = a0 + a @ c, b0 + b @ c  # integral of an affine field = value at centroid
    zero = np.zeros(m.nq)
    # uniaxial u = (x, 0, ...): eps_xx = 1, energy density lambda + 2 mu
    u = _vec(m, lambda q: np.vstack([q[0]] + [zero] * (d - 1)))
    assert abs(u @ (K @ u) - (int_lam + 2 * int_mu)) < 1e-12
    # simple shear u = (y, 0, ...): eps_xy = 1/2, energy density mu
    u = _vec(m, lambda q: np.vstack([q[1]] + [zero] * (d - 1)))
    assert abs(u @ (K @ u) - int_mu) < 1e-12
    # dilatation u = x: eps = I, energy density d^2 lambda + 2 d mu
    u = _vec(m, lambda q: q.copy())
    assert abs(u @ (K @ u) - (d * d * int_lam + 2 * d * int_mu)) < 1e-11
    # rigid rotation about the z axis: in the kernel for any fields
    u = _vec(m, lambda q: np.vstack([-q[1], q[0]] + [zero] * (d - 2)))
    assert np.abs(K @ u).max() < 1e-12 * abs(K).max()


def test_linear_in_the_fields():
    m = _mesh(3)
    rng = np.random.default_rng(74)
    l1, l2, m1, m2 = (rng.uniform(0.5, 2.0, m.nq) for _ in range(4))
    K1, _ = _K(m, l1, m1)
    K2, _ = _K(m, l2, m2)
    K3, (rp, ci, v, av) = _K(m, l1 + l2, m1 + m2)
    assert abs(K1 + K2 - K3).max() <= 1e-14 * abs(K3).max()


def test_rows_variant():
    m = _mesh(2)
    rng = np.random.default_rng(75)
    lam, mu = rng.uniform(0.5, 2, m.nq), rng.uniform(0.5, 2, m.nq)
    rp, ci, v, av = oracle.assemble_lame(m.q, m.me, lam, mu)
    rows = np.array([5, 0, 2 * m.nq - 1, 17])
    rr, cr, vr, ar = oracle.assemble_lame(m.q, m.me, lam, mu, rows=rows)
    for s, r in enumerate(rows):
        assert np.array_equal(cr[rr[s]:rr[s + 1]], ci[rp[r]:rp[r + 1]])
        assert np.array_equal(vr[rr[s]:rr[s + 1]], v[rp[r]:rp[r + 1]])
