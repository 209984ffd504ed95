"""Pins of the P_k mass oracle (Appendix D) against what the mathematics fixes.

The oracle builds C from the paper's polynomial representation of the basis
in barycentric coordinates.  The checks below reach the same quantities by
other routes: textbook P2 matrices, the partition of unity, a Lagrange basis
obtained by inverting a Cartesian Vandermonde matrix on the reference
simplex with exact monomial integrals, and the exact integration of
products of polynomials of degree <= k over the unit square and cube.  The
exact rational route pins every degree k = 1..6 in 2D and 3D bit for bit.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
from helpers import floored_err, to_scipy
from paper_1401_3301_amd import meshgen as mg

GOLD = os.path.join(os.path.dirname(__file__), "golden", "pk_textbook.json")


def test_local_numbering():
    """Vertices first, then decreasing lexicographic; same count as (d+k)!/(d!k!)."""
    for d in (2, 3):
        for k in range(1, 7):
            a = oracle.pk_alpha(d, k)
            assert a.shape == (math.comb(d + k, d), d + 1)
            assert np.all(a.sum(1) == k)
            assert np.array_equal(a[:d + 1], k * np.eye(d + 1, dtype=np.int32))
            rest = [tuple(x) for x in a[d + 1:]]
            assert rest == sorted(rest, reverse=True)
            assert len(set(map(tuple, a))) == len(a)
            # the generator enumerates the same order
            assert [tuple(x) for x in a] == mg.pk_local_indices(d, k)


def test_p2_triangle_textbook():
    g = json.load(open(GOLD))["p2_triangle"]
    C = oracle.pk_coeff(2, 2)
    # int_K phi_a phi_b = d! |K| C; golden is |K| num / den
    np.testing.assert_allclose(2.0 * C, np.array(g["num"]) / g["den"], rtol=1e-15, atol=1e-17)


def test_p2_tetrahedron_integrals():
    g = json.load(open(GOLD))["p2_tetrahedron_integrals"]
    C = oracle.pk_coeff(3, 2)
    np.testing.assert_allclose(6.0 * C.sum(1), np.array(g["num"]) / g["den"], rtol=1e-14,
                               atol=1e-17)


@pytest.mark.parametrize("d", [2, 3])
def test_p1_case_is_the_magic_formula(d):
    """k = 1: d! C_ab = d! (1 + delta_ab) / (d+2)! (magic formula, Section 2)."""
    C = oracle.pk_coeff(d, 1)
    ref = (1.0 + np.eye(d + 1)) / math.factorial(d + 2)
    np.testing.assert_allclose(math.factorial(d) * C, math.factorial(d) * ref, rtol=1e-15)


@pytest.mark.parametrize("d,k", [(d, k) for d in (2, 3) for k in range(1, 7)])
def test_partition_of_unity_and_symmetry(d, k):
    C = oracle.pk_coeff(d, k)
    assert np.array_equal(C, C.T)
    # sum_ab int phi_a phi_b = int 1 = |K|  =>  sum C = 1/d!
    assert abs(C.sum() * math.factorial(d) - 1.0) < 1e-13
    # the basis is linearly independent: C is a Gram matrix, positive definite
    assert np.linalg.eigvalsh(C).min() > 0


def _vandermonde_C(d, k):
    """C through a different route: Lagrange basis on the reference simplex
    (vertex 0 at the origin, vertex i at e_i) by inverting the Vandermonde
    matrix of Cartesian monomials x^m, |m| <= k, at the lattice points
    sum_i alpha_i P_i / k, and int_ref x^m = m! / (d + |m|)! exactly."""
    alpha = oracle.pk_alpha(d, k)
    P = np.vstack([np.zeros(d), np.eye(d)])
    pts = alpha @ P / k                                   # (n, d)
    mons = [m for m in itertools.product(range(k + 1), repeat=d) if sum(m) <= k]
    V = np.array([[np.prod(p ** np.array(m)) for m in mons] for p in pts])
    coef = np.linalg.solve(V, np.eye(len(pts)))          # phi_j = sum_m coef[m, j] x^m

    def integ(m):
        return math.prod(math.factorial(x) for x in m) / math.factorial(d + sum(m))

    Q = np.array([[integ(tuple(a + b for a, b in zip(m1, m2))) for m2 in mons] for m1 in mons])
    M = coef.T @ Q @ coef                                 # int_ref phi_a phi_b, |ref| = 1/d!
    return M                                              # = d! |ref| C = C


@pytest.mark.parametrize("d,k", [(2, 1), (2, 2), (2, 3), (2, 4), (3, 1), (3, 2), (3, 3), (3, 4)])
def test_vandermonde_route(d, k):
    C = oracle.pk_coeff(d, k)
    M = _vandermonde_C(d, k)
    np.testing.assert_allclose(C, M, rtol=0, atol=1e-11 * np.abs(C).max())


def _exact_C(d, k):
    """C in exact rational arithmetic by the Vandermonde route: the Lagrange
    basis on the reference simplex from Gauss-Jordan elimination of the
    Cartesian-monomial Vandermonde matrix at the lattice points (fractions
    throughout), then int_ref x^m = m! / (d + |m|)! for every product.  No
    barycentric product formula and no magic formula are involved."""
    from fractions import Fraction as F

    alpha = oracle.pk_alpha(d, k)
    n = len(alpha)
    pts = [[F(int(a[i + 1]), k) for i in range(d)] for a in alpha]
    mons = [m for m in itertools.product(range(k + 1), repeat=d) if sum(m) <= k]
    assert len(mons) == n
    A = [[math.prod((p[i] ** m[i] for i in range(d)), start=F(1)) for m in mons]
         + [F(int(r == j)) for j in range(n)] for r, p in enumerate(pts)]
    for c in range(n):
        piv = next(r for r in range(c, n) if A[r][c] != 0)
        A[c], A[piv] = A[piv], A[c]
        inv = 1 / A[c][c]
        A[c] = [x * inv for x in A[c]]
        for r in range(n):
            if r != c and A[r][c] != 0:
                f = A[r][c]
                A[r] = [x - f * y for x, y in zip(A[r], A[c])]
    coef = [row[n:] for row in A]                         # phi_j = sum_m coef[m][j] x^m

    def integ(m):
        return F(math.prod(math.factorial(x) for x in m), math.factorial(d + sum(m)))

    Q = [[integ(tuple(a + b for a, b in zip(m1, m2))) for m2 in mons] for m1 in mons]
    QC = [[sum(Q[i][l] * coef[l][j] for l in range(n)) for j in range(n)] for i in range(n)]
    return [[sum(coef[l][a] * QC[l][b] for l in range(n)) for b in range(n)] for a in range(n)]


@pytest.mark.parametrize("d,k", [(d, k) for d in (2, 3) for k in range(1, 7)])
def test_exact_rational_route(d, k):
    """Every degree of Table D.1, 2D and 3D: the oracle's C (exact integers
    over the common denominator, rounded once) equals the exactly computed
    rational C of an independent route, rounded to the nearest double, bit
    for bit."""
    C = oracle.pk_coeff(d, k)
    M = np.array([[float(x) for x in row] for row in _exact_C(d, k)])
    assert np.array_equal(C, M), np.abs(C - M).max()


def _poly_integral_unit(d, c1, c2):
    """int over [0,1]^d of u v for u = sum c1[m] x^m, v = sum c2[m] x^m."""
    tot = 0.0
    for m1, a in c1.items():
        for m2, b in c2.items():
            tot += a * b * math.prod(1.0 / (x + y + 1) for x, y in zip(m1, m2))
    return tot


def _rand_poly(d, k, rng):
    mons = [m for m in itertools.product(range(k + 1), repeat=d) if sum(m) <= k]
    return {m: rng.uniform(-1, 1) for m in mons}


def _eval(c, q):
    out = np.zeros(q.shape[1])
    for m, a in c.items():
        out += a * np.prod(q ** np.array(m)[:, None], axis=0)
    return out


@pytest.mark.parametrize("d,k,n", [(2, 1, 5), (2, 2, 4), (2, 3, 3), (2, 4, 2), (2, 5, 2),
                                   (2, 6, 2), (3, 1, 3), (3, 2, 2), (3, 3, 2), (3, 4, 1),
                                   (3, 5, 1), (3, 6, 1)])
def test_exact_integration_of_polynomials(d, k, n):
    """P_k reproduces polynomials of degree <= k, so with U, V their nodal
    values U^T M V = int_Omega u v exactly; on the (jittered-inside) unit
    square / cube the integral is a sum of 1/((p+1)(q+1)...)."""
    m1 = mg.jittered_square(n, 0.2, seed=21) if d == 2 else mg.kuhn_cube(n, 0.15, seed=22)
    m = mg.pk_mesh(m1, k)
    rp, ci, v, _ = oracle.pk_mass(m.q, m.me, k)
    M = to_scipy(rp, ci, v, m.nq)
    rng = np.random.default_rng(100 * d + k)
    for _ in range(3):
        cu, cv = _rand_poly(d, k, rng), _rand_poly(d, k, rng)
        U, V = _eval(cu, m.q), _eval(cv, m.q)
        ref = _poly_integral_unit(d, cu, cv)
        got = U @ (M @ V)
        scale = np.abs(U) @ (abs(M) @ np.abs(V))
        assert abs(got - ref) <= 1e-13 * scale, (got, ref)


def test_pk_mesh_k1_is_the_p1_mesh_and_matches_p1_mass():
    """k = 1: the P_k mesh is the P1 mesh and the P_k mass is the P1 mass
    matrix of the magic formula (entries agree to rounding)."""
    m1 = mg.kuhn_cube(3, 0.15, seed=5, perm_seed=6)
    m = mg.pk_mesh(m1, 1)
    assert np.array_equal(m.me, m1.me) and np.array_equal(m.q, m1.q)
    rp, ci, v, av = oracle.pk_mass(m.q, m.me, 1)
    rp1, ci1, v1, av1 = oracle.assemble(m1.q, m1.me, "MASS")
    assert np.array_equal(rp, rp1) and np.array_equal(ci, ci1)
    assert floored_err(v, v1, av1) < 1e-14


def test_rows_variant_and_errors():
    m = mg.pk_mesh(mg.jittered_square(3, 0.2, seed=2), 3)
    rp, ci, v, av = oracle.pk_mass(m.q, m.me, 3)
    rows = np.array([m.nq - 1, 0, 17, 5])
    rr, cr, vr, ar = oracle.pk_mass_rows(m.q, m.me, 3, rows)
    for s, r in enumerate(rows):
        assert np.array_equal(cr[rr[s]:rr[s + 1]], ci[rp[r]:rp[r + 1]])
        assert np.array_equal(vr[rr[s]:rr[s + 1]], v[rp[r]:rp[r + 1]])
    bad = m.me.copy()
    bad[4, 0] = bad[0, 0]
    with pytest.raises(oracle.OracleError) as e:
        oracle.pk_mass(m.q, bad, 3)
    assert e.value.name == "ERR_INDEX"
    q = m.q.copy()
    q[:, m.me[1, 0]] = q[:, m.me[0, 0]]      # collapse element 0
    with pytest.raises(oracle.OracleError) as e:
        oracle.pk_mass(q, m.me, 3)
    assert e.value.name == "ERR_DEGENERATE"


def test_generator_places_nodes_on_the_lattice():
    """Input check: every local node sits at sum alpha_i P_i / k of its element
    and nodes on shared sub-simplices are shared (no duplicates)."""
    for d, k, m1 in [(2, 3, mg.jittered_square(3, 0.2, seed=1)), (3, 2, mg.kuhn_cube(2, 0.1, seed=2))]:
        m = mg.pk_mesh(m1, k)
        alpha = np.array(mg.pk_local_indices(d, k))
        for e in range(m.nme):
            P = m1.q[:, m1.me[:, e]]                      # (d, d+1)
            want = P @ alpha.T / k                        # (d, ndfe)
            np.testing.assert_allclose(m.q[:, m.me[:, e]], want, atol=1e-15)
        uq = np.unique(np.round(m.q.T, 12), axis=0)
        assert len(uq) == m.nq
