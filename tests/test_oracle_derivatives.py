"""Pins of the oracle's JVP / VJP of the assembly map (complex-step
differentiation of the element matrices).

Checks: central finite differences of the assembled matrix; the scaling
laws of the operators (E(s q) = s^(d-2) E(q) for stiffness, s^d for the mass:
along dq = q the derivative is (d-2) A resp. d A) and invariance under
translations and rotations; the VJP with G = a b^T equals the pinned
gradient of J = a^T (S + M_w) b; and the adjoint identity
<G, JVP(dq, dw)> = <VJP(G), (dq, dw)>.
"""
import numpy as np
import pytest

import oracle
from helpers import floored_err
from paper_1401_3301_amd import meshgen as mg


def _mesh(d):
    return mg.jittered_square(5, 0.2, seed=131) if d == 2 else mg.kuhn_cube(3, 0.15, seed=132,
                                                                          perm_seed=133)


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("op", ["MASS", "MASS_W", "STIFF"])
def test_jvp_against_finite_differences(d, op):
    m = _mesh(d)
    rng = np.random.default_rng(134)
    dq = rng.standard_normal(m.q.shape) * 0.01
    w = mg.lognormal_field(m.nq, 135)
    dw = rng.standard_normal(m.nq) if op == "MASS_W" else None
    rp, ci, v, av = oracle.jvp(m.q, m.me, op, dq, w if op == "MASS_W" else None, dw)
    h = 1e-5
    kw = {"w": w + h * dw} if op == "MASS_W" else {}
    _, _, vp, _ = oracle.assemble(m.q + h * dq, m.me, op, **kw)
    kw = {"w": w - h * dw} if op == "MASS_W" else {}
    _, _, vm, _ = oracle.assemble(m.q - h * dq, m.me, op, **kw)
    fd = (vp - vm) / (2 * h)
    assert np.abs(v - fd).max() <= 1e-6 * np.abs(v).max()


@pytest.mark.parametrize("d", [2, 3])
def test_scaling_and_rigid_motions(d):
    m = _mesh(d)
    for op, power in (("STIFF", d - 2), ("MASS", d)):
        _, _, A, Aabs = oracle.assemble(m.q, m.me, op)
        _, _, dA, _ = oracle.jvp(m.q, m.me, op, m.q.copy())
        assert floored_err(dA, power * A, Aabs) < 1e-12
        shift = np.tile(np.array([[0.3], [-0.2], [0.1]])[:d], (1, m.nq))
        _, _, dT, _ = oracle.jvp(m.q, m.me, op, shift)
        assert np.abs(dT).max() == 0.0
        R = np.zeros((d, d))
        R[0, 1], R[1, 0] = -1.0, 1.0          # infinitesimal rotation in the (x, y) plane
        _, _, dR, _ = oracle.jvp(m.q, m.me, op, R @ m.q)
        assert np.abs(dR).max() <= 1e-13 * np.abs(A).max()


@pytest.mark.parametrize("d", [2, 3])
def test_vjp_of_rank_one_equals_the_pinned_gradient(d):
    m = _mesh(d)
    rng = np.random.default_rng(136)
    a, b = rng.standard_normal(m.nq), rng.standard_normal(m.nq)
    w = mg.lognormal_field(m.nq, 137)
    J, gw, gq = oracle.grad(m.q, m.me, w, a, b)
    dq = np.zeros((d, m.nq))
    for op in ("STIFF", "MASS_W"):
        rp, ci, _, _ = oracle.assemble(m.q, m.me, op, w=w)
        rows = np.repeat(np.arange(m.nq), np.diff(rp))
        G = a[rows] * b[ci]
        vq, vw, _, _ = oracle.vjp(m.q, m.me, op, rp, ci, G, w=w)
        dq += vq
        if op == "MASS_W":
            assert np.abs(vw - gw).max() <= 1e-12 * np.abs(gw).max()
    assert np.abs(dq - gq).max() <= 1e-12 * np.abs(gq).max()


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("op", ["MASS", "MASS_W", "STIFF"])
def test_adjoint_identity(d, op):
    m = _mesh(d)
    rng = np.random.default_rng(138)
    w = mg.lognormal_field(m.nq, 139) if op == "MASS_W" else None
    rp, ci, _, _ = oracle.assemble(m.q, m.me, op, w=w)
    G = rng.standard_normal(len(ci))
    dq = rng.standard_normal(m.q.shape)
    dw = rng.standard_normal(m.nq) if op == "MASS_W" else None
    _, _, dA, _ = oracle.jvp(m.q, m.me, op, dq, w, dw)
    vq, vw, _, _ = oracle.vjp(m.q, m.me, op, rp, ci, G, w=w)
    lhs = G @ dA
    rhs = np.sum(vq * dq) + (vw @ dw if op == "MASS_W" else 0.0)
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(G) @ np.abs(dA))


def test_vjp_vertex_subset():
    m = _mesh(3)
    rng = np.random.default_rng(140)
    rp, ci, _, _ = oracle.assemble(m.q, m.me, "STIFF")
    G = rng.standard_normal(len(ci))
    full, _, _, _ = oracle.vjp(m.q, m.me, "STIFF", rp, ci, G)
    sel = np.array([0, 5, m.nq - 1])
    part, _, _, _ = oracle.vjp(m.q, m.me, "STIFF", rp, ci, G, vertices=sel)
    assert np.array_equal(part[:, sel], full[:, sel])
