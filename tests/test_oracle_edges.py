"""CPU: the oracle on degenerate-size inputs, the cases the GPU edge tests
compare against.  An element list without elements gives empty CSR rows
(nq of them, or d*nq for elasticity) and zero derivatives; a vertex that no
element uses gets an empty row (the reading of unused vertices)."""
import numpy as np
import pytest

import oracle
from paper_1401_3301_amd import meshgen as mg


@pytest.mark.parametrize("d", [2, 3])
def test_no_elements(d):
    nq = 6
    q = np.random.default_rng(d).standard_normal((d, nq))
    me = np.zeros((d + 1, 0), np.int32)
    for op in ("MASS", "MASS_W", "STIFF", "ELAS"):
        rp, ci, v, _ = oracle.assemble(q, me, op, w=np.ones(nq) if op == "MASS_W" else None)
        rows = d * nq if op == "ELAS" else nq
        assert rp.tolist() == [0] * (rows + 1) and len(ci) == 0 and len(v) == 0
    assert oracle.assemble_general(q, me, oracle.general_coef(d, np.eye(d)))[0].tolist() == [0] * (nq + 1)
    assert oracle.assemble_lame(q, me, np.ones(nq), np.ones(nq))[0].tolist() == [0] * (d * nq + 1)
    assert oracle.boundary_mass(q, np.zeros((d, 0), np.int32), None)[0].tolist() == [0] * (nq + 1)
    n_p2 = (d + 1) * (d + 2) // 2
    assert oracle.pk_mass(q, np.zeros((n_p2, 0), np.int32), 2, nq=nq)[0].tolist() == [0] * (nq + 1)
    assert oracle.jvp(q, me, "STIFF", np.zeros_like(q))[0].tolist() == [0] * (nq + 1)
    dq, dw, _, _ = oracle.vjp(q, me, "MASS_W", np.zeros(nq + 1, np.int64), np.zeros(0, np.int64),
                              np.zeros(0), w=np.ones(nq))
    assert dq.shape == (d, nq) and not dq.any() and not dw.any()


def test_unused_vertex_rows_are_empty():
    base = mg.jittered_square(3, 0.2, seed=1)
    q = np.hstack([base.q, [[5.0], [5.0]]])          # vertex base.nq is used by no element
    rp, ci, v, _ = oracle.assemble(q, base.me, "STIFF")
    assert rp[-1] == rp[-2] and base.nq not in set(ci.tolist())
    rp_ref, ci_ref, v_ref, _ = oracle.assemble(base.q, base.me, "STIFF")
    assert np.array_equal(rp[:-1], rp_ref) and np.array_equal(ci, ci_ref) and np.array_equal(v, v_ref)
    rp, ci, _, _ = oracle.assemble(q, base.me, "ELAS")
    assert rp[-1] == rp[-3]                          # both dof rows of the unused vertex empty
