"""GPU checks of the long-row routes: a vertex with 40 neighbours stays in a
block (every operator on the block layouts); a vertex with 300 neighbours is
beyond the block caps, so its row is assembled by the row-gather tile kernel
beside the pair kernel, and the symbolic phase builds it on its workgroup
path."""
import numpy as np
import pytest

import oracle
from helpers import assert_parity
from paper_1401_3301_amd import meshgen as mg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from paper_1401_3301_amd import femasm  # noqa: E402

DEV = torch.device("cuda:0")


def _fan(n, seed=0):
    """n triangles around vertex 0 of a jittered disk, plus a ring of outer
    triangles so that every row but 0 stays short."""
    rng = np.random.default_rng(seed)
    ang = np.linspace(0, 2 * np.pi, n, endpoint=False) + rng.uniform(-0.01, 0.01, n)
    r2 = 2.0
    q = np.hstack([[[0.0], [0.0]], np.vstack([np.cos(ang), np.sin(ang)]),
                   r2 * np.vstack([np.cos(ang + np.pi / n), np.sin(ang + np.pi / n)])])
    inner = [[0, 1 + i, 1 + (i + 1) % n] for i in range(n)]
    outer = []
    for i in range(n):
        a, b, c = 1 + i, 1 + (i + 1) % n, 1 + n + i
        outer += [[a, c, b]]
    me = np.ascontiguousarray(np.array(inner + outer, np.int32).T)
    return mg.Mesh(2, np.ascontiguousarray(q), me)


def test_long_row_keeps_the_block_layouts():
    """A vertex with 40 neighbours (rows up to 511 entries fit a block): every
    operator, the pair-only ones included, runs on the block layouts and
    matches the oracle."""
    mesh = _fan(40)
    me = torch.from_numpy(mesh.me).to(DEV)
    q = torch.from_numpy(mesh.q).to(DEV)
    w = mg.lognormal_field(mesh.nq, 3)
    plan = femasm.Plan(me, mesh.nq)
    assert plan.max_row == 41 and plan.layouts() == 1
    for op in ("MASS", "MASS_W", "STIFF", "ELAS"):
        wt = w if op == "MASS_W" else None
        v = plan.numeric(op, q, wt).cpu().numpy()
        plan.sync_status()
        _, _, ov, oav = oracle.assemble(mesh.q, mesh.me, op, w=wt)
        assert_parity(v, ov, oav, what=f"fan40 {op}")
    lam, mu = np.ones(mesh.nq) * 1.5, np.ones(mesh.nq) * 0.25
    v = plan.elasticity_nodal(q, lam, mu).cpu().numpy()
    _, _, ov, oav = oracle.assemble_lame(mesh.q, mesh.me, lam, mu)
    assert_parity(v, ov, oav, what="fan40 nodal Lame")
    coef = oracle.general_coef(2, np.eye(2))
    v = plan.general(q, coef).cpu().numpy()
    _, _, ov, oav = oracle.assemble_general(mesh.q, mesh.me, coef)
    assert_parity(v, ov, oav, what="fan40 general")
    dq = np.random.default_rng(4).standard_normal(mesh.q.shape) * 0.01
    v = plan.jvp("STIFF", q, dq).cpu().numpy()
    _, _, ov, oav = oracle.jvp(mesh.q, mesh.me, "STIFF", dq)
    assert_parity(v, ov, oav, what="fan40 JVP")


def test_row_beyond_255_entries():
    """A vertex with 300 neighbours: the symbolic phase's workgroup path builds
    its row; values as the oracle's."""
    mesh = _fan(300)
    plan = femasm.Plan(torch.from_numpy(mesh.me).to(DEV), mesh.nq)
    assert plan.max_row == 301
    q = torch.from_numpy(mesh.q).to(DEV)
    for op in ("STIFF", "ELAS"):
        rp, ci = (x.cpu().numpy() for x in plan.pattern(op))
        v = plan.numeric(op, q).cpu().numpy()
        plan.sync_status()
        orp, oci, ov, oav = oracle.assemble(mesh.q, mesh.me, op)
        assert np.array_equal(rp, orp) and np.array_equal(ci, oci)
        assert_parity(v, ov, oav, what=f"fan300 {op}")
