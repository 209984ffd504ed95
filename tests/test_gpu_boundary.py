"""GPU parity of the boundary (d-1)-simplex mass and weighted mass through
fem_boundary_symbolic / fem_boundary_mass, against the oracle, on the
boundary facets of the 2D and 3D workloads (the 128^3 cube's surface: 196,608
triangles, compared entry by entry).
"""
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

MESHES = {
    "square300": lambda: mg.jittered_square(300, 0.2, seed=4),
    "cube14": lambda: mg.kuhn_cube(14, 0.15, seed=7),
    "cube9_perm": lambda: mg.kuhn_cube(9, 0.15, seed=3, perm_seed=33),
    "cube128_perm": lambda: mg.config_large_3d()["mesh"],
}


def _run(mesh, w):
    f = mg.boundary_facets(mesh)
    plan = femasm.BoundaryPlan(torch.from_numpy(f).to(DEV), mesh.nq)
    rp, ci = plan.pattern()
    q = torch.from_numpy(np.ascontiguousarray(mesh.q)).to(DEV)
    v = plan.mass(q, w)
    plan.sync_status()
    return f, plan, q, rp.cpu().numpy(), ci.cpu().numpy(), v.cpu().numpy()


@pytest.mark.parametrize("name", sorted(MESHES))
@pytest.mark.parametrize("weighted", [False, True])
def test_boundary_parity(name, weighted):
    mesh = MESHES[name]()
    w = mg.lognormal_field(mesh.nq, 120) if weighted else None
    print(f"case {name} weighted={weighted}", flush=True)
    f, plan, q, rp, ci, v = _run(mesh, w)
    orp, oci, ov, oav = oracle.boundary_mass(mesh.q, f, w)
    assert np.array_equal(rp, orp) and np.array_equal(ci, oci)
    assert len(ci) > 3 * 1024
    assert_parity(v, ov, oav, what=f"boundary mass {name}")
    area = 4.0 if mesh.d == 2 else 6.0
    if not weighted:
        assert abs(v.sum() - area) < 1e-11
    v2 = plan.mass(q, w).cpu().numpy()
    assert np.array_equal(v, v2)


def test_plan_kinds_and_errors():
    mesh = MESHES["cube9_perm"]()
    f, plan, q, rp, ci, v = _run(mesh, None)
    out = torch.empty(max(plan.nnz, 1), dtype=torch.float64, device=DEV)
    # a boundary plan is not a P_k plan and the other way round
    assert femasm.load_library().fem_pk_mass(plan.handle, q.data_ptr(), out.data_ptr(), None) == 1
    pk = femasm.PkPlan(torch.from_numpy(mesh.me).to(DEV), mesh.nq, 3, 1)
    assert femasm.load_library().fem_boundary_mass(pk.handle, q.data_ptr(), None,
                                                   out.data_ptr(), None) == 1
    # a collapsed facet: its measure is 0 and the status word is set
    qd = mesh.q.copy()
    qd[:, f[1, 0]] = qd[:, f[0, 0]]
    plan.mass(torch.from_numpy(qd).to(DEV))
    with pytest.raises(femasm.FemError) as e:
        plan.sync_status()
    assert e.value.name == "FEM_ERR_DEGENERATE"
    bad = f.copy()
    bad[2, 0] = bad[0, 0]
    with pytest.raises(femasm.FemError) as e:
        femasm.BoundaryPlan(torch.from_numpy(bad).to(DEV), mesh.nq)
    assert e.value.name == "FEM_ERR_INDEX"
