"""GPU parity on unstructured meshes and on rows far longer than a grid's.

The paper's algorithms take any conforming simplicial mesh.  Here: Delaunay
triangulations of random points (scipy) in 2D and 3D with their elements in a
random order (maximum vertex valence well above a grid's), a 2D fan with one
vertex in 1000 triangles and a 3D double fan with one vertex in 600
tetrahedra (rows longer than the symbolic phase's single-wavefront path, so
they take its workgroup path, and beyond the block caps, so the row-gather
tile kernel assembles them beside the pair kernel).  Every operator is
compared with the oracle entry by entry: pattern bit-exact, values within the
floored 1e-12 bound.
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


def delaunay(d, npts, seed):
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(seed)
    pts = rng.random((npts, d))
    tri = Delaunay(pts)
    me = tri.simplices.T.astype(np.int32)
    me = me[:, rng.permutation(me.shape[1])]
    return mg.Mesh(d, np.ascontiguousarray(pts.T), np.ascontiguousarray(me))


def fan2d(m):
    t = 2 * np.pi * np.arange(m) / m
    q = np.concatenate([[[0.0], [0.0]], np.stack([np.cos(t), np.sin(t)])], axis=1)
    i = np.arange(m)
    me = np.stack([np.zeros(m, int), 1 + i, 1 + (i + 1) % m]).astype(np.int32)
    return mg.Mesh(2, q, me)


def fan3d(m):
    """Vertex 0 at the origin, a ring of m vertices, apexes above and below:
    2m tetrahedra around vertex 0."""
    t = 2 * np.pi * np.arange(m) / m
    ring = np.stack([np.cos(t), np.sin(t), 0.1 * np.sin(3 * t)])
    q = np.concatenate([[[0.0], [0.0], [0.0]], ring, [[0.0], [0.0], [1.0]], [[0.0], [0.0], [-1.0]]],
                       axis=1)
    i = np.arange(m)
    a, b = 1 + i, 1 + (i + 1) % m
    top, bot = np.full(m, m + 1), np.full(m, m + 2)
    me = np.concatenate([np.stack([np.zeros(m, int), a, b, top]),
                         np.stack([np.zeros(m, int), b, a, bot])], axis=1).astype(np.int32)
    return mg.Mesh(3, q, me)


MESHES = {
    "delaunay2d": lambda: delaunay(2, 4000, 11),
    "delaunay3d": lambda: delaunay(3, 2500, 12),
    "fan2d_1000": lambda: fan2d(1000),
    "fan3d_300": lambda: fan3d(300),
}


@pytest.fixture(scope="module", params=sorted(MESHES))
def mesh_case(request):
    mesh = MESHES[request.param]()
    me = torch.from_numpy(mesh.me).to(DEV)
    plan = femasm.Plan(me, mesh.nq)
    return request.param, mesh, plan


def test_unstructured_layouts_in_use(mesh_case):
    """Every mesh here keeps its block layouts: the Delaunay meshes entirely
    (rows up to 511 entries fit a block), the fans with their hub rows left
    over to the row-gather tile kernel."""
    name, mesh, plan = mesh_case
    assert plan.layouts() == 1, f"{name}: no block layouts"


@pytest.mark.parametrize("op", ["MASS", "MASS_W", "STIFF", "ELAS"])
def test_unstructured_parity(mesh_case, op):
    name, mesh, plan = mesh_case
    w = mg.lognormal_field(mesh.nq, 7)
    q = torch.from_numpy(mesh.q).to(DEV)
    wt = torch.from_numpy(w).to(DEV)
    rp, ci = (x.cpu().numpy() for x in plan.pattern(op))
    v = plan.numeric(op, q, wt, 1.3, 0.6).cpu().numpy()
    plan.sync_status()
    orp, oci, ov, oav = oracle.assemble(mesh.q, mesh.me, op, w=w if op == "MASS_W" else None,
                                        lam=1.3, mu=0.6)
    assert np.array_equal(rp, orp), f"{name} {op} row_ptr"
    assert np.array_equal(ci, oci), f"{name} {op} col_idx"
    e = assert_parity(v, ov, oav, what=f"{name} {op}")
    print(f"{name} {op}: max row {plan.max_row}, layouts state {plan.layouts()}, floored err {e:.2e}")


def test_first_call_before_layouts_matches():
    """A numeric call made while the block layouts are still being built runs
    the row-gather kernel; its values equal those after the layouts are
    published bit for bit."""
    mesh = mg.kuhn_cube(40, 0.15, seed=3, perm_seed=4)
    me = torch.from_numpy(mesh.me).to(DEV)
    q = torch.from_numpy(mesh.q).to(DEV)
    for op in ("STIFF", "ELAS"):
        plan = femasm.Plan(me, mesh.nq, wait_layouts=False)
        state0 = plan.layouts()
        v0 = plan.numeric(op, q).clone()
        plan.layouts(wait=True)
        assert plan.layouts() == 1
        v1 = plan.numeric(op, q)
        torch.cuda.synchronize()
        assert torch.equal(v0, v1), f"{op}: first call (layout state {state0}) differs"
        print(f"{op}: first call made in layout state {state0}")


def test_vertex_in_too_many_elements():
    """The symbolic phase lists a vertex's candidates in LDS: more than
    16384/(d+1) incident elements is refused with FEM_ERR_OVERFLOW."""
    mesh = fan2d(5500)   # 3 * 5500 > 16384 candidates in row 0
    with pytest.raises(femasm.FemError) as e:
        femasm.Plan(torch.from_numpy(mesh.me).to(DEV), mesh.nq)
    assert e.value.name == "FEM_ERR_OVERFLOW"
    ok = fan2d(5400)     # 16200 candidates: accepted
    plan = femasm.Plan(torch.from_numpy(ok.me).to(DEV), ok.nq)
    assert plan.max_row == 5401


def test_unstructured_next_operators(mesh_case):
    """Nodal-Lame elasticity, the general operator and the JVP against the
    oracle.  On the Delaunay meshes they run on the block layouts; on the fans
    (hub rows left over) the pair-only operators report FEM_ERR_OVERFLOW and
    the JVP takes its row-gather form."""
    name, mesh, plan = mesh_case
    d = mesh.d
    rng = np.random.default_rng(17)
    q = torch.from_numpy(mesh.q).to(DEV)
    lam = np.exp(0.3 * rng.standard_normal(mesh.nq))
    mu = 0.5 * np.exp(0.3 * rng.standard_normal(mesh.nq))
    A = np.eye(d) * 2 + rng.uniform(-0.5, 0.5, (d, d))
    coef = oracle.general_coef(d, A, rng.uniform(-1, 1, d), rng.uniform(-1, 1, d), 0.8)
    dq = 0.01 * rng.standard_normal(mesh.q.shape)
    jv = plan.jvp("STIFF", q, dq).cpu().numpy()
    plan.sync_status()
    _, _, ov, oav = oracle.jvp(mesh.q, mesh.me, "STIFF", dq)
    assert_parity(jv, ov, oav, what=f"{name} JVP")
    if name.startswith("fan"):
        with pytest.raises(femasm.FemError) as e:
            plan.elasticity_nodal(q, lam, mu)
        assert e.value.name == "FEM_ERR_OVERFLOW"
        with pytest.raises(femasm.FemError) as e:
            plan.general(q, coef)
        assert e.value.name == "FEM_ERR_OVERFLOW"
        return
    v = plan.elasticity_nodal(q, lam, mu).cpu().numpy()
    _, _, ov, oav = oracle.assemble_lame(mesh.q, mesh.me, lam, mu)
    assert_parity(v, ov, oav, what=f"{name} nodal Lame")
    v = plan.general(q, coef).cpu().numpy()
    plan.sync_status()
    _, _, ov, oav = oracle.assemble_general(mesh.q, mesh.me, coef)
    assert_parity(v, ov, oav, what=f"{name} general")
