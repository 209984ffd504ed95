"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Bar: CSR pattern bit-exact; values within 1e-12 of the oracle per entry,
relative to max(|v*|, sum of |contributions| into that entry) (the floored
bound: plain relative error is ill-posed for entries that cancel).  Small and
medium meshes (several row tiles plus a ragged tail) are compared entry by
entry; the full-size 2D (2048^2 cells) and 3D (128^3 cubes, permuted
elements) workloads, in the launch configuration the benchmark times, are
compared on sampled rows that the oracle computes one by one and on
size-independent properties.
"""
import numpy as np
import pytest

import oracle
from helpers import assert_parity, floored_err
from paper_1401_3301_amd import meshgen as mg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from paper_1401_3301_amd import femasm  # noqa: E402

DEV = torch.device("cuda:0")
OPS = ["MASS", "MASS_W", "STIFF", "ELAS"]


def _gpu(mesh, w=None):
    me = torch.from_numpy(np.ascontiguousarray(mesh.me)).to(DEV)
    q = torch.from_numpy(np.ascontiguousarray(mesh.q)).to(DEV)
    wt = None if w is None else torch.from_numpy(np.ascontiguousarray(w)).to(DEV)
    return me, q, wt


def _run(mesh, op, w=None, lam=1.0, mu=0.5):
    me, q, wt = _gpu(mesh, w)
    plan = femasm.Plan(me, mesh.nq)
    rp, ci = plan.pattern(op)
    v = plan.numeric(op, q, wt, lam, mu)
    plan.sync_status()
    return plan, rp.cpu().numpy(), ci.cpu().numpy(), v.cpu().numpy()


def _full_parity(mesh, op, w=None, lam=1.0, mu=0.5, what=""):
    plan, rp, ci, v = _run(mesh, op, w, lam, mu)
    orp, oci, ov, oav = oracle.assemble(mesh.q, mesh.me, op, w=w, lam=lam, mu=mu)
    assert np.array_equal(rp, orp), f"{what} row_ptr"
    assert np.array_equal(ci, oci), f"{what} col_idx"
    return assert_parity(v, ov, oav, what=f"{what} {op}")


SMALL = {
    "square64": lambda: mg.jittered_square(64, 0.2, seed=1),
    "square37_down": lambda: mg.jittered_square(37, 0.2, seed=5, diagonals="down"),
    "cube9_perm": lambda: mg.kuhn_cube(9, 0.15, seed=3, perm_seed=33),
    "cube14": lambda: mg.kuhn_cube(14, 0.15, seed=7),
}


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("op", OPS)
def test_parity_small(name, op):
    mesh = SMALL[name]()
    w = mg.lognormal_field(mesh.nq, 21) if op == "MASS_W" else None
    e = _full_parity(mesh, op, w, lam=1.0, mu=0.5, what=name)
    print(f"{name} {op} floored err {e:.2e}")


def test_parity_lame_parameters():
    mesh = mg.kuhn_cube(5, 0.15, seed=9, perm_seed=1)
    _full_parity(mesh, "ELAS", lam=3.7, mu=0.21, what="lame")
    mesh2 = mg.jittered_square(11, 0.2, seed=9)
    _full_parity(mesh2, "ELAS", lam=0.3, mu=2.5, what="lame2d")


@pytest.mark.parametrize("op", OPS)
def test_deterministic_and_symmetric(op):
    mesh = mg.kuhn_cube(10, 0.15, seed=4, perm_seed=44)
    w = mg.lognormal_field(mesh.nq, 5)
    me, q, wt = _gpu(mesh, w)
    plan = femasm.Plan(me, mesh.nq)
    v1 = plan.numeric(op, q, wt).clone()
    v2 = plan.numeric(op, q, wt).clone()
    torch.cuda.synchronize()
    assert torch.equal(v1, v2), "values differ between two runs"
    rp, ci = plan.pattern(op)
    import scipy.sparse as sp
    n = rp.numel() - 1
    A = sp.csr_matrix((v1.cpu().numpy(), ci.cpu().numpy(), rp.cpu().numpy()), shape=(n, n))
    assert (A != A.T).nnz == 0, "not exactly symmetric"


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("name", ["square64", "cube9_perm", "cube14"])
def test_kernel_families_agree_bitwise(name, op, monkeypatch):
    """The vertex-pair kernel, the record-block kernel (scalar operators) and
    the row-gather kernel sum every entry in the same order with the same
    expressions: their values agree bit for bit (and with the default)."""
    mesh = SMALL[name]()
    w = mg.lognormal_field(mesh.nq, 3)
    me, q, wt = _gpu(mesh, w)
    # the record-block layout is built only on request when the pair layouts exist
    monkeypatch.setenv("FEMASM_BLOCK_LAYOUT", "1")
    plan = femasm.Plan(me, mesh.nq)
    v_def = plan.numeric(op, q, wt, 1.3, 0.7).clone()
    kernels = ["pair", "rowgather"] + ([] if op == "ELAS" else ["block"])
    for kern in kernels:
        monkeypatch.setenv("FEMASM_KERNEL", kern)
        v = plan.numeric(op, q, wt, 1.3, 0.7).clone()
        torch.cuda.synchronize()
        assert torch.equal(v, v_def), f"{kern} differs from the default kernel"


def test_slot_map_consistency():
    mesh = mg.kuhn_cube(6, 0.15, seed=8, perm_seed=80)
    me, q, _ = _gpu(mesh)
    plan = femasm.Plan(me, mesh.nq)
    slot = plan.slot_map().cpu().numpy().reshape(mesh.nme, 4, 4)   # [k, b, a]
    rp, ci = (x.cpu().numpy() for x in plan.pattern("STIFF"))
    rows = np.repeat(np.arange(mesh.nq), np.diff(rp))
    for a in range(4):
        for b in range(4):
            s = slot[:, b, a]
            assert np.array_equal(rows[s], mesh.me[a]) and np.array_equal(ci[s], mesh.me[b])
    # `sparse` semantics: scattering the oracle's element matrices through the
    # slot map reproduces the oracle CSR
    orp, oci, ov, oav = oracle.assemble(mesh.q, mesh.me, "STIFF")
    acc = np.zeros(len(ci))
    for k in range(mesh.nme):
        E = oracle.element_matrix(mesh.q[:, mesh.me[:, k]].T, "STIFF")
        for a in range(4):
            for b in range(4):
                acc[slot[k, b, a]] += E[a, b]
    assert floored_err(acc, ov, oav) < 1e-12


# ------------------------------------------------------------- edge cases
def test_empty_mesh_and_unused_vertices():
    q = np.array([[0.0, 1.0, 0.0, 3.0], [0.0, 0.0, 1.0, 3.0]])
    me = np.zeros((3, 0), np.int32)
    plan = femasm.Plan(torch.from_numpy(me).to(DEV), 4)
    rp, ci = plan.pattern("STIFF")
    assert rp.cpu().tolist() == [0, 0, 0, 0, 0] and ci.numel() == 0
    v = plan.numeric("STIFF", torch.from_numpy(q).to(DEV))
    assert v.numel() == 0
    mesh = mg.Mesh(2, q, np.array([[0], [1], [2]], np.int32))
    _full_parity(mesh, "STIFF", what="unused")
    _full_parity(mesh, "ELAS", what="unused")


def test_error_paths():
    mesh = mg.jittered_square(4, 0.1, seed=2)
    me = mesh.me.copy()
    me[1, 3] = mesh.nq
    with pytest.raises(femasm.FemError) as ei:
        femasm.Plan(torch.from_numpy(me).to(DEV), mesh.nq)
    assert ei.value.name == "FEM_ERR_INDEX"
    assert oracle.validate(2, mesh.nq, me) == ei.value.code
    me = mesh.me.copy()
    me[2, 7] = me[1, 7]
    with pytest.raises(femasm.FemError) as ei:
        femasm.Plan(torch.from_numpy(me).to(DEV), mesh.nq)
    assert ei.value.name == "FEM_ERR_INDEX" and oracle.validate(2, mesh.nq, me) == ei.value.code
    # degenerate element: reported by the status word after the fact
    q = mesh.q.copy()
    q[:, mesh.me[1, 5]] = q[:, mesh.me[0, 5]]
    me_t, q_t, _ = _gpu(mg.Mesh(2, q, mesh.me))
    plan = femasm.Plan(me_t, mesh.nq)
    for op in ("STIFF", "MASS", "ELAS"):
        plan.numeric(op, q_t)
        with pytest.raises(femasm.FemError) as ei:
            plan.sync_status()
        assert ei.value.name == "FEM_ERR_DEGENERATE"
        plan.sync_status()          # the word is cleared on read
    with pytest.raises(oracle.OracleError) as eo:
        oracle.assemble(q, mesh.me, "STIFF")
    assert eo.value.code == 3
    # bad arguments
    with pytest.raises(femasm.FemError) as ei:
        femasm.fem_assemble_symbolic(4, 10, 1, 0)
    assert ei.value.name == "FEM_ERR_ARG"
    with pytest.raises(femasm.FemError) as ei:
        femasm.fem_assemble_numeric(plan.handle, 7, q_t.data_ptr(), None, 1.0, 0.5, q_t.data_ptr())
    assert ei.value.name == "FEM_ERR_ARG"
    with pytest.raises(femasm.FemError):
        plan.numeric("MASS_W", q_t, None)


# --------------------------------------------- full-size workloads, sampled
def _sampled_check(mesh, op, plan, v, rp, ci, w=None, nsample=256, seed=0):
    m = mesh.d if op == "ELAS" else 1
    nrows = m * mesh.nq
    rng = np.random.default_rng(seed)
    rows = np.unique(np.concatenate([rng.choice(nrows, nsample, replace=False),
                                     [0, nrows - 1, nrows // 2]]))
    srp, sci, sv, sav = oracle.assemble_rows(mesh.q, mesh.me, op, rows, w=w)
    worst = 0.0
    for s, r in enumerate(rows):
        a, b = rp[r], rp[r + 1]
        assert np.array_equal(ci[a:b], sci[srp[s]:srp[s + 1]]), f"row {r} pattern"
        worst = max(worst, floored_err(v[a:b], sv[srp[s]:srp[s + 1]], sav[srp[s]:srp[s + 1]]))
    assert worst <= 1e-12, worst
    return worst


@pytest.fixture(scope="module")
def big3d():
    return mg.config_large_3d()["mesh"]


@pytest.fixture(scope="module")
def big2d():
    c = mg.config_large_2d()
    return c["mesh"], c["w"]


@pytest.mark.parametrize("op", ["STIFF", "ELAS"])
def test_full_size_3d(big3d, op):
    mesh = big3d
    plan, rp, ci, v = _run(mesh, op)
    n = 128
    E = 3 * n * (n + 1) ** 2 + 3 * n * n * (n + 1) + n ** 3
    m = 3 if op == "ELAS" else 1
    assert len(v) == m * m * (mesh.nq + 2 * E)
    worst = _sampled_check(mesh, op, plan, v, rp, ci)
    print(f"3D full size {op}: sampled worst floored err {worst:.2e}")
    if op == "STIFF":
        # constants are in the kernel of S: every row sums to ~0
        rs = np.add.reduceat(v, rp[:-1])
        scale = np.add.reduceat(np.abs(v), rp[:-1])
        assert (np.abs(rs) <= 1e-12 * scale).all()


@pytest.mark.parametrize("op", ["STIFF", "MASS_W", "ELAS"])
def test_full_size_2d(big2d, op):
    mesh, w = big2d
    plan, rp, ci, v = _run(mesh, op, w if op == "MASS_W" else None)
    if op != "ELAS":
        assert len(v) == 3 * mesh.nq + 2 * mesh.nme - 2
    worst = _sampled_check(mesh, op, plan, v, rp, ci, w=w if op == "MASS_W" else None)
    print(f"2D full size {op}: sampled worst floored err {worst:.2e}")
