"""GPU parity of the pair kernel across its layout settings: rows per block
(FEMASM_PAIR_ROWS / FEMASM_ELAS_ROWS, 16..128), 64-pair tasks per
wavefront (FEMASM_PAIR_SLOTS / FEMASM_ELAS_SLOTS, 1, 2 or 4) and the 3D
element caps (FEMASM_PAIR_ELEMS / FEMASM_ELAS_ELEMS), read when a plan is
built.  Every setting must give the oracle's matrix: the settings
change the blocking, the task deal and the descriptor's packed wavefront
task starts, never the summation order of an entry."""
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
    "square70": lambda: mg.jittered_square(70, 0.2, seed=12),
    "cube11_perm": lambda: mg.kuhn_cube(11, 0.15, seed=13, perm_seed=5),
}
# (rows, slots, 3D element cap or None for the default)
KNOBS = [(16, 1, None), (56, 4, None), (128, 2, None), (128, 4, None), (64, 2, 100), (96, 4, 250)]


@pytest.mark.parametrize("rows,slots,elems", KNOBS,
                         ids=[f"R{r}-s{s}" + (f"-e{e}" if e else "") for r, s, e in KNOBS])
@pytest.mark.parametrize("name", list(MESHES))
def test_layout_settings_keep_parity(monkeypatch, name, rows, slots, elems):
    for var in ("FEMASM_PAIR_ROWS", "FEMASM_ELAS_ROWS"):
        monkeypatch.setenv(var, str(rows))
    for var in ("FEMASM_PAIR_SLOTS", "FEMASM_ELAS_SLOTS"):
        monkeypatch.setenv(var, str(slots))
    if elems:
        for var in ("FEMASM_PAIR_ELEMS", "FEMASM_ELAS_ELEMS"):
            monkeypatch.setenv(var, str(elems))
    mesh = MESHES[name]()
    d = mesh.d
    print(f"layout {name} rows {rows} slots {slots}", flush=True)
    me = torch.from_numpy(np.ascontiguousarray(mesh.me)).to(DEV)
    q = torch.from_numpy(np.ascontiguousarray(mesh.q)).to(DEV)
    w = mg.lognormal_field(mesh.nq, 31)
    plan = femasm.Plan(me, mesh.nq)
    assert plan.layouts() == 1, f"{name}: no block layouts"
    for op in ("MASS", "MASS_W", "STIFF", "ELAS"):
        wt = w if op == "MASS_W" else None
        rp, ci = plan.pattern(op)
        v = plan.numeric(op, q, wt, 1.3, 0.4).cpu().numpy()
        plan.sync_status()
        orp, oci, ov, oav = oracle.assemble(mesh.q, mesh.me, op, w=wt, lam=1.3, mu=0.4)
        assert np.array_equal(rp.cpu().numpy(), orp) and np.array_equal(ci.cpu().numpy(), oci)
        assert_parity(v, ov, oav, what=f"{name} R{rows} s{slots} {op}")
    rng = np.random.default_rng(8)
    coef = oracle.general_coef(d, rng.uniform(-1, 1, (d, d)) + 2 * np.eye(d),
                               rng.uniform(-1, 1, d), rng.uniform(-1, 1, d), 0.7)
    v = plan.general(q, coef).cpu().numpy()
    plan.sync_status()
    _, _, ov, oav = oracle.assemble_general(mesh.q, mesh.me, coef)
    assert_parity(v, ov, oav, what=f"{name} R{rows} s{slots} general")
    lam = mg.lognormal_field(mesh.nq, 32)
    mu = mg.lognormal_field(mesh.nq, 33)
    v = plan.elasticity_nodal(q, lam, mu).cpu().numpy()
    plan.sync_status()
    _, _, ov, oav = oracle.assemble_lame(mesh.q, mesh.me, lam, mu)
    assert_parity(v, ov, oav, what=f"{name} R{rows} s{slots} nodal Lame")
    dq = rng.standard_normal(mesh.q.shape) * 0.01
    v = plan.jvp("STIFF", q, dq).cpu().numpy()
    plan.sync_status()
    _, _, ov, oav = oracle.jvp(mesh.q, mesh.me, "STIFF", dq)
    assert_parity(v, ov, oav, what=f"{name} R{rows} s{slots} JVP")
