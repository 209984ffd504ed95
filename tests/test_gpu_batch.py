"""Batched assembly: 256 meshes (128 jittered squares, 128 Kuhn cubes,
element counts log-uniform in [1e3, 2e5]) in persistent launches.

Checks: batched values are bitwise equal to per-mesh fem_assemble_numeric
values for every mesh, for both kernel families (vertex pairs in one launch
over both dimensions, row-gather), pair layouts rebuilt with other block
sizes and every tuning parameter set; a subset matches the oracle; a captured
hipGraph replays to the eager result several times with eager work in
between.
"""
import numpy as np
import pytest

import oracle
from helpers import assert_parity
from paper_1401_3301_amd import meshgen as mg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1401_3301_amd import femasm  # noqa: E402

DEV = torch.device("cuda:0")


@pytest.fixture(scope="module")
def batch():
    cfg = mg.config_batch()
    meshes, ws = cfg["meshes"], cfg["w"]
    mes = [torch.from_numpy(m.me).to(DEV) for m in meshes]
    B = femasm.Batch(mes, [m.nq for m in meshes])
    q_cat = torch.from_numpy(np.concatenate([m.q.ravel() for m in meshes])).to(DEV)
    w_cat = torch.from_numpy(np.concatenate(ws)).to(DEV)
    return B, meshes, ws, q_cat, w_cat


def _per_mesh(B, op, q_cat, w_cat):
    offs = B.offsets(op)
    out = torch.full((offs.nnz[-1],), np.nan, dtype=torch.float64, device=DEV)
    for i in range(len(B)):
        h = B.plan_handle(i)
        femasm.fem_assemble_numeric(h, femasm.FEM_OP[op], q_cat.data_ptr() + 8 * offs.q[i],
                                    w_cat.data_ptr() + 8 * offs.w[i], 1.0, 0.5,
                                    out.data_ptr() + 8 * offs.nnz[i])
    return out


def test_batch_sizes(batch):
    B, meshes, *_ = batch
    assert len(B) == 256
    n = np.array([m.nme for m in meshes])
    assert n.min() >= 500 and n.max() <= 2.6e5
    assert sum(m.d == 2 for m in meshes) == 128


@pytest.mark.parametrize("op", ["MASS_W", "STIFF", "ELAS"])
def test_batched_equals_per_mesh(batch, op):
    B, meshes, ws, q_cat, w_cat = batch
    ref = _per_mesh(B, op, q_cat, w_cat)
    default = ("pair",) + femasm.PAIR_LAYOUT_DEFAULT[1 if op == "ELAS" else 0]
    split = ("pair_split",) + default[1:]
    for params in [default, split, ("pair", 40, 96, 1), ("rowgather", 256, 2), ("rowgather", 128, 4),
                   ("rowgather", 64, 8), ("rowgather", 256, 1)]:
        B.configure(params, op)
        out = torch.full_like(ref, np.nan)
        B.numeric(op, q_cat, w_cat, out=out)
        B.sync_status()
        assert torch.equal(out, ref), f"{op} batched != per-mesh with params {params}"
    B.configure(default, op)


@pytest.mark.parametrize("op", ["MASS_W", "STIFF", "ELAS"])
def test_batched_vs_oracle_subset(batch, op):
    B, meshes, ws, q_cat, w_cat = batch
    vals = B.numeric(op, q_cat, w_cat).cpu().numpy()
    offs = B.offsets(op)
    for i in (0, 5, 127, 128, 200, 255):
        m = meshes[i]
        w = ws[i] if op == "MASS_W" else None
        orp, oci, ov, oav = oracle.assemble(m.q, m.me, op, w=w)
        v = vals[offs.nnz[i]:offs.nnz[i + 1]]
        assert len(v) == len(ov)
        assert_parity(v, ov, oav, what=f"mesh {i} {op}")
        rp, ci = femasm.Plan(torch.from_numpy(m.me).to(DEV), m.nq).pattern(op)
        assert np.array_equal(rp.cpu().numpy(), orp) and np.array_equal(ci.cpu().numpy(), oci)


@pytest.mark.parametrize("kernel", ["pair", "pair_split", "rowgather"])
def test_graph_capture_replay(batch, kernel):
    B, meshes, ws, q_cat, w_cat = batch
    B.configure((kernel, 56, 128, 2) if kernel.startswith("pair") else (kernel, 256, 2))
    offs = B.offsets("STIFF")
    out_s = torch.empty(offs.nnz[-1], dtype=torch.float64, device=DEV)
    out_m = torch.empty(offs.nnz[-1], dtype=torch.float64, device=DEV)
    ref_s = B.numeric("STIFF", q_cat, w_cat).clone()
    ref_m = B.numeric("MASS_W", q_cat, w_cat).clone()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        B.numeric("STIFF", q_cat, w_cat, out=out_s)       # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        B.numeric("MASS_W", q_cat, w_cat, out=out_m)
        B.numeric("STIFF", q_cat, w_cat, out=out_s)
    for rep in range(4):
        out_s.fill_(-1.0)
        out_m.fill_(-1.0)
        B.numeric("ELAS", q_cat, w_cat)                   # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out_s, ref_s), f"replay {rep} STIFF"
        assert torch.equal(out_m, ref_m), f"replay {rep} MASS_W"
    B.configure(("pair", 56, 128, 2))


def test_autotuner(batch, tmp_path):
    from paper_1401_3301_amd import autotune
    B, meshes, ws, q_cat, w_cat = batch
    ref = _per_mesh(B, "STIFF", q_cat, w_cat)
    cache = str(tmp_path / "tune.json")
    params, times = autotune.tune(B, "STIFF", q_cat, w_cat, reps=2, cache_path=cache)
    assert params in autotune.candidates("STIFF") and len(times) >= 8
    assert sum(k.startswith("pair") for k in times) >= 12   # layout variants timed, both forms
    assert B.params == params
    out = B.numeric("STIFF", q_cat, w_cat)
    assert torch.equal(out, ref)
    B.configure(("rowgather", 64, 1))
    again, _ = autotune.tune(B, "STIFF", q_cat, w_cat, cache_path=cache)   # from the cache
    assert again == params and B.params == params
    B.configure(("pair", 56, 128, 2))
