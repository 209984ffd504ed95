"""GPU: calls on a side stream with inputs the binding must convert (float32
coordinates and weights, upstream gradients in float32) give the values of
the same calls on the default stream, bit for bit, and the temporaries the
binding creates belong to the side stream (the caching allocator cannot hand
them out again while the side stream still reads them): the default stream
is kept busy meanwhile and new tensors are allocated between the calls."""
import numpy as np
import pytest

from paper_1401_3301_amd import meshgen as mg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

from paper_1401_3301_amd import femasm  # noqa: E402

DEV = torch.device("cuda:0")


def test_side_stream_with_converted_inputs():
    mesh = mg.kuhn_cube(20, 0.15, seed=6, perm_seed=7)
    plan = femasm.Plan(torch.from_numpy(mesh.me).to(DEV), mesh.nq)
    q64 = torch.from_numpy(mesh.q).to(DEV)
    q32 = q64.float()
    w32 = torch.from_numpy(mg.lognormal_field(mesh.nq, 3)).to(DEV).float()
    ref = {op: plan.numeric(op, q32, w32).clone() for op in ("MASS_W", "STIFF", "ELAS")}
    G32 = torch.randn(plan.query("STIFF")[1], device=DEV, dtype=torch.float32)
    gq_ref, _ = plan.vjp("STIFF", q32, G32)
    gq_ref = gq_ref.clone()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    busy = torch.randn(4096, 4096, device=DEV)
    for rep in range(3):
        got = {op: plan.numeric(op, q32, w32, stream=side) for op in ref}
        gq, _ = plan.vjp("STIFF", q32, G32, stream=side)
        # the default stream allocates and works while the side stream runs
        for _ in range(4):
            busy = busy @ busy.T / 4096.0
        junk = [torch.full((1 << 20,), 7.0, device=DEV) for _ in range(8)]
        torch.cuda.current_stream().wait_stream(side)
        for op in ref:
            assert torch.equal(got[op], ref[op]), f"{op} on the side stream, repetition {rep}"
        assert torch.equal(gq, gq_ref), f"VJP on the side stream, repetition {rep}"
        del junk
    # a raw stream handle works the same way
    v = plan.numeric("STIFF", q32, stream=side.cuda_stream)
    torch.cuda.current_stream().wait_stream(side)
    assert torch.equal(v, ref["STIFF"])


def test_debug_mode_reports_at_the_call(monkeypatch):
    """FEMASM_DEBUG=1: a numeric call on a mesh with a degenerate element
    returns FEM_ERR_DEGENERATE itself (the status word is read and cleared),
    a good call returns normally; without it the error waits for
    fem_plan_sync_status."""
    m = mg.jittered_square(6, 0.1, seed=2)
    plan = femasm.Plan(torch.from_numpy(m.me).to(DEV), m.nq)
    q = torch.from_numpy(m.q).to(DEV)
    qb = m.q.copy()
    qb[:, m.me[1, 5]] = qb[:, m.me[0, 5]]
    qb = torch.from_numpy(qb).to(DEV)
    monkeypatch.setenv("FEMASM_DEBUG", "1")
    plan.numeric("STIFF", q)
    with pytest.raises(femasm.FemError) as e:
        plan.numeric("STIFF", qb)
    assert e.value.name == "FEM_ERR_DEGENERATE"
    plan.sync_status()   # already cleared by the call
    monkeypatch.delenv("FEMASM_DEBUG")
    plan.numeric("STIFF", qb)   # no error at the call
    with pytest.raises(femasm.FemError) as e:
        plan.sync_status()
    assert e.value.name == "FEM_ERR_DEGENERATE"
