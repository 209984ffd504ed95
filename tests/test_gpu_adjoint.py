"""Adjoint of J = a^T (S(q) + M_w(q)) b on the GPU.

Against the oracle gradient (complex-step shape derivative, exact dJ/dw) on
whole small meshes and, on the 55^3 Kuhn cube (998,250 tets), on vertex stars:
the gradient at vertex i only involves the elements around i, so the oracle
evaluated on the star of i gives the exact entries for i.

Against central finite differences (step 1e-6) of J computed by the GPU
forward assembly on 100 seeded entries drawn from {w_i} and {q_(v,i)}.  J is
linear in w and |J| is large compared with one dJ/dw_i, so the w entries use
the star of i and the mass term only (the stiffness term does not depend on
w); the q entries use the star of i with both terms.  Criterion:
|g_adj - g_fd| <= 1e-6 * max(|g_fd|, 1e-3 * max|g|).
"""
import numpy as np
import pytest

import oracle
from paper_1401_3301_amd import meshgen as mg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1401_3301_amd import femasm  # noqa: E402
from paper_1401_3301_amd.autograd import bilinear_energy  # noqa: E402

DEV = torch.device("cuda:0")


def _t(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def _floored(g, g_ref, scale):
    num = np.abs(g - g_ref)
    den = np.maximum(np.abs(g_ref), scale)
    return float(np.where(num == 0, 0.0, num / np.where(den > 0, den, 1e-300)).max())


@pytest.mark.parametrize("which", ["2d", "3d"])
def test_adjoint_vs_oracle_small(which):
    m = mg.jittered_square(20, 0.2, seed=61) if which == "2d" else \
        mg.kuhn_cube(8, 0.15, seed=62, perm_seed=63)
    rng = np.random.default_rng(64)
    a, b = rng.standard_normal(m.nq), rng.standard_normal(m.nq)
    w = mg.lognormal_field(m.nq, 65)
    plan = femasm.Plan(_t(m.me), m.nq)
    gw, gq = plan.backward(_t(m.q), _t(w), _t(a), _t(b))
    plan.sync_status()
    J, ow, oq, aw, aq = oracle.grad(m.q, m.me, w, a, b, with_abs=True)
    ew = _floored(gw.cpu().numpy(), ow, aw)
    eq = _floored(gq.cpu().numpy(), oq, aq)
    print(f"{which}: dJ/dw err {ew:.2e}  dJ/dq err {eq:.2e}")
    assert ew <= 1e-12 and eq <= 1e-12
    # J itself through the forward kernels
    Jt = bilinear_energy(_t(m.q), _t(w), _t(a), _t(b), plan)
    assert abs(Jt.item() - J) <= 1e-12 * (abs(J) + 1)


def test_autograd_function():
    m = mg.kuhn_cube(5, 0.15, seed=71)
    rng = np.random.default_rng(72)
    a, b = _t(rng.standard_normal(m.nq)), _t(rng.standard_normal(m.nq))
    plan = femasm.Plan(_t(m.me), m.nq)
    q = _t(m.q).requires_grad_(True)
    w = _t(mg.lognormal_field(m.nq, 73)).requires_grad_(True)
    J = bilinear_energy(q, w, a, b, plan)
    gq, gw = torch.autograd.grad(J * 2.0, (q, w))
    rw, rq = plan.backward(q.detach(), w.detach(), a, b)
    assert torch.equal(gq, 2.0 * rq) and torch.equal(gw, 2.0 * rw)


def _star(m, i):
    ks = np.flatnonzero((m.me == i).any(axis=0))
    verts = np.unique(m.me[:, ks])
    loc = {v: j for j, v in enumerate(verts)}
    me_loc = np.vectorize(loc.get)(m.me[:, ks]).astype(np.int32)
    return verts, me_loc, loc[i]


def _J_star(plan, q_loc, w_loc, a_loc, b_loc, ops):
    J = 0.0
    for op in ops:
        v = plan.numeric(op, _t(q_loc), _t(w_loc))
        J += plan.bilinear(op, v, _t(a_loc), _t(b_loc)).item()
    return J


@pytest.fixture(scope="module")
def adjoint_case():
    c = mg.config_adjoint()
    m = c["mesh"]
    plan = femasm.Plan(_t(m.me), m.nq)
    gw, gq = plan.backward(_t(m.q), _t(c["w"]), _t(c["a"]), _t(c["b"]))
    plan.sync_status()
    return c, gw.cpu().numpy(), gq.cpu().numpy()


def test_adjoint_full_size_vs_oracle_stars(adjoint_case):
    c, gw, gq = adjoint_case
    m = c["mesh"]
    assert m.nme == 998250 and m.nq == 175616
    rng = np.random.default_rng(56)
    worst = 0.0
    for i in rng.choice(m.nq, 40, replace=False):
        verts, me_loc, il = _star(m, i)
        J, ow, oq, aw, aq = oracle.grad(m.q[:, verts], me_loc, c["w"][verts], c["a"][verts],
                                         c["b"][verts], with_abs=True)
        worst = max(worst, _floored(np.array([gw[i]]), np.array([ow[il]]), np.array([aw[il]])))
        worst = max(worst, _floored(gq[:, i], oq[:, il], aq[:, il]))
    print(f"full-size adjoint vs oracle (40 stars): worst floored err {worst:.2e}")
    assert worst <= 1e-12


def test_adjoint_full_size_vs_finite_differences(adjoint_case):
    c, gw, gq = adjoint_case
    m = c["mesh"]
    rng = np.random.default_rng(c["fd_seed"])
    h = 1e-6
    gmax_w, gmax_q = np.abs(gw).max(), np.abs(gq).max()
    entries = rng.integers(0, 4 * m.nq, size=100)      # 0..nq-1 -> w_i, else q_(v,i)
    worst = 0.0
    for e in entries:
        kind, i = divmod(int(e), m.nq)
        verts, me_loc, il = _star(m, i)
        plan = femasm.Plan(_t(me_loc), len(verts))
        ql, wl = m.q[:, verts].copy(), c["w"][verts].copy()
        al, bl = c["a"][verts], c["b"][verts]
        if kind == 0:
            wp, wm = wl.copy(), wl.copy()
            wp[il] += h
            wm[il] -= h
            fd = (_J_star(plan, ql, wp, al, bl, ["MASS_W"]) -
                  _J_star(plan, ql, wm, al, bl, ["MASS_W"])) / (2 * h)
            g, gmax = gw[i], gmax_w
        else:
            v = kind - 1
            qp, qm = ql.copy(), ql.copy()
            qp[v, il] += h
            qm[v, il] -= h
            fd = (_J_star(plan, qp, wl, al, bl, ["STIFF", "MASS_W"]) -
                  _J_star(plan, qm, wl, al, bl, ["STIFF", "MASS_W"])) / (2 * h)
            g, gmax = gq[v, i], gmax_q
        rel = abs(g - fd) / max(abs(fd), 1e-3 * gmax)
        worst = max(worst, rel)
        assert rel <= 1e-6, (kind, i, g, fd, rel)
    print(f"adjoint vs central FD (100 entries): worst {worst:.2e}")
