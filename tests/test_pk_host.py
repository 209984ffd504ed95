"""CPU checks of the library's host-side P_k plan (pk_host.h).

The CSR pattern, the per-tile element lists and the per-entry contribution
items are compared with a brute force over the P_k mesh; the library's C
(its own evaluation of the formula of Appendix D) with the oracle's; and the
sum the kernel performs, replayed here in numpy on the library's layout,
with the oracle's assembled matrix.
"""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
from helpers import floored_err
from paper_1401_3301_amd import meshgen as mg

HERE = os.path.dirname(os.path.abspath(__file__))
TILE = 1024


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("pkshim") / "pk_host_shim.so")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-pthread",
                           os.path.join(HERE, "pk_host_shim.cpp"), "-o", out])
    return ctypes.CDLL(out)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _build(shim, m, k):
    me = np.ascontiguousarray(m.me, np.int32)
    sizes = np.zeros(6, np.int64)
    st = shim.pkh_build(m.d, k, ctypes.c_int64(m.nq), ctypes.c_int64(m.nme), _p(me), _p(sizes))
    if st:
        return st, None
    nnz, ntiles, nitems, ebits, ntri, _ = (int(x) for x in sizes)
    L = dict(rp=np.zeros(m.nq + 1, np.int32), ci=np.zeros(nnz, np.int32),
             tile_item=np.zeros(ntiles + 1, np.int64), coff=np.zeros(ntiles * TILE, np.uint16),
             item=np.zeros(nitems, np.uint32), ctri=np.zeros(ntri), ebits=ebits)
    shim.pkh_get(*(_p(L[x]) for x in ("rp", "ci", "tile_item", "coff", "item", "ctri")))
    return 0, L


def _tri(n, a, b):
    lo, hi = min(a, b), max(a, b)
    return lo * n - lo * (lo - 1) // 2 + (hi - lo)


def _entry_items(L, s, nnz):
    t = s // TILE
    i0 = L["tile_item"][t]
    c0 = int(L["coff"][s])
    c1 = int(L["coff"][s + 1]) if (s + 1) % TILE and s + 1 < nnz else int(L["tile_item"][t + 1] - i0)
    it = L["item"][i0 + c0:i0 + c1].astype(np.int64)
    eb = L["ebits"]
    return it & ((1 << eb) - 1), it >> eb


CASES = [(2, 2, 3), (2, 3, 2), (2, 5, 1), (3, 2, 2), (3, 3, 1), (3, 1, 2),
         # more than 4096 nodes: the builder's multi-threaded row passes
         (2, 2, 33), (3, 1, 16)]


@pytest.mark.parametrize("d,k,n", CASES)
def test_layout_against_brute_force(shim, d, k, n):
    m1 = mg.jittered_square(n, 0.2, seed=3) if d == 2 else mg.kuhn_cube(n, 0.1, seed=4, perm_seed=5)
    m = mg.pk_mesh(m1, k)
    st, L = _build(shim, m, k)
    assert st == 0
    N = m.me.shape[0]
    # brute force: contributions of each (i, j) in ascending element order
    contrib = {}
    for e in range(m.nme):
        for a in range(N):
            for b in range(N):
                contrib.setdefault((int(m.me[a, e]), int(m.me[b, e])), []).append((e, _tri(N, a, b)))
    rows = {}
    for (i, j) in contrib:
        rows.setdefault(i, []).append(j)
    rp, ci = L["rp"], L["ci"]
    nnz = len(ci)
    assert nnz == len(contrib)
    for i in range(m.nq):
        assert list(ci[rp[i]:rp[i + 1]]) == sorted(rows.get(i, []))
    for s in range(nnz):
        i = int(np.searchsorted(rp, s, side="right") - 1)
        els, codes = _entry_items(L, s, nnz)
        assert list(zip(els.tolist(), codes.tolist())) == contrib[(i, int(ci[s]))]
    assert L["ebits"] == 32 - math.ceil(math.log2(N * (N + 1) // 2))


@pytest.mark.parametrize("d,k", [(d, k) for d in (2, 3) for k in range(1, 7)])
def test_library_coefficients_match_oracle(shim, d, k):
    m = mg.pk_mesh(mg.jittered_square(1) if d == 2 else mg.kuhn_cube(1), k)
    st, L = _build(shim, m, k)
    assert st == 0
    C = oracle.pk_coeff(d, k)
    N = C.shape[0]
    iu = np.triu_indices(N)
    np.testing.assert_allclose(L["ctri"], C[iu], rtol=1e-15, atol=1e-18)


@pytest.mark.parametrize("d,k,n", [(2, 3, 4), (3, 2, 3)])
def test_kernel_sum_replayed_on_cpu(shim, d, k, n):
    """The sum k_pk_mass performs (products |det B_K| * C added in item
    order) replayed in numpy on the library layout equals the oracle."""
    m1 = mg.jittered_square(n, 0.2, seed=8) if d == 2 else mg.kuhn_cube(n, 0.15, seed=9)
    m = mg.pk_mesh(m1, k)
    st, L = _build(shim, m, k)
    assert st == 0
    P = np.stack([m.q[:, m.me[a]] for a in range(d + 1)])       # (d+1, d, nme)
    B = np.stack([P[a] - P[0] for a in range(1, d + 1)], axis=1)  # (d, d, nme)
    vol = np.abs(np.linalg.det(np.moveaxis(B, -1, 0)))
    nnz = len(L["ci"])
    val = np.zeros(nnz)
    for s in range(nnz):
        els, codes = _entry_items(L, s, nnz)
        acc = 0.0
        for e, c in zip(els, codes):
            acc += vol[e] * L["ctri"][c]
        val[s] = acc
    rp, ci, v, av = oracle.pk_mass(m.q, m.me, k)
    assert np.array_equal(rp, L["rp"]) and np.array_equal(ci, L["ci"])
    assert floored_err(val, v, av) < 1e-13


def test_refusals(shim):
    m = mg.pk_mesh(mg.jittered_square(2), 2)
    bad = m.me.copy()
    bad[3, 1] = bad[0, 1]
    assert _build(shim, mg.Mesh(2, m.q, bad), 2)[0] == 2
    bad = m.me.copy()
    bad[5, 0] = m.nq
    assert _build(shim, mg.Mesh(2, m.q, bad), 2)[0] == 2


@pytest.mark.parametrize("d", [2, 3])
def test_boundary_facet_layout(shim, d):
    """Boundary facets ((d-1)-simplices, k = 1): pattern and items against a
    brute force, and C of the segment / triangle mass."""
    m1 = mg.jittered_square(5, 0.2, seed=6) if d == 2 else mg.kuhn_cube(3, 0.1, seed=7)
    f = mg.boundary_facets(m1)
    fm = mg.Mesh(d - 1, m1.q, f)
    me = np.ascontiguousarray(f, np.int32)
    sizes = np.zeros(6, np.int64)
    st = shim.pkh_build(d - 1, 1, ctypes.c_int64(m1.nq), ctypes.c_int64(f.shape[1]), _p(me),
                        _p(sizes))
    assert st == 0
    nnz, ntiles, nitems, ebits, ntri, _ = (int(x) for x in sizes)
    L = dict(rp=np.zeros(m1.nq + 1, np.int32), ci=np.zeros(nnz, np.int32),
             tile_item=np.zeros(ntiles + 1, np.int64), coff=np.zeros(ntiles * TILE, np.uint16),
             item=np.zeros(nitems, np.uint32), ctri=np.zeros(ntri), ebits=ebits)
    shim.pkh_get(*(_p(L[x]) for x in ("rp", "ci", "tile_item", "coff", "item", "ctri")))
    N = d
    contrib = {}
    for e in range(f.shape[1]):
        for a in range(N):
            for b in range(N):
                contrib.setdefault((int(f[a, e]), int(f[b, e])), []).append((e, _tri(N, a, b)))
    assert nnz == len(contrib)
    for s in range(nnz):
        i = int(np.searchsorted(L["rp"], s, side="right") - 1)
        els, codes = _entry_items(L, s, nnz)
        assert list(zip(els.tolist(), codes.tolist())) == contrib[(i, int(L["ci"][s]))]
    n = d - 1
    C = (1 + np.eye(N)) / math.factorial(n + 2)
    np.testing.assert_allclose(L["ctri"], C[np.triu_indices(N)], rtol=1e-15)
    assert fm.nme == f.shape[1]
