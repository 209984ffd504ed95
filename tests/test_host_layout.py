"""CPU checks of the library's host-side layout builders (blocks_host.h).

The vertex-block layout (rows, touched vertices, block elements, 32-bit
incidence records) and the vertex-pair lists built from it (tasks of 64
pairs, entries in ascending element order, packed-triangle codes, mirror
pairs, dummy padding, caps on rows / CSR entries / touched vertices) are
compared with a brute force over the mesh written here in Python.  The
builders are compiled from the library's own header through a small shim.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

from paper_1401_3301_amd import meshgen as mg

HERE = os.path.dirname(os.path.abspath(__file__))
PAD = 0xFFFF
REC_PAD = 0xFFFFFFFF


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("shim") / "host_layout_shim.so")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-pthread",
                           os.path.join(HERE, "host_layout_shim.cpp"), "-o", out])
    return ctypes.CDLL(out)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _pattern(mesh):
    d, nq, nme = mesh.d, mesh.nq, mesh.nme
    me = np.ascontiguousarray(mesh.me, dtype=np.int32)
    nl = d + 1
    r = np.repeat(me, nl, axis=0).ravel()
    c = np.tile(me, (nl, 1)).ravel()
    a = sp.csr_matrix((np.ones(len(r), np.int8), (r, c)), shape=(nq, nq))
    a.sort_indices()
    rp, ci = a.indptr.astype(np.int32), a.indices.astype(np.int32)
    v = me.ravel()
    k = np.tile(np.arange(nme, dtype=np.int32), nl)
    o = np.lexsort((k, v))
    inc_k = np.ascontiguousarray(k[o])
    ip = np.zeros(nq + 1, np.int64)
    ip[1:] = np.cumsum(np.bincount(v, minlength=nq))
    return me, rp, ci, ip, inc_k


def _build(shim, mesh, R, max_pairs=0, max_nodes=0, waves=8, slots=2, tri=False, dedup=True,
           chunk_min=8192, pair_mode=False, max_elems=1023, max_ent=0, max_inc=0):
    me, rp, ci, ip, inc_k = _pattern(mesh)
    sizes = np.zeros(10, np.int64)
    st = shim.hl_build(mesh.d, ctypes.c_int64(mesh.nq), ctypes.c_int64(mesh.nme), _p(me), _p(rp),
                       _p(ci), _p(ip), _p(inc_k), R, ctypes.c_int64(max_pairs), max_nodes, waves,
                       slots, int(tri), int(dedup), ctypes.c_int64(chunk_min), int(pair_mode),
                       max_elems, ctypes.c_int64(max_ent), ctypes.c_int64(max_inc), _p(sizes))
    assert st == 0, f"builder refused the mesh (status {st})"
    nb, nrows, nnodes, nelem, nrec, ntask, nent, _, nleft, nwrec = (int(x) for x in sizes)
    B = dict(rows=np.zeros(nrows, np.int32), row_ptr=np.zeros(nb + 1, np.int32),
             nodes=np.zeros(nnodes, np.int32), node_ptr=np.zeros(nb + 1, np.int32),
             elem=np.zeros(nelem, np.uint16), elem_ptr=np.zeros(nb + 1, np.int32),
             rec=np.zeros(nrec, np.uint32), rec_ptr=np.zeros(nb + 1, np.int64),
             maxdeg=np.zeros(nb, np.int32))
    shim.hl_blocks(*(_p(B[k]) for k in ("rows", "row_ptr", "nodes", "node_ptr", "elem",
                                        "elem_ptr", "rec", "rec_ptr", "maxdeg")))
    Pr = dict(wt=np.zeros(nb * (waves + 1), np.int32), task_cnt=np.zeros(ntask, np.int32),
              task_ent=np.zeros(ntask, np.int64), hdr=np.zeros(ntask * 64, np.uint16),
              hdr2=np.zeros(ntask * 64, np.uint16), ent=np.zeros(nent, np.uint16),
              ent_ptr=np.zeros(nb + 1, np.int64))
    shim.hl_pairs(*(_p(Pr[k]) for k in ("wt", "task_cnt", "task_ent", "hdr", "hdr2", "ent",
                                        "ent_ptr")))
    B["wrec"] = np.zeros(nwrec, np.uint64)
    B["leftover"] = np.zeros(nleft, np.int32)
    Pr["blk_ok"] = np.zeros(nb, np.uint8)
    shim.hl_pair_mode(_p(B["wrec"]), _p(B["leftover"]), _p(Pr["blk_ok"]))
    return (me, rp, ci, ip, inc_k), nb, B, Pr


def _tri(a, b, nl):
    lo, hi = min(a, b), max(a, b)
    return lo * nl - lo * (lo - 1) // 2 + (hi - lo)


def _check(mesh, built, R, max_pairs, max_nodes, waves, slots, tri, dedup, pair_mode=False,
           max_elems=1023, max_inc=0):
    (me, rp, ci, ip, inc_k), nb, B, Pr = built
    d, nq, nme, nl = mesh.d, mesh.nq, mesh.nme, mesh.d + 1
    used = np.diff(rp) > 0
    owner = np.full(nq, -1)
    covered = np.zeros(len(ci), np.int64)
    left = set(int(x) for x in B["leftover"])
    if not pair_mode:
        assert not left
    for v in left:   # a vertex is left over only when it cannot be a block row
        lv = rp[v + 1] - rp[v]
        assert lv > 511 or (max_pairs and lv > max_pairs) or (max_nodes and lv > max_nodes) or \
            ip[v + 1] - ip[v] > max_elems or (max_inc and nl * (ip[v + 1] - ip[v]) > max_inc)
    for b in range(nb):
        rows = B["rows"][B["row_ptr"][b]:B["row_ptr"][b + 1]]
        assert 0 < len(rows) <= R and np.all(np.diff(rows) > 0)
        assert np.all(owner[rows] == -1) and not (set(rows.tolist()) & left)
        owner[rows] = b
        lens = rp[rows + 1] - rp[rows]
        if max_pairs:
            assert lens.sum() <= max_pairs
        if max_inc:   # growth cap: (d+1) x the rows' stars
            assert nl * (ip[rows + 1] - ip[rows]).sum() <= max_inc
        # block elements: every element around a row, ascending
        ks = np.unique(np.concatenate([inc_k[ip[i]:ip[i + 1]] for i in rows]))
        el = B["elem"][4 * B["elem_ptr"][b]:4 * B["elem_ptr"][b + 1]].reshape(-1, 4)[:, :nl]
        assert len(el) == len(ks) <= 1023
        nodes = B["nodes"][B["node_ptr"][b]:B["node_ptr"][b + 1]]
        assert np.array_equal(nodes[:len(rows)], rows)
        halo = nodes[len(rows):]
        assert np.all(np.diff(halo) > 0)
        assert set(np.unique(me[:, ks])) == set(nodes.tolist())
        if max_nodes:
            assert len(nodes) <= max_nodes
        assert np.array_equal(nodes[el], me[:, ks].T)
        # incidence records, interleaved t * nrows + r: 32-bit (record mode)
        # and wide (12-bit column positions, both modes)
        nr, deg = len(rows), B["maxdeg"][b]
        forms = [("wrec", 12, 4095, 0xFFFFFFFFFFFFFFFF)]
        if not pair_mode:
            forms.append(("rec", 5, 31, REC_PAD))
        for key, width, mask, pad in forms:
            rec = B[key][B["rec_ptr"][b]:B["rec_ptr"][b + 1]]
            assert len(rec) == nr * deg
            for r, i in enumerate(rows):
                inc = inc_k[ip[i]:ip[i + 1]]
                for t in range(deg):
                    x = int(rec[t * nr + r])
                    if t >= len(inc):
                        assert x == pad
                        continue
                    k = inc[t]
                    assert x & 1023 == np.searchsorted(ks, k)
                    al = (x >> 10) & 3
                    assert me[al, k] == i
                    cols = ci[rp[i]:rp[i + 1]]
                    for a in range(nl):
                        assert cols[(x >> (12 + width * a)) & mask] == me[a, k]
        # pair tasks: wavefront ranges, headers, entries
        t0s = Pr["wt"][b * (waves + 1):(b + 1) * (waves + 1)]
        if not Pr["blk_ok"][b]:   # beyond a cap: no tasks, its rows are left over
            assert pair_mode and t0s[0] == t0s[-1]
            left |= set(rows.tolist())
            continue
        assert np.all(np.diff(t0s) >= 0) and np.all(np.diff(t0s) <= slots)
        ne_b = len(ks)
        for t in range(t0s[0], t0s[-1]):
            C, base = Pr["task_cnt"][t], Pr["task_ent"][t]
            assert Pr["ent_ptr"][b] <= base and base + 64 * C <= Pr["ent_ptr"][b + 1]
            for j in range(64):
                h = int(Pr["hdr"][t * 64 + j])
                lst = [int(Pr["ent"][base + u * 64 + j]) for u in range(C)]
                if h == PAD:
                    assert all(x == ne_b for x in lst) and Pr["hdr2"][t * 64 + j] == PAD
                    continue
                r, p = h & 127, h >> 7
                i = rows[r]
                col = ci[rp[i] + p]
                covered[rp[i] + p] += 1
                got = [x for x in lst if x != ne_b]
                assert all(x == ne_b for x in lst[len(got):])
                want = []
                for ep, k in enumerate(ks):
                    vs = list(me[:, k])
                    if i in vs and col in vs:
                        a, bb = vs.index(i), vs.index(col)
                        code = (_tri(a, bb, nl) << 10) if tri else ((a << 10) | (bb << 12))
                        want.append(ep | code)
                assert got == want
                h2 = int(Pr["hdr2"][t * 64 + j])
                if h2 != PAD:
                    assert dedup
                    r2, p2 = h2 & 127, h2 >> 7
                    assert r2 > r and rows[r2] == col and ci[rp[col] + p2] == i
                    covered[rp[col] + p2] += 1
                elif dedup:
                    assert not (col in rows and np.searchsorted(rows, col) > r)
    assert np.all((owner[used] >= 0) | np.isin(np.nonzero(used)[0], sorted(left)))
    assert np.all(owner[~used] == -1)
    rows_of = np.repeat(np.arange(nq), np.diff(rp))
    in_left = np.isin(rows_of, sorted(left))
    assert np.all(covered[~in_left] == 1), "every CSR entry is listed or mirrored exactly once"
    assert np.all(covered[in_left] == 0), "rows left over are not in any task"
    return left


CASES = [
    # (mesh, R, max_pairs, max_nodes, waves, slots, tri, dedup[, chunk_min])
    ("square12", 16, 0, 0, 8, 2, False, True),
    ("square12", 16, 512, 64, 8, 2, True, True, 40),      # four id chunks grown in parallel
    ("cube5_perm", 56, 1024, 256, 8, 2, True, True, 50),
    ("square12", 40, 512, 60, 4, 4, True, True),
    ("cube5_perm", 56, 1024, 256, 8, 2, True, True),
    ("cube5_perm", 20, 512, 0, 8, 1, False, False),
    ("cube4", 64, 1024, 70, 8, 2, False, True),
    ("cube4", 8, 0, 0, 4, 1, True, False),
]
MESHES = {
    "square12": lambda: mg.jittered_square(12, 0.2, seed=3),
    "cube5_perm": lambda: mg.kuhn_cube(5, 0.15, seed=4, perm_seed=9),
    "cube4": lambda: mg.kuhn_cube(4, 0.0, seed=0),
}


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-R{c[1]}-p{c[2]}-n{c[3]}-w{c[4]}s{c[5]}"
                                              f"-{'tri' if c[6] else 'ab'}-{'dd' if c[7] else 'nodd'}"
                                              f"{'-chunks' if len(c) > 8 else ''}"
                                              for c in CASES])
def test_layout_against_brute_force(shim, case):
    name, R, max_pairs, max_nodes, waves, slots, tri, dedup = case[:8]
    chunk_min = case[8] if len(case) > 8 else 8192
    mesh = MESHES[name]()
    built = _build(shim, mesh, R, max_pairs, max_nodes, waves, slots, tri, dedup, chunk_min)
    _check(mesh, built, R, max_pairs, max_nodes, waves, slots, tri, dedup)


def test_unused_vertices_and_refusals(shim):
    # a vertex no element uses gets no block; a row longer than 32 entries
    # (a fan of 40 triangles around vertex 0) makes the builder refuse
    q = np.array([[0.0, 1.0, 0.0, 5.0], [0.0, 0.0, 1.0, 5.0]])
    mesh = mg.Mesh(2, q, np.array([[0], [1], [2]], np.int32))
    built = _build(shim, mesh, 16)
    _check(mesh, built, 16, 0, 0, 8, 2, False, True)
    assert built[1] == 1
    n = 40
    ang = np.linspace(0, 2 * np.pi, n, endpoint=False)
    qf = np.vstack([np.r_[0.0, np.cos(ang)], np.r_[0.0, np.sin(ang)]])
    mef = np.array([[0] * n, list(range(1, n + 1)), [j % n + 1 for j in range(1, n + 1)]],
                   np.int32)
    me, rp, ci, ip, inc_k = _pattern(mg.Mesh(2, qf, mef))
    sizes = np.zeros(10, np.int64)
    st = shim.hl_build(2, ctypes.c_int64(n + 1), ctypes.c_int64(n), _p(me), _p(rp), _p(ci),
                       _p(ip), _p(inc_k), 16, ctypes.c_int64(0), 0, 8, 2, 0, 1, ctypes.c_int64(8192),
                       0, 1023, ctypes.c_int64(0), ctypes.c_int64(0), _p(sizes))
    assert st == 1
    # pair mode keeps the mesh: the fan's centre is left over only when its
    # row exceeds a cap (here the 32-entry CSR cap of a block)
    fan = mg.Mesh(2, qf, mef)
    built = _build(shim, fan, 16, max_pairs=32, pair_mode=True, tri=True)
    left = _check(fan, built, 16, 32, 0, 8, 2, True, True, pair_mode=True)
    assert left == {0}
    built = _build(shim, fan, 16, max_pairs=1024, pair_mode=True, tri=True)
    assert _check(fan, built, 16, 1024, 0, 8, 2, True, True, pair_mode=True) == set()


def _delaunay(d, npts, seed):
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(seed)
    pts = rng.random((npts, d))
    me = Delaunay(pts).simplices.T.astype(np.int32)
    me = me[:, rng.permutation(me.shape[1])]
    return mg.Mesh(d, np.ascontiguousarray(pts.T), np.ascontiguousarray(me))


PAIR_CASES = [
    # (mesh, R, max_pairs, max_nodes, tri, max_elems, max_ent, max_inc)
    ("delaunay3d", 64, 1024, 256, True, 700, 8192, 8192),
    ("delaunay3d", 64, 1024, 256, False, 600, 8192, 8192),
    ("delaunay2d", 128, 1024, 256, True, 1023, 8192, 8192),
    ("delaunay3d", 56, 1024, 256, True, 700, 2500, 0),     # blocks beyond the entry cap
    ("delaunay3d", 64, 1024, 256, True, 700, 2500, 2500),  # growth held under it
    ("delaunay3d", 56, 1024, 24, True, 40, 8192, 8192),    # vertices beyond the node and element caps
    ("delaunay3d", 64, 1024, 256, True, 700, 8192, 120),   # stars beyond the growth cap
    ("cube5_perm", 64, 1024, 256, True, 700, 8192, 8192),
]
PAIR_MESHES = {
    "delaunay3d": lambda: _delaunay(3, 600, 5),
    "delaunay2d": lambda: _delaunay(2, 1500, 6),
    "cube5_perm": lambda: mg.kuhn_cube(5, 0.15, seed=4, perm_seed=9),
}


@pytest.mark.parametrize("case", PAIR_CASES, ids=[f"{c[0]}-R{c[1]}-n{c[3]}-e{c[5]}-ent{c[6]}"
                                                  f"-inc{c[7]}" for c in PAIR_CASES])
def test_pair_mode_against_brute_force(shim, case):
    """Pair mode on unstructured meshes (rows up to 511 entries): every CSR
    entry of a block row is listed or mirrored once; vertices beyond a cap and
    the rows of blocks beyond the task or entry caps are left over, and only
    those; with the growth cap (max_inc, as the library sets it) each block's
    rows hold (d+1) x star sizes within it."""
    name, R, max_pairs, max_nodes, tri, max_elems, max_ent, max_inc = case
    mesh = PAIR_MESHES[name]()
    built = _build(shim, mesh, R, max_pairs, max_nodes, 8, 2, tri, True, pair_mode=True,
                   max_elems=max_elems, max_ent=max_ent, max_inc=max_inc)
    left = _check(mesh, built, R, max_pairs, max_nodes, 8, 2, tri, True, pair_mode=True,
                  max_elems=max_elems, max_inc=max_inc)
    nb, Pr = built[1], built[3]
    print(f"{name}: max row {np.diff(built[0][1]).max()}, {nb} blocks, "
          f"{nb - int(Pr['blk_ok'].sum())} over a cap, {len(left)} rows left over")
    if case[6] == 8192 and case[5] >= 600 and case[7] == 8192:
        assert not left   # default caps: every row of these meshes is in a block
    if max_inc == 120:
        assert left   # the mesh has stars above 30 elements


def _unpack_wave_starts(wp, waves):
    return [0] + [(wp >> (6 * (w - 1))) & 63 for w in range(1, waves + 1)]


def test_wave_start_packing(shim):
    # the descriptor's wavefront task starts: a full block of 8 wavefronts x
    # 4 tasks ends at task 32, which must survive the packing, as must every
    # monotone start sequence within that bound and any first task
    shim.hl_pack_wave_starts.restype = ctypes.c_uint64
    rng = np.random.default_rng(11)
    seqs = [np.arange(0, 33, 4), np.zeros(9, int), np.full(9, 7)]
    for _ in range(200):
        inc = rng.integers(0, 5, 8)
        seqs.append(np.concatenate([[0], np.cumsum(inc)]))
    for s in seqs:
        t0 = int(rng.integers(0, 1 << 20))
        wt = np.ascontiguousarray(np.asarray(s) + t0, np.int32)
        wp = shim.hl_pack_wave_starts(_p(wt), 8)
        assert _unpack_wave_starts(wp, 8) == list(np.asarray(s) - s[0]), s
        assert wp < (1 << 48)
    # the starts of a layout the builder made, with 4 tasks per wavefront
    mesh = MESHES["cube5_perm"]()
    built = _build(shim, mesh, 64, 2048, 256, 8, 4, True, True)
    wt = built[3]["wt"].reshape(-1, 9)
    for row in wt:
        wp = shim.hl_pack_wave_starts(_p(np.ascontiguousarray(row)), 8)
        assert _unpack_wave_starts(wp, 8) == list(row - row[0])


@pytest.mark.parametrize("n,nkeys,threads", [(0, 5, 4), (7, 1, 4), (1000, 37, 1), (200_000, 50, 8),
                                             (300_000, 2_000_000, 8), (150_000, 150_001, 3)])
def test_stable_key_sort(shim, n, nkeys, threads):
    # the symbolic phase's parallel counting sort against a stable argsort
    rng = np.random.default_rng(n + nkeys)
    keys = np.ascontiguousarray(rng.integers(0, nkeys, n), np.int64)
    if n > 10:
        keys[: n // 10] = nkeys - 1          # a heavy key and an empty key range
    order = np.zeros(n, np.int64)
    ptr = np.zeros(nkeys + 1, np.int64)
    shim.hl_key_sort(ctypes.c_int64(n), ctypes.c_int64(nkeys), _p(keys), threads, _p(order),
                     _p(ptr))
    assert np.array_equal(order, np.argsort(keys, kind="stable"))
    ref = np.zeros(nkeys + 1, np.int64)
    ref[1:] = np.cumsum(np.bincount(keys, minlength=nkeys))
    assert np.array_equal(ptr, ref)


def test_incidence_order_of_a_mesh(shim):
    # element slots k*(d+1)+a keyed by their vertex: each vertex's incidences
    # in ascending element number, the order the numeric phase sums in
    mesh = mg.kuhn_cube(6, 0.1, seed=3, perm_seed=4)
    nl = mesh.d + 1
    keys = np.ascontiguousarray(mesh.me.T.ravel(), np.int64)    # r = k*nl + a
    order = np.zeros(len(keys), np.int64)
    ptr = np.zeros(mesh.nq + 1, np.int64)
    shim.hl_key_sort(ctypes.c_int64(len(keys)), ctypes.c_int64(mesh.nq), _p(keys), 8, _p(order),
                     _p(ptr))
    for v in range(0, mesh.nq, 7):
        ks = order[ptr[v]:ptr[v + 1]] // nl
        assert np.all(np.diff(ks) > 0)
        assert set(ks.tolist()) == set(np.nonzero((mesh.me == v).any(axis=0))[0].tolist())


@pytest.mark.parametrize("nt,throw_at", [(1, -1), (8, -1), (8, 0), (8, 5), (3, 2)])
def test_run_threads_joins_and_rethrows(shim, nt, throw_at):
    # the builders' thread helper: all indices run and are joined; a worker's
    # exception is rethrown on the calling thread (the entry points turn it
    # into FEM_ERR_NOMEM instead of terminating the process)
    ran = np.zeros(nt, np.int32)
    st = shim.hl_run_threads(nt, throw_at, _p(ran))
    assert st == (1 if throw_at >= 0 else 0)
    assert ran.tolist() == [1] * nt
