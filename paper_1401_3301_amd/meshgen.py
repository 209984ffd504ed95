"""Seeded synthetic P1 meshes and nodal fields.

This module only builds inputs: vertex coordinates ``q`` (shape ``(d, nq)``,
float64, C-contiguous, so ``q[v, j]`` is coordinate ``v`` of vertex ``j``),
connectivity ``me`` (shape ``(d+1, nme)``, int32, 0-based, ``me[a, k]`` is
local vertex ``a`` of element ``k``) and random nodal fields.  It holds none
of the assembly arithmetic (no volumes, gradients or element matrices), so the
CPU oracle and the GPU library can both consume its output without sharing
any part of the method.

The paper benchmarks on unit-disk and unit-ball meshes whose generator it does
not give (Section 6); these jittered grids stand in for them with the same
element/vertex ratios (about 2 in 2D and 6 in 3D).

Rules (all seeds feed ``numpy.random.default_rng``):

* 2D ``jittered_square(n, jit, seed)``: ``(n+1)^2`` vertices on the unit
  square, vertex id ``j*(n+1)+i`` at ``(i*h, j*h)``, ``h = 1/n``.  Draw order
  from one generator: first the per-vertex jitter (uniform in
  ``[-jit*h, jit*h)`` for x then y), applied to interior vertices only, then
  one Bernoulli(1/2) diagonal choice per cell (cells in row-major order).
  Cell ``(i, j)`` with corners a=(i,j), b=(i+1,j), c=(i+1,j+1), e=(i,j+1)
  gives triangles (a,b,c),(a,c,e) for choice 0 and (a,b,e),(b,c,e) for
  choice 1; elements are numbered cell by cell.
* 3D ``kuhn_cube(n, jit, seed)``: ``(n+1)^3`` vertices on the unit cube, id
  ``(k*(n+1)+j)*(n+1)+i``; the jitter is drawn as in 2D (x, y, z).  Each cube
  is split into the 6 Kuhn tetrahedra, one per permutation (p0,p1,p2) of the
  axes, with vertices c, c+e_p0, c+e_p0+e_p1, c+(1,1,1); the permutations are
  taken in lexicographic order, elements cube by cube (cubes in id order).
  ``perm_seed`` optionally permutes the element order (columns of ``me``).
* ``delaunay_mesh(d, npts, seed)``: Delaunay triangulation of random
  points (unstructured meshes, vertex valence up to several tens).
* P_k meshes ``pk_mesh(mesh, k)`` (Appendix D): the nodal points of P_k
  Lagrange elements on the straight simplices of a P1 mesh.  Local node
  ``I(alpha)`` of an element is the multi-index ``alpha`` in N^(d+1),
  ``|alpha| = k`` (``alpha_i`` pairs with local vertex ``i``): indices
  ``0..d`` are the vertices ``alpha = k e_i``, the others follow in
  decreasing lexicographic order of ``(alpha_0, ..., alpha_d)``.  The node of
  ``alpha`` lies at ``sum_i alpha_i P_i / k``.  Global ids: the P1 vertices
  keep theirs; every other node is identified by its support (the vertices
  with ``alpha_i > 0`` and their exponents), so neighbouring elements share
  it, and numbered after the vertices in increasing order of that support
  (smallest vertex id first).  Its coordinates are those computed by the
  lowest-numbered element that has it.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Mesh", "jittered_square", "kuhn_cube", "lognormal_field", "normal_field",
    "config_small_2d", "config_large_2d", "config_large_3d", "config_batch",
    "config_adjoint", "interior_mask", "pk_local_indices", "pk_mesh", "config_pk",
    "boundary_facets",
]


@dataclass
class Mesh:
    d: int
    q: np.ndarray          # (d, nq) float64
    me: np.ndarray         # (d+1, nme) int32
    n: int = 0             # grid cells per side
    meta: dict = field(default_factory=dict)

    @property
    def nq(self) -> int:
        return int(self.q.shape[1])

    @property
    def nme(self) -> int:
        return int(self.me.shape[1])


def _jitter(rng, d, n, jit):
    nq = (n + 1) ** d
    h = 1.0 / n
    # one block of draws: (d, nq), x row first
    delta = rng.uniform(-jit * h, jit * h, size=(d, nq)) if jit > 0 else np.zeros((d, nq))
    return delta


def interior_mask(d: int, n: int) -> np.ndarray:
    """Boolean mask of vertices strictly inside the unit square/cube."""
    idx = np.arange(n + 1)
    inner = (idx > 0) & (idx < n)
    if d == 2:
        m = inner[None, :] & inner[:, None]          # [j, i]
    else:
        m = inner[None, None, :] & inner[None, :, None] & inner[:, None, None]  # [k, j, i]
    return m.reshape(-1)


def jittered_square(n: int, jit: float = 0.0, seed: int = 0,
                    diagonals: str = "random") -> Mesh:
    """2D jittered grid; ``diagonals`` is 'random' (seeded), 'up' (a-c) or 'down' (b-e)."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    i = np.tile(np.arange(n + 1), n + 1)
    j = np.repeat(np.arange(n + 1), n + 1)
    q = np.stack([i * h, j * h]).astype(np.float64)
    delta = _jitter(rng, 2, n, jit)
    mask = interior_mask(2, n)
    q[:, mask] += delta[:, mask]
    if diagonals == "random":
        choice = rng.integers(0, 2, size=n * n)
    elif diagonals == "up":
        choice = np.zeros(n * n, dtype=np.int64)
    elif diagonals == "down":
        choice = np.ones(n * n, dtype=np.int64)
    else:
        raise ValueError(diagonals)
    ci = np.tile(np.arange(n), n)
    cj = np.repeat(np.arange(n), n)
    a = cj * (n + 1) + ci
    b = a + 1
    c = a + (n + 1) + 1
    e = a + (n + 1)
    t0 = np.where(choice == 0, np.stack([a, b, c]), np.stack([a, b, e]))
    t1 = np.where(choice == 0, np.stack([a, c, e]), np.stack([b, c, e]))
    me = np.empty((3, 2 * n * n), dtype=np.int32)
    me[:, 0::2] = t0
    me[:, 1::2] = t1
    return Mesh(2, np.ascontiguousarray(q), me, n, {"jit": jit, "seed": seed})


def kuhn_cube(n: int, jit: float = 0.0, seed: int = 0,
              perm_seed: int | None = None) -> Mesh:
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    n1 = n + 1
    i = np.tile(np.arange(n1), n1 * n1)
    j = np.tile(np.repeat(np.arange(n1), n1), n1)
    k = np.repeat(np.arange(n1), n1 * n1)
    q = np.stack([i * h, j * h, k * h]).astype(np.float64)
    delta = _jitter(rng, 3, n, jit)
    mask = interior_mask(3, n)
    q[:, mask] += delta[:, mask]
    ci = np.tile(np.arange(n), n * n)
    cj = np.tile(np.repeat(np.arange(n), n), n)
    ck = np.repeat(np.arange(n), n * n)
    base = (ck * n1 + cj) * n1 + ci
    step = (1, n1, n1 * n1)           # id offsets of unit steps in x, y, z
    perms = list(itertools.permutations(range(3)))
    me = np.empty((4, 6 * n ** 3), dtype=np.int32)
    for t, p in enumerate(perms):
        v1 = base + step[p[0]]
        v2 = v1 + step[p[1]]
        v3 = base + 1 + n1 + n1 * n1
        me[0, t::6] = base
        me[1, t::6] = v1
        me[2, t::6] = v2
        me[3, t::6] = v3
    meta = {"jit": jit, "seed": seed, "perm_seed": perm_seed}
    if perm_seed is not None:
        perm = np.random.default_rng(perm_seed).permutation(me.shape[1])
        me = np.ascontiguousarray(me[:, perm])
    return Mesh(3, np.ascontiguousarray(q), me, n, meta)


def pk_local_indices(d: int, k: int) -> list[tuple[int, ...]]:
    """Local numbering of the P_k nodes of a d-simplex: the list of multi-indices
    alpha (length d+1, sum k), vertices first, then decreasing lexicographic."""
    if k < 1:
        raise ValueError("k >= 1")
    allm = [a for a in itertools.product(range(k, -1, -1), repeat=d + 1) if sum(a) == k]
    verts = [tuple(k if i == v else 0 for i in range(d + 1)) for v in range(d + 1)]
    rest = [a for a in allm if a not in verts]     # product order is decreasing lex
    return verts + rest


def pk_mesh(mesh: Mesh, k: int) -> Mesh:
    """P_k mesh on the simplices of the P1 mesh ``mesh`` (rules in the module
    docstring).  ``me`` has shape (n_dfe, nme), n_dfe = (d+k)!/(d! k!)."""
    d, nq1, nme = mesh.d, mesh.nq, mesh.nme
    loc = pk_local_indices(d, k)
    ndfe = len(loc)
    me1 = mesh.me.astype(np.int64)
    big = np.iinfo(np.int64).max
    # support key of every (element, non-vertex local node): (vertex, exponent)
    # pairs sorted by vertex id, padded with (big, 0)
    keys = np.full((ndfe - d - 1, nme, 2 * (d + 1)), big, dtype=np.int64)
    for r, a in enumerate(loc[d + 1:]):
        verts = np.where(np.array(a)[:, None] > 0, me1, big)          # (d+1, nme)
        expo = np.broadcast_to(np.array(a, dtype=np.int64)[:, None], (d + 1, nme))
        order = np.argsort(verts, axis=0, kind="stable")
        vs = np.take_along_axis(verts, order, axis=0)
        es = np.take_along_axis(expo, order, axis=0)
        es = np.where(vs == big, 0, es)
        keys[r, :, 0::2] = vs.T
        keys[r, :, 1::2] = es.T
    flat = keys.reshape(-1, 2 * (d + 1))
    uniq, inv = np.unique(flat, axis=0, return_inverse=True)
    inv = inv.reshape(ndfe - d - 1, nme)
    nq = nq1 + len(uniq)
    me = np.empty((ndfe, nme), dtype=np.int32)
    me[:d + 1] = mesh.me
    me[d + 1:] = nq1 + inv
    q = np.empty((d, nq), dtype=np.float64)
    q[:, :nq1] = mesh.q
    # first element (lowest number) holding each new node, and its local row
    flat_id = inv.ravel()
    elem_of = np.tile(np.arange(nme), ndfe - d - 1)
    row_of = np.repeat(np.arange(ndfe - d - 1), nme)
    first = np.full(len(uniq), np.iinfo(np.int64).max)
    np.minimum.at(first, flat_id, elem_of * (ndfe - d - 1) + row_of)
    fe, fr = first // (ndfe - d - 1), first % (ndfe - d - 1)
    for r, a in enumerate(loc[d + 1:]):
        sel = fr == r
        if not np.any(sel):
            continue
        e = fe[sel]
        pts = np.zeros((d, len(e)))
        for i in range(d + 1):
            if a[i]:
                pts += a[i] * mesh.q[:, mesh.me[i, e]]
        q[:, nq1 + np.nonzero(sel)[0]] = pts / k
    meta = dict(mesh.meta)
    meta["k"] = k
    return Mesh(d, np.ascontiguousarray(q), me, mesh.n, meta)


def boundary_facets(mesh: Mesh) -> np.ndarray:
    """The (d-1)-simplices that belong to exactly one element (the boundary of
    a conforming mesh), as a (d, nf) int32 array; each facet lists its
    vertices in ascending id, facets in ascending order of that tuple."""
    d, me = mesh.d, mesh.me.astype(np.int64)
    faces = []
    for drop in range(d + 1):
        keep = [a for a in range(d + 1) if a != drop]
        faces.append(np.sort(me[keep].T, axis=1))
    f = np.concatenate(faces)
    uniq, cnt = np.unique(f, axis=0, return_counts=True)
    return np.ascontiguousarray(uniq[cnt == 1].T.astype(np.int32))


def delaunay_mesh(d: int, npts: int, seed: int, perm_seed: int | None = None,
                  morton: bool = True) -> Mesh:
    """Unstructured mesh: the Delaunay triangulation (scipy / Qhull) of
    ``npts`` uniform random points in the unit square or cube (seeded).  With
    ``morton`` the points are numbered along a Morton (Z-order) curve of
    their coordinates quantised to 2^16 (2D) or 2^10 (3D) cells per axis --
    the locality order a mesh generator would give them; ``perm_seed``
    optionally permutes the element order."""
    from scipy.spatial import Delaunay
    rng = np.random.default_rng(seed)
    pts = rng.random((npts, d))
    if morton:
        bits = 16 if d == 2 else 10
        cell = np.minimum((pts * (1 << bits)).astype(np.int64), (1 << bits) - 1)
        code = np.zeros(npts, np.int64)
        for b in range(bits):
            for x in range(d):
                code |= ((cell[:, x] >> b) & 1) << (b * d + x)
        pts = pts[np.argsort(code, kind="stable")]
    me = Delaunay(pts).simplices.T.astype(np.int32)
    if perm_seed is not None:
        me = me[:, np.random.default_rng(perm_seed).permutation(me.shape[1])]
    return Mesh(d, np.ascontiguousarray(pts.T), np.ascontiguousarray(me))


def lognormal_field(nq: int, seed: int, sigma: float = 0.5) -> np.ndarray:
    """Nodal weight w_i = exp(sigma * Z_i), Z ~ N(0,1) (median 1)."""
    z = np.random.default_rng(seed).standard_normal(nq)
    return np.exp(sigma * z)


def normal_field(nq: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(nq)


# ---------------------------------------------------------------------------
# Workload presets.  Each returns plain arrays; sizes are exact for the rules
# above.
# ---------------------------------------------------------------------------

def config_small_2d() -> dict:
    """2D mass + stiffness, 64x64 cells, random diagonals, jitter 0.2h."""
    m = jittered_square(64, 0.2, seed=1)
    return {"name": "square64_2d", "mesh": m, "ops": ("MASS", "STIFF")}


def config_large_2d() -> dict:
    """2D stiffness / weighted mass / elasticity on 2048x2048 cells."""
    m = jittered_square(2048, 0.2, seed=2)
    w = lognormal_field(m.nq, seed=21)
    return {"name": "square2048_2d", "mesh": m, "w": w, "lam": 1.0, "mu": 0.5,
            "ops": ("STIFF", "MASS_W", "ELAS")}


def config_large_3d(n: int = 128) -> dict:
    """3D stiffness / elasticity, 128^3 cubes x 6 Kuhn tets, permuted elements."""
    m = kuhn_cube(n, 0.15, seed=3, perm_seed=33)
    return {"name": f"cube{n}_3d_perm", "mesh": m, "lam": 1.0, "mu": 0.5,
            "ops": ("STIFF", "ELAS")}


def batch_sizes(count: int = 256, seed: int = 4, lo: float = 1e3, hi: float = 2e5):
    """Target element counts log-uniform in [lo, hi] and the grid sizes that
    realise them (first half 2D, second half 3D)."""
    rng = np.random.default_rng(seed)
    e = np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))
    dims, ns = [], []
    for b in range(count):
        if b < count // 2:
            dims.append(2)
            ns.append(max(1, int(round(math.sqrt(e[b] / 2.0)))))
        else:
            dims.append(3)
            ns.append(max(1, int(round((e[b] / 6.0) ** (1.0 / 3.0)))))
    return dims, ns


def config_batch(count: int = 256, seed: int = 4) -> dict:
    """256 independent meshes, half triangles / half tets, own seeds and w."""
    dims, ns = batch_sizes(count, seed)
    meshes, ws = [], []
    for b in range(count):
        if dims[b] == 2:
            m = jittered_square(ns[b], 0.2, seed=4000 + b)
        else:
            m = kuhn_cube(ns[b], 0.15, seed=4000 + b)
        meshes.append(m)
        ws.append(lognormal_field(m.nq, seed=5000 + b))
    return {"name": f"batch{count}_mixed", "meshes": meshes, "w": ws,
            "ops": ("MASS_W", "STIFF")}


def config_pk(k: int, n: int, jit: float = 0.15, seed: int = 6) -> dict:
    """3D P_k mass (Appendix D, Table D.1): P_k nodes on a jittered Kuhn cube
    of n^3 cubes, elements in cube order."""
    m = pk_mesh(kuhn_cube(n, jit, seed=seed), k)
    return {"name": f"cube{n}_3d_p{k}", "mesh": m, "k": k, "ops": ("MASS",)}


def config_adjoint(n: int = 55) -> dict:
    """3D Kuhn cube (about 1M tets) with a, b ~ N(0,1) and lognormal w."""
    m = kuhn_cube(n, 0.15, seed=5)
    a = normal_field(m.nq, 51)
    b = normal_field(m.nq, 52)
    w = lognormal_field(m.nq, 53)
    return {"name": f"cube{n}_3d_adjoint", "mesh": m, "a": a, "b": b, "w": w,
            "fd_seed": 55}
