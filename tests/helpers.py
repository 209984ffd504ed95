"""Shared test helpers: CSR wrapping and the floored per-entry tolerance."""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# Per-entry bound: |v - v*| <= REL * max(|v*|, sum_of_|contributions|).  A plain
# relative error is ill-posed for entries that cancel to (near) zero, so the
# bound is floored by the magnitude of what was summed into the entry.
REL = 1e-12


def to_scipy(rp, ci, v, n):
    return sp.csr_matrix((v, ci, rp), shape=(n, n))


def floored_err(v, v_ref, absv_ref):
    """Max over entries of |v - v_ref| / max(|v_ref|, absv_ref); 0/0 -> 0."""
    v = np.asarray(v, float)
    v_ref = np.asarray(v_ref, float)
    den = np.maximum(np.abs(v_ref), np.asarray(absv_ref, float))
    num = np.abs(v - v_ref)
    ok0 = (num == 0)
    rel = np.where(ok0, 0.0, num / np.where(den > 0, den, 1.0))
    rel = np.where((den == 0) & ~ok0, np.inf, rel)
    return float(rel.max()) if rel.size else 0.0


def assert_parity(v, v_ref, absv_ref, rel=REL, what=""):
    e = floored_err(v, v_ref, absv_ref)
    assert e <= rel, f"{what}: floored relative error {e:.3e} > {rel:.1e}"
    return e


def plain_rel_err(v, v_ref, absv_ref, floor=1e-8):
    """Plain max relative error |v - v*| / |v*| over the entries whose value is
    not a cancellation residue: |v*| >= floor * (sum of |contributions|)."""
    v = np.asarray(v, float)
    v_ref = np.asarray(v_ref, float)
    keep = np.abs(v_ref) >= floor * np.asarray(absv_ref, float)
    keep &= v_ref != 0
    if not keep.any():
        return 0.0
    return float((np.abs(v[keep] - v_ref[keep]) / np.abs(v_ref[keep])).max())


def oracle_rows_parallel(q, me, op, nrows, w=None, lam=1.0, mu=0.5, nthreads=None, nparts=None):
    """The full oracle CSR, built as contiguous row ranges on host threads.

    Each range is one call of the oracle's row-restricted assembly (the same
    element loop and `sparse` sum, keeping the triplets of its rows); the
    ctypes call releases the GIL, so the ranges run in parallel.  The ranges
    are concatenated in row order, which gives exactly the CSR of a single
    full assembly."""
    import concurrent.futures as cf
    import os

    import oracle

    nt = nthreads or max(1, min(16, os.cpu_count() or 1))
    nparts = nparts or 2 * nt
    bounds = np.linspace(0, nrows, nparts + 1).astype(np.int64)

    def part(i):
        rows = np.arange(bounds[i], bounds[i + 1], dtype=np.int64)
        if len(rows) == 0:
            z = np.zeros(0, np.int64)
            return np.zeros(1, np.int64), z, np.zeros(0), np.zeros(0)
        return oracle.assemble_rows(q, me, op, rows, w=w, lam=lam, mu=mu)

    with cf.ThreadPoolExecutor(nt) as ex:
        parts = list(ex.map(part, range(nparts)))
    rp = np.zeros(nrows + 1, np.int64)
    o = 0
    for i, (prp, _, _, _) in enumerate(parts):
        rp[bounds[i] + 1:bounds[i + 1] + 1] = prp[1:] + o
        o += prp[-1]
    ci = np.concatenate([p[1] for p in parts])
    v = np.concatenate([p[2] for p in parts])
    av = np.concatenate([p[3] for p in parts])
    return rp, ci, v, av
