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
