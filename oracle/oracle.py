"""ctypes front end of the C oracle (oracle.c).  TEST INFRASTRUCTURE ONLY.

Inputs are plain numpy arrays in the layouts of the paper's Table of mesh
data (Section 2), 0-based and row-major: q is (d, nq) float64, me is
(d+1, nme) int32.  Outputs are numpy CSR arrays with int64 indices.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OP = {"MASS": 0, "MASS_W": 1, "STIFF": 2, "ELAS": 3}
STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_INDEX", 3: "ERR_DEGENERATE",
          4: "ERR_OVERFLOW", 5: "ERR_NOMEM"}


class OracleError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"oracle {where}: {STATUS.get(code, code)}")
        self.code = code
        self.name = STATUS.get(code, str(code))


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain IEEE double: no fused multiply-add)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = C.CDLL(_LIB)
        P = C.c_void_p
        i64 = C.c_int64
        lib.oracle_validate.argtypes = [C.c_int, i64, i64, P]
        lib.oracle_assemble.argtypes = [C.c_int, i64, i64, P, P, C.c_int, P, C.c_double,
                                        C.c_double, i64, P, P, P, P, P]
        lib.oracle_assemble_rows.argtypes = [C.c_int, i64, i64, P, P, C.c_int, P, C.c_double,
                                             C.c_double, i64, P, i64, P, P, P, P, P]
        lib.oracle_grad.argtypes = [C.c_int, i64, i64, P, P, P, P, P, P, P, P, P, P]
        lib.oracle_element_matrix.argtypes = [C.c_int, C.c_int, P, P, C.c_double, C.c_double, P]
        lib.oracle_assemble_lame.argtypes = [C.c_int, i64, i64, P, P, P, P, i64, P, i64, P, P, P,
                                             P, P]
        lib.oracle_assemble_general.argtypes = [C.c_int, i64, i64, P, P, P, i64, P, i64, P, P, P,
                                                P, P]
        lib.oracle_boundary_mass.argtypes = [C.c_int, i64, i64, P, P, P, i64, P, P, P, P, P]
        lib.oracle_jvp.argtypes = [C.c_int, i64, i64, P, P, C.c_int, P, P, P, i64, P, P, P, P, P]
        lib.oracle_vjp.argtypes = [C.c_int, i64, i64, P, P, C.c_int, P, P, P, P, P, P, P, P, P]
        lib.oracle_pk_coeff.argtypes = [C.c_int, C.c_int, P]
        lib.oracle_pk_alpha.argtypes = [C.c_int, C.c_int, P]
        lib.oracle_pk_mass.argtypes = [C.c_int, C.c_int, i64, i64, P, P, i64, P, P, P, P, P]
        lib.oracle_pk_mass_rows.argtypes = [C.c_int, C.c_int, i64, i64, P, P, i64, P, i64, P,
                                            P, P, P, P]
        for f in (lib.oracle_validate, lib.oracle_assemble, lib.oracle_assemble_rows,
                  lib.oracle_grad, lib.oracle_element_matrix, lib.oracle_pk_coeff,
                  lib.oracle_pk_alpha, lib.oracle_pk_mass, lib.oracle_pk_mass_rows,
                  lib.oracle_assemble_lame, lib.oracle_assemble_general,
                  lib.oracle_boundary_mass, lib.oracle_jvp, lib.oracle_vjp):
            f.restype = C.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _mesh_arrays(q, me):
    q = np.ascontiguousarray(q, dtype=np.float64)
    me = np.ascontiguousarray(me, dtype=np.int32)
    d = me.shape[0] - 1
    return d, q, me


def validate(d: int, nq: int, me) -> int:
    me = np.ascontiguousarray(me, dtype=np.int32)
    return _load().oracle_validate(d, nq, me.shape[1] if me.ndim == 2 else 0, _ptr(me))


def assemble(q, me, op: str, w=None, lam: float = 1.0, mu: float = 0.5, nq: int | None = None):
    """Full CSR: returns (row_ptr, col_idx, val, absval) with absval the
    per-entry sum of |contribution| (used for the floored tolerance)."""
    d, q, me = _mesh_arrays(q, me)
    nq = q.shape[1] if nq is None else nq
    nme = me.shape[1]
    m = d if op == "ELAS" else 1
    cap = max(1, nme * ((d + 1) * m) ** 2)
    rp = np.zeros(m * nq + 1, np.int64)
    ci = np.zeros(cap, np.int64)
    v = np.zeros(cap, np.float64)
    av = np.zeros(cap, np.float64)
    nnz = C.c_int64(0)
    wv = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    st = _load().oracle_assemble(d, nq, nme, _ptr(q), _ptr(me), OP[op], _ptr(wv), lam, mu, cap,
                                 C.byref(nnz), _ptr(rp), _ptr(ci), _ptr(v), _ptr(av))
    if st:
        raise OracleError(st, "assemble")
    n = nnz.value
    return rp, ci[:n].copy(), v[:n].copy(), av[:n].copy()


def assemble_rows(q, me, op: str, rows, w=None, lam: float = 1.0, mu: float = 0.5):
    """CSR restricted to the global rows listed in ``rows`` (in that order)."""
    d, q, me = _mesh_arrays(q, me)
    nq = q.shape[1]
    nme = me.shape[1]
    m = d if op == "ELAS" else 1
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cap = max(1, len(rows) * 64 * m * m * 4)
    while True:
        rp = np.zeros(len(rows) + 1, np.int64)
        ci = np.zeros(cap, np.int64)
        v = np.zeros(cap, np.float64)
        av = np.zeros(cap, np.float64)
        nnz = C.c_int64(0)
        wv = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        st = _load().oracle_assemble_rows(d, nq, nme, _ptr(q), _ptr(me), OP[op], _ptr(wv), lam,
                                          mu, len(rows), _ptr(rows), cap, C.byref(nnz), _ptr(rp),
                                          _ptr(ci), _ptr(v), _ptr(av))
        if st == 4:
            cap *= 4
            continue
        if st:
            raise OracleError(st, "assemble_rows")
        n = nnz.value
        return rp, ci[:n].copy(), v[:n].copy(), av[:n].copy()


def assemble_lame(q, me, lam, mu, rows=None):
    """Elasticity with nodal Lame fields lam, mu (nq,) as CSR over the d*nq
    dof rows (or only the global dof rows listed in ``rows``)."""
    d, q, me = _mesh_arrays(q, me)
    nq, nme = q.shape[1], me.shape[1]
    lam = np.ascontiguousarray(lam, np.float64)
    mu = np.ascontiguousarray(mu, np.float64)
    rsel = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nout = d * nq if rsel is None else len(rsel)
    cap = max(1, nme * ((d + 1) * d) ** 2) if rsel is None else max(1, len(rsel) * 64 * d * 4)
    while True:
        rp = np.zeros(nout + 1, np.int64)
        ci = np.zeros(cap, np.int64)
        v = np.zeros(cap, np.float64)
        av = np.zeros(cap, np.float64)
        nnz = C.c_int64(0)
        st = _load().oracle_assemble_lame(d, nq, nme, _ptr(q), _ptr(me), _ptr(lam), _ptr(mu),
                                          0 if rsel is None else len(rsel), _ptr(rsel), cap,
                                          C.byref(nnz), _ptr(rp), _ptr(ci), _ptr(v), _ptr(av))
        if st == 4 and rsel is not None:
            cap *= 4
            continue
        if st:
            raise OracleError(st, "assemble_lame")
        n = nnz.value
        return rp, ci[:n].copy(), v[:n].copy(), av[:n].copy()


def general_coef(d, A=None, b=None, c=None, a0=0.0):
    """Packed coefficients [A (d*d, row-major), b (d), c (d), a0]."""
    A = np.zeros((d, d)) if A is None else np.asarray(A, float).reshape(d, d)
    b = np.zeros(d) if b is None else np.asarray(b, float).reshape(d)
    c = np.zeros(d) if c is None else np.asarray(c, float).reshape(d)
    return np.ascontiguousarray(np.concatenate([A.ravel(), b, c, [float(a0)]]))


def assemble_general(q, me, coef, rows=None):
    """General operator -div(A grad u) + div(b u) + c.grad u + a0 u (constant
    coefficients, weak form) as CSR over the nq rows (or the listed rows)."""
    d, q, me = _mesh_arrays(q, me)
    nq, nme = q.shape[1], me.shape[1]
    coef = np.ascontiguousarray(coef, np.float64)
    assert coef.shape == (d * d + 2 * d + 1,)
    rsel = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nout = nq if rsel is None else len(rsel)
    cap = max(1, nme * (d + 1) ** 2) if rsel is None else max(1, len(rsel) * 64)
    while True:
        rp = np.zeros(nout + 1, np.int64)
        ci = np.zeros(cap, np.int64)
        v = np.zeros(cap, np.float64)
        av = np.zeros(cap, np.float64)
        nnz = C.c_int64(0)
        st = _load().oracle_assemble_general(d, nq, nme, _ptr(q), _ptr(me), _ptr(coef),
                                             0 if rsel is None else len(rsel), _ptr(rsel), cap,
                                             C.byref(nnz), _ptr(rp), _ptr(ci), _ptr(v), _ptr(av))
        if st == 4 and rsel is not None:
            cap *= 4
            continue
        if st:
            raise OracleError(st, "assemble_general")
        n = nnz.value
        return rp, ci[:n].copy(), v[:n].copy(), av[:n].copy()


def boundary_mass(q, facets, w=None):
    """Mass (w None) or weighted mass on (d-1)-simplices ``facets`` ((d, nf)
    int32) embedded in R^d; CSR over the nq vertices."""
    q = np.ascontiguousarray(q, np.float64)
    facets = np.ascontiguousarray(facets, np.int32)
    d, nq = q.shape
    nf = facets.shape[1]
    cap = max(1, nf * d * d)
    rp = np.zeros(nq + 1, np.int64)
    ci = np.zeros(cap, np.int64)
    v = np.zeros(cap, np.float64)
    av = np.zeros(cap, np.float64)
    nnz = C.c_int64(0)
    wv = None if w is None else np.ascontiguousarray(w, np.float64)
    st = _load().oracle_boundary_mass(d, nq, nf, _ptr(q), _ptr(facets), _ptr(wv), cap,
                                      C.byref(nnz), _ptr(rp), _ptr(ci), _ptr(v), _ptr(av))
    if st:
        raise OracleError(st, "boundary_mass")
    k = nnz.value
    return rp, ci[:k].copy(), v[:k].copy(), av[:k].copy()


def jvp(q, me, op: str, dq, w=None, dw=None):
    """Directional derivative dA of the assembled operator (MASS, MASS_W or
    STIFF) along (dq, dw), as CSR (row_ptr, col_idx, val, absval)."""
    d, q, me = _mesh_arrays(q, me)
    nq, nme = q.shape[1], me.shape[1]
    dq = np.ascontiguousarray(dq, np.float64)
    wv = None if w is None else np.ascontiguousarray(w, np.float64)
    dwv = None if dw is None else np.ascontiguousarray(dw, np.float64)
    cap = max(1, nme * (d + 1) ** 2)
    rp = np.zeros(nq + 1, np.int64)
    ci = np.zeros(cap, np.int64)
    v = np.zeros(cap, np.float64)
    av = np.zeros(cap, np.float64)
    nnz = C.c_int64(0)
    st = _load().oracle_jvp(d, nq, nme, _ptr(q), _ptr(me), OP[op], _ptr(wv), _ptr(dq), _ptr(dwv),
                            cap, C.byref(nnz), _ptr(rp), _ptr(ci), _ptr(v), _ptr(av))
    if st:
        raise OracleError(st, "jvp")
    n = nnz.value
    return rp, ci[:n].copy(), v[:n].copy(), av[:n].copy()


def vjp(q, me, op: str, rp, ci, G, w=None, vertices=None, want_w=True):
    """Gradient of L = sum_s G_s A_s (A the operator's CSR values on the
    pattern rp, ci) with respect to q (d, nq) and w (nq,); only the listed
    vertices when given.  Returns (dq, dw, dq_abs, dw_abs)."""
    d, q, me = _mesh_arrays(q, me)
    nq, nme = q.shape[1], me.shape[1]
    rp = np.ascontiguousarray(rp, np.int64)
    ci = np.ascontiguousarray(ci, np.int64)
    G = np.ascontiguousarray(G, np.float64)
    wv = None if w is None else np.ascontiguousarray(w, np.float64)
    want = None
    if vertices is not None:
        want = np.zeros(nq, np.uint8)
        want[np.asarray(vertices)] = 1
    dq = np.zeros((d, nq))
    dqa = np.zeros((d, nq))
    dw = np.zeros(nq) if (op == "MASS_W" and want_w) else None
    dwa = np.zeros(nq) if dw is not None else None
    st = _load().oracle_vjp(d, nq, nme, _ptr(q), _ptr(me), OP[op], _ptr(wv), _ptr(rp), _ptr(ci),
                            _ptr(G), _ptr(want), _ptr(dq), _ptr(dw), _ptr(dqa), _ptr(dwa))
    if st:
        raise OracleError(st, "vjp")
    return dq, dw, dqa, dwa


def grad(q, me, w, a, b, want_w: bool = True, want_q: bool = True, with_abs: bool = False):
    """J = a^T (S + M_w) b with dJ/dw (nq,) and dJ/dq (d, nq); with_abs also
    returns the per-entry sums of |element contribution|."""
    d, q, me = _mesh_arrays(q, me)
    nq = q.shape[1]
    w = np.ascontiguousarray(w, np.float64)
    a = np.ascontiguousarray(a, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    J = C.c_double(0.0)
    gw = np.zeros(nq) if want_w else None
    gq = np.zeros((d, nq)) if want_q else None
    aw = np.zeros(nq) if (want_w and with_abs) else None
    aq = np.zeros((d, nq)) if (want_q and with_abs) else None
    st = _load().oracle_grad(d, nq, me.shape[1], _ptr(q), _ptr(me), _ptr(w), _ptr(a), _ptr(b),
                             C.byref(J), _ptr(gw), _ptr(gq), _ptr(aw), _ptr(aq))
    if st:
        raise OracleError(st, "grad")
    if with_abs:
        return J.value, gw, gq, aw, aq
    return J.value, gw, gq


def element_matrix(P, op: str, wloc=None, lam: float = 1.0, mu: float = 0.5):
    """Local matrix of one simplex with vertex coordinates P ((d+1) x d)."""
    P = np.ascontiguousarray(P, np.float64)
    d = P.shape[1]
    m = d if op == "ELAS" else 1
    n = (d + 1) * m
    E = np.zeros((n, n))
    wl = None if wloc is None else np.ascontiguousarray(wloc, np.float64)
    st = _load().oracle_element_matrix(d, OP[op], _ptr(P), _ptr(wl), lam, mu, _ptr(E))
    if st:
        raise OracleError(st, "element_matrix")
    return E


# ---------------------------------------------------------------------------
# P_k Lagrange mass (Appendix D)
# ---------------------------------------------------------------------------

def pk_ndfe(d: int, k: int) -> int:
    """Local P_k nodes of a d-simplex, (d+k)!/(d! k!)."""
    return math.comb(d + k, d)


def pk_alpha(d: int, k: int) -> np.ndarray:
    """Multi-indices of the local nodes, (ndfe, d+1), in the oracle's numbering."""
    out = np.zeros((pk_ndfe(d, k), d + 1), np.int32)
    st = _load().oracle_pk_alpha(d, k, _ptr(out))
    if st:
        raise OracleError(st, "pk_alpha")
    return out


def pk_coeff(d: int, k: int) -> np.ndarray:
    """C with int_K phi_a phi_b = d! |K| C[a, b] (local numbering of pk_alpha)."""
    n = pk_ndfe(d, k)
    out = np.zeros((n, n))
    st = _load().oracle_pk_coeff(d, k, _ptr(out))
    if st:
        raise OracleError(st, "pk_coeff")
    return out


def pk_mass(q, me, k: int, nq: int | None = None):
    """P_k mass matrix as CSR (row_ptr, col_idx, val, absval); me is (ndfe, nme)."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    me = np.ascontiguousarray(me, dtype=np.int32)
    d = q.shape[0]
    nq = q.shape[1] if nq is None else nq
    nme = me.shape[1]
    cap = max(1, nme * me.shape[0] ** 2)
    rp = np.zeros(nq + 1, np.int64)
    ci = np.zeros(cap, np.int64)
    v = np.zeros(cap, np.float64)
    av = np.zeros(cap, np.float64)
    nnz = C.c_int64(0)
    st = _load().oracle_pk_mass(d, k, nq, nme, _ptr(q), _ptr(me), cap, C.byref(nnz), _ptr(rp),
                                _ptr(ci), _ptr(v), _ptr(av))
    if st:
        raise OracleError(st, "pk_mass")
    n = nnz.value
    return rp, ci[:n].copy(), v[:n].copy(), av[:n].copy()


def pk_mass_rows(q, me, k: int, rows):
    """P_k mass matrix restricted to the global rows listed in ``rows``."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    me = np.ascontiguousarray(me, dtype=np.int32)
    d, nq, nme = q.shape[0], q.shape[1], me.shape[1]
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cap = max(1, len(rows) * 256)
    while True:
        rp = np.zeros(len(rows) + 1, np.int64)
        ci = np.zeros(cap, np.int64)
        v = np.zeros(cap, np.float64)
        av = np.zeros(cap, np.float64)
        nnz = C.c_int64(0)
        st = _load().oracle_pk_mass_rows(d, k, nq, nme, _ptr(q), _ptr(me), len(rows), _ptr(rows),
                                         cap, C.byref(nnz), _ptr(rp), _ptr(ci), _ptr(v), _ptr(av))
        if st == 4:
            cap *= 4
            continue
        if st:
            raise OracleError(st, "pk_mass_rows")
        n = nnz.value
        return rp, ci[:n].copy(), v[:n].copy(), av[:n].copy()
