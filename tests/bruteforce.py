"""Brute-force element matrices by numerical quadrature (test helper).

An independent route to the P1 element matrices, used to pin the oracle on
tiny meshes.  It shares nothing with the oracle's closed forms:

* barycentric coordinates come from solving the (d+1) x (d+1) system
  [1 ... 1; x_0 ... x_d] lambda = [1; x] (numpy.linalg), so their gradients
  are the columns 1..d of the inverse of that matrix;
* integrals are taken with a collapsed (Duffy) tensor Gauss-Legendre rule on
  the reference simplex, exact for the polynomial degrees involved;
* elasticity uses the linearised strain of Section 5.1 written out from its
  tensor definition (eps_ij = (d_j u_i + d_i u_j)/2), the Voigt vector with
  doubled shear strains and the paper's isotropic matrix C;
* assembly uses scipy.sparse's COO -> CSR conversion, which sums duplicate
  (I, J) pairs: the `sparse` primitive of Section 3.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _gauss01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def duffy_rule(d: int, n: int = 5):
    """Points (npts, d) and weights on the reference simplex {x_i >= 0, sum <= 1}."""
    x, w = _gauss01(n)
    if d == 2:
        U, V = np.meshgrid(x, x, indexing="ij")
        WU, WV = np.meshgrid(w, w, indexing="ij")
        pts = np.stack([U, V * (1 - U)], -1).reshape(-1, 2)
        wts = (WU * WV * (1 - U)).reshape(-1)
    else:
        U, V, W = np.meshgrid(x, x, x, indexing="ij")
        WU, WV, WW = np.meshgrid(w, w, w, indexing="ij")
        pts = np.stack([U, V * (1 - U), W * (1 - U) * (1 - V)], -1).reshape(-1, 3)
        wts = (WU * WV * WW * (1 - U) ** 2 * (1 - V)).reshape(-1)
    return pts, wts


def barycentric(P):
    """P: (d+1, d) vertices.  Returns (Minv, absdet) with lambda(x) = Minv @ [1, x]."""
    d = P.shape[1]
    M = np.vstack([np.ones(d + 1), P.T])
    Minv = np.linalg.inv(M)
    return Minv


def voigt_strain(grad_u):
    """grad_u[i, j] = d u_i / d x_j  ->  Voigt vector with doubled shears."""
    d = grad_u.shape[0]
    eps = 0.5 * (grad_u + grad_u.T)
    if d == 2:
        return np.array([eps[0, 0], eps[1, 1], 2 * eps[0, 1]])
    return np.array([eps[0, 0], eps[1, 1], eps[2, 2], 2 * eps[0, 1], 2 * eps[1, 2],
                     2 * eps[0, 2]])


def elasticity_C(d, lam, mu):
    if d == 2:
        C = np.zeros((3, 3))
        C[:2, :2] = lam
        C[0, 0] += 2 * mu
        C[1, 1] += 2 * mu
        C[2, 2] = mu
    else:
        C = np.zeros((6, 6))
        C[:3, :3] = lam
        for i in range(3):
            C[i, i] += 2 * mu
        for i in range(3, 6):
            C[i, i] = mu
    return C


def element_matrix(P, op, wloc=None, lam=1.0, mu=0.5, nquad=5):
    P = np.asarray(P, float)
    d = P.shape[1]
    nl = d + 1
    Minv = barycentric(P)
    grads = Minv[:, 1:]                       # grads[a] = grad lambda_a
    B = (P[1:] - P[0]).T
    jac = abs(np.linalg.det(B))
    pts, wts = duffy_rule(d, nquad)
    X = P[0][None, :] + pts @ B.T             # physical points
    lam_at = (Minv @ np.vstack([np.ones(len(X)), X.T]))   # (nl, npts)
    W = wts * jac
    if op in ("MASS", "MASS_W"):
        wh = np.ones(len(X)) if op == "MASS" else np.asarray(wloc) @ lam_at
        E = np.einsum("ap,bp,p,p->ab", lam_at, lam_at, wh, W)
        return E
    vol = W.sum()
    if op == "STIFF":
        return vol * grads @ grads.T
    # ELAS: row (a, l) = test function lambda_a e_l, column (b, n)
    m = d
    C = elasticity_C(d, lam, mu)
    E = np.zeros((nl * m, nl * m))
    strains = {}
    for a in range(nl):
        for l in range(m):
            gu = np.zeros((d, d))
            gu[l, :] = grads[a]
            strains[(a, l)] = voigt_strain(gu)
    for a in range(nl):
        for l in range(m):
            for b in range(nl):
                for n in range(m):
                    E[a * m + l, b * m + n] = vol * strains[(b, n)] @ C @ strains[(a, l)]
    return E


def assemble(q, me, op, w=None, lam=1.0, mu=0.5):
    """Global CSR via scipy.sparse (duplicates summed by the library)."""
    d = me.shape[0] - 1
    nq = q.shape[1]
    m = d if op == "ELAS" else 1
    I, J, K = [], [], []
    for k in range(me.shape[1]):
        vid = me[:, k]
        P = q[:, vid].T
        wl = None if w is None else w[vid]
        E = element_matrix(P, op, wl, lam, mu)
        for a in range(d + 1):
            for l in range(m):
                for b in range(d + 1):
                    for n in range(m):
                        I.append(m * vid[a] + l)
                        J.append(m * vid[b] + n)
                        K.append(E[a * m + l, b * m + n])
    A = sp.coo_matrix((K, (I, J)), shape=(m * nq, m * nq)).tocsr()
    A.sort_indices()
    return A


def simplex_volumes(q, me):
    d = me.shape[0] - 1
    out = np.empty(me.shape[1])
    for k in range(me.shape[1]):
        P = q[:, me[:, k]].T
        out[k] = abs(np.linalg.det((P[1:] - P[0]).T)) / (2 if d == 2 else 6)
    return out
