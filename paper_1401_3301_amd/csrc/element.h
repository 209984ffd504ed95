// Per-element closed forms of the P1 element matrices, device side.
//
// Geometry (Appendix C.1 of the paper): with B_k = [q^1-q^0, ..., q^d-q^0],
// the barycentric gradients solve B_k^T G_k = [-1 | I_d].  Written with
// cofactors: g_a = c_a / det B_k where
//   d = 2:  c_1 = ( e2.y, -e2.x),  c_2 = (-e1.y,  e1.x)
//   d = 3:  c_1 = e2 x e3,  c_2 = e3 x e1,  c_3 = e1 x e2
// (e_i = q^i - q^0) and c_0 = -(c_1 + ... + c_d); det B_k = e1 . c_1 in 3D.
// |K| = |det| / d!, so the closed forms need a single division per element:
//   stiffness   |K| g_a.g_b          = c_a.c_b / (d! |det|)          (Section 4.2)
//   mass        |K| d!(1+delta)/(d+2)! = |det| (1+delta) / (d+2)!   (magic formula)
//   weighted    |det| (1+delta) (w^s + (w_a + w_b)) / (d+3)!          (Section 4.1)
//   elasticity  [lambda c_al c_bn + mu (delta_ln c_a.c_b + c_an c_bl)] / (d! |det|)
// The elasticity form is the lemma of Section 5.1 with Q^{n,l}, S^{n,l}
// multiplied out: Q^{n,l} picks g_al g_bn, S^{n,l} gives the strain product;
// it is evaluated as a combination of summed outer products (below).
// Every expression is written so that swapping (a,l) with (b,n) yields the
// same operations on swapped operands, which makes each element matrix, and
// therefore the assembled matrix, exactly symmetric.  Contraction of a*b+c
// into fused multiply-adds is switched off and the fused operations are
// spelled out with fma(), so every kernel that includes these routines rounds
// identically (batched and single-mesh values agree bit for bit).
#pragma once

#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

namespace femasm {

template <int D>
struct Elem {
    double c[D + 1][D];  // cofactor vectors
    double det;
};

__device__ __forceinline__ void elem_geometry(const double (&P)[3][2], Elem<2> &E) {
    const double e1x = P[1][0] - P[0][0], e1y = P[1][1] - P[0][1];
    const double e2x = P[2][0] - P[0][0], e2y = P[2][1] - P[0][1];
    E.c[1][0] = e2y;
    E.c[1][1] = -e2x;
    E.c[2][0] = -e1y;
    E.c[2][1] = e1x;
    E.c[0][0] = -(E.c[1][0] + E.c[2][0]);
    E.c[0][1] = -(E.c[1][1] + E.c[2][1]);
    E.det = fma(e1x, e2y, -(e1y * e2x));
}

__device__ __forceinline__ void elem_geometry(const double (&P)[4][3], Elem<3> &E) {
    double e[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int x = 0; x < 3; ++x) e[i][x] = P[i + 1][x] - P[0][x];
    // c_1 = e2 x e3, c_2 = e3 x e1, c_3 = e1 x e2
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double *u = e[(i + 1) % 3];
        const double *v = e[(i + 2) % 3];
        E.c[i + 1][0] = fma(u[1], v[2], -(u[2] * v[1]));
        E.c[i + 1][1] = fma(u[2], v[0], -(u[0] * v[2]));
        E.c[i + 1][2] = fma(u[0], v[1], -(u[1] * v[0]));
    }
#pragma unroll
    for (int x = 0; x < 3; ++x) E.c[0][x] = -(E.c[1][x] + E.c[2][x] + E.c[3][x]);
    E.det = fma(e[0][2], E.c[1][2], fma(e[0][1], E.c[1][1], e[0][0] * E.c[1][0]));
}

// Only the determinant (mass operators).
__device__ __forceinline__ double elem_det(const double (&P)[3][2]) {
    const double e1x = P[1][0] - P[0][0], e1y = P[1][1] - P[0][1];
    const double e2x = P[2][0] - P[0][0], e2y = P[2][1] - P[0][1];
    return fma(e1x, e2y, -(e1y * e2x));
}

__device__ __forceinline__ double elem_det(const double (&P)[4][3]) {
    double e[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int x = 0; x < 3; ++x) e[i][x] = P[i + 1][x] - P[0][x];
    const double c0 = fma(e[1][1], e[2][2], -(e[1][2] * e[2][1]));
    const double c1 = fma(e[1][2], e[2][0], -(e[1][0] * e[2][2]));
    const double c2 = fma(e[1][0], e[2][1], -(e[1][1] * e[2][0]));
    return fma(e[0][2], c2, fma(e[0][1], c1, e[0][0] * c0));
}

template <int D>
__device__ __forceinline__ double cdot(const double (&a)[D], const double (&b)[D]) {
    double s = a[0] * b[0];
#pragma unroll
    for (int x = 1; x < D; ++x) s = fma(a[x], b[x], s);
    return s;
}

// Scaled cofactors for elasticity: ch_a = c_a / sqrt(d! |det|), so that
// ch_al * ch_bn = |K| g_al g_bn.  The lemma of Section 5.1 then reads
//   E[(a,l),(b,n)] = lambda X_ln + mu (delta_ln tr X + X_nl),  X = ch_a ch_b^T,
// and summing X over the elements of a vertex pair before combining needs one
// fused multiply-add per entry and element.  X_ji is exactly X_ij^T (the
// products commute), so the assembled matrix stays exactly symmetric.
template <int D>
__device__ __forceinline__ double elas_scale(double det);
template <>
__device__ __forceinline__ double elas_scale<2>(double det) {
    return 1.0 / sqrt(2.0 * fabs(det));
}
template <>
__device__ __forceinline__ double elas_scale<3>(double det) {
    return 1.0 / sqrt(6.0 * fabs(det));
}

// Final elasticity value of entry (l, n) of a vertex-pair block from the
// summed X (xln = X_ln, xnl = X_nl, tr = X_00 + X_11 [+ X_22] in that order).
__device__ __forceinline__ double elas_combine(double xln, double xnl, double tr, bool diag,
                                               double lam, double mu) {
    return fma(lam, xln, mu * (diag ? tr + xnl : xnl));
}

// Nodal (P1) Lame fields: with per-element means lambda_K = lambda^s/(d+1),
// mu_K = mu^s/(d+1) the sums XL = sum lambda_K X_K, XM = sum mu_K X_K give
// the entry (l, n) of a vertex pair as XL_ln + (tr XM delta_ln + XM_nl).
__device__ __forceinline__ double elas_combine_nodal(double xl_ln, double xm_nl, double trm,
                                                     bool diag) {
    return xl_ln + (diag ? trm + xm_nl : xm_nl);
}

template <int D>
struct Fact {
    static constexpr double dfact = D == 2 ? 2.0 : 6.0;           // d!
    static constexpr double d1fact = D == 2 ? 6.0 : 24.0;         // (d+1)!
    static constexpr double mass_den = D == 2 ? 24.0 : 120.0;     // (d+2)!
    static constexpr double massw_den = D == 2 ? 120.0 : 720.0;   // (d+3)!
};

}  // namespace femasm
