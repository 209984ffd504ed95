/*
 * Plain FP64 CPU oracle for P1 finite-element assembly.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header or table with the GPU library; it is a slow, obviously
 * correct restatement of what the paper (Cuvelier, Japhet, Scarella, "An
 * efficient way to assemble finite element matrices in vector languages")
 * defines:
 *
 *   A = sum over elements K of  P_K^T E(K) P_K,
 *
 * the classical element loop of Section 3 (Algorithms "base" / OptV1), with
 * every element matrix E(K) obtained from the paper's own ingredients:
 *   - gradients of the barycentric coordinates by solving B_k^T G_k = G_hat
 *     (Appendix C.1, "gradient systems"), here by Gaussian elimination with
 *     partial pivoting, one element at a time;
 *   - |K| = |det B_k| / d!;
 *   - mass and weighted mass from the "magic formula" (Section 2) applied to
 *     the P1 interpolant of w (Section 4.1);
 *   - stiffness |K| <grad l_b, grad l_a> (Section 4.2);
 *   - elasticity through the lemma of Section 5.1 / Appendix B:
 *     lambda <g_b, Q^{n,l} g_a> + mu <g_b, S^{n,l} g_a>, with the Voigt
 *     matrices B_l, C_0, C_1 written out, times |K| (constant Lame
 *     parameters: the P1 interpolant of a constant is that constant), or
 *     with nodal Lame fields, times |K|/(d+1) and the vertex sums lambda^s,
 *     mu^s of the fields (the P1-interpolated coefficients of Section 5.1).
 * and the language-level `sparse` of Section 3: triplets (I, J, K) with
 * duplicates summed.  Here the triplets are sorted by (row, column, element
 * number) and summed in that order, so every global entry is the sum of its
 * element contributions in ascending element order, starting from 0.0.
 * Structural zeros are kept: the pattern is every (I, J) pair that appears
 * in a triplet, whatever its value.
 *
 * Alongside each entry the oracle returns its magnitude scale: the sum over
 * the contributing elements of the size of the terms each contribution is
 * made of, |K| max_c |g_c|^2 for stiffness, (|lambda| + 2|mu|) times that for
 * elasticity, |K| sum_g |w_g| x magic factor for the masses.  Any correct
 * way of computing the gradients and summing rounds relative to this scale,
 * also where a contribution or an entry cancels to (near) zero, so the
 * tolerance of the parity tests is floored by it.
 *
 * Vector case (elasticity, m = d): alternate numbering of Section 5, global
 * dof r = m*i + l for vertex i and component l (0-based), local index
 * a*m + l for local vertex a.
 *
 * Gradient (adjoint) oracle: for J(q, w) = a^T (S(q) + M_w(q)) b it returns
 * dJ/dw (exact: J is linear in w, each coefficient is a magic-formula
 * integral) and dJ/dq by complex-step differentiation of each element's
 * contribution to J (imaginary step 1e-30, so no truncation or cancellation
 * error), accumulated per vertex in ascending element order.
 *
 * Derivatives of the assembly map (JVP and VJP of the mass, weighted mass
 * and stiffness operators) by complex-step differentiation of each element
 * matrix: see the end of the file.
 *
 * Mass and weighted mass on boundary facets ((d-1)-simplices, the Neumann /
 * Robin terms of the remark after Algorithm AssemblyMassWP1): measure from
 * the Gram determinant; see the end of the file.
 *
 * General second-order operator of the introduction with constant
 * coefficients (weak form, full non-symmetric matrix): see the end of the file.
 *
 * P_k Lagrange mass (Appendix D): element matrix d! |K| C with the constant
 * C of the paper's polynomial representation of the basis, evaluated in
 * exact integer arithmetic; local numbering and the rest at the end of the
 * file.
 *
 * Status codes are this file's own and are restated, not included, by the
 * library under test: 0 ok, 1 bad argument, 2 bad index / repeated vertex,
 * 3 degenerate element (det B_k == 0), 4 overflow, 5 out of memory.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_OK = 0, OR_ERR_ARG = 1, OR_ERR_INDEX = 2, OR_ERR_DEGENERATE = 3,
       OR_ERR_OVERFLOW = 4, OR_ERR_NOMEM = 5 };
enum { OR_MASS = 0, OR_MASS_W = 1, OR_STIFF = 2, OR_ELAS = 3 };

#define MAXD 3
#define MAXNL (MAXD + 1)
#define MAXLOC (MAXNL * MAXD)

static double factorial(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= (double)i;
    return f;
}

/* Magic formula (Section 2): integral over K of prod lambda_i^{n_i}
 * = d! |K| prod(n_i!) / (d + sum n_i)!.  Returns the factor multiplying |K|. */
static double magic_factor(int d, const int *expo) {
    double num = factorial(d);
    int s = 0;
    for (int i = 0; i < d + 1; ++i) {
        num *= factorial(expo[i]);
        s += expo[i];
    }
    return num / factorial(d + s);
}

/* ------------------------------------------------------------------------ */
/* Geometry of one element (Appendix C.1), real and complex versions.        */
/* ------------------------------------------------------------------------ */

/* det of a d x d matrix by cofactor expansion along the first row. */
static double det_real(int d, double M[MAXD][MAXD]) {
    if (d == 1) return M[0][0];
    if (d == 2) return M[0][0] * M[1][1] - M[0][1] * M[1][0];
    double s = 0.0;
    for (int c = 0; c < 3; ++c) {
        int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        s += M[0][c] * (M[1][c1] * M[2][c2] - M[1][c2] * M[2][c1]);
    }
    return s;
}

static double complex det_cplx(int d, double complex M[MAXD][MAXD]) {
    if (d == 1) return M[0][0];
    if (d == 2) return M[0][0] * M[1][1] - M[0][1] * M[1][0];
    double complex s = 0.0;
    for (int c = 0; c < 3; ++c) {
        int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
        s += M[0][c] * (M[1][c1] * M[2][c2] - M[1][c2] * M[2][c1]);
    }
    return s;
}

/* Solve Bt X = R for X (d x (d+1)) by Gaussian elimination with partial
 * pivoting; Bt is d x d, R is d x (d+1).  Returns 0 on a zero pivot. */
static int solve_real(int d, double Bt[MAXD][MAXD], double R[MAXD][MAXNL],
                      double X[MAXD][MAXNL]) {
    double A[MAXD][MAXD], Y[MAXD][MAXNL];
    memcpy(A, Bt, sizeof(A));
    memcpy(Y, R, sizeof(Y));
    for (int col = 0; col < d; ++col) {
        int piv = col;
        for (int r = col + 1; r < d; ++r)
            if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
        if (A[piv][col] == 0.0) return 0;
        if (piv != col) {
            for (int c = 0; c < d; ++c) { double t = A[col][c]; A[col][c] = A[piv][c]; A[piv][c] = t; }
            for (int c = 0; c < d + 1; ++c) { double t = Y[col][c]; Y[col][c] = Y[piv][c]; Y[piv][c] = t; }
        }
        for (int r = col + 1; r < d; ++r) {
            double f = A[r][col] / A[col][col];
            for (int c = col; c < d; ++c) A[r][c] -= f * A[col][c];
            for (int c = 0; c < d + 1; ++c) Y[r][c] -= f * Y[col][c];
        }
    }
    for (int c = 0; c < d + 1; ++c) {
        for (int r = d - 1; r >= 0; --r) {
            double s = Y[r][c];
            for (int k = r + 1; k < d; ++k) s -= A[r][k] * X[k][c];
            X[r][c] = s / A[r][r];
        }
    }
    return 1;
}

static int solve_cplx(int d, double complex Bt[MAXD][MAXD], double complex R[MAXD][MAXNL],
                      double complex X[MAXD][MAXNL]) {
    double complex A[MAXD][MAXD], Y[MAXD][MAXNL];
    memcpy(A, Bt, sizeof(A));
    memcpy(Y, R, sizeof(Y));
    for (int col = 0; col < d; ++col) {
        int piv = col;  /* pivot on the real part: the imaginary part is a perturbation */
        for (int r = col + 1; r < d; ++r)
            if (fabs(creal(A[r][col])) > fabs(creal(A[piv][col]))) piv = r;
        if (creal(A[piv][col]) == 0.0) return 0;
        if (piv != col) {
            for (int c = 0; c < d; ++c) { double complex t = A[col][c]; A[col][c] = A[piv][c]; A[piv][c] = t; }
            for (int c = 0; c < d + 1; ++c) { double complex t = Y[col][c]; Y[col][c] = Y[piv][c]; Y[piv][c] = t; }
        }
        for (int r = col + 1; r < d; ++r) {
            double complex f = A[r][col] / A[col][col];
            for (int c = col; c < d; ++c) A[r][c] -= f * A[col][c];
            for (int c = 0; c < d + 1; ++c) Y[r][c] -= f * Y[col][c];
        }
    }
    for (int c = 0; c < d + 1; ++c) {
        for (int r = d - 1; r >= 0; --r) {
            double complex s = Y[r][c];
            for (int k = r + 1; k < d; ++k) s -= A[r][k] * X[k][c];
            X[r][c] = s / A[r][r];
        }
    }
    return 1;
}

/* Element geometry: B_k (columns q^i - q^0), |K| = |det B_k|/d!, and
 * G[i][a] = d lambda_a / d x_i from B_k^T G = G_hat with
 * G_hat = [-1 | I_d].  Returns 0 for a degenerate element. */
static int element_geometry(int d, const double P[MAXNL][MAXD], double *vol,
                            double G[MAXD][MAXNL]) {
    double B[MAXD][MAXD], Bt[MAXD][MAXD], Ghat[MAXD][MAXNL];
    for (int i = 0; i < d; ++i)
        for (int c = 0; c < d; ++c) B[i][c] = P[c + 1][i] - P[0][i];
    double det = det_real(d, B);
    if (det == 0.0) return 0;
    for (int i = 0; i < d; ++i)
        for (int c = 0; c < d; ++c) Bt[i][c] = B[c][i];
    for (int i = 0; i < d; ++i) {
        Ghat[i][0] = -1.0;
        for (int a = 1; a < d + 1; ++a) Ghat[i][a] = (a - 1 == i) ? 1.0 : 0.0;
    }
    if (!solve_real(d, Bt, Ghat, G)) return 0;
    *vol = fabs(det) / factorial(d);
    return 1;
}

/* Voigt strain selection matrix B_l (Appendix B), 0-based component l. */
static void voigt_B(int d, int l, double Bl[6][MAXD]) {
    memset(Bl, 0, sizeof(double) * 6 * MAXD);
    const double dl1 = (l == 0), dl2 = (l == 1), dl3 = (l == 2);
    if (d == 2) {
        Bl[0][0] = dl1;
        Bl[1][1] = dl2;
        Bl[2][0] = dl2; Bl[2][1] = dl1;
    } else {
        Bl[0][0] = dl1;
        Bl[1][1] = dl2;
        Bl[2][2] = dl3;
        Bl[3][0] = dl2; Bl[3][1] = dl1;
        Bl[4][1] = dl3; Bl[4][2] = dl2;
        Bl[5][0] = dl3; Bl[5][2] = dl1;
    }
}

/* C_0 (ones block on the normal strains) and C_1 (2 I_d then I_{2d-3}). */
static void voigt_C(int d, double C0[6][6], double C1[6][6]) {
    int nv = 3 * (d - 1);
    memset(C0, 0, sizeof(double) * 36);
    memset(C1, 0, sizeof(double) * 36);
    for (int i = 0; i < d; ++i) {
        for (int j = 0; j < d; ++j) C0[i][j] = 1.0;
        C1[i][i] = 2.0;
    }
    for (int i = d; i < nv; ++i) C1[i][i] = 1.0;
}

/* Q^{n,l} = B_n^T C_0 B_l and S^{n,l} = B_n^T C_1 B_l (Appendix B). */
static void mat_QS(int d, int n, int l, double Q[MAXD][MAXD], double S[MAXD][MAXD]) {
    double Bn[6][MAXD], Bl[6][MAXD], C0[6][6], C1[6][6];
    int nv = 3 * (d - 1);
    voigt_B(d, n, Bn);
    voigt_B(d, l, Bl);
    voigt_C(d, C0, C1);
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            double q = 0.0, s = 0.0;
            for (int u = 0; u < nv; ++u)
                for (int v = 0; v < nv; ++v) {
                    q += Bn[u][i] * C0[u][v] * Bl[v][j];
                    s += Bn[u][i] * C1[u][v] * Bl[v][j];
                }
            Q[i][j] = q;
            S[i][j] = s;
        }
}

/* Full local matrix E (nloc x nloc, nloc = (d+1)*m), row index a*m+l (test
 * function psi_{l,a}), column index b*m+n (trial function psi_{n,b}). */
static int element_matrix(int d, int op, const double P[MAXNL][MAXD], const double *wloc,
                          double lam, double mu, double E[MAXLOC][MAXLOC],
                          double Eabs[MAXLOC][MAXLOC]) {
    double vol, G[MAXD][MAXNL];
    if (!element_geometry(d, P, &vol, G)) return 0;
    const int nl = d + 1;
    double g2max = 0.0;  /* largest squared gradient norm on the element */
    for (int a = 0; a < nl; ++a) {
        double g2 = 0.0;
        for (int i = 0; i < d; ++i) g2 += G[i][a] * G[i][a];
        if (g2 > g2max) g2max = g2;
    }
    if (op == OR_MASS || op == OR_MASS_W) {
        for (int a = 0; a < nl; ++a)
            for (int b = 0; b < nl; ++b) {
                double s = 0.0, sa = 0.0;
                if (op == OR_MASS) {
                    int ex[MAXNL] = {0, 0, 0, 0};
                    ex[a] += 1; ex[b] += 1;
                    s = sa = magic_factor(d, ex);
                } else {
                    /* w_h = sum_g w_g lambda_g (P1 interpolant, Section 4.1) */
                    for (int g = 0; g < nl; ++g) {
                        int ex[MAXNL] = {0, 0, 0, 0};
                        ex[a] += 1; ex[b] += 1; ex[g] += 1;
                        s += wloc[g] * magic_factor(d, ex);
                        sa += fabs(wloc[g]) * magic_factor(d, ex);
                    }
                }
                E[a][b] = vol * s;
                Eabs[a][b] = vol * sa;
            }
        return 1;
    }
    if (op == OR_STIFF) {
        for (int a = 0; a < nl; ++a)
            for (int b = 0; b < nl; ++b) {
                double s = 0.0;
                for (int i = 0; i < d; ++i) s += G[i][b] * G[i][a];
                E[a][b] = vol * s;
                Eabs[a][b] = vol * g2max;
            }
        return 1;
    }
    /* OR_ELAS */
    const int m = d;
    for (int l = 0; l < m; ++l)
        for (int n = 0; n < m; ++n) {
            double Q[MAXD][MAXD], S[MAXD][MAXD];
            mat_QS(d, n, l, Q, S);
            for (int a = 0; a < nl; ++a)
                for (int b = 0; b < nl; ++b) {
                    /* <g_b, Q g_a> and <g_b, S g_a> */
                    double xq = 0.0, xs = 0.0;
                    for (int i = 0; i < d; ++i)
                        for (int j = 0; j < d; ++j) {
                            xq += G[i][b] * Q[i][j] * G[j][a];
                            xs += G[i][b] * S[i][j] * G[j][a];
                        }
                    E[a * m + l][b * m + n] = vol * (lam * xq + mu * xs);
                    Eabs[a * m + l][b * m + n] = vol * (fabs(lam) + 2.0 * fabs(mu)) * g2max;
                }
        }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Validation and the `sparse` step.                                          */
/* ------------------------------------------------------------------------ */

int oracle_validate(int d, int64_t nq, int64_t nme, const int32_t *me) {
    if (d < 2 || d > 3 || nq < 0 || nme < 0) return OR_ERR_ARG;
    if (nme > 0 && !me) return OR_ERR_ARG;
    for (int64_t k = 0; k < nme; ++k) {
        for (int a = 0; a <= d; ++a) {
            int32_t v = me[(int64_t)a * nme + k];
            if (v < 0 || (int64_t)v >= nq) return OR_ERR_INDEX;
            for (int b = 0; b < a; ++b)
                if (me[(int64_t)b * nme + k] == v) return OR_ERR_INDEX;
        }
    }
    return OR_OK;
}

typedef struct {
    int64_t row, col, seq;
    double val, aval;
} triplet_t;

static int cmp_triplet(const void *pa, const void *pb) {
    const triplet_t *a = (const triplet_t *)pa, *b = (const triplet_t *)pb;
    if (a->row != b->row) return a->row < b->row ? -1 : 1;
    if (a->col != b->col) return a->col < b->col ? -1 : 1;
    if (a->seq != b->seq) return a->seq < b->seq ? -1 : 1;
    return 0;
}

static void gather_element(int d, int64_t nq, int64_t nme, const double *q, const int32_t *me,
                           int64_t k, double P[MAXNL][MAXD], int32_t *vid) {
    for (int a = 0; a <= d; ++a) {
        vid[a] = me[(int64_t)a * nme + k];
        for (int i = 0; i < d; ++i) P[a][i] = q[(int64_t)i * nq + vid[a]];
    }
}

/* Core: assemble the rows selected by `sel` (sel[r] = output position + 1,
 * or 0 for rows to skip; NULL = all rows).  Output is CSR over the selected
 * rows in output-position order.  cap bounds the number of nonzeros. */
static int assemble_core(int d, int64_t nq, int64_t nme, const double *q, const int32_t *me,
                         int op, const double *w, double lam, double mu,
                         const double *lam_nodal, const double *mu_nodal,
                         const int64_t *sel, int64_t nout,
                         int64_t cap, int64_t *nnz_out, int64_t *row_ptr, int64_t *col_idx,
                         double *val, double *absval) {
    int st = oracle_validate(d, nq, nme, me);
    if (st != OR_OK) return st;
    if (op < OR_MASS || op > OR_ELAS) return OR_ERR_ARG;
    if (op == OR_MASS_W && !w) return OR_ERR_ARG;
    if (nme > 0 && !q) return OR_ERR_ARG;
    const int m = (op == OR_ELAS) ? d : 1;
    const int nl = d + 1, nloc = nl * m;

    /* pass 1: count selected triplets */
    int64_t ntrip = 0;
    for (int64_t k = 0; k < nme; ++k)
        for (int a = 0; a < nl; ++a)
            for (int l = 0; l < m; ++l) {
                int64_t r = (int64_t)m * me[(int64_t)a * nme + k] + l;
                if (!sel || sel[r]) ntrip += nloc;
            }
    triplet_t *T = (triplet_t *)malloc(sizeof(triplet_t) * (ntrip > 0 ? ntrip : 1));
    if (!T) return OR_ERR_NOMEM;

    /* pass 2: element loop in ascending k (Section 3, Algorithms base/OptV1):
     * local matrix stored column-wise, triplet number = seq */
    int64_t t = 0;
    for (int64_t k = 0; k < nme; ++k) {
        int32_t vid[MAXNL];
        double P[MAXNL][MAXD], wloc[MAXNL] = {0, 0, 0, 0}, E[MAXLOC][MAXLOC], Ea[MAXLOC][MAXLOC];
        int need = 0;
        for (int a = 0; a < nl && !need; ++a)
            for (int l = 0; l < m; ++l) {
                int64_t r = (int64_t)m * me[(int64_t)a * nme + k] + l;
                if (!sel || sel[r]) need = 1;
            }
        if (!need) continue;
        gather_element(d, nq, nme, q, me, k, P, vid);
        if (op == OR_MASS_W)
            for (int a = 0; a < nl; ++a) wloc[a] = w[vid[a]];
        double lamk = lam, muk = mu;
        if (lam_nodal) {
            /* P1 interpolants of the Lame fields (Section 5.1): the integral
             * of lambda_h over K is |K| lambda^s / (d+1) */
            double ls = 0.0, ms = 0.0;
            for (int a = 0; a < nl; ++a) {
                ls += lam_nodal[vid[a]];
                ms += mu_nodal[vid[a]];
            }
            lamk = ls / (double)nl;
            muk = ms / (double)nl;
        }
        if (!element_matrix(d, op, P, wloc, lamk, muk, E, Ea)) {
            free(T);
            return OR_ERR_DEGENERATE;
        }
        for (int b = 0; b < nl; ++b)
            for (int n = 0; n < m; ++n)
                for (int a = 0; a < nl; ++a)
                    for (int l = 0; l < m; ++l) {
                        int64_t r = (int64_t)m * vid[a] + l;
                        if (sel && !sel[r]) continue;
                        T[t].row = sel ? sel[r] - 1 : r;
                        T[t].col = (int64_t)m * vid[b] + n;
                        T[t].seq = t;
                        T[t].val = E[a * m + l][b * m + n];
                        T[t].aval = Ea[a * m + l][b * m + n];
                        ++t;
                    }
    }
    /* `sparse`: sort by (row, col, seq), sum duplicates in that order */
    qsort(T, (size_t)t, sizeof(triplet_t), cmp_triplet);
    int64_t nnz = 0;
    for (int64_t i = 0; i < t; ++i)
        if (i == 0 || T[i].row != T[i - 1].row || T[i].col != T[i - 1].col) ++nnz;
    if (nnz > cap) {
        free(T);
        return OR_ERR_OVERFLOW;
    }
    for (int64_t r = 0; r <= nout; ++r) row_ptr[r] = 0;
    int64_t s = -1;
    for (int64_t i = 0; i < t; ++i) {
        if (i == 0 || T[i].row != T[i - 1].row || T[i].col != T[i - 1].col) {
            ++s;
            col_idx[s] = T[i].col;
            val[s] = 0.0;
            if (absval) absval[s] = 0.0;
            row_ptr[T[i].row + 1] += 1;
        }
        val[s] += T[i].val;
        if (absval) absval[s] += T[i].aval;
    }
    for (int64_t r = 0; r < nout; ++r) row_ptr[r + 1] += row_ptr[r];
    *nnz_out = nnz;
    free(T);
    return OR_OK;
}

/* Full assembly: CSR with nrows = m*nq rows.  row_ptr has nrows+1 entries;
 * col_idx/val/absval have room for cap entries ((d+1)^2 m^2 nme suffices). */
int oracle_assemble(int d, int64_t nq, int64_t nme, const double *q, const int32_t *me,
                    int op, const double *w, double lam, double mu, int64_t cap,
                    int64_t *nnz_out, int64_t *row_ptr, int64_t *col_idx, double *val,
                    double *absval) {
    if (d < 2 || d > 3) return OR_ERR_ARG;
    const int m = (op == OR_ELAS) ? d : 1;
    return assemble_core(d, nq, nme, q, me, op, w, lam, mu, NULL, NULL, NULL, (int64_t)m * nq,
                         cap, nnz_out, row_ptr, col_idx, val, absval);
}

/* Elasticity with nodal (P1) Lame fields lam_nodal[nq], mu_nodal[nq]:
 * element matrix |K|/(d+1) (lambda^s <g_b, Q g_a> + mu^s <g_b, S g_a>),
 * lambda^s the sum of the field over the element's vertices (Section 5.1).
 * rows: NULL for all d*nq rows, else nsel distinct global rows. */
int oracle_assemble_lame(int d, int64_t nq, int64_t nme, const double *q, const int32_t *me,
                         const double *lam_nodal, const double *mu_nodal, int64_t nsel,
                         const int64_t *rows, int64_t cap, int64_t *nnz_out, int64_t *row_ptr,
                         int64_t *col_idx, double *val, double *absval) {
    if (d < 2 || d > 3 || !lam_nodal || !mu_nodal) return OR_ERR_ARG;
    if (!rows)
        return assemble_core(d, nq, nme, q, me, OR_ELAS, NULL, 0.0, 0.0, lam_nodal, mu_nodal,
                             NULL, (int64_t)d * nq, cap, nnz_out, row_ptr, col_idx, val, absval);
    const int64_t nrows = (int64_t)d * nq;
    if (nsel < 0) return OR_ERR_ARG;
    int64_t *sel = (int64_t *)calloc((size_t)(nrows > 0 ? nrows : 1), sizeof(int64_t));
    if (!sel) return OR_ERR_NOMEM;
    for (int64_t s = 0; s < nsel; ++s) {
        if (rows[s] < 0 || rows[s] >= nrows || sel[rows[s]]) {
            free(sel);
            return OR_ERR_ARG;
        }
        sel[rows[s]] = s + 1;
    }
    int st = assemble_core(d, nq, nme, q, me, OR_ELAS, NULL, 0.0, 0.0, lam_nodal, mu_nodal, sel,
                           nsel, cap, nnz_out, row_ptr, col_idx, val, absval);
    free(sel);
    return st;
}

/* Selected rows only (sampled checks on large meshes).  rows[0..nsel) are
 * distinct global row numbers; output CSR row s is global row rows[s]. */
int oracle_assemble_rows(int d, int64_t nq, int64_t nme, const double *q, const int32_t *me,
                         int op, const double *w, double lam, double mu, int64_t nsel,
                         const int64_t *rows, int64_t cap, int64_t *nnz_out, int64_t *row_ptr,
                         int64_t *col_idx, double *val, double *absval) {
    if (d < 2 || d > 3 || nsel < 0) return OR_ERR_ARG;
    const int m = (op == OR_ELAS) ? d : 1;
    const int64_t nrows = (int64_t)m * nq;
    int64_t *sel = (int64_t *)calloc((size_t)(nrows > 0 ? nrows : 1), sizeof(int64_t));
    if (!sel) return OR_ERR_NOMEM;
    for (int64_t s = 0; s < nsel; ++s) {
        if (rows[s] < 0 || rows[s] >= nrows || sel[rows[s]]) {
            free(sel);
            return OR_ERR_ARG;
        }
        sel[rows[s]] = s + 1;
    }
    int st = assemble_core(d, nq, nme, q, me, op, w, lam, mu, NULL, NULL, sel, nsel, cap, nnz_out,
                           row_ptr, col_idx, val, absval);
    free(sel);
    return st;
}

/* Element contribution to J = a^T (S + M_w) b, in complex arithmetic so that
 * a complex perturbation of one coordinate yields the derivative exactly.
 * |K| = sign(Re det) det / d! keeps the expression analytic. */
static int element_J_cplx(int d, double complex P[MAXNL][MAXD], const double *wl,
                          const double *al, const double *bl, double complex *J) {
    double complex B[MAXD][MAXD], Bt[MAXD][MAXD], R[MAXD][MAXNL], G[MAXD][MAXNL];
    for (int i = 0; i < d; ++i)
        for (int c = 0; c < d; ++c) B[i][c] = P[c + 1][i] - P[0][i];
    double complex det = det_cplx(d, B);
    if (creal(det) == 0.0) return 0;
    for (int i = 0; i < d; ++i)
        for (int c = 0; c < d; ++c) Bt[i][c] = B[c][i];
    for (int i = 0; i < d; ++i) {
        R[i][0] = -1.0;
        for (int a = 1; a < d + 1; ++a) R[i][a] = (a - 1 == i) ? 1.0 : 0.0;
    }
    if (!solve_cplx(d, Bt, R, G)) return 0;
    double complex vol = (creal(det) < 0 ? -det : det) / factorial(d);
    double complex s = 0.0;
    for (int a = 0; a <= d; ++a)
        for (int b = 0; b <= d; ++b) {
            double complex st = 0.0;
            for (int i = 0; i < d; ++i) st += G[i][b] * G[i][a];
            double mw = 0.0;
            for (int g = 0; g <= d; ++g) {
                int ex[MAXNL] = {0, 0, 0, 0};
                ex[a] += 1; ex[b] += 1; ex[g] += 1;
                mw += wl[g] * magic_factor(d, ex);
            }
            s += al[a] * bl[b] * (st + mw);
        }
    *J = vol * s;
    return 1;
}

/* J = a^T (S + M_w) b and its gradients.  dJdw has nq entries, dJdq has
 * d*nq entries laid out like q (dJdq[v*nq + j]).  Either may be NULL.  The
 * *_abs arrays (optional) receive the sum of |element contribution| per
 * entry, the scale that floors the parity tolerance. */
int oracle_grad(int d, int64_t nq, int64_t nme, const double *q, const int32_t *me,
                const double *w, const double *a, const double *b, double *J_out,
                double *dJdw, double *dJdq, double *dJdw_abs, double *dJdq_abs) {
    int st = oracle_validate(d, nq, nme, me);
    if (st != OR_OK) return st;
    if (!q || !w || !a || !b) return OR_ERR_ARG;
    const double hstep = 1e-30;
    if (dJdw) memset(dJdw, 0, sizeof(double) * (size_t)nq);
    if (dJdq) memset(dJdq, 0, sizeof(double) * (size_t)(d * nq));
    if (dJdw_abs) memset(dJdw_abs, 0, sizeof(double) * (size_t)nq);
    if (dJdq_abs) memset(dJdq_abs, 0, sizeof(double) * (size_t)(d * nq));
    double Jsum = 0.0;
    for (int64_t k = 0; k < nme; ++k) {
        int32_t vid[MAXNL];
        double P[MAXNL][MAXD], wl[MAXNL], al[MAXNL], bl[MAXNL];
        gather_element(d, nq, nme, q, me, k, P, vid);
        for (int g = 0; g <= d; ++g) { wl[g] = w[vid[g]]; al[g] = a[vid[g]]; bl[g] = b[vid[g]]; }
        double complex Pc[MAXNL][MAXD], Jk;
        for (int g = 0; g <= d; ++g)
            for (int i = 0; i < d; ++i) Pc[g][i] = P[g][i];
        if (!element_J_cplx(d, Pc, wl, al, bl, &Jk)) return OR_ERR_DEGENERATE;
        Jsum += creal(Jk);
        if (dJdq) {
            for (int g = 0; g <= d; ++g)
                for (int i = 0; i < d; ++i) {
                    double complex Pp[MAXNL][MAXD];
                    memcpy(Pp, Pc, sizeof(Pp));
                    Pp[g][i] += I * hstep;
                    double complex Jp;
                    if (!element_J_cplx(d, Pp, wl, al, bl, &Jp)) return OR_ERR_DEGENERATE;
                    dJdq[(int64_t)i * nq + vid[g]] += cimag(Jp) / hstep;
                    if (dJdq_abs) dJdq_abs[(int64_t)i * nq + vid[g]] += fabs(cimag(Jp) / hstep);
                }
        }
        if (dJdw) {
            double vol, G[MAXD][MAXNL];
            if (!element_geometry(d, P, &vol, G)) return OR_ERR_DEGENERATE;
            for (int g = 0; g <= d; ++g) {
                double s = 0.0;
                for (int aa = 0; aa <= d; ++aa)
                    for (int bb = 0; bb <= d; ++bb) {
                        int ex[MAXNL] = {0, 0, 0, 0};
                        ex[aa] += 1; ex[bb] += 1; ex[g] += 1;
                        s += al[aa] * bl[bb] * magic_factor(d, ex);
                    }
                dJdw[vid[g]] += vol * s;
                if (dJdw_abs) dJdw_abs[vid[g]] += fabs(vol * s);
            }
        }
    }
    if (J_out) *J_out = Jsum;
    return OR_OK;
}

/* Element matrix of one element given its vertex coordinates P (row-major
 * (d+1) x d) — exposed so tests can pin it on reference simplices. */
int oracle_element_matrix(int d, int op, const double *P, const double *wloc, double lam,
                          double mu, double *E_out) {
    if (d < 2 || d > 3 || op < OR_MASS || op > OR_ELAS) return OR_ERR_ARG;
    double Pl[MAXNL][MAXD], E[MAXLOC][MAXLOC], Ea[MAXLOC][MAXLOC];
    for (int a = 0; a <= d; ++a)
        for (int i = 0; i < d; ++i) Pl[a][i] = P[a * d + i];
    if (!element_matrix(d, op, Pl, wloc, lam, mu, E, Ea)) return OR_ERR_DEGENERATE;
    const int m = (op == OR_ELAS) ? d : 1, nloc = (d + 1) * m;
    for (int i = 0; i < nloc; ++i)
        for (int j = 0; j < nloc; ++j) E_out[i * nloc + j] = E[i][j];
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* P_k Lagrange mass matrix (Appendix D).                                     */
/*                                                                            */
/* Local numbering I of the multi-indices alpha in N^{d+1}, |alpha| = k        */
/* (alpha_i is the exponent of the barycentric coordinate of local vertex i): */
/* local nodes 0..d are the vertices alpha = k e_i, the others follow in      */
/* decreasing lexicographic order of (alpha_0, ..., alpha_d).                  */
/*                                                                            */
/* The basis function of alpha is prod_l prod_{j < alpha_l} (k lambda_l - j)/  */
/* (j+1), a polynomial in the barycentric coordinates, so alpha! phi_alpha =   */
/* prod_l p_{alpha_l}(lambda_l) with p_m(x) = prod_{j<m} (k x - j) has integer */
/* coefficients; the magic formula then gives                                 */
/*   int_K phi_alpha phi_beta = d! |K| C_{alpha,beta},                         */
/*   C_{alpha,beta} = sum_{mu,nu} a_mu(alpha) a_nu(beta)                       */
/*                    prod_i (mu_i + nu_i)! / (d + |mu| + |nu|)!,               */
/* evaluated here exactly in 128-bit integers over the common denominator     */
/* (d+2k)! alpha! beta!, and converted to double once at the end.             */
/* ------------------------------------------------------------------------ */

#define PK_MAXK 6
#define PK_MAXN 84 /* (3+6)! / (3! 6!) */

typedef __int128 i128;

static int pk_count(int d, int k) {
    int64_t n = 1;
    for (int i = 1; i <= d; ++i) n = n * (k + i) / i;
    return (int)n;
}

/* multi-indices in local order; returns their number */
static int pk_enumerate(int d, int k, int alpha[PK_MAXN][MAXNL]) {
    int all[PK_MAXN][MAXNL], n = 0, cur[MAXNL];
    /* decreasing lexicographic: odometer from (k,0,..,0) downwards */
    for (int a0 = k; a0 >= 0; --a0) {
        cur[0] = a0;
        if (d == 2) {
            for (int a1 = k - a0; a1 >= 0; --a1) {
                cur[1] = a1;
                cur[2] = k - a0 - a1;
                memcpy(all[n++], cur, sizeof(int) * MAXNL);
            }
        } else {
            for (int a1 = k - a0; a1 >= 0; --a1)
                for (int a2 = k - a0 - a1; a2 >= 0; --a2) {
                    cur[1] = a1;
                    cur[2] = a2;
                    cur[3] = k - a0 - a1 - a2;
                    memcpy(all[n++], cur, sizeof(int) * MAXNL);
                }
        }
    }
    int m = 0;
    for (int v = 0; v <= d; ++v) { /* vertices first */
        for (int i = 0; i <= d; ++i) alpha[m][i] = (i == v) ? k : 0;
        ++m;
    }
    for (int t = 0; t < n; ++t) {
        int isv = 0;
        for (int i = 0; i <= d; ++i) isv |= all[t][i] == k;
        if (!isv) memcpy(alpha[m++], all[t], sizeof(int) * MAXNL);
    }
    return m;
}

static i128 ifact(int n) {
    i128 f = 1;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

/* pc[m][i] = coefficient of x^i in p_m(x) = prod_{j<m} (k x - j) */
static void pk_univariate(int k, i128 pc[PK_MAXK + 1][PK_MAXK + 1]) {
    memset(pc, 0, sizeof(i128) * (PK_MAXK + 1) * (PK_MAXK + 1));
    pc[0][0] = 1;
    for (int m = 1; m <= k; ++m)
        for (int i = 0; i <= m; ++i) {
            i128 c = -(i128)(m - 1) * pc[m - 1][i];  /* times (-(m-1)) */
            if (i > 0) c += (i128)k * pc[m - 1][i - 1]; /* times k x */
            pc[m][i] = c;
        }
}

/* C (n x n, row-major, n = pk_count) */
int oracle_pk_coeff(int d, int k, double *C) {
    if (d < 2 || d > 3 || k < 1 || k > PK_MAXK || !C) return OR_ERR_ARG;
    int alpha[PK_MAXN][MAXNL];
    const int n = pk_enumerate(d, k, alpha);
    i128 pc[PK_MAXK + 1][PK_MAXK + 1];
    pk_univariate(k, pc);
    const i128 top = ifact(d + 2 * k);
    for (int x = 0; x < n; ++x)
        for (int y = 0; y < n; ++y) {
            const int *a = alpha[x], *b = alpha[y];
            i128 num = 0;
            int mu[MAXNL] = {0, 0, 0, 0}, nu[MAXNL];
            /* odometer over mu <= a (componentwise) */
            for (;;) {
                i128 am = 1;
                int smu = 0;
                for (int i = 0; i <= d; ++i) { am *= pc[a[i]][mu[i]]; smu += mu[i]; }
                if (am != 0) {
                    memset(nu, 0, sizeof(nu));
                    for (;;) {
                        i128 bn = 1;
                        int snu = 0;
                        for (int i = 0; i <= d; ++i) { bn *= pc[b[i]][nu[i]]; snu += nu[i]; }
                        if (bn != 0) {
                            i128 w = top / ifact(d + smu + snu);
                            for (int i = 0; i <= d; ++i) w *= ifact(mu[i] + nu[i]);
                            num += am * bn * w;
                        }
                        int i = 0;
                        while (i <= d && nu[i] == b[i]) nu[i++] = 0;
                        if (i > d) break;
                        nu[i] += 1;
                    }
                }
                int i = 0;
                while (i <= d && mu[i] == a[i]) mu[i++] = 0;
                if (i > d) break;
                mu[i] += 1;
            }
            i128 den = top;
            for (int i = 0; i <= d; ++i) den *= ifact(a[i]) * ifact(b[i]);
            C[x * n + y] = (double)((long double)num / (long double)den);
        }
    return OR_OK;
}

/* Local multi-indices (n x (d+1), row-major ints) in the numbering above. */
int oracle_pk_alpha(int d, int k, int32_t *out) {
    if (d < 2 || d > 3 || k < 1 || k > PK_MAXK || !out) return OR_ERR_ARG;
    int alpha[PK_MAXN][MAXNL];
    const int n = pk_enumerate(d, k, alpha);
    for (int x = 0; x < n; ++x)
        for (int i = 0; i <= d; ++i) out[x * (d + 1) + i] = alpha[x][i];
    return OR_OK;
}

/* P_k mass matrix of a P_k mesh: me is n x nme (n = (d+k)!/(d!k!)), local
 * nodes 0..d are the element's vertices (their coordinates define K).  Rows
 * selected as in assemble_core (sel NULL = all nq rows).  Element matrix
 * d! |K| C, triplets summed by `sparse` in ascending element order. */
static int pk_core(int d, int k, int64_t nq, int64_t nme, const double *q, const int32_t *me,
                   const int64_t *sel, int64_t nout, int64_t cap, int64_t *nnz_out,
                   int64_t *row_ptr, int64_t *col_idx, double *val, double *absval) {
    if (d < 2 || d > 3 || k < 1 || k > PK_MAXK || nq < 0 || nme < 0) return OR_ERR_ARG;
    if (nme > 0 && (!me || !q)) return OR_ERR_ARG;
    const int n = pk_count(d, k);
    for (int64_t e = 0; e < nme; ++e)
        for (int a = 0; a < n; ++a) {
            const int32_t v = me[(int64_t)a * nme + e];
            if (v < 0 || (int64_t)v >= nq) return OR_ERR_INDEX;
            for (int b = 0; b < a; ++b)
                if (me[(int64_t)b * nme + e] == v) return OR_ERR_INDEX;
        }
    double *C = (double *)malloc(sizeof(double) * n * n);
    if (!C) return OR_ERR_NOMEM;
    oracle_pk_coeff(d, k, C);
    int64_t ntrip = 0;
    for (int64_t e = 0; e < nme; ++e)
        for (int a = 0; a < n; ++a)
            if (!sel || sel[me[(int64_t)a * nme + e]]) ntrip += n;
    triplet_t *T = (triplet_t *)malloc(sizeof(triplet_t) * (ntrip > 0 ? ntrip : 1));
    if (!T) {
        free(C);
        return OR_ERR_NOMEM;
    }
    int64_t t = 0;
    const double dfact = factorial(d);
    for (int64_t e = 0; e < nme; ++e) {
        int need = 0;
        for (int a = 0; a < n && !need; ++a) need = !sel || sel[me[(int64_t)a * nme + e]];
        if (!need) continue;
        double P[MAXNL][MAXD], vol, G[MAXD][MAXNL];
        int32_t vid[MAXNL];
        gather_element(d, nq, nme, q, me, e, P, vid); /* local nodes 0..d: the vertices */
        if (!element_geometry(d, P, &vol, G)) {
            free(T);
            free(C);
            return OR_ERR_DEGENERATE;
        }
        for (int b = 0; b < n; ++b)
            for (int a = 0; a < n; ++a) {
                const int64_t r = me[(int64_t)a * nme + e];
                if (sel && !sel[r]) continue;
                T[t].row = sel ? sel[r] - 1 : r;
                T[t].col = me[(int64_t)b * nme + e];
                T[t].seq = t;
                T[t].val = dfact * vol * C[a * n + b];
                T[t].aval = fabs(T[t].val);
                ++t;
            }
    }
    free(C);
    qsort(T, (size_t)t, sizeof(triplet_t), cmp_triplet);
    int64_t nnz = 0;
    for (int64_t i = 0; i < t; ++i)
        if (i == 0 || T[i].row != T[i - 1].row || T[i].col != T[i - 1].col) ++nnz;
    if (nnz > cap) {
        free(T);
        return OR_ERR_OVERFLOW;
    }
    for (int64_t r = 0; r <= nout; ++r) row_ptr[r] = 0;
    int64_t s = -1;
    for (int64_t i = 0; i < t; ++i) {
        if (i == 0 || T[i].row != T[i - 1].row || T[i].col != T[i - 1].col) {
            ++s;
            col_idx[s] = T[i].col;
            val[s] = 0.0;
            if (absval) absval[s] = 0.0;
            row_ptr[T[i].row + 1] += 1;
        }
        val[s] += T[i].val;
        if (absval) absval[s] += T[i].aval;
    }
    for (int64_t r = 0; r < nout; ++r) row_ptr[r + 1] += row_ptr[r];
    *nnz_out = nnz;
    free(T);
    return OR_OK;
}

int oracle_pk_mass(int d, int k, int64_t nq, int64_t nme, const double *q, const int32_t *me,
                   int64_t cap, int64_t *nnz_out, int64_t *row_ptr, int64_t *col_idx,
                   double *val, double *absval) {
    return pk_core(d, k, nq, nme, q, me, NULL, nq, cap, nnz_out, row_ptr, col_idx, val, absval);
}

int oracle_pk_mass_rows(int d, int k, int64_t nq, int64_t nme, const double *q,
                        const int32_t *me, int64_t nsel, const int64_t *rows, int64_t cap,
                        int64_t *nnz_out, int64_t *row_ptr, int64_t *col_idx, double *val,
                        double *absval) {
    if (nsel < 0 || nq < 0) return OR_ERR_ARG;
    int64_t *sel = (int64_t *)calloc((size_t)(nq > 0 ? nq : 1), sizeof(int64_t));
    if (!sel) return OR_ERR_NOMEM;
    for (int64_t s = 0; s < nsel; ++s) {
        if (rows[s] < 0 || rows[s] >= nq || sel[rows[s]]) {
            free(sel);
            return OR_ERR_ARG;
        }
        sel[rows[s]] = s + 1;
    }
    int st = pk_core(d, k, nq, nme, q, me, sel, nsel, cap, nnz_out, row_ptr, col_idx, val, absval);
    free(sel);
    return st;
}


/* ------------------------------------------------------------------------ */
/* General second-order operator (the PDE of the introduction):              */
/*   -div(A grad u) + div(b u) + c . grad u + a0 u                            */
/* with constant A (d x d, row-major), b, c (d) and a0, in the weak form      */
/* obtained by testing with v and integrating the divergence terms by parts   */
/* (boundary terms left out):                                                 */
/*   int A grad u . grad v  -  int u b . grad v  +  int (c . grad u) v        */
/*   +  int a0 u v.                                                           */
/* Element matrix, row a (test lambda_a), column b (trial lambda_b):          */
/*   |K| g_a^T A g_b - |K|/(d+1) b.g_a + |K|/(d+1) c.g_b                       */
/*   + a0 |K| d! (1+delta_ab)/(d+2)!   (magic formula for int lambda).        */
/* Not symmetric in general: the full matrix is assembled (OptV, not OptVS).  */
/* coef = [A (d*d), b (d), c (d), a0].                                        */
/* ------------------------------------------------------------------------ */

static int general_element(int d, const double P[MAXNL][MAXD], const double *coef,
                           double E[MAXNL][MAXNL], double Ea[MAXNL][MAXNL]) {
    double vol, G[MAXD][MAXNL];
    if (!element_geometry(d, P, &vol, G)) return 0;
    const int nl = d + 1;
    const double *A = coef, *bv = coef + d * d, *cv = coef + d * d + d;
    const double a0v = coef[d * d + 2 * d];
    double anorm = 0.0, bn = 0.0, cn = 0.0, gmax = 0.0;
    for (int i = 0; i < d * d; ++i) anorm += fabs(A[i]);
    for (int i = 0; i < d; ++i) { bn += fabs(bv[i]); cn += fabs(cv[i]); }
    for (int a = 0; a < nl; ++a) {
        double g = 0.0;
        for (int i = 0; i < d; ++i) g += fabs(G[i][a]);
        if (g > gmax) gmax = g;
    }
    for (int a = 0; a < nl; ++a)
        for (int b = 0; b < nl; ++b) {
            double diff = 0.0;
            for (int i = 0; i < d; ++i)
                for (int j = 0; j < d; ++j) diff += G[i][a] * A[i * d + j] * G[j][b];
            double conv_b = 0.0, conv_c = 0.0;
            for (int i = 0; i < d; ++i) {
                conv_b += bv[i] * G[i][a];
                conv_c += cv[i] * G[i][b];
            }
            int ex[MAXNL] = {0, 0, 0, 0};
            ex[a] += 1;
            ex[b] += 1;
            const double mass = magic_factor(d, ex);
            E[a][b] = vol * diff - vol / nl * conv_b + vol / nl * conv_c + a0v * vol * mass;
            Ea[a][b] = vol * (anorm * gmax * gmax + (bn + cn) * gmax / nl + fabs(a0v) * mass);
        }
    return 1;
}

/* Full CSR of the general operator (nrows = nq), or of the nsel global rows
 * listed in rows (rows NULL: all). */
int oracle_assemble_general(int d, int64_t nq, int64_t nme, const double *q, const int32_t *me,
                            const double *coef, int64_t nsel, const int64_t *rows, int64_t cap,
                            int64_t *nnz_out, int64_t *row_ptr, int64_t *col_idx, double *val,
                            double *absval) {
    if (d < 2 || d > 3 || !coef || nsel < 0) return OR_ERR_ARG;
    int st = oracle_validate(d, nq, nme, me);
    if (st != OR_OK) return st;
    if (nme > 0 && !q) return OR_ERR_ARG;
    int64_t *sel = NULL;
    int64_t nout = nq;
    if (rows) {
        sel = (int64_t *)calloc((size_t)(nq > 0 ? nq : 1), sizeof(int64_t));
        if (!sel) return OR_ERR_NOMEM;
        for (int64_t s = 0; s < nsel; ++s) {
            if (rows[s] < 0 || rows[s] >= nq || sel[rows[s]]) {
                free(sel);
                return OR_ERR_ARG;
            }
            sel[rows[s]] = s + 1;
        }
        nout = nsel;
    }
    const int nl = d + 1;
    int64_t ntrip = 0;
    for (int64_t k = 0; k < nme; ++k)
        for (int a = 0; a < nl; ++a)
            if (!sel || sel[me[(int64_t)a * nme + k]]) ntrip += nl;
    triplet_t *T = (triplet_t *)malloc(sizeof(triplet_t) * (ntrip > 0 ? ntrip : 1));
    if (!T) {
        free(sel);
        return OR_ERR_NOMEM;
    }
    int64_t t = 0;
    for (int64_t k = 0; k < nme; ++k) {
        int need = 0;
        for (int a = 0; a < nl && !need; ++a) need = !sel || sel[me[(int64_t)a * nme + k]];
        if (!need) continue;
        int32_t vid[MAXNL];
        double P[MAXNL][MAXD], E[MAXNL][MAXNL], Ea[MAXNL][MAXNL];
        gather_element(d, nq, nme, q, me, k, P, vid);
        if (!general_element(d, P, coef, E, Ea)) {
            free(T);
            free(sel);
            return OR_ERR_DEGENERATE;
        }
        for (int b = 0; b < nl; ++b)
            for (int a = 0; a < nl; ++a) {
                const int64_t r = vid[a];
                if (sel && !sel[r]) continue;
                T[t].row = sel ? sel[r] - 1 : r;
                T[t].col = vid[b];
                T[t].seq = t;
                T[t].val = E[a][b];
                T[t].aval = Ea[a][b];
                ++t;
            }
    }
    free(sel);
    qsort(T, (size_t)t, sizeof(triplet_t), cmp_triplet);
    int64_t nnz = 0;
    for (int64_t i = 0; i < t; ++i)
        if (i == 0 || T[i].row != T[i - 1].row || T[i].col != T[i - 1].col) ++nnz;
    if (nnz > cap) {
        free(T);
        return OR_ERR_OVERFLOW;
    }
    for (int64_t r = 0; r <= nout; ++r) row_ptr[r] = 0;
    int64_t s = -1;
    for (int64_t i = 0; i < t; ++i) {
        if (i == 0 || T[i].row != T[i - 1].row || T[i].col != T[i - 1].col) {
            ++s;
            col_idx[s] = T[i].col;
            val[s] = 0.0;
            if (absval) absval[s] = 0.0;
            row_ptr[T[i].row + 1] += 1;
        }
        val[s] += T[i].val;
        if (absval) absval[s] += T[i].aval;
    }
    for (int64_t r = 0; r < nout; ++r) row_ptr[r + 1] += row_ptr[r];
    *nnz_out = nnz;
    free(T);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Mass and weighted mass on a mesh of n-simplices embedded in R^d, n < d   */
/* (boundary facets, n = d-1: Neumann / Robin terms).  The closed forms of   */
/* Section 4.1 hold with d replaced by n and |K| the n-dimensional measure,  */
/* sqrt(det(B^T B)) / n! for the d x n edge matrix B (Gram determinant):     */
/*   mass      n! |K| (1+delta_ab) / (n+2)!                                  */
/*   weighted  sum_g w_g int lambda_g lambda_a lambda_b (magic formula).     */
/* facets is (n+1) x nf, w NULL for the plain mass.                           */
/* ------------------------------------------------------------------------ */

static double gram_measure(int d, int n, const double P[MAXNL][MAXD]) {
    double B[MAXD][MAXD], G[MAXD][MAXD];
    for (int i = 0; i < d; ++i)
        for (int c = 0; c < n; ++c) B[i][c] = P[c + 1][i] - P[0][i];
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            double s = 0.0;
            for (int i = 0; i < d; ++i) s += B[i][a] * B[i][b];
            G[a][b] = s;
        }
    double det;
    if (n == 1) det = G[0][0];
    else det = G[0][0] * G[1][1] - G[0][1] * G[1][0];
    if (det <= 0.0) return 0.0;
    return sqrt(det) / factorial(n);
}

int oracle_boundary_mass(int d, int64_t nq, int64_t nf, const double *q, const int32_t *facets,
                         const double *w, int64_t cap, int64_t *nnz_out, int64_t *row_ptr,
                         int64_t *col_idx, double *val, double *absval) {
    if (d < 2 || d > 3 || nq < 0 || nf < 0 || (nf > 0 && (!q || !facets))) return OR_ERR_ARG;
    const int n = d - 1, nl = n + 1;
    for (int64_t k = 0; k < nf; ++k)
        for (int a = 0; a < nl; ++a) {
            const int32_t v = facets[(int64_t)a * nf + k];
            if (v < 0 || (int64_t)v >= nq) return OR_ERR_INDEX;
            for (int b = 0; b < a; ++b)
                if (facets[(int64_t)b * nf + k] == v) return OR_ERR_INDEX;
        }
    const int64_t ntrip = nf * nl * nl;
    triplet_t *T = (triplet_t *)malloc(sizeof(triplet_t) * (ntrip > 0 ? ntrip : 1));
    if (!T) return OR_ERR_NOMEM;
    int64_t t = 0;
    for (int64_t k = 0; k < nf; ++k) {
        double P[MAXNL][MAXD];
        int32_t vid[MAXNL];
        for (int a = 0; a < nl; ++a) {
            vid[a] = facets[(int64_t)a * nf + k];
            for (int i = 0; i < d; ++i) P[a][i] = q[(int64_t)i * nq + vid[a]];
        }
        const double vol = gram_measure(d, n, P);
        if (vol == 0.0) {
            free(T);
            return OR_ERR_DEGENERATE;
        }
        for (int b = 0; b < nl; ++b)
            for (int a = 0; a < nl; ++a) {
                double s = 0.0, sa = 0.0;
                if (!w) {
                    int ex[MAXNL] = {0, 0, 0, 0};
                    ex[a] += 1;
                    ex[b] += 1;
                    s = sa = magic_factor(n, ex);
                } else {
                    for (int g = 0; g < nl; ++g) {
                        int ex[MAXNL] = {0, 0, 0, 0};
                        ex[a] += 1;
                        ex[b] += 1;
                        ex[g] += 1;
                        s += w[vid[g]] * magic_factor(n, ex);
                        sa += fabs(w[vid[g]]) * magic_factor(n, ex);
                    }
                }
                T[t].row = vid[a];
                T[t].col = vid[b];
                T[t].seq = t;
                T[t].val = vol * s;
                T[t].aval = vol * sa;
                ++t;
            }
    }
    qsort(T, (size_t)t, sizeof(triplet_t), cmp_triplet);
    int64_t nnz = 0;
    for (int64_t i = 0; i < t; ++i)
        if (i == 0 || T[i].row != T[i - 1].row || T[i].col != T[i - 1].col) ++nnz;
    if (nnz > cap) {
        free(T);
        return OR_ERR_OVERFLOW;
    }
    for (int64_t r = 0; r <= nq; ++r) row_ptr[r] = 0;
    int64_t s = -1;
    for (int64_t i = 0; i < t; ++i) {
        if (i == 0 || T[i].row != T[i - 1].row || T[i].col != T[i - 1].col) {
            ++s;
            col_idx[s] = T[i].col;
            val[s] = 0.0;
            if (absval) absval[s] = 0.0;
            row_ptr[T[i].row + 1] += 1;
        }
        val[s] += T[i].val;
        if (absval) absval[s] += T[i].aval;
    }
    for (int64_t r = 0; r < nq; ++r) row_ptr[r + 1] += row_ptr[r];
    *nnz_out = nnz;
    free(T);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Derivatives of the assembly map (q, w) -> A for the mass, weighted mass   */
/* and stiffness operators, by complex-step differentiation of each element  */
/* matrix (imaginary step 1e-30: no truncation or cancellation error).       */
/*   JVP: dA = sum_K P_K^T dE(K) P_K, dE = Im E(q + i h dq, w + i h dw) / h,  */
/*        summed by `sparse` as the assembly is;                              */
/*   VJP: for L = sum_s G_s A_s, dL/dq and dL/dw accumulated per vertex in    */
/*        ascending element number, G_s read at the CSR entry of each local   */
/*        (row, column) pair (rp, ci: the operator's pattern).                 */
/* ------------------------------------------------------------------------ */

/* E (nl x nl) of MASS, MASS_W or STIFF in complex arithmetic. */
static int element_matrix_c(int d, int op, double complex P[MAXNL][MAXD],
                            const double complex *wl, double complex E[MAXNL][MAXNL]) {
    double complex B[MAXD][MAXD], Bt[MAXD][MAXD], R[MAXD][MAXNL], G[MAXD][MAXNL];
    for (int i = 0; i < d; ++i)
        for (int c = 0; c < d; ++c) B[i][c] = P[c + 1][i] - P[0][i];
    double complex det = det_cplx(d, B);
    if (creal(det) == 0.0) return 0;
    const int nl = d + 1;
    const double complex vol = (creal(det) < 0 ? -det : det) / factorial(d);
    if (op == OR_STIFF) {
        for (int i = 0; i < d; ++i)
            for (int c = 0; c < d; ++c) Bt[i][c] = B[c][i];
        for (int i = 0; i < d; ++i) {
            R[i][0] = -1.0;
            for (int a = 1; a < nl; ++a) R[i][a] = (a - 1 == i) ? 1.0 : 0.0;
        }
        if (!solve_cplx(d, Bt, R, G)) return 0;
    }
    for (int a = 0; a < nl; ++a)
        for (int b = 0; b < nl; ++b) {
            double complex s = 0.0;
            if (op == OR_STIFF) {
                for (int i = 0; i < d; ++i) s += G[i][b] * G[i][a];
            } else if (op == OR_MASS) {
                int ex[MAXNL] = {0, 0, 0, 0};
                ex[a] += 1; ex[b] += 1;
                s = magic_factor(d, ex);
            } else {
                for (int g = 0; g < nl; ++g) {
                    int ex[MAXNL] = {0, 0, 0, 0};
                    ex[a] += 1; ex[b] += 1; ex[g] += 1;
                    s += wl[g] * magic_factor(d, ex);
                }
            }
            E[a][b] = vol * s;
        }
    return 1;
}

static int64_t csr_find(const int64_t *rp, const int64_t *ci, int64_t r, int64_t c) {
    int64_t lo = rp[r], hi = rp[r + 1];
    while (lo < hi) {
        const int64_t m = (lo + hi) / 2;
        if (ci[m] < c) lo = m + 1; else hi = m;
    }
    return (lo < rp[r + 1] && ci[lo] == c) ? lo : -1;
}

int oracle_jvp(int d, int64_t nq, int64_t nme, const double *q, const int32_t *me, int op,
               const double *w, const double *dq, const double *dw, int64_t cap,
               int64_t *nnz_out, int64_t *row_ptr, int64_t *col_idx, double *val, double *absval) {
    int st = oracle_validate(d, nq, nme, me);
    if (st != OR_OK) return st;
    if (op != OR_MASS && op != OR_MASS_W && op != OR_STIFF) return OR_ERR_ARG;
    if (nme > 0 && (!q || !dq || (op == OR_MASS_W && (!w || !dw)))) return OR_ERR_ARG;
    const int nl = d + 1;
    const double h = 1e-30;
    triplet_t *T = (triplet_t *)malloc(sizeof(triplet_t) * (nme > 0 ? nme * nl * nl : 1));
    if (!T) return OR_ERR_NOMEM;
    int64_t t = 0;
    for (int64_t k = 0; k < nme; ++k) {
        int32_t vid[MAXNL];
        double complex P[MAXNL][MAXD], wl[MAXNL], E[MAXNL][MAXNL];
        for (int a = 0; a < nl; ++a) {
            vid[a] = me[(int64_t)a * nme + k];
            for (int i = 0; i < d; ++i)
                P[a][i] = q[(int64_t)i * nq + vid[a]] + I * h * dq[(int64_t)i * nq + vid[a]];
            wl[a] = op == OR_MASS_W ? w[vid[a]] + I * h * dw[vid[a]] : 0.0;
        }
        if (!element_matrix_c(d, op, P, wl, E)) {
            free(T);
            return OR_ERR_DEGENERATE;
        }
        for (int b = 0; b < nl; ++b)
            for (int a = 0; a < nl; ++a) {
                T[t].row = vid[a];
                T[t].col = vid[b];
                T[t].seq = t;
                T[t].val = cimag(E[a][b]) / h;
                T[t].aval = fabs(T[t].val);
                ++t;
            }
    }
    qsort(T, (size_t)t, sizeof(triplet_t), cmp_triplet);
    int64_t nnz = 0;
    for (int64_t i = 0; i < t; ++i)
        if (i == 0 || T[i].row != T[i - 1].row || T[i].col != T[i - 1].col) ++nnz;
    if (nnz > cap) {
        free(T);
        return OR_ERR_OVERFLOW;
    }
    for (int64_t r = 0; r <= nq; ++r) row_ptr[r] = 0;
    int64_t s = -1;
    for (int64_t i = 0; i < t; ++i) {
        if (i == 0 || T[i].row != T[i - 1].row || T[i].col != T[i - 1].col) {
            ++s;
            col_idx[s] = T[i].col;
            val[s] = 0.0;
            if (absval) absval[s] = 0.0;
            row_ptr[T[i].row + 1] += 1;
        }
        val[s] += T[i].val;
        if (absval) absval[s] += T[i].aval;
    }
    for (int64_t r = 0; r < nq; ++r) row_ptr[r + 1] += row_ptr[r];
    *nnz_out = nnz;
    free(T);
    return OR_OK;
}

/* VJP.  want[v] != 0 selects the vertices whose dq / dw are computed (NULL:
 * all); dq_out is d x nq (like q), dw_out nq; either may be NULL.  The *_abs
 * arrays receive the sums of |element contribution| (tolerance scale). */
int oracle_vjp(int d, int64_t nq, int64_t nme, const double *q, const int32_t *me, int op,
               const double *w, const int64_t *rp, const int64_t *ci, const double *G,
               const uint8_t *want, double *dq_out, double *dw_out, double *dq_abs,
               double *dw_abs) {
    int st = oracle_validate(d, nq, nme, me);
    if (st != OR_OK) return st;
    if (op != OR_MASS && op != OR_MASS_W && op != OR_STIFF) return OR_ERR_ARG;
    if (nme > 0 && (!q || !rp || !ci || !G || (op == OR_MASS_W && !w))) return OR_ERR_ARG;
    const int nl = d + 1;
    const double h = 1e-30;
    if (dq_out) memset(dq_out, 0, sizeof(double) * (size_t)(d * nq));
    if (dw_out) memset(dw_out, 0, sizeof(double) * (size_t)nq);
    if (dq_abs) memset(dq_abs, 0, sizeof(double) * (size_t)(d * nq));
    if (dw_abs) memset(dw_abs, 0, sizeof(double) * (size_t)nq);
    for (int64_t k = 0; k < nme; ++k) {
        int32_t vid[MAXNL];
        int need = 0;
        for (int a = 0; a < nl; ++a) {
            vid[a] = me[(int64_t)a * nme + k];
            need |= !want || want[vid[a]];
        }
        if (!need) continue;
        double Gk[MAXNL][MAXNL];
        for (int a = 0; a < nl; ++a)
            for (int b = 0; b < nl; ++b) {
                const int64_t s = csr_find(rp, ci, vid[a], vid[b]);
                if (s < 0) return OR_ERR_INDEX;
                Gk[a][b] = G[s];
            }
        double complex P0[MAXNL][MAXD], w0[MAXNL];
        for (int a = 0; a < nl; ++a) {
            for (int i = 0; i < d; ++i) P0[a][i] = q[(int64_t)i * nq + vid[a]];
            w0[a] = op == OR_MASS_W ? w[vid[a]] : 0.0;
        }
        for (int c = 0; c < nl; ++c) {
            if (want && !want[vid[c]]) continue;
            for (int i = 0; i < d + 1; ++i) {
                if (i == d && (op != OR_MASS_W || !dw_out)) continue;
                if (i < d && !dq_out) continue;
                double complex P[MAXNL][MAXD], wl[MAXNL], E[MAXNL][MAXNL];
                memcpy(P, P0, sizeof(P));
                memcpy(wl, w0, sizeof(wl));
                if (i < d) P[c][i] += I * h;
                else wl[c] += I * h;
                if (!element_matrix_c(d, op, P, wl, E)) return OR_ERR_DEGENERATE;
                double s = 0.0, sa = 0.0;
                for (int a = 0; a < nl; ++a)
                    for (int b = 0; b < nl; ++b) {
                        s += Gk[a][b] * (cimag(E[a][b]) / h);
                        sa += fabs(Gk[a][b] * (cimag(E[a][b]) / h));
                    }
                if (i < d) {
                    dq_out[(int64_t)i * nq + vid[c]] += s;
                    if (dq_abs) dq_abs[(int64_t)i * nq + vid[c]] += sa;
                } else {
                    dw_out[vid[c]] += s;
                    if (dw_abs) dw_abs[vid[c]] += sa;
                }
            }
        }
    }
    return OR_OK;
}
