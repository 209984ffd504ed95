// Adjoint of J(q, w) = a^T (S(q) + M_w(q)) b.
//
// Per element K with barycentric gradients g_c, |K| = |det B_k|/d!,
// u = sum_c a_c g_c and v = sum_c b_c g_c, the gradient systems of the
// paper's Appendix C.1 (B_k^T G_k = [-1 | I_d]) give, for a perturbation of
// the vertices, d g_a = -sum_c g_c (g_a . d q_c) and d|K| = |K| sum_c g_c . d q_c.
// Hence for local vertex c:
//   dJ/dq_c += |K| [ (u.v) g_c - (g_c.v) u - (g_c.u) v ]        (stiffness term)
//            + s_K g_c,    s_K = a_K^T E_mass_w(K) b_K           (mass term, E ~ |K|)
// and, since E_mass_w is linear in w with coefficients from the magic
// formula, with A = sum a, B = sum b, kk = |K| d!/(d+3)!:
//   dJ/dw_c += kk [ A B + a_c B + A b_c + sum_e a_e b_e + 2 a_c b_c ].
// Each vertex is handled by kLanes consecutive lanes: lane j adds the
// contributions of its incidences j, j+kLanes, ... (ascending element
// number), and the partial sums are combined as ((p0+p1)+(p2+p3)) through
// lane shuffles, so the result is deterministic without atomics.
#include "element.h"
#include "femasm_impl.h"
#include "rowgather.h"

namespace femasm {

constexpr int kLanes = 4;   // lanes per vertex

template <int D>
__global__ void __launch_bounds__(256)
    k_backward(MeshView mv, const double *__restrict__ av, const double *__restrict__ bv,
               uint32_t mask, double *__restrict__ dJdw, double *__restrict__ dJdq,
               int32_t *status) {
    constexpr int NL = D + 1;
    const int64_t gt = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t i = gt / kLanes;
    const int j = int(gt % kLanes);
    const bool stiff = mask & (1u << FEM_OP_STIFF);
    const bool mass = mask & (1u << FEM_OP_MASS_W);
    int bad = 0;
    double gw = 0.0, gq[D];
#pragma unroll
    for (int x = 0; x < D; ++x) gq[x] = 0.0;
    if (i < mv.nq) {
        const int64_t nq = mv.nq;
        for (int t = mv.inc_ptr[i] + j; t < mv.inc_ptr[i + 1]; t += kLanes) {
            const uint32_t ea = mv.inc_elem[t];
            const int64_t e = ea & 0x3fffffffu;
            const int al = int(ea >> 30);
            int v[NL];
            double P[NL][D], la[NL], lb[NL];
#pragma unroll
            for (int b = 0; b < NL; ++b) {
                v[b] = mv.pme[e * NL + b];
                la[b] = av[v[b]];
                lb[b] = bv[v[b]];
#pragma unroll
                for (int x = 0; x < D; ++x) P[b][x] = mv.q[x * nq + v[b]];
            }
            Elem<D> E;
            elem_geometry(P, E);
            if (E.det == 0.0) { bad = 1; continue; }
            const double rdet = 1.0 / E.det;
            const double vol = fabs(E.det) / Fact<D>::dfact;
            double g[NL][D];
#pragma unroll
            for (int b = 0; b < NL; ++b)
#pragma unroll
                for (int x = 0; x < D; ++x) g[b][x] = E.c[b][x] * rdet;
            double ga[D];
#pragma unroll
            for (int x = 0; x < D; ++x) {
                double cx[NL];
#pragma unroll
                for (int b = 0; b < NL; ++b) cx[b] = g[b][x];
                ga[x] = sel<D>(cx, al);
            }
            if (stiff) {
                double u[D], w2[D];
#pragma unroll
                for (int x = 0; x < D; ++x) {
                    u[x] = 0.0;
                    w2[x] = 0.0;
#pragma unroll
                    for (int b = 0; b < NL; ++b) {
                        u[x] += la[b] * g[b][x];
                        w2[x] += lb[b] * g[b][x];
                    }
                }
                const double uv = cdot<D>(u, w2), gv = cdot<D>(ga, w2), gu = cdot<D>(ga, u);
#pragma unroll
                for (int x = 0; x < D; ++x) gq[x] += vol * (uv * ga[x] - gv * u[x] - gu * w2[x]);
            }
            if (mass) {
                double wl[NL];
#pragma unroll
                for (int b = 0; b < NL; ++b) wl[b] = mv.w[v[b]];
                double A = 0.0, B = 0.0, ab = 0.0, ws = 0.0, aw = 0.0, bw = 0.0, abw = 0.0;
#pragma unroll
                for (int b = 0; b < NL; ++b) {
                    A += la[b];
                    B += lb[b];
                    ab += la[b] * lb[b];
                    ws += wl[b];
                    aw += la[b] * wl[b];
                    bw += lb[b] * wl[b];
                    abw += la[b] * lb[b] * wl[b];
                }
                const double kk = fabs(E.det) / Fact<D>::massw_den;
                // s_K = sum_ab a_a b_b kk (1+delta_ab)(w^s + w_a + w_b)
                const double sK = kk * (A * B * ws + aw * B + A * bw + ws * ab + 2.0 * abw);
#pragma unroll
                for (int x = 0; x < D; ++x) gq[x] += sK * ga[x];
                const double aa = sel<D>(la, al), bb = sel<D>(lb, al);
                gw += kk * (A * B + aa * B + A * bb + ab + 2.0 * aa * bb);
            }
        }
    }
    // ((p0 + p1) + (p2 + p3)): every lane of the group ends with the same bits
#pragma unroll
    for (int sh = 1; sh < kLanes; sh <<= 1) {
        gw += __shfl_xor(gw, sh, kLanes);
#pragma unroll
        for (int x = 0; x < D; ++x) gq[x] += __shfl_xor(gq[x], sh, kLanes);
    }
    if (i < mv.nq && j == 0) {
        if (dJdw) dJdw[i] = gw;
        if (dJdq)
#pragma unroll
            for (int x = 0; x < D; ++x) dJdq[x * mv.nq + i] = gq[x];
    }
    const unsigned long long any = __ballot(bad != 0);
    if (any != 0ull && (threadIdx.x & 63) == __ffsll((long long)any) - 1) atomicOr(status, bad);
}

}  // namespace femasm

using namespace femasm;

static fem_status fem_assemble_backward_impl(fem_plan plan, uint32_t op_mask, const double *q,
                                            const double *w, const double *a, const double *b,
                                            double *dJdw, double *dJdq, hipStream_t stream) {
    PhaseRange range("femasm: backward (adjoint)");
    const uint32_t allowed = (1u << FEM_OP_STIFF) | (1u << FEM_OP_MASS_W);
    if (!plan || (op_mask & ~allowed) || op_mask == 0) return FEM_ERR_ARG;
    if (plan->nq == 0) return FEM_OK;
    if (!q || !a || !b || ((op_mask & (1u << FEM_OP_MASS_W)) && !w)) return FEM_ERR_ARG;
    MeshView mv{};
    mv.rp = plan->rp;
    mv.inc_ptr = plan->inc_ptr;
    mv.inc_elem = plan->inc_elem;
    mv.inc_off = plan->inc_off;
    mv.pme = plan->pme;
    mv.q = q;
    mv.w = w;
    mv.values = nullptr;
    mv.nq = plan->nq;
    const unsigned grid = unsigned((plan->nq * kLanes + 255) / 256);
    if (plan->d == 2)
        hipLaunchKernelGGL(k_backward<2>, dim3(grid), dim3(256), 0, stream, mv, a, b, op_mask,
                           dJdw, dJdq, plan->status);
    else
        hipLaunchKernelGGL(k_backward<3>, dim3(grid), dim3(256), 0, stream, mv, a, b, op_mask,
                           dJdw, dJdq, plan->status);
    return hip_status(hipGetLastError());
}

extern "C" fem_status fem_assemble_backward(fem_plan plan, uint32_t op_mask, const double *q,
                                            const double *w, const double *a, const double *b,
                                            double *dJdw, double *dJdq, hipStream_t stream) {
    return debug_check(fem_assemble_backward_impl(plan, op_mask, q, w, a, b, dJdw, dJdq, stream),
                       stream, plan ? plan->status : nullptr);
}
