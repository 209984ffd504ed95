// Derivatives of the assembly map (q, w) -> A for the mass, weighted mass
// and stiffness operators: the directional derivative (JVP) and the
// gradient of L = sum_s G_s A_s (VJP) for an arbitrary upstream gradient G
// on the CSR entries.
//
// Per element, with g_c the barycentric gradients (g_c = c_c / det), |K| =
// |det|/d! and a perturbation dq_c of its vertices, the gradient systems of
// Appendix C.1 give d g_a = -N g_a with N = sum_c g_c dq_c^T, and
// d|K| = |K| t with t = tr N = sum_c g_c . dq_c.  Hence
//   stiffness  dE_ab = |K| [ t g_a.g_b - (N g_a).g_b - g_a.(N g_b) ]
//   mass       dE_ab = E_ab t          (E proportional to |K|)
//   weighted   dE_ab = E_ab t + |K| d!/(d+3)! (1+delta_ab) (dw^s + dw_a + dw_b)
// and, for L_K = sum_ab G_ab E_ab(K) with G_ab the upstream gradient at the
// entry (me[a,K], me[b,K]),
//   stiffness  dL_K/dq_c = |K| [ s g_c - sum_a z_a g_a ],  s = sum_ab G_ab g_a.g_b,
//              z = (G + G^T) y, y_a = g_a . g_c
//   masses     dL_K/dq_c = (sum_ab G_ab E_ab) g_c
//   weighted   dL_K/dw_c = |K| d!/(d+3)! [ sum G + tr G + (row_c + col_c of G) + 2 G_cc ].
// JVP: by default on the vertex-pair kernel (pair.hip: the tangent of the
// packed element matrix in the element phase, then the same ordered pair
// sums); else one thread per CSR row adds the tangent element rows of its
// vertex into an LDS tile of the workgroup's CSR range, in ascending element
// number (the row-gather scheme of the numeric phase), then the tile is
// written coalesced.  VJP: kVjpLanes lanes per vertex, each lane summing its
// share of the vertex's incidences, partial sums combined in a fixed order.
// Workspace VJP: the same terms evaluated once per element into a caller
// buffer, then summed per vertex with the same lanes and order, so the two
// forms agree bit for bit.
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <type_traits>

#include "element.h"
#include "femasm_impl.h"
#include "rowgather.h"

#pragma clang fp contract(off)

namespace femasm {

namespace {

// VJP: lanes per vertex; each lane walks every kVjpLanes-th incidence and the
// partials are combined by lane shuffles in a fixed order.  Eight lanes
// shorten each lane's chain of dependent gathers (incidence, element,
// slot map, upstream gradient) enough to hide more of their latency:
// 1.97 ms against 3.04 ms with four on the 128^3 cube; sixteen gain
// nothing more.
constexpr int kVjpLanes = 8;
constexpr int kVjpElemWG = 256;   // threads (elements) per workgroup of k_vjp_elem
constexpr int kGatherDepth = 4;    // incidences per lane in flight in k_vjp_gather

template <int D, int OP>
__global__ void __launch_bounds__(256) k_jvp(MeshView mv, const double *__restrict__ dq,
                                             const double *__restrict__ dw, int32_t *status) {
    constexpr int NL = D + 1;
    extern __shared__ double acc[];
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t r0 = tile * blockDim.x;
    const int64_t r1 = min(r0 + int64_t(blockDim.x), mv.nq);
    const int64_t base = mv.rp[r0];
    const int nacc = int(mv.rp[r1] - base);
    for (int s = threadIdx.x; s < nacc; s += blockDim.x) acc[s] = 0.0;
    __syncthreads();
    int bad = 0;
    const int64_t i = r0 + threadIdx.x;
    if (i < r1) {
        double *__restrict__ my = acc + (mv.rp[i] - base);
        const int64_t nq = mv.nq;
        for (int t = mv.inc_ptr[i]; t < mv.inc_ptr[i + 1]; ++t) {
            const uint32_t ea = mv.inc_elem[t];
            const uint64_t off = mv.inc_off[t];
            const int64_t e = ea & 0x3fffffffu;
            const int al = int(ea >> 30);
            int v[NL];
            double P[NL][D], dP[NL][D];
#pragma unroll
            for (int b = 0; b < NL; ++b) {
                v[b] = mv.pme[e * NL + b];
#pragma unroll
                for (int x = 0; x < D; ++x) {
                    P[b][x] = mv.q[x * nq + v[b]];
                    dP[b][x] = dq[x * nq + v[b]];
                }
            }
            Elem<D> E;
            elem_geometry(P, E);
            if (E.det == 0.0) {
                bad = 1;
                continue;
            }
            const double rdet = 1.0 / E.det;
            const double ad = fabs(E.det);
            double g[NL][D];
#pragma unroll
            for (int b = 0; b < NL; ++b)
#pragma unroll
                for (int x = 0; x < D; ++x) g[b][x] = E.c[b][x] * rdet;
            // N = sum_c g_c dq_c^T, t = tr N
            double N[D][D];
#pragma unroll
            for (int x = 0; x < D; ++x)
#pragma unroll
                for (int y = 0; y < D; ++y) {
                    double s = g[0][x] * dP[0][y];
#pragma unroll
                    for (int c = 1; c < NL; ++c) s = fma(g[c][x], dP[c][y], s);
                    N[x][y] = s;
                }
            double tr = N[0][0];
#pragma unroll
            for (int x = 1; x < D; ++x) tr += N[x][x];
            double ga[D];
#pragma unroll
            for (int x = 0; x < D; ++x) {
                double cx[NL];
#pragma unroll
                for (int b = 0; b < NL; ++b) cx[b] = g[b][x];
                ga[x] = sel<D>(cx, al);
            }
            if constexpr (OP == FEM_OP_STIFF) {
                const double vol = ad / Fact<D>::dfact;
                double Nga[D];
#pragma unroll
                for (int x = 0; x < D; ++x) Nga[x] = cdot<D>(N[x], ga);
#pragma unroll
                for (int b = 0; b < NL; ++b) {
                    double Ngb[D];
#pragma unroll
                    for (int x = 0; x < D; ++x) Ngb[x] = cdot<D>(N[x], g[b]);
                    const double de =
                        vol * ((tr * cdot<D>(ga, g[b]) - cdot<D>(Nga, g[b])) - cdot<D>(ga, Ngb));
                    const int pos = int((off >> (16 * b)) & 0xffffu);
                    my[pos] += de;
                }
            } else if constexpr (OP == FEM_OP_MASS) {
                const double k = ad / Fact<D>::mass_den;
#pragma unroll
                for (int b = 0; b < NL; ++b) {
                    const int pos = int((off >> (16 * b)) & 0xffffu);
                    my[pos] += ((b == al) ? 2.0 * k : k) * tr;
                }
            } else {
                double wl[NL], dwl[NL];
#pragma unroll
                for (int b = 0; b < NL; ++b) {
                    wl[b] = mv.w[v[b]];
                    dwl[b] = dw[v[b]];
                }
                double ws = wl[0], dws = dwl[0];
#pragma unroll
                for (int b = 1; b < NL; ++b) {
                    ws += wl[b];
                    dws += dwl[b];
                }
                const double k = ad / Fact<D>::massw_den;
                const double wa = sel<D>(wl, al), dwa = sel<D>(dwl, al);
#pragma unroll
                for (int b = 0; b < NL; ++b) {
                    const double f = (b == al) ? 2.0 * k : k;
                    const int pos = int((off >> (16 * b)) & 0xffffu);
                    my[pos] += f * ((ws + (wa + wl[b])) * tr + (dws + (dwa + dwl[b])));
                }
            }
        }
    }
    __syncthreads();
    for (int s = threadIdx.x; s < nacc; s += blockDim.x) mv.values[base + s] = acc[s];
    const unsigned long long any = __ballot(bad != 0);
    if (any != 0ull && (threadIdx.x & 63) == __ffsll((long long)any) - 1) atomicOr(status, bad);
}

// Geometry of one element for the VJP terms: barycentric gradients and
// |det B_K|.  False for a degenerate element (no contribution).
template <int D>
struct VjpGeom {
    double g[D + 1][D];
    double ad;
};

template <int D>
__device__ __forceinline__ bool vjp_geometry(const double (&P)[D + 1][D], VjpGeom<D> &V) {
    Elem<D> E;
    elem_geometry(P, E);
    if (E.det == 0.0) return false;
    const double rdet = 1.0 / E.det;
    V.ad = fabs(E.det);
#pragma unroll
    for (int b = 0; b < D + 1; ++b)
#pragma unroll
        for (int x = 0; x < D; ++x) V.g[b][x] = E.c[b][x] * rdet;
    return true;
}

// The VJP term of one element at its local vertex al: tq (d values, the
// contribution to dL/dq at that vertex) and, for the weighted mass, tw (to
// dL/dw).  Gk[a][b] is the upstream gradient at the element's entry (a, b);
// wl the element's nodal weights (weighted mass only).
template <int D, int OP>
__device__ __forceinline__ void vjp_term(const VjpGeom<D> &V, const double (&Gk)[D + 1][D + 1],
                                         const double (&wl)[D + 1], int al, double (&tq)[D],
                                         double &tw) {
    constexpr int NL = D + 1;
    double gc[D];
#pragma unroll
    for (int x = 0; x < D; ++x) {
        double cx[NL];
#pragma unroll
        for (int b = 0; b < NL; ++b) cx[b] = V.g[b][x];
        gc[x] = sel<D>(cx, al);
    }
    // sums of G used by the mass terms
    double gsum = 0.0, gtr = 0.0, rowc = 0.0, colc = 0.0, gcc = 0.0;
#pragma unroll
    for (int a = 0; a < NL; ++a) {
        gtr += Gk[a][a];
#pragma unroll
        for (int b = 0; b < NL; ++b) {
            gsum += Gk[a][b];
            if (a == al) rowc += Gk[a][b];
            if (b == al) colc += Gk[a][b];
        }
        if (a == al) gcc = Gk[a][a];
    }
    tw = 0.0;
    if constexpr (OP == FEM_OP_STIFF) {
        const double vol = V.ad / Fact<D>::dfact;
        double y[NL], s = 0.0;
#pragma unroll
        for (int a = 0; a < NL; ++a) y[a] = cdot<D>(V.g[a], gc);
#pragma unroll
        for (int a = 0; a < NL; ++a)
#pragma unroll
            for (int b = 0; b < NL; ++b) s = fma(Gk[a][b], cdot<D>(V.g[a], V.g[b]), s);
        double Uz[D];
#pragma unroll
        for (int x = 0; x < D; ++x) Uz[x] = 0.0;
#pragma unroll
        for (int a = 0; a < NL; ++a) {
            double z = 0.0;
#pragma unroll
            for (int b = 0; b < NL; ++b) z = fma(Gk[a][b] + Gk[b][a], y[b], z);
#pragma unroll
            for (int x = 0; x < D; ++x) Uz[x] = fma(z, V.g[a][x], Uz[x]);
        }
#pragma unroll
        for (int x = 0; x < D; ++x) tq[x] = vol * (s * gc[x] - Uz[x]);
    } else if constexpr (OP == FEM_OP_MASS) {
        const double sk = V.ad / Fact<D>::mass_den * (gsum + gtr);
#pragma unroll
        for (int x = 0; x < D; ++x) tq[x] = sk * gc[x];
    } else {
        double ws = wl[0];
#pragma unroll
        for (int b = 1; b < NL; ++b) ws += wl[b];
        const double kk = V.ad / Fact<D>::massw_den;
        // sum_ab G_ab (1+delta_ab)(w^s + w_a + w_b)
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < NL; ++a)
#pragma unroll
            for (int b = 0; b < NL; ++b)
                s = fma(Gk[a][b] * (a == b ? 2.0 : 1.0), ws + (wl[a] + wl[b]), s);
        const double sk = kk * s;
#pragma unroll
        for (int x = 0; x < D; ++x) tq[x] = sk * gc[x];
        tw = kk * ((gsum + gtr) + (rowc + colc) + 2.0 * gcc);
    }
}

// Where the VJP finds the upstream gradient of entry (a, b) of an element:
// through the caller's slot map (indexed by caller element number), or,
// when `slot` is null, through the plan's per-element column positions
// (indexed by plan element number, next to the connectivity the kernels
// read anyway) and the row pointers.  Both give the same address.
struct GAddr {
    const int32_t *slot;
    const void *vpos;   // 8-bit (PB 1) or 16-bit (PB 2) positions
};

// The upstream gradient block Gk[a][b] of plan element e with vertices v;
// PB: 0 slot map, 1 or 2 bytes per plan position.
template <int D, int PB>
__device__ __forceinline__ void vjp_gk(const MeshView &mv, const int32_t *__restrict__ porig,
                                       const GAddr &ga, const double *__restrict__ G, int64_t e,
                                       const int (&v)[D + 1], double (&Gk)[D + 1][D + 1]) {
    constexpr int NL = D + 1;
    if constexpr (PB == 0) {
        const int64_t k = porig[e];
#pragma unroll
        for (int b = 0; b < NL; ++b)
#pragma unroll
            for (int a = 0; a < NL; ++a) Gk[a][b] = G[ga.slot[k * NL * NL + b * NL + a]];
    } else {
        using T = typename std::conditional<PB == 1, uint8_t, uint16_t>::type;
        const T *pos = static_cast<const T *>(ga.vpos) + e * NL * NL;
#pragma unroll
        for (int a = 0; a < NL; ++a) {
            const int64_t r0 = mv.rp[v[a]];
#pragma unroll
            for (int b = 0; b < NL; ++b) Gk[a][b] = G[r0 + pos[b * NL + a]];
        }
    }
}

// Loads of one element (internal number e) for the VJP: coordinates, the
// upstream gradient block, nodal weights.
template <int D, int OP, int PB>
__device__ __forceinline__ void vjp_load(const MeshView &mv, const int32_t *__restrict__ porig,
                                         const GAddr &ga, const double *__restrict__ G, int64_t e,
                                         double (&P)[D + 1][D], double (&Gk)[D + 1][D + 1],
                                         double (&wl)[D + 1]) {
    constexpr int NL = D + 1;
    int v[NL];
#pragma unroll
    for (int b = 0; b < NL; ++b) {
        v[b] = mv.pme[e * NL + b];
#pragma unroll
        for (int x = 0; x < D; ++x) P[b][x] = mv.q[x * mv.nq + v[b]];
        wl[b] = OP == FEM_OP_MASS_W ? mv.w[v[b]] : 0.0;
    }
    vjp_gk<D, PB>(mv, porig, ga, G, e, v, Gk);
}

// Lane-strided sums of one vertex's incidence terms, combined by shuffles in
// a fixed tree; lane 0 of each group writes the vertex's outputs.
template <int D>
__device__ __forceinline__ void vjp_store(const MeshView &mv, int64_t i, int j, double (&gq)[D],
                                          double gw, double *__restrict__ dLdq,
                                          double *__restrict__ dLdw) {
#pragma unroll
    for (int sh = 1; sh < kVjpLanes; sh <<= 1) {
        gw += __shfl_xor(gw, sh, kVjpLanes);
#pragma unroll
        for (int x = 0; x < D; ++x) gq[x] += __shfl_xor(gq[x], sh, kVjpLanes);
    }
    if (i < mv.nq && j == 0) {
        if (dLdw) dLdw[i] = gw;
        if (dLdq)
#pragma unroll
            for (int x = 0; x < D; ++x) dLdq[x * mv.nq + i] = gq[x];
    }
}

template <int D, int OP, int PB>
__global__ void __launch_bounds__(256)
    k_vjp(MeshView mv, const int32_t *__restrict__ porig, GAddr ga,
          const double *__restrict__ G, double *__restrict__ dLdq, double *__restrict__ dLdw,
          int32_t *status) {
    constexpr int NL = D + 1;
    const int64_t gt = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t i = gt / kVjpLanes;
    const int j = int(gt % kVjpLanes);
    int bad = 0;
    double gw = 0.0, gq[D];
#pragma unroll
    for (int x = 0; x < D; ++x) gq[x] = 0.0;
    if (i < mv.nq) {
        const int64_t nq = mv.nq;
        for (int t = mv.inc_ptr[i] + j; t < mv.inc_ptr[i + 1]; t += kVjpLanes) {
            const uint32_t ea = mv.inc_elem[t];
            const int64_t e = ea & 0x3fffffffu;
            const int al = int(ea >> 30);
            int v[NL];
            double P[NL][D];
#pragma unroll
            for (int b = 0; b < NL; ++b) {
                v[b] = mv.pme[e * NL + b];
#pragma unroll
                for (int x = 0; x < D; ++x) P[b][x] = mv.q[x * nq + v[b]];
            }
            double Gk[NL][NL];
            vjp_gk<D, PB>(mv, porig, ga, G, e, v, Gk);
            Elem<D> E;
            elem_geometry(P, E);
            if (E.det == 0.0) {
                bad = 1;
                continue;
            }
            const double rdet = 1.0 / E.det;
            const double ad = fabs(E.det);
            double g[NL][D];
#pragma unroll
            for (int b = 0; b < NL; ++b)
#pragma unroll
                for (int x = 0; x < D; ++x) g[b][x] = E.c[b][x] * rdet;
            double gc[D];
#pragma unroll
            for (int x = 0; x < D; ++x) {
                double cx[NL];
#pragma unroll
                for (int b = 0; b < NL; ++b) cx[b] = g[b][x];
                gc[x] = sel<D>(cx, al);
            }
            // sums of G used by the mass terms
            double gsum = 0.0, gtr = 0.0, rowc = 0.0, colc = 0.0, gcc = 0.0;
#pragma unroll
            for (int a = 0; a < NL; ++a) {
                gtr += Gk[a][a];
#pragma unroll
                for (int b = 0; b < NL; ++b) {
                    gsum += Gk[a][b];
                    if (a == al) rowc += Gk[a][b];
                    if (b == al) colc += Gk[a][b];
                }
                if (a == al) gcc = Gk[a][a];
            }
            if constexpr (OP == FEM_OP_STIFF) {
                const double vol = ad / Fact<D>::dfact;
                double y[NL], s = 0.0;
#pragma unroll
                for (int a = 0; a < NL; ++a) y[a] = cdot<D>(g[a], gc);
#pragma unroll
                for (int a = 0; a < NL; ++a)
#pragma unroll
                    for (int b = 0; b < NL; ++b) s = fma(Gk[a][b], cdot<D>(g[a], g[b]), s);
                double Uz[D];
#pragma unroll
                for (int x = 0; x < D; ++x) Uz[x] = 0.0;
#pragma unroll
                for (int a = 0; a < NL; ++a) {
                    double z = 0.0;
#pragma unroll
                    for (int b = 0; b < NL; ++b) z = fma(Gk[a][b] + Gk[b][a], y[b], z);
#pragma unroll
                    for (int x = 0; x < D; ++x) Uz[x] = fma(z, g[a][x], Uz[x]);
                }
#pragma unroll
                for (int x = 0; x < D; ++x) gq[x] += vol * (s * gc[x] - Uz[x]);
            } else if constexpr (OP == FEM_OP_MASS) {
                const double sk = ad / Fact<D>::mass_den * (gsum + gtr);
#pragma unroll
                for (int x = 0; x < D; ++x) gq[x] += sk * gc[x];
            } else {
                double wl[NL];
#pragma unroll
                for (int b = 0; b < NL; ++b) wl[b] = mv.w[v[b]];
                double ws = wl[0];
#pragma unroll
                for (int b = 1; b < NL; ++b) ws += wl[b];
                const double kk = ad / Fact<D>::massw_den;
                // sum_ab G_ab (1+delta_ab)(w^s + w_a + w_b)
                double s = 0.0;
#pragma unroll
                for (int a = 0; a < NL; ++a)
#pragma unroll
                    for (int b = 0; b < NL; ++b)
                        s = fma(Gk[a][b] * (a == b ? 2.0 : 1.0), ws + (wl[a] + wl[b]), s);
                const double sk = kk * s;
#pragma unroll
                for (int x = 0; x < D; ++x) gq[x] += sk * gc[x];
                gw += kk * ((gsum + gtr) + (rowc + colc) + 2.0 * gcc);
            }
        }
    }
#pragma unroll
    for (int sh = 1; sh < kVjpLanes; sh <<= 1) {
        gw += __shfl_xor(gw, sh, kVjpLanes);
#pragma unroll
        for (int x = 0; x < D; ++x) gq[x] += __shfl_xor(gq[x], sh, kVjpLanes);
    }
    if (i < mv.nq && j == 0) {
        if (dLdw) dLdw[i] = gw;
        if (dLdq)
#pragma unroll
            for (int x = 0; x < D; ++x) dLdq[x * mv.nq + i] = gq[x];
    }
    const unsigned long long any = __ballot(bad != 0);
    if (any != 0ull && (threadIdx.x & 63) == __ffsll((long long)any) - 1) atomicOr(status, bad);
}

// Workspace VJP, element pass: one thread per element (plan order e) writes
// the terms of its d+1 vertices to work[(e*(d+1) + a)*NW + ...], NW = d
// (+1 for the weighted mass); zeros for a degenerate element.
template <int D, int OP, int PB>
__global__ void __launch_bounds__(kVjpElemWG)
    k_vjp_elem(MeshView mv, int64_t nme, const int32_t *__restrict__ porig, GAddr ga,
               const double *__restrict__ G, double *__restrict__ work, int32_t *status) {
    constexpr int NL = D + 1;
    constexpr int NW = D + (OP == FEM_OP_MASS_W ? 1 : 0);
    constexpr int NT = NL * NW;   // doubles per element
    // the workgroup's terms are staged in LDS and written out as one
    // contiguous run (a thread's own NT doubles would leave as NT stores
    // whose lanes lie NT * 8 bytes apart)
    __shared__ double stage[kVjpElemWG * NT];
    const int64_t e0 = int64_t(blockIdx.x) * kVjpElemWG;
    const int64_t e = e0 + threadIdx.x;
    int bad = 0;
    if (e < nme) {
        double P[NL][D], Gk[NL][NL], wl[NL];
        vjp_load<D, OP, PB>(mv, porig, ga, G, e, P, Gk, wl);
        VjpGeom<D> V;
        double *out = stage + threadIdx.x * NT;
        if (!vjp_geometry<D>(P, V)) {
            bad = 1;
#pragma unroll
            for (int u = 0; u < NT; ++u) out[u] = 0.0;
        } else {
#pragma unroll
            for (int al = 0; al < NL; ++al) {
                double tq[D], tw;
                vjp_term<D, OP>(V, Gk, wl, al, tq, tw);
#pragma unroll
                for (int x = 0; x < D; ++x) out[al * NW + x] = tq[x];
                if constexpr (OP == FEM_OP_MASS_W) out[al * NW + D] = tw;
            }
        }
    }
    __syncthreads();
    const int64_t n = (nme - e0 < kVjpElemWG ? nme - e0 : kVjpElemWG) * NT;
    double *dst = work + e0 * NT;
    for (int64_t u = threadIdx.x; u < n; u += kVjpElemWG) dst[u] = stage[u];
    const unsigned long long any = __ballot(bad != 0);
    if (any != 0ull && (threadIdx.x & 63) == __ffsll((long long)any) - 1) atomicOr(status, bad);
}

// Workspace VJP, vertex pass: the terms of each vertex's incidences summed in
// the order of k_vjp (same lanes, same tree), so the outputs are identical.
template <int D, int OP>
__global__ void __launch_bounds__(256)
    k_vjp_gather(MeshView mv, const double *__restrict__ work, double *__restrict__ dLdq,
                 double *__restrict__ dLdw) {
    constexpr int NL = D + 1;
    constexpr int NW = D + (OP == FEM_OP_MASS_W ? 1 : 0);
    const int64_t gt = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t i = gt / kVjpLanes;
    const int j = int(gt % kVjpLanes);
    double gw = 0.0, gq[D];
#pragma unroll
    for (int x = 0; x < D; ++x) gq[x] = 0.0;
    if (i < mv.nq) {
        const int t1 = mv.inc_ptr[i + 1];
        // kGatherDepth of the lane's incidences per step: their words, then
        // their records, are loaded together (past the lane's last incidence
        // the loads repeat the step's first and the adds are skipped), and
        // the terms are added in incidence order
        for (int t = mv.inc_ptr[i] + j; t < t1; t += kGatherDepth * kVjpLanes) {
            const double *in[kGatherDepth];
#pragma unroll
            for (int u = 0; u < kGatherDepth; ++u) {
                const int tu = t + u * kVjpLanes;
                const uint32_t ea = mv.inc_elem[tu < t1 ? tu : t];
                in[u] = work + (int64_t(ea & 0x3fffffffu) * NL + int(ea >> 30)) * NW;
            }
            double r[kGatherDepth][NW];
#pragma unroll
            for (int u = 0; u < kGatherDepth; ++u)
#pragma unroll
                for (int x = 0; x < NW; ++x) r[u][x] = in[u][x];
#pragma unroll
            for (int u = 0; u < kGatherDepth; ++u)
                if (t + u * kVjpLanes < t1) {
#pragma unroll
                    for (int x = 0; x < D; ++x) gq[x] += r[u][x];
                    if constexpr (OP == FEM_OP_MASS_W) gw += r[u][D];
                }
        }
    }
    vjp_store<D>(mv, i, j, gq, gw, dLdq, dLdw);
}

MeshView deriv_view(const fem_plan_s *p, const double *q, const double *w, double *values) {
    MeshView mv{};
    mv.rp = p->rp;
    mv.inc_ptr = p->inc_ptr;
    mv.inc_elem = p->inc_elem;
    mv.inc_off = p->inc_off;
    mv.pme = p->pme;
    mv.q = q;
    mv.w = w;
    mv.values = values;
    mv.nq = p->nq;
    return mv;
}

template <int D>
hipError_t launch_jvp(const fem_plan_s *p, int op, const MeshView &mv, const double *dq,
                      const double *dw, hipStream_t s) {
    const RowLaunch &L = p->launch[1];
    if (L.tiles == 0) return hipSuccess;
    const dim3 grid(unsigned(L.tiles)), block(L.rows_per_wg);
    if (op == FEM_OP_MASS)
        hipLaunchKernelGGL((k_jvp<D, FEM_OP_MASS>), grid, block, L.lds_bytes, s, mv, dq, dw, p->status);
    else if (op == FEM_OP_MASS_W)
        hipLaunchKernelGGL((k_jvp<D, FEM_OP_MASS_W>), grid, block, L.lds_bytes, s, mv, dq, dw,
                           p->status);
    else
        hipLaunchKernelGGL((k_jvp<D, FEM_OP_STIFF>), grid, block, L.lds_bytes, s, mv, dq, dw,
                           p->status);
    return hipGetLastError();
}

// PB of a gradient addresser: the slot map, or the plan's positions
int addr_kind(const fem_plan_s *p, const GAddr &ga) {
    return ga.slot ? 0 : (p->vpos_bytes.load(std::memory_order_acquire) == 1 ? 1 : 2);
}

template <int D, int OP, int PB>
void launch_vjp_t(const fem_plan_s *p, const MeshView &mv, const GAddr &ga, const double *G,
                  double *dLdq, double *dLdw, hipStream_t s) {
    const unsigned grid = unsigned((p->nq * kVjpLanes + 255) / 256);
    hipLaunchKernelGGL((k_vjp<D, OP, PB>), dim3(grid), dim3(256), 0, s, mv, p->porig, ga, G,
                       dLdq, dLdw, p->status);
}

template <int D, int OP>
void launch_vjp_pb(const fem_plan_s *p, const MeshView &mv, const GAddr &ga, const double *G,
                   double *dLdq, double *dLdw, hipStream_t s) {
    switch (addr_kind(p, ga)) {
    case 0: launch_vjp_t<D, OP, 0>(p, mv, ga, G, dLdq, dLdw, s); break;
    case 1: launch_vjp_t<D, OP, 1>(p, mv, ga, G, dLdq, dLdw, s); break;
    default: launch_vjp_t<D, OP, 2>(p, mv, ga, G, dLdq, dLdw, s); break;
    }
}

template <int D>
hipError_t launch_vjp(const fem_plan_s *p, int op, const MeshView &mv, const GAddr &ga,
                      const double *G, double *dLdq, double *dLdw, hipStream_t s) {
    if (op == FEM_OP_MASS)
        launch_vjp_pb<D, FEM_OP_MASS>(p, mv, ga, G, dLdq, dLdw, s);
    else if (op == FEM_OP_MASS_W)
        launch_vjp_pb<D, FEM_OP_MASS_W>(p, mv, ga, G, dLdq, dLdw, s);
    else
        launch_vjp_pb<D, FEM_OP_STIFF>(p, mv, ga, G, dLdq, dLdw, s);
    return hipGetLastError();
}

template <int D, int OP, int PB>
void launch_vjp_elem_t(const fem_plan_s *p, const MeshView &mv, const GAddr &ga,
                       const double *G, double *work, hipStream_t s) {
    const unsigned ge = unsigned((p->nme + kVjpElemWG - 1) / kVjpElemWG);
    hipLaunchKernelGGL((k_vjp_elem<D, OP, PB>), dim3(ge), dim3(kVjpElemWG), 0, s, mv, p->nme, p->porig,
                       ga, G, work, p->status);
}

template <int D, int OP>
hipError_t launch_vjp_ws_t(const fem_plan_s *p, const MeshView &mv, const GAddr &ga,
                           const double *G, double *work, double *dLdq, double *dLdw,
                           hipStream_t s) {
    if (p->nme > 0) {
        switch (addr_kind(p, ga)) {
        case 0: launch_vjp_elem_t<D, OP, 0>(p, mv, ga, G, work, s); break;
        case 1: launch_vjp_elem_t<D, OP, 1>(p, mv, ga, G, work, s); break;
        default: launch_vjp_elem_t<D, OP, 2>(p, mv, ga, G, work, s); break;
        }
    }
    const unsigned gv = unsigned((p->nq * kVjpLanes + 255) / 256);
    hipLaunchKernelGGL((k_vjp_gather<D, OP>), dim3(gv), dim3(256), 0, s, mv, work, dLdq, dLdw);
    return hipGetLastError();
}

template <int D>
hipError_t launch_vjp_ws(const fem_plan_s *p, int op, const MeshView &mv, const GAddr &ga,
                         const double *G, double *work, double *dLdq, double *dLdw,
                         hipStream_t s) {
    if (op == FEM_OP_MASS)
        return launch_vjp_ws_t<D, FEM_OP_MASS>(p, mv, ga, G, work, dLdq, dLdw, s);
    if (op == FEM_OP_MASS_W)
        return launch_vjp_ws_t<D, FEM_OP_MASS_W>(p, mv, ga, G, work, dLdq, dLdw, s);
    return launch_vjp_ws_t<D, FEM_OP_STIFF>(p, mv, ga, G, work, dLdq, dLdw, s);
}

// The plan's per-element column positions, from the incidence records: the
// incidence (vertex of local index a, element e) holds the positions of the
// element's vertices b within that vertex's row.
template <class T>
__global__ void k_vjp_positions(const uint32_t *__restrict__ inc_elem,
                                const uint64_t *__restrict__ inc_off, int64_t ninc, int NL,
                                T *__restrict__ vpos) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= ninc) return;
    const uint32_t ea = inc_elem[t];
    const int64_t e = ea & 0x3fffffffu;
    const int a = int(ea >> 30);
    const uint64_t off = inc_off[t];
    for (int b = 0; b < NL; ++b) vpos[e * NL * NL + b * NL + a] = T((off >> (16 * b)) & 0xffffu);
}

// The gradient addresser of a VJP call: the caller's map, or (slot null) the
// plan's positions, which fem_plan_vjp_positions must have built.
bool vjp_addr(const fem_plan_s *p, const int32_t *slot, GAddr *ga) {
    ga->slot = slot;
    ga->vpos = nullptr;
    if (slot) return true;
    if (p->vpos_bytes.load(std::memory_order_acquire) == 0) return false;
    ga->vpos = p->vpos;
    return true;
}

bool deriv_op(int32_t op) { return op == FEM_OP_MASS || op == FEM_OP_MASS_W || op == FEM_OP_STIFF; }

// Element-term buffer of fem_assemble_vjp_noalloc: a fixed device array, one
// copy per GPU the library runs on (each GPU holds it until the process
// ends).  128 MiB: 3D meshes of up to 1,048,576 elements for the weighted
// mass (128 B of terms per element), 1,398,101 for the mass and stiffness.
constexpr int64_t kVjpScratchBytes = int64_t(128) << 20;
__device__ __align__(256) double scratch[kVjpScratchBytes / sizeof(double)];

// Device address of `scratch` on each device, looked up once per device with
// that device current (host code never passes the array's own name: on the
// host it is a stand-in, not a device address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_address(int dev, double **out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// bytes of the element-term work array of the workspace VJP
int64_t vjp_work_bytes(const fem_plan_s *p, int32_t op) {
    const int64_t nw = p->d + (op == FEM_OP_MASS_W ? 1 : 0);
    return int64_t(sizeof(double)) * (p->d + 1) * nw * p->nme;
}

}  // namespace
}  // namespace femasm

using namespace femasm;

static fem_status fem_assemble_jvp_impl(fem_plan plan, int32_t op, const double *q, const double *w,
                                       const double *dq, const double *dw, double *dvalues,
                                       hipStream_t stream) {
    PhaseRange range("femasm: JVP");
    if (!plan || !deriv_op(op)) return FEM_ERR_ARG;
    if (plan->nnz == 0) return FEM_OK;
    if (!q || !dq || !dvalues || (op == FEM_OP_MASS_W && (!w || !dw))) return FEM_ERR_ARG;
    // the vertex-pair kernel (FEMASM_KERNEL=rowgather forces the row-gather one)
    const char *sel = getenv("FEMASM_KERNEL");
    if (!sel || strcmp(sel, "rowgather") != 0) {
        // the two JVP routes round differently: always the pair kernel when
        // the mesh has its layout
        wait_layouts(plan);
        const int jop = op == FEM_OP_MASS ? kOpJvpMass : op == FEM_OP_MASS_W ? kOpJvpMassW
                                                                            : kOpJvpStiff;
        hipError_t e = hipSuccess;
        if (launch_pair(plan, jop, q, w, 0.0, 0.0, dvalues, stream, &e, dw, nullptr, dq))
            return hip_status(e);
    }
    if (plan->launch[1].rows_per_wg == 0) return FEM_ERR_OVERFLOW;
    const MeshView mv = deriv_view(plan, q, w, dvalues);
    const hipError_t e = plan->d == 2 ? launch_jvp<2>(plan, op, mv, dq, dw, stream)
                                      : launch_jvp<3>(plan, op, mv, dq, dw, stream);
    return hip_status(e);
}

extern "C" fem_status fem_assemble_jvp(fem_plan plan, int32_t op, const double *q, const double *w,
                                       const double *dq, const double *dw, double *dvalues,
                                       hipStream_t stream) {
    return debug_check(fem_assemble_jvp_impl(plan, op, q, w, dq, dw, dvalues, stream),
                       stream, plan ? plan->status : nullptr);
}

static fem_status fem_assemble_vjp_impl(fem_plan plan, int32_t op, const double *q, const double *w,
                                       const double *G, const int32_t *slot, double *dLdq,
                                       double *dLdw, hipStream_t stream) {
    PhaseRange range("femasm: VJP");
    if (!plan || !deriv_op(op)) return FEM_ERR_ARG;
    if (plan->nq == 0) return FEM_OK;
    GAddr ga{slot, nullptr};
    if (!q || (plan->nnz > 0 && (!G || !vjp_addr(plan, slot, &ga))) || (op == FEM_OP_MASS_W && !w))
        return FEM_ERR_ARG;
    if (op != FEM_OP_MASS_W) dLdw = nullptr;
    const MeshView mv = deriv_view(plan, q, w, nullptr);
    const hipError_t e = plan->d == 2 ? launch_vjp<2>(plan, op, mv, ga, G, dLdq, dLdw, stream)
                                      : launch_vjp<3>(plan, op, mv, ga, G, dLdq, dLdw, stream);
    return hip_status(e);
}

extern "C" fem_status fem_assemble_vjp(fem_plan plan, int32_t op, const double *q, const double *w,
                                       const double *G, const int32_t *slot, double *dLdq,
                                       double *dLdw, hipStream_t stream) {
    return debug_check(fem_assemble_vjp_impl(plan, op, q, w, G, slot, dLdq, dLdw, stream),
                       stream, plan ? plan->status : nullptr);
}

extern "C" fem_status fem_plan_vjp_positions(fem_plan plan, hipStream_t stream) {
    if (!plan) return FEM_ERR_ARG;
    if (plan->vpos_bytes.load(std::memory_order_acquire) != 0) return FEM_OK;
    std::lock_guard<std::mutex> lock(plan->vpos_mu);
    if (plan->vpos_bytes.load(std::memory_order_acquire) != 0) return FEM_OK;
    const int NL = plan->d + 1;
    const int bytes = plan->max_row <= 256 ? 1 : 2;
    const int64_t n = int64_t(NL) * NL * plan->nme, ninc = int64_t(NL) * plan->nme;
    void *buf = nullptr;
    if (n > 0) {
        hipError_t e = hipMalloc(&buf, size_t(n) * bytes);
        if (e != hipSuccess) return hip_status(e);
        const unsigned grid = unsigned((ninc + 255) / 256);
        if (bytes == 1)
            hipLaunchKernelGGL(k_vjp_positions<uint8_t>, dim3(grid), dim3(256), 0, stream,
                               plan->inc_elem, plan->inc_off, ninc, NL,
                               static_cast<uint8_t *>(buf));
        else
            hipLaunchKernelGGL(k_vjp_positions<uint16_t>, dim3(grid), dim3(256), 0, stream,
                               plan->inc_elem, plan->inc_off, ninc, NL,
                               static_cast<uint16_t *>(buf));
        e = hipGetLastError();
        // complete before any stream may read it
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) {
            (void)hipFree(buf);
            return hip_status(e);
        }
    }
    plan->vpos = buf;
    plan->vpos_bytes.store(bytes, std::memory_order_release);
    return FEM_OK;
}

extern "C" fem_status fem_vjp_work_bytes(fem_plan plan, int32_t op, int64_t *bytes) {
    if (!plan || !deriv_op(op) || !bytes) return FEM_ERR_ARG;
    *bytes = vjp_work_bytes(plan, op);
    return FEM_OK;
}

extern "C" fem_status fem_assemble_vjp_ws(fem_plan plan, int32_t op, const double *q,
                                          const double *w, const double *G, const int32_t *slot,
                                          double *work, int64_t work_bytes, double *dLdq,
                                          double *dLdw, hipStream_t stream) {
    if (!plan || !deriv_op(op)) return FEM_ERR_ARG;
    if (plan->nq == 0) return FEM_OK;
    GAddr ga{slot, nullptr};
    if (!q || (plan->nnz > 0 && (!G || !vjp_addr(plan, slot, &ga))) || (op == FEM_OP_MASS_W && !w))
        return FEM_ERR_ARG;
    if (plan->nme > 0 && (!work || work_bytes < vjp_work_bytes(plan, op) ||
                          (reinterpret_cast<uintptr_t>(work) & 7u) != 0))
        return FEM_ERR_ARG;
    if (op != FEM_OP_MASS_W) dLdw = nullptr;
    const MeshView mv = deriv_view(plan, q, w, nullptr);
    const hipError_t e =
        plan->d == 2 ? launch_vjp_ws<2>(plan, op, mv, ga, G, work, dLdq, dLdw, stream)
                     : launch_vjp_ws<3>(plan, op, mv, ga, G, work, dLdq, dLdw, stream);
    return hip_status(e);
}

extern "C" fem_status fem_assemble_vjp_noalloc(fem_plan plan, int32_t op, const double *q,
                                               const double *w, const double *G,
                                               const int32_t *slot, double *dLdq, double *dLdw,
                                               hipStream_t stream) {
    if (!plan || !deriv_op(op)) return FEM_ERR_ARG;
    if (plan->nq == 0) return FEM_OK;
    GAddr ga{slot, nullptr};
    if (!q || (plan->nnz > 0 && (!G || !vjp_addr(plan, slot, &ga))) || (op == FEM_OP_MASS_W && !w))
        return FEM_ERR_ARG;
    if (vjp_work_bytes(plan, op) > kVjpScratchBytes) return FEM_ERR_OVERFLOW;
    double *work = nullptr;
    if (plan->nme > 0) {
        const hipError_t e = scratch_address(plan->device, &work);
        if (e != hipSuccess) return hip_status(e);
    }
    if (op != FEM_OP_MASS_W) dLdw = nullptr;
    const MeshView mv = deriv_view(plan, q, w, nullptr);
    const hipError_t e =
        plan->d == 2 ? launch_vjp_ws<2>(plan, op, mv, ga, G, work, dLdq, dLdw, stream)
                     : launch_vjp_ws<3>(plan, op, mv, ga, G, work, dLdq, dLdw, stream);
    return hip_status(e);
}
