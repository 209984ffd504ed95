// Pair kernel: every entry of the scalar CSR pattern (a "vertex pair" (i, j))
// is summed by one thread, in registers, over the elements that contain both
// vertices (the duplicate sum of the `sparse` step, Section 3).
//
// Work is organised in vertex blocks (blocks_host.h): the block's rows, every
// element around them, and per pair the list of those elements in ascending
// caller element number.  For one block a workgroup
//   1. computes each block element's values once (closed forms of Sections
//      4.1, 4.2 and 5.1, element.h) into LDS, plus an all-zero dummy element
//      that pads the pair lists;
//   2. lets every lane walk its pairs' lists and accumulate; all lanes of a
//      64-pair task run the same number of entries (no divergence);
//   3. places the finished values into an LDS image of the block's CSR value
//      range and writes it out with coalesced stores.
// Each pair's sum is taken in ascending element number with the same
// expressions as the row-gather kernel, so both give identical bits.
//
// The kernel is persistent: a fixed grid sized to the occupancy walks the
// blocks (each XCD a contiguous range, for L2 locality).  While one block is
// summed, the next block's lists and coordinates are already in flight into
// registers, and the vertex ids of the block after it as well, so the HBM
// latency of the dependent loads (block descriptor -> vertex ids ->
// coordinates) is hidden behind the previous block's work.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "blocks_host.h"
#include "element.h"
#include "femasm_impl.h"

#pragma clang fp contract(off)

namespace femasm {

namespace {

constexpr int kPairWG = kPairWaves * 64;
constexpr int kEntSlots = 8192 / 8 / kPairWG;   // uint4 entry slots per thread: <= 8192 entries
constexpr int kNodeSlots = 512 / kPairWG;       // touched vertices per thread
constexpr int kMaxPairNodes = 256;              // touched vertices per block: 8-bit local ids
// s_waitcnt operand: vmcnt(0), expcnt and lgkmcnt left at their maxima
constexpr int kWaitVmem = 0x0F70;
constexpr int kElemSlots = 1024 / kPairWG;      // elements per thread: <= 1023 (+ dummy)
static_assert(kEntSlots == 2 && kNodeSlots == 1 && kElemSlots == 2, "512-thread workgroups");
static_assert(kPairWaves * 4 < (1 << kWaveStartBits) && kPairWaves * kWaveStartBits <= 64,
              "task starts of up to 4 tasks per wavefront fit the descriptor");

struct PairView {
    const int32_t *desc;
    const int4 *rowinfo;
    const int32_t *nodes;
    const uint32_t *elem;
    const int32_t *task_cnt;
    const int32_t *task_eoff;
    const uint32_t *hdr;
    const uint16_t *ent;
    const double *q;
    const double *w;
    const double *w2;     // mu field (nodal Lame elasticity; w is the lambda field)
    double gco[kGeneralCoef];   // general operator: A (d x d, row-major), b, c, a0
    const double *dq;     // JVP operators: tangent coordinates (layout of q); w2 is then dw
    double *values;
    int32_t nb, max_nodes;
    uint32_t off_w, off_row, off_rowof, off_ev, off_ent;
};

// Per-element values kept in LDS (mostly an odd slot size: consecutive
// elements fall on different banks).  ELAS: scaled cofactors ch_a (and, with nodal Lame
// fields, the element means lambda_K, mu_K after them); the scalar
// operators: the packed upper triangle of the element matrix, entry (a, b),
// a <= b, at a*(d+1) - a*(a-1)/2 + (b-a) (the pair entries carry that index).
constexpr bool is_elas(int op) { return op == FEM_OP_ELAS || op == kOpElasNodal; }
constexpr bool is_jvp(int op) { return op == kOpJvpMass || op == kOpJvpMassW || op == kOpJvpStiff; }

template <int D, int OP>
struct PairOp {
    static constexpr int NL = D + 1;
    static constexpr int NV0 = OP == FEM_OP_ELAS      ? NL * D
                               : OP == kOpElasNodal ? NL * D + 2
                               : OP == kOpGeneral   ? NL * NL
                                                    : NL * (NL + 1) / 2;
    // 3D scalar operators: ten values, unpadded (their blocks are the largest
    // the LDS holds); the others an odd slot size
    static constexpr int NV = (D == 3 && NV0 == 10) ? NV0 : (NV0 | 1);
    static constexpr int M = is_elas(OP) ? D : 1;
    // register sums per pair (the general operator also sums its mirror's
    // transposed entries)
    static constexpr int NX = OP == kOpElasNodal ? 2 * M * M : OP == kOpGeneral ? 2 : M * M;
};

template <int NL>
__device__ __forceinline__ constexpr int tri_index(int a, int b) {
    return a * NL - a * (a - 1) / 2 + (b - a);
}

// Block descriptor, kDescInts ints per block: [0] first row, [1] rows,
// [2] first touched vertex, [3] touched vertices, [4] first element,
// [5] elements, [6] CSR entries of the rows, [7] first task, [8] entry
// count / 8, [9],[12] task starts of wavefronts 1..8 relative to the first
// task (6 bits each, low word first), [10..11] first entry, and the block's
// mesh within the coordinate, weight and value arrays (several meshes share
// one launch in the batched assembly): [14..15] coordinate offset, [16..17]
// weight offset, [18..19] value offset, [20..21] its vertex count n_q; 64-bit
// fields low word first.
constexpr int kDescInts = 24;
struct Desc {
    int r0, nr, n0, nn, e0, ne, nacc, t0, nent8;
    uint64_t wp;
    int64_t eb, qo, wo, vo, nq;
};

__device__ __forceinline__ int64_t lane64(int dv, int lo) {
    return int64_t(uint32_t(__builtin_amdgcn_readlane(dv, lo))) |
           (int64_t(__builtin_amdgcn_readlane(dv, lo + 1)) << 32);
}

// Descriptors travel as vector loads, lane k holding int k, and are read out
// with readlane an iteration later: a scalar load shares its wait counter
// with LDS operations and would stall the next LDS access on HBM latency.
__device__ __forceinline__ int load_desc_vec(const PairView &pv, int b, int lane) {
    return b >= 0 && lane < kDescInts ? pv.desc[int64_t(b) * kDescInts + lane] : 0;
}

__device__ __forceinline__ Desc desc_from(int dv) {
    Desc d;
    d.r0 = __builtin_amdgcn_readlane(dv, 0);
    d.nr = __builtin_amdgcn_readlane(dv, 1);
    d.n0 = __builtin_amdgcn_readlane(dv, 2);
    d.nn = __builtin_amdgcn_readlane(dv, 3);
    d.e0 = __builtin_amdgcn_readlane(dv, 4);
    d.ne = __builtin_amdgcn_readlane(dv, 5);
    d.nacc = __builtin_amdgcn_readlane(dv, 6);
    d.t0 = __builtin_amdgcn_readlane(dv, 7);
    d.nent8 = __builtin_amdgcn_readlane(dv, 8);
    d.wp = uint64_t(uint32_t(__builtin_amdgcn_readlane(dv, 9))) |
           (uint64_t(uint32_t(__builtin_amdgcn_readlane(dv, 12))) << 32);
    d.eb = lane64(dv, 10);
    d.qo = lane64(dv, 14);
    d.wo = lane64(dv, 16);
    d.vo = lane64(dv, 18);
    d.nq = lane64(dv, 20);
    return d;
}

// First task of wavefront w (0..kPairWaves) of a block, relative to its t0.
__device__ __forceinline__ int wave_task(uint64_t wp, int w) {
    return w == 0 ? 0 : int((wp >> (kWaveStartBits * (w - 1))) & ((1u << kWaveStartBits) - 1u));
}

template <int D, int OP>
__device__ __forceinline__ void element_values(const double (&P)[D + 1][D], const double *wl,
                                               const double *wl2, const double *gco,
                                               const double (&dP)[D + 1][D], double *out,
                                               int &bad) {
    constexpr int NL = D + 1;
    if constexpr (is_jvp(OP)) {
        // directional derivative of the packed element matrix along dP (and
        // dw = wl2): with g = c/det, N = sum_c g_c dP_c^T and t = tr N,
        //   stiffness  vol [ t g_a.g_b - (N g_a).g_b - g_a.(N g_b) ]
        //   mass       E_ab t;   weighted  E_ab t + f (dw^s + dw_a + dw_b)
        Elem<D> E;
        elem_geometry(P, E);
        const bool deg = E.det == 0.0;
        if (deg) bad = 1;
        const double rdet = deg ? 0.0 : 1.0 / E.det;
        const double ad = fabs(E.det);
        double g[NL][D];
#pragma unroll
        for (int b = 0; b < NL; ++b)
#pragma unroll
            for (int x = 0; x < D; ++x) g[b][x] = E.c[b][x] * rdet;
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
        double t = N[0][0];
#pragma unroll
        for (int x = 1; x < D; ++x) t += N[x][x];
        if constexpr (OP == kOpJvpStiff) {
            const double vol = ad / Fact<D>::dfact;
            double Ng[NL][D];
#pragma unroll
            for (int b = 0; b < NL; ++b)
#pragma unroll
                for (int x = 0; x < D; ++x) Ng[b][x] = cdot<D>(N[x], g[b]);
#pragma unroll
            for (int a = 0; a < NL; ++a)
#pragma unroll
                for (int b = a; b < NL; ++b)
                    out[tri_index<NL>(a, b)] =
                        vol * ((t * cdot<D>(g[a], g[b]) - cdot<D>(Ng[a], g[b])) - cdot<D>(g[a], Ng[b]));
        } else if constexpr (OP == kOpJvpMass) {
            const double k = deg ? 0.0 : ad / Fact<D>::mass_den;
#pragma unroll
            for (int a = 0; a < NL; ++a)
#pragma unroll
                for (int b = a; b < NL; ++b) out[tri_index<NL>(a, b)] = (a == b ? 2.0 * k : k) * t;
        } else {
            double ws = wl[0], dws = wl2[0];
#pragma unroll
            for (int b = 1; b < NL; ++b) {
                ws += wl[b];
                dws += wl2[b];
            }
            const double k = deg ? 0.0 : ad / Fact<D>::massw_den;
#pragma unroll
            for (int a = 0; a < NL; ++a)
#pragma unroll
                for (int b = a; b < NL; ++b) {
                    const double f = a == b ? 2.0 * k : k;
                    out[tri_index<NL>(a, b)] = f * ((ws + (wl[a] + wl[b])) * t + (dws + (wl2[a] + wl2[b])));
                }
        }
    } else if constexpr (OP == FEM_OP_MASS || OP == FEM_OP_MASS_W) {
        // the same operations as the row-gather kernel: (1+delta) k, and
        // f (w^s + (w_a + w_b)) with f = (1+delta) k
        const double det = elem_det(P);
        const bool deg = det == 0.0;
        if (deg) bad = 1;
        const double ad = fabs(det);
        // a degenerate element gets k = 0, so every value is a signed zero
        // (adding it leaves a sum unchanged, as skipping the element does)
        if constexpr (OP == FEM_OP_MASS) {
            const double k = deg ? 0.0 : ad / Fact<D>::mass_den;
#pragma unroll
            for (int a = 0; a < NL; ++a)
#pragma unroll
                for (int b = a; b < NL; ++b) out[tri_index<NL>(a, b)] = a == b ? 2.0 * k : k;
        } else {
            double ws = wl[0];
#pragma unroll
            for (int b = 1; b < NL; ++b) ws += wl[b];
            const double k = deg ? 0.0 : ad / Fact<D>::massw_den;
#pragma unroll
            for (int a = 0; a < NL; ++a)
#pragma unroll
                for (int b = a; b < NL; ++b) {
                    const double f = a == b ? 2.0 * k : k;
                    out[tri_index<NL>(a, b)] = f * (ws + (wl[a] + wl[b]));
                }
        }
    } else {
        Elem<D> E;
        elem_geometry(P, E);
        const bool deg = E.det == 0.0;
        if (deg) bad = 1;
        if constexpr (OP == FEM_OP_STIFF) {
            // degenerate: inv = 0, so every value is a signed zero
            const double inv = deg ? 0.0 : 1.0 / (Fact<D>::dfact * fabs(E.det));
#pragma unroll
            for (int a = 0; a < NL; ++a)
#pragma unroll
                for (int b = a; b < NL; ++b) out[tri_index<NL>(a, b)] = cdot<D>(E.c[a], E.c[b]) * inv;
        } else if constexpr (OP == kOpGeneral) {
            // full element matrix, row a (test), column b (trial), with
            // g = c/det and |K| = |det|/d!:
            //   |K| g_a^T A g_b        = c_a^T A c_b / (d! |det|)
            //   |K|/(d+1) b.g_a        = sign(det) b.c_a / (d+1)!
            //   |K|/(d+1) c.g_b        = sign(det) c.c_b / (d+1)!
            //   a0 |K| d!(1+delta)/(d+2)! = a0 |det| (1+delta) / (d+2)!
            const double *A = gco;
            double bv[D], cv[D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                bv[i] = gco[D * D + i];
                cv[i] = gco[D * D + D + i];
            }
            const double a0 = gco[D * D + 2 * D];
            const double ad = fabs(E.det);
            const double inv = deg ? 0.0 : 1.0 / (Fact<D>::dfact * ad);
            const double f1 = deg ? 0.0 : (E.det > 0.0 ? 1.0 : -1.0) / Fact<D>::d1fact;
            const double fm = deg ? 0.0 : a0 * ad / Fact<D>::mass_den;
            double Ac[NL][D], tb[NL], tc[NL];
#pragma unroll
            for (int b = 0; b < NL; ++b) {
#pragma unroll
                for (int i = 0; i < D; ++i) {
                    double s = A[i * D] * E.c[b][0];
#pragma unroll
                    for (int j = 1; j < D; ++j) s = fma(A[i * D + j], E.c[b][j], s);
                    Ac[b][i] = s;
                }
                tb[b] = cdot<D>(bv, E.c[b]) * f1;
                tc[b] = cdot<D>(cv, E.c[b]) * f1;
            }
#pragma unroll
            for (int a = 0; a < NL; ++a)
#pragma unroll
                for (int b = 0; b < NL; ++b)
                    out[a * NL + b] = ((cdot<D>(E.c[a], Ac[b]) * inv - tb[a]) + tc[b]) +
                                      (a == b ? 2.0 * fm : fm);
        } else {
            const double sc = deg ? 0.0 : elas_scale<D>(E.det);
#pragma unroll
            for (int a = 0; a < NL; ++a)
#pragma unroll
                for (int x = 0; x < D; ++x) out[a * D + x] = E.c[a][x] * sc;
            if constexpr (OP == kOpElasNodal) {
                // means of the P1 Lame fields over K: int_K lambda_h = |K| lambda^s/(d+1)
                double ls = wl[0], ms = wl2[0];
#pragma unroll
                for (int a = 1; a < NL; ++a) {
                    ls += wl[a];
                    ms += wl2[a];
                }
                out[NL * D] = ls / double(NL);
                out[NL * D + 1] = ms / double(NL);
            }
        }
    }
}

// The persistent loop of one workgroup: workgroup wg of nwg (a multiple of 8)
// walks its XCD's share of the layout's blocks.
template <int D, int OP, int S>
__device__ __forceinline__ void pair_run(const PairView &pv, double lam, double mu,
                                         int32_t *status, const int wg, const int nwg) {
    using O = PairOp<D, OP>;
    constexpr int NL = D + 1;
    constexpr int NV = O::NV;
    constexpr int M = O::M;
    constexpr int M2 = M * M;
    constexpr int NX = O::NX;
    constexpr bool kW = OP == FEM_OP_MASS_W || OP == kOpElasNodal || OP == kOpJvpMassW;
    constexpr bool kW2 = OP == kOpElasNodal || OP == kOpJvpMassW;
    constexpr bool kDQ = is_jvp(OP);
    constexpr bool kScalarSum = !(OP == FEM_OP_ELAS || OP == kOpElasNodal || OP == kOpGeneral);
    constexpr int kDqOff = (kW ? 1 : 0) + (kW2 ? 1 : 0);   // tangents after w and w2
    extern __shared__ __align__(16) unsigned char smem[];
    double *crd = reinterpret_cast<double *>(smem);
    double *wv = reinterpret_cast<double *>(smem + pv.off_w);
    int4 *rinf = reinterpret_cast<int4 *>(smem + pv.off_row);
    uint8_t *rowof = smem + pv.off_rowof;
    double *ev = reinterpret_cast<double *>(smem + pv.off_ev);
    uint16_t *ent = reinterpret_cast<uint16_t *>(smem + pv.off_ent);
    double *outb = ev;   // the output image reuses the element and entry buffers

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int MN = pv.max_nodes;
    // blocks of this workgroup: XCD x (workgroups x, x+8, ...) owns a
    // contiguous range of blocks, walked with stride J
    const int xcd = wg & 7, jj = wg >> 3, J = nwg >> 3;
    const int per = pv.nb >> 3, rem = pv.nb & 7;
    const int xs = xcd * per + (xcd < rem ? xcd : rem);
    const int xn = per + (xcd < rem ? 1 : 0);
    auto block_at = [&](int k) { return jj + k * J < xn ? xs + jj + k * J : -1; };

    // ---- prefetch registers
    // entry slots as named registers (an indexed array ends up in scratch)
    uint4 rent0 = make_uint4(0, 0, 0, 0), rent1 = rent0;
    uint32_t rel[kElemSlots];   // 4 x 8-bit local vertex ids per element
    int4 rrow = make_int4(0, 0, 0, 0);
    uint32_t rhd[S];   // pair | mirror << 16, split where it is used
    int rcntv = 0, reoffv = 0, rns = 0;   // task entry counts / offsets, lane s = slot s
    double rq[kNodeSlots][D];
    double rw[kNodeSlots], rw2[kNodeSlots];
    double rdq[kNodeSlots][D];
    int nid[kNodeSlots];

    auto load_nodes = [&](const Desc &d) {
#pragma unroll
        for (int u = 0; u < kNodeSlots; ++u) {
            const int n = u * kPairWG + tid;
            nid[u] = n < d.nn ? pv.nodes[d.n0 + n] : 0;
        }
    };
    auto issue_coords = [&](const Desc &d) {
#pragma unroll
        for (int u = 0; u < kNodeSlots; ++u) {
            if (u * kPairWG + tid < d.nn) {
#pragma unroll
                for (int x = 0; x < D; ++x) rq[u][x] = pv.q[d.qo + x * d.nq + nid[u]];
                if constexpr (kW) rw[u] = pv.w[d.wo + nid[u]];
                if constexpr (kW2) rw2[u] = pv.w2[d.wo + nid[u]];
                if constexpr (kDQ)
#pragma unroll
                    for (int x = 0; x < D; ++x) rdq[u][x] = pv.dq[d.qo + x * d.nq + nid[u]];
            }
        }
    };
    auto issue_raw = [&](const Desc &d) {
        const uint4 *src = reinterpret_cast<const uint4 *>(pv.ent + d.eb);
        const int tw0 = d.t0 + wave_task(d.wp, wave);
        rns = d.t0 + wave_task(d.wp, wave + 1) - tw0;
        rcntv = lane < rns ? pv.task_cnt[tw0 + lane] : 0;
        reoffv = lane < rns ? pv.task_eoff[tw0 + lane] : 0;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            rhd[s] = s < rns ? pv.hdr[int64_t(tw0 + s) * 64 + lane]
                             : kPairPad | (uint32_t(kPairPad) << 16);
        }
        if (tid < d.nent8) rent0 = src[tid];
        if (kPairWG + tid < d.nent8) rent1 = src[kPairWG + tid];
#pragma unroll
        for (int u = 0; u < kElemSlots; ++u) {
            const int e = u * kPairWG + tid;
            rel[u] = e < d.ne ? pv.elem[d.e0 + e] : 0u;
        }
        if (tid < d.nr) rrow = pv.rowinfo[d.r0 + tid];
    };

    // blocks k, k+1, k+2 of this workgroup: current, next, after next; the
    // descriptor registers run three blocks ahead
    int bc = block_at(0);
    if (bc < 0) return;
    int bn = block_at(1), bnn = block_at(2);
    Desc dc = desc_from(load_desc_vec(pv, bc, lane));
    load_nodes(dc);
    issue_coords(dc);
    issue_raw(dc);
    Desc dn = dc;
    if (bn >= 0) {
        dn = desc_from(load_desc_vec(pv, bn, lane));
        load_nodes(dn);
    }
    int dv_nn = load_desc_vec(pv, bnn, lane);

    Desc dp = dc;
    bool have_prev = false;
    int bad = 0;
    for (int k = 0;; ++k) {
        // Every load issued for this block landed during the previous block's
        // work: wait for all of them here, once.  Without this the compiler,
        // which cannot count loads issued under divergent conditions, waits
        // for everything outstanding further down, including the next
        // block's coordinate loads issued just before.
        __builtin_amdgcn_s_waitcnt(kWaitVmem);
        // L1: coordinates of the current block into LDS
#pragma unroll
        for (int u = 0; u < kNodeSlots; ++u) {
            const int n = u * kPairWG + tid;
            if (n < dc.nn) {
#pragma unroll
                for (int x = 0; x < D; ++x) crd[x * MN + n] = rq[u][x];
                if constexpr (kW) wv[n] = rw[u];
                if constexpr (kW2) wv[MN + n] = rw2[u];
                if constexpr (kDQ)
#pragma unroll
                    for (int x = 0; x < D; ++x) wv[kDqOff * MN + x * MN + n] = rdq[u][x];
            }
        }
        // L2: coordinates of the next block in flight
        if (bn >= 0) issue_coords(dn);
        // L3: output image of the previous block to HBM
        if (have_prev) {
            int kk = tid;
            if constexpr (M2 > 1) {
                // elasticity: M2 values per CSR entry, so each thread runs
                // many iterations; four at a time, their row lookups (two
                // dependent LDS reads each) in flight together
                for (; kk + 3 * kPairWG < M2 * dp.nacc; kk += 4 * kPairWG) {
                    int r[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) r[u] = rowof[(kk + u * kPairWG) / M2];
                    int4 ri[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) ri[u] = rinf[r[u]];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        pv.values[dp.vo + int64_t(M2) * ri[u].x + (kk + u * kPairWG - M2 * ri[u].z)] =
                            outb[kk + u * kPairWG];
                }
            }
            for (; kk < M2 * dp.nacc; kk += kPairWG) {
                const int4 ri = rinf[rowof[kk / M2]];
                pv.values[dp.vo + int64_t(M2) * ri.x + (kk - M2 * ri.z)] = outb[kk];
            }
        }
        __syncthreads();
        // L5: entry lists and rows of the current block into LDS
        {
            uint4 *e4 = reinterpret_cast<uint4 *>(ent);
            if (tid < dc.nent8) e4[tid] = rent0;
            if (kPairWG + tid < dc.nent8) e4[kPairWG + tid] = rent1;
        }
        if (tid < dc.nr) {
            rinf[tid] = rrow;
            for (int kk = 0; kk < rrow.y; ++kk) rowof[rrow.z + kk] = uint8_t(tid);
        }
        uint32_t hd[S], hd2[S];
        int cnt[S], eoff[S];
        const int ns = rns;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            hd[s] = rhd[s] & 0xffffu;
            hd2[s] = rhd[s] >> 16;
            cnt[s] = __builtin_amdgcn_readlane(rcntv, s);
            eoff[s] = __builtin_amdgcn_readlane(reoffv, s);
        }
        uint32_t el[kElemSlots];
#pragma unroll
        for (int u = 0; u < kElemSlots; ++u) el[u] = rel[u];
        // lists of the next block, vertex ids of the one after it and the
        // descriptor of the block after that: in flight during this block's
        // element and pair phases
        const int bnnn = block_at(k + 3);
        Desc dnn = dn;
        if (bn >= 0) issue_raw(dn);
        if (bnn >= 0) {
            dnn = desc_from(dv_nn);
            load_nodes(dnn);
        }
        const int dv_nnn = load_desc_vec(pv, bnnn, lane);
        __syncthreads();
        // L7: element phase.  The phases end at barriers, so each lasts as
        // long as its busiest wavefront: those with a second element pass
        // here, and in the pair sums wavefront 0 (the longest task of every
        // block, the one holding the diagonal pairs, goes to it).  They get
        // the higher issue priority for the phase against the other
        // workgroup's wavefronts on their SIMD.
        const bool two_passes = kPairWG + wave * 64 < dc.ne;
        if (two_passes) __builtin_amdgcn_s_setprio(2);
#pragma unroll
        for (int u = 0; u < kElemSlots; ++u) {
            const int e = u * kPairWG + tid;
            if (e < dc.ne) {
                const uint32_t vv = el[u];
                const int v[4] = {int(vv & 255u), int((vv >> 8) & 255u), int((vv >> 16) & 255u),
                                  int(vv >> 24)};
                double P[NL][D], dP[NL][D];
                double wl[NL], wl2[NL];
#pragma unroll
                for (int a = 0; a < NL; ++a) {
#pragma unroll
                    for (int x = 0; x < D; ++x) P[a][x] = crd[x * MN + v[a]];
                    if constexpr (kW) wl[a] = wv[v[a]];
                    if constexpr (kW2) wl2[a] = wv[MN + v[a]];
                    if constexpr (kDQ)
#pragma unroll
                        for (int x = 0; x < D; ++x) dP[a][x] = wv[kDqOff * MN + x * MN + v[a]];
                }
                element_values<D, OP>(P, wl, wl2, pv.gco, dP, ev + e * NV, bad);
            } else if (e == dc.ne) {
#pragma unroll
                for (int t = 0; t < NV; ++t) ev[e * NV + t] = 0.0;
            }
        }
        if (two_passes) __builtin_amdgcn_s_setprio(0);
        __syncthreads();
        // L10: pair sums
        if (wave == 0) __builtin_amdgcn_s_setprio(3);
        double X[S][NX];
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
            for (int t = 0; t < NX; ++t) X[s][t] = 0.0;
            if (s < ns && kScalarSum) {
                // four list entries per step: their values are read together
                // and added one after another in list (ascending element)
                // order, so a long list (a diagonal pair's) waits for one LDS
                // round trip per four entries instead of per entry
                const uint16_t *lst = ent + eoff[s] + lane;
                const int C = cnt[s], Cm = C - 1;
                auto val = [&](uint32_t x) { return ev[int(x & 1023u) * NV + int((x >> 10) & 15u)]; };
                uint32_t x0 = lst[0], x1 = lst[min(1, Cm) * 64], x2 = lst[min(2, Cm) * 64],
                         x3 = lst[min(3, Cm) * 64];
                double acc = 0.0;
                int t = 0;
                for (; t + 4 <= C; t += 4) {
                    const double v0 = val(x0), v1 = val(x1), v2 = val(x2), v3 = val(x3);
                    x0 = lst[min(t + 4, Cm) * 64];
                    x1 = lst[min(t + 5, Cm) * 64];
                    x2 = lst[min(t + 6, Cm) * 64];
                    x3 = lst[min(t + 7, Cm) * 64];
                    acc += v0;
                    acc += v1;
                    acc += v2;
                    acc += v3;
                }
                if (t < C) acc += val(x0);
                if (t + 1 < C) acc += val(x1);
                if (t + 2 < C) acc += val(x2);
                X[s][0] = acc;
            } else if (s < ns && OP == FEM_OP_ELAS) {
                // two list entries per step: both entries' rows of c-hat are
                // read together, then each accumulator takes the first entry's
                // product and the second's, in list order
                const uint16_t *lst = ent + eoff[s] + lane;
                const int C = cnt[s], Cm = C - 1;
                auto rows = [&](uint32_t x, double *A, double *B) {
                    const double *Ee = ev + int(x & 1023u) * NV;
                    const int a = int((x >> 10) & 3u), b = int((x >> 12) & 3u);
#pragma unroll
                    for (int c = 0; c < D; ++c) {
                        A[c] = Ee[a * D + c];
                        B[c] = Ee[b * D + c];
                    }
                };
                auto acc = [&](const double *A, const double *B) {
#pragma unroll
                    for (int l = 0; l < D; ++l)
#pragma unroll
                        for (int n = 0; n < D; ++n) X[s][l * D + n] = fma(A[l], B[n], X[s][l * D + n]);
                };
                uint32_t x0 = lst[0], x1 = lst[min(1, Cm) * 64];
                int t = 0;
                for (; t + 2 <= C; t += 2) {
                    double A0[D], B0[D], A1[D], B1[D];
                    rows(x0, A0, B0);
                    rows(x1, A1, B1);
                    x0 = lst[min(t + 2, Cm) * 64];
                    x1 = lst[min(t + 3, Cm) * 64];
                    acc(A0, B0);
                    acc(A1, B1);
                }
                if (t < C) {
                    double A0[D], B0[D];
                    rows(x0, A0, B0);
                    acc(A0, B0);
                }
            } else if (s < ns) {
                const uint16_t *lst = ent + eoff[s] + lane;
                const int C = cnt[s];
                uint32_t x = lst[0];
                uint32_t xn = C > 1 ? lst[64] : x;
                for (int t = 0; t < C; ++t) {
                    const uint32_t xnn = t + 2 < C ? lst[(t + 2) * 64] : xn;
                    const double *Ee = ev + int(x & 1023u) * NV;
                    if constexpr (OP == FEM_OP_ELAS) {
                        const int a = int((x >> 10) & 3u), b = int((x >> 12) & 3u);
                        double A[D], B[D];
#pragma unroll
                        for (int c = 0; c < D; ++c) {
                            A[c] = Ee[a * D + c];
                            B[c] = Ee[b * D + c];
                        }
#pragma unroll
                        for (int l = 0; l < D; ++l)
#pragma unroll
                            for (int n = 0; n < D; ++n)
                                X[s][l * D + n] = fma(A[l], B[n], X[s][l * D + n]);
                    } else if constexpr (OP == kOpElasNodal) {
                        const int a = int((x >> 10) & 3u), b = int((x >> 12) & 3u);
                        double A[D], B[D];
#pragma unroll
                        for (int c = 0; c < D; ++c) {
                            A[c] = Ee[a * D + c];
                            B[c] = Ee[b * D + c];
                        }
                        const double lk = Ee[NL * D], mk = Ee[NL * D + 1];
#pragma unroll
                        for (int l = 0; l < D; ++l)
#pragma unroll
                            for (int n = 0; n < D; ++n) {
                                const double xln = A[l] * B[n];
                                X[s][l * D + n] = fma(lk, xln, X[s][l * D + n]);
                                X[s][M2 + l * D + n] = fma(mk, xln, X[s][M2 + l * D + n]);
                            }
                    } else if constexpr (OP == kOpGeneral) {
                        const int a = int((x >> 10) & 3u), b = int((x >> 12) & 3u);
                        X[s][0] += Ee[a * NL + b];
                        X[s][1] += Ee[b * NL + a];
                    } else {
                        X[s][0] += Ee[(x >> 10) & 15u];
                    }
                    x = xn;
                    xn = xnn;
                }
            }
        }
        if (wave == 0) __builtin_amdgcn_s_setprio(0);
        __syncthreads();
        // L12: output image of the current block
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (s < ns && hd[s] != kPairPad) {
                const int r = int(hd[s] & 127u), p = int(hd[s] >> 7);
                const int4 ri = rinf[r];
                double *o = outb + M2 * ri.z + M * p;
                // the mirror pair (if any): the transposed block, or the same value
                double *o2 = nullptr;
                int len2 = 0;
                if (hd2[s] != kPairPad) {
                    const int4 r2 = rinf[hd2[s] & 127u];
                    o2 = outb + M2 * r2.z + M * int(hd2[s] >> 7);
                    len2 = r2.y;
                }
                if constexpr (OP == kOpElasNodal) {
                    double trm = X[s][M2];
#pragma unroll
                    for (int m = 1; m < D; ++m) trm += X[s][M2 + m * D + m];
#pragma unroll
                    for (int l = 0; l < D; ++l)
#pragma unroll
                        for (int n = 0; n < D; ++n) {
                            const double v = elas_combine_nodal(X[s][l * D + n],
                                                                X[s][M2 + n * D + l], trm, l == n);
                            o[l * D * ri.y + n] = v;
                            if (o2) o2[n * D * len2 + l] = v;
                        }
                } else if constexpr (OP == FEM_OP_ELAS) {
                    double tr = X[s][0];
#pragma unroll
                    for (int m = 1; m < D; ++m) tr += X[s][m * D + m];
#pragma unroll
                    for (int l = 0; l < D; ++l)
#pragma unroll
                        for (int n = 0; n < D; ++n) {
                            const double v = elas_combine(X[s][l * D + n], X[s][n * D + l], tr,
                                                          l == n, lam, mu);
                            o[l * D * ri.y + n] = v;
                            if (o2) o2[n * D * len2 + l] = v;
                        }
                } else if constexpr (OP == kOpGeneral) {
                    o[0] = X[s][0];
                    if (o2) o2[0] = X[s][1];
                } else {
                    o[0] = X[s][0];
                    if (o2) o2[0] = X[s][0];
                }
            }
        }
        __syncthreads();
        dp = dc;
        have_prev = true;
        if (bn < 0) break;
        bc = bn;
        dc = dn;
        bn = bnn;
        dn = dnn;
        bnn = bnnn;
        dv_nn = dv_nnn;
    }
    for (int kk = tid; kk < M2 * dp.nacc; kk += kPairWG) {
        const int4 ri = rinf[rowof[kk / M2]];
        pv.values[dp.vo + int64_t(M2) * ri.x + (kk - M2 * ri.z)] = outb[kk];
    }
    const unsigned long long any = __ballot(bad != 0);
    if (any != 0ull && (threadIdx.x & 63) == __ffsll((long long)any) - 1) atomicOr(status, bad);
}

template <int D, int OP, int S>
__global__ void __launch_bounds__(kPairWG) k_pair(PairView pv, double lam, double mu,
                                                  int32_t *status) {
    pair_run<D, OP, S>(pv, lam, mu, status, int(blockIdx.x), int(gridDim.x));
}

// The same kernel held to 128 VGPRs (four wavefronts per SIMD: two
// 512-thread workgroups per compute unit), for the stiffness JVP: its
// registers pass 128 by a few while its LDS allows two workgroups, and the
// handful of spilled registers cost less than the lost occupancy (measured
// on the 128^3 cube: 0.55 ms instead of 0.65; the weighted-mass JVP, whose
// LDS admits one workgroup anyway, only loses by it).
template <int D, int OP, int S>
__global__ void __launch_bounds__(kPairWG, 4) k_pair2(PairView pv, double lam, double mu,
                                                       int32_t *status) {
    pair_run<D, OP, S>(pv, lam, mu, status, int(blockIdx.x), int(gridDim.x));
}

// One persistent launch over a 2D and a 3D layout (a batch with meshes of
// both dimensions): every workgroup walks its share of the 2D blocks, then
// its share of the 3D blocks, so the two parts balance over the whole grid.
template <int OP, int S>
__global__ void __launch_bounds__(kPairWG) k_pair_mixed(PairView pv2, PairView pv3, double lam,
                                                        double mu, int32_t *status) {
    pair_run<2, OP, S>(pv2, lam, mu, status, int(blockIdx.x), int(gridDim.x));
    __syncthreads();   // the LDS is reused
    pair_run<3, OP, S>(pv3, lam, mu, status, int(blockIdx.x), int(gridDim.x));
}

template <class T>
fem_status up(T **dst, const std::vector<T> &src) {
    *dst = nullptr;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(dst), sizeof(T) * std::max<size_t>(1, src.size()));
    if (e == hipSuccess && !src.empty())
        e = copy_sync(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
    return hip_status(e);
}

uint32_t align16(size_t x) { return uint32_t((x + 15) & ~size_t(15)); }

struct PairLds {
    PairView pv;
    size_t bytes;
};

template <int D, int OP>
PairLds pair_lds(const PairPlan &P) {
    using O = PairOp<D, OP>;
    PairView pv{};
    size_t o = size_t(D) * P.max_nodes * sizeof(double);
    pv.off_w = align16(o);
    {
        // per-node fields after the coordinates: w, the second field, the
        // tangent coordinates (see k_pair)
        constexpr bool kW = OP == FEM_OP_MASS_W || OP == kOpElasNodal || OP == kOpJvpMassW;
        constexpr bool kW2 = OP == kOpElasNodal || OP == kOpJvpMassW;
        const int nf = (kW ? 1 : 0) + (kW2 ? 1 : 0) + (is_jvp(OP) ? D : 0);
        o = pv.off_w + size_t(nf) * P.max_nodes * sizeof(double);
    }
    pv.off_row = align16(o);
    o = pv.off_row + size_t(P.max_rows) * sizeof(int4);
    pv.off_rowof = align16(o);
    o = pv.off_rowof + size_t(P.max_nacc);
    pv.off_ev = align16(o);
    o = pv.off_ev + size_t(P.max_elems + 1) * O::NV * sizeof(double);
    pv.off_ent = align16(o);
    o = pv.off_ent + size_t(P.max_ent) * sizeof(uint16_t);
    o = std::max(o, pv.off_ev + size_t(O::M) * O::M * P.max_nacc * sizeof(double));
    return PairLds{pv, align16(o)};
}

template <int D, int OP>
PairView make_view(const PairPlan &P, const PairLds &L, const double *q, const double *w,
                   const double *w2, const double *gco, const double *dq, double *values) {
    PairView pv = L.pv;
    pv.desc = P.desc;
    pv.rowinfo = P.rowinfo;
    pv.nodes = P.nodes;
    pv.elem = P.elem;
    pv.task_cnt = P.task_cnt;
    pv.task_eoff = P.task_eoff;
    pv.hdr = P.hdr;
    pv.ent = P.ent;
    pv.q = q;
    pv.w = w;
    pv.w2 = w2;
    pv.dq = dq;
    for (int i = 0; i < kGeneralCoef; ++i) pv.gco[i] = gco ? gco[i] : 0.0;
    pv.values = values;
    pv.nb = P.nb;
    pv.max_nodes = P.max_nodes;
    return pv;
}

// Resident workgroups per CU of a kernel at this LDS size (cached per kernel).
int resident_wgs(const void *fn, size_t lds) {
    static std::mutex mu;
    static std::vector<std::pair<std::pair<const void *, size_t>, int>> cache;
    std::lock_guard<std::mutex> lock(mu);
    for (const auto &c : cache)
        if (c.first.first == fn && c.first.second == lds) return c.second;
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, kPairWG, lds) != hipSuccess || n < 1)
        n = 1;
    cache.push_back({{fn, lds}, n});
    return n;
}

int device_cus() {
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return std::max(cus, 8);
}

template <int D, int OP, int S>
hipError_t launch_pair_t(const PairPlan &P, const double *q, const double *w, const double *w2,
                         const double *gco, const double *dq, double lam, double mu,
                         double *values, int32_t *status, hipStream_t s) {
    PairLds L = pair_lds<D, OP>(P);
    if (L.bytes > 160 * 1024) return hipErrorNotSupported;   // caller falls back
    const PairView pv = make_view<D, OP>(P, L, q, w, w2, gco, dq, values);
    constexpr bool kTwo = OP == kOpJvpStiff;
    const void *fn;
    if constexpr (kTwo)
        fn = reinterpret_cast<const void *>(&k_pair2<D, OP, S>);
    else
        fn = reinterpret_cast<const void *>(&k_pair<D, OP, S>);
    // persistent grid: resident workgroups per CU x CUs, a multiple of the 8 XCDs
    int64_t grid = int64_t(resident_wgs(fn, L.bytes)) * device_cus() / 8 * 8;
    const int64_t need = (int64_t(P.nb) + 7) / 8 * 8;
    grid = std::max<int64_t>(8, std::min(grid, need));
    if constexpr (kTwo)
        hipLaunchKernelGGL((k_pair2<D, OP, S>), dim3(unsigned(grid)), dim3(kPairWG), L.bytes, s,
                           pv, lam, mu, status);
    else
        hipLaunchKernelGGL((k_pair<D, OP, S>), dim3(unsigned(grid)), dim3(kPairWG), L.bytes, s,
                           pv, lam, mu, status);
    return hipGetLastError();
}

template <int OP, int S>
hipError_t launch_pair_mixed_t(const PairPlan &P2, const PairPlan &P3, const double *q,
                               const double *w, double lam, double mu, double *values,
                               int32_t *status, hipStream_t s) {
    const PairLds L2 = pair_lds<2, OP>(P2), L3 = pair_lds<3, OP>(P3);
    const size_t bytes = std::max(L2.bytes, L3.bytes);
    if (bytes > 160 * 1024) return hipErrorNotSupported;
    const PairView pv2 = make_view<2, OP>(P2, L2, q, w, nullptr, nullptr, nullptr, values);
    const PairView pv3 = make_view<3, OP>(P3, L3, q, w, nullptr, nullptr, nullptr, values);
    const void *fn = reinterpret_cast<const void *>(&k_pair_mixed<OP, S>);
    int64_t grid = int64_t(resident_wgs(fn, bytes)) * device_cus() / 8 * 8;
    const int64_t need = (int64_t(std::max(P2.nb, P3.nb)) + 7) / 8 * 8;
    grid = std::max<int64_t>(8, std::min(grid, need));
    hipLaunchKernelGGL((k_pair_mixed<OP, S>), dim3(unsigned(grid)), dim3(kPairWG), bytes, s, pv2,
                       pv3, lam, mu, status);
    return hipGetLastError();
}

template <int D, int OP>
hipError_t launch_pair_s(const PairPlan &P, const double *q, const double *w, const double *w2,
                         const double *gco, const double *dq, double lam, double mu,
                         double *values, int32_t *status, hipStream_t s) {
    if (P.slots == 4)
        return launch_pair_t<D, OP, 4>(P, q, w, w2, gco, dq, lam, mu, values, status, s);
    if (P.slots == 1)
        return launch_pair_t<D, OP, 1>(P, q, w, w2, gco, dq, lam, mu, values, status, s);
    return launch_pair_t<D, OP, 2>(P, q, w, w2, gco, dq, lam, mu, values, status, s);
}

template <int D>
hipError_t launch_pair_d(const PairPlan &P, int op, const double *q, const double *w,
                         const double *w2, const double *gco, const double *dq, double lam,
                         double mu, double *values, int32_t *status, hipStream_t s) {
#define FEMASM_PAIR_CASE(OPC) \
    case OPC: return launch_pair_s<D, OPC>(P, q, w, w2, gco, dq, lam, mu, values, status, s);
    switch (op) {
        FEMASM_PAIR_CASE(FEM_OP_MASS)
        FEMASM_PAIR_CASE(FEM_OP_MASS_W)
        FEMASM_PAIR_CASE(FEM_OP_STIFF)
        FEMASM_PAIR_CASE(kOpElasNodal)
        FEMASM_PAIR_CASE(kOpGeneral)
        FEMASM_PAIR_CASE(kOpJvpMass)
        FEMASM_PAIR_CASE(kOpJvpMassW)
        FEMASM_PAIR_CASE(kOpJvpStiff)
        default: return launch_pair_s<D, FEM_OP_ELAS>(P, q, w, w2, gco, dq, lam, mu, values, status, s);
    }
#undef FEMASM_PAIR_CASE
}

}  // namespace

void free_pairs(PairPlan *p) {
    void *ptrs[] = {p->desc,      p->rowinfo, p->nodes, p->elem, p->task_cnt,  p->task_eoff,
                    p->hdr,       p->ent,     p->left_items, p->left_mesh};
    for (void *x : ptrs)
        if (x) (void)hipFree(x);
    *p = PairPlan();
}

fem_status upload_pairs(PairPlan &P, int R, int slots, bool tri, int d, int64_t nq, int64_t nme,
                        const int32_t *me, const int32_t *rp, const int32_t *ci, const int64_t *ip,
                        const int32_t *inc_k) {
    // mirror pairs inside a block are summed once (FEMASM_PAIR_DEDUP=0: off)
    bool dedup = true;
    if (const char *e = getenv("FEMASM_PAIR_DEDUP")) dedup = atoi(e) != 0;
    P = PairPlan();
    const int64_t max_pairs = int64_t(64) * kPairWaves * slots;
    // Element cap of a 3D block: the kernel keeps every block element's values
    // in LDS (11 doubles per element for the scalar operators, 13 for
    // elasticity) and its LDS size follows the largest block, so 700 / 600
    // elements keep it within the 80 KB that two workgroups per compute unit
    // allow (blocks grown against a chunk border would otherwise grow flat and
    // large).
    // FEMASM_PAIR_ELEMS / FEMASM_ELAS_ELEMS override the 3D caps.
    int ecap = d == 3 ? (tri ? 700 : 600) : kMaxBlockElems;
    if (d == 3)
        if (const char *e = getenv(tri ? "FEMASM_PAIR_ELEMS" : "FEMASM_ELAS_ELEMS"))
            ecap = std::max(64, std::min(kMaxBlockElems, atoi(e)));
    // vertices that fit no block (a star or row beyond these caps) and the
    // rows of blocks beyond the task or list-entry caps are left over: the
    // row-gather tile kernel assembles them
    // The list-entry cap of a block also bounds its growth (by the entries
    // before mirror pairs are merged), so that blocks seldom end up over it.
    const int64_t max_ent = int64_t(kEntSlots) * kPairWG * 8;
    BlockHost H = build_block_host(d, nq, nme, me, rp, ci, ip, inc_k, std::min(R, 128), 16,
                                   max_pairs, kMaxPairNodes, 8192, ecap, true, max_ent);
    if (!H.ok || H.nb == 0) return FEM_OK;   // row-gather kernel only
    PairHost PH = build_pair_host(H, d, rp, ci, kPairWaves, slots, 16, tri, dedup, max_ent);
    if (!PH.ok || H.max_nodes > std::min(kMaxPairNodes, kNodeSlots * kPairWG) ||
        H.max_elems + 1 > kElemSlots * kPairWG)
        return FEM_OK;
    std::vector<int32_t> left = H.leftover;
    for (int b = 0; b < H.nb; ++b)
        if (!PH.blk_ok[b])
            left.insert(left.end(), H.rows.begin() + H.row_ptr[b], H.rows.begin() + H.row_ptr[b + 1]);
    std::sort(left.begin(), left.end());
    std::vector<uint32_t> elem8(H.elem.size() / 4);
    for (size_t k = 0; k < elem8.size(); ++k)
        elem8[k] = uint32_t(H.elem[4 * k]) | (uint32_t(H.elem[4 * k + 1]) << 8) |
                   (uint32_t(H.elem[4 * k + 2]) << 16) | (uint32_t(H.elem[4 * k + 3]) << 24);
    int nb = 0;   // blocks with tasks (the others' rows are left over)
    for (int b = 0; b < H.nb; ++b) nb += PH.blk_ok[b];
    std::vector<int32_t> desc(size_t(nb) * kDescInts), task_eoff(PH.task_ent.size());
    std::vector<int4> rowinfo(H.rows.size());
    int64_t max_nacc = 0;
    for (int b = 0, ob = 0; b < H.nb; ++b) {
        if (!PH.blk_ok[b]) continue;
        int32_t o = 0;
        for (int r = H.row_ptr[b]; r < H.row_ptr[b + 1]; ++r) {
            const int32_t row = H.rows[r];
            const int32_t len = rp[row + 1] - rp[row];
            rowinfo[r] = make_int4(rp[row], len, o, 0);
            o += len;
        }
        max_nacc = std::max<int64_t>(max_nacc, o);
        const int32_t t0 = PH.wt[size_t(b) * (kPairWaves + 1)];
        int32_t *x = desc.data() + size_t(ob++) * kDescInts;
        x[0] = H.row_ptr[b];
        x[1] = H.row_ptr[b + 1] - H.row_ptr[b];
        x[2] = H.node_ptr[b];
        x[3] = H.node_ptr[b + 1] - H.node_ptr[b];
        x[4] = H.elem_ptr[b];
        x[5] = H.elem_ptr[b + 1] - H.elem_ptr[b];
        x[6] = o;
        x[7] = t0;
        const uint64_t wp = pack_wave_starts(&PH.wt[size_t(b) * (kPairWaves + 1)], kPairWaves);
        x[8] = int32_t((PH.ent_ptr[b + 1] - PH.ent_ptr[b]) / 8);
        x[9] = int32_t(uint32_t(wp & 0xffffffffu));
        x[12] = int32_t(uint32_t(wp >> 32));
        x[20] = int32_t(uint32_t(uint64_t(nq) & 0xffffffffu));   // one mesh: offsets 0
        x[21] = int32_t(uint64_t(nq) >> 32);
        x[10] = int32_t(uint32_t(uint64_t(PH.ent_ptr[b]) & 0xffffffffu));
        x[11] = int32_t(uint64_t(PH.ent_ptr[b]) >> 32);
        for (int t = t0; t < PH.wt[size_t(b) * (kPairWaves + 1) + kPairWaves]; ++t)
            task_eoff[t] = int32_t(PH.task_ent[t] - PH.ent_ptr[b]);
    }
    fem_status st = FEM_OK;
    if (st == FEM_OK) st = up(&P.desc, desc);
    if (st == FEM_OK) st = up(&P.rowinfo, rowinfo);
    if (st == FEM_OK) st = up(&P.nodes, H.nodes);
    if (st == FEM_OK) st = up(&P.elem, elem8);
    if (st == FEM_OK) st = up(&P.task_cnt, PH.task_cnt);
    if (st == FEM_OK) st = up(&P.task_eoff, task_eoff);
    {
        std::vector<uint32_t> hdr(PH.hdr.size());
        for (size_t k = 0; k < hdr.size(); ++k)
            hdr[k] = uint32_t(PH.hdr[k]) | (uint32_t(PH.hdr2[k]) << 16);
        if (st == FEM_OK) st = up(&P.hdr, hdr);
    }
    if (st == FEM_OK) st = up(&P.ent, PH.ent);
    if (st != FEM_OK) {
        free_pairs(&P);
        return st;
    }
    P.nb = nb;
    P.slots = slots;
    P.n_rows = int64_t(H.rows.size());
    P.n_nodes = int64_t(H.nodes.size());
    P.n_elems = int64_t(H.elem.size() / 4);
    P.n_tasks = int64_t(PH.task_cnt.size());
    P.n_ent = int64_t(PH.ent.size());
    P.h_desc = desc;
    P.h_left = std::move(left);
    P.max_rows = H.max_rows;
    P.max_nodes = H.max_nodes;
    P.max_elems = H.max_elems;
    P.max_nacc = max_nacc;
    P.max_ent = PH.max_ent;
    P.ok = true;
    return FEM_OK;
}

fem_status upload_leftover(PairPlan &P, const fem_plan_data *p, int M) {
    if (!P.ok || P.h_left.empty()) return FEM_OK;
    // tiles of consecutive leftover vertices: at most 256 dof rows (whole
    // vertices) and kLdsCap bytes of accumulators each
    const std::vector<int32_t> &rp = p->h_rp;
    auto vstart = [&](int64_t r) -> int64_t {
        const int64_t i = r / M, l = r - i * M;
        int64_t x = int64_t(M) * M * rp[i];
        if (l) x += l * M * int64_t(rp[i + 1] - rp[i]);
        return x;
    };
    const int R = 256 / M * M;
    std::vector<BatchItem> items;
    size_t lds = sizeof(double);
    const std::vector<int32_t> &L = P.h_left;
    for (size_t i = 0; i < L.size();) {
        const int64_t v0 = L[i];
        size_t j = i + 1;
        auto bytes_to = [&](int64_t v1) {   // vertices [v0, v1)
            return tile_lds_bytes(M, vstart(M * v1) - vstart(M * v0), M * (v1 - v0));
        };
        if (bytes_to(v0 + 1) > kLdsCap) {   // one vertex beyond the tile memory
            free_pairs(&P);
            return FEM_OK;                  // no pair layout: row-gather for every row
        }
        while (j < L.size() && L[j] == L[j - 1] + 1 && int64_t(M) * (L[j] + 1 - v0) <= R &&
               bytes_to(L[j] + 1) <= kLdsCap)
            ++j;
        const int64_t v1 = L[j - 1] + 1;
        BatchItem it;
        it.mesh = 0;
        it.nrows = int32_t(M * (v1 - v0));
        it.row0 = M * v0;
        items.push_back(it);
        lds = std::max(lds, bytes_to(v1));
        i = j;
    }
    BatchMesh bm;
    bm.rp = p->rp;
    bm.inc_ptr = p->inc_ptr;
    bm.inc_elem = p->inc_elem;
    bm.inc_off = p->inc_off;
    bm.pme = p->pme;
    bm.nq = p->nq;
    bm.q_off = bm.w_off = 0;
    bm.val_off[0] = bm.val_off[1] = 0;
    bm.d = p->d;
    bm.pad = 0;
    fem_status st = up(&P.left_items, items);
    if (st == FEM_OK) st = up(&P.left_mesh, std::vector<BatchMesh>(1, bm));
    if (st != FEM_OK) return st;
    P.n_left_items = int64_t(items.size());
    P.left_rpw = R;
    P.left_lds = lds;
    return FEM_OK;
}

hipError_t launch_pair_layout(const PairPlan &P, int d, int op, const double *q, const double *w,
                              double lam, double mu, double *values, int32_t *status,
                              hipStream_t s, const double *w2, const double *gco,
                              const double *dq) {
    return d == 2 ? launch_pair_d<2>(P, op, q, w, w2, gco, dq, lam, mu, values, status, s)
                  : launch_pair_d<3>(P, op, q, w, w2, gco, dq, lam, mu, values, status, s);
}

hipError_t launch_pair_mixed(const PairPlan &P2, const PairPlan &P3, int op, const double *q,
                             const double *w, double lam, double mu, double *values,
                             int32_t *status, hipStream_t s) {
    if (P2.slots != P3.slots) return hipErrorNotSupported;
#define FEMASM_MIXED(OPC, SS) \
    return launch_pair_mixed_t<OPC, SS>(P2, P3, q, w, lam, mu, values, status, s);
#define FEMASM_MIXED_S(OPC)                           \
    if (P2.slots == 4) { FEMASM_MIXED(OPC, 4) }       \
    if (P2.slots == 1) { FEMASM_MIXED(OPC, 1) }       \
    FEMASM_MIXED(OPC, 2)
    switch (op) {
        case FEM_OP_MASS: FEMASM_MIXED_S(FEM_OP_MASS)
        case FEM_OP_MASS_W: FEMASM_MIXED_S(FEM_OP_MASS_W)
        case FEM_OP_STIFF: FEMASM_MIXED_S(FEM_OP_STIFF)
        case FEM_OP_ELAS: FEMASM_MIXED_S(FEM_OP_ELAS)
        default: return hipErrorNotSupported;
    }
#undef FEMASM_MIXED_S
#undef FEMASM_MIXED
}

bool launch_pair(const fem_plan_data *p, int op, const double *q, const double *w, double lam,
                 double mu, double *values, hipStream_t s, hipError_t *err, const double *w2,
                 const double *gco, const double *dq) {
    // the (a, b)-coded layout serves elasticity and the non-symmetric operator
    if (!layouts_ready(p)) return false;   // still being built (or none)
    const PairPlan &P = is_elas(op) || op == kOpGeneral ? p->pvec : p->pscal;
    if (!P.ok) return false;
    // leftover rows: the row-gather tile kernel, which has the four P1 operators
    const bool p1 = op == FEM_OP_MASS || op == FEM_OP_MASS_W || op == FEM_OP_STIFF || op == FEM_OP_ELAS;
    if (P.n_left_items > 0 && !p1) return false;
    hipError_t e =
        launch_pair_layout(P, p->d, op, q, w, lam, mu, values, p->status, s, w2, gco, dq);
    if (e == hipErrorNotSupported) return false;
    if (e == hipSuccess && P.n_left_items > 0) {
        const fem_status st = launch_batch(op, P.left_mesh, P.left_items, P.n_left_items,
                                           P.left_rpw, P.left_lds, 1024, 0, 0, q, w, lam, mu,
                                           values, p->status, s);
        if (st != FEM_OK) e = hipErrorLaunchFailure;
    }
    *err = e;
    return true;
}

fem_status concat_pairs(PairPlan &out, const std::vector<const PairPlan *> &parts,
                        const std::vector<int64_t> &qo, const std::vector<int64_t> &wo,
                        const std::vector<int64_t> &vo, const std::vector<int64_t> &nq) {
    out = PairPlan();
    if (parts.empty()) return FEM_OK;
    int64_t rows = 0, nodes = 0, elems = 0, tasks = 0, ents = 0, nb = 0;
    for (const PairPlan *P : parts) {
        // no batched pair layout (also when a mesh has leftover rows)
        if (!P->ok || P->slots != parts[0]->slots || P->n_left_items > 0) return FEM_OK;
        rows += P->n_rows;
        nodes += P->n_nodes;
        elems += P->n_elems;
        tasks += P->n_tasks;
        ents += P->n_ent;
        nb += P->nb;
    }
    std::vector<int32_t> desc(size_t(nb) * kDescInts);
    auto put64 = [](int32_t *x, int64_t v) {
        x[0] = int32_t(uint32_t(uint64_t(v) & 0xffffffffu));
        x[1] = int32_t(uint64_t(v) >> 32);
    };
    fem_status st = FEM_OK;
    hipError_t e = hipSuccess;
    auto alloc = [&](auto **ptr, int64_t n) {
        if (e == hipSuccess)
            e = hipMalloc(reinterpret_cast<void **>(ptr), sizeof(**ptr) * size_t(std::max<int64_t>(1, n)));
    };
    alloc(&out.rowinfo, rows);
    alloc(&out.nodes, nodes);
    alloc(&out.elem, elems);
    alloc(&out.task_cnt, tasks);
    alloc(&out.task_eoff, tasks);
    alloc(&out.hdr, 64 * tasks);
    alloc(&out.ent, ents);
    int64_t r0 = 0, n0 = 0, e0 = 0, t0 = 0, eb = 0, b0 = 0;
    for (size_t m = 0; m < parts.size() && e == hipSuccess; ++m) {
        const PairPlan &P = *parts[m];
        auto cp = [&](auto *dst, const auto *src, int64_t n) {
            if (e == hipSuccess && n > 0)
                e = hipMemcpy(dst, src, sizeof(*src) * size_t(n), hipMemcpyDeviceToDevice);
        };
        cp(out.rowinfo + r0, P.rowinfo, P.n_rows);
        cp(out.nodes + n0, P.nodes, P.n_nodes);
        cp(out.elem + e0, P.elem, P.n_elems);
        cp(out.task_cnt + t0, P.task_cnt, P.n_tasks);
        cp(out.task_eoff + t0, P.task_eoff, P.n_tasks);
        cp(out.hdr + 64 * t0, P.hdr, 64 * P.n_tasks);
        cp(out.ent + eb, P.ent, P.n_ent);
        for (int b = 0; b < P.nb; ++b) {
            int32_t *x = desc.data() + size_t(b0 + b) * kDescInts;
            const int32_t *y = P.h_desc.data() + size_t(b) * kDescInts;
            std::copy(y, y + kDescInts, x);
            x[0] += int32_t(r0);
            x[2] += int32_t(n0);
            x[4] += int32_t(e0);
            x[7] += int32_t(t0);
            put64(x + 10, (int64_t(uint32_t(y[10])) | (int64_t(y[11]) << 32)) + eb);
            put64(x + 14, qo[m]);
            put64(x + 16, wo[m]);
            put64(x + 18, vo[m]);
            put64(x + 20, nq[m]);
        }
        r0 += P.n_rows;
        n0 += P.n_nodes;
        e0 += P.n_elems;
        t0 += P.n_tasks;
        eb += P.n_ent;
        b0 += P.nb;
        out.max_rows = std::max(out.max_rows, P.max_rows);
        out.max_nodes = std::max(out.max_nodes, P.max_nodes);
        out.max_elems = std::max(out.max_elems, P.max_elems);
        out.max_nacc = std::max(out.max_nacc, P.max_nacc);
        out.max_ent = std::max(out.max_ent, P.max_ent);
    }
    if (e == hipSuccess) st = up(&out.desc, desc);
    else st = hip_status(e);
    if (st != FEM_OK || rows >= (int64_t(1) << 31) || nodes >= (int64_t(1) << 31) ||
        tasks >= (int64_t(1) << 31)) {
        free_pairs(&out);
        return st;
    }
    out.nb = int(nb);
    out.slots = parts[0]->slots;
    out.n_rows = rows;
    out.n_nodes = nodes;
    out.n_elems = elems;
    out.n_tasks = tasks;
    out.n_ent = ents;
    out.h_desc = std::move(desc);
    out.ok = true;
    return FEM_OK;
}

}  // namespace femasm
