// Row-gather assembly of one tile of CSR rows (device side).
//
// One thread owns one CSR row (a vertex for scalar operators, a (vertex,
// component) dof for elasticity).  It walks the vertex's incidences in
// ascending element number, recomputes that element's geometry, and adds the
// element-matrix row of its local vertex into the row's segment of an LDS
// tile that mirrors the contiguous CSR value range of the workgroup's rows.
// Because a row is only ever touched by its own thread, in a fixed order, the
// sums are deterministic without atomics; the tile is then written to HBM
// with coalesced stores.
#pragma once

#include "element.h"
#include "femasm_impl.h"

#pragma clang fp contract(off)

namespace femasm {

// First CSR value position of dof row r (r = M*i + l) of an operator whose
// pattern is the scalar pattern expanded to M x M blocks.
template <int M>
__device__ __forceinline__ int64_t vrow_start(const int32_t *__restrict__ rp, int64_t r) {
    if (M == 1) return rp[r];
    const int64_t i = r / M;
    const int64_t l = r - i * M;
    int64_t s = int64_t(M) * M * rp[i];
    if (l) s += l * M * int64_t(rp[i + 1] - rp[i]);
    return s;
}

// Bijective block -> tile map that hands each of the 8 XCDs (blocks are
// dealt round-robin to them) a contiguous range of tiles, so neighbouring
// rows share an L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nb) {
    const int64_t xcd = b & 7, idx = b >> 3;
    const int64_t per = nb >> 3, rem = nb & 7;
    return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

// v[a] for a runtime index a, as a chain of conditional moves on scalars
// (keeps the operands in registers; an indexed array would go to scratch).
__device__ __forceinline__ double pick(double v0, double v1, double v2, int a) {
    double r = v0;
    r = (a == 1) ? v1 : r;
    r = (a == 2) ? v2 : r;
    return r;
}
__device__ __forceinline__ double pick(double v0, double v1, double v2, double v3, int a) {
    double r = v0;
    r = (a == 1) ? v1 : r;
    r = (a == 2) ? v2 : r;
    r = (a == 3) ? v3 : r;
    return r;
}
template <int D>
__device__ __forceinline__ double sel(const double (&v)[D + 1], int a) {
    if constexpr (D == 2)
        return pick(v[0], v[1], v[2], a);
    else
        return pick(v[0], v[1], v[2], v[3], a);
}

template <int D, int OP>
__device__ __forceinline__ void assemble_row_tile(const MeshView &mv, int64_t r0, int64_t r1,
                                                  double *__restrict__ acc, double lam, double mu,
                                                  int &bad) {
    constexpr int M = (OP == FEM_OP_ELAS) ? D : 1;
    constexpr int NL = D + 1;
    const int64_t base = vrow_start<M>(mv.rp, r0);
    const int64_t top = vrow_start<M>(mv.rp, r1);
    const int nacc = int(top - base);
    for (int s = threadIdx.x; s < nacc; s += blockDim.x) acc[s] = 0.0;
    // Elasticity tiles hold whole vertices (r0, r1 multiples of M).  After the
    // accumulators: per vertex its segment start and row length, and for each
    // group of M*M accumulators the vertex it belongs to (combining epilogue).
    int32_t *vinfo = nullptr;
    uint8_t *vof = nullptr;
    int nv = 0;
    if constexpr (OP == FEM_OP_ELAS) {
        nv = int((r1 - r0) / M);
        vinfo = reinterpret_cast<int32_t *>(acc + nacc);
        vof = reinterpret_cast<uint8_t *>(vinfo + 2 * nv);
        for (int v = threadIdx.x; v < nv; v += blockDim.x) {
            const int64_t i = r0 / M + v;
            const int b0 = int(vrow_start<M>(mv.rp, i * M) - base);
            const int len = mv.rp[i + 1] - mv.rp[i];
            vinfo[v] = b0;
            vinfo[nv + v] = len;
            for (int k = 0; k < len; ++k) vof[b0 / (M * M) + k] = uint8_t(v);
        }
    }
    __syncthreads();

    const int64_t r = r0 + threadIdx.x;
    if (r < r1) {
        const int64_t i = r / M;
        const int l = int(r - i * M);
        double *__restrict__ my = acc + (vrow_start<M>(mv.rp, r) - base);
        const int t0 = mv.inc_ptr[i], t1 = mv.inc_ptr[i + 1];
        const int64_t nq = mv.nq;
        for (int t = t0; t < t1; ++t) {
            const uint32_t ea = mv.inc_elem[t];
            const uint64_t off = mv.inc_off[t];
            const int64_t e = ea & 0x3fffffffu;
            const int al = int(ea >> 30);
            int v[NL];
#pragma unroll
            for (int b = 0; b < NL; ++b) v[b] = mv.pme[e * NL + b];
            double P[NL][D];
#pragma unroll
            for (int b = 0; b < NL; ++b)
#pragma unroll
                for (int x = 0; x < D; ++x) P[b][x] = mv.q[x * nq + v[b]];

            if constexpr (OP == FEM_OP_MASS || OP == FEM_OP_MASS_W) {
                const double det = elem_det(P);
                if (det == 0.0) { bad = 1; continue; }
                const double ad = fabs(det);
                if constexpr (OP == FEM_OP_MASS) {
                    const double k = ad / Fact<D>::mass_den;
#pragma unroll
                    for (int b = 0; b < NL; ++b) {
                        const int pos = int((off >> (16 * b)) & 0xffffu);
                        my[pos] += (b == al) ? 2.0 * k : k;
                    }
                } else {
                    double wl[NL];
#pragma unroll
                    for (int b = 0; b < NL; ++b) wl[b] = mv.w[v[b]];
                    double ws = wl[0];
#pragma unroll
                    for (int b = 1; b < NL; ++b) ws += wl[b];
                    const double k = ad / Fact<D>::massw_den;
                    const double wa = sel<D>(wl, al);
#pragma unroll
                    for (int b = 0; b < NL; ++b) {
                        const int pos = int((off >> (16 * b)) & 0xffffu);
                        const double f = (b == al) ? 2.0 * k : k;
                        my[pos] += f * (ws + (wa + wl[b]));
                    }
                }
            } else {
                Elem<D> E;
                elem_geometry(P, E);
                if (E.det == 0.0) { bad = 1; continue; }
                double ca[D];
#pragma unroll
                for (int x = 0; x < D; ++x) {
                    double cx[NL];
#pragma unroll
                    for (int b = 0; b < NL; ++b) cx[b] = E.c[b][x];
                    ca[x] = sel<D>(cx, al);
                }
                if constexpr (OP == FEM_OP_STIFF) {
                    const double inv = 1.0 / (Fact<D>::dfact * fabs(E.det));
#pragma unroll
                    for (int b = 0; b < NL; ++b) {
                        const int pos = int((off >> (16 * b)) & 0xffffu);
                        my[pos] += cdot<D>(ca, E.c[b]) * inv;
                    }
                } else {
                    // elasticity: X_ln += ch_al ch_bn for the columns (b, n)
                    const double sc = elas_scale<D>(E.det);
                    double cal;
                    if constexpr (D == 2)
                        cal = (l == 1) ? ca[1] : ca[0];
                    else
                        cal = pick(ca[0], ca[1], ca[2], l);
                    const double chal = cal * sc;
#pragma unroll
                    for (int b = 0; b < NL; ++b) {
                        const int pos = int((off >> (16 * b)) & 0xffffu);
#pragma unroll
                        for (int n = 0; n < D; ++n)
                            my[M * pos + n] = fma(chal, E.c[b][n] * sc, my[M * pos + n]);
                    }
                }
            }
        }
    }
    __syncthreads();
    if constexpr (OP == FEM_OP_ELAS) {
        for (int s = threadIdx.x; s < nacc; s += blockDim.x) {
            const int v = vof[s / (M * M)];
            const int b0 = vinfo[v], ml = M * vinfo[nv + v];
            const int sl = s - b0;
            const int l = sl / ml, rem = sl - l * ml, pos = rem / M, n = rem - pos * M;
            const double *x = acc + b0 + M * pos;
            double tr = x[0];
#pragma unroll
            for (int m = 1; m < M; ++m) tr += x[m * ml + m];
            mv.values[base + s] = elas_combine(x[l * ml + n], x[n * ml + l], tr, l == n, lam, mu);
        }
    } else {
        for (int s = threadIdx.x; s < nacc; s += blockDim.x) mv.values[base + s] = acc[s];
    }
}

}  // namespace femasm
