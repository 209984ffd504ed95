// P_k Lagrange mass matrix (Appendix D of the paper): symbolic phase and
// numeric kernels.
//
// For P_k Lagrange elements on straight simplices the element mass matrix is
// d! |K| C, with C an N x N constant (N = (d+k)!/(d! k!)) that follows from
// writing each basis function as a polynomial in the barycentric coordinates
// and integrating products with the magic formula of Section 2.  The numeric
// phase therefore needs, per element, only d! |K| = |det B_K| (from its d+1
// vertices), and per CSR entry the (element, local entry) pairs that feed it.
//
// Local numbering of an element's N nodes (the multi-indices alpha with
// |alpha| = k, alpha_i the exponent of the barycentric coordinate of local
// vertex i): local nodes 0..d are the vertices alpha = k e_i, the others
// follow in decreasing lexicographic order of (alpha_0, ..., alpha_d).
//
// Plan (built once from the connectivity, layout in pk_host.h): the CSR
// pattern, CSR entries cut into tiles of kPkTile consecutive entries with per
// entry its contributions (element, packed-triangle index of (a, b)) in
// ascending element number, the vertex rows of the connectivity (geometry)
// and C (packed upper triangle).
// Numeric phase: k_pk_vol writes |det B_K| for every element; k_pk_mass, a
// persistent kernel, keeps C in LDS, turns each tile's items (read
// coalesced) into products in LDS, and every thread sums the products of its
// entries from 0.0 in ascending element order and writes the values
// (coalesced).
#include <algorithm>
#include <cmath>
#include <memory>
#include <thread>

#include "element.h"
#include "femasm_impl.h"
#include "pk_host.h"

namespace femasm {

struct fem_pk_data {
    int d = 0, k = 0, n = 0, ntri = 0, ebits = 0;
    bool boundary = false;          // facets of dimension d-1 embedded in R^d (k = 1)
    int64_t nq = 0, nme = 0, nnz = 0, ntiles = 0, nitems = 0;
    int max_tile_items = 0;
    int device = 0;
    int32_t *rp = nullptr, *ci = nullptr;
    int32_t *gme = nullptr;         // (d+1) x nme vertex ids
    int64_t *tile_item = nullptr;   // [ntiles+1] first item of each tile
    uint16_t *coff = nullptr;       // [ntiles*kPkTile] first item of each entry, tile-relative
    uint32_t *item = nullptr;       // element | tri code << ebits
    double *ctri = nullptr;         // [ntri]
    double *vol = nullptr;          // [nme] |det B_K| (work array of the numeric phase)
    double *ev = nullptr;           // boundary plans: [nme*ntri] element matrices (work array)
    int32_t *status = nullptr;
    // k = 1 (volume meshes): the P1 plan whose mass kernels serve fem_pk_mass
    // (the P_k mass of degree 1 is the P1 mass), null if it could not be made
    fem_plan p1 = nullptr;
};

namespace {

template <class T>
fem_status pk_upload(T **dst, const std::vector<T> &src) {
    *dst = nullptr;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(dst), sizeof(T) * std::max<size_t>(src.size(), 1));
    if (e != hipSuccess) {
        *dst = nullptr;
        return hip_status(e);
    }
    if (!src.empty()) e = hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
    return hip_status(e);
}

void pk_free(fem_pk_data *p) {
    fem_plan_destroy(p->p1);
    p->p1 = nullptr;
    void *ptrs[] = {p->rp,   p->ci,   p->gme, p->tile_item, p->coff,
                    p->item, p->ctri, p->vol, p->ev,        p->status};
    for (void *x : ptrs)
        if (x) (void)hipFree(x);
}

// ---------------------------------------------------------------- kernels
template <int D>
__global__ __launch_bounds__(256) void k_pk_vol(const int32_t *__restrict__ gme, int64_t nme,
                                                const double *__restrict__ q, int64_t nq,
                                                double *__restrict__ vol, int32_t *status) {
    const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= nme) return;
    double P[D + 1][D];
#pragma unroll
    for (int a = 0; a <= D; ++a) {
        const int64_t v = gme[a * nme + e];
#pragma unroll
        for (int x = 0; x < D; ++x) P[a][x] = q[x * nq + v];
    }
    Elem<D> E;
    elem_geometry(P, E);
    vol[e] = fabs(E.det);
    if (E.det == 0.0) atomicOr(status, 1);
}

// Items of a tile are staged `chunk` at a time (at most kPkMaxChunk): read
// coalesced, turned into products |det B_K| * C[code] in LDS, then each
// thread adds the products of its entries (contiguous, ascending element) in
// order.  The first chunk and the entry offsets of the next tile are loaded
// into registers while the current tile is summed.
constexpr int kPkMaxChunk = 2048;
constexpr int kPkRegs = kPkMaxChunk / kPkThreads;

// Boundary facets ((D-1)-simplices in R^D): the packed element matrix of
// the mass (ctri times n!|K|) or of the weighted mass
// n!|K| (1+delta) (w^s + w_a + w_b) / (n+3)!, n = D-1, with n!|K| the
// length of a segment (D = 2) or |e1 x e2| of a triangle (D = 3).
template <int D, bool W>
__global__ __launch_bounds__(256) void k_bnd_elem(const int32_t *__restrict__ gme, int64_t nf,
                                                  const double *__restrict__ q, int64_t nq,
                                                  const double *__restrict__ w,
                                                  const double *__restrict__ ctri,
                                                  double *__restrict__ ev, int32_t *status) {
    constexpr int NL = D;                       // vertices of a facet
    constexpr int NT = NL * (NL + 1) / 2;
    constexpr double kDen = D == 2 ? 24.0 : 120.0;   // (n+3)!
    const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= nf) return;
    double P[NL][D];
    int64_t v[NL];
#pragma unroll
    for (int a = 0; a < NL; ++a) {
        v[a] = gme[a * nf + e];
#pragma unroll
        for (int x = 0; x < D; ++x) P[a][x] = q[x * nq + v[a]];
    }
    double m;
    if constexpr (D == 2) {
        const double dx = P[1][0] - P[0][0], dy = P[1][1] - P[0][1];
        m = sqrt(fma(dx, dx, dy * dy));
    } else {
        double e1[3], e2[3];
#pragma unroll
        for (int x = 0; x < 3; ++x) {
            e1[x] = P[1][x] - P[0][x];
            e2[x] = P[2][x] - P[0][x];
        }
        const double cx = fma(e1[1], e2[2], -(e1[2] * e2[1]));
        const double cy = fma(e1[2], e2[0], -(e1[0] * e2[2]));
        const double cz = fma(e1[0], e2[1], -(e1[1] * e2[0]));
        m = sqrt(fma(cx, cx, fma(cy, cy, cz * cz)));
    }
    if (m == 0.0) atomicOr(status, 1);
    double *out = ev + e * NT;
    if constexpr (!W) {
#pragma unroll
        for (int t = 0; t < NT; ++t) out[t] = m * ctri[t];
    } else {
        double wl[NL];
#pragma unroll
        for (int a = 0; a < NL; ++a) wl[a] = w[v[a]];
        double ws = wl[0];
#pragma unroll
        for (int a = 1; a < NL; ++a) ws += wl[a];
        const double k = m / kDen;
        int t = 0;
#pragma unroll
        for (int a = 0; a < NL; ++a)
#pragma unroll
            for (int b = a; b < NL; ++b, ++t) out[t] = (a == b ? 2.0 * k : k) * (ws + (wl[a] + wl[b]));
    }
}

__global__ __launch_bounds__(kPkThreads) void k_pk_mass(
    const int64_t *__restrict__ tile_item, const uint16_t *__restrict__ coff,
    const uint32_t *__restrict__ item, const double *__restrict__ ctri, int ntri, int ebits,
    int chunk, const double *__restrict__ vol, const double *__restrict__ ev, int64_t ntiles,
    int64_t nnz, double *__restrict__ values) {
    extern __shared__ double lds[];
    double *sc = lds;                    // C, packed triangle
    double *sp = lds + ntri;             // products of the current chunk
    const int tid = threadIdx.x;
    const uint32_t emask = (1u << ebits) - 1u;
    for (int t = tid; t < ntri; t += kPkThreads) sc[t] = ctri[t];

    int64_t i0 = 0;
    int ni = 0;
    int c0[kPkPer], c1[kPkPer];
    uint32_t x[kPkRegs];
    auto fetch = [&](int64_t t) {
        i0 = tile_item[t];
        ni = int(tile_item[t + 1] - i0);
#pragma unroll
        for (int j = 0; j < kPkPer; ++j) {
            const int l = tid + kPkThreads * j;
            const int64_t s = t * kPkTile + l;
            c0[j] = c1[j] = 0;
            if (s < nnz) {
                c0[j] = coff[s];
                c1[j] = (l + 1 < kPkTile && s + 1 < nnz) ? int(coff[s + 1]) : ni;
            }
        }
        const int cn = min(chunk, ni);
#pragma unroll
        for (int r = 0; r < kPkRegs; ++r) {
            const int u = tid + kPkThreads * r;
            x[r] = u < cn ? item[i0 + u] : 0u;
        }
    };
    int64_t tile = blockIdx.x;
    if (tile < ntiles) fetch(tile);
    for (; tile < ntiles; tile += gridDim.x) {
        const int64_t ti0 = i0;
        const int tni = ni;
        int a0[kPkPer], a1[kPkPer];
#pragma unroll
        for (int j = 0; j < kPkPer; ++j) {
            a0[j] = c0[j];
            a1[j] = c1[j];
        }
        __syncthreads();                 // sc ready; the previous tile is done with sp
        {
            const int cn = min(chunk, tni);
#pragma unroll
            for (int r = 0; r < kPkRegs; ++r) {
                const int u = tid + kPkThreads * r;
                if (u < cn)
                    sp[u] = ev ? ev[int64_t(x[r] & emask) * ntri + (x[r] >> ebits)]
                               : vol[x[r] & emask] * sc[x[r] >> ebits];
            }
        }
        if (tile + gridDim.x < ntiles) fetch(tile + gridDim.x);
        __syncthreads();
        double acc[kPkPer];
#pragma unroll
        for (int j = 0; j < kPkPer; ++j) {
            acc[j] = 0.0;
            const int hi = min(a1[j], chunk);
            for (int c = a0[j]; c < hi; ++c) acc[j] += sp[c];
        }
        for (int cb = chunk; cb < tni; cb += chunk) {     // tiles with more items than a chunk
            const int cn = min(chunk, tni - cb);
            __syncthreads();
            for (int u = tid; u < cn; u += kPkThreads) {
                const uint32_t xx = item[ti0 + cb + u];
                sp[u] = ev ? ev[int64_t(xx & emask) * ntri + (xx >> ebits)]
                           : vol[xx & emask] * sc[xx >> ebits];
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kPkPer; ++j) {
                const int lo = max(a0[j], cb), hi = min(a1[j], cb + cn);
                for (int c = lo; c < hi; ++c) acc[j] += sp[c - cb];
            }
        }
#pragma unroll
        for (int j = 0; j < kPkPer; ++j) {
            const int64_t s = tile * kPkTile + tid + kPkThreads * j;
            if (s < nnz) values[s] = acc[j];
        }
    }
}

// Pipelined form of k_pk_mass, for the plans with a large C (the highest
// degrees): the same sums in the same order, with three tiles in flight, so
// that the gathers of the element factors, which depend on the items, no
// longer wait a full memory latency at every tile.  What it holds for one
// tile in flight: its item range, the item offsets of the thread's entries,
// the items and, once gathered, their element factors (|det B_K|, or the
// element value).
struct PkTile {
    int64_t t, i0;
    int ni;
    uint32_t r0[kPkPer], r1[kPkPer];   // raw item offsets of the entry and the next one
    uint32_t x[kPkRegs];
    double f[kPkRegs];
};

__global__ __launch_bounds__(kPkThreads) void k_pk_mass_pipe(
    const int64_t *__restrict__ tile_item, const uint16_t *__restrict__ coff,
    const uint32_t *__restrict__ item, const double *__restrict__ ctri, int ntri, int ebits,
    int chunk, const double *__restrict__ vol, const double *__restrict__ ev, int64_t ntiles,
    int64_t nnz, double *__restrict__ values) {
    extern __shared__ double lds[];
    double *sc = lds;                    // C, packed triangle
    double *sp = lds + ntri;             // products of the current chunk
    const int tid = threadIdx.x;
    const uint32_t emask = (1u << ebits) - 1u;
    for (int t = tid; t < ntri; t += kPkThreads) sc[t] = ctri[t];

    // items (and entry offsets) of tile t
    // (the entry offsets are loaded unconditionally, clamped, and only
    // interpreted when the tile is summed: nothing here waits for a load)
    auto fetch = [&](PkTile &T, int64_t t) {
        T.t = t;
        T.i0 = tile_item[t];
        T.ni = int(tile_item[t + 1] - T.i0);
#pragma unroll
        for (int j = 0; j < kPkPer; ++j) {
            const int64_t s = t * kPkTile + tid + kPkThreads * j;
            T.r0[j] = coff[min(s, nnz - 1)];
            T.r1[j] = coff[min(s + 1, nnz - 1)];
        }
        const int cn = min(chunk, T.ni);
#pragma unroll
        for (int r = 0; r < kPkRegs; ++r) {
            const int u = tid + kPkThreads * r;
            T.x[r] = u < cn ? item[T.i0 + u] : 0u;
        }
    };
    // element factors of a fetched tile's first chunk
    // (one load per item, its address chosen first: two loads into the same
    // register on the two sides of a branch would make the compiler wait for
    // every load in flight before the second)
    const double *fsrc = ev ? ev : vol;
    auto gather = [&](PkTile &T) {
        const int cn = min(chunk, T.ni);
#pragma unroll
        for (int r = 0; r < kPkRegs; ++r) {
            const int u = tid + kPkThreads * r;
            const int64_t e = T.x[r] & emask;
            const int64_t o = ev ? e * ntri + (T.x[r] >> ebits) : e;
            T.f[r] = u < cn ? fsrc[o] : 0.0;
        }
    };

    // Three tiles in flight: A (items and factors in registers), B (items;
    // its factors are gathered while A is summed), C (items loaded while A is
    // summed).  Each load has a whole tile's work to arrive.
    const int64_t G = gridDim.x;
    int64_t tile = blockIdx.x;
    PkTile A, B, C;
    if (tile >= ntiles) return;
    fetch(A, tile);
    gather(A);
    fetch(B, min(tile + G, ntiles - 1));
    // one tile: X current, Y next, Z the one after (the roles rotate over
    // three unrolled steps, so no tile's registers are copied)
    auto step = [&](PkTile &X, PkTile &Y, PkTile &Z) __attribute__((always_inline)) {
        // the loads of the previous step (X's factors, Y's items) are in
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0); expcnt, lgkmcnt unlimited
        const int64_t ti0 = X.i0;
        const int tni = X.ni;
        // item range of each entry: [c0, c1), tile-relative
        int c0[kPkPer], c1[kPkPer];
#pragma unroll
        for (int j = 0; j < kPkPer; ++j) {
            const int l = tid + kPkThreads * j;
            const int64_t s = tile * kPkTile + l;
            c0[j] = s < nnz ? int(X.r0[j]) : 0;
            c1[j] = s < nnz ? ((l + 1 < kPkTile && s + 1 < nnz) ? int(X.r1[j]) : tni) : 0;
        }
        __syncthreads();                 // sc ready; the previous tile is done with sp
        {
            const int cn = min(chunk, tni);
#pragma unroll
            for (int r = 0; r < kPkRegs; ++r) {
                const int u = tid + kPkThreads * r;
                if (u < cn) sp[u] = ev ? X.f[r] : X.f[r] * sc[X.x[r] >> ebits];
            }
        }
        // (unconditional, the tile index clamped: the registers of a tile past
        // the end are never used, and no branch merges them)
        gather(Y);
        fetch(Z, min(tile + 2 * G, ntiles - 1));
        __syncthreads();
        double acc[kPkPer];
#pragma unroll
        for (int j = 0; j < kPkPer; ++j) {
            acc[j] = 0.0;
            const int hi = min(c1[j], chunk);
            for (int c = c0[j]; c < hi; ++c) acc[j] += sp[c];
        }
        for (int cb = chunk; cb < tni; cb += chunk) {     // tiles with more items than a chunk
            const int cn = min(chunk, tni - cb);
            __syncthreads();
            for (int u = tid; u < cn; u += kPkThreads) {
                const uint32_t xx = item[ti0 + cb + u];
                sp[u] = ev ? ev[int64_t(xx & emask) * ntri + (xx >> ebits)]
                           : vol[xx & emask] * sc[xx >> ebits];
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < kPkPer; ++j) {
                const int lo = max(c0[j], cb), hi = min(c1[j], cb + cn);
                for (int c = lo; c < hi; ++c) acc[j] += sp[c - cb];
            }
        }
#pragma unroll
        for (int j = 0; j < kPkPer; ++j) {
            const int64_t s = tile * kPkTile + tid + kPkThreads * j;
            if (s < nnz) values[s] = acc[j];
        }
    };
    for (;;) {
        if (tile >= ntiles) break;
        step(A, B, C);
        tile += G;
        if (tile >= ntiles) break;
        step(B, C, A);
        tile += G;
        if (tile >= ntiles) break;
        step(C, A, B);
        tile += G;
    }
}

// Items per chunk: as many as fit next to C in kPkLdsBudget bytes of LDS
// (a multiple of the workgroup size, between one per thread and kPkMaxChunk).
constexpr size_t kPkLdsBudget = 40 * 1024;
inline int pk_chunk(int ntri) {
    const int64_t room = int64_t(kPkLdsBudget / sizeof(double)) - ntri;
    const int64_t c = std::max<int64_t>(kPkThreads, std::min<int64_t>(kPkMaxChunk, room)) /
                      kPkThreads * kPkThreads;
    return int(c);
}

int pk_grid(const void *fn, size_t lds, int64_t ntiles) {
    static thread_local int cached[2] = {0, 0};
    static thread_local size_t cached_lds[2] = {0, 0};
    const int ci = fn == reinterpret_cast<const void *>(&k_pk_mass) ? 0 : 1;
    if (cached[ci] == 0 || cached_lds[ci] != lds) {
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, kPkThreads, lds) != hipSuccess ||
            n < 1)
            n = 1;
        cached[ci] = n;
        cached_lds[ci] = lds;
    }
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (cus < 1) cus = 1;
    return int(std::max<int64_t>(1, std::min<int64_t>(ntiles, int64_t(cached[ci]) * cus)));
}

}  // namespace
}  // namespace femasm

using namespace femasm;

struct fem_pk_plan_s : femasm::fem_pk_data {};

namespace {

// The P1 plan of a degree-1 mesh, its block layouts built (waited for), and
// its CSR pattern checked equal to the P_k plan's (rp, ci); null when any of
// that fails (fem_pk_mass then keeps the P_k kernels).
fem_plan pk_p1_plan(int d, int64_t nq, int64_t nme, const int32_t *me,
                    const std::vector<int32_t> &rp, const std::vector<int32_t> &ci,
                    hipStream_t stream) {
    fem_plan q1 = nullptr;
    if (fem_assemble_symbolic(d, nq, nme, me, stream, &q1) != FEM_OK) return nullptr;
    int32_t state = 0;
    int64_t nrows = 0, nnz = 0;
    bool same = fem_plan_layouts(q1, 1, &state) == FEM_OK &&
                fem_plan_query(q1, FEM_OP_MASS, &nrows, &nnz) == FEM_OK && nrows == nq &&
                nnz == int64_t(ci.size()) && rp.size() == size_t(nq) + 1;
    if (same) {
        int32_t *drp = nullptr, *dci = nullptr;
        std::vector<int32_t> hrp(rp.size()), hci(ci.size());
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&drp), sizeof(int32_t) * hrp.size());
        if (e == hipSuccess)
            e = hipMalloc(reinterpret_cast<void **>(&dci), sizeof(int32_t) * std::max<size_t>(1, hci.size()));
        same = e == hipSuccess && fem_plan_pattern(q1, FEM_OP_MASS, drp, dci, stream) == FEM_OK &&
               hipMemcpyAsync(hrp.data(), drp, sizeof(int32_t) * hrp.size(), hipMemcpyDeviceToHost,
                              stream) == hipSuccess &&
               hipMemcpyAsync(hci.data(), dci, sizeof(int32_t) * hci.size(), hipMemcpyDeviceToHost,
                              stream) == hipSuccess &&
               hipStreamSynchronize(stream) == hipSuccess && hrp == rp && hci == ci;
        if (drp) (void)hipFree(drp);
        if (dci) (void)hipFree(dci);
    }
    if (!same) {
        fem_plan_destroy(q1);
        return nullptr;
    }
    return q1;
}

// Plan over an N x nme connectivity of sdim-simplices (sdim = d for P_k
// meshes, d - 1 for boundary facets) with d coordinates per node.
fem_status pk_build(int sdim, int d, int k, bool boundary, int64_t nq, int64_t nme,
                    const int32_t *me, hipStream_t stream, fem_pk_plan *out) {
    const int n = int(pk_nodes(sdim, k).size());
    if (int64_t(n) * nme >= (int64_t(1) << 31) || nq >= (int64_t(1) << 31) - 1)
        return FEM_ERR_OVERFLOW;
    std::vector<int32_t> hme(size_t(n) * nme);
    if (nme > 0) {
        hipError_t e = hipMemcpyAsync(hme.data(), me, sizeof(int32_t) * hme.size(),
                                      hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_status(e);
    }
    unsigned hc = std::thread::hardware_concurrency();
    PkHost H = build_pk_host(sdim, k, nq, nme, hme.data(),
                             int(std::max(1u, std::min(hc ? hc : 4u, 16u))));
    if (H.status == 2) return FEM_ERR_INDEX;
    if (H.status != 0) return FEM_ERR_OVERFLOW;
    std::vector<int32_t> gme(size_t(sdim + 1) * nme);   // the vertex rows
    std::copy(hme.begin(), hme.begin() + gme.size(), gme.begin());

    std::unique_ptr<fem_pk_plan_s> p(new fem_pk_plan_s());
    p->d = d;
    p->k = k;
    p->n = n;
    p->boundary = boundary;
    p->ntri = H.ntri;
    p->ebits = H.ebits;
    p->nq = nq;
    p->nme = nme;
    p->nnz = H.nnz;
    p->ntiles = H.ntiles;
    p->nitems = int64_t(H.item.size());
    p->max_tile_items = H.max_tile_items;
    (void)hipGetDevice(&p->device);
    fem_status st = pk_upload(&p->rp, H.rp);
    if (st == FEM_OK) st = pk_upload(&p->ci, H.ci);
    if (st == FEM_OK) st = pk_upload(&p->gme, gme);
    if (st == FEM_OK) st = pk_upload(&p->tile_item, H.tile_item);
    if (st == FEM_OK) st = pk_upload(&p->coff, H.coff);
    if (st == FEM_OK) st = pk_upload(&p->item, H.item);
    if (st == FEM_OK) st = pk_upload(&p->ctri, H.ctri);
    if (st == FEM_OK && !boundary) st = pk_upload(&p->vol, std::vector<double>(size_t(nme), 0.0));
    if (st == FEM_OK && boundary)
        st = pk_upload(&p->ev, std::vector<double>(size_t(nme) * H.ntri, 0.0));
    if (st == FEM_OK) st = pk_upload(&p->status, std::vector<int32_t>(1, 0));
    if (st != FEM_OK) {
        pk_free(p.get());
        return st;
    }
    if (!boundary && k == 1 && nme > 0) p->p1 = pk_p1_plan(d, nq, nme, me, H.rp, H.ci, stream);
    *out = p.release();
    return FEM_OK;
}

fem_status pk_sum(fem_pk_plan plan, double *values, hipStream_t stream) {
    const int chunk = pk_chunk(plan->ntri);
    const size_t lds = sizeof(double) * (size_t(plan->ntri) + size_t(chunk));
    // Large C (3D P5 and P6: 1596 and 3570 packed entries) takes the
    // pipelined kernel, the others the plain one (measured on 10^6 nodes:
    // P5 0.41 ms instead of 0.46, P6 0.50 instead of 0.61; P1-P4 were slower
    // pipelined, P1 0.40 instead of 0.30, P4 0.314 instead of 0.310)
    const bool pipe = plan->ntri >= 1024;
    const void *fn = pipe ? reinterpret_cast<const void *>(&k_pk_mass_pipe)
                          : reinterpret_cast<const void *>(&k_pk_mass);
    const int grid = pk_grid(fn, lds, plan->ntiles);
    if (pipe)
        hipLaunchKernelGGL(k_pk_mass_pipe, dim3(grid), dim3(kPkThreads), lds, stream,
                           plan->tile_item, plan->coff, plan->item, plan->ctri, plan->ntri,
                           plan->ebits, chunk, plan->boundary ? nullptr : plan->vol,
                           plan->boundary ? plan->ev : nullptr, plan->ntiles, plan->nnz, values);
    else
        hipLaunchKernelGGL(k_pk_mass, dim3(grid), dim3(kPkThreads), lds, stream, plan->tile_item,
                           plan->coff, plan->item, plan->ctri, plan->ntri, plan->ebits, chunk,
                           plan->boundary ? nullptr : plan->vol,
                           plan->boundary ? plan->ev : nullptr, plan->ntiles, plan->nnz, values);
    return hip_status(hipGetLastError());
}

}  // namespace

static fem_status fem_pk_symbolic_impl(int32_t d, int32_t k, int64_t nq, int64_t nme,
                                      const int32_t *me, hipStream_t stream, fem_pk_plan *out) {
    if (!out || (d != 2 && d != 3) || k < 1 || k > kPkMaxK || nq < 0 || nme < 0 ||
        (nme > 0 && !me))
        return FEM_ERR_ARG;
    return pk_build(d, d, k, false, nq, nme, me, stream, out);
}

extern "C" fem_status fem_pk_symbolic(int32_t d, int32_t k, int64_t nq, int64_t nme,
                                      const int32_t *me, hipStream_t stream, fem_pk_plan *out) {
    PhaseRange range("femasm: P_k symbolic");
    // host allocations (or threads) can fail for very large meshes: report
    // it, never throw across the ABI
    try {
        return fem_pk_symbolic_impl(d, k, nq, nme, me, stream, out);
    } catch (...) {
        return FEM_ERR_NOMEM;
    }
}

static fem_status fem_boundary_symbolic_impl(int32_t d, int64_t nq, int64_t nf,
                                            const int32_t *facets, hipStream_t stream,
                                            fem_pk_plan *out) {
    if (!out || (d != 2 && d != 3) || nq < 0 || nf < 0 || (nf > 0 && !facets)) return FEM_ERR_ARG;
    return pk_build(d - 1, d, 1, true, nq, nf, facets, stream, out);
}

extern "C" fem_status fem_boundary_symbolic(int32_t d, int64_t nq, int64_t nf,
                                            const int32_t *facets, hipStream_t stream,
                                            fem_pk_plan *out) {
    // host allocations (or threads) can fail for very large meshes: report
    // it, never throw across the ABI
    try {
        return fem_boundary_symbolic_impl(d, nq, nf, facets, stream, out);
    } catch (...) {
        return FEM_ERR_NOMEM;
    }
}

extern "C" fem_status fem_boundary_mass(fem_pk_plan plan, const double *q, const double *w,
                                        double *values, hipStream_t stream) {
    PhaseRange range("femasm: boundary mass");
    if (!plan || !plan->boundary || (plan->nme > 0 && !q) || (plan->nnz > 0 && !values))
        return FEM_ERR_ARG;
    if (plan->nnz == 0) return FEM_OK;
    const unsigned g = unsigned((plan->nme + 255) / 256);
    if (plan->d == 2) {
        if (w)
            hipLaunchKernelGGL((k_bnd_elem<2, true>), dim3(g), dim3(256), 0, stream, plan->gme,
                               plan->nme, q, plan->nq, w, plan->ctri, plan->ev, plan->status);
        else
            hipLaunchKernelGGL((k_bnd_elem<2, false>), dim3(g), dim3(256), 0, stream, plan->gme,
                               plan->nme, q, plan->nq, w, plan->ctri, plan->ev, plan->status);
    } else {
        if (w)
            hipLaunchKernelGGL((k_bnd_elem<3, true>), dim3(g), dim3(256), 0, stream, plan->gme,
                               plan->nme, q, plan->nq, w, plan->ctri, plan->ev, plan->status);
        else
            hipLaunchKernelGGL((k_bnd_elem<3, false>), dim3(g), dim3(256), 0, stream, plan->gme,
                               plan->nme, q, plan->nq, w, plan->ctri, plan->ev, plan->status);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_status(e);
    return pk_sum(plan, values, stream);
}

extern "C" fem_status fem_pk_query(fem_pk_plan plan, int64_t *nrows, int64_t *nnz, int32_t *ndfe) {
    if (!plan) return FEM_ERR_ARG;
    if (nrows) *nrows = plan->nq;
    if (nnz) *nnz = plan->nnz;
    if (ndfe) *ndfe = plan->n;
    return FEM_OK;
}

extern "C" fem_status fem_pk_pattern(fem_pk_plan plan, int32_t *row_ptr, int32_t *col_idx,
                                     hipStream_t stream) {
    if (!plan || !row_ptr || (plan->nnz > 0 && !col_idx)) return FEM_ERR_ARG;
    hipError_t e = hipMemcpyAsync(row_ptr, plan->rp, sizeof(int32_t) * (plan->nq + 1),
                                  hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess && plan->nnz > 0)
        e = hipMemcpyAsync(col_idx, plan->ci, sizeof(int32_t) * plan->nnz, hipMemcpyDeviceToDevice,
                           stream);
    return hip_status(e);
}

extern "C" fem_status fem_pk_mass(fem_pk_plan plan, const double *q, double *values,
                                  hipStream_t stream) {
    PhaseRange range("femasm: P_k mass");
    if (!plan || plan->boundary || (plan->nme > 0 && !q) || (plan->nnz > 0 && !values))
        return FEM_ERR_ARG;
    if (plan->nnz == 0) return FEM_OK;
    if (plan->p1)   // degree 1: the P1 mass kernels (same pattern, same summation order)
        return fem_assemble_numeric(plan->p1, FEM_OP_MASS, q, nullptr, 0.0, 0.0, values, stream);
    if (plan->nme > 0) {
        const unsigned g = unsigned((plan->nme + 255) / 256);
        if (plan->d == 2)
            hipLaunchKernelGGL(k_pk_vol<2>, dim3(g), dim3(256), 0, stream, plan->gme, plan->nme, q,
                               plan->nq, plan->vol, plan->status);
        else
            hipLaunchKernelGGL(k_pk_vol<3>, dim3(g), dim3(256), 0, stream, plan->gme, plan->nme, q,
                               plan->nq, plan->vol, plan->status);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_status(e);
    }
    return pk_sum(plan, values, stream);
}

extern "C" fem_status fem_pk_sync_status(fem_pk_plan plan, hipStream_t stream) {
    if (!plan) return FEM_ERR_ARG;
    // degree 1: the P1 plan's status word first (read and cleared)
    const fem_status s1 = plan->p1 ? fem_plan_sync_status(plan->p1, stream) : FEM_OK;
    if (s1 != FEM_OK && s1 != FEM_ERR_DEGENERATE) return s1;
    int32_t word = 0;
    hipError_t e = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = hipMemcpy(&word, plan->status, sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && word != 0) {
        const int32_t zero = 0;
        e = hipMemcpy(plan->status, &zero, sizeof(int32_t), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return hip_status(e);
    return word || s1 == FEM_ERR_DEGENERATE ? FEM_ERR_DEGENERATE : FEM_OK;
}

extern "C" void fem_pk_destroy(fem_pk_plan plan) {
    if (!plan) return;
    pk_free(plan);
    delete plan;
}
