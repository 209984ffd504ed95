// Block kernel for the scalar operators (mass, weighted mass, stiffness).
//
// One 128-thread workgroup per vertex block (see blocks_host.h):
//   1. stage the coordinates (and weights) of the block's touched vertices in
//      LDS with batched loads, zero the LDS accumulator of the block's rows;
//   2. for each chunk of 128 block elements: every thread computes one
//      element's geometry once and stores its element matrix in LDS (the
//      next chunk's vertex ids are already being loaded);
//   3. every thread that owns a row walks that row's incidences falling in the
//      chunk (ascending element number; the records were staged in LDS) and
//      adds the element-matrix row into its private accumulator segment;
//   4. the accumulators are written to the rows' CSR value ranges.
// A row is summed by one thread in ascending caller element number, as in the
// row-gather kernel, and element values are computed with the same routines,
// so both kernels produce the same bits.
#include <algorithm>
#include <cstdlib>
#include <string>
#include <thread>

#include "blocks_host.h"
#include "element.h"
#include "femasm_impl.h"
#include "rowgather.h"

#pragma clang fp contract(off)

namespace femasm {

// Threads per workgroup = rows per block (at most) = block elements per
// element phase; a kernel template parameter (64 or 128).
constexpr int kMaxWG = 128;

struct BlockView {
    const int32_t *rp;
    const int32_t *rows;
    const int32_t *row_ptr;
    const int32_t *acc_off;
    const int32_t *nacc;
    const int32_t *nodes;
    const int32_t *node_ptr;
    const uint2 *elem;
    const int32_t *elem_ptr;
    const uint32_t *rec;
    const int64_t *rec_ptr;
    const int32_t *maxdeg;
    const double *q;
    const double *w;
    double *values;
    int64_t nq;
    int32_t max_nodes;
    uint32_t off_w, off_ev, off_acc, off_rowoff, off_rowg, off_rowof, off_rec;
};

// Per-element values kept in LDS for the row phase: the full (d+1)x(d+1)
// stiffness matrix (a row is then contiguous), |det|/(d+2)! for the mass,
// and |det|/(d+3)!, w^s and the d+1 vertex weights for the weighted mass.
// Each element's slot is padded to an odd number of doubles so that threads
// with consecutive element indices fall on different LDS banks.
template <int D, int OP>
struct BlockOp {
    static constexpr int NL = D + 1;
    static constexpr int NV0 = OP == FEM_OP_MASS ? 1 : (OP == FEM_OP_MASS_W ? NL + 2 : NL * NL);
    static constexpr int NV = NV0 | 1;
};

template <int D, int OP, int kWG>
__global__ void __launch_bounds__(kWG) k_block(BlockView bv, int32_t *status) {
    constexpr int kChunk = kWG;
    constexpr int NL = D + 1;
    constexpr int NV = BlockOp<D, OP>::NV;
    extern __shared__ __align__(16) unsigned char smem[];
    double *crd = reinterpret_cast<double *>(smem);
    double *wv = reinterpret_cast<double *>(smem + bv.off_w);
    double *ev = reinterpret_cast<double *>(smem + bv.off_ev);
    double *acc = reinterpret_cast<double *>(smem + bv.off_acc);
    int32_t *row_off = reinterpret_cast<int32_t *>(smem + bv.off_rowoff);
    int32_t *row_g = reinterpret_cast<int32_t *>(smem + bv.off_rowg);
    uint8_t *rowof = smem + bv.off_rowof;
    uint32_t *recs = reinterpret_cast<uint32_t *>(smem + bv.off_rec);

    const int b = int(xcd_tile(blockIdx.x, gridDim.x));
    const int tid = threadIdx.x;
    const int r0 = bv.row_ptr[b], nr = bv.row_ptr[b + 1] - r0;
    const int n0 = bv.node_ptr[b], nn = bv.node_ptr[b + 1] - n0;
    const int e0 = bv.elem_ptr[b], ne = bv.elem_ptr[b + 1] - e0;
    const uint32_t *recg = bv.rec + bv.rec_ptr[b];
    const int nrec = bv.maxdeg[b] * nr;
    const int nacc = bv.nacc[b];
    const int64_t nq = bv.nq;
    const int MN = bv.max_nodes;

    // ---- global loads of the prologue, issued together: the block's
    // incidence records, the first chunk's element vertices, the row's CSR
    // range, and the touched-vertex ids
    for (int base = 0; base < nrec; base += 8 * kWG) {
        uint32_t rr[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = base + u * kWG + tid;
            rr[u] = i < nrec ? recg[i] : kRecPad;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = base + u * kWG + tid;
            if (i < nrec) recs[i] = rr[u];
        }
    }
    uint2 vnext = tid < ne ? bv.elem[e0 + tid] : make_uint2(0u, 0u);
    int myoff = 0, mylen = 0, g = 0;
    if (tid < nr) {
        const int row = bv.rows[r0 + tid];
        myoff = bv.acc_off[r0 + tid];
        g = bv.rp[row];
        mylen = bv.rp[row + 1] - g;
    }
    for (int base = 0; base < nn; base += 4 * kWG) {
        int64_t gi[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int n = base + u * kWG + tid;
            gi[u] = n < nn ? bv.nodes[n0 + n] : 0;
        }
        double c[4][D], wq[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (base + u * kWG + tid < nn) {
#pragma unroll
                for (int x = 0; x < D; ++x) c[u][x] = bv.q[x * nq + gi[u]];
                if constexpr (OP == FEM_OP_MASS_W) wq[u] = bv.w[gi[u]];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int n = base + u * kWG + tid;
            if (n < nn) {
#pragma unroll
                for (int x = 0; x < D; ++x) crd[x * MN + n] = c[u][x];
                if constexpr (OP == FEM_OP_MASS_W) wv[n] = wq[u];
            }
        }
    }
    if (tid < nr) {
        row_off[tid] = myoff;
        row_g[tid] = g;
        for (int k = 0; k < mylen; ++k) {
            acc[myoff + k] = 0.0;
            rowof[myoff + k] = uint8_t(tid);
        }
    }
    double *myacc = acc + myoff;
    const uint32_t *myrec = recs + tid;   // record t of this row at myrec[t * nr]
    const int maxdeg = tid < nr ? nrec / nr : 0;
    int t = 0;  // records consumed so far
    uint32_t cur = kRecPad;
    int bad = 0;

    for (int c0 = 0; c0 < ne; c0 += kChunk) {
        __syncthreads();  // crd/acc ready (first chunk); ev free (later chunks)
        // ---- element phase: one element per thread
        const uint2 vv = vnext;
        {
            const int en = c0 + kChunk + tid;
            if (en < ne) vnext = bv.elem[e0 + en];
        }
        if (c0 + tid < ne) {
            const int v[4] = {int(vv.x & 0xffffu), int(vv.x >> 16), int(vv.y & 0xffffu),
                              int(vv.y >> 16)};
            double P[NL][D];
#pragma unroll
            for (int a = 0; a < NL; ++a)
#pragma unroll
                for (int x = 0; x < D; ++x) P[a][x] = crd[x * MN + v[a]];
            double *out = ev + tid * NV;
            if constexpr (OP == FEM_OP_MASS || OP == FEM_OP_MASS_W) {
                const double det = elem_det(P);
                if (det == 0.0) bad = 1;
                if constexpr (OP == FEM_OP_MASS) {
                    out[0] = det == 0.0 ? 0.0 : fabs(det) / Fact<D>::mass_den;
                } else {
                    double wl[NL];
#pragma unroll
                    for (int a = 0; a < NL; ++a) wl[a] = wv[v[a]];
                    double ws = wl[0];
#pragma unroll
                    for (int a = 1; a < NL; ++a) ws += wl[a];
                    out[0] = det == 0.0 ? 0.0 : fabs(det) / Fact<D>::massw_den;
                    out[1] = ws;
#pragma unroll
                    for (int a = 0; a < NL; ++a) out[2 + a] = wl[a];
                }
            } else {
                Elem<D> E;
                elem_geometry(P, E);
                const bool deg = E.det == 0.0;
                if (deg) bad = 1;
                const double inv = deg ? 0.0 : 1.0 / (Fact<D>::dfact * fabs(E.det));
#pragma unroll
                for (int a = 0; a < NL; ++a)
#pragma unroll
                    for (int c = a; c < NL; ++c) {
                        const double val = deg ? 0.0 : cdot<D>(E.c[a], E.c[c]) * inv;
                        out[a * NL + c] = val;
                        out[c * NL + a] = val;
                    }
            }
        }
        __syncthreads();
        // ---- row phase: this row's incidences inside the chunk, ascending;
        // the next record is read ahead of the current accumulation
        const uint32_t cend = uint32_t(c0 + kChunk);
        if (c0 == 0) cur = t < maxdeg ? myrec[0] : kRecPad;
        while (cur != kRecPad && (cur & 1023u) < cend) {
            const uint32_t rec = cur;
            ++t;
            cur = t < maxdeg ? myrec[t * nr] : kRecPad;
            const int le = int(rec & 1023u) - c0;
            const int al = int((rec >> 10) & 3u);
            int pos[NL];
#pragma unroll
            for (int c = 0; c < NL; ++c) pos[c] = int((rec >> (12 + 5 * c)) & 31u);
            double val[NL];
            if constexpr (OP == FEM_OP_MASS) {
                const double k = ev[le];
#pragma unroll
                for (int c = 0; c < NL; ++c) val[c] = (c == al) ? 2.0 * k : k;
            } else if constexpr (OP == FEM_OP_MASS_W) {
                const double *E = ev + le * NV;
                const double k = E[0], ws = E[1];
                double wa = E[2];
#pragma unroll
                for (int c = 1; c < NL; ++c) wa = (c == al) ? E[2 + c] : wa;
#pragma unroll
                for (int c = 0; c < NL; ++c) {
                    const double f = (c == al) ? 2.0 * k : k;
                    val[c] = f * (ws + (wa + E[2 + c]));
                }
            } else {
                const double *E = ev + le * NV + al * NL;
#pragma unroll
                for (int c = 0; c < NL; ++c) val[c] = E[c];
            }
            double old[NL];
#pragma unroll
            for (int c = 0; c < NL; ++c) old[c] = myacc[pos[c]];
#pragma unroll
            for (int c = 0; c < NL; ++c) myacc[pos[c]] = old[c] + val[c];
        }
    }
    __syncthreads();
    // ---- write the block's rows
    for (int s = tid; s < nacc; s += kWG) {
        const int r = rowof[s];
        bv.values[int64_t(row_g[r]) + (s - row_off[r])] = acc[s];
    }
    const unsigned long long any = __ballot(bad != 0);
    if (any != 0ull && (threadIdx.x & 63) == __ffsll((long long)any) - 1) atomicOr(status, bad);
}


template <class T>
static fem_status up(T **dst, const std::vector<T> &src) {
    *dst = nullptr;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(dst), sizeof(T) * std::max<size_t>(1, src.size()));
    if (e == hipSuccess && !src.empty())
        e = copy_sync(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
    return hip_status(e);
}

void free_blocks(BlockPlan *b) {
    void *ptrs[] = {b->rows, b->row_ptr, b->acc_off, b->nacc, b->nodes, b->node_ptr,
                    b->elem, b->elem_ptr, b->rec, b->rec_ptr, b->maxdeg};
    for (void *x : ptrs)
        if (x) (void)hipFree(x);
    *b = BlockPlan();
}

static fem_status upload_layout(BlockPlan &B, const BlockHost &H, const int32_t *rp,
                                bool with_records) {
    std::vector<int32_t> acc_off(H.rows.size()), nacc(H.nb);
    for (int b = 0; b < H.nb; ++b) {
        int32_t o = 0;
        for (int r = H.row_ptr[b]; r < H.row_ptr[b + 1]; ++r) {
            acc_off[r] = o;
            o += rp[H.rows[r] + 1] - rp[H.rows[r]];
        }
        nacc[b] = o;
    }
    fem_status st = FEM_OK;
    if (st == FEM_OK) st = up(&B.rows, H.rows);
    if (st == FEM_OK) st = up(&B.row_ptr, H.row_ptr);
    if (st == FEM_OK) st = up(&B.nodes, H.nodes);
    if (st == FEM_OK) st = up(&B.node_ptr, H.node_ptr);
    if (st == FEM_OK) st = up(&B.elem, H.elem);
    if (st == FEM_OK) st = up(&B.elem_ptr, H.elem_ptr);
    if (st == FEM_OK) st = up(&B.acc_off, acc_off);
    if (st == FEM_OK) st = up(&B.nacc, nacc);
    if (with_records) {
        if (st == FEM_OK) st = up(&B.rec, H.rec);
        if (st == FEM_OK) st = up(&B.rec_ptr, H.rec_ptr);
        if (st == FEM_OK) st = up(&B.maxdeg, H.maxdeg);
    }
    if (st != FEM_OK) {
        free_blocks(&B);
        return st;
    }
    B.nb = H.nb;
    B.max_rows = H.max_rows;
    B.max_nodes = H.max_nodes;
    B.max_elems = H.max_elems;
    B.max_nacc = H.max_nacc;
    // two waves per workgroup measured faster than one at 64 rows per block;
    // FEMASM_BLOCK_WG=64 selects single-wave workgroups when the rows fit
    B.wg = 128;
    if (const char *env = getenv("FEMASM_BLOCK_WG"))
        if (atoi(env) == 64 && H.max_rows <= 64) B.wg = 64;
    B.max_rec = 0;
    for (int b = 0; b < H.nb; ++b)
        B.max_rec = std::max<int64_t>(B.max_rec, H.rec_ptr[b + 1] - H.rec_ptr[b]);
    B.ok = true;
    return FEM_OK;
}

fem_status upload_blocks(fem_plan_data *p, int d, int64_t nq, int64_t nme, const int32_t *me,
                         const int32_t *rp, const int32_t *ci, const int64_t *ip,
                         const int32_t *inc_k) {
    // record layout (scalar operators): FEMASM_BLOCK_ROWS (16..128) rows
    // per block when set, else 64
    int R = 64;
    if (const char *env = getenv("FEMASM_BLOCK_ROWS")) R = std::max(16, std::min(kMaxWG, atoi(env)));
    // pair layouts: FEMASM_PAIR_ROWS / FEMASM_ELAS_ROWS rows per block when
    // set (16..128), else in 3D 64 for both (measured on the 128^3 cube:
    // 64 rows 8 % faster than 56 for stiffness, 3 % faster than 48 for
    // elasticity, whose blocks the element cap then ends first; larger
    // blocks no faster, and beyond 72 rows the lists outgrow the LDS of two
    // workgroups per compute unit), in 2D 128 for both (2D rows are short: the largest blocks the row
    // field allows cut element replication; measured on the 2048^2 square:
    // 128 rows 40 % faster than 56 for the scalar operators, 20 % faster
    // than 64 for elasticity); FEMASM_PAIR_SLOTS / FEMASM_ELAS_SLOTS (1, 2
    // or 4) tasks of 64 pairs per wavefront, else 2 (measured on the 128^3
    // cube).
    // A block also stops at 512 * slots CSR entries.
    auto env_int = [](const char *name, int dflt, int lo, int hi) {
        const char *e = getenv(name);
        return e ? std::max(lo, std::min(hi, atoi(e))) : dflt;
    };
    auto slots_of = [](int v) { return v >= 4 ? 4 : (v <= 1 ? 1 : 2); };
    const int Rs = env_int("FEMASM_PAIR_ROWS", d == 3 ? 64 : 128, 16, 128);
    const int Ss = slots_of(env_int("FEMASM_PAIR_SLOTS", 2, 1, 4));
    const int Re = env_int("FEMASM_ELAS_ROWS", d == 3 ? 64 : 128, 16, 128);
    const int Se = slots_of(env_int("FEMASM_ELAS_SLOTS", 2, 1, 4));
    // the two pair layouts are independent: built concurrently, each thread
    // on the plan's device.  The record-block layout serves the scalar
    // operators only when the scalar pair layout cannot be built (or when
    // FEMASM_BLOCK_LAYOUT=1 asks for it, for comparisons of the kernel
    // families), so it is built only then.
    fem_status sb = FEM_OK, ss = FEM_OK, sv = FEM_OK;
    const int dev = p->device;
    run_threads(2, [&](int t) {
        (void)hipSetDevice(dev);
        if (t == 0)
            sv = upload_pairs(p->pvec, Re, Se, false, d, nq, nme, me, rp, ci, ip, inc_k);
        else
            ss = upload_pairs(p->pscal, Rs, Ss, true, d, nq, nme, me, rp, ci, ip, inc_k);
    });
    if (ss == FEM_OK && (!p->pscal.ok || env_int("FEMASM_BLOCK_LAYOUT", 0, 0, 1) == 1)) {
        BlockHost H = build_block_host(d, nq, nme, me, rp, ci, ip, inc_k, R, 16);
        if (H.ok && H.nb > 0) sb = upload_layout(p->blk, H, rp, true);
    }
    fem_status st = sb != FEM_OK ? sb : (ss != FEM_OK ? ss : sv);
    if (st != FEM_OK) {
        free_blocks(&p->blk);
        free_pairs(&p->pscal);
        free_pairs(&p->pvec);
    }
    return st;
}

static uint32_t align16(size_t x) { return uint32_t((x + 15) & ~size_t(15)); }

template <int D, int OP, int kWG>
static hipError_t launch_block_w(const fem_plan_data *p, const double *q, const double *w,
                                 double *values, hipStream_t s) {
    const BlockPlan &B = p->blk;
    BlockView bv;
    bv.rp = p->rp;
    bv.rows = B.rows;
    bv.row_ptr = B.row_ptr;
    bv.acc_off = B.acc_off;
    bv.nacc = B.nacc;
    bv.nodes = B.nodes;
    bv.node_ptr = B.node_ptr;
    bv.elem = reinterpret_cast<const uint2 *>(B.elem);
    bv.elem_ptr = B.elem_ptr;
    bv.rec = B.rec;
    bv.rec_ptr = B.rec_ptr;
    bv.maxdeg = B.maxdeg;
    bv.q = q;
    bv.w = w;
    bv.values = values;
    bv.nq = p->nq;
    bv.max_nodes = B.max_nodes;
    size_t o = size_t(D) * B.max_nodes * sizeof(double);
    bv.off_w = align16(o);
    o = bv.off_w + (OP == FEM_OP_MASS_W ? B.max_nodes * sizeof(double) : 0);
    bv.off_ev = align16(o);
    o = bv.off_ev + size_t(kWG) * BlockOp<D, OP>::NV * sizeof(double);
    bv.off_acc = align16(o);
    o = bv.off_acc + size_t(B.max_nacc) * sizeof(double);
    bv.off_rowoff = align16(o);
    o = bv.off_rowoff + size_t(B.max_rows) * sizeof(int32_t);
    bv.off_rowg = align16(o);
    o = bv.off_rowg + size_t(B.max_rows) * sizeof(int32_t);
    bv.off_rowof = align16(o);
    o = bv.off_rowof + size_t(B.max_nacc);
    bv.off_rec = align16(o);
    o = bv.off_rec + size_t(B.max_rec) * sizeof(uint32_t);
    const size_t lds = align16(o);
    static thread_local bool attr_set[2][4] = {};
    if (!attr_set[D - 2][OP]) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_block<D, OP, kWG>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        attr_set[D - 2][OP] = true;
    }
    hipLaunchKernelGGL((k_block<D, OP, kWG>), dim3(unsigned(B.nb)), dim3(kWG), lds, s, bv,
                       p->status);
    return hipGetLastError();
}

template <int D, int OP>
static hipError_t launch_block_t(const fem_plan_data *p, const double *q, const double *w,
                                 double *values, hipStream_t s) {
    if (p->blk.wg == 64) return launch_block_w<D, OP, 64>(p, q, w, values, s);
    return launch_block_w<D, OP, 128>(p, q, w, values, s);
}

bool launch_block(const fem_plan_data *p, int op, const double *q, const double *w,
                  double *values, hipStream_t s, hipError_t *err) {
    if (!layouts_ready(p) || !p->blk.ok || op == FEM_OP_ELAS) return false;
    hipError_t e;
    if (p->d == 2) {
        switch (op) {
            case FEM_OP_MASS: e = launch_block_t<2, FEM_OP_MASS>(p, q, w, values, s); break;
            case FEM_OP_MASS_W: e = launch_block_t<2, FEM_OP_MASS_W>(p, q, w, values, s); break;
            default: e = launch_block_t<2, FEM_OP_STIFF>(p, q, w, values, s); break;
        }
    } else {
        switch (op) {
            case FEM_OP_MASS: e = launch_block_t<3, FEM_OP_MASS>(p, q, w, values, s); break;
            case FEM_OP_MASS_W: e = launch_block_t<3, FEM_OP_MASS_W>(p, q, w, values, s); break;
            default: e = launch_block_t<3, FEM_OP_STIFF>(p, q, w, values, s); break;
        }
    }
    *err = e;
    return true;
}

}  // namespace femasm
