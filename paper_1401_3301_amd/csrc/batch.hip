// Batched assembly: many independent meshes, one persistent launch.
//
// The batch owns one plan per mesh and a device work list of (mesh, row
// tile) items per dof multiplicity (scalar / elasticity), ordered by
// decreasing work (longest-processing-time first).  A fixed grid of
// workgroups walks the list cyclically (workgroup g takes items g, g+G,
// ...), so the launch needs no counters or resets and can be captured in a
// hipGraph and replayed.  Each item runs the same row-gather tile routine as
// the single-mesh kernel, so batched values equal per-mesh values bit for bit.
#include <algorithm>
#include <atomic>
#include <memory>
#include <numeric>

#include "femasm_impl.h"
#include "host_threads.h"
#include "rowgather.h"

namespace femasm {

template <int OP>
__global__ void __launch_bounds__(256)
    k_batch(const BatchMesh *__restrict__ meshes, const BatchItem *__restrict__ items,
            int64_t nitems, int vec, const double *__restrict__ q_cat,
            const double *__restrict__ w_cat, double lam, double mu,
            double *__restrict__ values_cat, int32_t *status) {
    extern __shared__ double acc[];
    int bad = 0;
    for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const BatchItem item = items[it];
        const BatchMesh bm = meshes[item.mesh];
        MeshView mv;
        mv.rp = bm.rp;
        mv.inc_ptr = bm.inc_ptr;
        mv.inc_elem = bm.inc_elem;
        mv.inc_off = bm.inc_off;
        mv.pme = bm.pme;
        mv.q = q_cat + bm.q_off;
        mv.w = w_cat ? w_cat + bm.w_off : nullptr;
        mv.values = values_cat + (vec ? bm.val_off[1] : bm.val_off[0]);
        mv.nq = bm.nq;
        const int64_t r0 = item.row0;
        const int64_t r1 = r0 + item.nrows;
        if (bm.d == 2)
            assemble_row_tile<2, OP>(mv, r0, r1, acc, lam, mu, bad);
        else
            assemble_row_tile<3, OP>(mv, r0, r1, acc, lam, mu, bad);
        __syncthreads();
    }
    const unsigned long long any = __ballot(bad != 0);
    if (any != 0ull && (threadIdx.x & 63) == __ffsll((long long)any) - 1) atomicOr(status, bad);
}

fem_status launch_batch(int op, const BatchMesh *meshes, const BatchItem *items, int64_t nitems,
                        int rows_per_wg, size_t lds_bytes, int grid, int, int,
                        const double *q_cat, const double *w_cat, double lam, double mu,
                        double *values_cat, int32_t *status, hipStream_t stream) {
    if (nitems == 0) return FEM_OK;
    const int vec = op == FEM_OP_ELAS ? 1 : 0;
    const dim3 g(unsigned(std::max<int64_t>(1, std::min<int64_t>(grid, nitems))));
    const dim3 b(rows_per_wg);
    switch (op) {
        case FEM_OP_MASS:
            hipLaunchKernelGGL(k_batch<FEM_OP_MASS>, g, b, lds_bytes, stream, meshes, items, nitems,
                               vec, q_cat, w_cat, lam, mu, values_cat, status);
            break;
        case FEM_OP_MASS_W:
            hipLaunchKernelGGL(k_batch<FEM_OP_MASS_W>, g, b, lds_bytes, stream, meshes, items,
                               nitems, vec, q_cat, w_cat, lam, mu, values_cat, status);
            break;
        case FEM_OP_STIFF:
            hipLaunchKernelGGL(k_batch<FEM_OP_STIFF>, g, b, lds_bytes, stream, meshes, items,
                               nitems, vec, q_cat, w_cat, lam, mu, values_cat, status);
            break;
        default:
            hipLaunchKernelGGL(k_batch<FEM_OP_ELAS>, g, b, lds_bytes, stream, meshes, items, nitems,
                               vec, q_cat, w_cat, lam, mu, values_cat, status);
            break;
    }
    return hip_status(hipGetLastError());
}

}  // namespace femasm

using namespace femasm;

struct fem_batch_s {
    std::vector<fem_plan> plans;
    std::vector<int64_t> q_off, w_off, row_off[2], nnz_off[2];
    BatchMesh *d_meshes = nullptr;
    BatchItem *d_items[2] = {nullptr, nullptr};
    int64_t nitems[2] = {0, 0};
    size_t lds[2] = {0, 0};
    int block_threads = 256;
    int wg_per_cu = 2;
    int cus = 256;
    int32_t *status = nullptr;
    bool has_d[4] = {false, false, false, false};
    // batched pair layouts [scalar / elasticity][d] and the kernel in use
    PairPlan pairs[2][4];
    int kernel = FEM_BATCH_PAIR;
};

static void free_batch(fem_batch_s *b) {
    for (fem_plan p : b->plans) fem_plan_destroy(p);
    b->plans.clear();
    if (b->d_meshes) (void)hipFree(b->d_meshes);
    for (int v = 0; v < 2; ++v)
        if (b->d_items[v]) (void)hipFree(b->d_items[v]);
    if (b->status) (void)hipFree(b->status);
    b->d_meshes = nullptr;
    b->d_items[0] = b->d_items[1] = nullptr;
    b->status = nullptr;
    for (auto &row : b->pairs)
        for (PairPlan &P : row) free_pairs(&P);
}

// One pair layout per (scalar / elasticity, d) over all meshes of that d
// (vec_only >= 0: only that kind).
static fem_status build_pair_layouts(fem_batch_s *B, int vec_only = -1) {
    for (int vec = 0; vec < 2; ++vec)
        for (int d = 2; d <= 3; ++d) {
            if (vec_only >= 0 && vec != vec_only) continue;
            free_pairs(&B->pairs[vec][d]);
            std::vector<const PairPlan *> parts;
            std::vector<int64_t> qo, wo, vo, nq;
            for (size_t m = 0; m < B->plans.size(); ++m) {
                const fem_plan p = B->plans[m];
                if (p->d != d || p->nq == 0) continue;
                parts.push_back(vec ? &p->pvec : &p->pscal);
                qo.push_back(B->q_off[m]);
                wo.push_back(B->w_off[m]);
                vo.push_back(B->nnz_off[vec][m]);
                nq.push_back(p->nq);
            }
            fem_status st = concat_pairs(B->pairs[vec][d], parts, qo, wo, vo, nq);
            if (st != FEM_OK) return st;
        }
    return FEM_OK;
}

// (Re)builds the two work lists for the current block size.  Each mesh is
// cut into tiles of R rows, R the largest of block_threads, /2, /4, ... (at
// least 16) whose LDS tile fits the cap.
static fem_status build_items(fem_batch_s *B) {
    for (int vec = 0; vec < 2; ++vec) {
        std::vector<BatchItem> items;
        std::vector<int64_t> work;
        size_t worst = 8;
        for (size_t m = 0; m < B->plans.size(); ++m) {
            const fem_plan p = B->plans[m];
            const int M = vec ? p->d : 1;
            const int64_t nrows = int64_t(M) * p->nq;
            auto vstart = [&](int64_t r) -> int64_t {
                int64_t i = r / M, l = r - i * M;
                int64_t s = int64_t(M) * M * p->h_rp[i];
                if (l) s += l * M * int64_t(p->h_rp[i + 1] - p->h_rp[i]);
                return s;
            };
            // elasticity tiles hold whole vertices: R a multiple of M
            int R = B->block_threads;
            for (;; R /= 2) {
                const int Rm = R / M * M;
                size_t need = 0;
                for (int64_t r0 = 0; r0 < nrows; r0 += Rm) {
                    const int64_t r1 = std::min(nrows, r0 + Rm);
                    need = std::max(need, tile_lds_bytes(M, vstart(r1) - vstart(r0), r1 - r0));
                }
                if (need <= kLdsCap) break;
                if (R <= 16) return FEM_ERR_OVERFLOW;
            }
            R = R / M * M;
            for (int64_t r0 = 0; r0 < nrows; r0 += R) {
                const int64_t r1 = std::min(nrows, r0 + R);
                const int64_t span = vstart(r1) - vstart(r0);
                worst = std::max(worst, tile_lds_bytes(M, span, r1 - r0));
                items.push_back(BatchItem{int32_t(m), int32_t(r1 - r0), r0});
                work.push_back(span * (p->d + 1));
            }
        }
        std::vector<size_t> order(items.size());
        std::iota(order.begin(), order.end(), size_t(0));
        std::stable_sort(order.begin(), order.end(),
                         [&](size_t a, size_t b) { return work[a] > work[b]; });
        std::vector<BatchItem> sorted(items.size());
        for (size_t k = 0; k < order.size(); ++k) sorted[k] = items[order[k]];
        if (B->d_items[vec]) (void)hipFree(B->d_items[vec]);
        B->d_items[vec] = nullptr;
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&B->d_items[vec]),
                                 sizeof(BatchItem) * std::max<size_t>(1, sorted.size()));
        if (e == hipSuccess && !sorted.empty())
            e = hipMemcpy(B->d_items[vec], sorted.data(), sizeof(BatchItem) * sorted.size(),
                          hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_status(e);
        B->nitems[vec] = int64_t(sorted.size());
        B->lds[vec] = worst;
    }
    return FEM_OK;
}

static fem_status fem_batch_create_impl(int32_t nmesh, const int32_t *d, const int64_t *nq,
                                       const int64_t *nme, const int32_t *const *me,
                                       hipStream_t stream, fem_batch *out) {
    if (!out || nmesh < 1 || !d || !nq || !nme || !me) return FEM_ERR_ARG;
    std::unique_ptr<fem_batch_s> B(new fem_batch_s());
    for (int v = 0; v < 2; ++v) {
        B->row_off[v].assign(nmesh + 1, 0);
        B->nnz_off[v].assign(nmesh + 1, 0);
    }
    B->q_off.assign(nmesh + 1, 0);
    B->w_off.assign(nmesh + 1, 0);
    std::vector<BatchMesh> hm(nmesh);
    // the meshes' plans are independent: a few are built at a time (a small
    // mesh leaves a plan build's own threads idle), each on the caller's
    // device; the batch takes them in mesh order, so it does not depend on
    // the workers
    std::vector<fem_plan> plans(nmesh, nullptr);
    std::vector<fem_status> pst(nmesh, FEM_OK);
    int dev0 = 0;
    (void)hipGetDevice(&dev0);
    std::atomic<int32_t> next{0};
    run_threads(std::min<int32_t>(8, nmesh), [&](int) {
        (void)hipSetDevice(dev0);
        for (int32_t m; (m = next.fetch_add(1)) < nmesh;)
        {
            pst[m] = fem_assemble_symbolic(d[m], nq[m], nme[m], me[m], stream, &plans[m]);
            // the batch concatenates the meshes' block layouts
            if (pst[m] == FEM_OK) wait_layouts(plans[m]);
        }
    });
    for (int32_t m = 0; m < nmesh; ++m)
        if (pst[m] != FEM_OK) {
            for (fem_plan x : plans) fem_plan_destroy(x);
            free_batch(B.get());
            return pst[m];
        }
    for (int32_t m = 0; m < nmesh; ++m) {
        fem_plan p = plans[m];
        B->plans.push_back(p);
        B->has_d[p->d] = true;
        B->q_off[m + 1] = B->q_off[m] + int64_t(p->d) * p->nq;
        B->w_off[m + 1] = B->w_off[m] + p->nq;
        B->row_off[0][m + 1] = B->row_off[0][m] + p->nq;
        B->row_off[1][m + 1] = B->row_off[1][m] + int64_t(p->d) * p->nq;
        B->nnz_off[0][m + 1] = B->nnz_off[0][m] + p->nnz;
        B->nnz_off[1][m + 1] = B->nnz_off[1][m] + int64_t(p->d) * p->d * p->nnz;
        BatchMesh &bm = hm[m];
        bm.rp = p->rp;
        bm.inc_ptr = p->inc_ptr;
        bm.inc_elem = p->inc_elem;
        bm.inc_off = p->inc_off;
        bm.pme = p->pme;
        bm.nq = p->nq;
        bm.q_off = B->q_off[m];
        bm.w_off = B->w_off[m];
        bm.val_off[0] = B->nnz_off[0][m];
        bm.val_off[1] = B->nnz_off[1][m];
        bm.d = p->d;
        bm.pad = 0;
    }
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&B->d_meshes), sizeof(BatchMesh) * nmesh);
    if (e == hipSuccess)
        e = hipMemcpy(B->d_meshes, hm.data(), sizeof(BatchMesh) * nmesh, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&B->status), sizeof(int32_t));
    if (e == hipSuccess) e = hipMemset(B->status, 0, sizeof(int32_t));
    int dev = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&B->cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) {
        free_batch(B.get());
        return hip_status(e);
    }
    fem_status st = build_items(B.get());
    if (st == FEM_OK) st = build_pair_layouts(B.get());
    if (st != FEM_OK) {
        free_batch(B.get());
        return st;
    }
    *out = B.release();
    return FEM_OK;
}

extern "C" fem_status fem_batch_create(int32_t nmesh, const int32_t *d, const int64_t *nq,
                                       const int64_t *nme, const int32_t *const *me,
                                       hipStream_t stream, fem_batch *out) {
    PhaseRange range("femasm: batch create");
    // host allocations (or threads) can fail for very large batches: report
    // it, never throw across the ABI
    try {
        return fem_batch_create_impl(nmesh, d, nq, nme, me, stream, out);
    } catch (...) {
        return FEM_ERR_NOMEM;
    }
}

extern "C" fem_status fem_batch_set_kernel(fem_batch batch, int32_t kernel) {
    if (!batch || (kernel != FEM_BATCH_ROWGATHER && kernel != FEM_BATCH_PAIR &&
                   kernel != FEM_BATCH_PAIR_SPLIT))
        return FEM_ERR_ARG;
    batch->kernel = kernel;
    return FEM_OK;
}

extern "C" fem_status fem_batch_offsets(fem_batch batch, int32_t op, int64_t *q_off,
                                        int64_t *w_off, int64_t *row_off, int64_t *nnz_off) {
    if (!batch || op < FEM_OP_MASS || op > FEM_OP_ELAS) return FEM_ERR_ARG;
    const int vec = op == FEM_OP_ELAS ? 1 : 0;
    const size_t n = batch->plans.size() + 1;
    if (q_off) std::copy(batch->q_off.begin(), batch->q_off.end(), q_off);
    if (w_off) std::copy(batch->w_off.begin(), batch->w_off.end(), w_off);
    if (row_off) std::copy(batch->row_off[vec].begin(), batch->row_off[vec].begin() + n, row_off);
    if (nnz_off) std::copy(batch->nnz_off[vec].begin(), batch->nnz_off[vec].begin() + n, nnz_off);
    return FEM_OK;
}

extern "C" fem_status fem_batch_plan(fem_batch batch, int32_t index, fem_plan *plan) {
    if (!batch || !plan || index < 0 || size_t(index) >= batch->plans.size()) return FEM_ERR_ARG;
    *plan = batch->plans[index];
    return FEM_OK;
}

extern "C" fem_status fem_batch_set_params(fem_batch batch, int32_t block_threads,
                                           int32_t wg_per_cu) {
    if (!batch || (block_threads != 64 && block_threads != 128 && block_threads != 256) ||
        wg_per_cu < 1 || wg_per_cu > 8)
        return FEM_ERR_ARG;
    const int old_bt = batch->block_threads, old_w = batch->wg_per_cu;
    batch->block_threads = block_threads;
    batch->wg_per_cu = wg_per_cu;
    fem_status st = build_items(batch);
    if (st != FEM_OK) {
        batch->block_threads = old_bt;
        batch->wg_per_cu = old_w;
        (void)build_items(batch);
    }
    return st;
}

extern "C" fem_status fem_batch_set_pair_layout(fem_batch batch, int32_t op, int32_t rows_3d,
                                                int32_t rows_2d, int32_t slots) {
    if (!batch || op < FEM_OP_MASS || op > FEM_OP_ELAS || rows_3d < 16 || rows_3d > 128 ||
        rows_2d < 16 || rows_2d > 128 || (slots != 1 && slots != 2 && slots != 4))
        return FEM_ERR_ARG;
    const bool vec = op == FEM_OP_ELAS;
    std::vector<fem_status> st(batch->plans.size(), FEM_OK);
    std::atomic<size_t> next{0};
    int dev0 = 0;
    (void)hipGetDevice(&dev0);
    try {
        run_threads(int(std::min<size_t>(8, batch->plans.size())), [&](int) {
            (void)hipSetDevice(dev0);
            for (size_t m; (m = next.fetch_add(1)) < batch->plans.size();) {
                fem_plan p = batch->plans[m];
                st[m] = rebuild_pair_layout(p, vec, p->d == 3 ? rows_3d : rows_2d, slots);
            }
        });
    } catch (...) {
        return FEM_ERR_NOMEM;
    }
    for (fem_status x : st)
        if (x != FEM_OK) return x;
    return build_pair_layouts(batch, vec ? 1 : 0);
}

static fem_status fem_batch_numeric_impl(fem_batch batch, int32_t op, const double *q_cat,
                                        const double *w_cat, double lambda, double mu,
                                        double *values_cat, hipStream_t stream) {
    PhaseRange range("femasm: batch numeric");
    if (!batch || op < FEM_OP_MASS || op > FEM_OP_ELAS || !q_cat || !values_cat)
        return FEM_ERR_ARG;
    if (op == FEM_OP_MASS_W && !w_cat) return FEM_ERR_ARG;
    const int vec = op == FEM_OP_ELAS ? 1 : 0;
    for (fem_plan p : batch->plans) {
        const int64_t M = vec ? p->d : 1;
        if (M * M * p->nnz >= (int64_t(1) << 31)) return FEM_ERR_OVERFLOW;
    }
    if (batch->kernel == FEM_BATCH_PAIR || batch->kernel == FEM_BATCH_PAIR_SPLIT) {
        // one persistent pair launch over both dimensions (one per dimension
        // when the mixed launch does not fit); any layout missing or too
        // large for LDS: the row-gather launch below covers every mesh
        bool ok = true;
        for (int d = 2; d <= 3; ++d)
            if (batch->has_d[d] && !batch->pairs[vec][d].ok) ok = false;
        if (ok && batch->kernel == FEM_BATCH_PAIR && batch->has_d[2] && batch->has_d[3]) {
            const hipError_t e = launch_pair_mixed(batch->pairs[vec][2], batch->pairs[vec][3], op,
                                                   q_cat, w_cat, lambda, mu, values_cat,
                                                   batch->status, stream);
            if (e == hipSuccess) return FEM_OK;
            if (e != hipErrorNotSupported) return hip_status(e);
        }
        for (int d = 2; d <= 3 && ok; ++d) {
            if (!batch->has_d[d]) continue;
            const hipError_t e = launch_pair_layout(batch->pairs[vec][d], d, op, q_cat, w_cat,
                                                    lambda, mu, values_cat, batch->status, stream);
            if (e == hipErrorNotSupported) ok = false;
            else if (e != hipSuccess) return hip_status(e);
        }
        if (ok) return FEM_OK;
    }
    return launch_batch(op, batch->d_meshes, batch->d_items[vec], batch->nitems[vec],
                        batch->block_threads, batch->lds[vec], batch->cus * batch->wg_per_cu,
                        batch->has_d[2], batch->has_d[3], q_cat, w_cat, lambda, mu, values_cat,
                        batch->status, stream);
}

extern "C" fem_status fem_batch_numeric(fem_batch batch, int32_t op, const double *q_cat,
                                        const double *w_cat, double lambda, double mu,
                                        double *values_cat, hipStream_t stream) {
    const fem_status st =
        fem_batch_numeric_impl(batch, op, q_cat, w_cat, lambda, mu, values_cat, stream);
    return debug_check(st, stream, batch ? batch->status : nullptr);
}

extern "C" fem_status fem_batch_sync_status(fem_batch batch, hipStream_t stream) {
    if (!batch) return FEM_ERR_ARG;
    int32_t word = 0;
    hipError_t e = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = hipMemcpy(&word, batch->status, sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && word != 0) e = hipMemset(batch->status, 0, sizeof(int32_t));
    if (e != hipSuccess) return hip_status(e);
    return word ? FEM_ERR_DEGENERATE : FEM_OK;
}

extern "C" void fem_batch_destroy(fem_batch batch) {
    if (!batch) return;
    free_batch(batch);
    delete batch;
}
