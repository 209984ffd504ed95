// Symbolic phase: the plan of one mesh.
//
// The CSR pattern of `sparse` (Section 3), the per-vertex incidence lists
// with the column positions of every element vertex, and the locality-ordered
// connectivity are built on the GPU (pattern.hip) before the call returns;
// they are all the row-gather kernel needs, so a numeric assembly can follow
// at once.  The vertex-block layouts of the faster block kernels need more
// host-side work (breadth-first blocks, per-pair element lists): a host
// thread builds and uploads them after the call has returned and publishes
// them when complete.  Until then the numeric calls of the four P1 operators
// run the row-gather kernel, which sums every entry in the same order with
// the same expressions and so gives the same bits; the operators that have
// only a block-kernel form wait for the layouts.
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <thread>

#include "femasm_impl.h"
#include "host_threads.h"

namespace femasm {

fem_status hip_status(hipError_t e) {
    if (e == hipSuccess) return FEM_OK;
    if (e == hipErrorOutOfMemory) return FEM_ERR_NOMEM;
    return FEM_ERR_DEVICE;
}

namespace {

int worker_count() {
    unsigned hc = std::thread::hardware_concurrency();
    int n = hc == 0 ? 4 : static_cast<int>(hc);
    return std::max(1, std::min(n, 16));
}

// Runs fn(begin, end) over [0, n) split into contiguous chunks.
template <class F>
void parallel_ranges(int64_t n, F fn) {
    int nt = worker_count();
    if (n < 4096 || nt == 1) {
        fn(int64_t(0), n);
        return;
    }
    run_chunks(nt, n, fn);
}

void free_plan_arrays(fem_plan_data *p) {
    if (p->layout_thread.joinable()) p->layout_thread.join();
    void *ptrs[] = {p->rp,       p->ci,      p->pme,    p->porig, p->inc_ptr,
                    p->inc_elem, p->inc_off, p->status, p->part, p->vpos};
    for (void *x : ptrs)
        if (x) (void)hipFree(x);
    p->rp = p->ci = p->pme = p->porig = p->inc_ptr = nullptr;
    p->inc_elem = nullptr;
    p->inc_off = nullptr;
    p->status = nullptr;
    p->part = nullptr;
    p->vpos = nullptr;
    p->vpos_bytes.store(0);
    free_blocks(&p->blk);
    free_pairs(&p->pscal);
    free_pairs(&p->pvec);
}

}  // namespace

RowLaunch row_launch_for(const std::vector<int32_t> &h_rp, int64_t nq, int M, size_t lds_cap) {
    RowLaunch best;
    const int64_t nrows = int64_t(M) * nq;
    auto vstart = [&](int64_t r) -> int64_t {
        int64_t i = r / M, l = r - i * M;
        int64_t s = int64_t(M) * M * h_rp[i];
        if (l) s += l * M * int64_t(h_rp[i + 1] - h_rp[i]);
        return s;
    };
    for (int R0 : {256, 128, 64}) {
        const int R = R0 / M * M;   // elasticity tiles hold whole vertices
        int64_t tiles = (nrows + R - 1) / R;
        size_t bytes = sizeof(double);
        for (int64_t t = 0; t < tiles; ++t) {
            int64_t r0 = t * R, r1 = std::min(nrows, r0 + R);
            bytes = std::max(bytes, tile_lds_bytes(M, vstart(r1) - vstart(r0), r1 - r0));
        }
        best.rows_per_wg = R;
        best.lds_bytes = bytes;
        best.tiles = tiles;
        if (bytes <= lds_cap) return best;
    }
    best.rows_per_wg = 0;  // does not fit
    return best;
}

fem_status debug_check(fem_status st, hipStream_t s, int32_t *status_word) {
    const char *env = getenv("FEMASM_DEBUG");
    if (!env || !*env || strcmp(env, "0") == 0 || st != FEM_OK) return st;
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return hip_status(e);
    if (!status_word) return FEM_OK;
    int32_t word = 0;
    e = hipMemcpy(&word, status_word, sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && word != 0) {
        const int32_t zero = 0;
        e = hipMemcpy(status_word, &zero, sizeof(int32_t), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return hip_status(e);
    return word ? FEM_ERR_DEGENERATE : FEM_OK;
}

void wait_layouts(fem_plan_data *p) {
    std::unique_lock<std::mutex> lock(p->layout_mu);
    p->layout_cv.wait(lock, [&] { return p->layout_state.load() != kLayoutBuilding; });
}

}  // namespace femasm

using namespace femasm;

extern "C" const char *fem_status_str(fem_status s) {
    switch (s) {
        case FEM_OK: return "FEM_OK";
        case FEM_ERR_ARG: return "FEM_ERR_ARG";
        case FEM_ERR_INDEX: return "FEM_ERR_INDEX";
        case FEM_ERR_DEGENERATE: return "FEM_ERR_DEGENERATE";
        case FEM_ERR_OVERFLOW: return "FEM_ERR_OVERFLOW";
        case FEM_ERR_NOMEM: return "FEM_ERR_NOMEM";
        case FEM_ERR_DEVICE: return "FEM_ERR_DEVICE";
    }
    return "FEM_ERR_UNKNOWN";
}

// What the host-built block layouts need, copied back from the plan's
// device arrays: the connectivity in caller layout, the CSR columns and the
// incidences as caller element numbers.
struct LayoutInput {
    std::vector<int32_t> me, ci, inc_k;
    std::vector<int64_t> ip;
};

static fem_status layout_input(const fem_plan_s *p, LayoutInput &in) {
    const int NL = p->d + 1;
    const int64_t nq = p->nq, nme = p->nme, ninc = int64_t(NL) * nme, nnz = p->nnz;
    std::vector<int32_t> pme(static_cast<size_t>(ninc)), porig(static_cast<size_t>(nme)),
        ip32(static_cast<size_t>(nq + 1));
    std::vector<uint32_t> ielem(static_cast<size_t>(ninc));
    in.ci.resize(static_cast<size_t>(nnz));
    hipError_t e = hipSuccess;
    auto d2h = [&](void *dst, const void *src, size_t bytes) {
        if (e == hipSuccess && bytes > 0) e = copy_sync(dst, src, bytes, hipMemcpyDeviceToHost);
    };
    d2h(pme.data(), p->pme, sizeof(int32_t) * pme.size());
    d2h(porig.data(), p->porig, sizeof(int32_t) * porig.size());
    d2h(in.ci.data(), p->ci, sizeof(int32_t) * in.ci.size());
    d2h(ip32.data(), p->inc_ptr, sizeof(int32_t) * ip32.size());
    d2h(ielem.data(), p->inc_elem, sizeof(uint32_t) * ielem.size());
    if (e != hipSuccess) return hip_status(e);
    in.me.resize(static_cast<size_t>(ninc));
    in.inc_k.resize(static_cast<size_t>(ninc));
    in.ip.resize(static_cast<size_t>(nq + 1));
    parallel_ranges(nme, [&](int64_t b, int64_t en) {
        for (int64_t q = b; q < en; ++q)
            for (int a = 0; a < NL; ++a) in.me[size_t(a * nme + porig[q])] = pme[size_t(q * NL + a)];
    });
    parallel_ranges(ninc, [&](int64_t b, int64_t en) {
        for (int64_t t = b; t < en; ++t) in.inc_k[t] = porig[ielem[t] & 0x3fffffffu];
    });
    for (int64_t i = 0; i <= nq; ++i) in.ip[i] = ip32[i];
    return FEM_OK;
}

// The layout thread: copies the plan's incidences and connectivity back to
// the host, builds the block layouts there (blocks_host.h), uploads them and
// publishes them.  Device copies run on streams of their own.
static void build_layouts(fem_plan_s *p) {
    PhaseRange range("femasm: block layouts (host thread)");
    fem_plan_data L;   // the layouts under construction
    L.device = p->device;
    fem_status st = FEM_OK;
    try {
        (void)hipSetDevice(p->device);
        LayoutInput in;
        st = layout_input(p, in);
        if (st == FEM_OK) {
            st = upload_blocks(&L, p->d, p->nq, p->nme, in.me.data(), p->h_rp.data(), in.ci.data(),
                               in.ip.data(), in.inc_k.data());
            if (st == FEM_OK) st = upload_leftover(L.pscal, p, 1);
            if (st == FEM_OK) st = upload_leftover(L.pvec, p, p->d);
        }
    } catch (...) {
        st = FEM_ERR_NOMEM;
    }
    const bool any = st == FEM_OK && (L.pscal.ok || L.pvec.ok || L.blk.ok);
    if (!any) {
        free_blocks(&L.blk);
        free_pairs(&L.pscal);
        free_pairs(&L.pvec);
    }
    {
        std::lock_guard<std::mutex> lock(p->layout_mu);
        if (any) {
            p->blk = L.blk;
            p->pscal = std::move(L.pscal);
            p->pvec = std::move(L.pvec);
        }
        p->layout_status = st;
        p->layout_state.store(any ? kLayoutReady : kLayoutNone, std::memory_order_release);
    }
    p->layout_cv.notify_all();
}

fem_status femasm::rebuild_pair_layout(fem_plan_data *pd, bool vec, int R, int slots) {
    PhaseRange range("femasm: pair layout rebuild");
    fem_plan_s *p = static_cast<fem_plan_s *>(pd);
    wait_layouts(p);
    if (p->nme == 0 || p->nnz == 0) return FEM_OK;
    try {
        LayoutInput in;
        fem_status st = layout_input(p, in);
        if (st != FEM_OK) return st;
        PairPlan P;
        st = upload_pairs(P, R, slots, !vec, p->d, p->nq, p->nme, in.me.data(), p->h_rp.data(),
                          in.ci.data(), in.ip.data(), in.inc_k.data());
        if (st == FEM_OK) st = upload_leftover(P, p, vec ? p->d : 1);
        if (st != FEM_OK) {
            free_pairs(&P);
            return st;
        }
        std::lock_guard<std::mutex> lock(p->layout_mu);
        PairPlan &dst = vec ? p->pvec : p->pscal;
        free_pairs(&dst);
        dst = std::move(P);
        if (dst.ok) p->layout_state.store(kLayoutReady, std::memory_order_release);
        return FEM_OK;
    } catch (...) {
        return FEM_ERR_NOMEM;
    }
}

static fem_status fem_assemble_symbolic_impl(int32_t d, int64_t nq, int64_t nme, const int32_t *me,
                                            hipStream_t stream, fem_plan *out) {
    if (!out || (d != 2 && d != 3) || nq < 0 || nme < 0 || (nme > 0 && !me))
        return FEM_ERR_ARG;
    const int NL = d + 1;
    if (nme >= (int64_t(1) << 30) || int64_t(NL) * nme >= (int64_t(1) << 31) ||
        nq >= (int64_t(1) << 31) - 1)
        return FEM_ERR_OVERFLOW;
    // the plan's device arrays are freed with it unless it is handed out
    // (also when an exception unwinds through here)
    struct PlanFree {
        void operator()(fem_plan_s *x) const {
            free_plan_arrays(x);
            delete x;
        }
    };
    std::unique_ptr<fem_plan_s, PlanFree> p(new fem_plan_s());
    p->d = d;
    p->nq = nq;
    p->nme = nme;
    (void)hipGetDevice(&p->device);
    fem_status st = build_pattern_gpu(p.get(), me, stream);
    if (st != FEM_OK) {
        p->layout_state.store(kLayoutNone);
        return st;
    }
    for (int M : {1, d}) p->launch[M] = row_launch_for(p->h_rp, nq, M, kLdsCap);
    // FEMASM_LAYOUTS=sync builds the block layouts before returning
    const char *mode = getenv("FEMASM_LAYOUTS");
    if (nme == 0 || p->nnz == 0) {
        p->layout_state.store(kLayoutNone);
    } else if (mode && strcmp(mode, "sync") == 0) {
        build_layouts(p.get());
    } else {
        fem_plan_s *raw = p.get();
        p->layout_thread = std::thread([raw] { build_layouts(raw); });
    }
    *out = p.release();
    return FEM_OK;
}

extern "C" fem_status fem_assemble_symbolic(int32_t d, int64_t nq, int64_t nme, const int32_t *me,
                                            hipStream_t stream, fem_plan *out) {
    // host allocations (or threads) can fail for very large meshes: report
    // it, never throw across the ABI
    try {
        return fem_assemble_symbolic_impl(d, nq, nme, me, stream, out);
    } catch (...) {
        return FEM_ERR_NOMEM;
    }
}

extern "C" fem_status fem_plan_query(fem_plan plan, int32_t op, int64_t *nrows, int64_t *nnz) {
    if (!plan || op < FEM_OP_MASS || op > FEM_OP_ELAS) return FEM_ERR_ARG;
    const int64_t M = op == FEM_OP_ELAS ? plan->d : 1;
    if (nrows) *nrows = M * plan->nq;
    if (nnz) *nnz = M * M * plan->nnz;
    return FEM_OK;
}

extern "C" fem_status fem_plan_info(fem_plan plan, int32_t *d, int64_t *nq, int64_t *nme,
                                    int32_t *max_row) {
    if (!plan) return FEM_ERR_ARG;
    if (d) *d = plan->d;
    if (nq) *nq = plan->nq;
    if (nme) *nme = plan->nme;
    if (max_row) *max_row = plan->max_row;
    return FEM_OK;
}

extern "C" fem_status fem_plan_layouts(fem_plan plan, int32_t wait, int32_t *state) {
    if (!plan) return FEM_ERR_ARG;
    if (wait) wait_layouts(plan);
    const int s = plan->layout_state.load(std::memory_order_acquire);
    if (state) *state = s;
    if (s == kLayoutBuilding) return FEM_OK;
    std::lock_guard<std::mutex> lock(plan->layout_mu);
    return plan->layout_status;
}

extern "C" fem_status fem_plan_sync_status(fem_plan plan, hipStream_t stream) {
    if (!plan) return FEM_ERR_ARG;
    int32_t word = 0;
    hipError_t e = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = hipMemcpy(&word, plan->status, sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess && word != 0) {
        const int32_t zero = 0;
        e = hipMemcpy(plan->status, &zero, sizeof(int32_t), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return hip_status(e);
    return word ? FEM_ERR_DEGENERATE : FEM_OK;
}

extern "C" void fem_plan_destroy(fem_plan plan) {
    if (!plan) return;
    free_plan_arrays(plan);
    delete plan;
}
