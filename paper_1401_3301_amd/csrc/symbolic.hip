// Symbolic phase: validation, CSR pattern, per-vertex incidence lists with
// slot offsets, and a locality-ordered copy of the connectivity.
//
// The pattern is the `sparse` structure of Section 3 of the paper: row i
// holds every vertex that shares an element with vertex i.  The numeric
// kernels never search it: for every (vertex i, element k, local vertex a
// with me[a,k] == i) the plan stores k's position in plan order and the
// positions, inside row i, of all d+1 vertices of k.  Incidences of a vertex
// are listed in ascending caller element number, which fixes the summation
// order of every CSR entry.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <memory>
#include <thread>

#include "femasm_impl.h"
#include "host_threads.h"
#include "symbolic_host.h"

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

template <class T>
fem_status upload(T **dst, const std::vector<T> &src) {
    *dst = nullptr;
    size_t bytes = sizeof(T) * std::max<size_t>(src.size(), 1);
    hipError_t e = hipMalloc(reinterpret_cast<void **>(dst), bytes);
    if (e != hipSuccess) {
        *dst = nullptr;
        return hip_status(e);
    }
    if (!src.empty()) {
        e = hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_status(e);
    }
    return FEM_OK;
}

void free_plan_arrays(fem_plan_data *p) {
    void *ptrs[] = {p->rp,       p->ci,      p->pme,    p->porig, p->inc_ptr,
                    p->inc_elem, p->inc_off, p->status, p->part};
    for (void *x : ptrs)
        if (x) (void)hipFree(x);
    p->rp = p->ci = p->pme = p->porig = p->inc_ptr = nullptr;
    p->inc_elem = p->inc_off = nullptr;
    p->status = nullptr;
    p->part = nullptr;
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

static fem_status fem_assemble_symbolic_impl(int32_t d, int64_t nq, int64_t nme, const int32_t *me,
                                            hipStream_t stream, fem_plan *out) {
    if (!out || (d != 2 && d != 3) || nq < 0 || nme < 0 || (nme > 0 && !me))
        return FEM_ERR_ARG;
    const int NL = d + 1;
    if (nme >= (int64_t(1) << 30) || int64_t(NL) * nme >= (int64_t(1) << 31) ||
        nq >= (int64_t(1) << 31) - 1)
        return FEM_ERR_OVERFLOW;

    // ---- connectivity to the host (the plan is built once per mesh)
    std::vector<int32_t> hme(size_t(NL) * nme);
    if (nme > 0) {
        hipError_t e = hipMemcpyAsync(hme.data(), me, sizeof(int32_t) * hme.size(),
                                      hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_status(e);
    }

    // ---- validation: indices in range, no repeated vertex in an element
    std::atomic<int> bad{0};
    parallel_ranges(nme, [&](int64_t b, int64_t e) {
        for (int64_t k = b; k < e && !bad.load(std::memory_order_relaxed); ++k) {
            for (int a = 0; a < NL; ++a) {
                int32_t v = hme[size_t(a) * nme + k];
                if (v < 0 || v >= nq) { bad = 1; break; }
                for (int c = 0; c < a; ++c)
                    if (hme[size_t(c) * nme + k] == v) { bad = 1; break; }
            }
        }
    });
    if (bad) return FEM_ERR_INDEX;

    // ---- incidences: vertex -> (element, local vertex), ascending element
    // (element slots k*(d+1)+a sorted stably by their vertex)
    const int64_t ninc = int64_t(NL) * nme;
    std::vector<int64_t> ip;
    std::vector<int32_t> inc_k(ninc);
    std::vector<uint8_t> inc_a(ninc);
    stable_key_sort(
        ninc, nq, worker_count(),
        [&](int64_t r) { return int64_t(hme[size_t(r % NL) * nme + r / NL]); },
        [&](int64_t pos, int64_t r) {
            inc_k[pos] = int32_t(r / NL);
            inc_a[pos] = uint8_t(r % NL);
        },
        ip);

    // ---- pattern: row i = sorted unique vertices of the elements around i,
    // and for every incidence the positions of its element's vertices in the
    // row.  One sort per row: each thread keeps the columns of its contiguous
    // row range until the row offsets are known, then copies them into place.
    std::vector<int32_t> rowlen(nq, 0);
    std::vector<uint32_t> ioff(ninc);
    std::atomic<int> too_long{0};
    const int nrt = nq < 4096 ? 1 : worker_count();
    const int64_t rchunk = (nq + nrt - 1) / nrt;
    std::vector<std::vector<int32_t>> tcols(nrt);
    {
        auto rows_of = [&](int t) {
            std::vector<int32_t> buf;
            std::vector<int32_t> &out = tcols[t];
            for (int64_t i = t * rchunk, e = std::min(nq, (t + 1) * rchunk); i < e; ++i) {
                buf.clear();
                for (int64_t s = ip[i]; s < ip[i + 1]; ++s) {
                    const int64_t k = inc_k[s];
                    for (int b = 0; b < NL; ++b) buf.push_back(hme[size_t(b) * nme + k]);
                }
                std::sort(buf.begin(), buf.end());
                buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
                rowlen[i] = int32_t(buf.size());
                if (buf.size() > 255) {
                    too_long = 1;
                    return;
                }
                out.insert(out.end(), buf.begin(), buf.end());
                for (int64_t s = ip[i]; s < ip[i + 1]; ++s) {
                    const int64_t k = inc_k[s];
                    uint32_t packed = 0;
                    for (int b = 0; b < NL; ++b) {
                        const int32_t v = hme[size_t(b) * nme + k];
                        packed |= uint32_t(std::lower_bound(buf.begin(), buf.end(), v) - buf.begin())
                                  << (8 * b);
                    }
                    ioff[s] = packed;
                }
            }
        };
        run_threads(nrt, rows_of);
    }
    if (too_long) return FEM_ERR_OVERFLOW;
    std::vector<int32_t> rp(nq + 1, 0);
    int64_t nnz = 0;
    int max_row = 0;
    for (int64_t i = 0; i < nq; ++i) {
        rp[i] = int32_t(nnz);
        nnz += rowlen[i];
        max_row = std::max(max_row, rowlen[i]);
        if (nnz >= (int64_t(1) << 31)) return FEM_ERR_OVERFLOW;
    }
    rp[nq] = int32_t(nnz);
    std::vector<int32_t> ci(nnz);
    run_threads(nrt, [&](int t) {
        if (tcols[t].empty()) return;
        std::copy(tcols[t].begin(), tcols[t].end(), ci.begin() + rp[std::min(nq, t * rchunk)]);
        std::vector<int32_t>().swap(tcols[t]);
    });

    // ---- device plan.  The block layouts need only the pattern and the
    // incidences: they are built on another thread while this one orders the
    // elements and uploads the plan arrays (no return before the join).
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
    p->nnz = nnz;
    p->max_row = max_row;
    (void)hipGetDevice(&p->device);
    fem_status sb = FEM_OK;
    std::thread layouts;
    struct Joiner {
        std::thread &t;
        ~Joiner() {
            if (t.joinable()) t.join();
        }
    } join_layouts{layouts};   // also on an exception below
    if (nme > 0)
        layouts = std::thread([&] {
            (void)hipSetDevice(p->device);
            try {
                sb = upload_blocks(p.get(), d, nq, nme, hme.data(), rp.data(), ci.data(),
                                   ip.data(), inc_k.data());
            } catch (...) {
                sb = FEM_ERR_NOMEM;
            }
        });

    // ---- locality order of elements: by smallest vertex id (counting sort,
    // stable in caller element number)
    std::vector<int32_t> porig(nme), pinv(nme);
    {
        std::vector<int64_t> kptr;
        stable_key_sort(
            nme, nq, worker_count(),
            [&](int64_t k) {
                int32_t m0 = hme[size_t(k)];
                for (int a = 1; a < NL; ++a) m0 = std::min(m0, hme[size_t(a) * nme + k]);
                return int64_t(m0);
            },
            [&](int64_t q, int64_t k) {
                porig[q] = int32_t(k);
                pinv[k] = int32_t(q);
            },
            kptr);
    }
    std::vector<int32_t> pme(size_t(NL) * nme);
    parallel_ranges(nme, [&](int64_t b, int64_t e) {
        for (int64_t q = b; q < e; ++q) {
            int64_t k = porig[q];
            for (int a = 0; a < NL; ++a) pme[size_t(q) * NL + a] = hme[size_t(a) * nme + k];
        }
    });
    std::vector<uint32_t> ielem(ninc);
    std::vector<int32_t> ip32(nq + 1);
    parallel_ranges(ninc, [&](int64_t b, int64_t e) {
        for (int64_t t = b; t < e; ++t) ielem[t] = uint32_t(pinv[inc_k[t]]) | (uint32_t(inc_a[t]) << 30);
    });
    for (int64_t i = 0; i <= nq; ++i) ip32[i] = int32_t(ip[i]);

    fem_status st = FEM_OK;
    if (st == FEM_OK) st = upload(&p->rp, rp);
    if (st == FEM_OK) st = upload(&p->ci, ci);
    if (st == FEM_OK) st = upload(&p->pme, pme);
    if (st == FEM_OK) st = upload(&p->porig, porig);
    if (st == FEM_OK) st = upload(&p->inc_ptr, ip32);
    if (st == FEM_OK) st = upload(&p->inc_elem, ielem);
    if (st == FEM_OK) st = upload(&p->inc_off, ioff);
    if (st == FEM_OK) st = upload(&p->status, std::vector<int32_t>(1, 0));
    if (st == FEM_OK) st = upload(&p->part, std::vector<double>(size_t((int64_t(d) * nq + 255) / 256 + 1), 0.0));
    if (layouts.joinable()) layouts.join();
    if (st == FEM_OK) st = sb;
    if (st != FEM_OK) return st;   // p's deleter frees what was uploaded
    p->h_rp = std::move(rp);
    for (int M : {1, d}) p->launch[M] = row_launch_for(p->h_rp, nq, M, kLdsCap);
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
