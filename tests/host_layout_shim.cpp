// Test shim: exposes the host-side block and pair-list builders of the
// library (paper_1401_3301_amd/csrc/blocks_host.h) through a C interface so
// that tests/test_host_layout.py can check them on the CPU, against a brute
// force written in Python.  Not part of the library.
#include <algorithm>
#include <cstdint>
#include <cstring>

#include "../paper_1401_3301_amd/csrc/blocks_host.h"

using namespace femasm;

template <class T>
static void put(void *dst, const std::vector<T> &v);

static BlockHost g_h;
static PairHost g_p;

extern "C" int hl_build(int d, int64_t nq, int64_t nme, const int32_t *me, const int32_t *rp,
                        const int32_t *ci, const int64_t *ip, const int32_t *inc_k, int R,
                        int64_t max_pairs, int max_nodes, int waves, int slots, int tri,
                        int dedup, int64_t chunk_min, int pair_mode, int max_elems,
                        int64_t max_ent, int64_t max_inc, int64_t *sizes) {
    g_h = build_block_host(d, nq, nme, me, rp, ci, ip, inc_k, R, 4, max_pairs, max_nodes,
                           chunk_min, max_elems, pair_mode != 0, max_inc);
    if (!g_h.ok) return 1;
    g_p = build_pair_host(g_h, d, rp, ci, waves, slots, 2, tri != 0, dedup != 0, max_ent);
    if (!g_p.ok) return 2;
    sizes[0] = g_h.nb;
    sizes[1] = int64_t(g_h.rows.size());
    sizes[2] = int64_t(g_h.nodes.size());
    sizes[3] = int64_t(g_h.elem.size());
    sizes[4] = int64_t(g_h.rec.size());
    sizes[5] = int64_t(g_p.task_cnt.size());
    sizes[6] = int64_t(g_p.ent.size());
    sizes[7] = g_h.max_nodes;
    sizes[8] = int64_t(g_h.leftover.size());
    sizes[9] = int64_t(g_h.wrec.size());
    return 0;
}

extern "C" void hl_pair_mode(uint64_t *wrec, int32_t *leftover, uint8_t *blk_ok) {
    put(wrec, g_h.wrec);
    put(leftover, g_h.leftover);
    put(blk_ok, g_p.blk_ok);
}

template <class T>
static void put(void *dst, const std::vector<T> &v) {
    if (!v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(T));
}

extern "C" void hl_blocks(int32_t *rows, int32_t *row_ptr, int32_t *nodes, int32_t *node_ptr,
                          uint16_t *elem, int32_t *elem_ptr, uint32_t *rec, int64_t *rec_ptr,
                          int32_t *maxdeg) {
    put(rows, g_h.rows);
    put(row_ptr, g_h.row_ptr);
    put(nodes, g_h.nodes);
    put(node_ptr, g_h.node_ptr);
    put(elem, g_h.elem);
    put(elem_ptr, g_h.elem_ptr);
    put(rec, g_h.rec);
    put(rec_ptr, g_h.rec_ptr);
    put(maxdeg, g_h.maxdeg);
}

extern "C" void hl_pairs(int32_t *wt, int32_t *task_cnt, int64_t *task_ent, uint16_t *hdr,
                         uint16_t *hdr2, uint16_t *ent, int64_t *ent_ptr) {
    put(wt, g_p.wt);
    put(task_cnt, g_p.task_cnt);
    put(task_ent, g_p.task_ent);
    put(hdr, g_p.hdr);
    put(hdr2, g_p.hdr2);
    put(ent, g_p.ent);
    put(ent_ptr, g_p.ent_ptr);
}

extern "C" uint64_t hl_pack_wave_starts(const int32_t *wt, int waves) {
    return pack_wave_starts(wt, waves);
}

#include "../paper_1401_3301_amd/csrc/symbolic_host.h"

extern "C" void hl_key_sort(int64_t n, int64_t nkeys, const int64_t *keys, int nthreads,
                            int64_t *order, int64_t *ptr) {
    std::vector<int64_t> p;
    stable_key_sort(
        n, nkeys, nthreads, [&](int64_t r) { return keys[r]; },
        [&](int64_t pos, int64_t r) { order[pos] = r; }, p);
    std::memcpy(ptr, p.data(), sizeof(int64_t) * p.size());
}

#include <new>

#include "../paper_1401_3301_amd/csrc/host_threads.h"

// run_threads: every index runs; an exception thrown on one of them reaches
// the caller after all have been joined (returns 1 then).
extern "C" int hl_run_threads(int nt, int throw_at, int *ran) {
    try {
        run_threads(nt, [&](int t) {
            ran[t] = 1;
            if (t == throw_at) throw std::bad_alloc();
        });
    } catch (const std::bad_alloc &) {
        return 1;
    }
    return 0;
}
