// Host construction of the vertex-block layout used by the block kernels.
//
// Vertices (CSR rows) are grouped into compact blocks by breadth-first
// growth over the mesh graph, seeded at the lowest unassigned vertex (within
// contiguous id chunks grown in parallel for large meshes).  For
// each block the plan stores
//   - its rows (ascending vertex id) and its touched vertices: the rows first,
//     then every other vertex of an element around a row (ascending id);
//     "local vertex" = position in that list (16 bits);
//   - its elements: every element with a vertex among the rows, in ascending
//     caller element number, as d+1 local vertex ids (four 16-bit slots);
//   - per row, its incidences in ascending element position, as 32-bit
//     records: element position (bits 0-9), the row's local vertex index a
//     within that element (bits 10-11) and, for each local vertex b of the
//     element, the position of that vertex in the row's CSR columns (5 bits
//     each from bit 12).  Records are interleaved across the rows of the
//     block (record t of row r at t*nrows + r) and padded with ~0u.
// Blocks grow until they hold R rows or the next vertex would bring the
// element count above max_elems (at most kMaxBlockElems; or, when max_pairs > 0, the number of
// CSR entries of the block's rows above max_pairs; when max_nodes > 0, the
// number of touched vertices above max_nodes; when max_inc > 0, (d+1) times
// the sum of the rows' star sizes above max_inc -- that sum bounds the pair
// lists' entries before mirror pairs share a list).
// Every incidence also gets a wide record (`wrec`, 64 bits: element position
// bits 0-9, local vertex a bits 10-11, the column position of local vertex b
// in 12 bits from bit 12 + 12b), the input of the pair lists.
// Record mode (the record-block kernel, which must cover every row): a mesh
// with a row longer than 32 entries, or a vertex whose own star exceeds a
// cap, does not fit (ok == false).  Pair mode (pair_mode): such vertices --
// a row longer than kMaxPairRow entries or than max_pairs, a star above the
// element cap (or (d+1) times it above max_inc), a row with more vertices
// than max_nodes -- are left out of
// the blocks and listed in `leftover` (another kernel assembles their rows);
// the 32-bit records are not built.
#pragma once

#include <algorithm>
#include <cstdint>
#include <thread>
#include <vector>

#include "host_threads.h"

namespace femasm {

struct BlockHost {
    int nb = 0;
    std::vector<int32_t> rows, row_ptr;
    std::vector<int32_t> nodes, node_ptr;
    std::vector<uint16_t> elem;   // 4 per block element
    std::vector<int32_t> elem_ptr;
    std::vector<uint32_t> rec;
    std::vector<uint64_t> wrec;     // wide records, same interleaving as rec
    std::vector<int64_t> rec_ptr;
    std::vector<int32_t> leftover;  // pair mode: used vertices that are no block's row
    std::vector<int32_t> maxdeg;
    int max_rows = 0, max_nodes = 0, max_elems = 0;
    int64_t max_nacc = 0;
    int64_t total_elems = 0;
    bool ok = false;
};

constexpr uint32_t kRecPad = 0xffffffffu;
constexpr uint64_t kWRecPad = ~uint64_t(0);
constexpr int kMaxBlockElems = 1023;
constexpr int kMaxRowLen = 32;     // record mode: 5-bit column positions
constexpr int kMaxPairRow = 511;   // pair mode: 9-bit column positions of the pair headers

inline BlockHost build_block_host(int d, int64_t nq, int64_t nme, const int32_t *me,
                                  const int32_t *rp, const int32_t *ci, const int64_t *ip,
                                  const int32_t *inc_k, int R, int nthreads,
                                  int64_t max_pairs = 0, int max_nodes = 0,
                                  int64_t chunk_min = 8192, int max_elems = kMaxBlockElems,
                                  bool pair_mode = false, int64_t max_inc = 0) {
    const int ecap = std::min(max_elems, kMaxBlockElems);   // growth stops above it
    BlockHost H;
    const int NL = d + 1;
    // vertices that cannot be a block row (pair mode), else the whole mesh fails
    std::vector<uint8_t> excluded(nq, 0);
    for (int64_t i = 0; i < nq; ++i) {
        const int64_t len = rp[i + 1] - rp[i];
        if (!pair_mode) {
            if (len > kMaxRowLen) return H;
            continue;
        }
        if (len == 0) continue;
        if (len > kMaxPairRow || (max_pairs > 0 && len > max_pairs) ||
            (max_nodes > 0 && len > max_nodes) || ip[i + 1] - ip[i] > ecap ||
            (max_inc > 0 && NL * (ip[i + 1] - ip[i]) > max_inc)) {
            excluded[i] = 1;
            H.leftover.push_back(int32_t(i));
        }
    }

    // ---- breadth-first blocks over used vertices, capped in rows and elements.
    // The vertex ids are cut into contiguous chunks grown independently (one
    // thread each, with its own stamps; growth never leaves a chunk), and the
    // chunks' blocks are concatenated in chunk order, so the layout does not
    // depend on thread timing.
    // (at most 8 chunks: the blocks cut at chunk borders cost a little list
    // traffic in the numeric phase)
    const int nchunk = int(std::max<int64_t>(
        1, std::min<int64_t>(std::min(nthreads, 8), nq / std::max<int64_t>(1, chunk_min))));
    std::vector<int32_t> blk_of(nq, -1);   // chunk-local block of each taken vertex
    std::vector<std::vector<int32_t>> crow(nchunk), cptr(nchunk);
    std::vector<int> cfail(nchunk, 0);
    auto grow = [&](int c) {
        const int64_t v0 = nq * c / nchunk, v1 = nq * (c + 1) / nchunk;
        std::vector<int32_t> queue;
        std::vector<int32_t> estamp(nme, -1);   // block that last counted the element
        std::vector<int32_t> nstamp(max_nodes > 0 ? nq : 0, -1);   // ... the touched vertex
        std::vector<int32_t> &rows = crow[c], &rptr = cptr[c];
        queue.reserve(R);
        rptr.push_back(0);
        int nbc = 0;
        auto new_elems = [&](int32_t v, int b) {
            int n = 0;
            for (int64_t t = ip[v]; t < ip[v + 1]; ++t) n += estamp[inc_k[t]] != b;
            return n;
        };
        // touched vertices the elements of v would add (only when capped)
        auto new_nodes = [&](int32_t v, int b) {
            const int32_t prov = -2 - b;   // provisional mark, undone below
            int n = 0;
            for (int64_t t = ip[v]; t < ip[v + 1]; ++t) {
                const int32_t k = inc_k[t];
                if (estamp[k] == b) continue;
                for (int a = 0; a < d + 1; ++a) {
                    const int32_t u = me[int64_t(a) * nme + k];
                    if (nstamp[u] != b && nstamp[u] != prov) {
                        nstamp[u] = prov;
                        ++n;
                    }
                }
            }
            for (int64_t t = ip[v]; t < ip[v + 1]; ++t) {
                const int32_t k = inc_k[t];
                if (estamp[k] == b) continue;
                for (int a = 0; a < d + 1; ++a) {
                    const int32_t u = me[int64_t(a) * nme + k];
                    if (nstamp[u] == prov) nstamp[u] = -1;
                }
            }
            return n;
        };
        auto take = [&](int32_t v, int b) {
            blk_of[v] = b;
            for (int64_t t = ip[v]; t < ip[v + 1]; ++t) {
                const int32_t k = inc_k[t];
                if (max_nodes > 0 && estamp[k] != b)
                    for (int a = 0; a < d + 1; ++a) nstamp[me[int64_t(a) * nme + k]] = b;
                estamp[k] = b;
            }
        };
        for (int64_t seed = v0; seed < v1; ++seed) {
            if (blk_of[seed] != -1 || rp[seed + 1] == rp[seed] || excluded[seed]) continue;
            const int b = nbc;
            if (ip[seed + 1] - ip[seed] > kMaxBlockElems) {
                cfail[c] = 1;
                return;
            }
            queue.clear();
            queue.push_back(int32_t(seed));
            int nel = new_elems(int32_t(seed), b);
            int64_t npairs = rp[seed + 1] - rp[seed];
            // (d+1) x the stars of the rows: the list entries of the rows'
            // pairs before mirror pairs are merged (capped by max_inc)
            int64_t ninc = NL * (ip[seed + 1] - ip[seed]);
            int nnodes = max_nodes > 0 ? new_nodes(int32_t(seed), b) : 0;
            if (max_nodes > 0 && nnodes > max_nodes) {
                cfail[c] = 1;
                return;
            }
            take(int32_t(seed), b);
            size_t head = 0;
            bool full = false;
            while (head < queue.size() && int(queue.size()) < R && !full) {
                const int32_t v = queue[head++];
                for (int32_t s = rp[v]; s < rp[v + 1] && int(queue.size()) < R; ++s) {
                    const int32_t j = ci[s];
                    if (j < v0 || j >= v1 || blk_of[j] != -1 || rp[j + 1] == rp[j] || excluded[j])
                        continue;
                    const int add = new_elems(j, b);
                    const int64_t addp = rp[j + 1] - rp[j];
                    const int addn = max_nodes > 0 ? new_nodes(j, b) : 0;
                    const int64_t addi = NL * (ip[j + 1] - ip[j]);
                    if (nel + add > ecap || (max_pairs > 0 && npairs + addp > max_pairs) ||
                        (max_nodes > 0 && nnodes + addn > max_nodes) ||
                        (max_inc > 0 && ninc + addi > max_inc)) {
                        full = true;
                        break;
                    }
                    nel += add;
                    npairs += addp;
                    ninc += addi;
                    nnodes += addn;
                    take(j, b);
                    queue.push_back(j);
                }
            }
            std::sort(queue.begin(), queue.end());
            rows.insert(rows.end(), queue.begin(), queue.end());
            rptr.push_back(int32_t(rows.size()));
            nbc += 1;
        }
    };
    run_threads(nchunk, grow);
    H.row_ptr.push_back(0);
    for (int c = 0; c < nchunk; ++c) {
        if (cfail[c]) return BlockHost();
        for (size_t b = 1; b < cptr[c].size(); ++b) {
            H.rows.insert(H.rows.end(), crow[c].begin() + cptr[c][b - 1], crow[c].begin() + cptr[c][b]);
            H.row_ptr.push_back(int32_t(H.rows.size()));
            H.nb += 1;
        }
    }
    const int nb = H.nb;

    // ---- per-block lists, built in parallel into per-block vectors
    struct Blk {
        std::vector<int32_t> nodes;
        std::vector<uint16_t> elem;
        std::vector<uint32_t> rec;
        std::vector<uint64_t> wrec;
        int32_t maxdeg = 0;
        int64_t nacc = 0;
        bool ok = true;
    };
    std::vector<Blk> blks(nb);
    auto work = [&](int b0, int b1) {
        std::vector<int32_t> loc(nq, -1);
        std::vector<int32_t> elems, halo;
        // per block: element id -> position (open addressing, stamped by
        // block so nothing is cleared); per row: local vertex -> column position
        constexpr int kHash = 2048;   // > 2 * kMaxBlockElems
        std::vector<int32_t> hkey(kHash), hval(kHash), hgen(kHash, -1);
        std::vector<uint16_t> colpos;
        auto hslot = [](int32_t k) { return int((uint32_t(k) * 2654435761u) >> 21); };
        for (int b = b0; b < b1; ++b) {
            Blk &B = blks[b];
            const int32_t *rw = H.rows.data() + H.row_ptr[b];
            const int nr = H.row_ptr[b + 1] - H.row_ptr[b];
            elems.clear();
            for (int r = 0; r < nr; ++r)
                for (int64_t t = ip[rw[r]]; t < ip[rw[r] + 1]; ++t) elems.push_back(inc_k[t]);
            std::sort(elems.begin(), elems.end());
            elems.erase(std::unique(elems.begin(), elems.end()), elems.end());
            if (int(elems.size()) > kMaxBlockElems) {
                B.ok = false;
                continue;
            }
            for (int r = 0; r < nr; ++r) loc[rw[r]] = r;
            halo.clear();
            for (int32_t k : elems)
                for (int a = 0; a < NL; ++a) {
                    const int32_t v = me[int64_t(a) * nme + k];
                    if (loc[v] == -1) {
                        loc[v] = -2;
                        halo.push_back(v);
                    }
                }
            std::sort(halo.begin(), halo.end());
            B.nodes.assign(rw, rw + nr);
            for (size_t h = 0; h < halo.size(); ++h) {
                loc[halo[h]] = int32_t(nr + h);
                B.nodes.push_back(halo[h]);
            }
            if (B.nodes.size() > 65535) {
                B.ok = false;
            } else {
                B.elem.resize(elems.size() * 4, 0);
                for (size_t e = 0; e < elems.size(); ++e)
                    for (int a = 0; a < NL; ++a)
                        B.elem[e * 4 + a] = uint16_t(loc[me[int64_t(a) * nme + elems[e]]]);
                int maxdeg = 0;
                for (int r = 0; r < nr; ++r)
                    maxdeg = std::max<int>(maxdeg, int(ip[rw[r] + 1] - ip[rw[r]]));
                B.maxdeg = maxdeg;
                if (!pair_mode) B.rec.assign(size_t(maxdeg) * nr, kRecPad);
                B.wrec.assign(size_t(maxdeg) * nr, kWRecPad);
                for (size_t e = 0; e < elems.size(); ++e) {
                    int h = hslot(elems[e]);
                    while (hgen[h] == b) h = (h + 1) & (kHash - 1);
                    hgen[h] = b;
                    hkey[h] = elems[e];
                    hval[h] = int32_t(e);
                }
                colpos.resize(B.nodes.size());
                for (int r = 0; r < nr; ++r) {
                    const int32_t row = rw[r];
                    const int32_t *c0 = ci + rp[row], *c1 = ci + rp[row + 1];
                    B.nacc += c1 - c0;
                    // every column of a block row is a touched vertex of the block
                    for (const int32_t *c = c0; c < c1; ++c) colpos[loc[*c]] = uint16_t(c - c0);
                    int t = 0;
                    for (int64_t s = ip[row]; s < ip[row + 1]; ++s, ++t) {
                        const int32_t k = inc_k[s];
                        int h = hslot(k);
                        while (hgen[h] == b && hkey[h] != k) h = (h + 1) & (kHash - 1);
                        if (hgen[h] != b) {   // cannot happen: k is a block element
                            B.ok = false;
                            break;
                        }
                        uint32_t recv = uint32_t(hval[h]);
                        uint64_t wide = uint64_t(hval[h]);
                        for (int a = 0; a < NL; ++a) {
                            const int32_t v = me[int64_t(a) * nme + k];
                            recv |= uint32_t(colpos[loc[v]]) << (12 + 5 * a);
                            wide |= uint64_t(colpos[loc[v]]) << (12 + 12 * a);
                            if (v == row) {
                                recv |= uint32_t(a) << 10;
                                wide |= uint64_t(a) << 10;
                            }
                        }
                        if (!pair_mode) B.rec[size_t(t) * nr + r] = recv;
                        B.wrec[size_t(t) * nr + r] = wide;
                    }
                }
            }
            for (int32_t v : B.nodes) loc[v] = -1;
        }
    };
    run_chunks(std::min(nthreads, nb / 64 + 1), nb,
               [&](int64_t b0, int64_t b1) { work(int(b0), int(b1)); });
    // offsets of every block's lists, then the lists copied into place in
    // parallel (block order, so the result does not depend on the threads)
    H.node_ptr.assign(size_t(nb) + 1, 0);
    H.elem_ptr.assign(size_t(nb) + 1, 0);
    H.rec_ptr.assign(size_t(nb) + 1, 0);
    H.maxdeg.resize(nb);
    for (int b = 0; b < nb; ++b) {
        const Blk &B = blks[b];
        if (!B.ok) return BlockHost();
        H.node_ptr[b + 1] = H.node_ptr[b] + int32_t(B.nodes.size());
        H.elem_ptr[b + 1] = H.elem_ptr[b] + int32_t(B.elem.size() / 4);
        H.rec_ptr[b + 1] = H.rec_ptr[b] + int64_t(B.wrec.size());
        H.maxdeg[b] = B.maxdeg;
        H.max_rows = std::max(H.max_rows, H.row_ptr[b + 1] - H.row_ptr[b]);
        H.max_nodes = std::max(H.max_nodes, int(B.nodes.size()));
        H.max_elems = std::max(H.max_elems, int(B.elem.size() / 4));
        H.max_nacc = std::max(H.max_nacc, B.nacc);
    }
    H.nodes.resize(size_t(H.node_ptr[nb]));
    H.elem.resize(size_t(H.elem_ptr[nb]) * 4);
    if (!pair_mode) H.rec.resize(size_t(H.rec_ptr[nb]));
    H.wrec.resize(size_t(H.rec_ptr[nb]));
    run_chunks(std::min(nthreads, nb / 64 + 1), nb, [&](int64_t b0, int64_t b1) {
        for (int64_t b = b0; b < b1; ++b) {
            Blk &B = blks[b];
            std::copy(B.nodes.begin(), B.nodes.end(), H.nodes.begin() + H.node_ptr[b]);
            std::copy(B.elem.begin(), B.elem.end(), H.elem.begin() + size_t(H.elem_ptr[b]) * 4);
            std::copy(B.rec.begin(), B.rec.end(), H.rec.begin() + H.rec_ptr[b]);
            std::copy(B.wrec.begin(), B.wrec.end(), H.wrec.begin() + H.rec_ptr[b]);
            B = Blk();
        }
    });
    H.total_elems = H.elem_ptr.back();
    H.ok = true;
    return H;
}

// Vertex-pair work lists of the elasticity block kernel, derived from the
// incidence records of a BlockHost.  A "pair" is one CSR entry (row r of the
// block, column position p): the d x d block of the vector operator that one
// thread sums in registers.  For each pair the plan lists the block elements
// that contain both vertices, in ascending element position, as 16-bit
// entries: element position (bits 0-9), local index a of the row vertex
// (bits 10-11) and b of the column vertex (bits 12-13), or, with `tri`, the
// index of (min(a,b), max(a,b)) in the packed upper triangle of the element
// matrix (bits 10-13; symmetric operators).  Lists are padded
// with entries naming position ne (the block's element count), a dummy
// element whose scaled cofactors the kernel sets to zero.
// Pairs are sorted by list length (longest first, stable) and cut into tasks
// of 64 (one per wavefront lane); a task's entries are stored entry-major
// (entry t of lane j at t*64 + j) up to the task's longest list.  Tasks are
// dealt to kWaves wavefronts, at most kSlots each, longest-first onto the
// least-loaded wavefront, and stored wavefront by wavefront.  hdr holds, per
// task lane, r | p << 7 (0xffff for an empty lane).
// With `dedup`, a pair (r, p) whose column vertex is row r2 > r of the same
// block also stands for its mirror (r2, p2) (same elements, transposed
// block, equal for symmetric operators); the mirror is not listed and hdr2
// holds r2 | p2 << 7 for its writer (0xffff otherwise).
struct PairHost {
    std::vector<int32_t> wt;        // [nb*(kWaves+1)] first task of each wavefront (global)
    std::vector<int32_t> task_cnt;  // entries per lane of each task
    std::vector<int64_t> task_ent;  // first entry of each task (global)
    std::vector<uint16_t> hdr;      // [ntask*64]
    std::vector<uint16_t> hdr2;     // [ntask*64] mirror target (dedup)
    std::vector<uint16_t> ent;
    std::vector<int64_t> ent_ptr;   // [nb+1]
    std::vector<uint8_t> blk_ok;    // [nb] 0: the block exceeds a cap (no tasks; its rows
                                    // go to another kernel)
    int64_t max_ent = 0;
    bool ok = false;
};

constexpr uint16_t kPairPad = 0xffffu;

// The task starts of wavefronts 1..waves of one block, relative to the
// block's first task (wt[0]), packed kWaveStartBits bits each, wavefront 1 in
// the low bits.  A block holds at most waves * slots <= 8 * 4 = 32 tasks, so
// a start is at most 32 and fits the 6-bit field.
constexpr int kWaveStartBits = 6;

inline uint64_t pack_wave_starts(const int32_t *wt, int waves) {
    uint64_t wp = 0;
    for (int w = 1; w <= waves; ++w)
        wp |= uint64_t(uint32_t(wt[w] - wt[0])) << (kWaveStartBits * (w - 1));
    return wp;
}

// A block whose rows need more than kWaves * kSlots tasks, more than 128
// rows, or (max_ent > 0) more than max_ent list entries gets no tasks and
// blk_ok[b] = 0.
inline PairHost build_pair_host(const BlockHost &H, int d, const int32_t *rp, const int32_t *ci,
                                int kWaves, int kSlots, int nthreads, bool tri = false,
                                bool dedup = false, int64_t max_ent = 0) {
    PairHost P;
    const int NL = d + 1;
    const int nb = H.nb;
    struct Blk {
        std::vector<int32_t> cnt;        // per task
        std::vector<int32_t> eoff;       // per task, local entry offset
        std::vector<int32_t> wfirst;     // [kWaves+1], local task index
        std::vector<uint16_t> hdr, hdr2, ent;
        bool ok = true;
    };
    std::vector<Blk> blks(nb);
    auto work = [&](int b0, int b1) {
        std::vector<int32_t> off, lst_ptr, fill, order, mir;
        std::vector<uint16_t> lst;
        for (int b = b0; b < b1; ++b) {
            Blk &B = blks[b];
            const int32_t *rw = H.rows.data() + H.row_ptr[b];
            const int nr = H.row_ptr[b + 1] - H.row_ptr[b];
            if (nr > 128) {
                B.ok = false;
                continue;
            }
            off.assign(nr + 1, 0);
            for (int r = 0; r < nr; ++r) off[r + 1] = off[r] + rp[rw[r] + 1] - rp[rw[r]];
            const int np = off[nr];
            const uint64_t *rec = H.wrec.data() + H.rec_ptr[b];
            const int maxdeg = H.maxdeg[b];
            // list lengths, then lists (records of a row come in ascending element position)
            lst_ptr.assign(np + 1, 0);
            for (int r = 0; r < nr; ++r)
                for (int t = 0; t < maxdeg; ++t) {
                    const uint64_t x = rec[size_t(t) * nr + r];
                    if (x == kWRecPad) break;
                    for (int a = 0; a < NL; ++a)
                        lst_ptr[off[r] + int((x >> (12 + 12 * a)) & 4095u) + 1]++;
                }
            for (int q = 0; q < np; ++q) lst_ptr[q + 1] += lst_ptr[q];
            lst.assign(lst_ptr[np], 0);
            fill.assign(lst_ptr.begin(), lst_ptr.end() - 1);
            for (int r = 0; r < nr; ++r)
                for (int t = 0; t < maxdeg; ++t) {
                    const uint64_t x = rec[size_t(t) * nr + r];
                    if (x == kWRecPad) break;
                    const uint32_t ep = uint32_t(x & 1023u), al = uint32_t((x >> 10) & 3u);
                    for (int a = 0; a < NL; ++a) {
                        const int q = off[r] + int((x >> (12 + 12 * a)) & 4095u);
                        uint32_t code = (al << 10) | (uint32_t(a) << 12);
                        if (tri) {
                            const uint32_t lo = std::min<uint32_t>(al, a), hi = std::max<uint32_t>(al, a);
                            code = (lo * NL - lo * (lo - 1) / 2 + (hi - lo)) << 10;
                        }
                        lst[fill[q]++] = uint16_t(ep | code);
                    }
                }
            // mirrors: column vertex = row r2 of this block; r2 > r writes both
            mir.assign(np, -1);
            order.clear();
            for (int r = 0; r < nr; ++r) {
                const int32_t row = rw[r];
                for (int p = 0; p < off[r + 1] - off[r]; ++p) {
                    const int q = off[r] + p;
                    const int32_t c = ci[rp[row] + p];
                    const int32_t *it = std::lower_bound(rw, rw + nr, c);
                    const int r2 = (it != rw + nr && *it == c) ? int(it - rw) : -1;
                    if (dedup && r2 >= 0 && r2 < r) continue;   // written by its mirror
                    if (dedup && r2 > r) {
                        const int p2 = int(std::lower_bound(ci + rp[c], ci + rp[c + 1], row) - (ci + rp[c]));
                        mir[q] = r2 | (p2 << 7);
                    }
                    order.push_back(q);
                }
            }
            const int nlisted = int(order.size());
            std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
                return lst_ptr[x + 1] - lst_ptr[x] > lst_ptr[y + 1] - lst_ptr[y];
            });
            const int ntask = (nlisted + 63) / 64;
            if (ntask > kWaves * kSlots) {
                B.ok = false;
                continue;
            }
            // longest-first onto the least-loaded wavefront with a free slot
            std::vector<std::vector<int>> wl(kWaves);
            std::vector<int64_t> load(kWaves, 0);
            for (int t = 0; t < ntask; ++t) {
                const int q0 = order[size_t(t) * 64];
                const int c = lst_ptr[q0 + 1] - lst_ptr[q0];
                int best = -1;
                for (int w = 0; w < kWaves; ++w)
                    if (int(wl[w].size()) < kSlots && (best < 0 || load[w] < load[best])) best = w;
                wl[best].push_back(t);
                load[best] += c;
            }
            // list entries of the block (each task stores its longest list 64 times)
            if (max_ent > 0) {
                int64_t nent = 0;
                for (int t = 0; t < ntask; ++t) {
                    const int q0 = order[size_t(t) * 64];
                    nent += int64_t(lst_ptr[q0 + 1] - lst_ptr[q0]) * 64;
                }
                if (nent > max_ent) {
                    B.ok = false;
                    continue;
                }
            }
            B.wfirst.push_back(0);
            for (int w = 0; w < kWaves; ++w) {
                for (int t : wl[w]) {
                    const int q0 = order[size_t(t) * 64];
                    const int c = lst_ptr[q0 + 1] - lst_ptr[q0];
                    B.cnt.push_back(c);
                    B.eoff.push_back(int32_t(B.ent.size()));
                    const size_t e0 = B.ent.size();
                    B.ent.resize(e0 + size_t(c) * 64, uint16_t(H.elem_ptr[b + 1] - H.elem_ptr[b]));
                    for (int j = 0; j < 64; ++j) {
                        const int k = t * 64 + j;
                        if (k >= nlisted) {
                            B.hdr.push_back(kPairPad);
                            B.hdr2.push_back(kPairPad);
                            continue;
                        }
                        const int q = order[k];
                        const int r = int(std::upper_bound(off.begin(), off.end(), q) - off.begin()) - 1;
                        B.hdr.push_back(uint16_t(r | ((q - off[r]) << 7)));
                        B.hdr2.push_back(mir[q] >= 0 ? uint16_t(mir[q]) : kPairPad);
                        for (int u = lst_ptr[q]; u < lst_ptr[q + 1]; ++u)
                            B.ent[e0 + size_t(u - lst_ptr[q]) * 64 + j] = lst[u];
                    }
                }
                B.wfirst.push_back(int32_t(B.cnt.size()));
            }
        }
    };
    run_chunks(std::min(nthreads, nb / 64 + 1), nb,
               [&](int64_t b0, int64_t b1) { work(int(b0), int(b1)); });
    // task and entry offsets of every block, then the lists copied into
    // place in parallel (block order)
    std::vector<int64_t> tptr(size_t(nb) + 1, 0);
    P.ent_ptr.assign(size_t(nb) + 1, 0);
    P.blk_ok.assign(size_t(nb), 1);
    for (int b = 0; b < nb; ++b) {
        Blk &B = blks[b];
        if (!B.ok) {   // no tasks: its rows are assembled elsewhere
            P.blk_ok[b] = 0;
            B = Blk();
            B.wfirst.assign(size_t(kWaves) + 1, 0);
        }
        tptr[b + 1] = tptr[b] + int64_t(B.cnt.size());
        P.ent_ptr[b + 1] = P.ent_ptr[b] + int64_t(B.ent.size());
        P.max_ent = std::max<int64_t>(P.max_ent, int64_t(B.ent.size()));
    }
    if (tptr[nb] >= (int64_t(1) << 31)) return PairHost();
    P.wt.resize(size_t(nb) * (kWaves + 1));
    P.task_cnt.resize(size_t(tptr[nb]));
    P.task_ent.resize(size_t(tptr[nb]));
    P.hdr.resize(size_t(tptr[nb]) * 64);
    P.hdr2.resize(size_t(tptr[nb]) * 64);
    P.ent.resize(size_t(P.ent_ptr[nb]));
    run_chunks(std::min(nthreads, nb / 64 + 1), nb, [&](int64_t b0, int64_t b1) {
        for (int64_t b = b0; b < b1; ++b) {
            Blk &B = blks[b];
            const int32_t t0 = int32_t(tptr[b]);
            const int64_t e0 = P.ent_ptr[b];
            for (int w = 0; w <= kWaves; ++w) P.wt[size_t(b) * (kWaves + 1) + w] = t0 + B.wfirst[w];
            for (size_t u = 0; u < B.cnt.size(); ++u) {
                P.task_cnt[size_t(t0) + u] = B.cnt[u];
                P.task_ent[size_t(t0) + u] = e0 + B.eoff[u];
            }
            std::copy(B.hdr.begin(), B.hdr.end(), P.hdr.begin() + size_t(t0) * 64);
            std::copy(B.hdr2.begin(), B.hdr2.end(), P.hdr2.begin() + size_t(t0) * 64);
            std::copy(B.ent.begin(), B.ent.end(), P.ent.begin() + e0);
            B = Blk();
        }
    });
    P.ok = true;
    return P;
}

}  // namespace femasm
