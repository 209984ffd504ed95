// Host side of the P_k mass assembly (Appendix D): local node numbering, the
// coefficient matrix C, and the plan layout read by the kernels of pk.hip.
// Plain C++ (no HIP), so the layout can be checked on the CPU.
//
// Local numbering of an element's N = (d+k)!/(d! k!) nodes: the
// multi-indices alpha in N^(d+1) with |alpha| = k (alpha_i is the exponent of
// the barycentric coordinate of local vertex i); local nodes 0..d are the
// vertices alpha = k e_i, the others follow in decreasing lexicographic order
// of (alpha_0, ..., alpha_d).
//
// Layout (build_pk_host):
//   rp, ci        CSR pattern: row i holds every node sharing an element with
//                 node i, columns ascending
//   CSR entries are cut into tiles of kPkTile consecutive entries.
//   tile_item[t]  first contribution item of tile t (its items are
//                 tile_item[t] .. tile_item[t+1]-1)
//   coff[s]       first item of entry s, relative to tile_item[t]
//   item[u]       one contribution: element number (bits 0 .. ebits-1) |
//                 index of (min(a,b), max(a,b)) in the packed upper triangle
//                 of C (bits ebits .. 31), a and b the local nodes of the row
//                 and column node; ebits = 32 - (bits of ntri-1), and the
//                 items of an entry are in ascending element number
//   ctri          packed upper triangle of C (row-major, a <= b)
#pragma once

#include <algorithm>
#include <array>
#include <atomic>
#include <cstdint>
#include <map>
#include <thread>
#include <vector>

#include "host_threads.h"
#include "symbolic_host.h"

namespace femasm {

constexpr int kPkMaxK = 6;
constexpr int kPkThreads = 256;        // threads of a k_pk_mass workgroup
constexpr int kPkPer = 4;              // CSR entries per thread and tile
constexpr int kPkTile = kPkThreads * kPkPer;   // CSR entries per tile

using PkMono = std::array<int, 4>;
using PkPoly = std::map<PkMono, __int128>;

// Local nodes of a d-simplex (d = 1, 2, 3) in the numbering above.
inline std::vector<PkMono> pk_nodes(int d, int k) {
    std::vector<PkMono> all, out;
    // every composition of k into d+1 parts, decreasing lexicographic
    PkMono cur{0, 0, 0, 0};
    auto rec = [&](auto &&self, int i, int left) -> void {
        if (i == d) {
            cur[i] = left;
            all.push_back(cur);
            return;
        }
        for (int a = left; a >= 0; --a) {
            cur[i] = a;
            self(self, i + 1, left - a);
        }
    };
    rec(rec, 0, k);
    for (int v = 0; v <= d; ++v) {
        PkMono a{0, 0, 0, 0};
        a[v] = k;
        out.push_back(a);
    }
    for (const PkMono &m : all)
        if (std::find(out.begin(), out.begin() + d + 1, m) == out.begin() + d + 1) out.push_back(m);
    return out;
}

inline __int128 pk_fact(int n) {
    __int128 f = 1;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

// alpha! phi_alpha as a polynomial in the barycentric coordinates: the
// product over l of prod_{j < alpha_l} (k lambda_l - j).
inline PkPoly pk_scaled_basis(int d, int k, const PkMono &alpha) {
    PkPoly p;
    p[PkMono{0, 0, 0, 0}] = 1;
    for (int l = 0; l <= d; ++l)
        for (int j = 0; j < alpha[l]; ++j) {
            PkPoly r;
            for (const auto &t : p) {
                PkMono up = t.first;
                up[l] += 1;
                r[up] += t.second * k;              // k lambda_l term
                if (j) r[t.first] -= t.second * j;  // -j term
            }
            p.swap(r);
        }
    return p;
}

// Packed upper triangle of C, C[a][b] = int_K phi_a phi_b / (d! |K|), from
// the magic formula int_K lambda^m = d! |K| m! / (d + |m|)!, evaluated in
// integers over the denominator (d+2k)! alpha! beta! and rounded once.
inline std::vector<double> pk_ctri(int d, int k) {
    const std::vector<PkMono> nodes = pk_nodes(d, k);
    const int n = int(nodes.size());
    std::vector<PkPoly> P(n);
    for (int a = 0; a < n; ++a) P[a] = pk_scaled_basis(d, k, nodes[a]);
    const __int128 top = pk_fact(d + 2 * k);
    std::vector<double> out;
    out.reserve(size_t(n) * (n + 1) / 2);
    for (int a = 0; a < n; ++a)
        for (int b = a; b < n; ++b) {
            __int128 num = 0;
            for (const auto &x : P[a])
                for (const auto &y : P[b]) {
                    int deg = 0;
                    __int128 f = 1;
                    for (int i = 0; i <= d; ++i) {
                        f *= pk_fact(x.first[i] + y.first[i]);
                        deg += x.first[i] + y.first[i];
                    }
                    num += x.second * y.second * f * (top / pk_fact(d + deg));
                }
            __int128 den = top;
            for (int i = 0; i <= d; ++i) den *= pk_fact(nodes[a][i]) * pk_fact(nodes[b][i]);
            out.push_back(double(static_cast<long double>(num) / static_cast<long double>(den)));
        }
    return out;
}

inline int pk_tri_index(int n, int a, int b) {
    const int lo = std::min(a, b), hi = std::max(a, b);
    return lo * n - lo * (lo - 1) / 2 + (hi - lo);
}

template <class F>
void pk_parallel(int64_t n, int nthreads, F fn) {
    const int nt = std::max(1, nthreads);
    if (n < 4096 || nt == 1) {
        fn(int64_t(0), n);
        return;
    }
    run_chunks(nt, n, fn);
}

// Bits of an item that hold the element number, for n local nodes.
inline int pk_ebits(int n) {
    const int ntri = n * (n + 1) / 2;
    int cbits = 1;
    while ((1 << cbits) < ntri) ++cbits;
    return 32 - cbits;
}

struct PkHost {
    int status = 0;   // 0 ok, 2 bad index / repeated node, 4 overflow
    int n = 0, ntri = 0, ebits = 0;
    int64_t nnz = 0, ntiles = 0;
    int max_tile_items = 0;
    std::vector<int32_t> rp, ci;
    std::vector<int64_t> tile_item;
    std::vector<uint16_t> coff;
    std::vector<uint32_t> item;
    std::vector<double> ctri;
};

// me: host, N x nme (row-major, me[a*nme + e]); d is the simplex dimension
// (1 for boundary segments, 2 for boundary triangles or 2D meshes, 3).
inline PkHost build_pk_host(int d, int k, int64_t nq, int64_t nme, const int32_t *me,
                            int nthreads) {
    PkHost H;
    const int n = int(pk_nodes(d, k).size());
    H.n = n;
    H.ntri = n * (n + 1) / 2;
    H.ebits = pk_ebits(n);
    if (nme > (int64_t(1) << H.ebits)) {
        H.status = 4;
        return H;
    }
    auto node = [&](int a, int64_t e) { return me[size_t(a) * nme + e]; };

    // validation: indices in range, no node repeated within an element
    std::atomic<int> bad{0};
    pk_parallel(nme, nthreads, [&](int64_t b, int64_t e) {
        std::vector<int32_t> v(n);
        for (int64_t x = b; x < e && !bad.load(std::memory_order_relaxed); ++x) {
            for (int a = 0; a < n; ++a) {
                v[a] = node(a, x);
                if (v[a] < 0 || v[a] >= nq) bad = 1;
            }
            std::sort(v.begin(), v.end());
            if (std::adjacent_find(v.begin(), v.end()) != v.end()) bad = 1;
        }
    });
    if (bad) {
        H.status = 2;
        return H;
    }

    // incidences node -> (element, local node), ascending element: the
    // element slots e*n+a sorted stably by their node
    std::vector<int64_t> ip;
    std::vector<int32_t> inc_e(size_t(n) * nme);
    std::vector<uint8_t> inc_a(size_t(n) * nme);
    stable_key_sort(
        int64_t(n) * nme, nq, nthreads, [&](int64_t r) { return int64_t(node(int(r % n), r / n)); },
        [&](int64_t pos, int64_t r) {
            inc_e[pos] = int32_t(r / n);
            inc_a[pos] = uint8_t(r % n);
        },
        ip);

    // pattern: row i = sorted distinct nodes of the elements around i, and
    // the number of contributions of every entry.  One sort per row: each
    // thread keeps the columns and counts of its contiguous row range until
    // the row offsets are known, then copies them into place.
    std::vector<int32_t> rowlen(nq, 0);
    const int nrt = nq < 4096 ? 1 : std::max(1, nthreads);
    const int64_t rchunk = (nq + nrt - 1) / nrt;
    std::vector<std::vector<int32_t>> tcols(nrt), tcnt(nrt);
    {
        auto rows_of = [&](int t) {
            std::vector<int32_t> buf;
            for (int64_t i = t * rchunk, e = std::min(nq, (t + 1) * rchunk); i < e; ++i) {
                buf.clear();
                for (int64_t u = ip[i]; u < ip[i + 1]; ++u)
                    for (int b = 0; b < n; ++b) buf.push_back(node(b, inc_e[u]));
                std::sort(buf.begin(), buf.end());
                buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
                rowlen[i] = int32_t(buf.size());
                const size_t base = tcols[t].size();
                tcols[t].insert(tcols[t].end(), buf.begin(), buf.end());
                tcnt[t].resize(base + buf.size(), 0);
                for (int64_t u = ip[i]; u < ip[i + 1]; ++u)
                    for (int bb = 0; bb < n; ++bb) {
                        const int32_t j = node(bb, inc_e[u]);
                        tcnt[t][base + (std::lower_bound(buf.begin(), buf.end(), j) - buf.begin())] += 1;
                    }
            }
        };
        run_threads(nrt, rows_of);
    }
    H.rp.assign(nq + 1, 0);
    int64_t nnz = 0;
    for (int64_t i = 0; i < nq; ++i) {
        H.rp[i] = int32_t(nnz);
        nnz += rowlen[i];
        if (nnz >= (int64_t(1) << 31)) {
            H.status = 4;
            return H;
        }
    }
    H.rp[nq] = int32_t(nnz);
    H.nnz = nnz;

    // contributions of every entry, ascending element: (element, tri code)
    H.ci.assign(nnz, 0);
    std::vector<int64_t> cptr(nnz + 1, 0);
    run_threads(nrt, [&](int t) {
        if (tcols[t].empty()) return;
        const int64_t o = H.rp[std::min(nq, t * rchunk)];
        std::copy(tcols[t].begin(), tcols[t].end(), H.ci.begin() + o);
        for (size_t x = 0; x < tcnt[t].size(); ++x) cptr[o + int64_t(x) + 1] = tcnt[t][x];
        std::vector<int32_t>().swap(tcols[t]);
        std::vector<int32_t>().swap(tcnt[t]);
    });
    for (int64_t s = 0; s < nnz; ++s) cptr[s + 1] += cptr[s];
    const int64_t ncontrib = cptr[nnz];
    std::vector<int32_t> celem(ncontrib);
    std::vector<uint16_t> ccode(ncontrib);
    pk_parallel(nq, nthreads, [&](int64_t b, int64_t e) {
        std::vector<int64_t> fill;
        for (int64_t i = b; i < e; ++i) {
            const int32_t *c0 = H.ci.data() + H.rp[i], *c1 = H.ci.data() + H.rp[i + 1];
            fill.assign(cptr.begin() + H.rp[i], cptr.begin() + H.rp[i + 1]);
            for (int64_t t = ip[i]; t < ip[i + 1]; ++t) {
                const int32_t x = inc_e[t];
                const int a = inc_a[t];
                for (int bb = 0; bb < n; ++bb) {
                    const int64_t pos = std::lower_bound(c0, c1, node(bb, x)) - c0;
                    const int64_t u = fill[pos]++;
                    celem[u] = x;
                    ccode[u] = uint16_t(pk_tri_index(n, a, bb));
                }
            }
        }
    });

    // tiles of kPkTile entries: tile-relative item offsets, packed items
    const int64_t ntiles = (nnz + kPkTile - 1) / kPkTile;
    H.ntiles = ntiles;
    H.tile_item.assign(ntiles + 1, 0);
    H.coff.assign(size_t(ntiles) * kPkTile, 0);
    H.item.assign(ncontrib, 0);
    for (int64_t t = 0; t <= ntiles; ++t) {
        H.tile_item[t] = cptr[std::min<int64_t>(nnz, t * kPkTile)];
        if (t > 0) {
            const int64_t c = H.tile_item[t] - H.tile_item[t - 1];
            if (c > 65535) {
                H.status = 4;
                return H;
            }
            H.max_tile_items = std::max(H.max_tile_items, int(c));
        }
    }
    for (int64_t s = 0; s < nnz; ++s) H.coff[s] = uint16_t(cptr[s] - H.tile_item[s / kPkTile]);
    pk_parallel(ncontrib, nthreads, [&](int64_t b, int64_t e) {
        for (int64_t u = b; u < e; ++u)
            H.item[u] = uint32_t(celem[u]) | (uint32_t(ccode[u]) << H.ebits);
    });
    H.ctri = pk_ctri(d, k);
    return H;
}

}  // namespace femasm
