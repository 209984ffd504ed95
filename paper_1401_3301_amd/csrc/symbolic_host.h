// Host-side integer steps of the symbolic phase that are shared by more than
// one plan builder: a parallel, stable counting sort of records by an integer
// key.  The symbolic phase uses it twice: for the vertex -> (element, local
// vertex) incidence lists (records = element slots k*(d+1)+a, key = the
// vertex, so each vertex's incidences come out in ascending element number)
// and for the locality order of the elements (records = elements, key = the
// smallest vertex id, ties in ascending element number).
#pragma once

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <vector>

#include "host_threads.h"

namespace femasm {

// Sorts the records 0..n-1 by key(r) in [0, nkeys), stably (records with
// equal keys keep ascending r), calling emit(pos, r) once per record with its
// position in the sorted order, and fills ptr[0..nkeys] with the first
// position of every key (ptr[nkeys] = n).  Two levels: records are first
// scattered into buckets of 2^S consecutive keys (per-thread counts over
// contiguous record chunks, so a bucket holds its records in ascending r),
// then every bucket is counting-sorted by the low S bits of the key.  Work
// and memory are O(n + nkeys); the scratch is one uint32 per record, so
// n must stay below 2^32.
template <class KeyF, class EmitF>
void stable_key_sort(int64_t n, int64_t nkeys, int nthreads, KeyF key, EmitF emit,
                     std::vector<int64_t> &ptr) {
    ptr.assign(size_t(nkeys) + 1, 0);
    if (n == 0 || nkeys == 0) return;
    int S = 6;
    while ((nkeys >> S) > 4096 && S < 24) ++S;
    const int64_t nbk = ((nkeys - 1) >> S) + 1;
    const int T = int(std::max<int64_t>(1, std::min<int64_t>(nthreads, n / 65536 + 1)));
    const int64_t chunk = (n + T - 1) / T;
    std::vector<int64_t> cnt(size_t(T) * nbk, 0);   // [thread][bucket]
    run_threads(T, [&](int t) {
        int64_t *c = cnt.data() + size_t(t) * nbk;
        for (int64_t r = t * chunk, e = std::min(n, r + chunk); r < e; ++r) c[key(r) >> S] += 1;
    });
    // bucket-major, then thread order: the start of (bucket, thread)
    std::vector<int64_t> bstart(size_t(nbk) + 1, 0);
    {
        int64_t o = 0;
        for (int64_t b = 0; b < nbk; ++b) {
            bstart[b] = o;
            for (int t = 0; t < T; ++t) {
                const int64_t x = cnt[size_t(t) * nbk + b];
                cnt[size_t(t) * nbk + b] = o;
                o += x;
            }
        }
        bstart[nbk] = o;
    }
    std::vector<uint32_t> tmp(static_cast<size_t>(n));
    run_threads(T, [&](int t) {
        int64_t *c = cnt.data() + size_t(t) * nbk;
        for (int64_t r = t * chunk, e = std::min(n, r + chunk); r < e; ++r)
            tmp[c[key(r) >> S]++] = uint32_t(r);
    });
    // buckets: counting sort by the low key bits, handed out dynamically
    std::atomic<int64_t> next{0};
    const int TB = int(std::max<int64_t>(1, std::min<int64_t>(nthreads, nbk)));
    run_threads(TB, [&](int) {
        std::vector<int64_t> h(size_t(1) << S);
        for (int64_t b; (b = next.fetch_add(1)) < nbk;) {
            const int64_t k0 = b << S, k1 = std::min(nkeys, k0 + (int64_t(1) << S));
            std::fill(h.begin(), h.end(), 0);
            for (int64_t i = bstart[b]; i < bstart[b + 1]; ++i) h[key(tmp[i]) - k0] += 1;
            int64_t o = bstart[b];
            for (int64_t k = k0; k < k1; ++k) {
                ptr[k] = o;
                const int64_t x = h[k - k0];
                h[k - k0] = o;
                o += x;
            }
            for (int64_t i = bstart[b]; i < bstart[b + 1]; ++i) {
                const int64_t r = tmp[i];
                emit(h[key(r) - k0]++, r);
            }
        }
    });
    ptr[nkeys] = n;
}

}  // namespace femasm
