// Thread helpers of the host-side plan builders.  Every builder thread is
// joined before the helper returns, and an exception thrown on any of them
// (std::bad_alloc for a very large mesh) is rethrown on the calling thread,
// where the library's entry points turn it into a status code.
#pragma once

#include <algorithm>
#include <cstdint>
#include <exception>
#include <thread>
#include <vector>

namespace femasm {

// fn(t) for t = 0..nt-1, t = 0 on the calling thread.  If a thread cannot be
// started, its index runs on the calling thread instead.  After all have
// finished, the exception of the lowest index that threw is rethrown.
template <class F>
void run_threads(int nt, F fn) {
    nt = std::max(1, nt);
    std::vector<std::exception_ptr> err(static_cast<size_t>(nt));
    auto guarded = [&](int t) {
        try {
            fn(t);
        } catch (...) {
            err[size_t(t)] = std::current_exception();
        }
    };
    std::vector<std::thread> th;
    int started = 1;
    try {
        th.reserve(size_t(nt - 1));
        for (; started < nt; ++started) th.emplace_back(guarded, started);
    } catch (...) {
        // fewer threads than asked for: the rest run below
    }
    guarded(0);
    for (int t = started; t < nt; ++t) guarded(t);
    for (auto &x : th) x.join();
    for (auto &e : err)
        if (e) std::rethrow_exception(e);
}

// fn(b, e) over [0, n) cut into nt contiguous chunks (empty chunks skipped).
template <class F>
void run_chunks(int nt, int64_t n, F fn) {
    nt = int(std::max<int64_t>(1, std::min<int64_t>(nt, n)));
    const int64_t chunk = (n + nt - 1) / nt;
    run_threads(nt, [&](int t) {
        const int64_t b = t * chunk, e = std::min(n, b + chunk);
        if (b < e) fn(b, e);
    });
}

}  // namespace femasm
