"""The library's host-side plan builders (blocks_host.h, pk_host.h,
symbolic_host.h) under ThreadSanitizer (the parallel block growth over
vertex-id chunks, the per-block list builders and the parallel key sort)
and AddressSanitizer + UBSan, on the CPU.  The
shims are compiled with g++ for the host only; each sanitized build runs a
small driver over meshes that exercise several chunks."""
import os
import shutil
import subprocess
import textwrap

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1401_3301_amd", "csrc")

DRIVER = textwrap.dedent(r"""
    #include <cstdio>
    #include <cstdint>
    #include <vector>
    #include <algorithm>
    #include "blocks_host.h"
    #include "pk_host.h"
    #include "symbolic_host.h"
    using namespace femasm;
    // Kuhn cube of n^3 cubes: connectivity, CSR pattern and incidences
    static void kuhn(int n, std::vector<int32_t> &me, int64_t &nq, int64_t &nme) {
        const int n1 = n + 1;
        nq = int64_t(n1) * n1 * n1;
        nme = 6LL * n * n * n;
        me.assign(4 * nme, 0);
        const int perm[6][3] = {{0,1,2},{0,2,1},{1,0,2},{1,2,0},{2,0,1},{2,1,0}};
        const int step[3] = {1, n1, n1 * n1};
        int64_t e = 0;
        for (int k = 0; k < n; ++k) for (int j = 0; j < n; ++j) for (int i = 0; i < n; ++i) {
            const int base = (k * n1 + j) * n1 + i;
            for (int t = 0; t < 6; ++t, ++e) {
                const int v1 = base + step[perm[t][0]], v2 = v1 + step[perm[t][1]];
                const int v3 = base + 1 + n1 + n1 * n1;
                me[0 * nme + e] = base; me[1 * nme + e] = v1; me[2 * nme + e] = v2; me[3 * nme + e] = v3;
            }
        }
    }
    int main() {
        std::vector<int32_t> me;
        int64_t nq, nme;
        kuhn(12, me, nq, nme);
        std::vector<int64_t> ip(nq + 1, 0);
        for (int64_t e = 0; e < nme; ++e) for (int a = 0; a < 4; ++a) ip[me[a * nme + e] + 1]++;
        for (int64_t i = 0; i < nq; ++i) ip[i + 1] += ip[i];
        std::vector<int32_t> inc(ip[nq]);
        std::vector<int64_t> fill(ip.begin(), ip.end() - 1);
        for (int64_t e = 0; e < nme; ++e) for (int a = 0; a < 4; ++a) inc[fill[me[a * nme + e]]++] = int32_t(e);
        std::vector<int32_t> rp(nq + 1, 0), ci;
        for (int64_t i = 0; i < nq; ++i) {
            std::vector<int32_t> cols;
            for (int64_t t = ip[i]; t < ip[i + 1]; ++t) for (int a = 0; a < 4; ++a) cols.push_back(me[a * nme + inc[t]]);
            std::sort(cols.begin(), cols.end());
            cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
            ci.insert(ci.end(), cols.begin(), cols.end());
            rp[i + 1] = int32_t(ci.size());
        }
        int bad = 0;
        for (int chunk_min : {8192, 200}) {
            BlockHost H = build_block_host(3, nq, nme, me.data(), rp.data(), ci.data(), ip.data(),
                                           inc.data(), 56, 8, 1024, 256, chunk_min, 700);
            PairHost P = build_pair_host(H, 3, rp.data(), ci.data(), 8, 2, 8, true, true);
            if (!H.ok || !P.ok) bad = 1;
            std::printf("blocks %d (chunk_min %d) tasks %zu\n", H.nb, chunk_min, P.task_cnt.size());
        }
        // the parallel stable key sort: incidences as the symbolic phase
        // builds them (against the serial ones above), then a large random
        // key set over several threads and buckets
        {
            std::vector<int64_t> ptr;
            std::vector<int32_t> inc2(4 * nme);
            stable_key_sort(4 * nme, nq, 8, [&](int64_t r) { return int64_t(me[(r % 4) * nme + r / 4]); },
                            [&](int64_t pos, int64_t r) { inc2[pos] = int32_t(r / 4); }, ptr);
            if (inc2 != inc || ptr != ip) bad = 1;
            const int64_t n = 400000, nk = 1500000;
            std::vector<int64_t> keys(n), order(n, -1);
            uint64_t x = 88172645463325252ull;
            for (auto &k : keys) { x ^= x << 13; x ^= x >> 7; x ^= x << 17; k = int64_t(x % nk); }
            stable_key_sort(n, nk, 8, [&](int64_t r) { return keys[r]; },
                            [&](int64_t pos, int64_t r) { order[pos] = r; }, ptr);
            for (int64_t i = 1; i < n; ++i)
                if (keys[order[i - 1]] > keys[order[i]] ||
                    (keys[order[i - 1]] == keys[order[i]] && order[i - 1] > order[i])) { bad = 1; break; }
            std::printf("key sort ok %d\n", bad == 0);
        }
        // P_k plan on the same connectivity read as P1 (k = 1)
        PkHost K = build_pk_host(3, 1, nq, nme, me.data(), 8);
        if (K.status) bad = 1;
        std::printf("pk nnz %ld\n", long(K.nnz));
        // more than 4096 nodes: the multi-threaded row passes of the P_k builder
        kuhn(16, me, nq, nme);
        PkHost K2 = build_pk_host(3, 1, nq, nme, me.data(), 8);
        if (K2.status || K2.nnz != K2.rp.back()) bad = 1;
        return bad;
    }
""")


def _run(tmp_path, flags, env=None):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    src = tmp_path / "driver.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-pthread", *flags, "-I", CSRC, str(src), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitizer" in (r.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr[-2000:]
    e = dict(os.environ)
    e.update(env or {})
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=e, timeout=600)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "blocks" in r.stdout
    return r


def test_thread_sanitizer(tmp_path):
    r = _run(tmp_path, ["-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1"})
    assert "WARNING: ThreadSanitizer" not in r.stderr


def test_address_and_undefined_sanitizers(tmp_path):
    _run(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
         {"ASAN_OPTIONS": "detect_leaks=1"})
