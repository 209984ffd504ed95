// Test shim: exposes the host-side P_k plan builder of the library
// (paper_1401_3301_amd/csrc/pk_host.h) through a C interface so that
// tests/test_pk_host.py can check it on the CPU.  Not part of the library.
#include <cstdint>
#include <cstring>

#include "../paper_1401_3301_amd/csrc/pk_host.h"

using namespace femasm;

static PkHost g_h;

extern "C" int pkh_build(int d, int k, int64_t nq, int64_t nme, const int32_t *me, int64_t *sizes) {
    g_h = build_pk_host(d, k, nq, nme, me, 2);
    if (g_h.status) return g_h.status;
    sizes[0] = g_h.nnz;
    sizes[1] = g_h.ntiles;
    sizes[2] = int64_t(g_h.item.size());
    sizes[3] = g_h.ebits;
    sizes[4] = g_h.ntri;
    sizes[5] = g_h.max_tile_items;
    return 0;
}

template <class T>
static void put(void *dst, const std::vector<T> &v) {
    if (!v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(T));
}

extern "C" void pkh_get(int32_t *rp, int32_t *ci, int64_t *tile_item, uint16_t *coff,
                        uint32_t *item, double *ctri) {
    put(rp, g_h.rp);
    put(ci, g_h.ci);
    put(tile_item, g_h.tile_item);
    put(coff, g_h.coff);
    put(item, g_h.item);
    put(ctri, g_h.ctri);
}
