// Symbolic phase on the GPU: validation, per-vertex incidence lists, the
// element locality order, the CSR pattern of `sparse` (Section 3: row i holds
// every vertex that shares an element with vertex i, columns ascending and
// unique) and, for every incidence, the positions of its element's vertices
// inside the row.
//
//   1. incidences: element slots r = k(d+1) + a keyed by their vertex
//      me[a,k] and radix-sorted stably, so each vertex lists its incidences
//      in ascending caller element number; the first position of every
//      vertex comes from the boundaries of the sorted keys;
//   2. element order: elements radix-sorted stably by their smallest vertex
//      id (plan order), with the plan-order connectivity gathered;
//   3. rows: the candidates of row i are the d+1 vertices of each of its
//      incident elements.  One wavefront per row holds up to 256 of them in
//      registers and marks every candidate that repeats an earlier one
//      (an all-pairs comparison through lane shuffles); the remaining
//      "first occurrences" are the row's columns.  A counting pass gives the
//      row lengths, a scan the row pointer, and a filling pass the rank of
//      every candidate among the distinct values (its column position),
//      which it writes as the column list and as the incidence's positions.
//      Longer rows take one workgroup each, candidates in LDS.
// Every step is deterministic: the sorts are stable, ranks depend only on
// values, and the few atomics only count.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstring>
#include <vector>

#include "femasm_impl.h"

namespace femasm {

namespace {

constexpr int kPatWG = 256;
constexpr int kRowSlots = 4;                 // candidates per lane in the wavefront pass
constexpr int kRowCap = 64 * kRowSlots;      // longest candidate list of the wavefront pass
constexpr int kLongCap = 16384;              // ... of the workgroup pass (64 KB of LDS)

__global__ void k_validate(const int32_t *__restrict__ me, int64_t nme, int NL, int64_t nq,
                           int32_t *__restrict__ flag) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= nme) return;
    int32_t v[4];
    int bad = 0;
    for (int a = 0; a < NL; ++a) {
        v[a] = me[int64_t(a) * nme + k];
        if (v[a] < 0 || v[a] >= nq) bad = 1;
        for (int c = 0; c < a; ++c)
            if (v[c] == v[a]) bad = 1;
    }
    if (bad) atomicOr(flag, 1);
}

// slot r = k*NL + a -> (vertex, r)
__global__ void k_slot_keys(const int32_t *__restrict__ me, int64_t nme, int NL,
                            uint32_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= int64_t(NL) * nme) return;
    const int64_t k = r / NL, a = r - k * NL;
    keys[r] = uint32_t(me[a * nme + k]);
    vals[r] = uint32_t(r);
}

// element k -> (smallest vertex id, k)
__global__ void k_elem_keys(const int32_t *__restrict__ me, int64_t nme, int NL,
                            uint32_t *__restrict__ keys, uint32_t *__restrict__ vals) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= nme) return;
    int32_t m = me[k];
    for (int a = 1; a < NL; ++a) m = min(m, me[int64_t(a) * nme + k]);
    keys[k] = uint32_t(m);
    vals[k] = uint32_t(k);
}

// ptr[v] = first position t of the sorted keys with key >= v (v = 0..nkeys):
// thread t writes the keys in (key[t-1], key[t]], thread n those after the last.
__global__ void k_key_bounds(const uint32_t *__restrict__ skeys, int64_t n, int64_t nkeys,
                             int32_t *__restrict__ ptr) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t > n) return;
    const int64_t lo = t == 0 ? 0 : int64_t(skeys[t - 1]) + 1;
    const int64_t hi = t == n ? nkeys : int64_t(skeys[t]);
    for (int64_t v = lo; v <= hi; ++v) ptr[v] = int32_t(t);
}

// plan order: porig[q] = caller element, pinv its inverse, pme element-major
__global__ void k_elem_order(const uint32_t *__restrict__ order, int64_t nme, int NL,
                             const int32_t *__restrict__ me, int32_t *__restrict__ porig,
                             int32_t *__restrict__ pinv, int32_t *__restrict__ pme) {
    const int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= nme) return;
    const int64_t k = order[q];
    porig[q] = int32_t(k);
    pinv[k] = int32_t(q);
    for (int a = 0; a < NL; ++a) pme[q * NL + a] = me[int64_t(a) * nme + k];
}

__global__ void k_inc_elem(const uint32_t *__restrict__ sslot, int64_t n, int NL,
                           const int32_t *__restrict__ pinv, uint32_t *__restrict__ inc_elem) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const uint32_t r = sslot[t];
    const uint32_t k = r / uint32_t(NL), a = r - k * uint32_t(NL);
    inc_elem[t] = uint32_t(pinv[k]) | (a << 30);
}

// Candidate u of row i: vertex b = u mod NL of the row's incidence u / NL,
// read from the plan-order connectivity (an element's vertices are
// contiguous there, and the elements around a vertex lie close together in
// plan order; the caller's layout would cost d+1 scattered reads).
__device__ __forceinline__ uint32_t candidate(const int32_t *__restrict__ pme, int NL,
                                              const uint32_t *__restrict__ inc_elem, int64_t t0,
                                              int u) {
    const int s = u / NL, b = u - s * NL;
    const int64_t q = inc_elem[t0 + s] & 0x3fffffffu;
    return uint32_t(pme[q * NL + b]);
}

// One wavefront per row (rows with at most kRowCap candidates).  Count pass:
// rowlen[i] = number of distinct candidates; rows beyond the cap are listed in
// `longrows` for the workgroup pass.  Fill pass: ci and the 16-bit positions.
template <bool FILL>
__global__ void __launch_bounds__(kPatWG)
    k_row_pattern(const int32_t *__restrict__ pme, int NL, int64_t nq,
                  const int32_t *__restrict__ ip, const uint32_t *__restrict__ inc_elem,
                  int64_t *__restrict__ rowlen, const int64_t *__restrict__ rp64,
                  int32_t *__restrict__ ci, uint16_t *__restrict__ pos16,
                  int32_t *__restrict__ longrows, int32_t *__restrict__ nlong) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = int64_t(gridDim.x) * (kPatWG / 64);
    for (int64_t i = int64_t(blockIdx.x) * (kPatWG / 64) + (threadIdx.x >> 6); i < nq; i += waves) {
        const int64_t t0 = ip[i];
        const int n = NL * (ip[i + 1] - ip[i]);
        if (n > kRowCap) {
            if (!FILL && lane == 0) {
                rowlen[i] = 0;
                longrows[atomicAdd(nlong, 1)] = int32_t(i);
            }
            continue;
        }
        uint32_t c[kRowSlots];
        bool dup[kRowSlots];
#pragma unroll
        for (int s = 0; s < kRowSlots; ++s) {
            const int u = lane + 64 * s;
            c[s] = u < n ? candidate(pme, NL, inc_elem, t0, u) : 0xffffffffu;
            dup[s] = false;
        }
        // dup: an earlier candidate has the same vertex
#pragma unroll
        for (int js = 0; js < kRowSlots; ++js) {
            if (64 * js >= n) break;
            const int jn = min(64, n - 64 * js);
            for (int jl = 0; jl < jn; ++jl) {
                const uint32_t y = __shfl(c[js], jl, 64);
                const int j = 64 * js + jl;
#pragma unroll
                for (int s = 0; s < kRowSlots; ++s) dup[s] |= (y == c[s]) & (j < lane + 64 * s);
            }
        }
        uint64_t first[kRowSlots];
        int cnt = 0;
#pragma unroll
        for (int s = 0; s < kRowSlots; ++s) {
            first[s] = __ballot((lane + 64 * s < n) && !dup[s]);
            cnt += __popcll(first[s]);
        }
        if constexpr (!FILL) {
            if (lane == 0) rowlen[i] = cnt;
        } else {
            // rank among the distinct values = column position
            int less[kRowSlots];
#pragma unroll
            for (int s = 0; s < kRowSlots; ++s) less[s] = 0;
#pragma unroll
            for (int js = 0; js < kRowSlots; ++js) {
                if (64 * js >= n) break;
                const int jn = min(64, n - 64 * js);
                for (int jl = 0; jl < jn; ++jl) {
                    const uint32_t y = __shfl(c[js], jl, 64);
                    const int f = int((first[js] >> jl) & 1ull);
#pragma unroll
                    for (int s = 0; s < kRowSlots; ++s) less[s] += f & int(y < c[s]);
                }
            }
            const int64_t r0 = rp64[i];
#pragma unroll
            for (int s = 0; s < kRowSlots; ++s) {
                const int u = lane + 64 * s;
                if (u < n) {
                    if ((first[s] >> lane) & 1ull) ci[r0 + less[s]] = int32_t(c[s]);
                    const int sl = u / NL, b = u - sl * NL;
                    pos16[(t0 + sl) * 4 + b] = uint16_t(less[s]);
                }
            }
        }
    }
}

// One workgroup per long row, its candidates in LDS (n <= kLongCap).
template <bool FILL>
__global__ void __launch_bounds__(kPatWG)
    k_row_pattern_long(const int32_t *__restrict__ pme, int NL,
                       const int32_t *__restrict__ ip, const uint32_t *__restrict__ inc_elem,
                       const int32_t *__restrict__ longrows, int64_t *__restrict__ rowlen,
                       const int64_t *__restrict__ rp64, int32_t *__restrict__ ci,
                       uint16_t *__restrict__ pos16, int32_t *__restrict__ flag) {
    extern __shared__ uint32_t lds[];
    uint32_t *cand = lds;                                     // [kLongCap]
    uint8_t *isfirst = reinterpret_cast<uint8_t *>(lds + kLongCap);   // [kLongCap]
    __shared__ int red[kPatWG];
    const int64_t i = longrows[blockIdx.x];
    const int64_t t0 = ip[i];
    const int n = NL * (ip[i + 1] - ip[i]);
    if (n > kLongCap) {   // uniform over the workgroup
        if (threadIdx.x == 0) atomicOr(flag, 2);
        return;
    }
    for (int u = threadIdx.x; u < n; u += kPatWG) cand[u] = candidate(pme, NL, inc_elem, t0, u);
    __syncthreads();
    int cnt = 0;
    for (int u = threadIdx.x; u < n; u += kPatWG) {
        const uint32_t x = cand[u];
        int d = 0;
        for (int j = 0; j < u && !d; ++j) d = cand[j] == x;
        isfirst[u] = uint8_t(!d);
        cnt += !d;
    }
    red[threadIdx.x] = cnt;
    __syncthreads();
    for (int w = kPatWG / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if constexpr (!FILL) {
        if (threadIdx.x == 0) rowlen[i] = red[0];
    } else {
        const int64_t r0 = rp64[i];
        for (int u = threadIdx.x; u < n; u += kPatWG) {
            const uint32_t x = cand[u];
            int less = 0;
            for (int j = 0; j < n; ++j) less += int(isfirst[j]) & int(cand[j] < x);
            if (isfirst[u]) ci[r0 + less] = int32_t(x);
            const int sl = u / NL, b = u - sl * NL;
            pos16[(t0 + sl) * 4 + b] = uint16_t(less);
        }
    }
}

__global__ void k_rp32(const int64_t *__restrict__ rp64, int64_t n, int32_t *__restrict__ rp) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) rp[i] = int32_t(rp64[i]);
}

unsigned grid_for(int64_t n, int wg = kPatWG) { return unsigned((n + wg - 1) / wg); }

// Device scratch of the build, freed on every return path.
struct Scratch {
    std::vector<void *> ptrs;
    ~Scratch() {
        for (void *x : ptrs) (void)hipFree(x);
    }
    template <class T>
    hipError_t get(T **p, size_t count) {
        *p = nullptr;
        const hipError_t e = hipMalloc(reinterpret_cast<void **>(p), sizeof(T) * std::max<size_t>(count, 1));
        if (e == hipSuccess) ptrs.push_back(*p);
        else *p = nullptr;
        return e;
    }
};

int key_bits(int64_t nkeys) {
    int b = 1;
    while (b < 32 && (int64_t(1) << b) < nkeys) ++b;
    return b;
}

}  // namespace

fem_status build_pattern_gpu(fem_plan_data *p, const int32_t *me, hipStream_t s) {
    PhaseRange range("femasm: symbolic (GPU pattern)");
    const int d = p->d, NL = d + 1;
    const int64_t nq = p->nq, nme = p->nme, ninc = int64_t(NL) * nme;
    Scratch tmp;
    hipError_t e = hipSuccess;
#define FEM_TRY(x)                              \
    do {                                        \
        e = (x);                                \
        if (e != hipSuccess) return hip_status(e); \
    } while (0)
    // plan arrays (owned by the plan from here on; freed with it)
    FEM_TRY(hipMalloc(reinterpret_cast<void **>(&p->status), sizeof(int32_t) * 2));
    FEM_TRY(hipMemsetAsync(p->status, 0, sizeof(int32_t) * 2, s));
    FEM_TRY(hipMalloc(reinterpret_cast<void **>(&p->inc_ptr), sizeof(int32_t) * (nq + 1)));
    FEM_TRY(hipMalloc(reinterpret_cast<void **>(&p->rp), sizeof(int32_t) * (nq + 1)));
    FEM_TRY(hipMalloc(reinterpret_cast<void **>(&p->porig), sizeof(int32_t) * std::max<int64_t>(nme, 1)));
    FEM_TRY(hipMalloc(reinterpret_cast<void **>(&p->pme), sizeof(int32_t) * std::max<int64_t>(ninc, 1)));
    FEM_TRY(hipMalloc(reinterpret_cast<void **>(&p->inc_elem), sizeof(uint32_t) * std::max<int64_t>(ninc, 1)));
    FEM_TRY(hipMalloc(reinterpret_cast<void **>(&p->inc_off), sizeof(uint64_t) * std::max<int64_t>(ninc, 1)));
    const size_t npart = size_t((int64_t(d) * nq + 255) / 256 + 1);
    FEM_TRY(hipMalloc(reinterpret_cast<void **>(&p->part), sizeof(double) * npart));

    // ---- validation
    int32_t *flag = p->status + 1;   // scratch word next to the status word
    if (nme > 0)
        hipLaunchKernelGGL(k_validate, dim3(grid_for(nme)), dim3(kPatWG), 0, s, me, nme, NL, nq, flag);
    int32_t hflag = 0;
    FEM_TRY(hipGetLastError());
    FEM_TRY(hipMemcpyAsync(&hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    FEM_TRY(hipStreamSynchronize(s));
    if (hflag) return FEM_ERR_INDEX;

    // ---- incidences (stable radix sort of the element slots by vertex)
    uint32_t *keys, *vals, *skeys, *svals;
    FEM_TRY(tmp.get(&keys, size_t(ninc)));
    FEM_TRY(tmp.get(&vals, size_t(ninc)));
    FEM_TRY(tmp.get(&skeys, size_t(ninc)));
    FEM_TRY(tmp.get(&svals, size_t(ninc)));
    size_t tbytes = 0, tb2 = 0;
    FEM_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, tbytes, keys, skeys, vals, svals, int(ninc),
                                               0, key_bits(nq), s));
    FEM_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, tb2, keys, skeys, vals, svals,
                                               int(std::max<int64_t>(nme, 1)), 0, key_bits(nq), s));
    void *cub_tmp;
    FEM_TRY(tmp.get(reinterpret_cast<char **>(&cub_tmp), std::max(tbytes, tb2)));
    const size_t cub_bytes = std::max(tbytes, tb2);
    if (ninc > 0) {
        hipLaunchKernelGGL(k_slot_keys, dim3(grid_for(ninc)), dim3(kPatWG), 0, s, me, nme, NL, keys, vals);
        FEM_TRY(hipGetLastError());
        size_t tb = cub_bytes;
        FEM_TRY(hipcub::DeviceRadixSort::SortPairs(cub_tmp, tb, keys, skeys, vals, svals, int(ninc), 0,
                                                   key_bits(nq), s));
    }
    hipLaunchKernelGGL(k_key_bounds, dim3(grid_for(ninc + 1)), dim3(kPatWG), 0, s, skeys, ninc, nq,
                       p->inc_ptr);
    FEM_TRY(hipGetLastError());

    // ---- element order (stable radix sort by smallest vertex id)
    int32_t *pinv;
    FEM_TRY(tmp.get(&pinv, size_t(nme)));
    if (nme > 0) {
        hipLaunchKernelGGL(k_elem_keys, dim3(grid_for(nme)), dim3(kPatWG), 0, s, me, nme, NL, keys, vals);
        FEM_TRY(hipGetLastError());
        size_t tb = cub_bytes;
        // sorted element keys/order go into the first nme words of keys/vals' partners
        uint32_t *ekeys = keys + nme, *eorder = vals + nme;
        if (ninc < 2 * nme) {   // cannot happen (ninc = (d+1) nme), kept for clarity
            return FEM_ERR_ARG;
        }
        FEM_TRY(hipcub::DeviceRadixSort::SortPairs(cub_tmp, tb, keys, ekeys, vals, eorder, int(nme),
                                                   0, key_bits(nq), s));
        hipLaunchKernelGGL(k_elem_order, dim3(grid_for(nme)), dim3(kPatWG), 0, s, eorder, nme, NL, me,
                           p->porig, pinv, p->pme);
        FEM_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_inc_elem, dim3(grid_for(ninc)), dim3(kPatWG), 0, s, svals, ninc, NL, pinv,
                           p->inc_elem);
        FEM_TRY(hipGetLastError());
    }

    // ---- rows: count, scan, fill
    int64_t *rowlen, *rp64;
    int32_t *longrows, *nlong;
    FEM_TRY(tmp.get(&rowlen, size_t(nq + 1)));
    FEM_TRY(tmp.get(&rp64, size_t(nq + 1)));
    FEM_TRY(tmp.get(&longrows, size_t(nq)));
    FEM_TRY(tmp.get(&nlong, 1));
    FEM_TRY(hipMemsetAsync(nlong, 0, sizeof(int32_t), s));
    FEM_TRY(hipMemsetAsync(rowlen, 0, sizeof(int64_t) * (nq + 1), s));
    FEM_TRY(hipMemsetAsync(p->inc_off, 0, sizeof(uint64_t) * std::max<int64_t>(ninc, 1), s));
    const int32_t *ip = p->inc_ptr;
    uint16_t *pos16 = reinterpret_cast<uint16_t *>(p->inc_off);
    const unsigned rgrid = unsigned(std::min<int64_t>(std::max<int64_t>(grid_for(nq, kPatWG / 64), 1), 8192));
    if (nq > 0) {
        hipLaunchKernelGGL(k_row_pattern<false>, dim3(rgrid), dim3(kPatWG), 0, s, p->pme, NL, nq, ip,
                           p->inc_elem, rowlen, rp64, p->ci, pos16, longrows, nlong);
        FEM_TRY(hipGetLastError());
    }
    int32_t hlong = 0;
    FEM_TRY(hipMemcpyAsync(&hlong, nlong, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    FEM_TRY(hipStreamSynchronize(s));
    const size_t long_lds = size_t(kLongCap) * 5;
    if (hlong > 0) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_row_pattern_long<false>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(long_lds));
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_row_pattern_long<true>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(long_lds));
        hipLaunchKernelGGL(k_row_pattern_long<false>, dim3(unsigned(hlong)), dim3(kPatWG), long_lds, s,
                           p->pme, NL, ip, p->inc_elem, longrows, rowlen, rp64, p->ci, pos16, flag);
        FEM_TRY(hipGetLastError());
    }
    {
        size_t tb = 0;
        FEM_TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, rowlen, rp64, int(nq + 1), s));
        void *st;
        FEM_TRY(tmp.get(reinterpret_cast<char **>(&st), tb));
        FEM_TRY(hipcub::DeviceScan::ExclusiveSum(st, tb, rowlen, rp64, int(nq + 1), s));
    }
    int64_t nnz = 0;
    FEM_TRY(hipMemcpyAsync(&nnz, rp64 + nq, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FEM_TRY(hipMemcpyAsync(&hflag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    FEM_TRY(hipStreamSynchronize(s));
    if (hflag) return FEM_ERR_OVERFLOW;   // a vertex in more than kLongCap/(d+1) elements
    if (nnz >= (int64_t(1) << 31)) return FEM_ERR_OVERFLOW;
    p->nnz = nnz;
    FEM_TRY(hipMalloc(reinterpret_cast<void **>(&p->ci), sizeof(int32_t) * std::max<int64_t>(nnz, 1)));
    if (nq > 0) {
        hipLaunchKernelGGL(k_row_pattern<true>, dim3(rgrid), dim3(kPatWG), 0, s, p->pme, NL, nq, ip,
                           p->inc_elem, rowlen, rp64, p->ci, pos16, longrows, nlong);
        FEM_TRY(hipGetLastError());
    }
    if (hlong > 0) {
        hipLaunchKernelGGL(k_row_pattern_long<true>, dim3(unsigned(hlong)), dim3(kPatWG), long_lds, s,
                           p->pme, NL, ip, p->inc_elem, longrows, rowlen, rp64, p->ci, pos16, flag);
        FEM_TRY(hipGetLastError());
    }
    hipLaunchKernelGGL(k_rp32, dim3(grid_for(nq + 1)), dim3(kPatWG), 0, s, rp64, nq + 1, p->rp);
    FEM_TRY(hipGetLastError());
    FEM_TRY(hipMemsetAsync(flag, 0, sizeof(int32_t), s));

    // ---- host copy of the row pointer (launch geometry)
    p->h_rp.resize(size_t(nq + 1));
    FEM_TRY(hipMemcpyAsync(p->h_rp.data(), p->rp, sizeof(int32_t) * (nq + 1), hipMemcpyDeviceToHost, s));
    FEM_TRY(hipStreamSynchronize(s));
#undef FEM_TRY
    int max_row = 0;
    for (int64_t i = 0; i < nq; ++i) max_row = std::max(max_row, p->h_rp[i + 1] - p->h_rp[i]);
    p->max_row = max_row;
    return FEM_OK;
}

}  // namespace femasm
