// Numeric phase and the small helper kernels of a plan.
#include <cstring>

#include "femasm_impl.h"
#include "rowgather.h"

namespace femasm {

__device__ __forceinline__ void flag_bad(int32_t *status, int bad) {
    // one vector atomic per wavefront that met a degenerate element
    const unsigned long long any = __ballot(bad != 0);
    if (any != 0ull && (threadIdx.x & 63) == __ffsll((long long)any) - 1) atomicOr(status, bad);
}

template <int D, int OP>
__global__ void __launch_bounds__(256) k_numeric(MeshView mv, double lam, double mu,
                                                 int32_t *status) {
    constexpr int M = (OP == FEM_OP_ELAS) ? D : 1;
    extern __shared__ double acc[];
    const int64_t nrows = int64_t(M) * mv.nq;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t r0 = tile * blockDim.x;
    const int64_t r1 = min(r0 + int64_t(blockDim.x), nrows);
    int bad = 0;
    assemble_row_tile<D, OP>(mv, r0, r1, acc, lam, mu, bad);
    flag_bad(status, bad);
}

template <int D, int OP>
static hipError_t launch_numeric(const fem_plan_s *p, const MeshView &mv, double lam, double mu,
                                 hipStream_t s) {
    constexpr int M = (OP == FEM_OP_ELAS) ? D : 1;
    const RowLaunch &L = p->launch[M];
    if (L.tiles == 0) return hipSuccess;
    hipLaunchKernelGGL((k_numeric<D, OP>), dim3(unsigned(L.tiles)), dim3(L.rows_per_wg),
                       L.lds_bytes, s, mv, lam, mu, p->status);
    return hipGetLastError();
}

// Vector pattern: dof row (i, l) = M*i + l, columns M*j + n.
__global__ void k_pattern_vec(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                              int64_t nq, int M, int32_t *__restrict__ vrp,
                              int32_t *__restrict__ vci) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nrows = int64_t(M) * nq;
    if (r > nrows) return;
    const int64_t i = r / M, l = r - (r / M) * M;
    if (r == nrows) {
        vrp[r] = int32_t(int64_t(M) * M * rp[nq]);
        return;
    }
    const int64_t deg = rp[i + 1] - rp[i];
    const int64_t s0 = int64_t(M) * M * rp[i] + l * M * deg;
    vrp[r] = int32_t(s0);
    for (int64_t p = 0; p < deg; ++p) {
        const int32_t j = ci[rp[i] + p];
        for (int n = 0; n < M; ++n) vci[s0 + M * p + n] = int32_t(int64_t(M) * j + n);
    }
}

// slot[k*(d+1)^2 + b*(d+1) + a] = CSR position of (me[a,k], me[b,k]).
__global__ void k_slot_map(const int32_t *__restrict__ rp, const int32_t *__restrict__ inc_ptr,
                           const uint32_t *__restrict__ inc_elem,
                           const uint64_t *__restrict__ inc_off,
                           const int32_t *__restrict__ porig, int64_t nq, int NL,
                           int32_t *__restrict__ slot) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    for (int t = inc_ptr[i]; t < inc_ptr[i + 1]; ++t) {
        const uint32_t ea = inc_elem[t];
        const int64_t k = porig[ea & 0x3fffffffu];
        const int a = int(ea >> 30);
        for (int b = 0; b < NL; ++b) {
            const int pos = int((inc_off[t] >> (16 * b)) & 0xffffu);
            slot[k * NL * NL + int64_t(b) * NL + a] = rp[i] + pos;
        }
    }
}

// J = a^T A b: per-row partial sums, then one workgroup adds them in row
// order (fixed tree), so the result is reproducible.
__global__ void k_bilinear_rows(const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                const double *__restrict__ vals, const double *__restrict__ a,
                                const double *__restrict__ b, int64_t nq, int M,
                                double *__restrict__ part) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    __shared__ double red[256];
    double s = 0.0;
    if (r < int64_t(M) * nq) {
        const int64_t i = r / M, l = r - (r / M) * M;
        const int64_t deg = rp[i + 1] - rp[i];
        const int64_t s0 = int64_t(M) * M * rp[i] + l * M * deg;
        double acc = 0.0;
        for (int64_t p = 0; p < deg; ++p) {
            const int64_t j = ci[rp[i] + p];
            for (int n = 0; n < M; ++n) acc += vals[s0 + M * p + n] * b[M * j + n];
        }
        s = a[r] * acc;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (unsigned w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_sum_parts(const double *__restrict__ part, int64_t n, double *__restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    // thread t sums a contiguous chunk, chunks then combined by a fixed tree
    const int64_t chunk = (n + blockDim.x - 1) / blockDim.x;
    const int64_t b0 = threadIdx.x * chunk, b1 = min(n, b0 + chunk);
    for (int64_t k = b0; k < b1; ++k) s += part[k];
    red[threadIdx.x] = s;
    __syncthreads();
    for (unsigned w = blockDim.x / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

}  // namespace femasm

using namespace femasm;

static MeshView plan_view(const fem_plan_s *p, const double *q, const double *w, double *values) {
    MeshView mv;
    mv.rp = p->rp;
    mv.inc_ptr = p->inc_ptr;
    mv.inc_elem = p->inc_elem;
    mv.inc_off = p->inc_off;
    mv.pme = p->pme;
    mv.q = q;
    mv.w = w;
    mv.values = values;
    mv.nq = p->nq;
    return mv;
}

static fem_status fem_assemble_numeric_impl(fem_plan plan, int32_t op, const double *q,
                                           const double *w, double lambda, double mu,
                                           double *values, hipStream_t stream) {
    PhaseRange range("femasm: numeric");
    if (!plan || op < FEM_OP_MASS || op > FEM_OP_ELAS) return FEM_ERR_ARG;
    const int64_t M = op == FEM_OP_ELAS ? plan->d : 1;
    if (M * M * plan->nnz >= (int64_t(1) << 31)) return FEM_ERR_OVERFLOW;
    if (plan->nnz > 0 && (!q || !values)) return FEM_ERR_ARG;
    if (op == FEM_OP_MASS_W && plan->nnz > 0 && !w) return FEM_ERR_ARG;
    if (plan->launch[M].rows_per_wg == 0) return FEM_ERR_OVERFLOW;
    hipError_t e = hipSuccess;
    // FEMASM_KERNEL=pair|block|rowgather forces one kernel family (A/B
    // comparisons).  By default the pair kernel (measured fastest for all
    // four operators), else the record-block kernel (scalar operators), else
    // the row-gather kernel.
    const char *sel = getenv("FEMASM_KERNEL");
    const bool any = !sel || !*sel;
    if (plan->nq > 0) {
        if ((any || !strcmp(sel, "pair")) && launch_pair(plan, op, q, w, lambda, mu, values, stream, &e))
            return hip_status(e);
        if ((any || !strcmp(sel, "block")) && launch_block(plan, op, q, w, values, stream, &e))
            return hip_status(e);
    }
    const MeshView mv = plan_view(plan, q, w, values);
    if (plan->d == 2) {
        switch (op) {
            case FEM_OP_MASS: e = launch_numeric<2, FEM_OP_MASS>(plan, mv, lambda, mu, stream); break;
            case FEM_OP_MASS_W: e = launch_numeric<2, FEM_OP_MASS_W>(plan, mv, lambda, mu, stream); break;
            case FEM_OP_STIFF: e = launch_numeric<2, FEM_OP_STIFF>(plan, mv, lambda, mu, stream); break;
            default: e = launch_numeric<2, FEM_OP_ELAS>(plan, mv, lambda, mu, stream); break;
        }
    } else {
        switch (op) {
            case FEM_OP_MASS: e = launch_numeric<3, FEM_OP_MASS>(plan, mv, lambda, mu, stream); break;
            case FEM_OP_MASS_W: e = launch_numeric<3, FEM_OP_MASS_W>(plan, mv, lambda, mu, stream); break;
            case FEM_OP_STIFF: e = launch_numeric<3, FEM_OP_STIFF>(plan, mv, lambda, mu, stream); break;
            default: e = launch_numeric<3, FEM_OP_ELAS>(plan, mv, lambda, mu, stream); break;
        }
    }
    return hip_status(e);
}

extern "C" fem_status fem_assemble_numeric(fem_plan plan, int32_t op, const double *q,
                                           const double *w, double lambda, double mu,
                                           double *values, hipStream_t stream) {
    return debug_check(fem_assemble_numeric_impl(plan, op, q, w, lambda, mu, values, stream),
                       stream, plan ? plan->status : nullptr);
}

static fem_status fem_assemble_elasticity_nodal_impl(fem_plan plan, const double *q,
                                                   const double *lam, const double *mu,
                                                   double *values, hipStream_t stream) {
    PhaseRange range("femasm: numeric (nodal Lame)");
    if (!plan) return FEM_ERR_ARG;
    const int64_t nnz = int64_t(plan->d) * plan->d * plan->nnz;
    if (nnz >= (int64_t(1) << 31)) return FEM_ERR_OVERFLOW;
    if (nnz > 0 && (!q || !lam || !mu || !values)) return FEM_ERR_ARG;
    if (nnz == 0) return FEM_OK;
    wait_layouts(plan);   // these operators run on the block layouts only
    hipError_t e = hipSuccess;
    if (launch_pair(plan, kOpElasNodal, q, lam, 0.0, 0.0, values, stream, &e, mu))
        return hip_status(e);
    return FEM_ERR_OVERFLOW;   // no vertex-pair layout for this mesh
}

extern "C" fem_status fem_assemble_elasticity_nodal(fem_plan plan, const double *q,
                                                   const double *lam, const double *mu,
                                                   double *values, hipStream_t stream) {
    return debug_check(fem_assemble_elasticity_nodal_impl(plan, q, lam, mu, values, stream),
                       stream, plan ? plan->status : nullptr);
}

static fem_status fem_assemble_general_impl(fem_plan plan, const double *q, const double *coef,
                                          double *values, hipStream_t stream) {
    PhaseRange range("femasm: numeric (general operator)");
    if (!plan || !coef) return FEM_ERR_ARG;
    if (plan->nnz > 0 && (!q || !values)) return FEM_ERR_ARG;
    if (plan->nnz == 0) return FEM_OK;
    const int d = plan->d;
    double gco[kGeneralCoef] = {};
    for (int i = 0; i < d * d + 2 * d + 1; ++i) gco[i] = coef[i];
    wait_layouts(plan);   // these operators run on the block layouts only
    hipError_t e = hipSuccess;
    if (launch_pair(plan, kOpGeneral, q, nullptr, 0.0, 0.0, values, stream, &e, nullptr, gco))
        return hip_status(e);
    return FEM_ERR_OVERFLOW;   // no vertex-pair layout for this mesh
}

extern "C" fem_status fem_assemble_general(fem_plan plan, const double *q, const double *coef,
                                          double *values, hipStream_t stream) {
    return debug_check(fem_assemble_general_impl(plan, q, coef, values, stream),
                       stream, plan ? plan->status : nullptr);
}

extern "C" fem_status fem_plan_pattern(fem_plan plan, int32_t op, int32_t *row_ptr,
                                       int32_t *col_idx, hipStream_t stream) {
    if (!plan || op < FEM_OP_MASS || op > FEM_OP_ELAS || !row_ptr) return FEM_ERR_ARG;
    const int M = op == FEM_OP_ELAS ? plan->d : 1;
    if (int64_t(M) * M * plan->nnz >= (int64_t(1) << 31)) return FEM_ERR_OVERFLOW;
    if (plan->nnz > 0 && !col_idx) return FEM_ERR_ARG;
    hipError_t e;
    if (M == 1) {
        e = hipMemcpyAsync(row_ptr, plan->rp, sizeof(int32_t) * (plan->nq + 1),
                           hipMemcpyDeviceToDevice, stream);
        if (e == hipSuccess && plan->nnz > 0)
            e = hipMemcpyAsync(col_idx, plan->ci, sizeof(int32_t) * plan->nnz,
                               hipMemcpyDeviceToDevice, stream);
    } else {
        const int64_t n = int64_t(M) * plan->nq + 1;
        hipLaunchKernelGGL(k_pattern_vec, dim3(unsigned((n + 255) / 256)), dim3(256), 0, stream,
                           plan->rp, plan->ci, plan->nq, M, row_ptr, col_idx);
        e = hipGetLastError();
    }
    return hip_status(e);
}

extern "C" fem_status fem_plan_slot_map(fem_plan plan, int32_t *slot, hipStream_t stream) {
    if (!plan || (plan->nme > 0 && !slot)) return FEM_ERR_ARG;
    if (plan->nq == 0) return FEM_OK;
    hipLaunchKernelGGL(k_slot_map, dim3(unsigned((plan->nq + 255) / 256)), dim3(256), 0, stream,
                       plan->rp, plan->inc_ptr, plan->inc_elem, plan->inc_off, plan->porig,
                       plan->nq, plan->d + 1, slot);
    return hip_status(hipGetLastError());
}

extern "C" fem_status fem_csr_bilinear(fem_plan plan, int32_t op, const double *values,
                                       const double *a, const double *b, double *out,
                                       hipStream_t stream) {
    if (!plan || op < FEM_OP_MASS || op > FEM_OP_ELAS || !out || !a || !b) return FEM_ERR_ARG;
    const int M = op == FEM_OP_ELAS ? plan->d : 1;
    const int64_t nrows = int64_t(M) * plan->nq;
    const int64_t nblk = (nrows + 255) / 256;
    if (nblk == 0) {
        hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, stream, out, int64_t(0), out);
        return hip_status(hipGetLastError());
    }
    double *part = plan->part;  // plan-owned, sized for the vector operator
    hipLaunchKernelGGL(k_bilinear_rows, dim3(unsigned(nblk)), dim3(256), 0, stream, plan->rp,
                       plan->ci, values, a, b, plan->nq, M, part);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, stream, part, nblk, out);
    return hip_status(hipGetLastError());
}
