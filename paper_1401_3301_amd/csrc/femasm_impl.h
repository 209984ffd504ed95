// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/femasm.h"

namespace femasm {

// Largest dynamic LDS block a numeric workgroup may request.
constexpr size_t kLdsCap = 64 * 1024;

// Launch geometry of the row-gather kernel for one dof multiplicity M
// (1 for scalar operators, d for elasticity): rows per workgroup and the
// LDS bytes the largest row tile needs.
struct RowLaunch {
    int rows_per_wg = 0;
    size_t lds_bytes = 0;
    int64_t tiles = 0;
};

struct fem_plan_data {
    int d = 0;
    int64_t nq = 0, nme = 0, nnz = 0;
    int max_row = 0;
    int device = 0;
    // device arrays (owned)
    int32_t *rp = nullptr;        // [nq+1] scalar CSR row pointer
    int32_t *ci = nullptr;        // [nnz]  scalar CSR columns
    int32_t *pme = nullptr;       // [(d+1)*nme] connectivity, plan order, element-major
    int32_t *porig = nullptr;     // [nme] plan element -> caller element number
    int32_t *inc_ptr = nullptr;   // [nq+1] vertex -> incidence range
    uint32_t *inc_elem = nullptr; // [(d+1)*nme] plan element | (local vertex << 30)
    uint32_t *inc_off = nullptr;  // [(d+1)*nme] byte b = position of local vertex b in the row
    int32_t *status = nullptr;    // [1] sticky error word
    double *part = nullptr;       // [d*nq/256 + 1] row-block partial sums of fem_csr_bilinear
    std::vector<int32_t> h_rp;    // host copy of rp (launch geometry)
    RowLaunch launch[4];          // indexed by M
};

}  // namespace femasm

struct fem_plan_s : femasm::fem_plan_data {};

namespace femasm {

fem_status hip_status(hipError_t e);
RowLaunch row_launch_for(const std::vector<int32_t> &h_rp, int64_t nq, int M, size_t lds_cap);

// Device-side view of one mesh for the shared tile routine.
struct MeshView {
    const int32_t *rp;
    const int32_t *inc_ptr;
    const uint32_t *inc_elem;
    const uint32_t *inc_off;
    const int32_t *pme;
    const double *q;
    const double *w;
    double *values;
    int64_t nq;
};

// One work item of the batched launch.
struct BatchItem {
    int32_t mesh;
    int32_t nrows;  // rows in this tile (<= threads per workgroup)
    int64_t row0;   // first dof row of the tile within the mesh
};

struct BatchMesh {
    const int32_t *rp;
    const int32_t *inc_ptr;
    const uint32_t *inc_elem;
    const uint32_t *inc_off;
    const int32_t *pme;
    int64_t nq;
    int64_t q_off;
    int64_t w_off;
    int64_t val_off[2];   // scalar / vector operator
    int32_t d;
    int32_t pad;
};

fem_status launch_batch(int op, const BatchMesh *meshes, const BatchItem *items, int64_t nitems,
                        int rows_per_wg, size_t lds_bytes, int grid, int has_d2, int has_d3,
                        const double *q_cat, const double *w_cat, double lam, double mu,
                        double *values_cat, int32_t *status, hipStream_t stream);

}  // namespace femasm
