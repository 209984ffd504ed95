// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <mutex>
#include <thread>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/femasm.h"

namespace femasm {

// A named profiler range (roctx) over a phase of the library, shown by
// rocprofv3 --marker-trace; next to free when no profiler is attached.
// Host time: for the asynchronous entry points it covers the launches.
struct PhaseRange {
    explicit PhaseRange(const char *name) { roctxRangePushA(name); }
    ~PhaseRange() { roctxRangePop(); }
    PhaseRange(const PhaseRange &) = delete;
    PhaseRange &operator=(const PhaseRange &) = delete;
};

// Largest dynamic LDS block a numeric workgroup may request.
constexpr size_t kLdsCap = 64 * 1024;

// LDS bytes of a row-gather tile of `rows` dof rows spanning `span` CSR values:
// the accumulators, plus the elasticity epilogue tables (M > 1).
inline size_t tile_lds_bytes(int M, int64_t span, int64_t rows) {
    size_t b = size_t(span) * sizeof(double);
    if (M > 1) b += 8 * size_t((rows + M - 1) / M) + size_t(span / (M * M)) + 16;
    return b;
}

// Launch geometry of the row-gather kernel for one dof multiplicity M
// (1 for scalar operators, d for elasticity): rows per workgroup and the
// LDS bytes the largest row tile needs.
struct RowLaunch {
    int rows_per_wg = 0;
    size_t lds_bytes = 0;
    int64_t tiles = 0;
};

// Vertex-block layout of the block kernels (see blocks_host.h).
struct BlockPlan {
    bool ok = false;
    int nb = 0;
    int max_rows = 0, max_nodes = 0, max_elems = 0;
    int64_t max_nacc = 0;
    int64_t max_rec = 0;          // largest record array of a block
    int wg = 128;                 // threads per workgroup of the block kernel
    int32_t *rows = nullptr;      // [rows] owned rows, grouped by block
    int32_t *row_ptr = nullptr;   // [nb+1]
    int32_t *acc_off = nullptr;   // [rows] local accumulator offset of each owned row
    int32_t *nacc = nullptr;      // [nb] accumulator length of each block
    int32_t *nodes = nullptr;     // touched vertices, grouped by block
    int32_t *node_ptr = nullptr;  // [nb+1]
    uint16_t *elem = nullptr;     // 4 local vertex ids per block element
    int32_t *elem_ptr = nullptr;  // [nb+1]
    uint32_t *rec = nullptr;      // interleaved incidence records
    int64_t *rec_ptr = nullptr;   // [nb+1]
    int32_t *maxdeg = nullptr;    // [nb]
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
    const uint64_t *inc_off;
    const int32_t *pme;
    int64_t nq;
    int64_t q_off;
    int64_t w_off;
    int64_t val_off[2];   // scalar / vector operator
    int32_t d;
    int32_t pad;
};

// Vertex-pair layout of the pair kernel (see blocks_host.h and pair.hip).
struct PairPlan {
    bool ok = false;
    int nb = 0;
    int slots = 2;                // tasks of 64 pairs per wavefront at most (1, 2 or 4)
    int max_rows = 0, max_nodes = 0, max_elems = 0;
    int64_t max_nacc = 0, max_ent = 0;
    int32_t *desc = nullptr;      // [nb*24] block descriptors (pair.hip)
    int4 *rowinfo = nullptr;      // [rows] (rp[row], row length, local offset, 0)
    int32_t *nodes = nullptr;     // touched vertices, grouped by block
    uint32_t *elem = nullptr;     // 4 x 8-bit local vertex ids per block element
    int32_t *task_cnt = nullptr;  // entries per lane of each task
    int32_t *task_eoff = nullptr; // first entry of each task, relative to its block
    // [ntask*64] per task lane: low half the pair r | p << 7 (0xffff: empty),
    // high half the mirror pair written by the same lane (0xffff: none)
    uint32_t *hdr = nullptr;
    uint16_t *ent = nullptr;      // entry lists, entry-major within a task
    int64_t n_rows = 0, n_nodes = 0, n_elems = 0, n_tasks = 0, n_ent = 0;   // array lengths
    std::vector<int32_t> h_desc;  // host copy of desc (batched layouts are built from it)
    // Vertices whose rows no block covers (ascending; a star or row beyond the
    // block caps), assembled by the row-gather tile kernel over `left_items`
    // (tiles of consecutive such rows) in the same launch sequence.
    std::vector<int32_t> h_left;
    BatchItem *left_items = nullptr;
    BatchMesh *left_mesh = nullptr;   // the plan as a one-mesh batch
    int64_t n_left_items = 0;
    int left_rpw = 0;                 // threads (dof rows) per tile
    size_t left_lds = 0;
};
constexpr int kPairWaves = 8;     // wavefronts per workgroup of the pair kernel
// Internal operator code of elasticity with nodal (P1) Lame fields
// (fem_assemble_elasticity_nodal); the vertex-pair kernel only.
constexpr int kOpElasNodal = 4;
// Internal operator code of the general second-order operator
// (fem_assemble_general); the vertex-pair kernel only.
constexpr int kOpGeneral = 5;
constexpr int kGeneralCoef = 16;   // A (d*d), b (d), c (d), a0, padded
// Internal operator codes of the directional derivatives (fem_assemble_jvp)
// of the mass, weighted mass and stiffness on the vertex-pair kernel.
constexpr int kOpJvpMass = 6;
constexpr int kOpJvpMassW = 7;
constexpr int kOpJvpStiff = 8;

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
    uint64_t *inc_off = nullptr;  // [(d+1)*nme] bits 16b..16b+15: position of local vertex b in the row
    int32_t *status = nullptr;    // [2] sticky error word, then a scratch word of the symbolic phase
    double *part = nullptr;       // [d*nq/256 + 1] row-block partial sums of fem_csr_bilinear
    // [(d+1)^2*nme] per plan element e, at e*(d+1)^2 + b*(d+1) + a: the
    // position of vertex b within the CSR row of vertex a -- 8-bit when no
    // row has more than 256 entries, else 16-bit (vpos_bytes, 0 until
    // fem_plan_vjp_positions builds it; published with release order)
    void *vpos = nullptr;
    std::atomic<int> vpos_bytes{0};
    std::mutex vpos_mu;
    std::vector<int32_t> h_rp;    // host copy of rp (launch geometry)
    RowLaunch launch[4];          // indexed by M
    BlockPlan blk;                // block-kernel layout (scalar operators)
    PairPlan pscal;               // pair-kernel layout, scalar operators
    PairPlan pvec;                // pair-kernel layout, elasticity
    // The block layouts above are built on a host thread after the symbolic
    // call returns (kLayout* states); until they are published the numeric
    // calls take the row-gather kernel, which produces the same bits.
    std::atomic<int> layout_state{0};
    fem_status layout_status = FEM_OK;   // of the build (FEM_OK unless it failed)
    std::mutex layout_mu;
    std::condition_variable layout_cv;
    std::thread layout_thread;
};
constexpr int kLayoutBuilding = 0;   // the host thread is still building
constexpr int kLayoutReady = 1;      // published: the block kernels may run
constexpr int kLayoutNone = 2;       // finished; no layout (row-gather only)

// Synchronous copies of the layout builders on a stream of their own that
// does not synchronise with the null stream (the layout thread runs while
// the caller's work proceeds).
inline hipError_t copy_sync(void *dst, const void *src, size_t bytes, hipMemcpyKind kind) {
    hipStream_t st = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(dst, src, bytes, kind, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    const hipError_t e2 = hipStreamDestroy(st);
    return e != hipSuccess ? e : e2;
}

// FEMASM_DEBUG=1 in the environment: the asynchronous entry points
// synchronise their stream after their launches and report a launch or
// kernel error, or a degenerate element (the status word, then cleared),
// from the call itself.  A debugging aid; off by default.
fem_status debug_check(fem_status st, hipStream_t s, int32_t *status_word);

// True when the block layouts are published (acquire: their arrays are
// complete and visible).
inline bool layouts_ready(const fem_plan_data *p) {
    return p->layout_state.load(std::memory_order_acquire) == kLayoutReady;
}
// Blocks until the layout build has finished (ready or none).
void wait_layouts(fem_plan_data *p);
// Rebuilds one pair layout of the plan (vec: elasticity) with R rows per
// block and `slots` tasks per wavefront, synchronously; not concurrently
// with numeric calls on the plan.
fem_status rebuild_pair_layout(fem_plan_data *p, bool vec, int R, int slots);

// CSR pattern, incidences and element order on the GPU (pattern.hip).
// Allocates and fills rp, ci, pme, porig, inc_ptr, inc_elem, inc_off,
// status and part of p (freed with the plan), sets nnz, max_row and h_rp.
// Synchronous on stream s.
fem_status build_pattern_gpu(fem_plan_data *p, const int32_t *me, hipStream_t s);

}  // namespace femasm

struct fem_plan_s : femasm::fem_plan_data {};

namespace femasm {

fem_status hip_status(hipError_t e);
fem_status upload_blocks(fem_plan_data *p, int d, int64_t nq, int64_t nme, const int32_t *me,
                         const int32_t *rp, const int32_t *ci, const int64_t *ip,
                         const int32_t *inc_k);
void free_blocks(BlockPlan *b);
void free_pairs(PairPlan *p);
fem_status upload_pairs(PairPlan &P, int R, int slots, bool tri, int d, int64_t nq, int64_t nme,
                        const int32_t *me, const int32_t *rp, const int32_t *ci, const int64_t *ip,
                        const int32_t *inc_k);
// Row-gather tiles of the leftover rows of a pair layout (M = dof per vertex).
fem_status upload_leftover(PairPlan &P, const fem_plan_data *p, int M);
// Launches the pair kernel; returns false (nothing launched) when the plan
// has no pair layout for this operator.
// w2: the mu field of kOpElasNodal (w is then the lambda field).
// gco: host coefficients of kOpGeneral (kGeneralCoef doubles).
// dq: the tangent coordinates of the JVP operators (d*nq, layout of q).
bool launch_pair(const fem_plan_data *p, int op, const double *q, const double *w, double lam,
                 double mu, double *values, hipStream_t s, hipError_t *err,
                 const double *w2 = nullptr, const double *gco = nullptr,
                 const double *dq = nullptr);
// Launches the pair kernel over a layout of dimension d (hipErrorNotSupported:
// its LDS need exceeds the workgroup limit, nothing launched).
hipError_t launch_pair_layout(const PairPlan &P, int d, int op, const double *q, const double *w,
                              double lam, double mu, double *values, int32_t *status,
                              hipStream_t s, const double *w2 = nullptr,
                              const double *gco = nullptr, const double *dq = nullptr);
// One persistent launch over a 2D and a 3D pair layout (the batched
// assembly of meshes of both dimensions; the four P1 operators, equal slot
// counts; hipErrorNotSupported: nothing launched).
hipError_t launch_pair_mixed(const PairPlan &P2, const PairPlan &P3, int op, const double *q,
                             const double *w, double lam, double mu, double *values,
                             int32_t *status, hipStream_t s);
// Concatenates per-mesh pair layouts into one (block descriptors carry each
// mesh's coordinate / weight / value offsets and vertex count).  out.ok is
// false when some part has no layout or the slot counts differ.
fem_status concat_pairs(PairPlan &out, const std::vector<const PairPlan *> &parts,
                        const std::vector<int64_t> &qo, const std::vector<int64_t> &wo,
                        const std::vector<int64_t> &vo, const std::vector<int64_t> &nq);
// Launches the block kernel for a scalar operator; returns false (nothing
// launched) when the plan has no block layout.
bool launch_block(const fem_plan_data *p, int op, const double *q, const double *w,
                  double *values, hipStream_t s, hipError_t *err);
bool launch_block(const fem_plan_data *p, int op, const double *q, const double *w,
                  double *values, hipStream_t s, hipError_t *err, double lam, double mu);
RowLaunch row_launch_for(const std::vector<int32_t> &h_rp, int64_t nq, int M, size_t lds_cap);

// Device-side view of one mesh for the shared tile routine.
struct MeshView {
    const int32_t *rp;
    const int32_t *inc_ptr;
    const uint32_t *inc_elem;
    const uint64_t *inc_off;
    const int32_t *pme;
    const double *q;
    const double *w;
    double *values;
    int64_t nq;
};

fem_status launch_batch(int op, const BatchMesh *meshes, const BatchItem *items, int64_t nitems,
                        int rows_per_wg, size_t lds_bytes, int grid, int has_d2, int has_d3,
                        const double *q_cat, const double *w_cat, double lam, double mu,
                        double *values_cat, int32_t *status, hipStream_t stream);

}  // namespace femasm
