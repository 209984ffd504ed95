/*
 * femasm.h - C ABI of the MI355X (gfx950) P1 finite-element assembly library.
 *
 * What it computes (Cuvelier, Japhet, Scarella, "An efficient way to
 * assemble finite element matrices in vector languages"):
 *
 *   A = sum over elements K of  P_K^T E(K) P_K            (Section 3)
 *
 * for a conforming mesh of d-simplices (d = 2 triangles, d = 3 tetrahedra)
 * with P1 Lagrange elements.  E(K) is one of
 *   FEM_OP_MASS    integral of lambda_a lambda_b            (magic formula, Section 2)
 *   FEM_OP_MASS_W  integral of w_h lambda_a lambda_b, w_h the P1 interpolant of
 *                  the nodal weight w (closed form of Section 4.1)
 *   FEM_OP_STIFF   |K| <grad lambda_b, grad lambda_a>      (Section 4.2)
 *   FEM_OP_ELAS    isotropic linear elasticity with constant Lame parameters
 *                  lambda, mu (lemma of Section 5.1, Appendix B), vector dofs
 *                  in the alternate numbering r = d*i + l (Section 5)
 * and the duplicate (I, J) contributions are summed into CSR (the `sparse`
 * primitive of Section 3), deterministically: every entry is the sum of its
 * element contributions in ascending element number, starting from 0.0, so
 * values are bitwise reproducible from run to run and A is exactly
 * symmetric.  The pattern is structural (explicit zeros are kept).
 *
 * Around that path: elasticity with nodal Lame fields and the general
 * second-order operator on the same plan; the adjoint of a^T (S + M_w) b and
 * the JVP / VJP of the assembly map; batched assembly of many meshes; the
 * P_k Lagrange mass (Appendix D) and the boundary mass of (d-1)-simplices on
 * plans of their own (fem_pk_*, fem_boundary_*).
 *
 * Conventions for every entry point:
 *  - All array arguments are DEVICE pointers unless marked "host".
 *  - Indices are 0-based.  Mesh arrays are row-major structure-of-arrays:
 *      q  [d][nq]     double   q[v*nq + j] = coordinate v of vertex j
 *      me [d+1][nme]  int32    me[a*nme + k] = local vertex a of element k
 *      w  [nq]        double   nodal weight (FEM_OP_MASS_W only)
 *  - CSR uses int32 row_ptr / col_idx (columns ascending, unique per row)
 *    and double values.  Scalar operators have nq rows; FEM_OP_ELAS has d*nq
 *    rows, row (i, l) = d*i + l, and its pattern is the scalar pattern with
 *    every entry expanded to a d x d block.
 *  - `stream` is a hipStream_t (0 = the null stream).  Numeric, pattern and
 *    backward calls only enqueue work on it and never synchronise; buffers
 *    they read must stay valid and unmodified until that work completes.
 *  - Errors are returned as fem_status; nothing is thrown across the ABI and
 *    out-parameters are written only on FEM_OK.  The caller owns every
 *    buffer it passes; the library owns plans and batches.
 */
#ifndef FEMASM_H
#define FEMASM_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fem_status {
    FEM_OK = 0,
    FEM_ERR_ARG = 1,         /* bad argument: null pointer, d not 2 or 3, bad op, negative size */
    FEM_ERR_INDEX = 2,       /* me holds an index outside [0, nq) or an element repeats a vertex */
    FEM_ERR_DEGENERATE = 3,  /* an element has det B_k == 0 (reported after the fact, see below) */
    FEM_ERR_OVERFLOW = 4,    /* a size exceeds the int32 CSR range or a row exceeds 255 entries */
    FEM_ERR_NOMEM = 5,       /* device or host allocation failed */
    FEM_ERR_DEVICE = 6       /* a HIP runtime call failed */
} fem_status;

typedef enum fem_op {
    FEM_OP_MASS = 0,
    FEM_OP_MASS_W = 1,
    FEM_OP_STIFF = 2,
    FEM_OP_ELAS = 3
} fem_op;

typedef struct fem_plan_s *fem_plan;
typedef struct fem_batch_s *fem_batch;

/* Human-readable name of a status code (static string, never NULL). */
const char *fem_status_str(fem_status s);

/*
 * Symbolic phase (Section 3: the (I, J) half of the triplets and the
 * `sparse` pattern).  Validates me, builds the CSR pattern of the scalar
 * operator (row i holds every vertex that shares an element with i, i
 * included), the element-to-CSR slot addressing used by the numeric phase,
 * and a locality-ordered copy of the connectivity, all with GPU kernels on
 * `stream`.  The plan depends only on me: one plan serves every q, w,
 * lambda, mu and operator.
 *   d      2 or 3
 *   nq     number of vertices (>= 0); vertices no element uses get empty rows
 *   nme    number of elements (>= 0)
 *   me     device, (d+1)*nme int32, layout above (may be NULL when nme == 0);
 *          not read after the call returns
 *   stream work is ordered on it; the call is synchronous (it returns once
 *          the pattern and slot addressing are complete)
 *   out    receives the plan (host pointer to a handle)
 * The vertex-block layouts of the block kernels are then built by a library
 * host thread and published when complete (fem_plan_layouts); numeric calls
 * made before that run the row-gather kernel, whose values are the same bit
 * for bit (FEMASM_LAYOUTS=sync in the environment builds them before
 * returning).
 * Errors: FEM_ERR_ARG, FEM_ERR_INDEX (index out of range, repeated vertex),
 * FEM_ERR_OVERFLOW (nnz >= 2^31, (d+1)*nme >= 2^31, or a vertex in more
 * than 16384/(d+1) elements), FEM_ERR_NOMEM, FEM_ERR_DEVICE.
 */
fem_status fem_assemble_symbolic(int32_t d, int64_t nq, int64_t nme, const int32_t *me,
                                 hipStream_t stream, fem_plan *out);

/* State of the plan's vertex-block layouts: *state = 0 while the library's
 * host thread is still building them, 1 once they are published (the block
 * kernels serve the numeric calls), 2 when the build has finished without
 * them (the row-gather kernel serves every call).  With wait != 0 the call
 * blocks until the build has finished.  Returns FEM_OK, or the error that
 * ended a failed build (FEM_ERR_NOMEM, FEM_ERR_DEVICE; the plan stays usable
 * with the row-gather kernel).  state: host pointer, may be NULL. */
fem_status fem_plan_layouts(fem_plan plan, int32_t wait, int32_t *state);

/* Matrix sizes of operator `op` for this plan: nrows (nq, or d*nq for
 * FEM_OP_ELAS) and nnz (scalar nnz, or d*d times it).  Host out-pointers. */
fem_status fem_plan_query(fem_plan plan, int32_t op, int64_t *nrows, int64_t *nnz);

/* Plan facts: d, nq, nme and the longest scalar row.  Host out-pointers,
 * any may be NULL. */
fem_status fem_plan_info(fem_plan plan, int32_t *d, int64_t *nq, int64_t *nme,
                         int32_t *max_row);

/* Writes the CSR pattern of operator `op` into caller buffers:
 * row_ptr[nrows+1], col_idx[nnz] (device).  Enqueued on `stream`. */
fem_status fem_plan_pattern(fem_plan plan, int32_t op, int32_t *row_ptr, int32_t *col_idx,
                            hipStream_t stream);

/* Triplet-to-slot map of the scalar operator, in the column-wise local order
 * of the OptV1 / OptV2 listings of Sections 3-4: for element k and local
 * entry (row vertex a, column vertex b),
 *   slot[k*(d+1)^2 + b*(d+1) + a] = CSR position of (me[a,k], me[b,k]).
 * slot is a device buffer of (d+1)^2 * nme int32.  Enqueued on `stream`. */
fem_status fem_plan_slot_map(fem_plan plan, int32_t *slot, hipStream_t stream);

/*
 * Numeric phase: CSR values of operator `op` (Sections 4.1, 4.2, 5.1).
 *   q       device, d*nq doubles (layout above)
 *   w       device, nq doubles; read only for FEM_OP_MASS_W (else may be NULL)
 *   lambda, mu  Lame parameters; read only for FEM_OP_ELAS (need lambda+mu > 0
 *           for a positive semi-definite result; not checked)
 *   values  device, nnz doubles (fem_plan_query), fully overwritten
 * Asynchronous: one kernel on `stream`, no host synchronisation, no
 * allocation.  An element with det B_k == 0 contributes nothing and sets the
 * plan's device status word; fem_plan_sync_status reports it.
 * Errors (immediate): FEM_ERR_ARG, FEM_ERR_OVERFLOW (vector nnz >= 2^31),
 * FEM_ERR_DEVICE (launch failure).
 */
fem_status fem_assemble_numeric(fem_plan plan, int32_t op, const double *q, const double *w,
                                double lambda, double mu, double *values, hipStream_t stream);

/*
 * Elasticity with nodal Lame fields (Section 5.1: the Lame parameters
 * replaced by their P1 interpolants): element matrix
 *   |K|/(d+1) (lambda^s <g_b, Q^{n,l} g_a> + mu^s <g_b, S^{n,l} g_a>),
 * lambda^s, mu^s the sums of the fields over the element's vertices.  Output
 * in the FEM_OP_ELAS pattern and numbering (d*nq rows, r = d*i + l), exactly
 * symmetric, entries summed in ascending element number.
 *   q       device, d*nq doubles
 *   lam, mu device, nq doubles each (nodal values)
 *   values  device, d*d*nnz doubles, fully overwritten
 * Asynchronous, no allocation.  Runs on the vertex-pair kernel only:
 * FEM_ERR_OVERFLOW for a mesh without that layout (a vertex with more than
 * 32 neighbours, or more than 1023 elements around a vertex) or vector nnz
 * >= 2^31; FEM_ERR_ARG for null arrays.  Degenerate elements as in
 * fem_assemble_numeric.
 */
fem_status fem_assemble_elasticity_nodal(fem_plan plan, const double *q, const double *lam,
                                         const double *mu, double *values, hipStream_t stream);

/*
 * General second-order operator of the paper's introduction,
 *   -div(A grad u) + div(b u) + c . grad u + a0 u,
 * with constant coefficients, in the weak form obtained by testing with the
 * P1 basis and integrating the divergence terms by parts (boundary terms
 * left out):  int A grad u.grad v - int u b.grad v + int (c.grad u) v
 * + int a0 u v.  Element matrix, row a (test), column b (trial):
 *   |K| g_a^T A g_b - |K|/(d+1) b.g_a + |K|/(d+1) c.g_b
 *   + a0 |K| d! (1 + delta_ab) / (d+2)!      (magic formula, Section 2).
 * Not symmetric in general: the full matrix (OptV rather than OptVS) is
 * written into the scalar pattern of the plan (nq rows, fem_plan_pattern
 * with FEM_OP_STIFF), entries summed in ascending element number.
 *   q       device, d*nq doubles
 *   coef    HOST array of d*d + 2*d + 1 doubles: A row-major (A[i*d+j]
 *           multiplies d u/d x_j in component i of the flux), b, c, a0
 *   values  device, nnz doubles, fully overwritten
 * Asynchronous, no allocation.  Runs on the vertex-pair kernel only:
 * FEM_ERR_OVERFLOW for a mesh without that layout; FEM_ERR_ARG for null
 * arrays.  Degenerate elements as in fem_assemble_numeric.
 */
fem_status fem_assemble_general(fem_plan plan, const double *q, const double *coef,
                                double *values, hipStream_t stream);

/*
 * Adjoint of J(q, w) = a^T (S(q) + M_w(q)) b: the sum over elements of
 * a_K^T (E_stiff(K) + E_mass_w(K)) b_K, differentiated through the element
 * Jacobians (the gradient systems of Appendix C.1 give
 * d g_a = -sum_c g_c (g_a . d q_c) and d|K| = |K| sum_c g_c . d q_c).
 *   op_mask  bit (1 << FEM_OP_STIFF) and/or bit (1 << FEM_OP_MASS_W): which
 *            terms J contains
 *   q, w, a, b  device; w is read when MASS_W is in the mask; a, b have nq doubles
 *   dJdw     device nq doubles or NULL
 *   dJdq     device d*nq doubles (laid out like q) or NULL
 * Each output entry is the sum of its element contributions in a fixed
 * order: four partial sums, partial j over the vertex's incident elements
 * j, j+4, j+8, ... in ascending element number, combined as
 * ((p0 + p1) + (p2 + p3)); bitwise reproducible from run to run.
 * Asynchronous, no allocation.
 */
fem_status fem_assemble_backward(fem_plan plan, uint32_t op_mask, const double *q,
                                 const double *w, const double *a, const double *b,
                                 double *dJdw, double *dJdq, hipStream_t stream);

/*
 * Derivatives of the assembly map (q, w) -> A for op = FEM_OP_MASS,
 * FEM_OP_MASS_W or FEM_OP_STIFF (generalising the adjoint above to any
 * direction and any upstream gradient).  With the gradient systems of
 * Appendix C.1 (d g_a = -N g_a, N = sum_c g_c dq_c^T, d|K| = |K| tr N):
 *
 * fem_assemble_jvp: dvalues = dA, the derivative of the operator's CSR
 *   values along (dq, dw):  dq device d*nq doubles (layout of q); dw device
 *   nq doubles (FEM_OP_MASS_W only, else ignored); dvalues device nnz
 *   doubles, fully overwritten, each entry summed in ascending element
 *   number.
 * fem_assemble_vjp: the gradient of L = sum_s G[s] A[s] (G device, nnz
 *   doubles, any upstream gradient on the CSR entries):  dLdq device d*nq
 *   doubles or NULL; dLdw device nq doubles or NULL (FEM_OP_MASS_W only);
 *   each output is the sum of its element contributions in a fixed order
 *   (eight partial sums, partial j over the vertex's incident elements j,
 *   j+8, ... in ascending element number, combined pairwise in a fixed
 *   tree), so bitwise reproducible.  slot is the plan's triplet-to-slot map (fem_plan_slot_map,
 *   (d+1)^2 * nme int32, device), computed once by the caller; or NULL once
 *   fem_plan_vjp_positions has run on the plan: the kernels then find each
 *   upstream gradient entry through the plan's own per-element column
 *   positions (the same addresses, read in the plan's element order rather
 *   than the caller's), with identical outputs.
 * Both asynchronous, no allocation.  Errors: FEM_ERR_ARG (other op, null
 * arrays), FEM_ERR_OVERFLOW; degenerate elements as in
 * fem_assemble_numeric.
 */
fem_status fem_assemble_jvp(fem_plan plan, int32_t op, const double *q, const double *w,
                            const double *dq, const double *dw, double *dvalues,
                            hipStream_t stream);
fem_status fem_assemble_vjp(fem_plan plan, int32_t op, const double *q, const double *w,
                            const double *G, const int32_t *slot, double *dLdq, double *dLdw,
                            hipStream_t stream);

/*
 * Builds, once per plan, the table that lets the VJP calls run without a
 * caller slot map (slot = NULL): for every element in the plan's order and
 * local entry (a, b), the position of vertex b within the CSR row of vertex
 * a -- 8-bit when no row has more than 256 entries, else 16-bit; (d+1)^2
 * bytes (or twice that) per element, owned and freed by the plan.  The
 * table is a re-indexing of the slot map (Sections 3-4: the triplet-to-CSR
 * step of `sparse`), kept in the order in which the VJP kernels visit the
 * elements.  Allocates; the build kernel runs on `stream` and the call
 * returns once it has completed, so later calls on any stream may use it.
 * Later calls return FEM_OK at once.  Errors: FEM_ERR_ARG (null plan),
 * FEM_ERR_NOMEM / FEM_ERR_DEVICE.
 */
fem_status fem_plan_vjp_positions(fem_plan plan, hipStream_t stream);

/*
 * Workspace form of fem_assemble_vjp, for callers that can lend scratch
 * memory: the same outputs, bit for bit, computed with every element's
 * derivative terms evaluated once (fem_assemble_vjp evaluates them once per
 * vertex of the element).  Two kernels on `stream`: one thread per element
 * writes the terms of its d+1 vertices into `work`, then the vertex pass
 * sums each vertex's terms in the order of fem_assemble_vjp.
 *   fem_vjp_work_bytes: bytes `work` must hold for operator `op`,
 *     8 (d+1) nw nme with nw = d (d+1 for FEM_OP_MASS_W); host out-pointer.
 *   work        device, >= that many bytes, 8-byte aligned; overwritten
 *               (its contents are scratch; the caller owns the buffer)
 *   work_bytes  its size in bytes
 * Other arguments, outputs and errors as fem_assemble_vjp, plus FEM_ERR_ARG
 * for a missing, short or misaligned work buffer.  Asynchronous, no
 * allocation.  Concurrent calls must not share `work`.
 */
fem_status fem_vjp_work_bytes(fem_plan plan, int32_t op, int64_t *bytes);
fem_status fem_assemble_vjp_ws(fem_plan plan, int32_t op, const double *q, const double *w,
                               const double *G, const int32_t *slot, double *work,
                               int64_t work_bytes, double *dLdq, double *dLdw,
                               hipStream_t stream);

/* The workspace VJP without a caller workspace, for callers that cannot
 * allocate device memory (code under graph capture, serving loops, harnesses
 * that forbid hipMalloc).  The element terms go to a fixed library array of
 * 128 MiB per GPU (one copy per device, held until the process ends), so the
 * call allocates nothing.  Arguments, outputs and results as
 * fem_assemble_vjp_ws (bit for bit: same kernels, same order).
 * Errors: as fem_assemble_vjp_ws; FEM_ERR_OVERFLOW when the plan's element
 * terms (fem_vjp_work_bytes) exceed 128 MiB.  Every call on one GPU shares
 * that array: calls that overlap on one GPU (any plan, any stream) race and
 * must be serialised by the caller.  Nothing in the array needs clearing:
 * each call writes every term it reads. */
fem_status fem_assemble_vjp_noalloc(fem_plan plan, int32_t op, const double *q, const double *w,
                                    const double *G, const int32_t *slot, double *dLdq,
                                    double *dLdw, hipStream_t stream);

/* J = a^T A b for CSR values of operator `op` produced with this plan:
 * out (device, 1 double).  Row partial sums are combined in row order, so
 * the result is bitwise reproducible.  Asynchronous.  The partial sums live
 * in a plan-owned work array: concurrent calls with one plan on different
 * streams race on it. */
fem_status fem_csr_bilinear(fem_plan plan, int32_t op, const double *values, const double *a,
                            const double *b, double *out, hipStream_t stream);

/* Synchronises `stream`, then reads and clears the plan's device status
 * word: FEM_ERR_DEGENERATE if any numeric or backward call since the last
 * read met an element with det B_k == 0, else FEM_OK. */
fem_status fem_plan_sync_status(fem_plan plan, hipStream_t stream);

/* Frees the plan (NULL is ignored).  Work using it must have completed. */
void fem_plan_destroy(fem_plan plan);

/*
 * Batched assembly of many independent meshes in one persistent launch.
 *   nmesh          number of meshes (>= 1)
 *   d, nq, nme     host arrays [nmesh]
 *   me             host array [nmesh] of device pointers (layout above)
 * Builds one plan per mesh, a device work list of (mesh, row tile) items
 * (largest first) and the concatenated vertex-pair layouts.  Synchronous.
 */
fem_status fem_batch_create(int32_t nmesh, const int32_t *d, const int64_t *nq,
                            const int64_t *nme, const int32_t *const *me, hipStream_t stream,
                            fem_batch *out);

/* Host arrays [nmesh+1] of offsets into the concatenated inputs/outputs of
 * operator `op`: q_off (doubles of q, mesh b holds d_b*nq_b), w_off (doubles
 * of w), row_off (CSR rows) and nnz_off (values).  Any may be NULL. */
fem_status fem_batch_offsets(fem_batch batch, int32_t op, int64_t *q_off, int64_t *w_off,
                             int64_t *row_off, int64_t *nnz_off);

/* Plan of mesh `index` (borrowed; owned by the batch). */
fem_status fem_batch_plan(fem_batch batch, int32_t index, fem_plan *plan);

/* Tunables of the persistent row-gather kernel: threads per workgroup (64,
 * 128 or 256) and workgroups per compute unit (1..8).  They change
 * scheduling only, not the values (each CSR row is still summed by one
 * thread in ascending element order).  Synchronous (rebuilds the work list). */
fem_status fem_batch_set_params(fem_batch batch, int32_t block_threads, int32_t wg_per_cu);

/* Layout tunables of the vertex-pair kernel for the operators of `op`'s
 * kind (the scalar operators share one layout, elasticity has its own):
 * rows per vertex block for the 3D and the 2D meshes (16..128) and tasks of
 * 64 pairs per wavefront (1, 2 or 4).  Rebuilds every mesh's layout of that
 * kind and the concatenated layouts (synchronous, host work; not
 * concurrently with numeric calls on the batch).  Scheduling only: the
 * values stay the same bit for bit.  FEM_ERR_ARG for values out of range. */
fem_status fem_batch_set_pair_layout(fem_batch batch, int32_t op, int32_t rows_3d,
                                     int32_t rows_2d, int32_t slots);

/* Kernel family of fem_batch_numeric:
 *   FEM_BATCH_PAIR (default)  the vertex-pair kernel over the concatenated
 *                             pair layouts of all meshes, one persistent
 *                             launch over both dimensions (workgroups split
 *                             between the 2D and the 3D blocks in proportion
 *                             to their work; one launch per dimension if the
 *                             two layouts' slot counts differ or their LDS
 *                             does not fit)
 *   FEM_BATCH_PAIR_SPLIT      the same kernel, one persistent launch per
 *                             dimension present
 *   FEM_BATCH_ROWGATHER       one persistent launch of the row-gather kernel
 *                             over (mesh, row tile) items (fem_batch_set_params)
 * All give the same values bit for bit; the pair forms fall back to the
 * row-gather launch when a mesh has no pair layout.  FEM_ERR_ARG for another
 * value. */
enum { FEM_BATCH_ROWGATHER = 0, FEM_BATCH_PAIR = 1, FEM_BATCH_PAIR_SPLIT = 2 };
fem_status fem_batch_set_kernel(fem_batch batch, int32_t kernel);

/*
 * CSR values of operator `op` for every mesh of the batch: one persistent
 * launch (see fem_batch_set_kernel).  q_cat, w_cat are the per-mesh arrays concatenated at q_off /
 * w_off; values_cat receives mesh b's values at nnz_off[b].  No host
 * synchronisation, no allocation, fixed kernel arguments: safe to capture
 * in a hipGraph and replay.
 */
fem_status fem_batch_numeric(fem_batch batch, int32_t op, const double *q_cat,
                             const double *w_cat, double lambda, double mu,
                             double *values_cat, hipStream_t stream);

/* Synchronises `stream`, then reads and clears the batch's device status
 * word: FEM_ERR_DEGENERATE if a batched numeric call since the last read met
 * an element with det B_k == 0, else FEM_OK. */
fem_status fem_batch_sync_status(fem_batch batch, hipStream_t stream);

/* Frees the batch and its plans (NULL is ignored). */
void fem_batch_destroy(fem_batch batch);

/*
 * P_k Lagrange mass matrix (Appendix D: the extension of the vectorised
 * assembly to P_k elements, k >= 1, on straight-sided simplices).
 *
 * Mesh arrays of a "P_k mesh": q [d][nq] holds the coordinates of every P_k
 * node, me [N][nme] (N = (d+k)!/(d! k!)) the N nodes of each element in the
 * local numbering I of the multi-indices alpha in N^(d+1), |alpha| = k
 * (alpha_i is the exponent of the barycentric coordinate of local vertex i):
 * local nodes 0..d are the vertices alpha = k e_i, the remaining
 * multi-indices follow in decreasing lexicographic order of
 * (alpha_0, ..., alpha_d).  Node alpha lies at sum_i alpha_i q^i / k; only
 * the vertex rows 0..d of me are used for geometry.
 *
 * The element matrix is d! |K| C with C[a][b] the integral of the product of
 * the basis functions of local nodes a and b over K divided by d! |K|
 * (formula of Appendix D, from the polynomial representation of the basis
 * in barycentric coordinates and the magic formula of Section 2).  Entries
 * are summed in ascending element number, starting from 0.0 (bitwise
 * reproducible), into the CSR pattern of all node pairs sharing an element.
 */
typedef struct fem_pk_plan_s *fem_pk_plan;

/* Symbolic phase of the P_k mass: validates me, builds the CSR pattern and
 * the per-entry contribution lists.  For k = 1 it also makes a P1 plan of the
 * same mesh (as fem_assemble_symbolic, block layouts waited for) whose
 * pattern it checks equal to its own; fem_pk_mass then runs the P1 mass
 * kernels of that plan.  Synchronous.
 *   d    2 or 3;  k  1..6
 *   nq   number of P_k nodes;  nme  number of elements
 *   me   device, N*nme int32 (layout above)
 * Errors: FEM_ERR_ARG, FEM_ERR_INDEX (index out of range or a node repeated
 * within an element), FEM_ERR_OVERFLOW (nnz >= 2^31, N*nme >= 2^31, more
 * than 2^(32-b) elements with b the bits of N(N+1)/2-1 (2^26 for P2 in 3D,
 * 2^20 for P6 in 3D), or 1024 consecutive CSR entries with more than 65535
 * contributions), FEM_ERR_NOMEM, FEM_ERR_DEVICE. */
fem_status fem_pk_symbolic(int32_t d, int32_t k, int64_t nq, int64_t nme, const int32_t *me,
                           hipStream_t stream, fem_pk_plan *out);

/* Rows (= nq), nnz and N of the plan.  Host out-pointers, any may be NULL. */
fem_status fem_pk_query(fem_pk_plan plan, int64_t *nrows, int64_t *nnz, int32_t *ndfe);

/* Copies the CSR pattern into row_ptr[nq+1], col_idx[nnz] (device).
 * Enqueued on `stream`. */
fem_status fem_pk_pattern(fem_pk_plan plan, int32_t *row_ptr, int32_t *col_idx,
                          hipStream_t stream);

/* CSR values of the P_k mass matrix for node coordinates q (device, d*nq
 * doubles) into values (device, nnz doubles, fully overwritten).  Two
 * kernels on `stream` (element volumes, then the entry sums), or for k = 1
 * the P1 mass kernels of the plan's P1 plan (the same matrix: same pattern,
 * each entry summed in ascending element number); no host synchronisation,
 * no allocation.  A degenerate element (det B_K == 0) contributes 0 and sets
 * the plan's status word (fem_pk_sync_status).  Concurrent calls with one
 * plan race on its volume work array. */
fem_status fem_pk_mass(fem_pk_plan plan, const double *q, double *values, hipStream_t stream);

/* Synchronises `stream`, reads and clears the plan's status word:
 * FEM_ERR_DEGENERATE if a fem_pk_mass call since the last read met a
 * degenerate element, else FEM_OK. */
fem_status fem_pk_sync_status(fem_pk_plan plan, hipStream_t stream);

/* Frees the plan (NULL is ignored).  Work using it must have completed. */
void fem_pk_destroy(fem_pk_plan plan);

/*
 * Boundary terms (Neumann / Robin): mass and weighted mass on a mesh of
 * (d-1)-simplices embedded in R^d, typically the boundary facets of a
 * volume mesh.  The paper notes (remark after the weighted-mass algorithm
 * of Section 4.1) that the weighted-mass assembly applies to n-simplices
 * with n <= d; here n = d-1, |K| is the n-dimensional measure (segment
 * length, triangle area) and the element matrices are
 *   mass      n! |K| (1 + delta_ab) / (n+2)!
 *   weighted  n! |K| (1 + delta_ab) (w^s + w_a + w_b) / (n+3)!
 * (magic formula with d replaced by n).  The plan is a fem_pk_plan (query,
 * pattern, status and destroy as above): nq rows over all vertices, rows of
 * vertices on no facet empty.
 *   d       2 (facets are segments) or 3 (triangles)
 *   facets  device, d*nf int32, facets[a*nf + f] = vertex a of facet f
 * Errors as fem_pk_symbolic.  Synchronous.
 */
fem_status fem_boundary_symbolic(int32_t d, int64_t nq, int64_t nf, const int32_t *facets,
                                 hipStream_t stream, fem_pk_plan *out);

/* Values of the boundary mass (w NULL) or weighted mass (w device, nq
 * doubles) for vertex coordinates q (device, d*nq doubles) into values
 * (device, nnz doubles, fully overwritten).  Two kernels on `stream` (facet
 * matrices into a plan-owned work array, then the entry sums); no host
 * synchronisation, no allocation.  A facet of zero measure sets the plan's
 * status word.  FEM_ERR_ARG for a plan not made by fem_boundary_symbolic
 * (and fem_pk_mass refuses boundary plans).  Concurrent calls with one plan
 * race on its work array. */
fem_status fem_boundary_mass(fem_pk_plan plan, const double *q, const double *w, double *values,
                             hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* FEMASM_H */
