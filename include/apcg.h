/*
 * apcg.h -- C ABI of the asynchronous, device-resident PCG library for
 * AMD Instinct MI355X (gfx950).
 *
 * The library implements the programming model of Faibussowitsch, Adams,
 * Mills, Zampini and Zhang, "Safe, Seamless, And Scalable Integration Of
 * Asynchronous GPU Streams In PETSc" (arXiv 2306.17801), for the
 * preconditioned conjugate-gradient hot path:
 *
 *   - an execution context owns one HIP stream and is the only way work is
 *     ordered (Section 3.1); the stream itself is never handed out
 *     (Section 2.1 explains why exposing it is unsafe);
 *   - every operation declares which objects it reads and writes, and
 *     operations on different contexts touching a common object are ordered
 *     write-write, write-read and read-write by call order, while reads are
 *     not ordered among themselves (Section 3.1.2, the formal ordering rule);
 *   - scalars produced by reductions stay on the device as futures and feed
 *     later operations without a host round trip (Sections 2.3 and 3.2.2);
 *   - the PCG iteration keeps alpha, beta, the residual norm and the
 *     convergence flag on the device; kernels queued after convergence
 *     return immediately, which is the device-side convergence check the
 *     paper leaves as future work (Section 5).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *   - Every function returns apcg_status.  APCG_SUCCESS (0) means the call
 *     was accepted (for asynchronous calls: enqueued).  On any other value
 *     nothing was enqueued and apcg_last_error() returns a message
 *     (thread-local, valid until the next failing call on the thread).
 *   - A vector that a call writes (a solve's x, MatMult's y) may share no
 *     memory with the vectors it reads: the same handle twice or two
 *     overlapping address ranges [d, d + n) return APCG_ERR_INVALID_ARG.
 *   - Numerical failures of asynchronous work (breakdown, NaN, iteration
 *     limit) are not return codes: they are written to device-resident
 *     solve-info words and read with apcg_info_get().
 *   - A NULL context argument means the per-device globally blocking
 *     context: the call waits for all earlier work on every context of the
 *     device and has finished when it returns (Section 3.1, "globally
 *     blocking" streams; Section 3.2.2, Eval without a context).
 *   - Pointers named dev_* are device (HBM) pointers; pointers named host_*
 *     are ordinary host memory.  Vector and matrix memory is BORROWED: the
 *     caller allocates it (e.g. as PyTorch tensors) and keeps it alive until
 *     every operation using it has finished (apcg_ctx_synchronize or an
 *     accessor).  Library objects (contexts, scalars, wrappers, info
 *     arrays) are owned by the library; destroying them is always safe,
 *     their resources are released once the device no longer uses them
 *     (Section 3.2.2, lifetime of ManagedMemory).
 *   - Floating point is IEEE binary64 throughout the solver; indices are
 *     int32 (row pointers and column indices), sizes int64 where a vector
 *     may exceed 2^31 elements.
 *   - Thread safety: the object registry is internally locked; a single
 *     context must not be used by two host threads at the same time.
 */
#ifndef APCG_H
#define APCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define APCG_ABI_VERSION 1

/* ---------------------------------------------------------------------- */
/* Status codes returned by every call                                     */
/* ---------------------------------------------------------------------- */
typedef int32_t apcg_status;
#define APCG_SUCCESS 0
#define APCG_ERR_INVALID_ARG 1   /* NULL handle, size mismatch, bad enum ...   */
#define APCG_ERR_INVALID_STATE 2 /* e.g. object used after destroy            */
#define APCG_ERR_HIP 3           /* the HIP runtime reported an error          */
#define APCG_ERR_OUT_OF_MEMORY 4
#define APCG_ERR_UNSUPPORTED 5   /* valid request the library does not serve   */

/* ---------------------------------------------------------------------- */
/* Solve-status bits written by the device (apcg_solve_info.status)        */
/* ---------------------------------------------------------------------- */
#define APCG_SOLVE_RUNNING 0         /* no terminal state reached           */
#define APCG_SOLVE_CONVERGED 1       /* ||r|| <= rtol * reference norm        */
#define APCG_SOLVE_MAXIT 2           /* iteration limit reached               */
#define APCG_SOLVE_BREAKDOWN_PAP 4   /* p.Ap <= 0: operator not SPD           */
#define APCG_SOLVE_BREAKDOWN_RZ 8    /* r.z <= 0: preconditioner not SPD      */
#define APCG_SOLVE_NAN 16            /* a non-finite norm or inner product    */
#define APCG_SOLVE_STALL 32          /* no progress within the stall window   */
#define APCG_SOLVE_FALLBACK 64       /* fell back to Jacobi-PCG               */
#define APCG_SOLVE_SETUP_ERROR 128   /* missing or non-positive diagonal      */

/* ---------------------------------------------------------------------- */
/* Opaque handles                                                          */
/* ---------------------------------------------------------------------- */
typedef struct apcg_ctx_s *apcg_ctx;       /* device + one managed stream   */
typedef struct apcg_scalar_s *apcg_scalar; /* one device-resident double    */
typedef struct apcg_vec_s *apcg_vec;       /* borrowed dense double vector  */
typedef struct apcg_mat_s *apcg_mat;       /* borrowed CSR matrix           */
typedef struct apcg_info_s *apcg_info;     /* device-resident solve results */
typedef struct apcg_timer_s *apcg_timer;   /* pair of stream timestamps     */

/* Stream types (Section 3.1). */
#define APCG_STREAM_DEFAULT 0         /* asynchronous w.r.t. host and other contexts */
#define APCG_STREAM_GLOBAL_BLOCKING 1 /* waits for all contexts; done on return      */

/* Join modes for apcg_ctx_join. */
#define APCG_JOIN_DESTROY 0 /* parent waits for the children, children destroyed    */
#define APCG_JOIN_SYNC 1    /* parent waits; host also waits for the children        */
#define APCG_JOIN_NO_SYNC 2 /* parent waits for the children; nothing else          */

/* ---------------------------------------------------------------------- */
/* Execution contexts (Section 3.1, core stream-control listing; fork and  */
/* join appear in the paper only as API names, read here as: children start */
/* after everything the parent has enqueued so far, and joining makes the   */
/* parent wait for everything the children enqueued).                       */
/* ---------------------------------------------------------------------- */

/* Creates a context on HIP device `device` with its own non-blocking stream
 * (default priority).  stream_type: APCG_STREAM_DEFAULT or
 * APCG_STREAM_GLOBAL_BLOCKING.  *out receives the handle. */
apcg_status apcg_ctx_create(int32_t device, int32_t stream_type, apcg_ctx *out);

/* Destroys the handle immediately; the stream and scratch memory are
 * released once the work already enqueued on it has finished. */
apcg_status apcg_ctx_destroy(apcg_ctx ctx);

/* Makes all later work of `waiter` start after all work enqueued on
 * `waitee` so far (no host wait). */
apcg_status apcg_ctx_wait_for(apcg_ctx waiter, apcg_ctx waitee);

/* *idle = 1 if every operation enqueued on ctx has finished, else 0.
 * Never blocks. */
apcg_status apcg_ctx_query_idle(apcg_ctx ctx, int32_t *idle);

/* Blocks the host until every operation enqueued on ctx has finished. */
apcg_status apcg_ctx_synchronize(apcg_ctx ctx);

/* Creates n children of the parent's device and stream type; each child's
 * first operation starts after everything enqueued on the parent so far.
 * children: caller-provided array of n handles (output). */
apcg_status apcg_ctx_fork(apcg_ctx parent, int32_t n, apcg_ctx *children);

/* The parent waits (on the device) for all work enqueued on the n children;
 * mode APCG_JOIN_DESTROY then destroys them (the handles become invalid),
 * APCG_JOIN_SYNC additionally blocks the host until the children are idle,
 * APCG_JOIN_NO_SYNC does nothing more. */
apcg_status apcg_ctx_join(apcg_ctx parent, int32_t n, int32_t mode, apcg_ctx *children);

/* *stream_type receives the context's stream type. */
apcg_status apcg_ctx_get_stream_type(apcg_ctx ctx, int32_t *stream_type);

/* ---------------------------------------------------------------------- */
/* Dependency marking on arbitrary objects (Section 3.1.2)                 */
/* ---------------------------------------------------------------------- */

/* Access modes of a marked operation. */
#define APCG_ACCESS_READ 1
#define APCG_ACCESS_WRITE 2
#define APCG_ACCESS_READ_WRITE 3

/* *stream receives the context's hipStream_t (as void *), for enqueuing the
 * caller's own work between apcg_mark_intent_begin and _end.  The stream
 * stays owned by the library: never destroy it, and never use it after the
 * context is destroyed. */
apcg_status apcg_ctx_get_stream(apcg_ctx ctx, void **stream);

/* Registers the device memory region [ptr, ptr + bytes) of `device` as an
 * object for dependency marking and returns its id (never 0, never reused).
 * Registering the same start pointer again with the same size returns the
 * existing id; with another size, or for a region that overlaps a
 * registered one, APCG_ERR_INVALID_ARG.  The library never dereferences
 * ptr.  A region registered here and a vector wrapping the same memory are
 * different objects for ordering; mark the vector through its own id. */
apcg_status apcg_memory_register(int32_t device, const void *ptr, int64_t bytes, uint64_t *id);

/* Finds the registered region of `device` containing ptr: *id and (if not
 * NULL) *start and *bytes; APCG_ERR_INVALID_ARG when there is none. */
apcg_status apcg_memory_lookup(int32_t device, const void *ptr, uint64_t *id, const void **start, int64_t *bytes);

/* Forgets a registered region (the caller's memory is untouched; pending
 * work on it keeps its own ordering). */
apcg_status apcg_memory_unregister(uint64_t id);

/* Ids of library objects, for marking the caller's own work on them. */
apcg_status apcg_vec_get_id(apcg_vec v, uint64_t *id);
apcg_status apcg_scalar_get_id(apcg_scalar s, uint64_t *id);
apcg_status apcg_mat_get_id(apcg_mat A, uint64_t *id);

/* Bracket the caller's own work on object `id` enqueued on ctx's stream
 * (Section 3.1.2, MarkIntent).  _begin makes ctx's stream wait (on the
 * device, no host wait) for the conflicting earlier accesses of other
 * contexts: a write waits for the last write and every read since it, a
 * read for the last write; reads are not ordered among themselves; earlier
 * operations of the same context are ordered by the stream.  _end records
 * the completion point of this access.  The begin/end pair must use the
 * same ctx, id and mode; description (may be NULL) names the operation in
 * error messages.  On a globally blocking context, _begin waits for the
 * whole device and _end for the stream. */
apcg_status apcg_mark_intent_begin(apcg_ctx ctx, uint64_t id, int32_t mode, const char *description);
apcg_status apcg_mark_intent_end(apcg_ctx ctx, uint64_t id, int32_t mode, const char *description);

/* ---------------------------------------------------------------------- */
/* Device scalars: futures of one double (Sections 3.2 and 3.2.2)          */
/* ---------------------------------------------------------------------- */

/* Allocates a device scalar on ctx's device and enqueues its
 * initialisation to 0 on ctx. */
apcg_status apcg_scalar_create(apcg_ctx ctx, apcg_scalar *out);

/* Releases the scalar once every operation that uses it has finished. */
apcg_status apcg_scalar_destroy(apcg_scalar s);

/* Enqueues s = value on ctx (value captured at call time; no host sync). */
apcg_status apcg_scalar_set(apcg_scalar s, double value, apcg_ctx ctx);

/* The host accessor ("front()" in the PCG listing of Section 3.3): waits
 * only for the last operation that wrote s, then copies its value to
 * *host_value. */
apcg_status apcg_scalar_get(apcg_scalar s, double *host_value);

/* Scalar arithmetic on the device (the fixed expressions the PCG loop
 * evaluates with Eval in Section 3.3: beta/betaold, beta/a, -a, 1/alpha).
 * out = op(a[, b]); b must be NULL for unary opcodes and non-NULL for
 * binary ones.  out may alias a or b.  Runs as one single-thread kernel on
 * ctx. */
#define APCG_SCALAR_COPY 0  /* out = a      */
#define APCG_SCALAR_NEG 1   /* out = -a     */
#define APCG_SCALAR_RECIP 2 /* out = 1 / a  */
#define APCG_SCALAR_SQRT 3  /* out = sqrt a */
#define APCG_SCALAR_ADD 4   /* out = a + b  */
#define APCG_SCALAR_SUB 5   /* out = a - b  */
#define APCG_SCALAR_MUL 6   /* out = a * b  */
#define APCG_SCALAR_DIV 7   /* out = a / b  */
apcg_status apcg_scalar_op(int32_t opcode, apcg_scalar out, apcg_scalar a, apcg_scalar b, apcg_ctx ctx);

/* Scalar expressions (Section 3.2.1: expression templates, Eval, CSE,
 * constant folding; MultiEval: several results of one program).
 * A program is a postfix token list over up to 16 input scalars producing
 * up to 16 output scalars: INPUT pushes input `arg`, CONST pushes `value`,
 * a unary op replaces the top, a binary op pops b then a and pushes a op b,
 * OUTPUT pops the top into output `arg`.  The stack must be empty at the
 * end and every output written exactly once. */
#define APCG_EXPR_INPUT 1
#define APCG_EXPR_CONST 2
#define APCG_EXPR_NEG 10
#define APCG_EXPR_RECIP 11 /* 1 / a */
#define APCG_EXPR_SQRT 12
#define APCG_EXPR_ABS 13
#define APCG_EXPR_EXP 14
#define APCG_EXPR_LOG 15
#define APCG_EXPR_SIN 16
#define APCG_EXPR_COS 17
#define APCG_EXPR_ADD 20
#define APCG_EXPR_SUB 21
#define APCG_EXPR_MUL 22
#define APCG_EXPR_DIV 23
#define APCG_EXPR_MIN 24 /* IEEE minNum: a NaN operand yields the other */
#define APCG_EXPR_MAX 25
#define APCG_EXPR_OUTPUT 30
typedef struct apcg_expr_token {
    int32_t op;
    int32_t arg;  /* input or output index */
    double value; /* CONST */
} apcg_expr_token;
typedef struct apcg_expr_s *apcg_expr;

/* Eval: compiles a program (host only, no device work) into a register
 * program: identical subexpressions are computed once (within and across
 * outputs), subexpressions of constants are folded when the operation is
 * correctly rounded (everything but EXP/LOG/SIN/COS), and only rewrites
 * that are exact in IEEE double are applied (x*1, 1*x, x/1, x-0, x+(-0),
 * -(-x)).  At most 256 tokens and 128 instructions; malformed programs are
 * APCG_ERR_INVALID_ARG. */
apcg_status apcg_expr_compile(const apcg_expr_token *prog, int32_t ntokens, int32_t ninputs, int32_t noutputs,
                              apcg_expr *out);

/* Instructions of the compiled program, constants folded and repeated
 * subexpressions shared during compilation (any pointer may be NULL). */
apcg_status apcg_expr_stats(apcg_expr e, int32_t *instructions, int32_t *folded, int32_t *shared);

/* Execute: one single-workgroup kernel on ctx's stream reads the inputs
 * and writes every output (ordered like any library operation: inputs
 * read, outputs written; a scalar may be both).  The scalars must live on
 * ctx's device.  inputs/outputs: arrays of ninputs / noutputs handles. */
apcg_status apcg_expr_execute(apcg_expr e, apcg_ctx ctx, const apcg_scalar *inputs, const apcg_scalar *outputs);

apcg_status apcg_expr_destroy(apcg_expr e);

/* ---------------------------------------------------------------------- */
/* Vectors (borrowed device memory)                                        */
/* ---------------------------------------------------------------------- */

/* Wraps n doubles at dev_ptr (device memory on `device`, 8-byte aligned;
 * n >= 0; dev_ptr may be NULL only when n == 0).  The library never frees
 * dev_ptr.  Writes made to the memory outside the library must be finished
 * before the next library call that uses the vector. */
apcg_status apcg_vec_wrap(int32_t device, double *dev_ptr, int64_t n, apcg_vec *out);

/* Destroys the wrapper (not the memory) once its pending uses finish. */
apcg_status apcg_vec_destroy(apcg_vec v);

/* out = x . y (Section 3.3, VecDotAsync).  Deterministic: a fixed two-stage
 * reduction tree, bitwise reproducible for a given n. */
apcg_status apcg_vec_dot_async(apcg_vec x, apcg_vec y, apcg_scalar out, apcg_ctx ctx);

/* out = ||x||_2 (Section 3.3, VecNormAsync with NORM_2). */
apcg_status apcg_vec_norm2_async(apcg_vec x, apcg_scalar out, apcg_ctx ctx);

/* y = y + s a x with s = -1 if negate else +1 (Section 3.3, VecAXPYAsync
 * with a and -a).  x and y must have equal length and must not overlap
 * unless they are the same vector. */
apcg_status apcg_vec_axpy_async(apcg_vec y, apcg_scalar a, int32_t negate, apcg_vec x, apcg_ctx ctx);

/* y = x + b y (Section 3.3, VecAYPX: p <- z + b p). */
apcg_status apcg_vec_aypx_async(apcg_vec y, apcg_scalar b, apcg_vec x, apcg_ctx ctx);

/* x = a x (Section 3.3, VecScaleAsync; Section 3.1.2, the scale-kernel
 * example). */
apcg_status apcg_vec_scale_async(apcg_vec x, apcg_scalar a, apcg_ctx ctx);

/* dst = src (VecCopyAsync, named in the paper's API list). */
apcg_status apcg_vec_copy_async(apcg_vec dst, apcg_vec src, apcg_ctx ctx);

/* x = value for every entry. */
apcg_status apcg_vec_set_async(apcg_vec x, double value, apcg_ctx ctx);

/* Host accessor (Section 3.3, accessors synchronise implicitly): waits for
 * the last operation that wrote x, then copies its n entries to host_out. */
apcg_status apcg_vec_copy_to_host(apcg_vec x, double *host_out);

/* Enqueues a copy of n host doubles into x on ctx; returns after the host
 * buffer has been consumed. */
apcg_status apcg_vec_copy_from_host(apcg_vec x, const double *host_in, apcg_ctx ctx);

/* ---------------------------------------------------------------------- */
/* CSR matrices (borrowed device memory)                                   */
/* ---------------------------------------------------------------------- */

/* Wraps an n x n CSR matrix: dev_rowptr int32[n+1] (dev_rowptr[0] == 0,
 * non-decreasing, dev_rowptr[n] == nnz), dev_col int32[nnz] in [0, n),
 * dev_val double[nnz].  host_rowptr (may be NULL) is a host copy of the row
 * pointers used to validate and to plan the SpMV schedule; if NULL the
 * library copies it once (synchronously).  The arrays are never modified
 * or freed by the library. */
apcg_status apcg_mat_wrap_csr(int32_t device, int32_t n, int64_t nnz, const int32_t *dev_rowptr,
                              const int32_t *dev_col, const double *dev_val, const int32_t *host_rowptr,
                              apcg_mat *out);

/* Destroys the wrapper once its pending uses finish. */
apcg_status apcg_mat_destroy(apcg_mat A);

/* y = A x (Section 3.3, MatMult / KSP_MatMultAsync). */
apcg_status apcg_mat_mult_async(apcg_mat A, apcg_vec x, apcg_vec y, apcg_ctx ctx);

/* SpMV schedule.
 *   schedule APCG_SPMV_ROWGROUP: lanes_per_row in {1,2,4,8,16,32,64} lanes
 *       of a 64-wide wavefront cooperate on one row;
 *   schedule APCG_SPMV_STREAM: the workgroup stages the nonzeros of
 *       block_size consecutive rows in LDS with coalesced loads, then each
 *       thread reduces one row (lanes_per_row is ignored).  Needs every such
 *       row block to hold at most 5376 nonzeros (about 21 per row at block
 *       256, 10 at block 512); apcg_mat_set_spmv_config rejects it otherwise.
 *   schedule APCG_SPMV_SELL (PCG solves): one wavefront per slice of 64
 *       consecutive rows, the slice's entries stored column-major in a
 *       library-owned copy (sliced ELLPACK, padded to the slice's longest
 *       row), so every load of a column index or value is one coalesced
 *       512-byte access.  The copy (12 bytes per stored entry) is allocated
 *       on first use and refilled from the CSR arrays at the start of every
 *       solve, so values may change between solves.  A lone MatMult
 *       reads the CSR arrays with row groups (this configuration's block
 *       size and grid, lanes per row from the mean row length).
 *   schedule APCG_SPMV_SDIA (PCG solves): sliced diagonals.  The rows of
 *       a 64-row slice share one sorted list of column offsets
 *       (column - row); a 64-bit mask per offset marks the rows that hold
 *       the entry, and only the values are stored per entry (column-major by
 *       offset), so the matrix stream is 8 bytes per stored entry instead of
 *       12, and the gathers of a wavefront read contiguous windows of the
 *       vectors.  Every row adds its entries in column order with the same
 *       fused multiply-adds as the row-per-thread and sliced schedules, so
 *       A p is bitwise the same.  Applicable when every row's columns are
 *       strictly increasing, no slice has more than 32 distinct offsets, and
 *       the padded value copy is smaller than the sliced one's column and
 *       value arrays; apcg_mat_set_spmv_config returns APCG_ERR_UNSUPPORTED
 *       otherwise.  Selecting it copies the column indices to the host once
 *       (synchronously) and snapshots the pattern: the columns must not
 *       change afterwards (values may, they are refilled at the start of
 *       every solve).  A lone MatMult reads the CSR arrays, as for
 *       APCG_SPMV_SELL.  lanes_per_row > 1 (any value up to 64 for this
 *       schedule: planes per task) selects plane marching when the
 *       pattern has a plane stride (an offset 64 Ps, Ps < 65536 slices,
 *       present with both signs in at least half of the slices): each
 *       wavefront walks lanes_per_row slices one plane apart and carries the
 *       +-plane windows between them instead of gathering them (blocks is
 *       then ignored); without a plane stride it is the plain kernel.  When
 *       the pattern is structurally symmetric (found by the same analysis)
 *       and the values are symmetric bit for bit (checked on the device at
 *       every refill), the marching product reads each entry left of the
 *       diagonal as its transpose, so only the slots on and right of the
 *       diagonal stream from memory; the sums are unchanged.  Once a refill
 *       finds the values unsymmetric, the matrix reads every slot from then
 *       on (until its schedule is analysed again, i.e. never for this
 *       handle).
 *   schedule APCG_SPMV_DIA (PCG solves): diagonals.  Applicable when the
 *       whole matrix has at most 9 distinct column offsets (column - row;
 *       the 5-, 7- and 9-point stencil matrices) and every row's columns are
 *       strictly increasing; apcg_mat_set_spmv_config returns
 *       APCG_ERR_UNSUPPORTED otherwise.  Diagonal k is a library-owned array
 *       of n (rounded up to 64) values, 0 where a row has no entry at that
 *       offset, refilled from the CSR values at the start of every solve;
 *       selecting the schedule copies the pattern to the host once
 *       (synchronously) and snapshots it.  lanes_per_row must be 1; each
 *       thread computes whole rows, workgroups own contiguous ranges of
 *       rows (multiples of 64), and every load address is the row plus a
 *       constant offset: no per-row or per-slice index loads.  A row's sum
 *       adds the diagonals in offset order (= column order), the absent
 *       entries adding exact zeros, so A p is bitwise that of the
 *       row-per-thread schedule.  When the offset set is symmetric and the
 *       values are symmetric bit for bit (checked on the device at every
 *       refill, as for APCG_SPMV_SDIA), the value of an entry left of the
 *       diagonal, (i, i - q), is read as its transpose's, i.e. from
 *       diagonal +q at row i - q, so only the diagonals on and right of
 *       the main one stream from memory.  A lone MatMult reads the CSR
 *       arrays, as for APCG_SPMV_SELL.
 * block_size in {256, 512} threads; blocks is the number of workgroups
 * (rounded up to a multiple of the 8 XCDs; 0 = library default).  Each
 * workgroup owns a contiguous range of rows and workgroups are renumbered so
 * each XCD owns a contiguous slice of the matrix. */
#define APCG_SPMV_ROWGROUP 0
#define APCG_SPMV_STREAM 1
#define APCG_SPMV_SELL 2
#define APCG_SPMV_SDIA 3
#define APCG_SPMV_DIA 4
typedef struct apcg_spmv_config {
    int32_t lanes_per_row;
    int32_t block_size;
    int32_t blocks;
    int32_t schedule;
} apcg_spmv_config;

apcg_status apcg_mat_set_spmv_config(apcg_mat A, const apcg_spmv_config *cfg);
apcg_status apcg_mat_get_spmv_config(apcg_mat A, apcg_spmv_config *cfg);

/* What the sliced-diagonal analysis found for A (it runs when
 * APCG_SPMV_SDIA is selected or a solve first needs the layout; this call
 * does not run it).  out[0]: 1 the layout applies, -1 it does not, 0 not
 * analysed; out[1]: value slots per slice (U); out[2]: offset/mask slots per
 * slice (8, 16 or 32); out[3]: plane stride in slices for marching (0:
 * none); out[4]: 1 if the pattern is structurally symmetric; out[5]: 1 while
 * the values have been found symmetric bit for bit at every refill so far
 * (the marching product then reads the entries left of the diagonal as
 * their transposes).  Reading out[5] waits for the device to go idle
 * (hipDeviceSynchronize) and copies one word back: a diagnostic, not for
 * hot loops. */
apcg_status apcg_mat_get_sdia_info(apcg_mat A, int32_t out[6]);

/* What the diagonal analysis found for A (it runs when APCG_SPMV_DIA is
 * selected; this call does not run it).  out[0]: 1 the layout applies, -1
 * it does not, 0 not analysed; out[1]: distinct offsets; out[2]: 1 if the
 * offset set is symmetric; out[3]: 1 while the values have been found
 * symmetric bit for bit at every refill so far (the product then reads the
 * entries left of the diagonal as their transposes).  Reading out[3] waits
 * for the device to go idle and copies one word back: a diagnostic. */
apcg_status apcg_mat_get_dia_info(apcg_mat A, int32_t out[4]);

/* Autotuner: times every candidate schedule of one PCG iteration (the
 * fused product kernel and the update kernel with their reductions; reps
 * iterations each, HIP events on ctx's stream), keeps the fastest in A and
 * returns it in *best (and the mean iteration time in *best_us).  Runs on
 * scratch vectors (ctx's workspace and one vector the library allocates and
 * frees); A's arrays are only read.  Blocks the host until the sweep ends. */
apcg_status apcg_mat_autotune(apcg_mat A, apcg_ctx ctx, int32_t reps, apcg_spmv_config *best,
                              double *best_us);

/* Times the two kernels of one PCG iteration at A's current SpMV
 * configuration: reps launches of the fused product kernel back to back,
 * then reps launches of the update kernel, each run between a pair of HIP
 * events on ctx's stream, in the autotuner's timing mode (every load,
 * reduction and store of the solve; the scalar decisions are not taken).
 * *product_us and *update_us receive the mean time per launch.  Same
 * scratch use as apcg_mat_autotune; blocks the host until the runs end. */
apcg_status apcg_mat_time_kernels(apcg_mat A, apcg_ctx ctx, int32_t reps, double *product_us, double *update_us);

/* ---------------------------------------------------------------------- */
/* Krylov solve (Section 3.3, the PCG loop; Section 4.1, Jacobi CG)        */
/* ---------------------------------------------------------------------- */

#define APCG_PC_NONE 0   /* z = r                                           */
#define APCG_PC_JACOBI 1 /* z = D^{-1} r                                     */

#define APCG_NORM_UNPRECONDITIONED 0 /* stop when ||r_k|| <= rtol ||b||       */
#define APCG_NORM_PRECONDITIONED 1   /* stop when ||z_k|| <= rtol ||D^-1 b||  */

/* Host orchestration of the iteration loop. */
#define APCG_MODE_GRAPH 0      /* K iterations per captured hipGraph,        */
                               /* host polls a pinned flag L graphs behind   */
#define APCG_MODE_STREAM 1     /* same kernels launched one by one           */
#define APCG_MODE_HOST_CHECK 2 /* host reads the convergence flag after     */
                               /* every iteration (the synchronous shape)   */
#define APCG_MODE_PERSISTENT 3 /* one workgroup runs the whole solve in one  */
                               /* launch (n <= APCG_PERSISTENT_MAX_N; the    */
                               /* latency-bound regime of Section 4.2)       */
#define APCG_MODE_AUTO 4       /* PERSISTENT when n <= APCG_PERSISTENT_MAX_N */
                               /* (and no kernel timing), else GRAPH         */
#define APCG_PERSISTENT_MAX_N 4096

typedef struct apcg_solve_opts {
    int32_t pc;              /* APCG_PC_*                                    */
    int32_t norm_type;       /* APCG_NORM_*                                  */
    int32_t mode;            /* APCG_MODE_*                                  */
    int32_t iters_per_graph; /* K (even, >= 2) for GRAPH; poll period STREAM */
    int32_t lookahead;       /* graphs/periods in flight before a poll (>=1) */
    int32_t x0_is_zero;      /* 1: skip r0 = b - A x0 and zero x on device   */
    int32_t kernel_timing;   /* 1: STREAM mode with HIP events around every  */
                             /*    product and update kernel (see            */
                             /*    apcg_ctx_kernel_times)                    */
    int32_t batch_block_size;/* apcg_ksp_solve_batched: threads per system   */
                             /*    (256, 512 or 1024; 0 = 512)               */
    int32_t batch_schedule;  /* APCG_BATCH_*                                 */
    int32_t batch_tile_rows; /* segmented batched solves: rows per tile, a    */
                             /*    multiple of 256 in [256, 8192] (0 = 1024); */
                             /*    changes the launch shape only, not a sum  */
    int32_t batch_tail_tile_rows; /* segmented batched solves: rows per tile */
                             /*    once the rows of the systems still running */
                             /*    fill fewer than two tiles per compute unit */
                             /*    (the last, largest systems run alone): a  */
                             /*    valid tile size below batch_tile_rows, 0 = */
                             /*    256 (when below), -1 = keep the tiles.  The */
                             /*    same bits either way                      */
    int32_t reserved[5];
} apcg_solve_opts;

/* Schedules of apcg_ksp_solve_batched. */
#define APCG_BATCH_AUTO 0       /* persistent when the batch is balanced enough */
#define APCG_BATCH_PERSISTENT 1 /* one launch; one workgroup per system        */
#define APCG_BATCH_SEGMENTED 2  /* the batch as one block-diagonal system      */

/* Fills *opts with the defaults: Jacobi, unpreconditioned norm, GRAPH mode,
 * K = 16, lookahead 2, x0 read from x, no kernel timing. */
apcg_status apcg_solve_opts_default(apcg_solve_opts *opts);

/* Host view of one solve's results. */
typedef struct apcg_solve_info {
    int32_t iterations;     /* products A p performed (PETSc's count)       */
    int32_t status;         /* APCG_SOLVE_* bits                             */
    int32_t fcg_iterations; /* iterations run by the flexible method         */
    int32_t half_steps;     /* TFQMR: half-steps m of the last iteration; 0 otherwise */
    double res_norm;        /* final stopping norm                           */
    double ref_norm;        /* ||b|| (or ||D^-1 b|| for the preconditioned norm) */
} apcg_solve_info;

/* Device array of `count` solve-info records on ctx's device. */
apcg_status apcg_info_create(int32_t device, int32_t count, apcg_info *out);
apcg_status apcg_info_destroy(apcg_info info);

/* Waits for the last operation that wrote the info array, then copies
 * record `index` to *out. */
apcg_status apcg_info_get(apcg_info info, int32_t index, apcg_solve_info *out);

/* Solves A x = b with preconditioned CG on ctx.  x holds x0 on entry
 * (ignored when opts->x0_is_zero) and the solution on exit.  Stops when the
 * chosen norm is <= rtol times its reference, or after maxit iterations
 * (maxit >= 0).  The result is written to info[info_index] on the device.
 * Workspace (6 n doubles plus a few scalars) is owned by ctx and reused.
 * With APCG_MODE_GRAPH/STREAM no kernel waits on the host: the host thread
 * returns once it has enqueued enough work to reach convergence or maxit,
 * having observed the device flag only through events `lookahead` periods
 * behind the queue.  With APCG_MODE_PERSISTENT (or AUTO at n <=
 * APCG_PERSISTENT_MAX_N) the whole solve is one launch of one 512-thread
 * workgroup that keeps each row's r, D^-1, p and A p in registers and shares
 * p through n doubles of the context's workspace; its sums run in another
 * fixed order than the multi-kernel modes' (same tests, same counts up to
 * rounding).  n > APCG_PERSISTENT_MAX_N with PERSISTENT returns
 * APCG_ERR_INVALID_ARG.  On a globally blocking context the call returns
 * after the solve has finished. */
apcg_status apcg_ksp_solve(apcg_ctx ctx, apcg_mat A, apcg_vec b, apcg_vec x, double rtol, int32_t maxit,
                           const apcg_solve_opts *opts, apcg_info info, int32_t info_index);

/* Tuning table (the autotuner's results kept and reused; a8 of the hot
 * path's autotuner row, not a passage of the paper).  A key is
 *   "<arch>|u<U>.d<D>.p<P>.s<S>.m<M>|n<floor(log2 n)>|r<round(4 nnz/n)>"
 * with U the most distinct column offsets (column - row) of any 64-row slice
 * (capped at 33), D the distinct offsets of the matrix (0 when more than 9),
 * P = 1 when an offset 64 k is present with both signs in at least half of
 * the slices (plane marching applies), S = 1 for a structurally symmetric
 * pattern and M the longest row.  A value is four int32 (for a product
 * schedule: apcg_spmv_config's fields in order) and the measured
 * microseconds.  The table is process-wide host memory guarded by a mutex.
 *
 * apcg_tune_key_pattern: the key of host CSR arrays for device architecture
 *   `arch` (gcnArchName), written to out (cap bytes incl. the terminating
 *   0).  Host only.  APCG_ERR_INVALID_ARG on bad arrays or a short buffer.
 * apcg_mat_tune_key: the key of A on its device (reads A's pattern back
 *   once, synchronously, and keeps the class with A).
 * apcg_tune_cache_insert / _lookup / _clear / _size: the table itself
 *   (lookup sets *found to 0 or 1; *us may be NULL).
 * apcg_tune_cache_load: merges the entries of a text file written by
 *   apcg_tune_cache_save (one "key TAB i0 i1 i2 i3 TAB us" line per entry,
 *   '#' lines ignored); a malformed file changes nothing and returns
 *   APCG_ERR_INVALID_ARG naming the line.  *entries (may be NULL): lines read.
 * apcg_tune_cache_save: writes the whole table (sorted by key) to path,
 *   through a temporary file renamed into place.
 * apcg_mat_autotune_cached: apcg_mat_autotune unless A's key is in the
 *   table with a configuration A accepts (apcg_mat_set_spmv_config
 *   succeeds), in which case that configuration is set without timing and
 *   *from_cache = 1; a fresh result is inserted under A's key. */
apcg_status apcg_tune_key_pattern(const char *arch, int32_t n, int64_t nnz, const int32_t *rowptr,
                                  const int32_t *col, char *out, int32_t cap);
apcg_status apcg_mat_tune_key(apcg_mat A, char *out, int32_t cap);
apcg_status apcg_tune_cache_insert(const char *key, const int32_t values[4], double us);
apcg_status apcg_tune_cache_lookup(const char *key, int32_t values[4], double *us, int32_t *found);
apcg_status apcg_tune_cache_clear(void);
apcg_status apcg_tune_cache_size(int32_t *entries);
apcg_status apcg_tune_cache_load(const char *path, int32_t *entries);
apcg_status apcg_tune_cache_save(const char *path, int32_t *entries);
apcg_status apcg_mat_autotune_cached(apcg_mat A, apcg_ctx ctx, int32_t reps, apcg_spmv_config *best,
                                     double *best_us, int32_t *from_cache);

/* Launch configuration of a batched solve, as the batched autotuner picks it. */
typedef struct apcg_batch_config {
    int32_t schedule;   /* APCG_BATCH_PERSISTENT or APCG_BATCH_SEGMENTED      */
    int32_t block_size; /* persistent: threads per system (256, 512, 1024)    */
    int32_t tile_rows;  /* segmented: rows per tile (apcg_solve_opts field)   */
    int32_t sdia;       /* 1: members read their sliced-diagonal copies       */
} apcg_batch_config;

/* Autotuner of the batched solves (the hot path's autotuner row: tile and
 * schedule shapes picked by timing, not a passage of the paper).  kind 0
 * times apcg_ksp_solve_batched (persistent at 256/512/1024 threads per
 * system; segmented at 256-4096 rows per tile, on CSR and on the
 * sliced-diagonal copies), kind 1 apcg_ksp_solve_batched_fcg_poly with the
 * constant polynomial (its eight Clenshaw steps still run; segmented
 * configurations only): `iters` iterations with rtol 0 on ctx's stream, HIP
 * events, the better of two runs after a warm-up.  That window has every
 * system running; over a whole solve the last systems run alone, latency-
 * bound, where the sliced-diagonal reads are faster, so a configuration on
 * the CSR arrays is picked only when it beats the best sliced-diagonal one
 * by more than 10% in the window.  x is used as scratch (its
 * contents are overwritten).  The result goes to the tuning table under
 *   "batch|<arch>|pcg|fcg|m<longest row>|r<round(4 nnz/n)>|s<log2 systems>|
 *    n<log2 rows>|x<log2 largest system>"
 * and a later call with the same key applies it without timing
 * (*from_cache = 1).  With sdia = 1 the members whose pattern allows it are
 * left on APCG_SPMV_SDIA; with sdia = 0 the members' schedules are restored,
 * except that a member that was on APCG_SPMV_SDIA is put on
 * APCG_SPMV_ROWGROUP (one lane per row), so that the batch reads the CSR
 * arrays.  The
 * caller passes *best's fields to apcg_solve_opts (batch_schedule,
 * batch_block_size, batch_tile_rows).  Blocks the host. */
apcg_status apcg_batch_autotune(apcg_ctx ctx, int32_t nsys, const apcg_mat *A, const apcg_vec *b, const apcg_vec *x,
                                int32_t kind, int32_t iters, apcg_batch_config *best, double *best_ms,
                                int32_t *from_cache);

/* No-allocation variant of apcg_ksp_solve with APCG_MODE_PERSISTENT, for
 * callers that cannot allocate device memory: code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc.  The same
 * one-workgroup Jacobi-PCG kernel (the same sums, the same tests), with its
 * direction vector in a fixed array of APCG_NOALLOC_MAX_N doubles compiled
 * into the library (one per device, held until the process ends) instead of
 * the context's workspace.  Allocates nothing and takes no library objects:
 * raw device pointers to CSR arrays (rowptr int32[n+1], col int32[nnz], val
 * f64[nnz], strictly increasing or not), b and x (f64[n]; x holds x0 unless
 * opts->x0_is_zero) and one device record `info` that receives the result;
 * all of them stay owned by the caller, who orders their other uses against
 * ctx's stream (the call does no dependency marking).  opts: pc, norm_type
 * and x0_is_zero are read (NULL: the defaults), mode is ignored.  Queues one
 * kernel on ctx's stream and returns.  Every call on one device shares that
 * device's array, so two calls that overlap in time on one device (two
 * contexts, or two host threads) race: the caller serialises them, e.g. by
 * using one context.  Errors (returned before anything is queued):
 * APCG_ERR_INVALID_ARG for a NULL context or pointer, a globally blocking
 * context, n < 0, n > APCG_NOALLOC_MAX_N, maxit < 0 or rtol < 0 or NaN;
 * APCG_ERR_UNSUPPORTED for another preconditioner. */
#define APCG_NOALLOC_MAX_N 4096
apcg_status apcg_ksp_solve_small_noalloc(apcg_ctx ctx, int32_t n, const int32_t *rowptr, const int32_t *col,
                                         const double *val, const double *b, double *x, double rtol, int32_t maxit,
                                         const apcg_solve_opts *opts, apcg_solve_info *info);

/* Latency floors of the device (Section 4.2: below about 1e5 nonzeros the
 * GPU solve is bound by latency).  Runs on a private stream of `device`,
 * blocks the host, and writes microseconds to out_us:
 *   [0] per launch of an empty kernel, `reps` launches back to back;
 *   [1] per node of a captured graph of min(reps, 1000) empty kernels;
 *   [2] per iteration of the one-workgroup persistent solve's
 *       synchronisation alone (three barriers, two workgroup sums),
 *       `reps` iterations in one launch;
 *   [3] host round trip: one empty kernel launched and waited for
 *       (min(reps, 200) times, host clock).
 * reps in [1, 100000]; APCG_ERR_INVALID_ARG otherwise. */
apcg_status apcg_latency_floors(int32_t device, int32_t reps, double out_us[4]);

/* TFQMR (Section 4, the paper's second benchmark method; Freund 1993) for
 * square, possibly nonsymmetric or indefinite A, left-preconditioned by
 * B = D^{-1} (opts->pc == APCG_PC_JACOBI: every a_ii present, finite and
 * nonzero, else APCG_SOLVE_SETUP_ERROR) or B = I (APCG_PC_NONE); two
 * products with A per iteration.  The arguments, modes, x0 handling, the
 * graph period K and the lookahead are those of apcg_ksp_solve;
 * opts->norm_type is ignored.  Test: after every half-step m the quasi-
 * residual bound tau_m sqrt(m + 1) (which bounds ||B (b - A x_m)||) is
 * compared with rtol ||B (b - A x0)||.  The record holds iterations (two
 * products each), half_steps (the last m), res_norm (the last bound) and
 * ref_norm (||B (b - A x0)||).  Breakdowns: r0.v = 0 (the denominator of
 * alpha) -> APCG_SOLVE_BREAKDOWN_PAP, r0.w = 0 (that of beta) ->
 * APCG_SOLVE_BREAKDOWN_RZ.  Workspace: 9 n doubles per context, kept
 * between solves.  The products read the matrix's sliced-diagonal copy when
 * its pattern allows one (see APCG_SPMV_SDIA; the first such solve of a
 * matrix copies the pattern to the host once, synchronously), else the CSR
 * arrays; both add every row's entries in column order, bitwise alike. */
apcg_status apcg_ksp_solve_tfqmr(apcg_ctx ctx, apcg_mat A, apcg_vec b, apcg_vec x, double rtol, int32_t maxit,
                                 const apcg_solve_opts *opts, apcg_info info, int32_t info_index);

/* Solves the nsys independent systems A[i] x[i] = b[i] with Jacobi-PCG (or
 * CG): same stopping rule, tests and order as apcg_ksp_solve (Section 3.3
 * loop, Section 4.1 Jacobi), every system with its own scalars and status.
 *   APCG_BATCH_PERSISTENT: ONE launch; each workgroup takes the next system
 *     from a device work queue ordered by decreasing estimated cost
 *     (nnz * sqrt(n)) and runs that system's whole iteration with
 *     workgroup-level reductions (opts->batch_block_size threads).  Best for
 *     many similar small systems.
 *   APCG_BATCH_SEGMENTED: the batch as one block-diagonal system cut into
 *     256-row tiles; per iteration a tile product, a per-system alpha, a
 *     tile update and a per-system test, K iterations per captured graph;
 *     stopped systems' tiles return at once.  Best when a few large systems
 *     dominate.  A system whose matrix is on APCG_SPMV_SDIA with 8
 *     offset slots per slice has its tile product read the sliced-diagonal
 *     copy (same row sums, bit for bit); every other system reads CSR.
 *     The tile product walks 5, 7 or 8 offset slots per row, the fewest
 *     that cover every such system of the batch.
 *   APCG_BATCH_AUTO: persistent when no system costs more than 1/CUs of the
 *     batch, else segmented.
 * A, b, x: arrays of nsys handles on ctx's device; the memory of each x[i]
 * may overlap no other x[j] and no b[j] (checked on the host over the
 * vectors' address ranges: APCG_ERR_INVALID_ARG); x[i] holds x0 (ignored with x0_is_zero) and receives
 * the solution; info must hold >= nsys records, record i for system i.
 * opts->mode APCG_MODE_GRAPH (default) replays captured graphs (cached while
 * the batch is unchanged).  The context keeps 6 sum(n_i) doubles of
 * workspace and the batch descriptors.  Returns once the work is enqueued
 * (after a one-time upload of the descriptors when the batch changed; the
 * segmented schedule polls the device's count of running systems one graph
 * behind, as apcg_ksp_solve does). */
apcg_status apcg_ksp_solve_batched(apcg_ctx ctx, int32_t nsys, const apcg_mat *A, const apcg_vec *b,
                                   const apcg_vec *x, double rtol, int32_t maxit, const apcg_solve_opts *opts,
                                   apcg_info info);

/* ---------------------------------------------------------------------- */
/* Learned polynomial preconditioner                                       */
/*                                                                         */
/* Preconditioner z = p(D^-1 A) D^-1 r with                                */
/*   p(t) = sum_{j=0..8} c_j T_j(2 t / lmax - 1),                          */
/* lmax = the Gershgorin upper bound of D^-1 A, inside flexible CG         */
/* (FCG(1)) -- the PCG loop of Section 3.3 with a variable preconditioner.  */
/* A 16 -> 64 -> 64 -> 9 tanh MLP (FP32) maps cheap matrix features to the */
/* nine coefficients.  Parameters are one float array of 5833 entries:     */
/* W1[64][16], b1[64], W2[64][64], b2[64], W3[9][64], b3[9] (row-major).   */
/* These calls take raw device pointers and are ordered on ctx only.       */
/* ---------------------------------------------------------------------- */

/* Features of one system (n >= 1, Jacobi diagonal > 0):
 * dev_feat[16] (float): log10 n, nnz/n, Gershgorin lower and upper bounds of
 *   D^-1 A, log10(max diag / min diag), std of ln diag, mean over rows of
 *   ln(max |offdiag| / min |offdiag|), the three smallest and three largest
 *   Ritz values / upper bound (with fewer than three, indices clamp to the
 *   ones that exist), log10(largest / smallest Ritz value), log10 of the
 *   relative residual after the steps (floored at 1e-30), log10(smallest
 *   Ritz / upper);
 * dev_lmax[1] (double): the Gershgorin upper bound.
 * Runs 12 Jacobi-PCG iterations from x0 = 0 on ctx's workspace (the
 * CG-Lanczos relation turns their alpha, beta into the Ritz values) plus two
 * passes over the rows. */
apcg_status apcg_pc_features(apcg_ctx ctx, apcg_mat A, apcg_vec b, float *dev_feat, double *dev_lmax);

/* Training label of one system, from its own Jacobi-PCG solve (x0 = 0, rtol,
 * maxit >= 1; the tridiagonal of all its iterations):
 * dev_label[3] (double): lmin = the smallest Ritz value of the solve (0 when
 *   it takes no iteration), a = 3 lmin clamped to [1e-3 lmax, lmax / 2]
 *   (lmax / 2 without iterations), lmax;
 * dev_G[81], dev_h[9] (float): the loss's quadratic form c'G c - 2 h'c + 1 =
 *   sum_q w_q t_q^2 (p(t_q) - p*(t_q))^2 / sum_q w_q t_q^2 p*(t_q)^2 over the
 *   16-point Gauss-Chebyshev rule (t_q, w_q = 1/16) on [a, lmax], where p*
 *   is the Chebyshev semi-iterative polynomial on [a, lmax] (its residual
 *   polynomial 1 - t p*(t) is the minimax one there). */
apcg_status apcg_pc_label(apcg_ctx ctx, apcg_mat A, apcg_vec b, double rtol, int32_t maxit, float *dev_G,
                          float *dev_h, double *dev_label);

/* Standardises the rows of dev_X[B][16] in place with the column means and
 * standard deviations dev_mean[16], dev_std[16]; compute_stats != 0 first
 * computes them from X (two passes; a zero deviation is replaced by 1). */
apcg_status apcg_mlp_standardize(apcg_ctx ctx, float *dev_X, int32_t B, float *dev_mean, float *dev_std,
                                 int32_t compute_stats);

/* dev_C[B][9] = MLP(dev_X[B][16]). */
apcg_status apcg_mlp_forward(apcg_ctx ctx, const float *dev_params, const float *dev_X, int32_t B, float *dev_C);

/* Mean loss over B systems (dev_loss[1]) and its gradient with respect to
 * the 5833 parameters (dev_grad), given each system's dev_G[B][81] and
 * dev_h[B][9] (from apcg_pc_label); penalty weight mu and floor eps of the positivity term
 * mu / 64 sum_q max(0, eps - p(t_q))^2 over 64 points of [0, lmax]. */
apcg_status apcg_mlp_loss_grad(apcg_ctx ctx, const float *dev_params, const float *dev_X, const float *dev_G,
                               const float *dev_h, int32_t B, float mu, float eps, float *dev_loss, float *dev_grad);

/* One Adam step (Kingma & Ba; beta1 0.9, beta2 0.999, eps 1e-8) on the
 * parameters with the loss gradient above; t >= 1 is the step number;
 * dev_adam_m, dev_adam_v (5833 each) hold the moment estimates. */
apcg_status apcg_mlp_train_step(apcg_ctx ctx, float *dev_params, float *dev_adam_m, float *dev_adam_v, int32_t t,
                                float lr, const float *dev_X, const float *dev_G, const float *dev_h, int32_t B,
                                float mu, float eps, float *dev_loss);

typedef struct apcg_fcg_opts {
    int32_t stall_min;  /* stall window floor (iterations)                    */
    int32_t fallback;   /* 1: continue with Jacobi-PCG after a breakdown,     */
                        /*    a stall or a non-positive polynomial            */
    double stall_frac;  /* window = max(stall_min, stall_frac * k)            */
    int32_t reserved[4];
} apcg_fcg_opts;

/* stall_min 50, stall_frac 0.1, fallback 1. */
apcg_status apcg_fcg_opts_default(apcg_fcg_opts *opts);

/* Solves A x = b with FCG(1) and the polynomial preconditioner above
 * (coefficients dev_coeffs[9], float, and dev_lmax, double, in device
 * memory, e.g. from apcg_mlp_forward and apcg_pc_features).  p is first
 * checked on 1024 points of [0, lmax]; if it is not positive there, or if
 * the iteration breaks down (p.Ap <= 0, r.z <= 0) or stalls (no new minimum
 * of ||r|| within the window), Jacobi-PCG continues from the current x for
 * the remaining iterations when fopts->fallback is set (status then carries
 * APCG_SOLVE_FALLBACK and the reason; iterations count both phases;
 * fcg_iterations the flexible ones).  Stopping: ||r|| <= rtol ||b||.
 * opts: mode (graph/stream), iters_per_graph, lookahead and x0_is_zero as
 * for apcg_ksp_solve.  The host waits once, at the end of the flexible
 * phase, to decide on the fallback. */
apcg_status apcg_ksp_solve_fcg_poly(apcg_ctx ctx, apcg_mat A, apcg_vec b, apcg_vec x, double rtol, int32_t maxit,
                                    const float *dev_coeffs, const double *dev_lmax, const apcg_solve_opts *opts,
                                    const apcg_fcg_opts *fopts, apcg_info info, int32_t info_index);

/* Solves the nsys independent systems A[i] x[i] = b[i], each with FCG(1) and
 * its own polynomial (dev_coeffs[nsys][9], float; dev_lmax[nsys], double),
 * the batch run as one block-diagonal iteration (tiles of 256 rows; K
 * iterations per captured graph; the host polls a device count of running
 * systems).  Every system follows apcg_ksp_solve_fcg_poly: the positivity
 * check, the breakdown and stall tests, and -- with fopts->fallback -- the
 * switch to Jacobi-PCG from its current x, taken on the device for that
 * system alone (its status then carries APCG_SOLVE_FALLBACK and the reason).
 * info[i] receives system i's record.  opts: mode (graph/stream),
 * iters_per_graph, lookahead, x0_is_zero.  The memory of each x[i] may
 * overlap no other x[j] and no b[j] (checked on the host:
 * APCG_ERR_INVALID_ARG).  A system whose matrix is on APCG_SPMV_SDIA with 8 offset slots per slice
 * has its products and Clenshaw steps read the sliced-diagonal copy (same
 * row sums, bit for bit; refilled at the start of every call). */
apcg_status apcg_ksp_solve_batched_fcg_poly(apcg_ctx ctx, int32_t nsys, const apcg_mat *A, const apcg_vec *b,
                                            const apcg_vec *x, double rtol, int32_t maxit, const float *dev_coeffs,
                                            const double *dev_lmax, const apcg_solve_opts *opts,
                                            const apcg_fcg_opts *fopts, apcg_info info);

/* Features of nsys systems at once (dev_feat[nsys][16], dev_lmax[nsys];
 * the same values as apcg_pc_features per system): one batched 12-step
 * Jacobi-PCG run from x0 = 0 on library scratch (the block-diagonal
 * iteration of apcg_ksp_solve_batched_fcg_poly with every system in Jacobi
 * mode), two passes of row statistics over all tiles and the Ritz values of
 * each system.  A system with b = 0 takes lmax as its only Ritz value. */
apcg_status apcg_pc_features_batched(apcg_ctx ctx, int32_t nsys, const apcg_mat *A, const apcg_vec *b,
                                     float *dev_feat, double *dev_lmax);

/* The learned batched solve: apcg_pc_features_batched, the network
 * (standardised with dev_mean / dev_std) for all systems at once, then
 * apcg_ksp_solve_batched_fcg_poly with the network's coefficients -- each
 * system with its own polynomial and its own fallback to Jacobi-PCG. */
apcg_status apcg_ksp_solve_batched_learned(apcg_ctx ctx, int32_t nsys, const apcg_mat *A, const apcg_vec *b,
                                           const apcg_vec *x, double rtol, int32_t maxit, const float *dev_params,
                                           const float *dev_mean, const float *dev_std, const apcg_solve_opts *opts,
                                           const apcg_fcg_opts *fopts, apcg_info info);

/* The learned solve in one call: features of (A, b), standardised with
 * dev_mean[16] / dev_std[16], the network dev_params[5833] -> coefficients,
 * then apcg_ksp_solve_fcg_poly with them (same options, result record and
 * fallback).  With opts->x0_is_zero the flexible solve starts
 * from the iterate of the feature run's 12 Jacobi-PCG steps from x0 = 0
 * (copied into x) rather than from 0, so those steps are not thrown away;
 * the record counts the flexible solve's iterations only.  Network arrays
 * are device pointers ordered on ctx only. */
apcg_status apcg_ksp_solve_learned(apcg_ctx ctx, apcg_mat A, apcg_vec b, apcg_vec x, double rtol, int32_t maxit,
                                   const float *dev_params, const float *dev_mean, const float *dev_std,
                                   const apcg_solve_opts *opts, const apcg_fcg_opts *fopts, apcg_info info,
                                   int32_t info_index);

/* Mean device time (microseconds) and launch count of the product kernel
 * (kind 0: fused SpMV + p.Ap) and the update kernel (kind 1: x, r update
 * with r.z and ||r||^2) measured by the last solve on ctx that ran with
 * kernel_timing = 1.  Blocks until that solve has finished. */
apcg_status apcg_ctx_kernel_times(apcg_ctx ctx, int32_t kind, double *mean_us, int32_t *count);

/* ---------------------------------------------------------------------- */
/* Timers and diagnostics                                                  */
/* ---------------------------------------------------------------------- */

apcg_status apcg_timer_create(apcg_timer *out);
apcg_status apcg_timer_destroy(apcg_timer t);
/* Records the start / stop timestamp on ctx's stream (no host wait). */
apcg_status apcg_timer_start(apcg_timer t, apcg_ctx ctx);
apcg_status apcg_timer_stop(apcg_timer t, apcg_ctx ctx);
/* Waits for the stop timestamp and returns stop - start in milliseconds. */
apcg_status apcg_timer_elapsed_ms(apcg_timer t, double *ms);

/* Library-wide counters of host-visible events. */
typedef struct apcg_counters {
    int64_t kernel_launches; /* kernels enqueued outside graphs              */
    int64_t graph_launches;  /* hipGraphLaunch calls                         */
    int64_t host_syncs;      /* host waits on streams/devices                */
    int64_t host_polls;      /* host waits on events queued >= 1 period back */
    int64_t d2h_copies;      /* device-to-host copies                        */
    int64_t h2d_copies;      /* host-to-device copies                        */
    int64_t stream_waits;    /* cross-context waits inserted by the registry */
    int64_t reserved[9];
} apcg_counters;

apcg_status apcg_counters_get(apcg_counters *out);
apcg_status apcg_counters_reset(void);

/* Device description for reports. */
typedef struct apcg_device_props {
    char name[64];
    char arch[32];           /* e.g. "gfx950"                                */
    int32_t compute_units;
    int32_t wavefront_size;
    int64_t global_mem_bytes;
    int32_t clock_khz;
    int32_t l2_bytes;
    int32_t lds_bytes_per_block;
    int32_t reserved[7];
} apcg_device_props;

apcg_status apcg_device_props_get(int32_t device, apcg_device_props *out);

/* Number of HIP devices visible (0 on a machine without GPU). */
apcg_status apcg_device_count(int32_t *count);

/* Message of the last failing call on this thread ("" if none). */
const char *apcg_last_error(void);

/* APCG_ABI_VERSION of the built library. */
int32_t apcg_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* APCG_H */
