/*
 * dagchol: task-DAG tiled Cholesky factorisation and solve on one MI355X.
 *
 * The programming model is the one of the paper's Section 2: data buffers are
 * registered as handles, tasks are submitted asynchronously with an access
 * mode (read-only, write-only, read-write) for every buffer argument, and the
 * dependency graph of the tasks follows from those modes plus the order of
 * submission; a wait call blocks until every submitted task has completed.
 * Section 3.2 gives the mode rule for parameters (unqualified pointer:
 * read-write, const pointer: read-only, output attribute: write-only, scalars
 * by value); Section 3.4 the register/unregister/acquire operations; Section
 * 5.1 the partitioning of a registered matrix into sub-matrix handles, the
 * idiom of tiled Cholesky; Section 5.3 task priorities as scheduling hints.
 *
 * The tasks run on the GPU.  The executor (DC_EXEC_LEVELS) splits each
 * flushed graph into levels on the host (every task's predecessors in
 * earlier levels) and runs each level as one launch of the panel kernel
 * (POTRF, the triangular solves, elementwise tasks) next to the GEMM/SYRK
 * kernels, on two streams; within a launch, workgroups take work items from
 * an atomic counter, urgent priority lanes first (Section 5.3's hints).
 * A device-side ready-queue executor (DC_EXEC_QUEUE: persistent kernels
 * whose workgroups pop ready items and decrement their successors'
 * dependency counters) is built but disabled: dc_init rejects it with
 * -ENOSYS (its first run on the GPU did not complete).
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Return value: 0 on success, a negative errno on failure, in which case
 *    the call had no effect:
 *      -EINVAL     bad argument: arity or access mode not matching the task
 *                  kind's signature, dtype or shape mismatch, null pointer;
 *      -ENOENT     unknown or unregistered handle or pointer (the paper's
 *                  generated task body rejects unregistered pointers);
 *      -EBUSY      a partitioned matrix used as a whole, or a handle still
 *                  referenced by pending tasks;
 *      -ENOMEM     host or device memory exhausted, or a capacity exceeded;
 *      -ENODEV     execution requested from a host-only runtime;
 *      -ENOSYS     a disabled feature was requested;
 *      -EIO        a HIP runtime call failed.
 *    The library never aborts the process (unlike the paper's generated
 *    code, which calls abort on these errors).
 *  - Numerical breakdown is not an error code: a factorisation of a matrix
 *    that is not numerically positive definite completes, and dc_get_info
 *    reports the 1-based global column of the first non-positive pivot
 *    (LAPACK convention); tasks that depend on the failed diagonal factor
 *    are skipped and the matrix contents are then unspecified.
 *  - Ownership: device buffers belong to the caller.  The library borrows
 *    them from register to unregister; they must stay allocated until the
 *    handle is unregistered (Section 3.4 warns that storage reclaimed before
 *    tasks complete is an error).  Handles, task descriptors and executor
 *    state belong to the runtime.  Scalar task arguments are copied at
 *    submission.
 *  - Layout: matrices are row-major with a leading dimension `ld` (elements
 *    between consecutive rows); only the lower triangle (row >= column) of a
 *    symmetric matrix is read or written.
 *  - Ordering: results equal those of executing the tasks one after another
 *    in submission order (the paper's "valid sequential program").
 *  - Threading: a runtime is not thread-safe; use one runtime per host
 *    thread.  All work is issued on the runtime's HIP stream.
 */
#ifndef DAGCHOL_H
#define DAGCHOL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dc_runtime dc_runtime;

/* Opaque handle; 0 is the null handle (like a failed data lookup). */
typedef int64_t dc_handle;

/* Access modes; read-write is the union of read and write. */
typedef enum { DC_R = 1, DC_W = 2, DC_RW = 3 } dc_mode;

typedef enum { DC_F64 = 0, DC_F32 = 1, DC_BF16 = 2 } dc_dtype;

/*
 * Task kinds and their buffer signatures (handles in this order):
 *   DC_POTRF      (D:RW)            D = L L^T in place, lower, one diagonal
 *                                   tile (FP64, or FP32 computed in FP64 and
 *                                   rounded on store); scalar: int64 global
 *                                   row offset of D (for the info column),
 *                                   optional.  The executor may run an FP64
 *                                   tile of order 257..512 as the blocked
 *                                   factorisation of its 2 x 2 sub-blocks
 *                                   (POTRF, TRSM, SYRK, POTRF on order <= 256;
 *                                   same result up to rounding), where the
 *                                   task's latency would otherwise set its
 *                                   level's length; the graph the caller
 *                                   submitted, its trace and its info column
 *                                   are unchanged.
 *   DC_TRSM       (L:R, X:RW)       X <- X L^{-T}, L lower non-unit.
 *   DC_SYRK       (X:R, C:RW)       lower(C) <- lower(C) - X X^T.
 *   DC_GEMM       (X:R, Y:R, C:RW)  C <- C - X Y^T.
 *   DC_TRSM_L     (L:R, B:RW)       B <- L^{-1} B (forward substitution).
 *   DC_TRSM_LT    (L:R, B:RW)       B <- L^{-T} B (backward substitution).
 *   DC_GEMM_RHS_N (L:R, Y:R, B:RW)  B <- B - L Y.
 *   DC_GEMM_RHS_T (L:R, Y:R, B:RW)  B <- B - L^T Y.
 *   DC_SCAL       (X:RW)            x <- factor * x, float vector; scalar:
 *                                   one float (the paper's scale_vector).
 *   DC_CAST       (S:R, D:W)        D <- S converted to D's dtype (round to
 *                                   nearest even), same shape.
 *   DC_RESID      (A:R, X:R, B:R, R:W)  R <- B - A X, A symmetric given by
 *                                   its lower triangle, FP64; each row is a
 *                                   compensated dot product (error-free
 *                                   products and sums), rounded once.
 *   DC_AXPY       (D:R, X:RW)       X <- X + D, FP64 matrices of one shape.
 *   DC_TRSM_CAST  (L:R, X:RW, S:W)  TRSM on an FP32 tile X that also writes
 *                                   S = BF16(X) (round to nearest even).
 *   DC_TRTRI      (L:R, W:W)        lower(W) <- L^{-1}, L lower non-unit,
 *                                   FP64, order 16..512.  The strictly upper
 *                                   part of W is scratch: it receives
 *                                   max |L| and per-column-block max |W|.
 *   DC_TRSM_INV   (L:R, W:R, X:RW)  X <- X L^{-T} computed as X W^T with W
 *                                   from DC_TRTRI of the same L (a dense
 *                                   MFMA product instead of a substitution).
 *                                   When max |L| * max |W| > 1024 (an
 *                                   ill-conditioned L, where the explicit
 *                                   inverse would lose accuracy) it solves
 *                                   with L by substitution like DC_TRSM.
 *                                   X FP64 or FP32.
 *   DC_TRSM_INV_CAST (L:R, W:R, X:RW, S:W)  TRSM_INV on an FP32 tile X that
 *                                   also writes S = BF16(X).
 *   DC_TRSM_L_INV  (L:R, W:R, S:R, D:W)  D <- L^{-1} S computed as W S, and
 *   DC_TRSM_LT_INV (L:R, W:R, S:R, D:W)  D <- L^{-T} S computed as W^T S,
 *                                   out of place (S and D distinct nb x r),
 *                                   with W from DC_TRTRI of the same L (FP64
 *                                   L, W, S and D, order 16..512); both fall
 *                                   back to substitution like DC_TRSM_INV.
 * Precisions (the dtypes of the handles select the kernel):
 *   POTRF: FP64 or FP32 storage, FP64 arithmetic.  TRSM: L FP64, X FP64 or FP32 (FP64 arithmetic, FP32 tiles
 *   rounded on store).  SYRK/GEMM: FP64 inputs update FP64 tiles with FP64
 *   MFMA; FP32 or BF16 inputs (both operands of one dtype) multiply with
 *   FP32 accumulation and the product is subtracted from an FP32 or FP64
 *   tile.  Solve tasks: B FP64, L FP64 or FP32, FP64 arithmetic.
 */
typedef enum {
  DC_POTRF = 0, DC_TRSM = 1, DC_SYRK = 2, DC_GEMM = 3,
  DC_TRSM_L = 4, DC_GEMM_RHS_N = 5, DC_TRSM_LT = 6, DC_GEMM_RHS_T = 7,
  DC_SCAL = 8, DC_CAST = 9, DC_RESID = 10, DC_AXPY = 11, DC_TRSM_CAST = 12,
  DC_TRTRI = 13, DC_TRSM_INV = 14, DC_TRSM_INV_CAST = 15,
  DC_TRSM_L_INV = 16, DC_TRSM_LT_INV = 17,
  DC_NUM_KINDS = 18
} dc_kind;

/* Executors (dc_config.executor). */
typedef enum { DC_EXEC_LEVELS = 0, DC_EXEC_QUEUE = 1 } dc_executor;

typedef struct {
  int device;            /* HIP device ordinal; -1: host-only runtime that
                            builds and inspects graphs but cannot execute */
  void *stream;          /* hipStream_t to issue work on; NULL: a stream the
                            runtime creates */
  int workers;           /* CUs the executor's kernels may use together;
                            0: every CU of the device */
  int64_t watchdog_ms;   /* reserved for DC_EXEC_QUEUE (a worker that waits
                            this long while no task completes would stop the
                            graph with -ETIMEDOUT); the level executor never
                            waits on the device; 0: 60000 */
  int trace;             /* nonzero: record a per-task trace at every wait */
  int executor;          /* dc_executor; 0 (DC_EXEC_LEVELS) by default;
                            DC_EXEC_QUEUE is rejected (-ENOSYS) */
  int lookahead;         /* lookahead depth of the level executor: a task
                            off the critical chains (the ones whose earliest
                            and latest levels, the downward and upward ranks
                            of Section 5.3's scheduling hints, differ) may be
                            placed at most this many levels after its
                            earliest one; 0 places every task at its earliest
                            level; dc_config_default sets 48; negative:
                            -EINVAL */
} dc_config;

/* Fills cfg with defaults (device 0, own stream, every CU, level executor,
 * 60 s watchdog, lookahead 48 levels). */
void dc_config_default(dc_config *cfg);

/* Creates a runtime.  Errors: -EINVAL (null pointer, unknown executor),
 * -ENOSYS (DC_EXEC_QUEUE on a device runtime), -EIO (HIP failure, e.g. no
 * such device), -ENOMEM. */
int dc_init(dc_runtime **rt, const dc_config *cfg);

/* Waits for pending work, frees runtime state (never user buffers). */
int dc_shutdown(dc_runtime *rt);

/* Registers a vector of nx elements at device address ptr (Section 2's
 * vector registration).  Errors: -EINVAL, -EBUSY (ptr already registered). */
int dc_vector_register(dc_runtime *rt, dc_handle *out, void *ptr, int64_t nx,
                       dc_dtype dtype);

/* Largest accepted leading dimension, in elements.  The GEMM kernels address
 * the rows of one 128-row unit through a 32-bit byte offset, which this bound
 * keeps below 2 GiB (a square FP64 matrix of this order would need 32 TiB). */
#define DC_MAX_LD ((int64_t)1 << 21)

/* Registers a rows x cols row-major matrix with leading dimension
 * cols <= ld <= DC_MAX_LD (Section 5.1's matrix).  Errors: -EINVAL, -EBUSY. */
int dc_matrix_register(dc_runtime *rt, dc_handle *out, void *ptr, int64_t rows,
                       int64_t cols, int64_t ld, dc_dtype dtype);

/* Partitions a registered matrix into ceil(rows/tile) x ceil(cols/tile)
 * sub-matrix handles (Section 5.1's filters): tile (I, J) starts at element
 * (I*tile, J*tile), keeps the parent's ld, and the last row/column of tiles
 * is ragged when tile does not divide the size.  tiles_out receives the
 * handles row-major (I * tcols + J) and must hold trows*tcols entries.
 * While partitioned, the parent cannot be used in tasks (-EBUSY).
 * Errors: -ENOENT, -EINVAL, -EBUSY (already partitioned or has pending
 * tasks). */
int dc_matrix_partition(dc_runtime *rt, dc_handle m, int64_t tile,
                        dc_handle *tiles_out);

/* Gathers the tiles back: flushes pending tasks if any touch them (the
 * graph's dependencies are fixed at that point), then drops the tile
 * handles; a flushed graph keeps running (its tasks hold the addresses, and
 * later graphs run after it in stream order).
 * Errors: -ENOENT, -EINVAL (not partitioned). */
int dc_matrix_unpartition(dc_runtime *rt, dc_handle m);

/* Number of tile rows and columns of a partitioned matrix. */
int dc_matrix_tiles(dc_runtime *rt, dc_handle m, int64_t *trows, int64_t *tcols);

/* Finds the top-level handle registered at ptr; *out = 0 and -ENOENT when
 * there is none (the lookup of the paper's generated task body). */
int dc_handle_lookup(dc_runtime *rt, const void *ptr, dc_handle *out);

/* Submits one task.  bufs/modes: nbuf handles with their access modes, in
 * the order of the kind's signature above; the modes must equal the
 * signature's (a W where RW is declared is accepted: W is RW without the
 * read).  cl_args: packed scalars, copied (at most 64 bytes).  priority: 0
 * is the most urgent; larger values run later when both are ready
 * (Section 5.3's hint); values above 3 are clamped.
 * Dependencies: a task that reads a handle waits for its last writer; a
 * task that writes a handle waits for the last writer and every reader since
 * (Section 2).  Sub-matrix handles of one partition are independent data.
 * Errors: -EINVAL, -ENOENT, -EBUSY, -ENOMEM. */
int dc_task_submit(dc_runtime *rt, dc_kind kind, int nbuf, const dc_handle *bufs,
                   const dc_mode *modes, const void *cl_args, size_t cl_args_size,
                   int priority);

/* Starts executing every submitted task (the executor's launches, ordered on
 * the runtime's stream) without waiting for them.  It first waits for the
 * previously flushed graph, if any.  Submissions after a flush form a new
 * graph that runs after the flushed one. */
int dc_flush(dc_runtime *rt);

/* Blocks until every submitted task has completed (Sections 2 and 3.3).
 * Errors: -EIO, -ENODEV (host-only runtime with pending tasks; the tasks are
 * discarded). */
int dc_wait_all(dc_runtime *rt);

/* Makes a handle's data valid for the host to access (Section 3.4's
 * acquire): if tasks that touch the handle (or one of its tiles) are
 * pending or in the flushed graph that may still run, it waits for every
 * submitted task (dc_wait_all); otherwise it returns at once.  dc_release
 * ends the access. */
int dc_acquire(dc_runtime *rt, dc_handle h, dc_mode mode);
int dc_release(dc_runtime *rt, dc_handle h);

/* Waits for the tasks that touch h (as dc_acquire), then forgets it (and
 * its tiles). */
int dc_unregister(dc_runtime *rt, dc_handle h);

/* Numerical status of a matrix handle after its tasks completed: 0, or the
 * 1-based global column of the first non-positive pivot. */
int dc_get_info(dc_runtime *rt, dc_handle m, int64_t *info);

/* Launch-path self test: fills the n int64 values at device address ptr
 * with 2 i + 1 on `stream` (a hipStream_t, NULL for the default stream)
 * and waits.  Errors: -EINVAL, -EIO. */
int dc_selftest(void *ptr, int64_t n, void *stream);

/* Text for a return code. */
const char *dc_strerror(int err);

/* Detail of the last -EIO on the calling thread (the failing HIP call and
 * its error name), or an empty string. */
const char *dc_last_error(void);

/* ---------------------------------------------------------------- graphs */

/* Inspection of the graph submitted since the last flush/wait (also on a
 * host-only runtime): number of tasks, of dependency edges, of edges present
 * only because of a write-after-read, and the task count of the longest
 * dependency chain. */
typedef struct {
  int64_t ntasks, nedges, nwar_edges, critical_path, nunits;
} dc_graph_stats;
int dc_graph_stats_get(dc_runtime *rt, dc_graph_stats *out);

/* Predecessors of pending task t (0-based submission index): writes up to
 * cap task indices, *count receives the total. */
int dc_graph_preds(dc_runtime *rt, int64_t t, int64_t *preds, int64_t cap,
                   int64_t *count);

/* Per-task trace of the last executed graph (config.trace != 0): for task t,
 * start and end times (ns, device clock), the workgroup that finished it and
 * its kind.  Errors: -ENOENT (no trace). */
int dc_trace_get(dc_runtime *rt, int64_t t, int64_t *start_ns, int64_t *end_ns,
                 int32_t *worker, int32_t *kind);

/* Diagnostics of the last flushed graph: host time spent laying out the
 * graph (ms), work units, and workgroups launched (queue executor: all
 * classes together; level executor: the largest level).  Any output pointer
 * may be NULL. */
int dc_last_launch(dc_runtime *rt, double *build_ms, int64_t *units, int32_t *workers);

/* Per-kernel timing.  While enabled, every launch of the executor's
 * kernels is bracketed by HIP events on the stream it is launched on (queue
 * executor: one launch per class spanning the graph; level executor: one per
 * level and kernel); each
 * completed graph adds the measured durations and the algorithmic work of
 * the units those launches ran.  Algorithmic work per task (the operation's
 * definition, independent of how the kernel computes it): POTRF m^3/3 + m^2/2
 * + m/6 flop; TRSM and the solve TRSMs m n^2; SYRK m(m+1)k; GEMM and the
 * solve GEMMs 2mnk; RESID 2 m^2 r; AXPY 2mn; SCAL m; CAST 0.  Bytes: every
 * operand read once and every output written once at its storage precision
 * (lower triangles for POTRF, SYRK's C and the L of the TRSMs). */
typedef struct {
  int64_t launches;   /* kernel launches timed */
  double ms;          /* sum of their durations */
  double flops;       /* algorithmic flops of the units they ran */
  double bytes;       /* algorithmic bytes of the units they ran */
} dc_kernel_stat;
typedef struct {
  dc_kernel_stat panel;   /* POTRF, TRSM, solve, cast, residual, axpy, scal */
  dc_kernel_stat gemm;    /* GEMM and SYRK */
} dc_kernel_stats;
/* enable != 0 switches timing on and clears the totals; 0 switches it off. */
int dc_kernel_timing(dc_runtime *rt, int enable);
/* Totals over the graphs completed since timing was enabled. */
int dc_kernel_stats_get(dc_runtime *rt, dc_kernel_stats *out);

/* ------------------------------------------------ high-level operations */

/* Each of these only submits tasks through dc_task_submit (the matrix must
 * be registered and not partitioned; it is partitioned with the given tile
 * size for the duration of the call) and then waits.
 *
 * dc_potrf: tiled right-looking Cholesky of the lower triangle of A in
 * place, in FP64: for k, POTRF(k); TRSM(i,k) for i>k; SYRK(i,k) and
 * GEMM(i,j,k) for k<j<i.  Result: dc_get_info(A).  With tile >= 16 the
 * panel solves of column k are TRSM(k+1,k) by substitution (it leads to the
 * next POTRF) and, for i >= k+2, TRTRI(k) into a workspace W_k followed by
 * TRSM_INV(i,k) (same result up to rounding; ill-conditioned diagonal tiles
 * fall back to substitution, see DC_TRSM_INV).  The runtime
 * keeps the workspace, (tiles - 1) * tile^2 doubles, until dc_shutdown;
 * -ENOMEM if it cannot be allocated.
 * upd selects the precision of the trailing updates (the mixed-precision
 * factor of dc_posv_ir, exposed on its own): DC_F64 as above; DC_F32 or
 * DC_BF16: the diagonal tiles are factored in A in FP64, the off-diagonal
 * tiles are copied to an FP32 workspace (and BF16 copies for DC_BF16),
 * solved there with FP64 arithmetic rounded to FP32, updated with FP32 or
 * BF16 products accumulated in FP32, and copied back into A (exactly).  The
 * result in A is then the mixed factor whose accuracy dc_posv_ir refines;
 * the runtime keeps that workspace (n^2 floats, n^2 BF16 values for
 * DC_BF16, and the inverse tiles) until dc_shutdown. */
int dc_potrf(dc_runtime *rt, dc_handle A, int64_t tile, dc_dtype upd);

/* dc_potrf_noalloc: for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation).  The
 * FP64 factorisation of dc_potrf without any device or pinned-memory
 * allocation (no hipMalloc, hipFree, hipHostMalloc or similar): the graph's
 * device layout (task descriptors, work items, level counters, status words)
 * is written to a fixed 16 MiB scratch array that the library keeps on every
 * device it runs on until the process ends, staged through a fixed host area
 * of the same size; both kernels of a level run on the runtime's stream.  The
 * panel solves are substitution TRSM tasks (no inverse workspace), so the
 * factor equals dc_potrf's up to rounding.  Host bookkeeping (handles, the
 * task list) uses the C++ heap as every call does.  The counters the kernels
 * start from are written by every call.  All calls on one device share its
 * scratch array, and all calls share the staging area: calls that overlap
 * race.  Errors: as dc_potrf; -ENOMEM (nothing runs) when the layout does not
 * fit the scratch (n = 32768 with tile 512 fits; tiles far smaller than 128
 * at large n do not); -EIO if the scratch's address could not be found when
 * the runtime was created. */
int dc_potrf_noalloc(dc_runtime *rt, dc_handle A, int64_t tile);

/* dc_potrs: solves L L^T X = B in place in B (n x r, FP64) with the factor
 * in the lower triangle of L: forward sweep TRSM_L/GEMM_RHS_N, backward
 * sweep TRSM_LT/GEMM_RHS_T. */
int dc_potrs(dc_runtime *rt, dc_handle L, dc_handle B, int64_t tile);

/* Mixed-precision solve with FP64-residual iterative refinement.  A (n x n
 * FP64, lower triangle) is left unchanged.  upd selects the precision of the
 * SYRK/GEMM updates (DC_F64, DC_F32 or DC_BF16); the diagonal POTRF tasks
 * stay FP64 and off-diagonal factor tiles are stored in FP32 when upd is not
 * DC_F64.  x0 = solve(b); then r = b - A x (FP64 storage, computed as a
 * compensated dot product per row, as accurate as twice-FP64 arithmetic
 * rounded once), d = solve(r), x += d, until ||d||_inf <= tol ||x||_inf for
 * every column (converged; that last d is still added), or, from the second
 * correction on, until the error left after adding d_i, estimated from the
 * contraction ratio as ||d_i||^2 / (||d_{i-1}|| - ||d_i||), is <= tol ||x||_inf
 * for every column (converged, d_i added; this saves the solve that would
 * only confirm it), stagnation (||d_i|| > 0.5 ||d_{i-1}|| in some column;
 * d_i is not added) or maxit steps.  If the factor breaks down or refinement does not converge,
 * the next wider precision is used (BF16 -> FP32 -> FP64).  B and X are
 * n x r FP64; X receives the solution. */
typedef struct {
  int iterations;        /* refinement steps before the one that met the
                            test, with the precision that was kept */
  int converged;         /* 1 if the stopping test was met */
  int final_prec;        /* dc_dtype actually used for the updates */
  int fallbacks;         /* precision changes made */
  double last_update;    /* ||d||_inf / ||x||_inf at the last step */
  double factor_ms;      /* device time of the last factorisation */
  double refine_ms;      /* device time of the solves and refinement */
} dc_ir_report;
int dc_posv_ir(dc_runtime *rt, dc_handle A, dc_handle B, dc_handle X,
               int64_t tile, dc_dtype upd, double tol, int maxit,
               dc_ir_report *rep);

/* Batched factorisation and solve: factors each of the count SPD matrices
 * A[i] (lower triangle, in place) with tile size tiles[i] (0: the matrix
 * order, i.e. one POTRF task) and, where B != NULL and B[i] != 0, solves
 * A[i] X = B[i] in place in B[i] (B FP64).  A[i] is FP64, or FP32 factored as
 * one tile (tiles[i] 0 or >= its order; FP64 arithmetic, the factor rounded
 * to FP32, the solve in FP64 arithmetic on the FP32 factor); FP64 and FP32
 * matrices may be mixed in one call.  All tasks of all matrices form one
 * graph, run by one flush of the executor.  info_out (optional) receives
 * each matrix's status (0 or the 1-based breakdown column).  Errors as for
 * dc_potrf; on an error no task runs. */
int dc_potrf_batched(dc_runtime *rt, int64_t count, const dc_handle *A, const dc_handle *B,
                     const int64_t *tiles, int64_t *info_out);

/* --------------------------------------------------------------- serving */

/* Continuous-batching solve server.  Requests (one SPD system each) are
 * admitted in arrival order as soon as one of `slots` slots and enough of the
 * server's device memory pool are free; each admitted request runs on its own
 * runtime and streams, so the work of requests in different slots overlaps on
 * the GPU.  Per request (A is read in place and must stay alive until the
 * request completes): factorisation into a workspace in the pool (FP64
 * diagonal tiles, off-diagonal updates at precision `upd`), solve and
 * FP64-residual refinement with the stopping tests of dc_posv_ir; a
 * breakdown or failed refinement restarts the request with the next wider
 * update precision (BF16 -> FP32 -> FP64).
 * The server object is driven by one host thread. */
typedef struct dc_server dc_server;

typedef struct {
  int device;          /* HIP device ordinal */
  int slots;           /* concurrent requests (1..64) */
  size_t pool_bytes;   /* device memory the server allocates for workspaces */
  int64_t tile;        /* tile size of the factorisations (<= 512) */
  int upd;             /* dc_dtype of the trailing updates */
  double tol;          /* refinement stopping threshold */
  int maxit;           /* refinement steps before giving up */
  int64_t whole_max;   /* requests of order <= whole_max (<= 512) are
                          factored as a single tile, larger ones with
                          `tile`; default 512, 0: every request uses
                          `tile` */
  int64_t mixed_min;   /* with upd FP32 or BF16: requests of order below
                          mixed_min use FP64 updates (their factorisation
                          costs less than the refinement steps the
                          low-precision factor needs); default 0: every
                          request uses upd */
  int64_t tile_large;  /* tile size (<= 512) of requests of order >=
                          large_min; default 512 */
  int64_t large_min;   /* order from which tile_large replaces tile;
                          default 4096 (at 4096 and above, 512-tiles
                          served 1.2-1.5x the requests per second of
                          256-tiles); 0: never */
} dc_server_config;

typedef struct {
  int64_t n, r;        /* order and right-hand-side count */
  const double *A;     /* device, n x n row-major FP64 (lower triangle read);
                          must stay valid until the request completes */
  const double *B;     /* device, n x r row-major FP64 */
  double *X;           /* device, n x r row-major FP64: the solution */
  double arrival;      /* arrival time in dc_server_now's clock (seconds) */
} dc_request;

typedef struct {
  int64_t id;          /* id returned by dc_server_submit */
  int status;          /* 0, or a negative errno if the request failed */
  int64_t info;        /* breakdown column of the (FP64) factorisation, or 0 */
  int converged, iterations, final_prec, restarts;
  double last_update;  /* ||d||_inf / ||x||_inf at the last step */
  double arrival, admitted, completed;   /* dc_server_now clock, seconds */
} dc_request_result;

/* Defaults: device 0, 4 slots, 64 GiB pool, tile 256 (512 from order
 * 4096), FP32 updates, tol 1e-12, 30 refinement steps. */
void dc_server_config_default(dc_server_config *cfg);
/* Errors: -EINVAL, -ENOMEM (pool allocation), -EIO. */
int dc_server_create(dc_server **srv, const dc_server_config *cfg);
/* Waits for the requests in flight, frees everything the server owns. */
int dc_server_destroy(dc_server *srv);
/* Seconds since the server was created (the clock of arrival/completion). */
double dc_server_now(dc_server *srv);
/* Queues a request; *id receives its id.  The request's A and B must hold
 * their values when this is called: the slots run on their own streams, and
 * nothing orders them after work the caller still has in flight on other
 * streams (synchronise first).  Errors: -EINVAL, -ENOMEM (its FP64 workspace
 * can never fit in the pool). */
int dc_server_submit(dc_server *srv, const dc_request *req, int64_t *id);
/* Never blocks: advances every request whose last step finished, admits
 * waiting requests, and copies up to cap completed results into results;
 * *ndone receives their number and *active (optional) the number of
 * requests still queued or running. */
int dc_server_progress(dc_server *srv, dc_request_result *results, int cap, int *ndone,
                       int *active);

#ifdef __cplusplus
}
#endif

#endif /* DAGCHOL_H */
