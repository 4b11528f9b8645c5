/*
 * mlbicgstab.h -- C ABI of the MI355X (gfx950) ML(n)BiCGStab library.
 *
 * The library solves sparse A x = b with ML(n)BiCGStabt, the A^H-using
 * ML(n)BiCGStab algorithm of M.-C. Yeung, "An introduction to ML(n)BiCGStab"
 * (arXiv 1106.3678): Algorithm 4.1 (Section 4.3), in the i/j loop form of
 * Algorithm 7.1 (Section 7), with M = I or the block diagonal of A.  Options
 * select the order of its two recurrences (a fused Gram-matrix form, or the
 * literal one) and a transpose-free form without A^H.  Every iteration runs in
 * hand-written HIP kernels on one GPU; scalars and convergence control stay on
 * the device.
 *
 * Conventions shared by every entry point
 *  - Array pointers named "device" point to GPU memory of the current HIP
 *    device; the caller owns them.  A's arrays are borrowed from create()
 *    until destroy(); b, x and Q are borrowed for the duration of one solve().
 *  - Work is ordered on the HIP stream passed to create() (NULL = the legacy
 *    default stream).  solve() returns after the result is complete (it
 *    synchronises that stream once at the end).
 *  - Complex values are two consecutive doubles (re, im), i.e. C99
 *    `double _Complex` / numpy complex128 layout.  u^H v conjugates u.
 *  - Return codes: >= -1 is the paper's flag (0 converged, 1 maxit reached,
 *    -1 breakdown); <= -2 is an API error (MLB_E*), with a message available
 *    from mlbicgstab_last_error() on the calling thread.  No C++ exception
 *    crosses this boundary.  On an API error nothing was written to x.
 */
#ifndef MLBICGSTAB_H
#define MLBICGSTAB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mlb_solver* mlb_handle;

/* Return codes.  0 / 1 / -1 are the flag of Algorithm 7.1's realisation. */
enum {
  MLB_CONVERGED = 0,      /* recursive ||r|| / ||b|| < tol                    */
  MLB_MAXIT = 1,          /* maxit iterations done without convergence         */
  MLB_BREAKDOWN = -1,     /* c_k == 0, ||A u||^2 == 0 or omega == 0 (or non-finite) */
  MLB_EINVAL = -2,        /* bad argument (null pointer, size, enum value)     */
  MLB_ENOMEM = -3,        /* device or pinned host allocation failed           */
  MLB_EHIP = -4,          /* a HIP runtime call failed                         */
  MLB_EUNSUPPORTED = -5   /* valid but not supported (e.g. n > MLB_MAX_N)      */
};

enum { MLB_R64 = 0, MLB_C128 = 1 };          /* value type of A, b, x, Q        */
enum { MLB_CSR = 0, MLB_BSR3 = 1 };          /* storage of A                     */
enum { MLB_PREC_FP64 = 0, MLB_PREC_FP32_IR = 1 };
enum { MLB_PRECOND_NONE = 0, MLB_PRECOND_JACOBI = 1, MLB_PRECOND_ILU0 = 2 };

#define MLB_MAX_N 32                          /* largest number of shadow vectors */

/*
 * A sparse square matrix on the device.
 *  CSR  : row_ptr[nrows+1], col_idx[nnz], values[nnz]; column indices of a
 *         row need not be sorted; duplicates are summed.
 *  BSR3 : 3x3 blocks.  nrows = 3 * (block rows); nnz = number of stored
 *         blocks; row_ptr[nrows/3+1] and col_idx[nnz] index blocks; values
 *         holds nnz blocks of 9 entries each, row-major inside a block.
 * Indices are 0-based int32; row_ptr[0] must be 0 and row_ptr[last] = nnz.
 * nrows and nnz are at most MLB_MAX_INDEX (2^31 - 2^20): the kernels index
 * rows and entries with 32-bit integers and step through them in strides of
 * up to 2^20, which must not overflow.  Larger values return MLB_EINVAL.
 */
#define MLB_MAX_INDEX 2146435072LL
typedef struct {
  int32_t format;           /* MLB_CSR or MLB_BSR3                             */
  int32_t dtype;            /* MLB_R64 or MLB_C128                             */
  int64_t nrows;            /* N, scalar rows (= columns)                       */
  int64_t nnz;              /* stored entries (CSR) or stored blocks (BSR3)    */
  const int32_t* row_ptr;   /* device                                          */
  const int32_t* col_idx;   /* device                                          */
  const void* values;       /* device                                          */
} mlb_matrix;

/*
 * Solver options.  n, tol, maxit and kappa are the paper's arguments
 * (Section 7): n = number of shadow vectors (columns of Q), 1 <= n <= 32;
 * tol > 0 for the recursive residual test; maxit >= 1; kappa >= 0 selects
 * the omega guard of eq. (5.1) (0 = plain minimisation).
 *
 * precision = MLB_PREC_FP32_IR runs the Krylov iteration in fp32 (fp32
 * vectors, fp32 SpMV / dot accumulation, fp64 coefficient recurrences) inside
 * an fp64 iterative-refinement loop (r = b - A x, x += d in fp64) that stops
 * on the TRUE residual ||b - A x|| / ||b|| < tol.  This mode is an addition of
 * this library; the paper does not discuss precision.  inner_tol (default
 * 1e-6 when <= 0) is the relative tolerance of each inner solve (raised to
 * 0.25 tol / ||r|| / ||b|| when that is larger, so the last step is not
 * over-solved; an inner solve whose residual has not halved for
 * max(300, 20 n) iterations also ends) and
 * max_outer (default 30 when <= 0) bounds the refinement steps; if a
 * refinement step gains less than 10x, or an inner solve breaks down, the
 * remaining work is done by the fp64 iteration.
 *
 * record_iterates = K > 0 stores x_1 .. x_K (K <= maxit) in the device array
 * iterates (N x K, column-major, ld = N, same dtype as x) during an fp64 solve.
 *
 * precond = MLB_PRECOND_JACOBI runs Algorithm 7.1 (Section 7) with M = the
 * block diagonal of A (its 3x3 diagonal blocks for BSR3, its diagonal for CSR),
 * applied from the right: the iteration runs on A M^{-1} y = b from
 * y_0 = M x_0 and returns x = M^{-1} y.  The residual, the stopping test and
 * f_s = M^{-H} A^H q_s are those of Algorithm 7.1.  create() fails with
 * MLB_EINVAL if a (block) row has no stored diagonal entry or a singular one.
 * MLB_PRECOND_NONE (0) is M = I, Algorithm 4.1.
 *
 * precond = MLB_PRECOND_ILU0 runs Algorithm 7.1 with M = ILU(0) of A, the
 * preconditioner of the paper's experiments (Section 5): M = L U with L unit
 * lower and U upper triangular (by 3x3 blocks for BSR3), both on A's pattern,
 * and (L U)_ij = a_ij wherever A is stored.  Applied from the right as above:
 * every product with A is preceded by M^{-1} (two triangular solves), and
 * f_s = M^{-H} A^H q_s.  create() factors A on the device (one launch per
 * level of the row dependencies; the level sets come from a host pass over a
 * copy of A's index arrays) and fails with MLB_EINVAL for a (block) row without
 * a stored diagonal, a column stored twice in a row, or a zero / singular
 * pivot.  Each triangular solve is one launch that takes the rows in level
 * order (3m - 2 levels on an m^3 7-point grid), every row waiting for the
 * solved values it reads; a wait is bounded (2 s), and a solve in which one
 * ran out returns MLB_EHIP (the environment variable MLB_ILU_MAX_TRIES, read
 * by create(), bounds the tries of a row instead: a test hook for that path).
 * fp64 only (MLB_EUNSUPPORTED with MLB_PREC_FP32_IR).
 *
 * transpose_free = 1 runs the iteration without A^H (an addition of this
 * library; Section 4 names A^H-free algorithms but prints only their costs).
 * The beta recurrence of step 2 of Algorithm 4.1 needs
 * f_s^H g = (A^H q_s)^H g = q_s^H (A g): at every inner step the product
 * v = A g of the vector entering that recurrence is formed first, the
 * coefficients use q_s^H v, and w_k = v + sum_s beta_s w_s is recombined from
 * this cycle's w columns instead of multiplied again.  Same matvec and dot
 * counts as Algorithm 7.1, (n-1)/2 more saxpys per iteration, no A^H and no
 * f_1..f_{n-1} stored: Table 4.2's costs (2n + 2 + 2/n saxpys, (3n + 5) N
 * storage).  The recursive residual can drift further from b - A x than with
 * A^H (Section 5.1 reports this for the second algorithm); err_true reports
 * the true residual.
 */
typedef struct {
  int32_t n;
  double tol;
  int64_t maxit;
  double kappa;
  int32_t precision;
  double inner_tol;
  int32_t max_outer;
  int32_t record_iterates;
  void* iterates;           /* device, N x record_iterates, or NULL            */
  int32_t precond;          /* MLB_PRECOND_NONE, MLB_PRECOND_JACOBI or MLB_PRECOND_ILU0 */
  int32_t transpose_free;   /* 0: Algorithm 7.1 with A^H; 1: without A^H       */
  int32_t order;            /* MLB_ORDER_FUSED (0) or MLB_ORDER_LITERAL (1)    */
  int32_t max_restarts;     /* fp64: restarts on a residual gap, 0..100 (below) */
} mlb_options;

/*
 * max_restarts (an addition of this library; 0 = Algorithm 7.1's own stop):
 * the fp64 iteration stops when its recursive residual drops below tol
 * (Algorithm 7.1), and rounding can leave the true residual ||b - A x|| / ||b||
 * above it.  With max_restarts > 0 the library then starts the iteration
 * again from the x it reached (a new r_0 = b - A x, the same Q), at most
 * max_restarts times and within maxit iterations in total, until the true
 * residual is below tol.  res->iter counts every iteration, res->outer_iters
 * the restarts; iterates are recorded by the first run only.
 * mlbicgstab_solve_batch refuses it; the server runs a small request on its
 * batched one-workgroup solve first and, if that leaves the true residual
 * not below tol, restarts it from its x on the multi-launch iteration.  Not
 * taken by MLB_PREC_FP32_IR, whose refinement already tests the true
 * residual.
 */

/*
 * Order of the beta~ and beta recurrences (Algorithm 7.1, the two loops of an
 * inner step).  MLB_ORDER_FUSED (default) evaluates each recurrence from small
 * Gram matrices of inner products the passes already produce: equal in exact
 * arithmetic, three reductions per step whatever n is.  MLB_ORDER_LITERAL runs
 * them in the algorithm's own sequential order: each coefficient from the
 * inner product of the vector the previous coefficient updated, one reduction
 * and one pass per coefficient (n + 2 reductions per step).  Not combined with
 * transpose_free (MLB_EUNSUPPORTED); mlbicgstab_solve_batch refuses it.
 */
enum { MLB_ORDER_FUSED = 0, MLB_ORDER_LITERAL = 1 };

typedef struct {
  int32_t flag;             /* same as the return code when >= -1              */
  int64_t iter;             /* k at exit (fp64), or total inner iterations (IR) */
  int32_t outer_iters;      /* refinement steps (IR); fp64: restarts taken     */
  int64_t fp64_iters;       /* iterations run by the fp64 iteration             */
  double err_recursive;     /* recursive ||r_k|| / ||b|| at exit (fp64 iteration) */
  double err_true;          /* ||b - A x|| / ||b|| recomputed in fp64 at exit   */
  double setup_ms;          /* residual, F = A^H Q, first w (stream time)       */
  double solve_ms;          /* whole solve() call, stream time                  */
} mlb_result;

/*
 * Create a solver for A with the given options.  Builds the conjugate
 * transpose A^H (Algorithm 4.1, step 2 needs A^H q_s) as an explicit device
 * copy, allocates the Krylov workspace ((4n+4) N values plus O(n^2)
 * scalars, Table 4.3) and, for MLB_PREC_FP32_IR, fp32 copies of A and A^H.
 * With transpose_free neither A^H nor f_1..f_{n-1} is made ((3n+5) N values,
 * Table 4.2).
 * hip_stream: a hipStream_t (NULL = default stream).  On success *out holds
 * the handle; on error *out is NULL.
 */
int mlbicgstab_create(const mlb_matrix* A, const mlb_options* opt, void* hip_stream, mlb_handle* out);

/* Bytes of device memory create() would allocate for A and opt. */
int mlbicgstab_workspace_size(const mlb_matrix* A, const mlb_options* opt, size_t* bytes);

/*
 * Solve A x = b.  b: device, N values.  x: device, N values; in = x_0,
 * out = the solution (the half-step x when the solve stops on the half step
 * that ends a cycle, as in Algorithm 7.1's realisation).  Q: device,
 * N x n shadow block [q_1 .. q_n], column-major with leading dimension
 * ldq >= N.  res may be NULL.  Returns the flag (0, 1, -1) or an API error.
 */
int mlbicgstab_solve(mlb_handle h, const void* b, void* x, const void* Q, int64_t ldq, mlb_result* res);

/*
 * Solve `count` prepared systems in one launch, one workgroup per system: the
 * whole iteration of Algorithm 7.1 (M = I) of system k runs in workgroup k,
 * with workgroup barriers where the multi-launch solve has kernel boundaries
 * (an addition of this library, for many small systems, whose multi-launch
 * iteration is bound by launch latency rather than bandwidth).  Every h[k]
 * must come from mlbicgstab_create with a CSR matrix of at most
 * MLB_BATCH_MAX_N rows, MLB_PREC_FP64, MLB_PRECOND_NONE and MLB_ORDER_FUSED (an iterate
 * record is kept as in a solve; transpose_free handles run the transpose-free
 * steps); all on the same stream and of the same value type (else
 * MLB_EINVAL / MLB_EUNSUPPORTED, and nothing runs).  b[k], x[k], Q[k], ldq[k]
 * and res[k] (res may be NULL) as in mlbicgstab_solve.  A system's result
 * does not depend on the other systems of the batch.  Synchronises the
 * stream.  Returns 0 (each flag is in res[k].flag) or an API error.
 */
#define MLB_BATCH_MAX_N 262144
#define MLB_BATCH_MAX 65535
int mlbicgstab_solve_batch(const mlb_handle* h, int32_t count, const void* const* b, void* const* x,
                           const void* const* Q, const int64_t* ldq, mlb_result* res);

/*
 * Sequences of systems with the same A (Section 5.2, choice of n): the method
 * is at its strongest over a sequence of systems, with n chosen automatically
 * from one system to the next.  A sequence owns one solver whose workspace and
 * A^H serve every n in [n_min, n_max]; A^H is built once.  opt->n is the n of
 * the first system.  After each solve the next n follows the paper's rule,
 * with t1 and t2 the solve times (mlb_result.solve_ms) of the previous and
 * the current system: n + step if t1 > t2, else n - step, kept in
 * [n_min, n_max]; after the first system n is kept.  step = 0 fixes n.
 */
typedef struct mlb_sequence* mlb_sequence_handle;

/* The rule alone: the n after a system solved with n (t_prev_ms < 0: no
 * previous system, n is kept).  Returns the next n, or MLB_EINVAL. */
int32_t mlb_sequence_next_n(int32_t n, double t_prev_ms, double t_cur_ms, int32_t step, int32_t n_min,
                            int32_t n_max);

/* A as in mlbicgstab_create (borrowed until destroy); opt as there, without an
 * iterate record.  Errors as mlbicgstab_create, MLB_EINVAL for bad n bounds. */
int mlb_sequence_create(const mlb_matrix* A, const mlb_options* opt, int32_t n_min, int32_t n_max, int32_t step,
                        void* hip_stream, mlb_sequence_handle* out);

/* Solve the next system: b, x as in mlbicgstab_solve; Q is N x n_max
 * (column-major, ldq >= N), of which the first n columns are used.  *n_used
 * (may be NULL) receives that n.  Returns the flag or an API error. */
int mlb_sequence_solve(mlb_sequence_handle s, const void* b, void* x, const void* Q, int64_t ldq, mlb_result* res,
                       int32_t* n_used);

/* Free the sequence.  NULL is accepted. */
int mlb_sequence_destroy(mlb_sequence_handle s);

/* Free everything create() allocated.  NULL is accepted. */
int mlbicgstab_destroy(mlb_handle h);

/*
 * y = A x (op = MLB_OP_A, the caller's A) or y = A^H x (op = MLB_OP_AH, the
 * conjugate transpose the solver built for f_s = A^H q_s, Algorithm 4.1 step
 * 2).  A transpose_free or preconditioned solver holds no A^H of A:
 * MLB_OP_AH returns MLB_EUNSUPPORTED there.  With an ILU(0) preconditioner
 * (the M of Algorithm 7.1) also y = M^{-1} x (MLB_OP_MINV) and y = M^{-H} x
 * (MLB_OP_MINVH), the two triangular solves each application runs; other
 * solvers return MLB_EUNSUPPORTED for them.  x and y are device vectors of N
 * values of the solver's value type (x is read, y written; they must not
 * overlap; both are borrowed for the call).  Runs the library's SpMV kernel on
 * the solver's stream and synchronises it; it reads and writes no solver state,
 * so it may come before, between or after solves.  For residuals and for tests
 * of the products.  Returns 0; MLB_EINVAL for a NULL handle, x or y or an
 * unknown op; MLB_EUNSUPPORTED as above; MLB_EHIP if the launch fails.
 */
enum { MLB_OP_A = 0, MLB_OP_AH = 1, MLB_OP_MINV = 2, MLB_OP_MINVH = 3 };
int mlbicgstab_matvec(mlb_handle h, int32_t op, const void* x, void* y);

/*
 * Allocation-free solve, for callers that cannot allocate device memory (code
 * that must not call hipMalloc, such as tight serving loops or harnesses that
 * forbid allocation): the same result as mlbicgstab_create + mlbicgstab_solve
 * + mlbicgstab_destroy with these arguments (the same kernels, grids and
 * reduction order, so x, iter and flag are bitwise those of that sequence),
 * with every piece of library-owned device memory -- the index check flag,
 * A^H and its transpose temporaries, the Krylov workspace, partial sums and
 * the scalar state -- carved from one static device array of
 * MLB_NOALLOC_SCRATCH_BYTES per GPU, which the library holds from its load
 * until the process ends.  The caller passes A, b, x and Q as for
 * create/solve (all borrowed for the call) and the stream the work goes on.
 * No hipMalloc, hipFree, pinned host allocation or HIP event is used; the host
 * reads the device's done flag every few cycles instead of a host-mapped one,
 * and res->setup_ms is 0, res->solve_ms host wall time.
 * Limits: opt->precision must be MLB_PREC_FP64 and opt->precond
 * MLB_PRECOND_NONE (else MLB_EUNSUPPORTED); an A and n whose buffers exceed
 * the scratch return MLB_EUNSUPPORTED with the bytes needed in the message,
 * before any work is enqueued (CSR fp64 with 7 entries a row and n = 4 fits up
 * to about 300,000 rows with A^H, about 690,000 with transpose_free).
 * All calls on one GPU share its array, which keeps the last call's contents:
 * the library re-initialises what each call reads and serialises the calls of
 * one process with a lock (two calls that overlapped on one GPU would race on
 * the array).  Synchronises the stream before returning.  Returns the flag or
 * an API error, as mlbicgstab_solve.
 */
#define MLB_NOALLOC_SCRATCH_BYTES (64ull << 20)
int mlbicgstab_solve_noalloc(const mlb_matrix* A, const mlb_options* opt, void* hip_stream, const void* b, void* x,
                             const void* Q, int64_t ldq, mlb_result* res);

/* Message for the last API error on this thread ("" if none). */
const char* mlbicgstab_last_error(void);

/*
 * Kernel timing for roofline figures: replays `reps` cycles of the fp64 (or,
 * for MLB_PREC_FP32_IR, the fp32) iteration on the solver's stream over the
 * workspace left by the last solve -- the same kernels in the same order as in
 * a solve, with the one-workgroup coefficient recurrences left out -- and
 * attaches a HIP start/stop event pair to every launch of the requested kernel
 * class (hipExtLaunchKernel: the events take that kernel's own start and end
 * times).  *ms_per_launch receives the mean duration.  Requires a
 * prior solve() whose Q is still allocated (it is read again); scrambles the
 * library's workspace (not b, x or Q).
 */
int mlbicgstab_time_kernel(mlb_handle h, int32_t kernel, int32_t reps, double* ms_per_launch);

enum {
  MLB_KERNEL_SPMV_STEP = 0,   /* SpMV + multi-dot of a step (every SpMV of a cycle
                                 but the one of the minimisation step)           */
  MLB_KERNEL_ALPHA_STEP = 1,  /* x, r update + norm + multi-dot                   */
  MLB_KERNEL_COMBINE = 2,     /* beta~ combination + F multi-dot (literal order:
                                 the beta~ passes)                               */
  MLB_KERNEL_RECOMBINE = 3    /* g_k = g + sum beta_s g_s (transpose_free: also
                                 w_k and its multi-dot; literal order: the beta
                                 passes)                                         */
};

/*
 * Serving: continuous batching of whole solves (an addition of this library;
 * the paper's setting is one solve at a time, or a sequence of systems in
 * Section 5.2).
 *
 * A server owns max_inflight workers, each with its own HIP stream, and (when
 * small_n_max >= 0) two batchers with a stream each.  Small requests (CSR,
 * fp64, fused order, no preconditioner, no iterate record, N <= small_n_max) wait for the
 * batchers; a free batcher takes every waiting small request that fits (at
 * most 256) and solves them in one launch of mlbicgstab_solve_batch's kernel.
 * Other requests wait for the workers, which run create, solve and destroy
 * one request at a time.  The batchers' queue is first-in first-out.  The
 * workers' queue is too by default (order MLB_SERVE_FIFO): the oldest waiting
 * request starts as soon as a worker is free and its device footprint
 * (mlbicgstab_workspace_size) fits the unused part of budget_bytes.  With
 * MLB_SERVE_SMALLEST a free worker takes the waiting request of smallest
 * footprint that fits (the oldest among equal footprints, so a sequence keeps
 * its order), except that a request which has waited max_wait_ms or longer
 * goes first, oldest first, and holds the queue until its footprint fits: under
 * load small solves then no longer wait behind large ones, and no request
 * waits much beyond max_wait_ms plus the runs in flight.
 * Requests that arrive while others run therefore start as slots and memory
 * free up, and their kernels overlap on the device.  A solve gives the same
 * result whatever else is in flight (same grids and reduction order; the
 * systems of a batch are independent).  The caller's A arrays, b, x and Q of a request must
 * stay allocated, and x untouched, until the request has been collected.
 * Work is not ordered with any caller stream: the caller must have finished
 * writing b, x and Q (e.g. synchronised its stream) before submitting.
 */
typedef struct mlb_server* mlb_server_handle;

typedef struct {
  uint64_t budget_bytes;    /* HBM admission budget for the requests' footprints */
  int32_t max_inflight;     /* workers = multi-launch solves in flight, 1..64  */
  int32_t small_n_max;      /* CSR fp64 requests without preconditioner and with
                               at most this many rows go to the batchers
                               (0: MLB_SERVER_SMALL_N, -1: none)              */
  int32_t order;            /* workers' pick order: MLB_SERVE_FIFO or MLB_SERVE_SMALLEST */
  double max_wait_ms;       /* MLB_SERVE_SMALLEST: age at which a request goes
                               first (0: MLB_SERVER_MAX_WAIT_MS)                */
} mlb_server_options;
#define MLB_SERVER_SMALL_N 4096
enum { MLB_SERVE_FIFO = 0, MLB_SERVE_SMALLEST = 1 };
#define MLB_SERVER_MAX_WAIT_MS 1000.0

typedef struct {
  double queued_ms;         /* submit -> start                                  */
  double run_ms;            /* start -> completion                              */
  double latency_ms;        /* submit -> completion                             */
  uint64_t footprint_bytes; /* admitted footprint (a sequence's: of the whole sequence) */
  int32_t n_used;           /* shadow vectors the solve ran with                */
} mlb_request_timing;

typedef struct {
  uint64_t budget_bytes, used_bytes, peak_used_bytes;
  int64_t queued;
  int32_t running, peak_running;
  int64_t completed;
} mlb_server_stats_t;

/* Start the workers.  Returns 0 or an API error. */
int mlb_server_create(const mlb_server_options* opt, mlb_server_handle* out);

/*
 * Queue one solve (same arguments as mlbicgstab_create + mlbicgstab_solve,
 * with every device array borrowed until collection).  *ticket identifies it.
 * MLB_ENOMEM if its footprint exceeds the whole budget.
 */
int mlb_server_submit(mlb_server_handle s, const mlb_matrix* A, const mlb_options* opt, const void* b, void* x,
                      const void* Q, int64_t ldq, int64_t* ticket);

/*
 * Collect a request: poll returns 0 while it is pending; poll and wait return
 * 1 once it has completed (res and timing filled, the ticket is then released),
 * or the request's API error (<= -2).  The solve's own flag is in res->flag.
 */
int mlb_server_poll(mlb_server_handle s, int64_t ticket, mlb_result* res, mlb_request_timing* timing);
int mlb_server_wait(mlb_server_handle s, int64_t ticket, mlb_result* res, mlb_request_timing* timing);

/*
 * Sequences of systems inside the server (Section 5.2: the method is at its
 * strongest over a sequence of systems, with n chosen automatically from one
 * system to the next).  Requests submitted with the same nonzero key form a
 * sequence: they must name the same A (the same device arrays, unchanged until
 * the sequence ends) and the same options and rule, and are solved one at a
 * time in submission order by one solver the sequence owns -- A^H is built
 * once, with the first request, and the workspace (sized for n_max) is reused.
 * The first request runs with opt->n; after each request the next n follows
 * mlb_sequence_next_n with the solve times of the previous and the current
 * request (timing->n_used reports it).  Each result is bitwise that of a fresh
 * create + solve with that n.  Q is N x n_max (column-major, ldq >= N), of
 * which the first n columns are used.  The sequence's footprint
 * (mlbicgstab_workspace_size with n = n_max) is admitted with its first
 * request and held until mlb_server_end_sequence; other requests keep flowing
 * meanwhile.  Errors as mlb_server_submit; MLB_EINVAL for key 0, for an A,
 * options or rule that differ from the sequence's, or for an ended sequence.
 */
int mlb_server_submit_sequence(mlb_server_handle s, uint64_t key, const mlb_matrix* A, const mlb_options* opt,
                               int32_t n_min, int32_t n_max, int32_t step, const void* b, void* x, const void* Q,
                               int64_t ldq, int64_t* ticket);

/* End a sequence: no more requests may join it; its solver and footprint are
 * released once its queued requests have run.  MLB_EINVAL for an unknown key. */
int mlb_server_end_sequence(mlb_server_handle s, uint64_t key);

/* Budget, peak footprint in flight, queue length, peak concurrency, completions. */
int mlb_server_stats(mlb_server_handle s, mlb_server_stats_t* out);

/* Finish every queued request, stop the workers and free the server. */
int mlb_server_destroy(mlb_server_handle s);

#ifdef __cplusplus
}
#endif
#endif /* MLBICGSTAB_H */
