/*
 * xamg.h -- C ABI of libxamg.so, an MI355X (gfx950) solve phase for sparse
 * linear systems with multiple right-hand sides, A X = B with X, B of size
 * n x m (Krasnopolsky and Medvedev, "XAMG: a library for solving linear
 * systems with multiple right-hand side vectors", Section 1, the equation
 * A X = B; Sections 2.1-2.2 for the methods and the multi-RHS design).
 *
 * The method: classical algebraic multigrid (Ruge-Stueben coarsening,
 * direct interpolation, Galerkin coarse operators), built once on the host,
 * used as a V(1,1) preconditioner with Jacobi or Chebyshev smoothing for CG
 * or BiCGStab (Section 2.1, Table 1); the m columns are independent systems
 * that share every matrix load (Section 2.2).  Optional reduced-precision
 * preconditioner and compressed indices follow Section 2.3 ("data
 * compression": mixed precision, smaller index types in row blocks).
 *
 * Conventions for every call:
 *   - Return value: XAMG_OK (0), XAMG_NOT_CONVERGED (+1, a warning: outputs
 *     valid) or a negative error code; a detail string for the last error
 *     of the calling thread is available from xamg_last_error().  No C++
 *     exception crosses this interface.
 *   - "host" pointers are ordinary CPU memory, "device" pointers are
 *     hipMalloc'ed (e.g. PyTorch CUDA/HIP tensors) memory of the current
 *     device.  The caller owns every pointer it passes; the library copies
 *     what it keeps.
 *   - Blocks of m vectors are stored row-major n x m ("interleaved"):
 *     element (i, j) at [i*m + j], contiguous, float64.
 *   - CSR matrices: int32 row_ptr (nrows + 1, row_ptr[0] = 0, nondecreasing),
 *     int32 col (nnz, strictly increasing within a row, 0 <= col < ncols),
 *     float64 val (nnz).  Square operators must store their diagonal.
 */
#ifndef XAMG_H
#define XAMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes --------------------------------------------------------- */
#define XAMG_OK 0
#define XAMG_NOT_CONVERGED 1 /* max_iters reached; X = last iterate, stats valid */
#define XAMG_EINVAL (-1)     /* bad argument: CSR, sizes, m, NaN/Inf in B, null */
#define XAMG_ENOMEM (-2)     /* host or device allocation failed */
#define XAMG_EHIP (-3)       /* HIP runtime error (code in xamg_last_error) */
#define XAMG_ENODEV (-4)     /* no usable gfx950 device */
#define XAMG_EBREAKDOWN (-5) /* singular coarse matrix, stalled coarsening, or a
                                Krylov breakdown that persists after restart */

#define XAMG_MAX_LEVELS 64
#define XAMG_MAX_M 32 /* columns per solve: 1..32 */

/* ---- enums --------------------------------------------------------------- */
enum { XAMG_CG = 0, XAMG_BICGSTAB = 1, XAMG_MG = 2, XAMG_PBICGSTAB = 3 };
enum { XAMG_JACOBI = 0, XAMG_CHEBYSHEV = 1, XAMG_GAUSS_SEIDEL = 2 };
enum { XAMG_FP64 = 0, XAMG_MIXED = 1 };
enum { XAMG_X0_ZERO = 0, XAMG_X0_GIVEN = 1 };
enum { XAMG_OP_A = 0, XAMG_OP_P = 1, XAMG_OP_R = 2 };

/* ---- data types ---------------------------------------------------------- */
typedef struct {
    int64_t nrows, ncols, nnz;
    const int32_t *row_ptr; /* host */
    const int32_t *col;     /* host */
    const double *val;      /* host */
} xamg_csr_t;

/* A multigrid hierarchy as plain host arrays (level 0 = the system matrix).
 * P[l] is n_l x n_{l+1} (prolongation), R[l] = P[l]^T is n_{l+1} x n_l,
 * A[l+1] = R[l] A[l] P[l].  lmax[l] estimates lambda_max(D_l^-1 A_l) and is
 * used by the Chebyshev smoother only (ignored for the coarsest level). */
typedef struct {
    int32_t nlevels;       /* 1..XAMG_MAX_LEVELS */
    const xamg_csr_t *A;   /* [nlevels] */
    const xamg_csr_t *P;   /* [nlevels - 1] */
    const xamg_csr_t *R;   /* [nlevels - 1] */
    const double *lmax;    /* [nlevels] */
} xamg_hierarchy_t;

/* Setup parameters of the classical AMG hierarchy (host). */
typedef struct {
    double theta;          /* strength threshold, default 0.25 */
    int32_t max_coarse;    /* stop when a level has <= this many rows, default 64 */
    int32_t max_levels;    /* error (XAMG_EBREAKDOWN) beyond this, default 40 */
    int32_t lanczos_steps; /* steps of the lambda_max estimate, default 10 */
    int32_t agg_levels;    /* aggressive coarsening on the first agg_levels levels
                              (the paper's mg_agg_num_levels, Section 2.4): a second
                              RS pass over the C points on their distance-two
                              strength, with multipass interpolation; default 0 */
    int32_t num_paths;     /* paths of length <= 2 that make a distance-two strong
                              connection (mg_num_paths), default 1 */
} xamg_setup_params_t;

/* Solver options. */
typedef struct {
    int32_t method;        /* XAMG_CG (default), XAMG_BICGSTAB, XAMG_MG: multigrid as
                              the solver (Table 1), x <- x + V(b - A x) per column
                              until the true relative residual is <= tol, or
                              XAMG_PBICGSTAB: pipelined BiCGStab (Section 2.1;
                              Cools and Vanroose 2017), BiCGStab's iterates with
                              recurrences in which neither product with A M waits
                              for a dot product; more work vectors (16 n x m FP64
                              blocks) and more vector traffic per iteration; a
                              breakdown stops the column (no restart).  Its
                              recurrences carry images under the preconditioner,
                              which must therefore be linear: it needs
                              precision XAMG_FP64 (EINVAL with XAMG_MIXED) */
    int32_t smoother;      /* XAMG_JACOBI (default), XAMG_CHEBYSHEV or XAMG_GAUSS_SEIDEL:
                              symmetric Gauss-Seidel (Section 2.1, Table 1; the
                              smoother of Section 3.1) in its l1-hybrid form --
                              Gauss-Seidel inside blocks of gs_block consecutive
                              rows, Jacobi across blocks, diagonal a_ii plus the
                              absolute couplings to other blocks (Baker et al.,
                              SISC 2011); one forward and one backward sweep per
                              smoothing step */
    double omega;          /* Jacobi damping, default 2/3 */
    int32_t cheby_degree;  /* Chebyshev polynomial degree, 1 or 2 (default 2) */
    double cheby_lo_frac;  /* interval [lo_frac * hi, hi], default 0.3 */
    double cheby_hi_frac;  /* hi = hi_frac * lmax, default 1.1 */
    int32_t precision;     /* XAMG_FP64 (default) or XAMG_MIXED: FP32 V-cycle */
    int32_t index_bits;    /* 32 (default) or 16: compressed preconditioner indices */
    int32_t max_iters;     /* default 1000 */
    int32_t x0_mode;       /* XAMG_X0_ZERO (default) or XAMG_X0_GIVEN */
    int32_t flexible;      /* CG beta: 0 Fletcher-Reeves, 1 flexible; MIXED forces 1 */
    int32_t check_every;   /* host convergence poll: every check_every iterations, or
                              0 (default): at the iteration predicted from the decay
                              of the largest active relative residual (16 bytes
                              copied per poll) */
    int32_t gs_block;      /* Gauss-Seidel block size in rows: 4, 8 (default) or 16 */
    int32_t precond;       /* 1 (default): the AMG V-cycle preconditions the Krylov
                              method; 0: no preconditioner (M = I; Table 1 lists the
                              Krylov solvers apart from their preconditioners).
                              MG requires 1. */
    int32_t merged;        /* CG in a merged form (Section 2.1: merged formulations
                              regroup the vector updates so that fewer passes read
                              and write the vectors); the recurrences, and so the
                              iterates, are those of the standard form.  0: standard
                              (q = A p; x += alpha p, r -= alpha q; z = M r;
                              p = z + beta p); 1: x's update of an iteration is
                              applied in the next iteration's p = z + beta p pass,
                              which reads the old p anyway (one vector read less
                              per iteration); 2: that pass rides in the SpMM as
                              well -- q = A (z + beta p), with the new p written to
                              a second buffer (one pass less per iteration, one
                              more n x m FP64 block of work memory).  Default 1;
                              BiCGStab and MG ignore it. */
    void *stream;          /* hipStream_t for all work; NULL = the null stream */
} xamg_options_t;

/* Per-column solve statistics. */
typedef struct {
    int32_t iters;       /* Krylov iterations the column was active */
    int32_t converged;   /* 1 if ||b - A x|| / ||b|| <= tol */
    double relres;       /* recurrence residual norm / ||b|| at exit */
    double true_relres;  /* ||b - A x|| / ||b|| recomputed at exit (FP64) */
    int32_t restarts;    /* times the column restarted: true-residual restarts
                            (the recurrence residual passed, the recomputed one
                            did not) plus BiCGStab breakdown restarts */
    int32_t reserved;    /* 0 */
    double ms;           /* host wall time (ms) of the solve that produced the column,
                            from its first launch to its final synchronisation (the
                            same for every column of a call; a batched solve reports
                            the whole batch); excludes the autotuning and work
                            allocation of a first call */
} xamg_stats_t;

typedef struct xamg_host_hierarchy xamg_host_hierarchy_t;
typedef struct xamg_handle xamg_handle_t;

/* ---- host setup (prerequisite, not part of the timed solve) -------------- */

/* Defaults: theta 0.25, max_coarse 64, max_levels 40, lanczos_steps 10,
 * agg_levels 0, num_paths 1. */
void xamg_default_setup_params(xamg_setup_params_t *p);

/* Build the classical AMG hierarchy of A on the host (Section 2.3: the
 * multigrid setup phase, which the paper delegates to hypre's classical
 * AMG; Section 1).  A is validated (EINVAL on a malformed or non-square CSR
 * or a missing diagonal).  params may be NULL for the defaults.  On success
 * *out owns all arrays; release with xamg_hierarchy_free.  EBREAKDOWN if
 * coarsening stalls (a level keeps > 0.9 of its rows) or needs more than
 * max_levels levels. */
int xamg_hierarchy_build(const xamg_csr_t *A, const xamg_setup_params_t *params,
                         xamg_host_hierarchy_t **out);

/* Fill *view with pointers into h (valid until xamg_hierarchy_free). */
int xamg_hierarchy_view(const xamg_host_hierarchy_t *h, xamg_hierarchy_t *view);

/* Copy the C/F split of level `level` (1 = C, 2 = F, one byte per row of
 * A[level]) into cf (host, caller-allocated). */
int xamg_hierarchy_cf(const xamg_host_hierarchy_t *h, int32_t level, int8_t *cf);

void xamg_hierarchy_free(xamg_host_hierarchy_t *h);

/* ---- device solver ------------------------------------------------------- */

/* Defaults as listed in xamg_options_t. */
void xamg_default_options(xamg_options_t *o);

/* Upload a hierarchy to the current device and prepare the solver (the
 * paper's construct_solver_hierarchy, Section 2.4).  H and its arrays are
 * host memory, deep-copied; the caller may free them on return.  Computes
 * D^-1 per level, the inverse of the coarsest matrix from its LU
 * factorisation (EBREAKDOWN if singular), FP32 copies and 16-bit index
 * encodings when the options ask for them.  opt may be NULL (defaults).
 * The coarsest level may have up to 1024 rows (its inverse is applied from
 * LDS up to 64 rows, from global memory above).  EINVAL on inconsistent
 * sizes, invalid CSR or a larger coarsest level; ENODEV without a gfx950
 * device; ENOMEM when device memory runs out. */
int xamg_setup(const xamg_hierarchy_t *H, const xamg_options_t *opt,
               xamg_handle_t **out);

/* Solve A X = B for m columns (1 <= m <= XAMG_MAX_M) to relative residual
 * ||b_j - A x_j|| / ||b_j|| <= tol per column (Section 2.4: solver->solve()).
 * B (n x m, device, read-only) and X (n x m, device, in/out: the initial
 * guess when x0_mode = GIVEN, overwritten with the solution) are caller
 * memory valid for the call.  stats (host, m entries) may be NULL.  The
 * call blocks until the solve ends; all device work runs on opt.stream.
 * A zero column of B yields a zero column of X, 0 iterations, converged.
 * Returns OK, NOT_CONVERGED, EINVAL (m out of range, tol <= 0, NaN/Inf in
 * B, null pointers), EBREAKDOWN (persistent Krylov breakdown), EHIP. */
int xamg_solve(xamg_handle_t *h, const double *B, double *X, int32_t m, double tol,
               xamg_stats_t *stats);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve
 * of xamg_solve, same arguments, same kernels and results, with no device
 * allocation and no autotuning inside the call.  Its work vectors, padding
 * copies, per-column state and partial sums live in one static device array
 * of XAMG_NOALLOC_SCRATCH_BYTES per device (held until the process ends);
 * a solve that needs more returns XAMG_EINVAL (the detail string gives the
 * bytes needed: roughly (5 + 4 C_G) n m 8 bytes for FP64 CG, C_G the grid
 * complexity).  Launch shapes are those already tuned for the padded m (by
 * an earlier xamg_solve or xamg_autotune on the handle), else the tuning
 * cache's choices for its operators (see xamg_autotune; a host lookup, no
 * timing), else the setup-time row-length guess.  Calls on one device share the array: calls that
 * overlap in time on one device race and must be serialised by the caller.
 * The kernel timer is inactive during this call. */
#define XAMG_NOALLOC_SCRATCH_BYTES (128u << 20)
int xamg_solve_noalloc(xamg_handle_t *h, const double *B, double *X, int32_t m, double tol,
                       xamg_stats_t *stats);

/* Apply one V(1,1) cycle from a zero guess, X = M^-1 B (device, n x m
 * interleaved, float64), with the smoother and precision of the handle.
 * m in {1, 2, 4, 8, 16, 32}. */
int xamg_vcycle(xamg_handle_t *h, const double *B, double *X, int32_t m);

/* Y = Op X for Op = A[level] (XAMG_OP_A), P[level] or R[level], in the
 * handle's FP64 copy (device pointers, row-major interleaved float64;
 * X has ncols(Op) rows, Y nrows(Op)).  m in {1, 2, 4, 8, 16, 32}. */
int xamg_spmm(xamg_handle_t *h, int32_t op, int32_t level, int32_t m,
              const double *X, double *Y);

/* Sizes of the uploaded hierarchy: out[0] = nlevels, then per level l
 * out[1 + 3l .. 3 + 3l] = n_l, nnz(A_l), nnz(P_l) (0 for the coarsest).
 * `cap` is the length of out; returns EINVAL if too short. */
int xamg_info(const xamg_handle_t *h, int64_t *out, int32_t cap);

/* Fraction of the nonzeros of A[level], P[level], R[level] (out[0..2],
 * host) stored with 16-bit column offsets in the reduced-precision copy;
 * 0 when the handle keeps 32-bit indices.  EINVAL for the coarsest level. */
int xamg_index16_fraction(const xamg_handle_t *h, int32_t level, double *out);

/* ---- batched uneven systems -------------------------------------------- */
typedef struct xamg_batch xamg_batch_t;

/* Group nsys CG handles (each with its own hierarchy, size and options)
 * for batched solves.  The handles stay owned by the caller and must
 * outlive the batch; a handle may appear once.  iters_per_launch (0 = 4) is
 * the number of CG iterations of every system in the batch's follow-up HIP
 * graph (see xamg_solve_batched).  EINVAL for handles whose method is not
 * CG, or repeated handles. */
int xamg_batch_create(xamg_handle_t *const *handles, int32_t nsys, int32_t iters_per_launch,
                      xamg_batch_t **out);

/* Solve all systems of the batch: B[s], X[s] (device, n_s x m[s], as in
 * xamg_solve), stats[s] (host, m[s] entries, or NULL / stats NULL).  The
 * iterations of every system run from captured HIP graphs (one branch per
 * system): the first launch runs as many iterations as the batch's previous
 * solve needed, so a repeated solve is normally one graph launch; then the
 * host reads 16 bytes per system, and graphs of iters_per_launch iterations
 * follow until each system has converged or reached its max_iters.
 * Converged systems' kernels exit immediately.  The true-residual checks of
 * all finished systems are enqueued together and waited for once.
 * Per-system results equal those of xamg_solve on the same handle.  Return:
 * the worst of the systems' codes (EBREAKDOWN, NOT_CONVERGED, OK); EINVAL
 * as xamg_solve. */
int xamg_solve_batched(xamg_batch_t *b, const double *const *B, double *const *X,
                       const int32_t *m, double tol, xamg_stats_t *const *stats);

int xamg_batch_destroy(xamg_batch_t *b);

/* Autotuner (Section 2.2's kernels, tuned for this device): for each
 * operator A_l, P_l, R_l of the copy the V-cycle uses (A_l twice: on the
 * residual pass and on the pre-smoothing pass, which gathers b against
 * A D^-1) and the Krylov operator, time the pass for m columns with 1, 2, 4
 * and 8 lane groups splitting a row's nonzeros, each with one block per
 * tile of rows or with a sweeping launch (at most 2048 blocks and no more
 * than the device holds at once, taking the tiles in block order); then,
 * one at a time on top of the fastest, the 32-bit indices of a 16-bit
 * encoded operator, twice the columns per lane, and 512-thread blocks, and
 * last the banded XCD walk with three segment lengths; a change is kept
 * when it is more than 3% faster.  Timed with HIP events on
 * the solver's stream.  Runs by itself
 * on the first solve for each padded m.  The choices are kept for the
 * process in a tuning cache per device, keyed by the operator's shape and
 * storage (rows, columns, nonzeros, stored row length, bandwidth, value and
 * index width), the pass, the pre-smoothing variant and m: a handle whose
 * operator matches a cached key takes that choice without timing, so equal
 * problems run on equal launch shapes and give bit-identical results.  This
 * call re-runs the tuning now, timing every choice afresh and replacing the
 * cached ones (enable = 1), or switches automatic tuning off (enable = 0;
 * the setup-time row-length heuristic stays in use).  m in {1, 2, 4, 8, 16,
 * 32}. */
int xamg_autotune(xamg_handle_t *h, int32_t m, int32_t enable);

/* Row splits in use for m columns: out[4l .. 4l+3] = split of A_l (the
 * residual and post-smoothing passes), of A_l's pre-smoothing pass (with
 * the Gauss-Seidel smoother: of its sweeps, lane groups per block of rows),
 * of P_l and of R_l (0 where the operator or pass does not exist): the lane
 * groups per row (1, 2, 4, 8) plus the flags 16 (a sweeping launch: no more
 * blocks than the device holds at once, each taking every gridDim-th tile),
 * 32 (blocks of 512 threads instead of 256: tiles of twice the rows), 64
 * (the operator's 32-bit column indices although it has 16-bit offsets),
 * 128 (twice the columns per lane: 32 instead of 16 bytes of a row's
 * columns per gathered nonzero) and 256 / 512 / 768 (the banded XCD walk:
 * the tiles cut into segments of one, a half or a quarter of the
 * operator's bandwidth, each segment into 8 chunks, the blocks of XCD k
 * taking chunk k of every segment in order); then out[4 nlevels] = the split of the Krylov operator, the FP64
 * copy of A_0 (a mixed-precision handle tunes it apart from the FP32 A_0 of
 * its V-cycle).  cap >= 4 * nlevels + 1. */
int xamg_tuning(const xamg_handle_t *h, int32_t m, int32_t *out, int32_t cap);

/* Set the row splits for m columns: the inverse of xamg_tuning, same layout
 * (in[4l .. 4l+3] for A_l, A_l's pre-smoothing pass, P_l and R_l; entries
 * 1..3 of the coarsest level are ignored), applied to the FP64 and the FP32
 * copies, and in[4 nlevels] to the FP64 A_0 of the Krylov method.  Each value
 * is 1, 2, 4 or 8 lane groups per row plus any of the flags 16, 32, 64, 128,
 * 256, 512, 768 (see xamg_tuning; a flag that does not apply, such as 128 where the row's
 * columns do not fill twice the lanes, is ignored); a split wider than a wavefront allows for m (lanes per
 * row x groups > 64) runs with the widest that fits.  Marks m as tuned, so
 * the values stay until xamg_autotune(h, m, 1).  For callers that tune
 * offline, and for tests that force every launch shape.  count >= 4 *
 * nlevels + 1.  Returns OK or EINVAL (null pointer, m, count or a value out of
 * range); the handle is unchanged on error. */
int xamg_set_tuning(xamg_handle_t *h, int32_t m, const int32_t *in, int32_t count);

/* Kernel timer: while enabled, every launch of the selected kernel during
 * xamg_solve is bracketed by HIP events on the solver's stream, and
 * xamg_timer_read returns the summed event time (ms) and the launch count
 * since the last enable.  kind: XAMG_TIMER_OFF, XAMG_TIMER_KRYLOV_SPMM (the
 * finest-level q = A p of CG with its fused (p, q) dot), XAMG_TIMER_PRESMOOTH
 * (the finest-level pre-smoothing pass from a zero guess).  For measurement
 * only; it adds two event records per timed launch. */
enum { XAMG_TIMER_OFF = 0, XAMG_TIMER_KRYLOV_SPMM = 1, XAMG_TIMER_PRESMOOTH = 2 };
int xamg_timer_enable(xamg_handle_t *h, int32_t kind);
int xamg_timer_read(xamg_handle_t *h, double *ms, int64_t *count);

/* Release every device and host resource of h (NULL is allowed). */
int xamg_destroy(xamg_handle_t *h);

/* ---- learned warm start ------------------------------------------------- *
 * The solve accepts an initial guess (Section 2.4 lists one as an optional
 * input beside the matrix and the right-hand side; x0_mode = XAMG_X0_GIVEN).
 * The network that produces one is an extension of this library, not part
 * of the paper's method.  These calls produce X0 from B with a
 * small bias-free 3D CNN on an N x N x N grid (row r = x + N y + N^2 z):
 * four 3x3x3 zero-padded convolutions, channels 1 -> 16 -> 16 -> 16 -> 1,
 * ReLU after the first three.  Weights and activations BF16 (round to
 * nearest even), accumulation FP32, master weights FP32.  Weights are one
 * flat FP32 array of XAMG_CNN_PARAMS values: W1 [16][1][27], W2 [16][16][27],
 * W3 [16][16][27], W4 [1][16][27] ([out][in][tap], tap t = (dz+1) 9 +
 * (dy+1) 3 + (dx+1) for neighbour offset (dx, dy, dz)).  Activations are
 * channels-last, BF16 stored as uint16: a[r * C + c].
 * All data pointers are device pointers unless stated otherwise. */
typedef struct xamg_cnn xamg_cnn_t;
#define XAMG_CNN_PARAMS 14688

/* Create a network for grid side N (a multiple of 16, 16..1024) with initial
 * weights w_init (host, XAMG_CNN_PARAMS floats).  stream: hipStream_t or
 * NULL.  Adam moments start at zero.  EINVAL for a bad N; ENOMEM/EHIP. */
int xamg_cnn_create(int32_t N, const float *w_init, void *stream, xamg_cnn_t **out);

/* Copy the FP32 master weights out / in (host arrays of XAMG_CNN_PARAMS). */
int xamg_cnn_get_weights(xamg_cnn_t *h, float *w_host);
int xamg_cnn_set_weights(xamg_cnn_t *h, const float *w_host);

/* Forward over S normalised samples x (S x n FP32, sample-major), writing
 * y_out (S x n FP32) unless NULL.  With targets t (S x n FP32) it also
 * back-propagates: the weight gradients of the mean relative squared error
 * L = (1/S) sum_s ||f(x_s) - t_s||^2 / ||t_s||^2 replace the gradient buffer
 * and *loss (host, may be NULL) receives L.  Activations and their
 * gradients are BF16; dL/dy and weight gradients FP32. */
int xamg_cnn_pass(xamg_cnn_t *h, const float *x, const float *t, int32_t S, float *y_out,
                  double *loss);

/* As xamg_cnn_pass with targets, but with the residual loss: the network's
 * output judged as a solver's initial guess, L = (1/S) sum_s ||x_s - A
 * f(x_s)||^2 / ||x_s||^2 with A the finest-level operator of `solver`
 * (same grid, n = N^3; symmetric, as CG's operator is: the gradient
 * dL/dy = -2 A (x - A y) / (||x||^2 S) uses A for A^T).  This is the
 * quantity xamg_warmstart's fallback judges; no solved targets are needed.
 * r = x - A y is formed with FP64 products and stored FP32.  EINVAL for a
 * null argument or a solver of another size. */
int xamg_cnn_pass_residual(xamg_cnn_t *h, xamg_handle_t *solver, const float *x, int32_t S,
                           double *loss);

/* Weight gradients of the last pass (host, XAMG_CNN_PARAMS floats). */
int xamg_cnn_get_grads(xamg_cnn_t *h, float *g_host);

/* One Adam step on the master weights with the last pass's gradients
 * (bias-corrected moments; lr > 0).  The BF16 copies are refreshed. */
int xamg_cnn_adam(xamg_cnn_t *h, float lr, float beta1, float beta2, float eps);

/* One layer alone (1..4), for checking against a reference.  mode 0:
 * forward of `in` (layer 1: n x 1 BF16; 2, 3: n x 16 BF16; 4: n x 16 BF16)
 * into `out` (layers 1-3: n x 16 BF16 after ReLU; layer 4: n FP32).
 * mode 1 (layers 2..4): input gradient of the gradient `in` at the layer's
 * output (layer 4: n FP32; 2, 3: n x 16 BF16), times (mask > 0) with `mask`
 * the layer's input activation, into `out` (n x 16 BF16).  mode 2: weight
 * gradient from `in` (gradient at the output, as in mode 1) and `mask` (the
 * layer's input activation); the result replaces the gradient buffer
 * (read with xamg_cnn_get_grads; other layers' entries are zero).
 * `in`, `mask` and `out` must be 16-byte aligned (XAMG_EINVAL otherwise). */
int xamg_cnn_layer(xamg_cnn_t *h, int32_t layer, int32_t mode, const void *in, const void *mask,
                   void *out);

/* X0 (n x m, interleaved as in xamg_solve) from B: column j is s_j f(b_j /
 * s_j) with s_j = ||b_j|| / sqrt(n) (a zero column gives zero).  With a
 * solver handle of the same n, every column whose initial residual
 * ||b_j - A x0_j|| is not below ||b_j|| is reset to zero and fallback[j]
 * (host, m entries, may be NULL) is 1, else 0.  1 <= m <= XAMG_MAX_M. */
int xamg_warmstart(xamg_cnn_t *h, xamg_handle_t *solver, const double *B, double *X0, int32_t m,
                   int32_t *fallback);

/* Kernel timer of the network (measurement only): while enabled, every
 * launch of the selected kernel is bracketed by HIP events on the network's
 * stream; xamg_cnn_timer_read returns the summed time (ms) and the launch
 * count since the last enable.  kind: XAMG_CNN_TIMER_OFF,
 * XAMG_CNN_TIMER_CONV16 (the MFMA 16 -> 16 forward convolutions),
 * XAMG_CNN_TIMER_WGRAD16 (the 16 x 16 weight-gradient reductions). */
enum { XAMG_CNN_TIMER_OFF = 0, XAMG_CNN_TIMER_CONV16 = 1, XAMG_CNN_TIMER_WGRAD16 = 2 };
int xamg_cnn_timer_enable(xamg_cnn_t *h, int32_t kind);
int xamg_cnn_timer_read(xamg_cnn_t *h, double *ms, int64_t *count);

int xamg_cnn_destroy(xamg_cnn_t *h);

/* Static description of a return code. */
const char *xamg_strerror(int code);

/* Detail of the last error on the calling thread ("" if none). */
const char *xamg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* XAMG_H */
