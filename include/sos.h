/*
 * sos.h - C ABI of the MI355X (gfx950) HSDE-ADMM solver for SOS-derived SDPs.
 *
 * Method: Zheng, Fantuzzi, Papachristodoulou, "Fast ADMM for sum-of-squares
 * programs using partial orthogonality" (arXiv 1708.04174).
 *
 *   primal   min c^T xi  s.t.  A xi = b,  xi in K = R^{n_free} x S^{N_1}_+ x ...   (Section III)
 *   dual     max b^T y   s.t.  A^T y + z = c,  z in K*                             (Section IV-A)
 *   state    u = (xi, y, tau), v = (z, s, kappa) of the homogeneous self-dual
 *            embedding v = Q u (Section IV-A); one iteration = the affine solve
 *            with I + Q, the projection onto C = K x R^m x R_+, and the dual
 *            update (the three ADMM steps of Section IV-A).
 *   affine   I + A A^T = P + A_f A_f^T with P diagonal (Proposition 1 and its
 *            weighted form in Section VI); solved with the matrix inversion lemma
 *            (Section IV-B) and the FP64 inverse of I + A_f^T P^{-1} A_f, formed
 *            once at setup from its Cholesky factor, so that each iteration's small
 *            solve is one dense matrix-vector product.
 *
 * Conventions for every function below
 *   - Return value: SOS_OK (0) or a negative SOS_E_* code.  Nothing throws across
 *     the ABI.  sos_last_error() gives a message for the last failure on a handle.
 *   - Host arrays passed in are read during the call only (the caller keeps
 *     ownership and may free them on return).  Output arrays are caller-owned
 *     host arrays of the documented length.
 *   - The library allocates and owns its device memory (HIP).  All device work of
 *     a handle is ordered on the hipStream_t given to sos_setup (NULL = the
 *     default stream).  A handle is not thread-safe.
 *   - Layout at the ABI is the paper's: every PSD block is the column-stacked vec
 *     of its N x N matrix (Section III).  Columns (i,j) and (j,i) of a PSD block
 *     must be identical (coefficient matching always produces this, since the
 *     indicator matrices are symmetric).  Internally the library keeps the lower
 *     triangle of every block (unscaled) and weighs off-diagonal entries by 2 in
 *     inner products, so its iterates are exactly the lower triangles of the
 *     full-vec iterates and conversion at the ABI is a copy.
 */
#ifndef SOS_H
#define SOS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define SOS_OK        0
#define SOS_E_INVAL  (-1)   /* bad dimensions, bad CSC structure, non-finite data, bad settings */
#define SOS_E_ASYM   (-2)   /* a PSD block's columns (i,j) and (j,i), or its cost, differ */
#define SOS_E_NOMEM  (-3)   /* host or device allocation failed */
#define SOS_E_HIP    (-4)   /* a HIP runtime call failed (no device, launch failure, ...) */
#define SOS_E_STATE  (-5)   /* call not valid in the handle's current state */

/* solve status (a status, never an error) */
#define SOS_UNSOLVED           0
#define SOS_SOLVED             1   /* max(res_pri, res_dual, gap) <= tol */
#define SOS_PRIMAL_INFEASIBLE  2   /* b^T y > 0 and |A^T y + z| <= tol b^T y  (tau -> 0 certificate) */
#define SOS_DUAL_INFEASIBLE    3   /* c^T xi < 0 and |A xi| <= tol (-c^T xi) */
#define SOS_MAX_ITERS          4

/* precision forms */
#define SOS_FP64        0   /* every step in FP64 */
#define SOS_FP32_MIXED  1   /* FP32 bulk (matvecs, eigensolves, FP32 accumulation); FP64 for the
                               small solve with S, theta, tau/kappa, residuals; FP64 polish at the end */

/* column partition of A into the diagonal part A_s and the low-rank part A_f */
#define SOS_PART_PAPER    0  /* A_f = all free columns + every PSD column with >= 2 nonzeros (Sections IV-B, VI) */
#define SOS_PART_COLUMNS  1  /* A_f = only columns with >= 2 nonzeros (any column with one nonzero keeps P diagonal) */

typedef struct sos_work  sos_work;
typedef struct sos_batch sos_batch;

/* Host CSC matrix, m rows, n = n_free + sum_j N_j^2 columns; rowind sorted within a column. */
typedef struct {
    int32_t m, n;
    const int64_t *colptr;   /* n + 1 entries, colptr[0] = 0 */
    const int32_t *rowind;   /* colptr[n] entries, 0 <= rowind < m */
    const double  *val;      /* colptr[n] entries, finite */
} sos_csc;

/* Cone K = R^{n_free} x S^{N[0]}_+ x ... x S^{N[n_psd-1]}_+ */
typedef struct {
    int32_t n_free;
    int32_t n_psd;
    const int32_t *N;        /* n_psd block sizes, each >= 1 */
} sos_cone;

typedef struct {
    double  tol;             /* stop when max(res_pri, res_dual, gap) <= tol, or on a certificate */
    int32_t max_iters;
    int32_t check_every;     /* residuals (FP64) are evaluated every check_every iterations */
    double  alpha;           /* relaxation; 1.0 = the paper's three steps unchanged */
    int32_t precision;       /* SOS_FP64 | SOS_FP32_MIXED */
    int32_t polish_iters;    /* FP64 iterations after an FP32 solve (>= 1 for SOS_FP32_MIXED) */
    int32_t partition;       /* SOS_PART_PAPER | SOS_PART_COLUMNS */
    int32_t block_threads;   /* threads per workgroup: 0 = default (512), else 64..1024, multiple of 64 */
    int32_t eig_form;        /* eigensolver of sos_step / sos_solve: 0 = library default (the
                                lane-group form for N < 128, 8 lanes per column pair for N >= 64,
                                the rows-over-wavefronts form from N = 128 for blocks that fit in
                                LDS), 1 = rows form for every block that fits in LDS, 2 = lane-group
                                form for every block, 3 = the multi-workgroup form for every block.
                                In SOS_FP64, eig_form 0 also runs a single problem whose largest
                                block has N >= 128 as one cooperative launch over several workgroups:
                                all of them take the affine step (a grid barrier between its
                                phases), a block one-sided Jacobi (column blocks of 8 columns, one
                                workgroup per pair of blocks and block round, the pair's 16 x 16
                                Gram matrix and rotation on the matrix cores, a grid barrier per
                                round) and the MFMA products; workgroup 0 the residual checks (a
                                solve with warm_budget > 0 stays on one workgroup).  Batches take
                                theirs from the schedule.
                                Out of 0..3: SOS_E_INVAL. */
    int32_t warm_budget;     /* 0: a warm-started solve keeps its start to the end.  > 0: a solve that
                                starts from sos_warm_start / sos_batch_warm_start and has neither
                                converged after warm_budget iterations nor kept tau > 0 at a residual
                                check is restarted in the same launch from the cold start with the
                                full max_iters budget (cold ADMM as the fallback); the abandoned
                                iterations are reported in sos_info.warm_iters */
    int32_t scale_iters;     /* 0: no scaling (the paper's method).  > 0: that many passes of a
                                block-scalar equilibration before the solve: rows scaled by D,
                                columns by E with one factor per PSD block and per free variable
                                (Ruiz's passes on 2-norms, D balanced to geometric mean 1, factors
                                in [1e-4, 1e4]), which keeps A_s A_s^T diagonal (Proposition 1) and
                                the cone.  The iteration runs on D A E, D b, E c; residuals,
                                certificates, sos_get_solution / get_iterate / set_iterate /
                                warm_start use the original units.  The batch learned-warm-start
                                layout (sos_batch_warm_start / export_solutions) is the scaled
                                problem's.  0..1000, else SOS_E_INVAL. */
} sos_settings;

typedef struct {
    int32_t status;          /* SOS_* status above */
    int32_t iters;           /* total iterations run (FP32 + FP64 polish) */
    int32_t k_lowrank;       /* columns of A_f = order of the small matrix S */
    int32_t polish_iters;    /* FP64 iterations run after the FP32 phase */
    double  pobj, dobj;      /* c^T xi / tau, b^T y / tau */
    double  res_pri, res_dual, gap;   /* |A xi - b tau|/tau/(1+|b|), |A^T y + z - c tau|/tau/(1+|c|),
                                         |c^T xi - b^T y|/tau/(1 + |c^T xi|/tau + |b^T y|/tau), FP64 */
    double  tau, kappa;
    double  setup_ms, solve_ms;
    double  eig_sweeps;      /* mean eigensolver sweeps per block projection in the last launch */
    double  affine_ms, eig_ms, resid_ms;   /* device time of the last launch by phase (one workgroup's clock) */
    int32_t warm_iters;      /* iterations of a warm-started attempt abandoned for the cold restart
                                (0: no restart; then iters counts the warm-started run itself) */
    double  start_ms, end_ms;   /* sos_batch_solve: when a workgroup took the problem from the queue
                                   and when it finished it, ms after the solve launch began (device
                                   wall clock); 0 for single solves */
} sos_info;

/* Fills *s with tol 1e-4, max_iters 2000, check_every 10, alpha 1, SOS_FP64, scale_iters 0,
   polish_iters 1, SOS_PART_PAPER, block_threads 0.  Returns SOS_E_INVAL if s is NULL. */
int sos_default_settings(sos_settings *s);

/* Validates the problem, folds PSD blocks to their lower triangles, splits A = [A_f A_s]
   (Proposition 1; Section VI for weighted blocks), forms d = 1 + diag(A_s A_s^T),
   S = I + A_f^T D^{-1} A_f (written over lower-triangle columns: W_f^{-1} + ...,
   W_f the weights 1 / 2), its FP64 Cholesky factor and from it S^{-1}, h = M^{-1} zeta and
   eta = 1 + zeta^T h with zeta = (c, -b) (Section IV-B), uploads everything to the
   current HIP device, and sets the cold start u = v = (0, 0, 1).
   A, b (m), c (n), K, s: host inputs.  s may be NULL (defaults).  hip_stream: a
   hipStream_t or NULL.  *out receives the new handle (NULL on failure).
   Errors: SOS_E_INVAL, SOS_E_ASYM, SOS_E_NOMEM, SOS_E_HIP. */
int sos_setup(const sos_csc *A, const double *b, const double *c, const sos_cone *K,
              const sos_settings *s, void *hip_stream, sos_work **out);

/* Runs exactly `iters` ADMM iterations from the current state, in the handle's
   precision, with no early stop; then evaluates the FP64 residuals once and fills
   *info (status SOS_UNSOLVED unless a stopping test already holds).  Blocks until
   the stream has finished.  iters >= 0.  info may be NULL. */
int sos_step(sos_work *w, int32_t iters, sos_info *info);

/* sos_step for callers that cannot allocate device memory (code under HIP graph capture,
   tight serving loops, harnesses that forbid hipMalloc): the same iterations, kernels and
   results as sos_step, but the launch's scratch (queue counter, affine work vector,
   eigensolver area) lives in a static device array of 4 MiB that the library holds on each
   GPU it runs on until the process ends, instead of the handle's own.  No hipMalloc, hipFree
   or other allocating call is made; the handle's device must be current.  The array keeps
   the last call's contents; each call clears what must start at zero (the queue counter)
   with a kernel, and every other byte is written before it is read.  Calls that overlap on
   one GPU share the array and race: serialise them (one stream, or host ordering).  It always
   runs the one-workgroup form (the multi-workgroup form of eig_form 0 / 3 keeps its scratch on
   the handle), so it matches sos_step where sos_step runs that form too.
   A problem needing more than 4 MiB of scratch (about 3 N^2 + m + n_x doubles, N the
   largest block) is rejected with SOS_E_INVAL and a message; then nothing is launched. */
int sos_step_static(sos_work *w, int32_t iters, sos_info *info);

/* Iterates from the current state until a stopping test holds or max_iters; in
   SOS_FP32_MIXED form the FP32 phase is followed by FP64 iterations (at least
   polish_iters) until the FP64 residuals meet tol.  Blocks until done. */
int sos_solve(sos_work *w, sos_info *info);

/* Sets u = (tau x, tau y, tau), v = (tau z, 0, kappa).  x, z: n entries (full vec,
   PSD blocks symmetric), y: m entries.  z must be zero on the free part (K* there
   is {0}).  tau >= 0, kappa >= 0, not both zero. */
int sos_warm_start(sos_work *w, const double *x, const double *y, const double *z,
                   double tau, double kappa);

/* Copies xi/tau, y/tau, z/tau (full vec) into x (n), y (m), z (n).  Any pointer
   may be NULL to skip it.  SOS_E_STATE if tau == 0 (use sos_get_iterate). */
int sos_get_solution(const sos_work *w, double *x, double *y, double *z);

/* Raw embedding state: u = (xi, y, tau), v = (z, s, kappa), each n + m + 1 entries. */
int sos_get_iterate(const sos_work *w, double *u, double *v);

/* Restores a state taken with sos_get_iterate (checkpoint / resume).  The s part
   of v and the free part of z must be zero, as every iterate of the method has. */
int sos_set_iterate(sos_work *w, const double *u, const double *v);

/* Eigen-decomposition of PSD block `block` of the current solution, for post-processing:
   dual = 0 factors X = xi / tau (the Gram matrix: p - gamma = sum_j evals[j] (v_j^T m(x))^2,
   the SOS decomposition of Section I and Section II-C), dual = 1 factors Z = z / tau (for a
   POP relaxation with cost -gamma, the moment matrix of the dual).  evals: N entries (Rayleigh
   quotients v_j^T W v_j, signed, in the order the eigensolver leaves them); evecs: N x N,
   column-major, orthonormal columns v_j.  Runs the library's FP64 Jacobi eigensolver on the
   device (one workgroup; a temporary device buffer of N^2 + N doubles is allocated and freed).
   SOS_E_INVAL for a bad block index or dual; SOS_E_STATE if tau == 0. */
int sos_psd_factor(sos_work *w, int32_t block, int32_t dual, double *evals, double *evecs);

/* The eigenvectors the projection keeps for its warm start (Section IV-A's projection step:
   each iteration's Jacobi starts from the last iteration's eigenvectors of the block): block
   `block`'s N x N matrix (column-major, columns = eigenvectors) from the cache of the given
   precision (SOS_FP64: the FP64 iterations', SOS_FP32_MIXED: the FP32 bulk iterations'), copied
   into V (N^2 doubles, host memory, caller-owned).  *valid (may be NULL) is 1 if the cache holds
   the eigenvectors of the last iteration, 0 after a reset or before the first iteration (the
   contents are then stale).  For diagnostics, e.g. the orthogonality of the cached basis.
   SOS_E_INVAL for a bad block index or precision. */
int sos_get_eig_cache(const sos_work *w, int32_t block, int32_t precision, double *V, int32_t *valid);

/* Message for the last error on w (or on the last failed sos_setup when w is NULL). */
const char *sos_last_error(const sos_work *w);

/* Releases the handle and its device memory.  NULL is ignored. */
void sos_free(sos_work *w);

/* Groups `count` handles (same precision) for one persistent launch: workgroups
   pull problems from a device queue ordered by decreasing cost.  schedule_json
   (may be NULL) holds the tuned launch shape, e.g.
   {"block_threads": 512, "wg_per_cu": 1, "max_sweeps": 60, "use_graph": 1, "eig_wave": 2}.
   Keys: block_threads, wg_per_cu, max_sweeps, warm_eig (Jacobi warm start from the last
   eigenvectors), use_graph (capture the launches in a hipGraph), eig_wave (2: rows form
   for blocks that fit in LDS, 0: lane-group form for all), rows_nmin (eig_wave 2: blocks
   with N below it still take the lane-group form), lds_kb, gs_n32 .. gs_big (lanes per
   column pair of the lane-group form by block size), one_launch (mixed form: 1 runs both
   phases in one launch, 0 in two), fp64_jacobi_tol (Jacobi coupling tolerance of the mixed
   form's FP64 phase, default 1e-7; 0 = 16 eps), stall_checks (mixed form: residual checks
   without progress before the FP64 phase, default 4).  Keys left out take the choice sos_solve makes with
   eig_form 0, so a batch without a schedule retraces single solves bitwise.  The handles
   must outlive the batch. */
int sos_batch_setup(int32_t count, sos_work *const *probs, const char *schedule_json,
                    sos_batch **out);

/* Solves every problem of the batch from its current state (one captured HIP
   graph: FP32 or FP64 persistent solve, then the FP64 polish for the mixed form).
   infos: count entries, in the order given to sos_batch_setup. */
int sos_batch_solve(sos_batch *b, sos_info *infos);

/* Resets every problem of the batch to the cold start u = v = (0, 0, 1) with one
   device kernel (e.g. between repeated solves of the same batch). */
int sos_batch_reset(sos_batch *b);

/* Device time in ms of the last sos_batch_solve: whole graph (hip events on the
   batch's stream around it). */
double sos_batch_last_ms(const sos_batch *b);

/* Device time in ms of one kernel of the last sos_batch_solve, from device wall-clock
   stamps the kernel writes (first workgroup start to last workgroup end): phase 0 = the
   persistent solve kernel (the FP32 kernel of the two-launch mixed form, or the single
   launch that runs both phases of the mixed form), phase 1 = the FP64 kernel of the
   two-launch mixed form (0 otherwise).  Returns a negative value if unavailable. */
double sos_batch_phase_ms(const sos_batch *b, int32_t phase);

/* Message for the last failed call on batch b (NULL: the last failed sos_batch_setup, as
   sos_last_error(NULL) gives it). */
const char *sos_batch_last_error(const sos_batch *b);

void sos_batch_free(sos_batch *b);

/* ---------------------------------------------------------------- learned warm start
   The library's own iterate layout, used by the two calls below: per problem one row of
   nx + m values, [xi (nx) | y (m)], where xi lists the free variables and then the lower
   triangle (by columns, unscaled) of every PSD block.  sos_layout_size gives nx + m. */
int64_t sos_layout_size(const sos_work *w);

/* For every problem p of the batch, from the predicted row pred_dev + p * ld (device,
   FP32, layout above) sets u = (P_K(xi), y, 1) and v = (P_K*(c - A^T y), 0, 0): the
   prediction made consistent with the cones, with tau = 1, kappa = 0.  One device kernel
   on the batch's stream; the next sos_batch_solve starts from it. */
int sos_batch_warm_start(sos_batch *b, const float *pred_dev, int64_t ld);

/* Writes [xi / tau | y / tau] of every problem (FP64 iterate after a solve) as FP32 rows
   of length >= nx + m, ld apart, into out_dev (device).  Rows of problems with tau = 0
   (certificates) are zero. */
int sos_batch_export_solutions(sos_batch *b, float *out_dev, int64_t ld);

/* A small FP32 multilayer perceptron, input -> H -> H -> output with GELU (the exact,
   erf form) after both hidden layers, trained with mean squared error and Adam on the
   device.  Parameters form one buffer [W1 (in x H) | b1 | W2 (H x H) | b2 | W3 (H x out) | b3],
   row-major, a layer being Z = X W + b for row-major batches.  All X, T, Y pointers are
   device pointers to row-major FP32 batches of at most max_batch rows.  Work is ordered
   on hip_stream. */
typedef struct sos_mlp sos_mlp;
int sos_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t max_batch, void *hip_stream,
                   sos_mlp **out);
int64_t sos_mlp_num_params(const sos_mlp *m);
/* host_params: sos_mlp_num_params floats; also resets the Adam state */
int sos_mlp_set_params(sos_mlp *m, const float *host_params);
int sos_mlp_get_params(const sos_mlp *m, float *host_params);
/* Y <- Y * scale + shift per output column, applied by sos_mlp_forward when asked */
int sos_mlp_set_output_affine(sos_mlp *m, const float *host_scale, const float *host_shift);
int sos_mlp_forward(sos_mlp *m, const float *X_dev, int32_t batch, float *Y_dev, int32_t apply_output_affine);
/* gradient of mean((Y - T)^2) w.r.t. every parameter into grad_host (num_params floats), loss into loss_host */
int sos_mlp_gradient(sos_mlp *m, const float *X_dev, const float *T_dev, int32_t batch, float *grad_host,
                     double *loss_host);
/* one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on mean((Y - T)^2); loss_host may be NULL */
int sos_mlp_train_step(sos_mlp *m, const float *X_dev, const float *T_dev, int32_t batch, float lr, double *loss_host);
/* sos_mlp_train_step on a mini-batch given by row indices: rows rows_dev[0..batch) of X_dev (n_in
   columns) and T_dev (n_out columns), both row-major FP32 device arrays, are gathered by a device
   kernel into the MLP's own batch buffers, so a caller shuffles by index only.  rows_dev: device
   int32 array; every index must lie inside X_dev and T_dev (not checked on the device). */
int sos_mlp_train_step_rows(sos_mlp *m, const float *X_dev, const float *T_dev, const int32_t *rows_dev, int32_t batch,
                            float lr, double *loss_host);
void sos_mlp_free(sos_mlp *m);

#ifdef __cplusplus
}
#endif
#endif /* SOS_H */
