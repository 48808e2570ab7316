// Internal layout shared by the host library and the gfx950 kernels.
//
// One problem on the device (all arrays device-resident):
//   xi = [ free variables (n_free) | block 0 lower | block 1 lower | ... ]   length nx
// where "lower" is the lower triangle of the block, by columns, UNSCALED: entry
// (i,j), i >= j, holds X_ij.  The full column-stacked vec of the paper counts every
// off-diagonal entry twice, so inner products and norms over xi carry the weight
// wgt = 2 off the diagonal (1 on it and on free variables), and the row gather
// A xi uses A's value times that weight.  Iterates therefore equal the lower
// triangles of the paper's full-vec iterates, and conversion at the ABI is a copy.
//   u  = [ xi | y (m) ]  (tau kept in FP64 in tk[0])
//   v  = [ z  ]          (s is identically zero for every iterate, kappa in tk[1])
// A = [A_f A_s]: A_s columns have at most one nonzero, so A_s A_s^T is diagonal
// (Proposition 1); A_f holds the free columns and every column with two or more
// nonzeros (weighted blocks, Section VI).
#pragma once
#include <stdint.h>

#define SOS_MAX_BLOCKS 64
#define SOS_KMAX_LDS 1024   // largest A_f width whose k-vector is kept in LDS; wider ones use the
                            // tail of the work area (sos_work_tail_doubles)
// doubles past the affine work vectors that a problem with an A_f of width k needs (0 if the
// k-vector and the small solve's partial sums fit in LDS)
static inline long long sos_work_tail_doubles(int k) {
    if (k <= SOS_KMAX_LDS) return 0;
    const long long kp = ((long long)k + 63) & ~63LL;
    return kp + (kp > 1024 ? kp : 1024);
}
// bytes of the per-device static scratch used by sos_step_static (queue counter, affine work
// vector and eigensolver area of one workgroup)
#define SOS_STATIC_SCRATCH_BYTES (4 << 20)

struct ProbDesc {
    int m, nx, nfree, k, nblk, nmax;
    int blk_N[SOS_MAX_BLOCKS];
    int blk_off[SOS_MAX_BLOCKS];      // svec offset of each PSD block inside xi

    // all of A in CSR over the lower-triangle columns, values already times wgt
    const int *rowptr, *colidx;
    const double *val64; const float *val32;
    // per column: row of its single nonzero (A_s), -1 if empty, -2-j for A_f column j (unscaled values)
    const int *colrow;
    const double *colval64; const float *colval32;
    // A_f in CSC (k columns) and CSR (rows -> A_f column index)
    const int *fptr, *frow;
    const int *fcol;                 // A_f column j is internal column fcol[j]
    const double *fval64; const float *fval32;
    const int *frptr, *frcol;
    const double *frval64; const float *frval32;
    // 1/d, d = 1 + diag(A_s A_s^T)
    const double *dinv64; const float *dinv32;
    // S^{-1}, S = W_f^{-1} + A_f^T D^{-1} A_f (W_f = wgt on the A_f columns): k x k,
    // symmetric, formed in FP64 from the Cholesky factor of S at setup
    const double *Sinv;
    // h = M^{-1} zeta (nx + m), b (m), c (nx), cw = wgt * c (nx), wgt (nx)
    const double *h64; const float *h32;
    const double *b64; const float *b32;
    const double *c64; const float *c32;
    const double *cw64; const float *cw32;
    const double *wgt64;
    // equilibrated problems: 1 / D per row and 1 / E per column, so that residuals and
    // certificates are measured in the original units (null: no equilibration)
    const double *rsc64, *csc64;
    double eta, nb, nc;

    // iterate
    double *u64, *v64;
    float  *u32, *v32;
    double *tk;          // [0] tau, [1] kappa, [2] 1 if vs holds eigenvectors of the last iteration,
                         // [3] 1 while the iterate is a warm start not yet judged
    double *vs64;        // per PSD block, its N x N eigenvectors from the last iteration (Jacobi warm start)
    float *vs32;
    double *out;         // SOS_OUT_* below
};

enum {
    SOS_OUT_STATUS = 0, SOS_OUT_ITERS, SOS_OUT_POBJ, SOS_OUT_DOBJ, SOS_OUT_RP, SOS_OUT_RD, SOS_OUT_GAP,
    SOS_OUT_TAU, SOS_OUT_KAPPA, SOS_OUT_CX, SOS_OUT_BY, SOS_OUT_TOTAL, SOS_OUT_SWEEPS, SOS_OUT_T_AFFINE, SOS_OUT_T_EIG, SOS_OUT_T_RES, SOS_OUT_WARM,
    SOS_OUT_T_START, SOS_OUT_T_END,   // device wall clock when a batch workgroup took the problem and finished it
    SOS_OUT_N
};

enum { RUN_STEP = 0, RUN_SOLVE = 1 };

struct RunParams {
    ProbDesc *probs;        // device array
    const int *order;       // queue order (indices into probs)
    int *counter;           // device queue head
    int count;
    int mode;               // RUN_STEP | RUN_SOLVE
    int iters;              // RUN_STEP: exact count; RUN_SOLVE: max iterations
    int min_iters;          // RUN_SOLVE: no stopping test before this many iterations
    int check_every;
    double tol, alpha;
    void *work;             // per-workgroup affine work area
    long long work_stride;  // bytes
    void *eig;              // per-workgroup eigensolver area (global)
    long long eig_stride;   // bytes
    int eig_ld;             // leading dimension of the eigensolver matrices
    int max_sweeps;
    int warm_eig;           // start each block's Jacobi sweeps from the previous iteration's eigenvectors
    int lds_budget;         // dynamic LDS bytes the launch may use
    int eig_wave;           // 2: blocks that fit in LDS use the rows-over-wavefronts eigensolver;
                            // 0: every block uses the lane-group form
    int lds_mat_off, lds_nmax, lds_nmax_g, rows_nmax;   // filled in by the launcher
    int rows_nmin;          // eig_wave 2: blocks with N below this still take the lane-group form
    int accumulate;         // 0: out[TOTAL] = iterations of this launch; 1: out[TOTAL] += them, and the
                            //    iteration budget is iters + out[WARM] - out[TOTAL] (at least min_iters)
    int warm_budget;        // > 0 (first launch of a solve): restart a warm start (tk[3] = 1) from the cold
                            //    start once it reaches this many iterations unsolved or shows tau = 0
    int gs_bucket[7];       // lanes per Jacobi column pair (8, 16 or 32) by block-size bucket:
                            // N < 32, < 64, < 96, < 128, < 192, < 256, >= 256
    int stall_checks;       // > 0: stop a problem that stopped improving (see the kernel) this many checks in a row
    double jacobi_tol;      // relative coupling a Jacobi pair must exceed to be rotated (0: 16 eps of the type)
    int jac_block;          // 8: the lane-group form sweeps in the block-cyclic order when G and V sit in
                            //    LDS (a workgroup barrier per block round); 0: the cyclic order
    int pair_need;          // LDS elements (of the launch's type) that G and V of a two-block problem's
                            //    blocks need together (the largest over the problems; 0: none)
    int lds_pair;           // filled in by the launcher: pair_need if the launch's LDS holds it, else 0;
                            //    a two-block problem that fits projects both blocks at once
    long long lds_bytes;    // filled in by the launcher: the launch's dynamic LDS bytes (0: unknown)
    unsigned long long *ts; // optional [start, end] wall-clock stamps of the launch (min / max over workgroups)
};

// Leading dimension of an N x N eigensolver matrix in LDS: columns padded to 8 mod 16 elements,
// so that a wavefront's reads of a round's columns fall in distinct banks.
#define SOS_LDS_LD(N) ((N) <= 8 ? (N) : ((((N) + 7) & ~15) + 8))
// LDS elements that G and V of two blocks N1, N2 take together, and block 2's sigma (0 unless both
// are at least 2); host and device code share it
#if defined(__HIP__)
__host__ __device__
#endif
static inline long long sos_pair_need(int N1, int N2) {
    if (N1 < 2 || N2 < 2) return 0;
    return 2LL * ((long long)N1 * SOS_LDS_LD(N1) + (long long)N2 * SOS_LDS_LD(N2)) + N2;
}

// Control block of a cooperative (multi-workgroup) launch on one problem, in device memory.
struct CoopCtl {
    unsigned int count, gen;   // grid barrier: arrivals, generation
    int err;                   // 1: a barrier wait ran past its spin limit (the launch's results are void)
    int status;                // residual-check status broadcast by workgroup 0
    int big[3];                // Jacobi sweep votes, by the launch's running sweep count modulo 3: the
                               // flag reset during sweep s (that of s + 1) was last read after sweep
                               // s - 2, before every workgroup passed the barriers of sweep s - 1
    int pad[1];
};
// Largest number of workgroups of a cooperative launch (per-workgroup partial sums in the scratch).
#define SOS_COOP_MAX_WG 1024

// host-side launchers implemented in sos_kernels.hip; a launcher returning -4 leaves the reason
// in sos_launch_message() (this thread)
const char *sos_launch_message();
int sos_launch_admm(int fp64, int threads, int grid, const RunParams &rp, void *stream);
// the mixed form in one launch (FP32 phase, widening, FP64 phase per problem); threads 256 or
// 512, else returns -1 and the caller launches the phases separately
int sos_launch_admm_mixed(int threads, int grid, const RunParams &rp32, const RunParams &rp64, void *stream);
int sos_launch_reset(int *counter, void *stream, unsigned long long *ts = nullptr);
int sos_launch_cast_state(const ProbDesc *probs_dev, const int *ids, int count, int to64, void *stream,
                          int max_len);
int sos_launch_reset_state(const ProbDesc *probs_dev, int count, int max_len, void *stream);
// grid: the number of workgroups whose scratch areas (work_stride, eig_stride apart) exist
int sos_launch_warm_start(int fp64, int threads, int grid, const RunParams &rp, const float *pred, long long ld,
                          void *stream);
// Multi-workgroup FP64 solve of problem 0 of rp (one cooperative launch of `grid` workgroups):
// every workgroup takes part in the affine step, the block Jacobi eigensolver (column blocks of 8,
// a pair of blocks per workgroup and block round) and the MFMA products; workgroup 0 runs the
// residual checks.  scratch: 3 nmax^2 + nmax doubles (G, V, W, sigma), 2 SOS_COOP_MAX_WG doubles
// of partial sums, 2 x (k rounded up to 64) doubles for the affine step.  ctl: zeroed by the
// launcher.  Returns 0, -1 (unsupported shape), -4 (launch failed).
int sos_launch_admm_coop(int threads, int grid, const RunParams &rp, CoopCtl *ctl, double *scratch, void *stream);
// Largest grid a cooperative launch of the given width may use on this device (0 if unsupported).
int sos_coop_max_grid(int threads, const RunParams &rp);
// Device address of the static scratch (SOS_STATIC_SCRATCH_BYTES) on the current device,
// looked up once per device; 0 on success, -4 if the lookup failed.
int sos_static_scratch(void **ptr);
// eigen-decomposition of PSD block blk of problem 0's solution (dual: of z instead of xi), one
// workgroup; evals (N) and evecs (N x N, column-major) device arrays
int sos_launch_psd_factor(int threads, const RunParams &rp, int blk, int dual, double *evals, double *evecs,
                          void *stream);
int sos_launch_export(int fp64, const ProbDesc *probs, int count, float *out, long long ld, int max_len, void *stream);
