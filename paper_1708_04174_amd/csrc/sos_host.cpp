// Host side of the C ABI declared in include/sos.h: validation, the fold from the
// paper's column-stacked vec to the weighted lower triangle, the A_f / A_s split, the cached
// factor of I + A_f^T D^{-1} A_f (Section IV-B), h = M^{-1} zeta, device upload,
// and the launches of the persistent solver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/sos.h"
#include "sos_internal.h"

namespace {

thread_local std::string g_setup_error;

// dynamic LDS a solver launch may take (gfx950: 160 KiB per workgroup, minus the static part)
const int kLdsBudget = 159 * 1024;   // of the 160 KiB per workgroup, the rest for static LDS
// Default eigensolver choice (single solves and schedules without these keys): the lane-group
// form below N = 128 (with G and V in LDS, the block-cyclic order: at N = 120 0.41 against 0.65
// ms per FP32 iteration for the rows form, even in FP64), and the rows-over-wavefronts form from
// 128 on for blocks that fit in LDS (even with the lane-group form there); lanes per column pair
// by block-size bucket (N < 32, 64, 96, 128, 192, 256, larger): 8 for 64 <= N < 128, as the
// autotuner picks there.
constexpr int kRowsNmin = 128;
// Jacobi coupling tolerance of the mixed form's FP64 phase (0: 16 eps of FP64).  That phase
// has to carry the iterate below the FP32 floor of the affine step and of the residuals; its
// stopping test and certificates are evaluated in FP64 on the iterate itself, whatever the
// eigensolver's accuracy.  Eigenvectors orthogonal to 1e-7 (sweeps stop once every coupling of
// a sweep is under 3e-4) measured as fast as FP32-level ones with the same statuses on the
// Lyapunov batch, and save about one sweep per projection against 16 eps.
constexpr double kMixedJacobiTol64 = 1e-7;
constexpr int kLanesPerPair[7] = {16, 16, 8, 8, 16, 16, 16};
// FP64 single solves take the multi-workgroup (cooperative) path from this largest block size on
// (eig_form 0); eig_form 3 takes it for every block
constexpr int kCoopNmin = 128;
// columns per Jacobi block of the multi-workgroup eigensolver (a pair of blocks is one 16-wide
// matrix-core tile)
constexpr int kCoopBcols = 8;
// the lane-group form's sweep order when G and V sit in LDS: 8 = block-cyclic, 0 = cyclic
constexpr int kJacBlock = 8;
// mixed form: the FP32 phase hands over after this many residual checks without a 10 % gain.
// An FP32-stored iterate has a residual floor of about eps_32 |A| |y| / tau (above 1e-4 on the
// Lyapunov family), so the hand-over should come soon after the floor is reached.
const int kStallChecks = 4;

double wall_clock_khz() {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
        return 100000.0;
    return (double)khz;
}

struct DeviceArena {
    std::vector<void *> ptrs;
    ~DeviceArena() { release(); }
    void release() {
        for (void *p : ptrs) (void)hipFree(p);
        ptrs.clear();
    }
    template <typename T>
    T *alloc(size_t n) {
        void *p = nullptr;
        size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
        if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return static_cast<T *>(p);
    }
};

int svec_index(int i, int j, int N) {   // i >= j, lower triangle by columns
    return j * N - (j * (j - 1)) / 2 + (i - j);
}

struct Status : std::exception {
    int code;
    std::string msg;
    Status(int c, std::string m) : code(c), msg(std::move(m)) {}
};

void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) throw Status(SOS_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T>
void upload(T *dst, const std::vector<T> &src, hipStream_t st) {
    if (!src.empty()) hip_check(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st),
                                "hipMemcpyAsync");
}

template <typename T>
std::vector<float> to_f32(const std::vector<T> &x) {
    std::vector<float> y(x.size());
    for (size_t i = 0; i < x.size(); ++i) y[i] = (float)x[i];
    return y;
}

}   // namespace

struct sos_work {
    sos_settings st{};
    hipStream_t stream = nullptr;
    std::string err;
    int m = 0, n_full = 0, nx = 0, nfree = 0, k = 0;
    std::vector<int> N, off_full, off_svec;
    int nmax = 0;
    DeviceArena mem;
    ProbDesc desc{};          // host copy
    ProbDesc *d_desc = nullptr;
    int *d_counter = nullptr, *d_order = nullptr;
    void *d_work = nullptr, *d_eig = nullptr;
    long long work_stride = 0, eig_stride = 0;
    int eig_ld = 0;
    int threads = 256;
    bool active64 = true;     // which copy of (u, v) holds the current iterate
    // multi-workgroup path (FP64 single solves with a large block): cooperative grid, scratch
    bool use_coop = false;
    int coop_grid = 0, coop_threads = 512;
    double *d_coop_scr = nullptr;
    CoopCtl *d_ctl = nullptr;
    // equilibration: the iteration runs on D A E; x = E x^, y = D y^, z = z^ / E
    std::vector<double> Drow; // m
    std::vector<double> Ecol; // nx (internal columns)
    double setup_ms = 0.0, last_ms = 0.0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

struct sos_batch {
    std::vector<sos_work *> probs;
    DeviceArena mem;
    ProbDesc *d_desc = nullptr;
    int *d_order = nullptr, *d_counter = nullptr;
    double *d_out = nullptr;
    void *d_work = nullptr, *d_eig = nullptr;
    long long work_stride = 0, eig_stride = 0;
    int eig_ld = 0, threads = 256, grid = 1, count = 0, fp64 = 1, wg_per_cu = 2, max_sweeps = 40;
    int pair_need = 0;   // LDS elements of the largest two-block problem's blocks together
    int max_len = 0;
    hipStream_t stream = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t evp[4] = {nullptr, nullptr, nullptr, nullptr};
    unsigned long long *d_ts = nullptr;   // wall-clock stamps of the solve and polish kernels
    double last_ms = 0.0, phase_ms[2] = {0.0, 0.0};
    bool use_graph = true;
    int warm_eig = 1, lds_budget = 0, eig_wave = 2, rows_nmin = 0;
    double jacobi_tol64 = 0.0;   // Jacobi tolerance of the mixed form's FP64 phase
    int stall_checks = 0;        // mixed form: checks without progress before the FP64 phase
    int jac_block = 8;           // lane-group form's sweep order (see RunParams::jac_block)
    int one_launch = 1;   // mixed form: both phases in one launch (threads 256 or 512)
    bool used_one_launch = false;
    int gs_bucket[7] = {16, 16, 16, 16, 16, 16, 16};
    sos_settings st{};
    std::string err;   // message of the last failed call on the batch
};

namespace {

void default_settings(sos_settings *s) {
    s->tol = 1e-4;
    s->max_iters = 2000;
    s->check_every = 10;
    s->alpha = 1.0;
    s->precision = SOS_FP64;
    s->polish_iters = 1;
    s->partition = SOS_PART_PAPER;
    s->block_threads = 0;
    s->eig_form = 0;
    s->warm_budget = 0;
    s->scale_iters = 0;
}

void check_settings(const sos_settings &s) {
    if (!(s.tol > 0.0) || s.max_iters < 0 || s.check_every < 1 || !(s.alpha > 0.0 && s.alpha < 2.0))
        throw Status(SOS_E_INVAL, "invalid settings (tol > 0, max_iters >= 0, check_every >= 1, 0 < alpha < 2)");
    if (s.precision != SOS_FP64 && s.precision != SOS_FP32_MIXED) throw Status(SOS_E_INVAL, "invalid precision");
    if (s.partition != SOS_PART_PAPER && s.partition != SOS_PART_COLUMNS) throw Status(SOS_E_INVAL, "invalid partition");
    if (s.block_threads != 0 && (s.block_threads < 64 || s.block_threads > 1024 || (s.block_threads & (s.block_threads - 1))))
        throw Status(SOS_E_INVAL, "block_threads must be 0 or a power of two in 64..1024");
    if (s.precision == SOS_FP32_MIXED && s.polish_iters < 1) throw Status(SOS_E_INVAL, "polish_iters >= 1 required");
    if (s.warm_budget < 0) throw Status(SOS_E_INVAL, "warm_budget must be >= 0");
    if (s.eig_form < 0 || s.eig_form > 3) throw Status(SOS_E_INVAL, "eig_form must be 0, 1, 2 or 3");
    if (s.scale_iters < 0 || s.scale_iters > 1000) throw Status(SOS_E_INVAL, "scale_iters must be in 0..1000");
}

// Dense Cholesky of the k x k SPD matrix S (row-major), lower factor in place.
void cholesky(std::vector<double> &S, int k) {
    for (int j = 0; j < k; ++j) {
        double d = S[(size_t)j * k + j];
        for (int p = 0; p < j; ++p) d -= S[(size_t)j * k + p] * S[(size_t)j * k + p];
        if (!(d > 0.0)) throw Status(SOS_E_INVAL, "I + A_f^T D^{-1} A_f is not positive definite");
        const double ljj = std::sqrt(d);
        S[(size_t)j * k + j] = ljj;
        for (int i = j + 1; i < k; ++i) {
            double s = S[(size_t)i * k + j];
            for (int p = 0; p < j; ++p) s -= S[(size_t)i * k + p] * S[(size_t)j * k + p];
            S[(size_t)i * k + j] = s / ljj;
        }
    }
}

// Block-scalar equilibration of the full-vec A: row factors D (m) and column factors E (n),
// E constant on every PSD block and per free variable.  Each pass divides every row by the
// square root of its 2-norm, then every column group by the square root of the root mean
// square of its columns' 2-norms, then rebalances D to geometric mean 1 (E takes the inverse
// factor; D A E is unchanged) and clamps both to [1e-4, 1e4].  A diagonal D keeps A_s A_s^T
// diagonal and one factor per block keeps the cone (Proposition 1).
void equilibrate(const sos_csc *A, const sos_cone *K, int passes, std::vector<double> &D, std::vector<double> &E) {
    const int m = A->m, n = A->n;
    std::vector<double> r2(m), c2(n);
    std::vector<int> gstart, gend;
    for (int j = 0; j < K->n_free; ++j) {
        gstart.push_back(j);
        gend.push_back(j + 1);
    }
    int off = K->n_free;
    for (int bk = 0; bk < K->n_psd; ++bk) {
        gstart.push_back(off);
        off += K->N[bk] * K->N[bk];
        gend.push_back(off);
    }
    for (int pass = 0; pass < passes; ++pass) {
        std::fill(r2.begin(), r2.end(), 0.0);
        for (int j = 0; j < n; ++j)
            for (long long e = A->colptr[j]; e < A->colptr[j + 1]; ++e) r2[A->rowind[e]] += A->val[e] * A->val[e] * E[j] * E[j];
        for (int i = 0; i < m; ++i) {
            const double r = std::sqrt(r2[i]) * D[i];
            if (r > 0.0) D[i] /= std::sqrt(r);
        }
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (long long e = A->colptr[j]; e < A->colptr[j + 1]; ++e) s += A->val[e] * A->val[e] * D[A->rowind[e]] * D[A->rowind[e]];
            c2[j] = s * E[j] * E[j];
        }
        for (size_t g = 0; g < gstart.size(); ++g) {
            double s = 0.0;
            for (int j = gstart[g]; j < gend[g]; ++j) s += c2[j];
            const double val = std::sqrt(s / (gend[g] - gstart[g]));
            if (val > 0.0)
                for (int j = gstart[g]; j < gend[g]; ++j) E[j] /= std::sqrt(val);
        }
        double lg = 0.0;
        for (int i = 0; i < m; ++i) lg += std::log(D[i]);
        const double gm = m > 0 ? std::exp(lg / m) : 1.0;
        for (int i = 0; i < m; ++i) D[i] = std::min(1e4, std::max(1e-4, D[i] / gm));
        for (int j = 0; j < n; ++j) E[j] = std::min(1e4, std::max(1e-4, E[j] * gm));
    }
}

void setup_coop(sos_work *w);

void build(sos_work *w, const sos_csc *A, const double *b, const double *c, const sos_cone *K) {
    if (!A || !b || !c || !K || !A->colptr || (!A->rowind && A->colptr[A->n] > 0))
        throw Status(SOS_E_INVAL, "null argument");
    const int m = A->m, n = A->n;
    if (m < 0 || n < 1 || K->n_free < 0 || K->n_psd < 0 || K->n_psd > SOS_MAX_BLOCKS)
        throw Status(SOS_E_INVAL, "bad dimensions (at most 64 PSD blocks)");
    long long ncheck = K->n_free;
    for (int j = 0; j < K->n_psd; ++j) {
        if (K->N[j] < 1 || K->N[j] > 2048) throw Status(SOS_E_INVAL, "PSD block size must be in 1..2048");
        ncheck += (long long)K->N[j] * K->N[j];
    }
    if (ncheck != n) throw Status(SOS_E_INVAL, "A has n != n_free + sum N_j^2 columns");
    if (A->colptr[0] != 0) throw Status(SOS_E_INVAL, "colptr[0] != 0");
    for (int j = 0; j < n; ++j) {
        if (A->colptr[j + 1] < A->colptr[j]) throw Status(SOS_E_INVAL, "colptr not monotone");
        for (long long e = A->colptr[j]; e < A->colptr[j + 1]; ++e) {
            const int r = A->rowind[e];
            if (r < 0 || r >= m) throw Status(SOS_E_INVAL, "row index out of range");
            if (e > A->colptr[j] && A->rowind[e - 1] >= r) throw Status(SOS_E_INVAL, "row indices not sorted/unique");
            if (!std::isfinite(A->val[e])) throw Status(SOS_E_INVAL, "non-finite value in A");
        }
    }
    for (int i = 0; i < m; ++i)
        if (!std::isfinite(b[i])) throw Status(SOS_E_INVAL, "non-finite b");
    for (int j = 0; j < n; ++j)
        if (!std::isfinite(c[j])) throw Status(SOS_E_INVAL, "non-finite c");

    w->m = m;
    w->n_full = n;
    w->nfree = K->n_free;
    w->N.assign(K->N, K->N + K->n_psd);
    w->nmax = 0;
    // symmetric column pairs, offsets
    int off = K->n_free, soff = K->n_free;
    for (int bk = 0; bk < K->n_psd; ++bk) {
        const int N = K->N[bk];
        w->off_full.push_back(off);
        w->off_svec.push_back(soff);
        w->nmax = std::max(w->nmax, N);
        for (int j = 0; j < N; ++j)
            for (int i = j + 1; i < N; ++i) {
                const int c1 = off + j * N + i, c2 = off + i * N + j;
                const long long l1 = A->colptr[c1 + 1] - A->colptr[c1], l2 = A->colptr[c2 + 1] - A->colptr[c2];
                if (l1 != l2 || c[c1] != c[c2]) throw Status(SOS_E_ASYM, "PSD block columns (i,j) and (j,i) differ");
                for (long long t = 0; t < l1; ++t)
                    if (A->rowind[A->colptr[c1] + t] != A->rowind[A->colptr[c2] + t] ||
                        A->val[A->colptr[c1] + t] != A->val[A->colptr[c2] + t])
                        throw Status(SOS_E_ASYM, "PSD block columns (i,j) and (j,i) differ");
            }
        off += N * N;
        soff += N * (N + 1) / 2;
    }
    const int nx = soff;
    w->nx = nx;

    // Optional block-scalar equilibration (Ruiz's passes with one column factor per PSD block,
    // so that partial orthogonality and the cone survive): the iteration runs on D A E, D b, E c
    std::vector<double> aval, bsc, csc_;
    std::vector<double> Dfull(m, 1.0), Efull(n, 1.0);
    sos_csc Ascaled;
    double nb0 = 0.0, nc0 = 0.0;   // norms of the original b and c (residuals are in its units)
    for (int i = 0; i < m; ++i) nb0 += b[i] * b[i];
    for (int j = 0; j < n; ++j) nc0 += c[j] * c[j];
    if (w->st.scale_iters > 0) {
        equilibrate(A, K, w->st.scale_iters, Dfull, Efull);
        const long long nnz = A->colptr[n];
        aval.resize(nnz);
        for (int j = 0; j < n; ++j)
            for (long long e = A->colptr[j]; e < A->colptr[j + 1]; ++e) aval[e] = A->val[e] * Dfull[A->rowind[e]] * Efull[j];
        bsc.resize(m);
        csc_.resize(n);
        for (int i = 0; i < m; ++i) bsc[i] = b[i] * Dfull[i];
        for (int j = 0; j < n; ++j) csc_[j] = c[j] * Efull[j];
        Ascaled = *A;
        Ascaled.val = aval.data();
        A = &Ascaled;
        b = bsc.data();
        c = csc_.data();
    }
    w->Drow = Dfull;

    // fold to the lower triangle: column e -> source column (i,j), i >= j; an off-diagonal
    // entry stands for both (i,j) and (j,i) of the full vec, hence weight 2
    std::vector<int> src_col(nx);
    std::vector<double> wgt(nx, 1.0);
    for (int e = 0; e < K->n_free; ++e) src_col[e] = e;
    for (int bk = 0; bk < K->n_psd; ++bk) {
        const int N = K->N[bk];
        for (int j = 0; j < N; ++j)
            for (int i = j; i < N; ++i) {
                const int e = w->off_svec[bk] + svec_index(i, j, N);
                src_col[e] = w->off_full[bk] + j * N + i;
                wgt[e] = (i == j) ? 1.0 : 2.0;
            }
    }
    w->Ecol.assign(nx, 1.0);
    for (int e = 0; e < nx; ++e) w->Ecol[e] = Efull[src_col[e]];
    std::vector<int> cnt(nx);
    std::vector<double> cs(nx), cw(nx);
    for (int e = 0; e < nx; ++e) {
        cnt[e] = (int)(A->colptr[src_col[e] + 1] - A->colptr[src_col[e]]);
        cs[e] = c[src_col[e]];
        cw[e] = cs[e] * wgt[e];
    }
    // partition
    std::vector<int> colrow(nx, -1), fcolof(nx, -1);
    std::vector<int> fcols;
    for (int e = 0; e < nx; ++e) {
        const bool lowrank = cnt[e] >= 2 || (w->st.partition == SOS_PART_PAPER && e < K->n_free);
        if (lowrank) {
            fcolof[e] = (int)fcols.size();
            colrow[e] = -2 - (int)fcols.size();
            fcols.push_back(e);
        }
    }
    const int k = (int)fcols.size();
    w->k = k;
    std::vector<double> colval(nx, 0.0), d(m, 1.0);
    for (int e = 0; e < nx; ++e) {
        if (colrow[e] <= -2) continue;
        if (cnt[e] == 1) {
            const long long p = A->colptr[src_col[e]];
            colrow[e] = A->rowind[p];
            colval[e] = A->val[p];
            d[colrow[e]] += wgt[e] * colval[e] * colval[e];
        }
    }
    // CSR of the whole svec A
    std::vector<int> rowptr(m + 1, 0);
    for (int e = 0; e < nx; ++e)
        for (long long p = A->colptr[src_col[e]]; p < A->colptr[src_col[e] + 1]; ++p) rowptr[A->rowind[p] + 1]++;
    for (int i = 0; i < m; ++i) rowptr[i + 1] += rowptr[i];
    std::vector<int> colidx(rowptr[m]);
    std::vector<double> val(rowptr[m]);
    {
        std::vector<int> fill(rowptr.begin(), rowptr.end() - 1);
        for (int e = 0; e < nx; ++e)
            for (long long p = A->colptr[src_col[e]]; p < A->colptr[src_col[e] + 1]; ++p) {
                const int r = A->rowind[p];
                colidx[fill[r]] = e;
                val[fill[r]++] = A->val[p] * wgt[e];
            }
    }
    // A_f in CSC and CSR
    std::vector<int> fptr(k + 1, 0), frow;
    std::vector<double> fval;
    for (int j = 0; j < k; ++j) {
        const int e = fcols[j];
        for (long long p = A->colptr[src_col[e]]; p < A->colptr[src_col[e] + 1]; ++p) {
            frow.push_back(A->rowind[p]);
            fval.push_back(A->val[p]);
        }
        fptr[j + 1] = (int)frow.size();
    }
    std::vector<int> frptr(m + 1, 0);
    for (int r : frow) frptr[r + 1]++;
    for (int i = 0; i < m; ++i) frptr[i + 1] += frptr[i];
    std::vector<int> frcol(frow.size());
    std::vector<double> frval(frow.size());
    {
        std::vector<int> fill(frptr.begin(), frptr.end() - 1);
        for (int j = 0; j < k; ++j)
            for (int p = fptr[j]; p < fptr[j + 1]; ++p) {
                frcol[fill[frow[p]]] = j;
                frval[fill[frow[p]]++] = fval[p];
            }
    }
    std::vector<double> dinv(m);
    for (int i = 0; i < m; ++i) dinv[i] = 1.0 / d[i];
    // S = W_f^{-1} + A_f^T D^{-1} A_f and its Cholesky factor.  In full-vec terms
    // A_f A_f^T sums both copies of an off-diagonal column, i.e. A_f W_f A_f^T with
    // W_f = diag(wgt), and the matrix inversion lemma then needs W_f^{-1} in place of I.
    std::vector<double> S((size_t)k * k, 0.0);
    for (int j = 0; j < k; ++j) S[(size_t)j * k + j] = 1.0 / wgt[fcols[j]];
    for (int r = 0; r < m; ++r)
        for (int p = frptr[r]; p < frptr[r + 1]; ++p)
            for (int q = frptr[r]; q < frptr[r + 1]; ++q)
                S[(size_t)frcol[p] * k + frcol[q]] += frval[p] * frval[q] * dinv[r];
    cholesky(S, k);
    // S^{-1} = L^{-T} L^{-1}, formed once in FP64 so that each iteration's solve with S is
    // one dense matrix-vector product: Li = L^{-1} (lower, by forward substitution on the
    // columns of I), then Sinv[i][j] = sum_{l >= max(i,j)} Li[l][i] Li[l][j]
    // (both loops stream rows, row-major)
    std::vector<double> Li((size_t)k * k, 0.0), Sinv((size_t)k * k, 0.0);
    for (int i = 0; i < k; ++i) {   // row i of L^{-1}: L[i][0..i] Li[0..i][j] = delta_ij
        double *li = &Li[(size_t)i * k];
        for (int p = 0; p < i; ++p) {
            const double lip = S[(size_t)i * k + p];
            const double *lp = &Li[(size_t)p * k];
            for (int j = 0; j <= p; ++j) li[j] -= lip * lp[j];
        }
        li[i] = 1.0;
        const double dinv_i = 1.0 / S[(size_t)i * k + i];
        for (int j = 0; j <= i; ++j) li[j] *= dinv_i;
    }
    for (int l = 0; l < k; ++l) {   // Sinv += row_l(Li)^T row_l(Li), lower triangle
        const double *ll = &Li[(size_t)l * k];
        for (int i = 0; i <= l; ++i) {
            const double a = ll[i];
            double *si = &Sinv[(size_t)i * k];
            for (int j = 0; j <= i; ++j) si[j] += a * ll[j];
        }
    }
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < i; ++j) Sinv[(size_t)j * k + i] = Sinv[(size_t)i * k + j];

    // h = M^{-1} zeta, zeta = (c, -b): the same Woodbury route, in FP64 on the host
    std::vector<double> bv(b, b + m);
    std::vector<double> x(m);
    for (int r = 0; r < m; ++r) {
        double acc = -bv[r];
        for (int p = rowptr[r]; p < rowptr[r + 1]; ++p) acc -= val[p] * cs[colidx[p]];
        x[r] = acc * dinv[r];
    }
    std::vector<double> zq(k, 0.0);
    for (int j = 0; j < k; ++j)
        for (int p = fptr[j]; p < fptr[j + 1]; ++p) zq[j] += fval[p] * x[frow[p]];
    for (int j = 0; j < k; ++j) {   // forward
        double s = zq[j];
        for (int p = 0; p < j; ++p) s -= S[(size_t)j * k + p] * zq[p];
        zq[j] = s / S[(size_t)j * k + j];
    }
    for (int j = k - 1; j >= 0; --j) {   // backward
        double s = zq[j];
        for (int p = j + 1; p < k; ++p) s -= S[(size_t)p * k + j] * zq[p];
        zq[j] = s / S[(size_t)j * k + j];
    }
    std::vector<double> h(nx + m);
    for (int r = 0; r < m; ++r) {
        double acc = 0.0;
        for (int p = frptr[r]; p < frptr[r + 1]; ++p) acc += frval[p] * zq[frcol[p]];
        h[nx + r] = x[r] - dinv[r] * acc;
    }
    for (int e = 0; e < nx; ++e) {
        double acc = cs[e];
        if (colrow[e] >= 0) acc += colval[e] * h[nx + colrow[e]];
        else if (colrow[e] <= -2) {
            const int j = -2 - colrow[e];
            for (int p = fptr[j]; p < fptr[j + 1]; ++p) acc += fval[p] * h[nx + frow[p]];
        }
        h[e] = acc;
    }
    double ch = 0.0, bh = 0.0, nb = 0.0, nc = 0.0;
    for (int e = 0; e < nx; ++e) {
        ch += cw[e] * h[e];
        nc += cw[e] * cs[e];
    }
    for (int r = 0; r < m; ++r) {
        bh += bv[r] * h[nx + r];
        nb += bv[r] * bv[r];
    }
    const double eta = 1.0 + ch - bh;

    // upload
    hipStream_t st = w->stream;
    ProbDesc &P = w->desc;
    std::memset(&P, 0, sizeof(P));
    P.m = m;
    P.nx = nx;
    P.nfree = K->n_free;
    P.k = k;
    P.nblk = K->n_psd;
    P.nmax = w->nmax;
    for (int bk = 0; bk < K->n_psd; ++bk) {
        P.blk_N[bk] = K->N[bk];
        P.blk_off[bk] = w->off_svec[bk];
    }
    DeviceArena &M = w->mem;
    auto up_i = [&](const std::vector<int> &v) {
        int *p = M.alloc<int>(v.size());
        if (!p) throw Status(SOS_E_NOMEM, "hipMalloc failed");
        upload(p, v, st);
        return p;
    };
    auto up_d = [&](const std::vector<double> &v) {
        double *p = M.alloc<double>(v.size());
        if (!p) throw Status(SOS_E_NOMEM, "hipMalloc failed");
        upload(p, v, st);
        return p;
    };
    auto up_f = [&](const std::vector<double> &v) {
        float *p = M.alloc<float>(v.size());
        if (!p) throw Status(SOS_E_NOMEM, "hipMalloc failed");
        std::vector<float> f = to_f32(v);
        upload(p, f, st);
        hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
        return p;
    };
    P.rowptr = up_i(rowptr);
    P.colidx = up_i(colidx);
    P.val64 = up_d(val);
    P.val32 = up_f(val);
    P.colrow = up_i(colrow);
    P.colval64 = up_d(colval);
    P.colval32 = up_f(colval);
    P.fptr = up_i(fptr);
    P.fcol = up_i(fcols);
    P.frow = up_i(frow);
    P.fval64 = up_d(fval);
    P.fval32 = up_f(fval);
    P.frptr = up_i(frptr);
    P.frcol = up_i(frcol);
    P.frval64 = up_d(frval);
    P.frval32 = up_f(frval);
    P.dinv64 = up_d(dinv);
    P.dinv32 = up_f(dinv);
    P.Sinv = up_d(Sinv);
    P.h64 = up_d(h);
    P.h32 = up_f(h);
    P.b64 = up_d(bv);
    P.b32 = up_f(bv);
    P.c64 = up_d(cs);
    P.c32 = up_f(cs);
    P.cw64 = up_d(cw);
    P.cw32 = up_f(cw);
    P.wgt64 = up_d(wgt);
    P.eta = eta;
    P.nb = w->st.scale_iters > 0 ? std::sqrt(nb0) : std::sqrt(nb);
    P.nc = w->st.scale_iters > 0 ? std::sqrt(nc0) : std::sqrt(nc);
    if (w->st.scale_iters > 0) {
        // residuals in the original units: rows times 1 / D, columns times 1 / E
        std::vector<double> rs(m), cs_(nx);
        for (int i = 0; i < m; ++i) rs[i] = 1.0 / Dfull[i];
        for (int e = 0; e < nx; ++e) cs_[e] = 1.0 / w->Ecol[e];
        P.rsc64 = up_d(rs);
        P.csc64 = up_d(cs_);
    }
    P.u64 = M.alloc<double>(nx + m);
    P.v64 = M.alloc<double>(nx);
    P.u32 = M.alloc<float>(nx + m);
    P.v32 = M.alloc<float>(nx);
    P.tk = M.alloc<double>(4);
    long long nvs = 0;
    for (int bk = 0; bk < K->n_psd; ++bk) nvs += (long long)K->N[bk] * K->N[bk];
    P.vs64 = M.alloc<double>(nvs);
    P.vs32 = M.alloc<float>(nvs);
    if (!P.vs64 || !P.vs32) throw Status(SOS_E_NOMEM, "hipMalloc failed");
    P.out = M.alloc<double>(SOS_OUT_N);
    if (!P.u64 || !P.v64 || !P.u32 || !P.v32 || !P.tk || !P.out) throw Status(SOS_E_NOMEM, "hipMalloc failed");
    hip_check(hipMemsetAsync(P.u64, 0, sizeof(double) * (nx + m), st), "hipMemsetAsync");
    hip_check(hipMemsetAsync(P.v64, 0, sizeof(double) * nx, st), "hipMemsetAsync");
    hip_check(hipMemsetAsync(P.u32, 0, sizeof(float) * (nx + m), st), "hipMemsetAsync");
    hip_check(hipMemsetAsync(P.v32, 0, sizeof(float) * nx, st), "hipMemsetAsync");
    const double tk0[4] = {1.0, 1.0, 0.0, 0.0};
    hip_check(hipMemcpyAsync(P.tk, tk0, sizeof(tk0), hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    w->d_desc = M.alloc<ProbDesc>(1);
    w->d_counter = M.alloc<int>(1);
    w->d_order = M.alloc<int>(1);
    if (!w->d_desc || !w->d_counter || !w->d_order) throw Status(SOS_E_NOMEM, "hipMalloc failed");
    hip_check(hipMemcpyAsync(w->d_desc, &P, sizeof(P), hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    const int zero = 0;
    hip_check(hipMemcpyAsync(w->d_order, &zero, sizeof(int), hipMemcpyHostToDevice, st), "hipMemcpyAsync");
    // per-workgroup areas for a single-problem launch
    w->eig_ld = std::max(w->nmax, 1);
    w->work_stride = (long long)(((m + 63) & ~63) + nx + 64 + sos_work_tail_doubles(k)) * sizeof(double);
    w->eig_stride = (long long)3 * w->eig_ld * std::max(w->nmax, 1) * sizeof(double) + 256;
    w->d_work = M.alloc<char>(w->work_stride);
    w->d_eig = M.alloc<char>(w->eig_stride);
    if (!w->d_work || !w->d_eig) throw Status(SOS_E_NOMEM, "hipMalloc failed");
    hip_check(hipStreamSynchronize(st), "hipStreamSynchronize");
    w->active64 = true;
    setup_coop(w);
    hip_check(hipEventCreate(&w->ev0), "hipEventCreate");
    hip_check(hipEventCreate(&w->ev1), "hipEventCreate");
}

RunParams single_params(sos_work *w, int mode, int iters, int min_iters, double tol);

// Multi-workgroup path: FP64, a block of at least kCoopNmin (eig_form 0) or any (eig_form 3), a
// device with cooperative launches.  Column blocks of kCoopBcols columns; one workgroup per pair
// of blocks, up to what the device holds at once.
void setup_coop(sos_work *w) {
    w->use_coop = false;
    if (w->st.precision != SOS_FP64 || w->N.empty()) return;
    if (!(w->st.eig_form == 3 || (w->st.eig_form == 0 && w->nmax >= kCoopNmin))) return;
    const int thr = (w->threads == 256 || w->threads == 512) ? w->threads : 512;
    RunParams rp = single_params(w, RUN_STEP, 0, 0, w->st.tol);
    const int gmax = sos_coop_max_grid(thr, rp);
    if (gmax < 1) {
        if (w->st.eig_form == 3) throw Status(SOS_E_INVAL, "multi-workgroup eigensolver unavailable on this device/shape");
        return;
    }
    const int nb = (w->nmax + kCoopBcols - 1) / kCoopBcols;
    const int pairs = (nb + (nb & 1)) / 2;
    w->coop_grid = std::max(1, std::min(gmax, pairs));
    w->coop_threads = thr;
    const size_t nm = (size_t)w->nmax;
    // G, V, W, sigma, two partial sums per workgroup, the affine step's two k-vectors
    const size_t kp = ((size_t)w->k + 63) & ~(size_t)63;
    w->d_coop_scr = w->mem.alloc<double>(3 * nm * nm + nm + 2 * SOS_COOP_MAX_WG + 2 * kp);
    w->d_ctl = w->mem.alloc<CoopCtl>(1);
    if (!w->d_coop_scr || !w->d_ctl) throw Status(SOS_E_NOMEM, "hipMalloc failed");
    w->use_coop = true;
}

// the FP64 iterations of a single solve over the cooperative grid; checks the barrier's flag
void run_coop(sos_work *w, const RunParams &rp) {
    if (sos_launch_admm_coop(w->coop_threads, w->coop_grid, rp, w->d_ctl, w->d_coop_scr, w->stream))
        throw Status(SOS_E_HIP, std::string("cooperative launch failed: ") + sos_launch_message());
    CoopCtl c;
    hip_check(hipMemcpyAsync(&c, w->d_ctl, sizeof(c), hipMemcpyDeviceToHost, w->stream), "copy");
    hip_check(hipStreamSynchronize(w->stream), "sync");
    if (c.err) throw Status(SOS_E_HIP, "multi-workgroup launch: a grid barrier wait timed out");
}

RunParams single_params(sos_work *w, int mode, int iters, int min_iters, double tol) {
    RunParams rp{};
    rp.probs = w->d_desc;
    rp.order = w->d_order;
    rp.counter = w->d_counter;
    rp.count = 1;
    rp.mode = mode;
    rp.iters = iters;
    rp.min_iters = min_iters;
    rp.check_every = w->st.check_every;
    rp.tol = tol;
    rp.alpha = w->st.alpha;
    rp.work = w->d_work;
    rp.work_stride = w->work_stride;
    rp.eig = w->d_eig;
    rp.eig_stride = w->eig_stride;
    rp.eig_ld = w->eig_ld;
    rp.max_sweeps = 60;
    rp.warm_eig = 1;
    rp.lds_budget = kLdsBudget;
    for (int i = 0; i < 7; ++i) rp.gs_bucket[i] = kLanesPerPair[i];
    rp.eig_wave = w->st.eig_form == 2 ? 0 : 2;
    rp.rows_nmin = w->st.eig_form == 0 ? kRowsNmin : 0;
    rp.jac_block = kJacBlock;
    rp.pair_need = w->N.size() == 2 ? (int)sos_pair_need(w->N[0], w->N[1]) : 0;
    return rp;
}

void run_single(sos_work *w, int fp64, const RunParams &rp) {
    if (sos_launch_reset(rp.counter, w->stream)) throw Status(SOS_E_HIP, std::string("reset launch failed: ") + sos_launch_message());
    if (sos_launch_admm(fp64, w->threads, 1, rp, w->stream)) throw Status(SOS_E_HIP, std::string("solver launch failed: ") + sos_launch_message());
}

void set_active(sos_work *w, bool to64) {
    if (w->active64 == to64) return;
    if (sos_launch_cast_state(w->d_desc, nullptr, 1, to64 ? 1 : 0, w->stream, w->nx + w->m))
        throw Status(SOS_E_HIP, std::string("cast launch failed: ") + sos_launch_message());
    w->active64 = to64;
}

void read_info(sos_work *w, const double *o, sos_info *info, int iters, int polish) {
    if (!info) return;
    info->status = (int)o[SOS_OUT_STATUS];
    info->iters = iters;
    info->k_lowrank = w->k;
    info->polish_iters = polish;
    info->pobj = o[SOS_OUT_POBJ];
    info->dobj = o[SOS_OUT_DOBJ];
    info->res_pri = o[SOS_OUT_RP];
    info->res_dual = o[SOS_OUT_RD];
    info->gap = o[SOS_OUT_GAP];
    info->tau = o[SOS_OUT_TAU];
    info->kappa = o[SOS_OUT_KAPPA];
    info->setup_ms = w->setup_ms;
    info->solve_ms = w->last_ms;
    info->eig_sweeps = o[SOS_OUT_SWEEPS];
    const double khz = wall_clock_khz();
    info->affine_ms = o[SOS_OUT_T_AFFINE] / khz;
    info->eig_ms = o[SOS_OUT_T_EIG] / khz;
    info->resid_ms = o[SOS_OUT_T_RES] / khz;
    info->warm_iters = (int)o[SOS_OUT_WARM];
    info->start_ms = info->end_ms = 0.0;
}

// Layout of a single-problem launch's scratch inside the static device array: the queue
// counter, then the affine work vector, then the eigensolver area, each 256-byte aligned.
long long static_scratch_bytes(const sos_work *w, long long *work_off, long long *eig_off) {
    const long long a = 256;
    *work_off = a;
    *eig_off = *work_off + (w->work_stride + a - 1) / a * a;
    return *eig_off + w->eig_stride;
}

// sos_step, with the launch's scratch either the handle's own (allocated at setup) or the
// static device array (no allocation of any kind on this path)
void step_impl(sos_work *w, int32_t iters, sos_info *info, bool static_scratch) {
    const int fp64 = w->st.precision == SOS_FP64;
    RunParams rp = single_params(w, RUN_STEP, iters, 0, w->st.tol);
    if (static_scratch) {
        long long work_off = 0, eig_off = 0;
        const long long need = static_scratch_bytes(w, &work_off, &eig_off);
        if (need > SOS_STATIC_SCRATCH_BYTES)
            throw Status(SOS_E_INVAL, "problem needs " + std::to_string(need) +
                                          " bytes of scratch; the static scratch holds " +
                                          std::to_string((long long)SOS_STATIC_SCRATCH_BYTES));
        void *base = nullptr;
        if (sos_static_scratch(&base)) throw Status(SOS_E_HIP, "address of the static device scratch not found");
        char *b = static_cast<char *>(base);
        rp.counter = reinterpret_cast<int *>(b);
        rp.work = b + work_off;
        rp.eig = b + eig_off;
    }
    set_active(w, fp64);
    hip_check(hipEventRecord(w->ev0, w->stream), "event");
    if (fp64 && w->use_coop && !static_scratch) {
        if (sos_launch_admm_coop(w->coop_threads, w->coop_grid, rp, w->d_ctl, w->d_coop_scr, w->stream))
            throw Status(SOS_E_HIP, std::string("cooperative launch failed: ") + sos_launch_message());
    } else {
        run_single(w, fp64, rp);
    }
    hip_check(hipEventRecord(w->ev1, w->stream), "event");
    double o[SOS_OUT_N];
    hip_check(hipMemcpyAsync(o, w->desc.out, sizeof(o), hipMemcpyDeviceToHost, w->stream), "copy");
    hip_check(hipStreamSynchronize(w->stream), "sync");
    float ms = 0.f;
    hip_check(hipEventElapsedTime(&ms, w->ev0, w->ev1), "event");
    w->last_ms = ms;
    if (fp64 && w->use_coop && !static_scratch) {
        CoopCtl c;
        hip_check(hipMemcpy(&c, w->d_ctl, sizeof(c), hipMemcpyDeviceToHost), "copy");
        if (c.err) throw Status(SOS_E_HIP, "multi-workgroup launch: a grid barrier wait timed out");
    }
    read_info(w, o, info, iters, 0);
}

template <typename F>
int guarded(sos_work *w, F &&f) {
    try {
        f();
        return SOS_OK;
    } catch (const Status &s) {
        if (w) w->err = s.msg;
        return s.code;
    } catch (const std::bad_alloc &) {
        if (w) w->err = "host allocation failed";
        return SOS_E_NOMEM;
    }
}

// as guarded, with the message kept on the batch handle (or, for a batch that does not exist
// yet, where sos_last_error(NULL) finds it)
template <typename F>
int guarded_b(sos_batch *B, F &&f) {
    try {
        f();
        return SOS_OK;
    } catch (const Status &s) {
        if (B) B->err = s.msg;
        else g_setup_error = s.msg;
        return s.code;
    } catch (const std::bad_alloc &) {
        if (B) B->err = "host allocation failed";
        else g_setup_error = "host allocation failed";
        return SOS_E_NOMEM;
    }
}

// full-vec host vector -> lower triangle (xi part of u or v), averaging (i,j) and (j,i)
void full_to_svec(const sos_work *w, const double *x, std::vector<double> &out) {
    out.assign(w->nx, 0.0);
    for (int e = 0; e < w->nfree; ++e) out[e] = x[e];
    for (size_t bk = 0; bk < w->N.size(); ++bk) {
        const int N = w->N[bk];
        const double *X = x + w->off_full[bk];
        for (int j = 0; j < N; ++j)
            for (int i = j; i < N; ++i) {
                const int e = w->off_svec[bk] + svec_index(i, j, N);
                out[e] = (i == j) ? X[j * N + i] : 0.5 * (X[j * N + i] + X[i * N + j]);
            }
    }
}

void svec_to_full(const sos_work *w, const std::vector<double> &s, double scale, double *x) {
    for (int e = 0; e < w->nfree; ++e) x[e] = s[e] * scale;
    for (size_t bk = 0; bk < w->N.size(); ++bk) {
        const int N = w->N[bk];
        double *X = x + w->off_full[bk];
        for (int j = 0; j < N; ++j)
            for (int i = j; i < N; ++i) {
                const double val = s[w->off_svec[bk] + svec_index(i, j, N)] * scale;
                X[j * N + i] = X[i * N + j] = val;
            }
    }
}

// iterate of the equilibrated problem (lower triangles, u = (x^, y^), v = z^) <-> original units
void to_original(const sos_work *w, std::vector<double> &u, std::vector<double> &v) {
    if (w->st.scale_iters <= 0) return;
    for (int e = 0; e < w->nx; ++e) {
        u[e] *= w->Ecol[e];
        v[e] /= w->Ecol[e];
    }
    for (int i = 0; i < w->m; ++i) u[w->nx + i] *= w->Drow[i];
}
void to_internal(const sos_work *w, std::vector<double> &u, std::vector<double> &v) {
    if (w->st.scale_iters <= 0) return;
    for (int e = 0; e < w->nx; ++e) {
        u[e] /= w->Ecol[e];
        v[e] *= w->Ecol[e];
    }
    for (int i = 0; i < w->m; ++i) u[w->nx + i] /= w->Drow[i];
}

void fetch_state(const sos_work *w, std::vector<double> &u, std::vector<double> &v, double tk[2]) {
    const int nu = w->nx + w->m, nv = w->nx;
    u.resize(nu);
    v.resize(nv);
    if (w->active64) {
        hip_check(hipMemcpyAsync(u.data(), w->desc.u64, nu * sizeof(double), hipMemcpyDeviceToHost, w->stream), "copy");
        hip_check(hipMemcpyAsync(v.data(), w->desc.v64, nv * sizeof(double), hipMemcpyDeviceToHost, w->stream), "copy");
    } else {
        std::vector<float> uf(nu), vf(nv);
        hip_check(hipMemcpyAsync(uf.data(), w->desc.u32, nu * sizeof(float), hipMemcpyDeviceToHost, w->stream), "copy");
        hip_check(hipMemcpyAsync(vf.data(), w->desc.v32, nv * sizeof(float), hipMemcpyDeviceToHost, w->stream), "copy");
        hip_check(hipStreamSynchronize(w->stream), "sync");
        for (int i = 0; i < nu; ++i) u[i] = uf[i];
        for (int i = 0; i < nv; ++i) v[i] = vf[i];
    }
    hip_check(hipMemcpyAsync(tk, w->desc.tk, 2 * sizeof(double), hipMemcpyDeviceToHost, w->stream), "copy");
    hip_check(hipStreamSynchronize(w->stream), "sync");
}

void push_state(sos_work *w, const std::vector<double> &u, const std::vector<double> &v, const double tk[2],
                bool warm_start = false) {
    const int nu = w->nx + w->m, nv = w->nx;
    std::vector<float> uf(u.begin(), u.end()), vf(v.begin(), v.end());
    hip_check(hipMemcpyAsync(w->desc.u64, u.data(), nu * sizeof(double), hipMemcpyHostToDevice, w->stream), "copy");
    hip_check(hipMemcpyAsync(w->desc.v64, v.data(), nv * sizeof(double), hipMemcpyHostToDevice, w->stream), "copy");
    hip_check(hipMemcpyAsync(w->desc.u32, uf.data(), nu * sizeof(float), hipMemcpyHostToDevice, w->stream), "copy");
    hip_check(hipMemcpyAsync(w->desc.v32, vf.data(), nv * sizeof(float), hipMemcpyHostToDevice, w->stream), "copy");
    // new iterate: cached eigenvectors are stale; a warm start is judged by the next solve
    const double tk4[4] = {tk[0], tk[1], 0.0, warm_start ? 1.0 : 0.0};
    hip_check(hipMemcpyAsync(w->desc.tk, tk4, sizeof(tk4), hipMemcpyHostToDevice, w->stream), "copy");
    hip_check(hipStreamSynchronize(w->stream), "sync");
    w->active64 = true;
}

double json_num(const char *js, const char *key, double dflt) {
    if (!js) return dflt;
    std::string pat = std::string("\"") + key + "\"";
    const char *p = std::strstr(js, pat.c_str());
    if (!p) return dflt;
    p = std::strchr(p + pat.size(), ':');
    if (!p) return dflt;
    return std::strtod(p + 1, nullptr);
}

int device_cu_count() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
    return n;
}

}   // namespace

extern "C" {

int sos_default_settings(sos_settings *s) {
    if (!s) return SOS_E_INVAL;
    default_settings(s);
    return SOS_OK;
}

int sos_setup(const sos_csc *A, const double *b, const double *c, const sos_cone *K, const sos_settings *s,
              void *hip_stream, sos_work **out) {
    if (!out) return SOS_E_INVAL;
    *out = nullptr;
    sos_work *w = nullptr;
    try {
        w = new sos_work();
    } catch (...) {
        g_setup_error = "host allocation failed";
        return SOS_E_NOMEM;
    }
    if (s) w->st = *s;
    else default_settings(&w->st);
    w->stream = reinterpret_cast<hipStream_t>(hip_stream);
    const auto t0 = std::chrono::steady_clock::now();
    int rc = guarded(w, [&] {
        check_settings(w->st);
        w->threads = w->st.block_threads ? w->st.block_threads : 512;
        build(w, A, b, c, K);
    });
    if (rc != SOS_OK) {
        g_setup_error = w->err;
        delete w;
        return rc;
    }
    w->setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = w;
    return SOS_OK;
}

int sos_step(sos_work *w, int32_t iters, sos_info *info) {
    if (!w || iters < 0) return SOS_E_INVAL;
    return guarded(w, [&] { step_impl(w, iters, info, false); });
}

int sos_step_static(sos_work *w, int32_t iters, sos_info *info) {
    if (!w || iters < 0) return SOS_E_INVAL;
    return guarded(w, [&] { step_impl(w, iters, info, true); });
}

int sos_solve(sos_work *w, sos_info *info) {
    if (!w) return SOS_E_INVAL;
    return guarded(w, [&] {
        double o[SOS_OUT_N];
        int total = 0, polish = 0;
        hip_check(hipEventRecord(w->ev0, w->stream), "event");
        if (w->st.precision == SOS_FP64) {
            set_active(w, true);
            RunParams r = single_params(w, RUN_SOLVE, w->st.max_iters, 0, w->st.tol);
            r.warm_budget = w->st.warm_budget;
            if (w->use_coop && r.warm_budget == 0) run_coop(w, r);
            else run_single(w, 1, r);
            hip_check(hipMemcpyAsync(o, w->desc.out, sizeof(o), hipMemcpyDeviceToHost, w->stream), "copy");
            hip_check(hipStreamSynchronize(w->stream), "sync");
            total = (int)o[SOS_OUT_ITERS];
        } else {
            // FP32 phase to tol or until it stops improving, then FP64 for the rest of the budget
            set_active(w, false);
            RunParams r32 = single_params(w, RUN_SOLVE, w->st.max_iters, 0, w->st.tol);
            r32.stall_checks = kStallChecks;
            r32.warm_budget = w->st.warm_budget;
            run_single(w, 0, r32);
            set_active(w, true);
            RunParams r64 = single_params(w, RUN_SOLVE, w->st.max_iters, w->st.polish_iters, w->st.tol);
            r64.accumulate = 1;
            r64.jacobi_tol = kMixedJacobiTol64;
            run_single(w, 1, r64);
            hip_check(hipMemcpyAsync(o, w->desc.out, sizeof(o), hipMemcpyDeviceToHost, w->stream), "copy");
            hip_check(hipStreamSynchronize(w->stream), "sync");
            polish = (int)o[SOS_OUT_ITERS];
            total = (int)o[SOS_OUT_TOTAL];
        }
        hip_check(hipEventRecord(w->ev1, w->stream), "event");
        hip_check(hipEventSynchronize(w->ev1), "event");
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, w->ev0, w->ev1), "event");
        w->last_ms = ms;
        read_info(w, o, info, total, polish);
    });
}

int sos_warm_start(sos_work *w, const double *x, const double *y, const double *z, double tau, double kappa) {
    if (!w || !x || !y || !z) return SOS_E_INVAL;
    return guarded(w, [&] {
        if (!(tau >= 0.0) || !(kappa >= 0.0) || (tau == 0.0 && kappa == 0.0) || !std::isfinite(tau) ||
            !std::isfinite(kappa))
            throw Status(SOS_E_INVAL, "tau, kappa must be >= 0 and not both zero");
        for (int e = 0; e < w->nfree; ++e)
            if (z[e] != 0.0) throw Status(SOS_E_INVAL, "z must vanish on the free variables");
        for (int i = 0; i < w->n_full; ++i)
            if (!std::isfinite(x[i]) || !std::isfinite(z[i])) throw Status(SOS_E_INVAL, "non-finite warm start");
        for (int i = 0; i < w->m; ++i)
            if (!std::isfinite(y[i])) throw Status(SOS_E_INVAL, "non-finite warm start");
        std::vector<double> xs, zs;
        full_to_svec(w, x, xs);
        full_to_svec(w, z, zs);
        std::vector<double> u(w->nx + w->m), v(w->nx);
        for (int e = 0; e < w->nx; ++e) {
            u[e] = tau * xs[e];
            v[e] = tau * zs[e];
        }
        for (int i = 0; i < w->m; ++i) u[w->nx + i] = tau * y[i];
        to_internal(w, u, v);
        const double tk[2] = {tau, kappa};
        push_state(w, u, v, tk, true);
    });
}

int sos_get_solution(const sos_work *w, double *x, double *y, double *z) {
    if (!w) return SOS_E_INVAL;
    return guarded(const_cast<sos_work *>(w), [&] {
        std::vector<double> u, v;
        double tk[2];
        fetch_state(w, u, v, tk);
        if (!(tk[0] > 0.0)) throw Status(SOS_E_STATE, "tau == 0: no solution to normalise (certificate state)");
        to_original(w, u, v);
        const double s = 1.0 / tk[0];
        if (x) svec_to_full(w, u, s, x);
        if (z) svec_to_full(w, v, s, z);
        if (y)
            for (int i = 0; i < w->m; ++i) y[i] = u[w->nx + i] * s;
    });
}

int sos_get_iterate(const sos_work *w, double *uo, double *vo) {
    if (!w || !uo || !vo) return SOS_E_INVAL;
    return guarded(const_cast<sos_work *>(w), [&] {
        std::vector<double> u, v;
        double tk[2];
        fetch_state(w, u, v, tk);
        to_original(w, u, v);
        const int n = w->n_full, m = w->m;
        svec_to_full(w, u, 1.0, uo);
        for (int i = 0; i < m; ++i) uo[n + i] = u[w->nx + i];
        uo[n + m] = tk[0];
        svec_to_full(w, v, 1.0, vo);
        for (int i = 0; i < m; ++i) vo[n + i] = 0.0;
        vo[n + m] = tk[1];
    });
}

int sos_set_iterate(sos_work *w, const double *uo, const double *vo) {
    if (!w || !uo || !vo) return SOS_E_INVAL;
    return guarded(w, [&] {
        const int n = w->n_full, m = w->m;
        for (int i = 0; i < m; ++i)
            if (vo[n + i] != 0.0) throw Status(SOS_E_INVAL, "the s part of v must be zero");
        for (int e = 0; e < w->nfree; ++e)
            if (vo[e] != 0.0) throw Status(SOS_E_INVAL, "z must vanish on the free variables");
        for (int i = 0; i < n + m + 1; ++i)
            if (!std::isfinite(uo[i]) || !std::isfinite(vo[i])) throw Status(SOS_E_INVAL, "non-finite state");
        std::vector<double> us, vs;
        full_to_svec(w, uo, us);
        full_to_svec(w, vo, vs);
        std::vector<double> u(w->nx + m), v(w->nx);
        for (int e = 0; e < w->nx; ++e) {
            u[e] = us[e];
            v[e] = vs[e];
        }
        for (int i = 0; i < m; ++i) u[w->nx + i] = uo[n + i];
        to_internal(w, u, v);
        const double tk[2] = {uo[n + m], vo[n + m]};
        push_state(w, u, v, tk);
    });
}

int sos_psd_factor(sos_work *w, int32_t block, int32_t dual, double *evals, double *evecs) {
    if (!w || !evals || !evecs) return SOS_E_INVAL;
    return guarded(w, [&] {
        if (block < 0 || block >= (int)w->N.size()) throw Status(SOS_E_INVAL, "block index out of range");
        if (dual != 0 && dual != 1) throw Status(SOS_E_INVAL, "dual must be 0 (X) or 1 (Z)");
        const int N = w->N[block];
        set_active(w, true);   // the kernel reads the FP64 iterate
        double tk[2];
        hip_check(hipMemcpyAsync(tk, w->desc.tk, sizeof(tk), hipMemcpyDeviceToHost, w->stream), "copy");
        hip_check(hipStreamSynchronize(w->stream), "sync");
        if (!(tk[0] > 0.0)) throw Status(SOS_E_STATE, "tau == 0: no solution to factor (certificate state)");
        DeviceArena tmp;
        double *d_val = tmp.alloc<double>(N), *d_vec = tmp.alloc<double>((size_t)N * N);
        if (!d_val || !d_vec) throw Status(SOS_E_NOMEM, "hipMalloc failed");
        RunParams rp = single_params(w, RUN_STEP, 0, 0, w->st.tol);
        if (sos_launch_psd_factor(w->threads, rp, block, dual, d_val, d_vec, w->stream))
            throw Status(SOS_E_HIP, std::string("factor launch failed: ") + sos_launch_message());
        hip_check(hipMemcpyAsync(evals, d_val, sizeof(double) * N, hipMemcpyDeviceToHost, w->stream), "copy");
        hip_check(hipMemcpyAsync(evecs, d_vec, sizeof(double) * N * N, hipMemcpyDeviceToHost, w->stream), "copy");
        hip_check(hipStreamSynchronize(w->stream), "sync");
        if (w->st.scale_iters > 0) {   // one factor e per block: X = e X^, Z = Z^ / e
            const double e = w->Ecol[w->off_svec[block]];
            for (int j = 0; j < N; ++j) evals[j] = dual ? evals[j] / e : evals[j] * e;
        }
    });
}

int sos_get_eig_cache(const sos_work *w, int32_t block, int32_t precision, double *V, int32_t *valid) {
    if (!w || !V) return SOS_E_INVAL;
    return guarded(const_cast<sos_work *>(w), [&] {
        if (block < 0 || block >= (int)w->N.size()) throw Status(SOS_E_INVAL, "block index out of range");
        if (precision != SOS_FP64 && precision != SOS_FP32_MIXED)
            throw Status(SOS_E_INVAL, "precision must be SOS_FP64 or SOS_FP32_MIXED");
        long long off = 0;
        for (int b = 0; b < block; ++b) off += (long long)w->N[b] * w->N[b];
        const size_t nn = (size_t)w->N[block] * w->N[block];
        if (precision == SOS_FP64) {
            hip_check(hipMemcpyAsync(V, w->desc.vs64 + off, sizeof(double) * nn, hipMemcpyDeviceToHost, w->stream), "copy");
        } else {
            std::vector<float> f(nn);
            hip_check(hipMemcpyAsync(f.data(), w->desc.vs32 + off, sizeof(float) * nn, hipMemcpyDeviceToHost, w->stream),
                      "copy");
            hip_check(hipStreamSynchronize(w->stream), "sync");
            for (size_t i = 0; i < nn; ++i) V[i] = f[i];
        }
        double tk3[3];
        hip_check(hipMemcpyAsync(tk3, w->desc.tk, sizeof(tk3), hipMemcpyDeviceToHost, w->stream), "copy");
        hip_check(hipStreamSynchronize(w->stream), "sync");
        if (valid) *valid = tk3[2] != 0.0 ? 1 : 0;
    });
}

const char *sos_last_error(const sos_work *w) { return w ? w->err.c_str() : g_setup_error.c_str(); }

void sos_free(sos_work *w) {
    if (!w) return;
    if (w->stream) (void)hipStreamSynchronize(w->stream);
    else (void)hipDeviceSynchronize();
    if (w->ev0) (void)hipEventDestroy(w->ev0);
    if (w->ev1) (void)hipEventDestroy(w->ev1);
    w->mem.release();
    delete w;
}

int sos_batch_setup(int32_t count, sos_work *const *probs, const char *schedule_json, sos_batch **out) {
    if (!out || count < 1 || !probs) return SOS_E_INVAL;
    *out = nullptr;
    sos_batch *B = new (std::nothrow) sos_batch();
    if (!B) return SOS_E_NOMEM;
    int rc = guarded_b(B, [&] {
        B->count = count;
        B->probs.assign(probs, probs + count);
        for (int i = 0; i < count; ++i)
            if (!probs[i]) throw Status(SOS_E_INVAL, "null handle in batch");
        B->st = probs[0]->st;
        B->fp64 = B->st.precision == SOS_FP64;
        for (int i = 1; i < count; ++i)
            if (probs[i]->st.precision != B->st.precision) throw Status(SOS_E_INVAL, "mixed precisions in one batch");
        B->threads = (int)json_num(schedule_json, "block_threads", B->st.block_threads ? B->st.block_threads : 512);
        B->wg_per_cu = (int)json_num(schedule_json, "wg_per_cu", 1);
        B->max_sweeps = (int)json_num(schedule_json, "max_sweeps", 60);
        B->use_graph = json_num(schedule_json, "use_graph", 1) != 0.0;
        B->warm_eig = (int)json_num(schedule_json, "warm_eig", 1);
        B->eig_wave = (int)json_num(schedule_json, "eig_wave", 2);
        B->one_launch = (int)json_num(schedule_json, "one_launch", 1);
        B->rows_nmin = (int)json_num(schedule_json, "rows_nmin", kRowsNmin);
        B->jacobi_tol64 = json_num(schedule_json, "fp64_jacobi_tol", kMixedJacobiTol64);
        B->stall_checks = (int)json_num(schedule_json, "stall_checks", kStallChecks);
        B->jac_block = (int)json_num(schedule_json, "jac_block", kJacBlock);
        if (B->jac_block != 0 && B->jac_block != 8) throw Status(SOS_E_INVAL, "schedule jac_block must be 0 or 8");
        if (B->stall_checks < 1) throw Status(SOS_E_INVAL, "schedule stall_checks must be >= 1");
        if (!(B->jacobi_tol64 >= 0.0 && B->jacobi_tol64 < 1e-3))
            throw Status(SOS_E_INVAL, "schedule fp64_jacobi_tol must be in [0, 1e-3)");
        if (B->rows_nmin < 0) throw Status(SOS_E_INVAL, "schedule rows_nmin must be >= 0");
        if (B->eig_wave != 0 && B->eig_wave != 2)
            throw Status(SOS_E_INVAL, "schedule eig_wave must be 0 (lane groups) or 2 (rows over wavefronts)");
        // LDS per workgroup: what wg_per_cu resident workgroups can share (160 KiB per CU, less
        // about 10 KiB of static LDS each), unless the schedule says otherwise
        const double lds_share = std::min<double>(kLdsBudget, 163840.0 / B->wg_per_cu - 1024.0);
        B->lds_budget = (int)(json_num(schedule_json, "lds_kb", lds_share / 1024.0) * 1024.0);
        if (B->lds_budget < 0 || B->lds_budget > kLdsBudget) throw Status(SOS_E_INVAL, "schedule lds_kb out of range");
        static const char *gs_keys[7] = {"gs_n32", "gs_n64", "gs_n96", "gs_n128", "gs_n192", "gs_n256", "gs_big"};
        for (int i = 0; i < 7; ++i) {
            B->gs_bucket[i] = (int)json_num(schedule_json, gs_keys[i], kLanesPerPair[i]);
            if (B->gs_bucket[i] != 8 && B->gs_bucket[i] != 16 && B->gs_bucket[i] != 32)
                throw Status(SOS_E_INVAL, "schedule lanes per pair must be 8, 16 or 32");
        }
        if (B->threads < 64 || B->threads > 1024 || (B->threads & (B->threads - 1)))
            throw Status(SOS_E_INVAL, "schedule block_threads must be a power of two in 64..1024");
        if (B->wg_per_cu < 1 || B->wg_per_cu > 16) throw Status(SOS_E_INVAL, "schedule wg_per_cu must be 1..16");
        hip_check(hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking), "hipStreamCreate");
        std::vector<ProbDesc> descs(count);
        int mmax = 0, nxmax = 0, nmax = 1;
        long long tailmax = 0;
        std::vector<double> cost(count);
        for (int i = 0; i < count; ++i) {
            descs[i] = probs[i]->desc;
            mmax = std::max(mmax, probs[i]->m);
            nxmax = std::max(nxmax, probs[i]->nx);
            nmax = std::max(nmax, probs[i]->nmax);
            tailmax = std::max(tailmax, sos_work_tail_doubles(probs[i]->k));
            double c3 = 0.0;
            for (int N : probs[i]->N) c3 += (double)N * N * N;
            cost[i] = c3 + probs[i]->nx + probs[i]->m;
            B->max_len = std::max(B->max_len, probs[i]->nx + probs[i]->m);
        }
        B->d_out = B->mem.alloc<double>((size_t)count * SOS_OUT_N);
        if (!B->d_out) throw Status(SOS_E_NOMEM, "hipMalloc failed");
        for (int i = 0; i < count; ++i) descs[i].out = B->d_out + (size_t)i * SOS_OUT_N;
        std::vector<int> order(count);
        for (int i = 0; i < count; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
        B->d_desc = B->mem.alloc<ProbDesc>(count);
        B->d_order = B->mem.alloc<int>(count);
        B->d_counter = B->mem.alloc<int>(1);
        B->d_ts = B->mem.alloc<unsigned long long>(4);
        if (!B->d_ts) throw Status(SOS_E_NOMEM, "hipMalloc failed");
        if (!B->d_desc || !B->d_order || !B->d_counter) throw Status(SOS_E_NOMEM, "hipMalloc failed");
        hip_check(hipMemcpy(B->d_desc, descs.data(), sizeof(ProbDesc) * count, hipMemcpyHostToDevice), "copy");
        hip_check(hipMemcpy(B->d_order, order.data(), sizeof(int) * count, hipMemcpyHostToDevice), "copy");
        const int cus = device_cu_count();
        B->grid = std::min(count, cus * B->wg_per_cu);
        B->eig_ld = nmax;
        B->pair_need = 0;
        for (int i = 0; i < count; ++i)
            if (probs[i]->N.size() == 2)
                B->pair_need = std::max(B->pair_need, (int)sos_pair_need(probs[i]->N[0], probs[i]->N[1]));
        B->work_stride = (long long)(((mmax + 63) & ~63) + nxmax + 64 + tailmax) * sizeof(double);
        B->eig_stride = (long long)3 * B->eig_ld * nmax * sizeof(double) + 256;
        B->d_work = B->mem.alloc<char>((size_t)B->work_stride * B->grid);
        B->d_eig = B->mem.alloc<char>((size_t)B->eig_stride * B->grid);
        if (!B->d_work || !B->d_eig) throw Status(SOS_E_NOMEM, "hipMalloc failed");
        hip_check(hipEventCreate(&B->ev0), "event");
        hip_check(hipEventCreate(&B->ev1), "event");
        for (auto &e : B->evp) hip_check(hipEventCreate(&e), "event");
    });
    if (rc != SOS_OK) {
        g_setup_error = B->err;   // the batch does not survive: sos_last_error(NULL) has the message
        if (B->stream) (void)hipStreamDestroy(B->stream);
        delete B;
        return rc;
    }
    *out = B;
    return SOS_OK;
}

const char *sos_batch_last_error(const sos_batch *B) { return B ? B->err.c_str() : g_setup_error.c_str(); }

static RunParams batch_params(sos_batch *B, int mode, int iters, int min_iters, double tol) {
    RunParams rp{};
    rp.probs = B->d_desc;
    rp.order = B->d_order;
    rp.counter = B->d_counter;
    rp.count = B->count;
    rp.mode = mode;
    rp.iters = iters;
    rp.min_iters = min_iters;
    rp.check_every = B->st.check_every;
    rp.tol = tol;
    rp.alpha = B->st.alpha;
    rp.work = B->d_work;
    rp.work_stride = B->work_stride;
    rp.eig = B->d_eig;
    rp.eig_stride = B->eig_stride;
    rp.eig_ld = B->eig_ld;
    rp.pair_need = B->pair_need;
    rp.max_sweeps = B->max_sweeps;
    rp.warm_eig = B->warm_eig;
    rp.eig_wave = B->eig_wave;
    rp.rows_nmin = B->rows_nmin;
    rp.lds_budget = B->lds_budget;
    rp.jac_block = B->jac_block;
    for (int i = 0; i < 7; ++i) rp.gs_bucket[i] = B->gs_bucket[i];
    return rp;
}

static void enqueue_batch(sos_batch *B) {
    // the solve kernels stamp their own start / end (device wall clock), which also works in a graph
    if (sos_launch_reset(B->d_counter, B->stream, B->d_ts)) throw Status(SOS_E_HIP, std::string("reset launch failed: ") + sos_launch_message());
    if (B->fp64) {
        RunParams rp = batch_params(B, RUN_SOLVE, B->st.max_iters, 0, B->st.tol);
        rp.warm_budget = B->st.warm_budget;
        rp.ts = B->d_ts;
        if (sos_launch_admm(1, B->threads, B->grid, rp, B->stream)) throw Status(SOS_E_HIP, std::string("launch failed: ") + sos_launch_message());
    } else {
        // FP32 phase: to tol, or until it stops improving; then FP64 for the rest of the budget
        RunParams rp = batch_params(B, RUN_SOLVE, B->st.max_iters, 0, B->st.tol);
        rp.stall_checks = B->stall_checks;
        rp.warm_budget = B->st.warm_budget;
        rp.ts = B->d_ts;
        RunParams rp2 = batch_params(B, RUN_SOLVE, B->st.max_iters, B->st.polish_iters, B->st.tol);
        rp2.accumulate = 1;
        rp2.jacobi_tol = B->jacobi_tol64;
        if (B->one_launch) {
            // both phases in one launch: each problem goes on to FP64 as soon as its own
            // FP32 phase ends
            const int rc = sos_launch_admm_mixed(B->threads, B->grid, rp, rp2, B->stream);
            if (rc == 0) {
                B->used_one_launch = true;
                return;
            }
            if (rc != -1) throw Status(SOS_E_HIP, std::string("launch failed: ") + sos_launch_message());
        }
        B->used_one_launch = false;
        if (sos_launch_admm(0, B->threads, B->grid, rp, B->stream)) throw Status(SOS_E_HIP, std::string("launch failed: ") + sos_launch_message());
        if (sos_launch_cast_state(B->d_desc, nullptr, B->count, 1, B->stream, B->max_len))
            throw Status(SOS_E_HIP, std::string("cast launch failed: ") + sos_launch_message());
        if (sos_launch_reset(B->d_counter, B->stream, B->d_ts + 2)) throw Status(SOS_E_HIP, std::string("reset launch failed: ") + sos_launch_message());
        rp2.ts = B->d_ts + 2;
        if (sos_launch_admm(1, B->threads, B->grid, rp2, B->stream)) throw Status(SOS_E_HIP, std::string("launch failed: ") + sos_launch_message());
    }
}

int sos_batch_solve(sos_batch *B, sos_info *infos) {
    if (!B || !infos) return SOS_E_INVAL;
    int rc = guarded_b(B, [&] {
        // the handles' current iterate must sit in the copy the solve starts from
        for (sos_work *w : B->probs) {
            set_active(w, B->fp64 != 0);
            hip_check(hipStreamSynchronize(w->stream), "sync");
        }
        if (B->use_graph && !B->exec) {
            hip_check(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal), "capture");
            try {
                enqueue_batch(B);
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(B->stream, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            hip_check(hipStreamEndCapture(B->stream, &B->graph), "end capture");
            hip_check(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0), "instantiate");
        }
        hip_check(hipEventRecord(B->ev0, B->stream), "event");
        if (B->use_graph) hip_check(hipGraphLaunch(B->exec, B->stream), "graph launch");
        else enqueue_batch(B);
        hip_check(hipEventRecord(B->ev1, B->stream), "event");
        std::vector<double> o((size_t)B->count * SOS_OUT_N);
        hip_check(hipMemcpyAsync(o.data(), B->d_out, o.size() * sizeof(double), hipMemcpyDeviceToHost, B->stream),
                  "copy");
        hip_check(hipStreamSynchronize(B->stream), "sync");
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, B->ev0, B->ev1), "event");
        B->last_ms = ms;
        unsigned long long ts[4];
        hip_check(hipMemcpy(ts, B->d_ts, sizeof(ts), hipMemcpyDeviceToHost), "copy");
        const double khz = wall_clock_khz();
        B->phase_ms[0] = ts[1] > ts[0] ? (double)(ts[1] - ts[0]) / khz : -1.0;
        B->phase_ms[1] = (B->fp64 || B->used_one_launch) ? 0.0 : (ts[3] > ts[2] ? (double)(ts[3] - ts[2]) / khz : -1.0);
        for (int i = 0; i < B->count; ++i) {
            sos_work *w = B->probs[i];
            w->active64 = true;
            w->last_ms = ms;
            const double *oi = o.data() + (size_t)i * SOS_OUT_N;
            read_info(w, oi, &infos[i], (int)oi[SOS_OUT_TOTAL], B->fp64 ? 0 : (int)oi[SOS_OUT_ITERS]);
            if (ts[1] > ts[0]) {
                infos[i].start_ms = (oi[SOS_OUT_T_START] - (double)ts[0]) / khz;
                infos[i].end_ms = (oi[SOS_OUT_T_END] - (double)ts[0]) / khz;
            }
        }
    });
    return rc;
}

int sos_batch_reset(sos_batch *B) {
    if (!B) return SOS_E_INVAL;
    return guarded_b(B, [&] {
        for (sos_work *w : B->probs) hip_check(hipStreamSynchronize(w->stream), "sync");
        if (sos_launch_reset_state(B->d_desc, B->count, B->max_len, B->stream))
            throw Status(SOS_E_HIP, std::string("reset launch failed: ") + sos_launch_message());
        hip_check(hipStreamSynchronize(B->stream), "sync");
        for (sos_work *w : B->probs) w->active64 = true;
    });
}

int sos_batch_warm_start(sos_batch *B, const float *pred_dev, int64_t ld) {
    if (!B || !pred_dev || ld < 1) return SOS_E_INVAL;
    return guarded_b(B, [&] {
        for (sos_work *w : B->probs) {
            if (ld < (int64_t)w->nx + w->m) throw Status(SOS_E_INVAL, "prediction rows shorter than nx + m");
            hip_check(hipStreamSynchronize(w->stream), "sync");
        }
        RunParams rp = batch_params(B, RUN_SOLVE, 0, 0, B->st.tol);
        if (sos_launch_warm_start(B->fp64, B->threads, B->grid, rp, pred_dev, (long long)ld, B->stream))
            throw Status(SOS_E_HIP, std::string("warm start launch failed: ") + sos_launch_message());
        hip_check(hipStreamSynchronize(B->stream), "sync");
        for (sos_work *w : B->probs) w->active64 = B->fp64 != 0;
    });
}

int sos_batch_export_solutions(sos_batch *B, float *out_dev, int64_t ld) {
    if (!B || !out_dev || ld < 1) return SOS_E_INVAL;
    return guarded_b(B, [&] {
        bool all64 = true;
        for (sos_work *w : B->probs) {
            if (ld < (int64_t)w->nx + w->m) throw Status(SOS_E_INVAL, "output rows shorter than nx + m");
            all64 = all64 && w->active64;
            hip_check(hipStreamSynchronize(w->stream), "sync");
        }
        if (!all64) throw Status(SOS_E_STATE, "export needs the FP64 iterate (after a solve)");
        if (sos_launch_export(1, B->d_desc, B->count, out_dev, (long long)ld, B->max_len, B->stream))
            throw Status(SOS_E_HIP, std::string("export launch failed: ") + sos_launch_message());
        hip_check(hipStreamSynchronize(B->stream), "sync");
    });
}

int64_t sos_layout_size(const sos_work *w) { return w ? (int64_t)w->nx + w->m : 0; }

double sos_batch_phase_ms(const sos_batch *B, int32_t phase) {
    if (!B || phase < 0 || phase > 1) return -1.0;
    return B->phase_ms[phase];
}

double sos_batch_last_ms(const sos_batch *B) { return B ? B->last_ms : 0.0; }

void sos_batch_free(sos_batch *B) {
    if (!B) return;
    if (B->stream) (void)hipStreamSynchronize(B->stream);
    if (B->exec) (void)hipGraphExecDestroy(B->exec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    if (B->ev0) (void)hipEventDestroy(B->ev0);
    if (B->ev1) (void)hipEventDestroy(B->ev1);
    for (auto &e : B->evp)
        if (e) (void)hipEventDestroy(e);
    B->mem.release();
    if (B->stream) (void)hipStreamDestroy(B->stream);
    delete B;
}

}   // extern "C"
