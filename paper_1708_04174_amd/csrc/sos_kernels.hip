// gfx950 kernels for HSDE-ADMM on SOS-derived SDPs.
//
// One workgroup owns one problem at a time and runs whole ADMM iterations on it
// (Section IV-A: affine solve with I + Q, projection onto C, dual update).  A
// persistent grid pulls problems from a device queue, so a batch of uneven
// problems is one launch and a single problem is the same launch with one entry.
//
// Affine solve (Section IV-B), per iteration, with omega = u + v:
//   rhs      w1 = omega_xi - c omega_tau,  w2 = omega_y + b omega_tau
//   P1       x = (w2 - A w1) / d                      (row gather over CSR of A)
//   P2       q = A_f^T x ;  z = (L L^T)^{-1} q         (FP64, cached Cholesky)
//   P3       sigma_2 = x - D^{-1} A_f z                (matrix inversion lemma)
//   P4       sigma_1 = w1 + A^T sigma_2                (one gather per A_s column)
//   theta    (c^T sigma_1 - b^T sigma_2) / eta          (rank-one zeta term)
//   P5       u_hat = sigma - theta h, u_hat_tau = omega_tau + theta,
//            w = u_hat - v; free/y/tau parts of u, v written directly,
//            PSD part of w parked in v for the projection.
// The identity u_hat_tau = omega_tau + theta follows from the rank-one formula:
// zeta^T u_hat = zeta^T sigma - theta zeta^T h = zeta^T sigma / eta = theta.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "sos_internal.h"

namespace {

template <typename T> struct TS;
template <> struct TS<double> {
    __device__ static double *u(const ProbDesc &P) { return P.u64; }
    __device__ static double *v(const ProbDesc &P) { return P.v64; }
    __device__ static const double *val(const ProbDesc &P) { return P.val64; }
    __device__ static const double *colval(const ProbDesc &P) { return P.colval64; }
    __device__ static const double *fval(const ProbDesc &P) { return P.fval64; }
    __device__ static const double *frval(const ProbDesc &P) { return P.frval64; }
    __device__ static const double *dinv(const ProbDesc &P) { return P.dinv64; }
    __device__ static const double *h(const ProbDesc &P) { return P.h64; }
    __device__ static const double *b(const ProbDesc &P) { return P.b64; }
    __device__ static const double *c(const ProbDesc &P) { return P.c64; }
    __device__ static const double *cw(const ProbDesc &P) { return P.cw64; }
    static constexpr double eps = 2.220446049250313e-16;
};
template <> struct TS<float> {
    __device__ static float *u(const ProbDesc &P) { return P.u32; }
    __device__ static float *v(const ProbDesc &P) { return P.v32; }
    __device__ static const float *val(const ProbDesc &P) { return P.val32; }
    __device__ static const float *colval(const ProbDesc &P) { return P.colval32; }
    __device__ static const float *fval(const ProbDesc &P) { return P.fval32; }
    __device__ static const float *frval(const ProbDesc &P) { return P.frval32; }
    __device__ static const float *dinv(const ProbDesc &P) { return P.dinv32; }
    __device__ static const float *h(const ProbDesc &P) { return P.h32; }
    __device__ static const float *b(const ProbDesc &P) { return P.b32; }
    __device__ static const float *c(const ProbDesc &P) { return P.c32; }
    __device__ static const float *cw(const ProbDesc &P) { return P.cw32; }
    static constexpr float eps = 1.1920929e-07f;
};

__device__ __forceinline__ double wave_sum(double x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    return __shfl(x, 0, 64);
}

// Sums (a, b) over the workgroup in a fixed order (deterministic), result in every thread.
template <int NT>
__device__ __forceinline__ void block_sum2(double &a, double &b, double *s_red) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_down(a, off, 64);
        b += __shfl_down(b, off, 64);
    }
    if (lane == 0) {
        s_red[2 * wid] = a;
        s_red[2 * wid + 1] = b;
    }
    __syncthreads();
    double ta = 0.0, tb = 0.0;
    for (int w = 0; w < NW; ++w) {
        ta += s_red[2 * w];
        tb += s_red[2 * w + 1];
    }
    a = ta;
    b = tb;
    __syncthreads();
}

template <int NT>
__device__ __forceinline__ void block_sum4(double *x, double *s_red) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int i = 0; i < 4; ++i)
        for (int off = 32; off > 0; off >>= 1) x[i] += __shfl_down(x[i], off, 64);
    if (lane == 0)
        for (int i = 0; i < 4; ++i) s_red[4 * wid + i] = x[i];
    __syncthreads();
    for (int i = 0; i < 4; ++i) {
        double t = 0.0;
        for (int w = 0; w < NW; ++w) t += s_red[4 * w + i];
        x[i] = t;
    }
    __syncthreads();
}

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// z <- (L L^T)^{-1} z in FP64 by one wavefront; z lives in LDS (k entries).
// Forward substitution by columns of L, backward by rows of L (= columns of L^T).
__device__ void chol_solve_wave(const double *__restrict__ Lcol, const double *__restrict__ Lrow,
                                const double *__restrict__ Ldinv, int k, double *z) {
    const int lane = threadIdx.x & 63;
    long long cs = 0;   // start of column j in the column-packed factor
    for (int j = 0; j < k; ++j) {
        const double yj = z[j] * Ldinv[j];
        const double *col = Lcol + cs;   // L[j..k-1][j]
        for (int i = j + 1 + lane; i < k; i += 64) z[i] -= col[i - j] * yj;
        wave_sync_lds();
        if (lane == 0) z[j] = yj;
        wave_sync_lds();
        cs += k - j;
    }
    for (int i = k - 1; i >= 0; --i) {
        const double xi = z[i] * Ldinv[i];
        const double *row = Lrow + (long long)i * (i + 1) / 2;   // L[i][0..i]
        for (int j = lane; j < i; j += 64) z[j] -= row[j] * xi;
        wave_sync_lds();
        if (lane == 0) z[i] = xi;
        wave_sync_lds();
    }
}

// ----------------------------------------------------------------------------- affine step
template <typename T, int NT>
__device__ void affine_phase(const ProbDesc &P, const RunParams &rp, T *__restrict__ wy, T *__restrict__ wx,
                             double *s_z, double *s_red) {
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    constexpr int NW = NT / 64;
    const int m = P.m, nx = P.nx, k = P.k, nfree = P.nfree;
    T *__restrict__ u = TS<T>::u(P);
    T *__restrict__ v = TS<T>::v(P);
    const T *__restrict__ val = TS<T>::val(P);
    const T *__restrict__ colval = TS<T>::colval(P);
    const T *__restrict__ fval = TS<T>::fval(P);
    const T *__restrict__ frval = TS<T>::frval(P);
    const T *__restrict__ dinv = TS<T>::dinv(P);
    const T *__restrict__ h = TS<T>::h(P);
    const T *__restrict__ b = TS<T>::b(P);
    const T *__restrict__ c = TS<T>::c(P);
    const T *__restrict__ cw = TS<T>::cw(P);
    const int *__restrict__ rowptr = P.rowptr;
    const int *__restrict__ colidx = P.colidx;
    const int *__restrict__ colrow = P.colrow;

    const double tau = P.tk[0], kap = P.tk[1];
    const double wtau = tau + kap;
    const T wt = (T)wtau;
    const T *__restrict__ uy = u + nx;

    // P1: x = (w2 - A w1) / d
    for (int a = tid; a < m; a += NT) {
        T acc = uy[a] + b[a] * wt;
        const int e1 = rowptr[a + 1];
        for (int e = rowptr[a]; e < e1; ++e) {
            const int j = colidx[e];
            acc -= val[e] * (u[j] + v[j] - c[j] * wt);
        }
        wy[a] = acc * dinv[a];
    }
    __syncthreads();

    // P2: q = A_f^T x, then the cached FP64 Cholesky solve
    if (k > 0) {
        const int *__restrict__ fptr = P.fptr;
        const int *__restrict__ frow = P.frow;
        for (int j = wid; j < k; j += NW) {
            double s = 0.0;
            for (int e = fptr[j] + lane; e < fptr[j + 1]; e += 64) s += (double)fval[e] * (double)wy[frow[e]];
            s = wave_sum(s);
            if (lane == 0) s_z[j] = s;
        }
        __syncthreads();
        if (wid == 0) chol_solve_wave(P.Lcol, P.Lrow, P.Ldinv, k, s_z);
        __syncthreads();
    }

    // P3: sigma_2 = x - D^{-1} A_f z ; partial b^T sigma_2
    double bs = 0.0;
    {
        const int *__restrict__ frptr = P.frptr;
        const int *__restrict__ frcol = P.frcol;
        for (int a = tid; a < m; a += NT) {
            T s2 = wy[a];
            if (k > 0) {
                double acc = 0.0;
                for (int e = frptr[a]; e < frptr[a + 1]; ++e) acc += (double)frval[e] * s_z[frcol[e]];
                s2 = s2 - (T)(acc * (double)dinv[a]);
            }
            wy[a] = s2;
            bs += (double)b[a] * (double)s2;
        }
    }
    __syncthreads();

    // P4: sigma_1 = w1 + A^T sigma_2 ; partial c^T sigma_1
    double cs = 0.0;
    {
        const int *__restrict__ fptr = P.fptr;
        const int *__restrict__ frow = P.frow;
        for (int e = tid; e < nx; e += NT) {
            const T w1 = u[e] + v[e] - c[e] * wt;
            const int r = colrow[e];
            T s1 = w1;
            if (r >= 0) {
                s1 = w1 + colval[e] * wy[r];
            } else if (r <= -2) {
                const int j = -2 - r;
                T acc = (T)0;
                for (int i = fptr[j]; i < fptr[j + 1]; ++i) acc += fval[i] * wy[frow[i]];
                s1 = w1 + acc;
            }
            wx[e] = s1;
            cs += (double)cw[e] * (double)s1;
        }
    }
    block_sum2<NT>(cs, bs, s_red);
    const double theta = (cs - bs) / P.eta;
    const T th = (T)theta;
    const T al = (T)rp.alpha;
    const bool relax = rp.alpha != 1.0;

    // P5: u_hat, w = u_hat - v, direct updates of the free, y and tau parts
    for (int e = tid; e < nx; e += NT) {
        T uh = wx[e] - th * h[e];
        if (relax) uh = al * uh + ((T)1 - al) * u[e];
        const T w = uh - v[e];
        if (e < nfree) {
            u[e] = w;
            v[e] = (T)0;
        } else {
            v[e] = w;   // parked for the PSD projection
        }
    }
    for (int a = tid; a < m; a += NT) {
        T uh = wy[a] - th * h[nx + a];
        if (relax) uh = al * uh + ((T)1 - al) * u[nx + a];
        u[nx + a] = uh;
    }
    if (tid == 0) {
        double uht = wtau + theta;
        if (relax) uht = rp.alpha * uht + (1.0 - rp.alpha) * tau;
        const double wtt = uht - kap;
        const double tn = wtt > 0.0 ? wtt : 0.0;
        P.tk[0] = tn;
        P.tk[1] = tn - wtt;
    }
    __syncthreads();
}

// ----------------------------------------------------------------------------- PSD projection
__device__ __forceinline__ int svec_idx(int i, int j, int N) {   // i >= j
    return j * N - (j * (j - 1)) / 2 + (i - j);
}

__device__ __forceinline__ void rr_pair(int r, int kk, int M, int &p, int &q) {
    if (kk == 0) {
        p = M - 1;
        q = r;
    } else {
        p = (r + kk) % (M - 1);
        q = (r - kk + (M - 1)) % (M - 1);
    }
    if (p > q) {
        const int t = p;
        p = q;
        q = t;
    }
}

// Projects one block: the lower triangle of W is read from vs, the lower triangle of
// P_{S+}(W) is written to us and v = u - w back to vs.  Cyclic two-sided Jacobi with round-robin parallel ordering;
// A and V are N x N row-major with leading dimension ld (global scratch of this workgroup).
template <typename T, int NT>
__device__ void project_block(T *__restrict__ vs, T *__restrict__ us, int N, T *__restrict__ A,
                              T *__restrict__ V, int ld, T *s_rot, int *s_flag, double *s_red, int max_sweeps) {
    const int tid = threadIdx.x;
    if (N == 1) {
        if (tid == 0) {
            const T w = vs[0];
            const T x = w > (T)0 ? w : (T)0;
            us[0] = x;
            vs[0] = x - w;
        }
        __syncthreads();
        return;
    }
    double fro2 = 0.0, dummy = 0.0;
    for (int idx = tid; idx < N * N; idx += NT) {
        const int i = idx / N, j = idx - (idx / N) * N;
        const int a = i > j ? i : j, bb = i > j ? j : i;
        const T x = vs[svec_idx(a, bb, N)];
        A[i * ld + j] = x;
        V[i * ld + j] = (i == j) ? (T)1 : (T)0;
        fro2 += (double)x * (double)x;
    }
    block_sum2<NT>(fro2, dummy, s_red);
    const T thresh = (T)(TS<T>::eps * sqrt(fro2) / (double)N);
    const int M = N + (N & 1);
    const int H = M / 2;
    T *s_c = s_rot, *s_s = s_rot + H, *s_t = s_rot + 2 * H, *s_app = s_rot + 3 * H, *s_aqq = s_rot + 4 * H,
      *s_apq = s_rot + 5 * H;

    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        if (tid == 0) *s_flag = 0;
        __syncthreads();
        for (int r = 0; r < M - 1; ++r) {
            for (int kk = tid; kk < H; kk += NT) {
                int p, q;
                rr_pair(r, kk, M, p, q);
                T cc = (T)1, ss = (T)0, tt = (T)0, app = 0, aqq = 0, apq = 0;
                if (q < N) {
                    app = A[p * ld + p];
                    aqq = A[q * ld + q];
                    apq = A[p * ld + q];
                    if (fabs(apq) > thresh) {
                        const T th = (aqq - app) / ((T)2 * apq);
                        const T sg = th >= (T)0 ? (T)1 : (T)-1;
                        tt = sg / (fabs(th) + sqrt((T)1 + th * th));
                        cc = (T)1 / sqrt((T)1 + tt * tt);
                        ss = tt * cc;
                        *s_flag = 1;
                    }
                }
                s_c[kk] = cc;
                s_s[kk] = ss;
                s_t[kk] = tt;
                s_app[kk] = app;
                s_aqq[kk] = aqq;
                s_apq[kk] = apq;
            }
            __syncthreads();
            // A <- A J, V <- V J  (rotate column pairs)
            for (int it = tid; it < N * H; it += NT) {
                const int i = it / H, kk = it - (it / H) * H;
                const T ss = s_s[kk];
                if (ss == (T)0) continue;
                const T cc = s_c[kk];
                int p, q;
                rr_pair(r, kk, M, p, q);
                const T aip = A[i * ld + p], aiq = A[i * ld + q];
                A[i * ld + p] = cc * aip - ss * aiq;
                A[i * ld + q] = ss * aip + cc * aiq;
                const T vip = V[i * ld + p], viq = V[i * ld + q];
                V[i * ld + p] = cc * vip - ss * viq;
                V[i * ld + q] = ss * vip + cc * viq;
            }
            __syncthreads();
            // A <- J^T A  (rotate row pairs)
            for (int it = tid; it < N * H; it += NT) {
                const int kk = it / N, j = it - (it / N) * N;
                const T ss = s_s[kk];
                if (ss == (T)0) continue;
                const T cc = s_c[kk];
                int p, q;
                rr_pair(r, kk, M, p, q);
                const T apj = A[p * ld + j], aqj = A[q * ld + j];
                A[p * ld + j] = cc * apj - ss * aqj;
                A[q * ld + j] = ss * apj + cc * aqj;
            }
            __syncthreads();
            // exact 2x2 results for the rotated pairs
            for (int kk = tid; kk < H; kk += NT) {
                if (s_s[kk] == (T)0) continue;
                int p, q;
                rr_pair(r, kk, M, p, q);
                const T tt = s_t[kk], apq = s_apq[kk];
                A[p * ld + p] = s_app[kk] - tt * apq;
                A[q * ld + q] = s_aqq[kk] + tt * apq;
                A[p * ld + q] = (T)0;
                A[q * ld + p] = (T)0;
            }
            __syncthreads();
        }
        const int any = *s_flag;
        __syncthreads();
        if (!any) break;
    }
    // rebuild X = V max(L, 0) V^T over the lower triangle; u = X, v = u - w
    const int nsv = N * (N + 1) / 2;
    for (int s = tid; s < nsv; s += NT) {
        // invert svec index: column j, row i >= j
        int j = 0, rem = s;
        while (rem >= N - j) {
            rem -= N - j;
            ++j;
        }
        const int i = j + rem;
        T acc = (T)0;
        for (int kk = 0; kk < N; ++kk) {
            const T lam = A[kk * ld + kk];
            if (lam > (T)0) acc += V[i * ld + kk] * lam * V[j * ld + kk];
        }
        const T x = acc;
        const T w = vs[s];
        us[s] = x;
        vs[s] = x - w;
    }
    __syncthreads();
}

// ----------------------------------------------------------------------------- residuals (FP64)
template <typename T, int NT>
__device__ int residual_phase(const ProbDesc &P, double tol, double *s_red, int iters_done) {
    const int tid = threadIdx.x;
    const int m = P.m, nx = P.nx;
    const T *__restrict__ u = TS<T>::u(P);
    const T *__restrict__ v = TS<T>::v(P);
    const double tau = P.tk[0], kap = P.tk[1];
    // rows: |A xi - b tau|^2, |A xi|^2, b^T y
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int a = tid; a < m; a += NT) {
        double ax = 0.0;
        for (int e = P.rowptr[a]; e < P.rowptr[a + 1]; ++e) ax += P.val64[e] * (double)u[P.colidx[e]];
        const double rp = ax - P.b64[a] * tau;
        acc[0] += rp * rp;
        acc[1] += ax * ax;
        acc[2] += P.b64[a] * (double)u[nx + a];
    }
    // columns: |A^T y + z - c tau|^2 and |A^T y + z|^2 folded into acc[3] / second pass, c^T xi
    double acc2[4] = {0.0, 0.0, 0.0, 0.0};
    for (int e = tid; e < nx; e += NT) {
        const int r = P.colrow[e];
        double aty = 0.0;
        if (r >= 0) {
            aty = P.colval64[e] * (double)u[nx + r];
        } else if (r <= -2) {
            const int j = -2 - r;
            for (int i = P.fptr[j]; i < P.fptr[j + 1]; ++i) aty += P.fval64[i] * (double)u[nx + P.frow[i]];
        }
        const double g = aty + (double)v[e];
        const double rd = g - P.c64[e] * tau;
        const double wg = P.wgt64[e];
        acc2[0] += wg * rd * rd;
        acc2[1] += wg * g * g;
        acc2[2] += P.cw64[e] * (double)u[e];
    }
    acc[3] = acc2[0];
    block_sum4<NT>(acc, s_red);
    acc2[0] = 0.0;
    block_sum4<NT>(acc2, s_red);
    const double sp = acc[0], sax = acc[1], by = acc[2], sd = acc[3], saty = acc2[1], cx = acc2[2];
    int status = 0;
    double rpn = INFINITY, rdn = INFINITY, gap = INFINITY, pobj = NAN, dobj = NAN;
    if (tau > 0.0) {
        rpn = sqrt(sp) / tau / (1.0 + P.nb);
        rdn = sqrt(sd) / tau / (1.0 + P.nc);
        gap = fabs(cx - by) / tau / (1.0 + fabs(cx) / tau + fabs(by) / tau);
        pobj = cx / tau;
        dobj = by / tau;
    }
    const double mx = fmax(rpn, fmax(rdn, gap));
    if (mx <= tol) status = 1;
    else if (by > 0.0 && sqrt(saty) <= tol * by) status = 2;
    else if (cx < 0.0 && sqrt(sax) <= tol * (-cx)) status = 3;
    if (tid == 0) {
        double *o = P.out;
        o[SOS_OUT_STATUS] = status;
        o[SOS_OUT_ITERS] = iters_done;
        o[SOS_OUT_POBJ] = pobj;
        o[SOS_OUT_DOBJ] = dobj;
        o[SOS_OUT_RP] = rpn;
        o[SOS_OUT_RD] = rdn;
        o[SOS_OUT_GAP] = gap;
        o[SOS_OUT_TAU] = tau;
        o[SOS_OUT_KAPPA] = kap;
        o[SOS_OUT_CX] = cx;
        o[SOS_OUT_BY] = by;
    }
    __syncthreads();
    return status;
}

// ----------------------------------------------------------------------------- persistent driver
template <typename T, int NT>
__global__ __launch_bounds__(NT) void admm_persistent(RunParams rp) {
    __shared__ int s_idx;
    __shared__ int s_flag;
    __shared__ double s_red[4 * (NT / 64)];
    __shared__ double s_z[SOS_KMAX_LDS];
    extern __shared__ char dyn_lds[];
    T *s_rot = reinterpret_cast<T *>(dyn_lds);

    char *wbase = reinterpret_cast<char *>(rp.work) + (long long)blockIdx.x * rp.work_stride;
    char *ebase = reinterpret_cast<char *>(rp.eig) + (long long)blockIdx.x * rp.eig_stride;

    for (;;) {
        if (threadIdx.x == 0) s_idx = atomicAdd(rp.counter, 1);
        __syncthreads();
        const int idx = __builtin_amdgcn_readfirstlane(s_idx);
        __syncthreads();
        if (idx >= rp.count) break;
        const int pid = __builtin_amdgcn_readfirstlane(rp.order[idx]);
        const ProbDesc &P = rp.probs[pid];
        T *wy = reinterpret_cast<T *>(wbase);
        T *wx = wy + ((P.m + 63) & ~63);
        T *EA = reinterpret_cast<T *>(ebase);
        T *EV = EA + (long long)rp.eig_ld * P.nmax;
        T *u = TS<T>::u(P);
        T *v = TS<T>::v(P);

        int it = 0;
        int status = 0;
        while (it < rp.iters) {
            affine_phase<T, NT>(P, rp, wy, wx, s_z, s_red);
            for (int bk = 0; bk < P.nblk; ++bk) {
                const int off = P.blk_off[bk];
                project_block<T, NT>(v + off, u + off, P.blk_N[bk], EA, EV, rp.eig_ld, s_rot, &s_flag, s_red,
                                     rp.max_sweeps);
            }
            ++it;
            if (rp.mode == RUN_SOLVE && it >= rp.min_iters && (it % rp.check_every == 0 || it == rp.iters)) {
                status = residual_phase<T, NT>(P, rp.tol, s_red, it);
                if (status) break;
            }
        }
        if (rp.mode == RUN_STEP || status == 0) {
            status = residual_phase<T, NT>(P, rp.tol, s_red, it);
            if (rp.mode == RUN_SOLVE && status == 0 && threadIdx.x == 0) P.out[SOS_OUT_STATUS] = 4;
        }
        if (threadIdx.x == 0) P.out[SOS_OUT_TOTAL] = (rp.accumulate ? P.out[SOS_OUT_TOTAL] : 0.0) + it;
        __syncthreads();
    }
}

__global__ void reset_counter(int *c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0;
}

// state conversion between the FP32 and FP64 copies of u and v
__global__ void cast_state(const ProbDesc *probs, const int *ids, int count, int to64) {
    const int p = blockIdx.y;
    if (p >= count) return;
    const ProbDesc P = probs[ids ? ids[p] : p];
    const int nu = P.nx + P.m, nv = P.nx;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nu; i += gridDim.x * blockDim.x) {
        if (to64) {
            P.u64[i] = (double)P.u32[i];
            if (i < nv) P.v64[i] = (double)P.v32[i];
        } else {
            P.u32[i] = (float)P.u64[i];
            if (i < nv) P.v32[i] = (float)P.v64[i];
        }
    }
}

// cold start u = v = (0, 0, 1) for every listed problem (both precisions)
__global__ void reset_state(const ProbDesc *probs, int count) {
    const int p = blockIdx.y;
    if (p >= count) return;
    const ProbDesc &P = probs[p];
    const int nu = P.nx + P.m, nv = P.nx;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nu; i += gridDim.x * blockDim.x) {
        P.u64[i] = 0.0;
        P.u32[i] = 0.0f;
        if (i < nv) {
            P.v64[i] = 0.0;
            P.v32[i] = 0.0f;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        P.tk[0] = 1.0;
        P.tk[1] = 1.0;
    }
}

template <typename T, int NT>
int launch_t(int grid, const RunParams &rp, hipStream_t st) {
    const int H = (rp.eig_ld + 2) / 2;
    const size_t lds = sizeof(T) * 6 * (size_t)H;
    hipLaunchKernelGGL((admm_persistent<T, NT>), dim3(grid), dim3(NT), lds, st, rp);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

}   // namespace

int sos_launch_admm(int fp64, int threads, int grid, const RunParams &rp, void *stream) {
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (fp64) {
        switch (threads) {
            case 64: return launch_t<double, 64>(grid, rp, st);
            case 128: return launch_t<double, 128>(grid, rp, st);
            case 256: return launch_t<double, 256>(grid, rp, st);
            case 512: return launch_t<double, 512>(grid, rp, st);
            case 1024: return launch_t<double, 1024>(grid, rp, st);
        }
    } else {
        switch (threads) {
            case 64: return launch_t<float, 64>(grid, rp, st);
            case 128: return launch_t<float, 128>(grid, rp, st);
            case 256: return launch_t<float, 256>(grid, rp, st);
            case 512: return launch_t<float, 512>(grid, rp, st);
            case 1024: return launch_t<float, 1024>(grid, rp, st);
        }
    }
    return -1;
}

int sos_launch_reset(int *counter, void *stream) {
    hipLaunchKernelGGL(reset_counter, dim3(1), dim3(64), 0, reinterpret_cast<hipStream_t>(stream), counter);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

int sos_launch_cast_state(const ProbDesc *probs_dev, const int *ids, int count, int to64, void *stream,
                          int max_len) {
    if (count <= 0) return 0;
    int gx = (max_len + 255) / 256;
    if (gx > 64) gx = 64;
    if (gx < 1) gx = 1;
    hipLaunchKernelGGL(cast_state, dim3(gx, count), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), probs_dev,
                       ids, count, to64);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}

int sos_launch_reset_state(const ProbDesc *probs_dev, int count, int max_len, void *stream) {
    if (count <= 0) return 0;
    int gx = (max_len + 255) / 256;
    if (gx > 64) gx = 64;
    if (gx < 1) gx = 1;
    hipLaunchKernelGGL(reset_state, dim3(gx, count), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), probs_dev,
                       count);
    return hipGetLastError() == hipSuccess ? 0 : -4;
}
