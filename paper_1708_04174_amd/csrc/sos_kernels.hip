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
#include <cstdio>
#include <mutex>
#include <type_traits>
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "sos_internal.h"

// Device scratch of the entry point that allocates nothing (sos_step_static): the queue
// counter, the affine work vector and the eigensolver area of its one workgroup.  Each GPU
// the library runs on holds its own copy until the process ends.  Host code never passes
// this name to a kernel (on the host it is a stand-in, not a device address): it takes the
// address sos_static_scratch looked up for the current device.
static __device__ __align__(256) char scratch[SOS_STATIC_SCRATCH_BYTES];

namespace {

// Pointer to LDS (address space 3).  Passing LDS buffers with this type lets the compiler
// emit LDS instructions; through a generic pointer it has to use flat accesses, which
// take the vector-memory path and are several times slower for LDS data.
template <typename T> struct Lds { typedef __attribute__((address_space(3))) T type; };
template <typename T> __device__ __forceinline__ typename Lds<T>::type *as_lds(void *p) {
    return (typename Lds<T>::type *)(p);
}

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
    __device__ static double *vstore(const ProbDesc &P) { return P.vs64; }
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
    __device__ static float *vstore(const ProbDesc &P) { return P.vs32; }
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

// z <- S^{-1} z in FP64 by the workgroup; z (k entries) and part (NT entries) in LDS.
// Each row's sum is split into nseg contiguous segments of the column range, one thread
// per (row, segment); reads of S^{-1} by column are coalesced across threads (S^{-1} is
// symmetric, so column i read down is row i).  Segment sums are added in a fixed order.
template <int NT>
__device__ __forceinline__ void schur_solve(const double *__restrict__ Sinv, int k, double *z, double *part) {
    const int tid = threadIdx.x;
    const int kp = (k + 63) & ~63;
    const int nseg = kp >= NT ? 1 : NT / kp;
    for (int t = tid; t < kp * nseg; t += NT) {
        const int i = t % kp, sg = t / kp;
        double acc = 0.0;
        if (i < k) {
            // eight loads of S^{-1} in flight at a time, four partial sums
            const int j0 = sg * k / nseg, j1 = (sg + 1) * k / nseg;
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            int j = j0;
            for (; j + 8 <= j1; j += 8) {
                double sv[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) sv[q] = Sinv[(long long)(j + q) * k + i];
                a0 += sv[0] * z[j] + sv[4] * z[j + 4];
                a1 += sv[1] * z[j + 1] + sv[5] * z[j + 5];
                a2 += sv[2] * z[j + 2] + sv[6] * z[j + 6];
                a3 += sv[3] * z[j + 3] + sv[7] * z[j + 7];
            }
            for (; j < j1; ++j) a0 += Sinv[(long long)j * k + i] * z[j];
            acc = (a0 + a1) + (a2 + a3);
        }
        part[t] = acc;   // t < kp nseg <= max(kp, NT) <= 1024
    }
    __syncthreads();
    for (int i = tid; i < k; i += NT) {
        double s = 0.0;
        for (int sg = 0; sg < nseg; ++sg) s += part[sg * kp + i];
        z[i] = s;
    }
}

// Cross-lane moves within rows of 16 lanes (DPP, no LDS round trip).
enum { DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_ROW_MIRROR = 0x140, DPP_HALF_MIRROR = 0x141 };
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// Sum over an aligned group of GS (8, 16 or 32) lanes.  Each step adds a lane's partial sum
// to its partner's, partners swapping roles; since a + b == b + a exactly, every lane of
// the group ends with the bitwise-same total, so branches on it stay uniform in the group.
template <int GS, typename T>
__device__ __forceinline__ T group_allsum(T x) {
    x += dpp_mov<DPP_XOR1>(x);
    x += dpp_mov<DPP_XOR2>(x);
    x += dpp_mov<DPP_HALF_MIRROR>(x);
    if constexpr (GS >= 16) x += dpp_mov<DPP_ROW_MIRROR>(x);
    if constexpr (GS >= 32) x += __shfl_xor(x, 16, 64);
    return x;
}

// ----------------------------------------------------------------------------- affine step
// T: storage type of u, v, A, b, c, h; AT: the type the affine step computes and
// accumulates in (the storage type; a variant with FP64 arithmetic on FP32 storage
// left the FP32 residual floor unchanged, since the floor comes from the stored iterate).
template <typename T, int NT, typename AT, typename WP>
__device__ __forceinline__ void affine_core(const ProbDesc &P, const RunParams &rp, WP wy, WP wx, WP w1s, double *s_z,
                                            double *s_red) {
    // WP an LDS pointer: w1 = u + v - c wt (the columns' part of the right-hand side) is staged
    // once, and the work vectors x / sigma_2 (wy) and sigma_1 (wx) stay in LDS; else all global
    constexpr bool kStaged = !std::is_same<WP, AT *>::value;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    constexpr int NW = NT / 64;
    const int m = P.m, nx = P.nx, k = P.k, nfree = P.nfree;
    // an A_f wider than the LDS k-vector: the k-vector and partial sums live past the work vectors
    // (the staged form is only taken with the k-vector in LDS)
    if constexpr (!kStaged)
        if (k > SOS_KMAX_LDS)
            s_z = reinterpret_cast<double *>(reinterpret_cast<char *>(wy) + sizeof(double) * ((long long)((m + 63) & ~63) + nx + 64));
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
    const AT wt = (AT)wtau;
    const T *__restrict__ uy = u + nx;
    if constexpr (kStaged) {
        for (int e = tid; e < nx; e += NT) w1s[e] = (AT)u[e] + (AT)v[e] - (AT)c[e] * wt;
        __syncthreads();
    }
    // the column's part (u + v - c wt) at column j, staged or read
    auto w1 = [&](int j) -> AT {
        if constexpr (kStaged) return w1s[j];
        else return (AT)u[j] + (AT)v[j] - (AT)c[j] * wt;
    };

    // P1: x = (w2 - A w1) / d.  A row has up to a few tens of nonzeros, each a chain of two
    // dependent loads (column index, then u, v, c there): four entries in flight at a time
    for (int a = tid; a < m; a += NT) {
        AT acc = (AT)uy[a] + (AT)b[a] * wt;
        AT acc1 = (AT)0, acc2 = (AT)0, acc3 = (AT)0;
        const int e1 = rowptr[a + 1];
        int e = rowptr[a];
        for (; e + 4 <= e1; e += 4) {
            const int j0 = colidx[e], j1 = colidx[e + 1], j2 = colidx[e + 2], j3 = colidx[e + 3];
            acc -= (AT)val[e] * w1(j0);
            acc1 -= (AT)val[e + 1] * w1(j1);
            acc2 -= (AT)val[e + 2] * w1(j2);
            acc3 -= (AT)val[e + 3] * w1(j3);
        }
        for (; e < e1; ++e) {
            const int j = colidx[e];
            acc -= (AT)val[e] * w1(j);
        }
        wy[a] = (acc + acc1 + (acc2 + acc3)) * (AT)dinv[a];
    }
    __syncthreads();

    // P2: q = A_f^T x, then z = S^{-1} q in FP64.  A column of A_f has a few nonzeros, so a
    // group of 8 lanes takes one column (DPP reduction within the group) and NT / 8 columns
    // are in flight at once: each column is a chain of dependent loads (fptr, frow, x)
    if (k > 0) {
        const int *__restrict__ fptr = P.fptr;
        const int *__restrict__ frow = P.frow;
        const int grp = tid >> 3, gl = tid & 7;
        for (int j = grp; j < k; j += NT / 8) {
            double s = 0.0;
            const int e1 = fptr[j + 1];
            for (int e = fptr[j] + gl; e < e1; e += 8) s += (double)fval[e] * (double)wy[frow[e]];
            s = group_allsum<8>(s);
            if (gl == 0) s_z[j] = s;
        }
        __syncthreads();
        schur_solve<NT>(P.Sinv, k, s_z, k <= SOS_KMAX_LDS ? s_z + SOS_KMAX_LDS : s_z + ((k + 63) & ~63));
        __syncthreads();
    }

    // P3: sigma_2 = x - D^{-1} A_f z ; partial b^T sigma_2
    double bs = 0.0;
    {
        const int *__restrict__ frptr = P.frptr;
        const int *__restrict__ frcol = P.frcol;
        for (int a = tid; a < m; a += NT) {
            AT s2 = wy[a];
            if (k > 0) {
                double acc = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
                const int e1 = frptr[a + 1];
                int e = frptr[a];
                for (; e + 4 <= e1; e += 4) {
                    acc += (double)frval[e] * s_z[frcol[e]];
                    acc1 += (double)frval[e + 1] * s_z[frcol[e + 1]];
                    acc2 += (double)frval[e + 2] * s_z[frcol[e + 2]];
                    acc3 += (double)frval[e + 3] * s_z[frcol[e + 3]];
                }
                for (; e < e1; ++e) acc += (double)frval[e] * s_z[frcol[e]];
                s2 = s2 - (AT)(((acc + acc1) + (acc2 + acc3)) * (double)dinv[a]);
            }
            wy[a] = s2;
            bs += (double)b[a] * (double)s2;
        }
    }
    __syncthreads();

    // P4: sigma_1 = w1 + A^T sigma_2 ; partial c^T sigma_1.  Columns with at most one nonzero
    // (A_s, empty) one per thread; the columns of A_f a group of 8 lanes each (as in P2)
    double cs = 0.0;
    {
        for (int e = tid; e < nx; e += NT) {
            const int r = colrow[e];
            if (r <= -2) continue;
            const AT we = w1(e);
            const AT s1 = r >= 0 ? we + (AT)colval[e] * wy[r] : we;
            wx[e] = s1;
            cs += (double)cw[e] * (double)s1;
        }
        const int *__restrict__ fptr = P.fptr;
        const int *__restrict__ frow = P.frow;
        const int *__restrict__ fcol = P.fcol;
        const int grp = tid >> 3, gl = tid & 7;
        for (int j = grp; j < k; j += NT / 8) {
            AT acc = (AT)0;
            const int i1 = fptr[j + 1];
            for (int i = fptr[j] + gl; i < i1; i += 8) acc += (AT)fval[i] * wy[frow[i]];
            acc = group_allsum<8>(acc);
            if (gl == 0) {
                const int e = fcol[j];
                const AT s1 = w1(e) + acc;
                wx[e] = s1;
                cs += (double)cw[e] * (double)s1;
            }
        }
    }
    block_sum2<NT>(cs, bs, s_red);
    const double theta = (cs - bs) / P.eta;
    const AT th = (AT)theta;
    const AT al = (AT)rp.alpha;
    const bool relax = rp.alpha != 1.0;

    // P5: u_hat, w = u_hat - v, direct updates of the free, y and tau parts
    for (int e = tid; e < nx; e += NT) {
        AT uh = wx[e] - th * (AT)h[e];
        if (relax) uh = al * uh + ((AT)1 - al) * (AT)u[e];
        const AT w = uh - (AT)v[e];
        if (e < nfree) {
            u[e] = (T)w;
            v[e] = (T)0;
        } else {
            v[e] = (T)w;   // parked for the PSD projection
        }
    }
    for (int a = tid; a < m; a += NT) {
        AT uh = wy[a] - th * (AT)h[nx + a];
        if (relax) uh = al * uh + ((AT)1 - al) * (AT)u[nx + a];
        u[nx + a] = (T)uh;
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

// The affine step of one problem by the workgroup.  wy, wx: its global work vectors; lds: the
// LDS area the eigensolver leaves free during the step (nullptr if none) and lds_cap its bytes.
// When x / sigma_2 (m), sigma_1 (nx) and the staged column part (nx) fit there, they live in LDS
// (the arithmetic is the same; only where the vectors live changes).
template <typename T, int NT, typename AT>
__device__ __noinline__ void affine_phase(const ProbDesc &P, const RunParams &rp, AT *__restrict__ wy, AT *__restrict__ wx,
                                          double *s_z, double *s_red, char *lds = nullptr, long long lds_cap = 0) {
    typedef typename Lds<AT>::type *LW;
    const long long mp = (P.m + 3) & ~3LL, nxp = (P.nx + 3) & ~3LL;
    if (lds && P.k <= SOS_KMAX_LDS && (long long)sizeof(AT) * (mp + 2 * nxp) <= lds_cap) {
        LW l = as_lds<AT>(lds);
        affine_core<T, NT, AT, LW>(P, rp, l, l + mp, l + mp + nxp, s_z, s_red);
    } else {
        affine_core<T, NT, AT, AT *>(P, rp, wy, wx, nullptr, s_z, s_red);
    }
}

// ----------------------------------------------------------------------------- PSD projection
__device__ __forceinline__ int svec_idx(int i, int j, int N) {   // i >= j
    return j * N - (j * (j - 1)) / 2 + (i - j);
}

// Round-robin (circle) pairing: in round r of M - 1 rounds, pair kk is (p, q), p < q;
// every index of 0..M-1 appears once per round and every unordered pair once per sweep.
__device__ __forceinline__ void rr_pair(int r, int kk, int M, int &p, int &q) {
    if (kk == 0) {
        p = M - 1;
        q = r;
    } else {   // (r + kk) mod (M - 1) and (r - kk) mod (M - 1), with 0 <= r < M - 1, 0 < kk < M / 2
        p = r + kk;
        if (p >= M - 1) p -= M - 1;
        q = r - kk;
        if (q < 0) q += M - 1;
    }
    if (p > q) {
        const int t = p;
        p = q;
        q = t;
    }
}

// lanes per column pair for a block of size N: the schedule's choice for N's bucket
// (buckets N < 32, 64, 96, 128, 192, 256, and above)
// Leading dimension of G and V when both sit in LDS: the smallest ld >= N with ld = 8 mod 16.
// A wavefront's groups read columns p, p - 1, ..., p - 7 of one round (8 consecutive rows
// each); with this stride the 8 column starts fall 8 banks apart modulo 64 banks (4-byte
// elements), and 16 apart within each half-wavefront for 8-byte elements, so the groups'
// reads of a column do not share banks.
__host__ __device__ __forceinline__ int lds_ld(int N) { return SOS_LDS_LD(N); }

__device__ __forceinline__ int lanes_per_pair(const RunParams &rp, int N) {
    const int b = N < 32 ? 0 : N < 64 ? 1 : N < 96 ? 2 : N < 128 ? 3 : N < 192 ? 4 : N < 256 ? 5 : 6;
    const int g = rp.gs_bucket[b];
    return (g == 8 || g == 32) ? g : 16;
}

struct EigScratch {
    typename Lds<int>::type *s_flag;
    typename Lds<int>::type *s_sweeps;    // Jacobi sweeps run (diagnostic)
    double *s_red;
    double jtol;                          // relative coupling a pair must exceed to rotate (0: 16 eps)
};

// Relative rotation threshold of the Jacobi sweeps: 16 eps of the type by default.
template <typename T>
__device__ __forceinline__ T jacobi_tol(double jtol) { return (T)(jtol > 0.0 ? jtol : 16.0 * TS<T>::eps); }

// Wave sum with lane 0's result broadcast, so every lane holds the bitwise-same value
// (a butterfly would leave lane-dependent rounding, and branches on it must not diverge).
__device__ __forceinline__ double wave_allsum(double x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    return __shfl(x, 0, 64);
}
__device__ __forceinline__ float wave_allsum(float x) {
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    return __shfl(x, 0, 64);
}

// Absolute floor of the coupling a pair must have to be rotated, in units of eps |W|_F
// times the larger column norm.  Columns whose norms sit near the rounding level of W keep
// picking up coupling of that size from every rotation of their partners (about eps |W|
// times sqrt(N) accumulated over a sweep); a floor below that level makes them trade
// rounding noise sweep after sweep.  Left unrotated, such a pair perturbs |W| by about
// this floor, i.e. at the rounding level of W.
__device__ __forceinline__ double jacobi_atol_factor(int N) { return 4.0 * sqrt((double)N); }

// Jacobi rotation for the column pair with squared norms al, be and inner product ga:
// rotate only while the pair is coupled beyond rounding, relative to both columns
// (ga^2 > tol2 al be) and absolutely (ga^2 > atol2 max(al, be)); then t = tan(theta) of the
// smaller of the two angles that make the pair orthogonal, t = 2 ga sgn(d) / (|d| + hypot(d, 2 ga))
// with d = be - al, c = 1 / sqrt(1 + t^2), s = c t.  FP32 uses the native reciprocal and
// root instructions (1 ulp; c^2 + s^2 = 1 to that level), FP64 the IEEE operations.
template <typename T>
__device__ __forceinline__ bool jacobi_rot(T al, T be, T ga, T tol2, T atol2, T &c, T &s);
template <>
__device__ __forceinline__ bool jacobi_rot<float>(float al, float be, float ga, float tol2, float atol2, float &c,
                                                  float &s) {
    const float g2 = ga * ga;
    if (!(g2 > tol2 * (al * be)) || !(g2 > atol2 * (al > be ? al : be))) return false;
    const float d = be - al;
    const float h = __builtin_amdgcn_sqrtf(d * d + 4.0f * g2);
    float t = 2.0f * ga * __builtin_amdgcn_rcpf(fabsf(d) + h);
    if (d < 0.0f) t = -t;
    c = __builtin_amdgcn_rsqf(1.0f + t * t);
    s = c * t;
    return true;
}
template <>
__device__ __forceinline__ bool jacobi_rot<double>(double al, double be, double ga, double tol2, double atol2,
                                                   double &c, double &s) {
    const double g2 = ga * ga;
    if (!(g2 > tol2 * (al * be)) || !(g2 > atol2 * (al > be ? al : be))) return false;
    // the hardware reciprocal and reciprocal square root, each refined by two Newton steps
    // (quadratic convergence: far below 1 ulp of error left), instead of the IEEE-exact
    // square root and divisions with their range scaling: the arguments here are positive,
    // finite and far from the extremes
    const double d = be - al;
    const double x = d * d + 4.0 * g2;   // > 0, since g2 > 0
    double r = __builtin_amdgcn_rsq(x);
    r = fma(0.5 * r, fma(-x * r, r, 1.0), r);
    r = fma(0.5 * r, fma(-x * r, r, 1.0), r);
    const double den = fabs(d) + x * r;   // |d| + sqrt(d^2 + 4 g^2)
    double inv = __builtin_amdgcn_rcp(den);
    inv = fma(inv, fma(-den, inv, 1.0), inv);
    inv = fma(inv, fma(-den, inv, 1.0), inv);
    double t = 2.0 * ga * inv;
    if (d < 0.0) t = -t;
    const double y = 1.0 + t * t;
    double cr = __builtin_amdgcn_rsq(y);
    cr = fma(0.5 * cr, fma(-y * cr, cr, 1.0), cr);
    cr = fma(0.5 * cr, fma(-y * cr, cr, 1.0), cr);
    c = cr;
    s = cr * t;
    return true;
}

// One-sided Jacobi rotation of the column pair (p, q) of G (and of V) by a group of GS
// lanes, each lane holding RPL rows of the columns in registers (N <= RPL GS).  V in global
// memory is read up front, so that its reads are in flight during the reduction and the
// rotation decision; V in LDS is read only once a rotation is decided (most pairs of a
// warm-started sweep are not rotated, and LDS bandwidth is what a round spends).  Returns
// as os_rotate_pair.
template <typename T, int GS, int RPL, typename GP, typename VP>
__device__ __forceinline__ int rotate_pair_regs(GP gp, GP gq, VP vp, VP vq, int N, T tol, T atol) {
    constexpr bool kPrefetchV = !std::is_same<VP, typename Lds<T>::type *>::value;
    const int gl = threadIdx.x & (GS - 1);
    T xp[RPL], xq[RPL], yp[RPL], yq[RPL];
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
        const int i = gl + GS * t;
        xp[t] = i < N ? gp[i] : (T)0;
        xq[t] = i < N ? gq[i] : (T)0;
        if (kPrefetchV) {
            yp[t] = i < N ? vp[i] : (T)0;
            yq[t] = i < N ? vq[i] : (T)0;
        }
    }
    T al = 0, be = 0, ga = 0;
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
        al += xp[t] * xp[t];
        be += xq[t] * xq[t];
        ga += xp[t] * xq[t];
    }
    al = group_allsum<GS>(al);
    be = group_allsum<GS>(be);
    ga = group_allsum<GS>(ga);
    T cc, ss;
    if (!jacobi_rot<T>(al, be, ga, tol * tol, atol * atol, cc, ss)) return 0;
    if (!kPrefetchV) {
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
            const int i = gl + GS * t;
            yp[t] = i < N ? vp[i] : (T)0;
            yq[t] = i < N ? vq[i] : (T)0;
        }
    }
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
        const int i = gl + GS * t;
        if (i < N) {
            gp[i] = cc * xp[t] - ss * xq[t];
            gq[i] = ss * xp[t] + cc * xq[t];
            vp[i] = cc * yp[t] - ss * yq[t];
            vq[i] = ss * yp[t] + cc * yq[t];
        }
    }
    return ga * ga > tol * (al * be) ? 2 : 1;
}

// One-sided Jacobi rotation of the column pair (p, q) of G (and of V) by a group of GS
// lanes; makes g_p and g_q orthogonal.  Returns 0 if no rotation was applied, 1 for a
// rotation of relative coupling at most sqrt(tol), 2 for a larger one.  Blocks of up to
// 16 GS rows keep the columns in registers (4, 8, 12 or 16 rows per lane, the fewest that
// hold N); larger ones stream them.
template <typename T, int GS, typename GP, typename VP>
__device__ __forceinline__ int os_rotate_pair(GP G, int ldg, VP V, int ldv, int N, int p, int q, T tol, T atol) {
    const int gl = threadIdx.x & (GS - 1);
    GP gp = G + (long long)p * ldg, gq = G + (long long)q * ldg;
    VP vp = V + (long long)p * ldv, vq = V + (long long)q * ldv;
    if (N <= 4 * GS) return rotate_pair_regs<T, GS, 4>(gp, gq, vp, vq, N, tol, atol);
    if (N <= 8 * GS) return rotate_pair_regs<T, GS, 8>(gp, gq, vp, vq, N, tol, atol);
    if (N <= 12 * GS) return rotate_pair_regs<T, GS, 12>(gp, gq, vp, vq, N, tol, atol);
    if (N <= 16 * GS) return rotate_pair_regs<T, GS, 16>(gp, gq, vp, vq, N, tol, atol);
    T al = 0, be = 0, ga = 0;
    for (int i = gl; i < N; i += GS) {
        const T a = gp[i], b = gq[i];
        al += a * a;
        be += b * b;
        ga += a * b;
    }
    al = group_allsum<GS>(al);
    be = group_allsum<GS>(be);
    ga = group_allsum<GS>(ga);
    T cc, ss;
    if (!jacobi_rot<T>(al, be, ga, tol * tol, atol * atol, cc, ss)) return 0;
    for (int i = gl; i < N; i += GS) {
        const T a = gp[i], b = gq[i];
        gp[i] = cc * a - ss * b;
        gq[i] = ss * a + cc * b;
        const T c = vp[i], d = vq[i];
        vp[i] = cc * c - ss * d;
        vq[i] = ss * c + cc * d;
    }
    return ga * ga > tol * (al * be) ? 2 : 1;
}

// ----------------------------------------------------------------------------- MFMA tiles
// The projection's two dense products run on the matrix cores, one 16 x 16 output tile per
// wavefront and 16 x 16 x 4 MFMA steps (FP32 MFMA with FP32 accumulation in the FP32 phase,
// FP64 MFMA in the FP64 phase).  Operand layout of one step D += A B (A 16 x 4, B 4 x 16):
// lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]; its four results r = 0..3 are
// D[row(l / 16, r)][l % 16], with row = 4 (l / 16) + r for FP32 and l / 16 + 4 r for FP64
// (layouts measured on gfx950).  Entries outside the N x N matrices are zero.
template <typename T> struct Mma;
template <> struct Mma<float> {
    typedef float acc __attribute__((ext_vector_type(4)));
    __device__ static __forceinline__ acc step(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int lg, int r) { return 4 * lg + r; }
};
template <> struct Mma<double> {
    typedef double acc __attribute__((ext_vector_type(4)));
    __device__ static __forceinline__ acc step(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int lg, int r) { return lg + 4 * r; }
};

// Output tiles a wavefront may hold in registers while W, stored where G goes, is still read.
constexpr int kMfmaHold = 8;

// G = W V for column-major N x N matrices, W symmetric.  In a chunk of 16 values of the
// summation index, lane group g = l / 16 takes k = k0 + 4 g + t in step t = 0..3, so each lane
// reads four consecutive entries of a column of V (and, W being symmetric, of a column of W)
// per chunk.  W in global memory (wglobal) is read by rows instead, W[k][i] for consecutive i
// across lanes, which keeps those reads coalesced.  hold: W occupies G's storage; every tile
// stays in registers until all wavefronts have finished reading W (needs at most kMfmaHold
// tiles per wavefront).  The caller ends with a barrier before G is read.
// Tiles go to workers w0 = 0..nw-1 (wavefronts; the default is this workgroup's, a grid-wide
// numbering spreads them over several workgroups), tile w0, w0 + nw, ...
template <typename T, int NT, typename WP, typename VP, typename GP>
__device__ __forceinline__ void mfma_wv(WP W, int ldw, bool wglobal, VP V, int ldv, GP G, int ldg, int N,
                                        bool hold, int w0 = -1, int nw = 0) {
    typedef typename Mma<T>::acc AC;
    const int lane = threadIdx.x & 63;
    const int wid = w0 >= 0 ? w0 : (int)(threadIdx.x >> 6);
    const int NW = w0 >= 0 ? nw : NT / 64;
    const int li = lane & 15, lg = lane >> 4;
    const int nt = (N + 15) >> 4, ntt = nt * nt;
    for (int base = 0; base < ntt; base += NW * kMfmaHold) {
        AC acc[kMfmaHold];
#pragma unroll
        for (int q = 0; q < kMfmaHold; ++q) {
            acc[q] = (AC)(T)0;
            const int tile = base + q * NW + wid;   // wavefront-uniform
            if (tile >= ntt) continue;
            const int i0 = (tile % nt) * 16, j0 = (tile / nt) * 16;
            const int i = i0 + li, j = j0 + li;   // this lane's row of A, column of B
            const bool iok = i < N, jok = j < N;
            for (int k0 = 0; k0 < N; k0 += 16) {
                const int kb = k0 + 4 * lg;
                T a[4], b[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const bool kok = kb + t < N;
                    a[t] = (iok && kok) ? (wglobal ? W[(long long)(kb + t) * ldw + i] : W[(long long)i * ldw + kb + t])
                                        : (T)0;
                    b[t] = (jok && kok) ? V[(long long)j * ldv + kb + t] : (T)0;
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) acc[q] = Mma<T>::step(a[t], b[t], acc[q]);
            }
        }
        if (hold) __syncthreads();   // every read of W done before G, its storage, is written
#pragma unroll
        for (int q = 0; q < kMfmaHold; ++q) {
            const int tile = base + q * NW + wid;
            if (tile >= ntt) continue;
            const int i0 = (tile % nt) * 16, j = (tile / nt) * 16 + li;
            if (j >= N) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + Mma<T>::row(lg, r);
                if (i < N) G[(long long)j * ldg + i] = acc[q][r];
            }
        }
    }
}

// Lower triangle of (W + V Sigma V^T) / 2 into us, and v = u - w into vs (both packed lower
// triangles by columns; vs holds w on entry).  Tiles on and below the diagonal, one per
// wavefront at a time; step t covers V's columns k0 + l / 16.
template <typename T, int NT, typename VP, typename SP>
__device__ __forceinline__ void mfma_rebuild(VP V, int ldv, SP sig, int N, T *__restrict__ vs, T *__restrict__ us,
                                             int w0 = -1, int nw = 0) {
    typedef typename Mma<T>::acc AC;
    const int lane = threadIdx.x & 63;
    const int wid = w0 >= 0 ? w0 : (int)(threadIdx.x >> 6);
    const int NW = w0 >= 0 ? nw : NT / 64;
    const int li = lane & 15, lg = lane >> 4;
    const int nt = (N + 15) >> 4, ntri = nt * (nt + 1) / 2;
    for (int tile = wid; tile < ntri; tile += NW) {
        int ta = 0, rem = tile;
        while (rem > ta) {
            rem -= ta + 1;
            ++ta;
        }
        const int i0 = ta * 16, j0 = rem * 16;   // tile row ta >= tile column rem
        const int i = i0 + li, j = j0 + li;
        const bool iok = i < N, jok = j < N, diag = ta == rem;
        AC acc = (AC)(T)0;
        int k0 = 0;
        for (; k0 + 16 <= N; k0 += 16) {
            T a[4], b[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int k = k0 + 4 * t + lg;
                const T vi = iok ? V[(long long)k * ldv + i] : (T)0;
                b[t] = diag ? vi : (jok ? V[(long long)k * ldv + j] : (T)0);
                a[t] = vi * sig[k];
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) acc = Mma<T>::step(a[t], b[t], acc);
        }
        for (; k0 < N; k0 += 4) {
            const int k = k0 + lg;
            const bool kok = k < N;
            const T vi = (iok && kok) ? V[(long long)k * ldv + i] : (T)0;
            const T b = diag ? vi : ((jok && kok) ? V[(long long)k * ldv + j] : (T)0);
            const T a = kok ? vi * sig[k] : (T)0;
            acc = Mma<T>::step(a, b, acc);
        }
        if (!jok) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int ii = i0 + Mma<T>::row(lg, r);
            if (ii < N && ii >= j) {
                const int s = svec_idx(ii, j, N);
                const T w = vs[s];
                const T x = (T)0.5 * (w + acc[r]);
                us[s] = x;
                vs[s] = x - w;
            }
        }
    }
}

// Projects one block: the lower triangle of W is read from vs, the lower triangle of
// P_{S+}(W) is written to us and v = u - w back to vs.
// P_{S+}(W) = (W + |W|) / 2 with |W| = V Sigma V^T: one-sided (Hestenes) Jacobi makes the
// columns of G = W V mutually orthogonal by plane rotations applied to G and V alike;
// then V holds eigenvectors of W and Sigma = diag(|g_j|) = |eigenvalues| (for a symmetric W
// the right singular vectors are eigenvectors, and the formula holds within any group of
// equal |lambda|).  Round-robin parallel ordering, a group of lanes per column pair, one
// barrier per round.  With a cached V from the previous ADMM iteration (warm) the sweeps
// start from G = W V, which is nearly orthogonal once the iterates settle.
// G, V: column-major N x N (column j at j*ld), in LDS or global scratch; Tm: N x N global.
// Between Jacobi rounds, within a wavefront: a code-motion barrier only.  A wavefront's LDS
// operations are performed in issue order, so a read issued after a write (by any lane of
// the same wavefront) returns the written value without waiting for the write to finish.
__device__ __forceinline__ void wave_order() { __builtin_amdgcn_wave_barrier(); }

// Exchange between the 8-lane groups g and g ^ B of a wavefront (lane l takes lane l ^ 8B): for
// B = 1 inside each row of 16 lanes, a DPP move (row_ror:8 swaps the row's halves) with no LDS
// traffic; for B = 2 and 4 across rows, an LDS permute.  (The gfx950 permlane swaps in place of
// the permutes measured slower.)
template <int B>
__device__ __forceinline__ unsigned group_xchg(unsigned x) {
    static_assert(B == 1 || B == 2 || B == 4, "groups g and g ^ B");
    if constexpr (B == 1) return (unsigned)__builtin_amdgcn_mov_dpp((int)x, 0x128, 0xF, 0xF, true);
    else return (unsigned)__shfl_xor((int)x, 8 * B, 64);
}
template <int B>
__device__ __forceinline__ float group_xchg(float x) {
    return __uint_as_float(group_xchg<B>(__float_as_uint(x)));
}
template <int B>
__device__ __forceinline__ double group_xchg(double x) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = group_xchg<B>((unsigned)u), hi = group_xchg<B>((unsigned)(u >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The 64 cross pairs of blocks P and Q (8 columns each) by one wavefront, columns in registers:
// group g keeps column 8P + g of G and V (RPL rows per lane) for the whole round; in step s it
// holds column 8Q + (g ^ gray(s)) of Q, gray(s) = s ^ (s >> 1) (0, 1, 3, 2, 6, 7, 5, 4: every
// column of Q once, and the groups' columns distinct in every step).  Consecutive Gray codes
// differ in one bit, so between steps each group exchanges its column of Q with the group
// g ^ 1 (four of the seven hand-overs, DPP moves inside rows of 16 lanes), g ^ 2 or g ^ 4 (LDS
// permutes); after the last step group g writes back column 8Q + (g ^ 4).  The 8 steps are
// unrolled, so each hand-over's kind is fixed at compile time.  With VQ the V column of Q travels
// the same way; without, it stays in LDS and only a step that rotates reads and writes it (the
// group that owns it next is in the same wavefront, whose LDS accesses are performed in order):
// fewer lane moves when few pairs rotate, LDS traffic when many do.  Columns and rows at or past N
// are zero (their products vanish; such columns are never rotated).  Returns 1 if a rotation had
// relative coupling above sqrt(tol).
template <typename T, int RPL, bool VQ, typename LP>
__device__ __forceinline__ int cross_block_regs(LP G, LP V, int ld, int N, int P, int Q, T tol, T atol) {
    const int gl = threadIdx.x & 7, grp = (threadIdx.x & 63) >> 3;
    const int p = P * 8 + grp;
    const bool pok = p < N;
    const int q0 = Q * 8 + grp;
    T xp[RPL], yp[RPL], xq[RPL], yq[VQ ? RPL : 1];
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
        const int i = gl + 8 * t;
        const bool iok = i < N;
        xp[t] = (pok && iok) ? G[(long long)p * ld + i] : (T)0;
        yp[t] = (pok && iok) ? V[(long long)p * ld + i] : (T)0;
        xq[t] = (q0 < N && iok) ? G[(long long)q0 * ld + i] : (T)0;
        if constexpr (VQ) yq[t] = (q0 < N && iok) ? V[(long long)q0 * ld + i] : (T)0;
    }
    int big = 0;
    const T tol2 = tol * tol, atol2 = atol * atol;
#pragma unroll
    for (int st = 0; st < 8; ++st) {
        T al = 0, be = 0, ga = 0;
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
            al += xp[t] * xp[t];
            be += xq[t] * xq[t];
            ga += xp[t] * xq[t];
        }
        al = group_allsum<8>(al);
        be = group_allsum<8>(be);
        ga = group_allsum<8>(ga);
        T cc, ss;
        if (jacobi_rot<T>(al, be, ga, tol2, atol2, cc, ss)) {   // then both columns are nonzero, so below N
            if (ga * ga > tol * (al * be)) big = 1;
            const long long qo = (long long)(Q * 8 + (grp ^ st ^ (st >> 1))) * ld;
#pragma unroll
            for (int t = 0; t < RPL; ++t) {
                const T a = xp[t], b = xq[t];
                xp[t] = cc * a - ss * b;
                xq[t] = ss * a + cc * b;
                if constexpr (VQ) {
                    const T c = yp[t], d = yq[t];
                    yp[t] = cc * c - ss * d;
                    yq[t] = ss * c + cc * d;
                } else {
                    const int i = gl + 8 * t;
                    if (i < N) {
                        const T c = yp[t], d = V[qo + i];
                        yp[t] = cc * c - ss * d;
                        V[qo + i] = ss * c + cc * d;
                    }
                }
            }
        }
        wave_order();
        // gray(st) ^ gray(st + 1), the lowest set bit of st + 1 (none after the last step)
        const int bit = (st + 1) & -(st + 1);
#pragma unroll
        for (int t = 0; t < RPL; ++t) {
            if (bit == 1) {
                xq[t] = group_xchg<1>(xq[t]);
                if constexpr (VQ) yq[t] = group_xchg<1>(yq[t]);
            } else if (bit == 2) {
                xq[t] = group_xchg<2>(xq[t]);
                if constexpr (VQ) yq[t] = group_xchg<2>(yq[t]);
            } else if (bit == 4) {
                xq[t] = group_xchg<4>(xq[t]);
                if constexpr (VQ) yq[t] = group_xchg<4>(yq[t]);
            }
        }
    }
    const int ql = Q * 8 + (grp ^ 4);
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
        const int i = gl + 8 * t;
        if (i < N) {
            if (pok) {
                G[(long long)p * ld + i] = xp[t];
                V[(long long)p * ld + i] = yp[t];
            }
            if (ql < N) {
                G[(long long)ql * ld + i] = xq[t];
                if constexpr (VQ) V[(long long)ql * ld + i] = yq[t];
            }
        }
    }
    return big;
}

// Block-cyclic sweep of the lane-group form (G and V in LDS): the columns form blocks of 8;
// first every block's own pairs (two blocks per wavefront, four 8-lane groups each per round of
// the block's round-robin), then block rounds over pairs of blocks (round-robin of the blocks), a
// wavefront per block pair covering its 64 cross pairs in 8 steps of 8 disjoint pairs (group g
// rotates columns 8P + g and 8Q + (g + s) mod 8 in step s, or 8Q + (g ^ gray(s)) in the register
// rounds).  Every column pair meets once per
// sweep, as in the cyclic order, but only the block rounds end in a workgroup barrier (N / 8 + 1
// per sweep instead of N - 1): inside a block round the wavefront's own LDS order suffices.
// Up to N = 128 a cross round keeps its columns in registers (cross_block_regs, 4 to 16 rows per
// lane): G and V up to N = 32, G alone above; larger blocks take the LDS steps.
// Returns 1 if some rotation had relative coupling above sqrt(tol).
template <typename T, int NT, typename LP>
__device__ __forceinline__ int block_cyclic_sweep(LP G, LP V, int ld, int N, T tol, T atol) {
    constexpr int NW = NT / 64;
    const int wid = threadIdx.x >> 6, grp = (threadIdx.x & 63) >> 3;
    const int nb = (N + 7) >> 3, nbp = nb + (nb & 1);
    int big = 0;
    // in-block pairs: a block has at most 4 disjoint pairs per round, so a wavefront takes two
    // blocks at once, one per half (lane groups 0-3 and 4-7)
    const int half = grp >> 2, hg = grp & 3;
    for (int B = 2 * wid + half; B - half < nb; B += 2 * NW) {
        const int c0 = B * 8, c = B < nb ? (N - c0 < 8 ? N - c0 : 8) : 0, M = c + (c & 1);
        for (int r = 0; r < 7; ++r) {   // the rounds of a full block; shorter blocks idle
            if (r < M - 1 && hg < M / 2) {
                int p, q;
                rr_pair(r, hg, M, p, q);
                if (q < c && os_rotate_pair<T, 8, LP, LP>(G, ld, V, ld, N, c0 + p, c0 + q, tol, atol) == 2) big = 1;
            }
            wave_order();
        }
    }
    __syncthreads();
    for (int R = 0; R < nbp - 1; ++R) {
        for (int pk = wid; pk < nbp / 2; pk += NW) {
            int P, Q;
            rr_pair(R, pk, nbp, P, Q);
            if (Q >= nb) continue;
            if (N <= 128) {
                if (N <= 32) big |= cross_block_regs<T, 4, true>(G, V, ld, N, P, Q, tol, atol);
                else if (N <= 64) big |= cross_block_regs<T, 8, false>(G, V, ld, N, P, Q, tol, atol);
                else if (N <= 96) big |= cross_block_regs<T, 12, false>(G, V, ld, N, P, Q, tol, atol);
                else big |= cross_block_regs<T, 16, false>(G, V, ld, N, P, Q, tol, atol);
                continue;
            }
            for (int st = 0; st < 8; ++st) {
                const int p = P * 8 + grp, q = Q * 8 + ((grp + st) & 7);
                if (p < N && q < N && os_rotate_pair<T, 8, LP, LP>(G, ld, V, ld, N, p, q, tol, atol) == 2) big = 1;
                wave_order();
            }
        }
        __syncthreads();
    }
    return big;
}

// One block-cyclic sweep (block_cyclic_sweep) of each of two matrices at once, G and V of both in
// LDS: the blocks of both share the passes of the in-block phase (a wavefront per block) and the
// block rounds share their workgroup barriers (the two matrices' block pairs spread over the
// wavefronts), so the smaller matrix's sweep runs on wavefronts the larger one leaves idle.  Each
// matrix's rotations and their order are those of its own sweep.  A matrix with act = 0 is left
// alone.  big1, big2: as block_cyclic_sweep's result, per matrix.
template <typename T, int NT, typename LP>
__device__ __forceinline__ void block_cyclic_sweep2(LP G1, LP V1, int ld1, int N1, T tol1, T atol1, bool act1, LP G2,
                                                    LP V2, int ld2, int N2, T tol2, T atol2, bool act2, int &big1,
                                                    int &big2) {
    constexpr int NW = NT / 64;
    const int wid = threadIdx.x >> 6, grp = (threadIdx.x & 63) >> 3;
    const int nb1 = act1 ? (N1 + 7) >> 3 : 0, nb2 = act2 ? (N2 + 7) >> 3 : 0;
    const int nbp1 = nb1 + (nb1 & 1), nbp2 = nb2 + (nb2 & 1);
    big1 = big2 = 0;
    // in-block pairs: two blocks per wavefront, one per half (as in block_cyclic_sweep)
    const int half = grp >> 2, hg = grp & 3;
    for (int Bk = 2 * wid + half; Bk - half < nb1 + nb2; Bk += 2 * NW) {
        const bool one = Bk < nb1;
        LP G = one ? G1 : G2;
        LP V = one ? V1 : V2;
        const int ld = one ? ld1 : ld2, N = one ? N1 : N2;
        const T tol = one ? tol1 : tol2, atol = one ? atol1 : atol2;
        const int c0 = (one ? Bk : Bk - nb1) * 8;
        const int c = Bk < nb1 + nb2 ? (N - c0 < 8 ? N - c0 : 8) : 0, M = c + (c & 1);
        for (int r = 0; r < 7; ++r) {   // the rounds of a full block; shorter blocks idle
            if (r < M - 1 && hg < M / 2) {
                int p, q;
                rr_pair(r, hg, M, p, q);
                if (q < c && os_rotate_pair<T, 8, LP, LP>(G, ld, V, ld, N, c0 + p, c0 + q, tol, atol) == 2) {
                    if (one) big1 = 1;
                    else big2 = 1;
                }
            }
            wave_order();
        }
    }
    __syncthreads();
    const int rounds = (nbp1 > nbp2 ? nbp1 : nbp2) - 1;
    const int h1 = nbp1 / 2, h2 = nbp2 / 2;
    for (int R = 0; R < rounds; ++R) {
        const int n1 = R < nbp1 - 1 ? h1 : 0, n2 = R < nbp2 - 1 ? h2 : 0;
        for (int pk = wid; pk < n1 + n2; pk += NW) {
            const bool one = pk < n1;
            const int nb = one ? nb1 : nb2, nbp = one ? nbp1 : nbp2, N = one ? N1 : N2;
            int P, Q;
            rr_pair(R, one ? pk : pk - n1, nbp, P, Q);
            if (Q >= nb) continue;
            LP G = one ? G1 : G2;
            LP V = one ? V1 : V2;
            const int ld = one ? ld1 : ld2;
            const T tol = one ? tol1 : tol2, atol = one ? atol1 : atol2;
            int b = 0;
            if (N <= 32) b = cross_block_regs<T, 4, true>(G, V, ld, N, P, Q, tol, atol);
            else if (N <= 64) b = cross_block_regs<T, 8, false>(G, V, ld, N, P, Q, tol, atol);
            else if (N <= 96) b = cross_block_regs<T, 12, false>(G, V, ld, N, P, Q, tol, atol);
            else if (N <= 128) b = cross_block_regs<T, 16, false>(G, V, ld, N, P, Q, tol, atol);
            else
                for (int st = 0; st < 8; ++st) {
                    const int p = P * 8 + grp, q = Q * 8 + ((grp + st) & 7);
                    if (p < N && q < N && os_rotate_pair<T, 8, LP, LP>(G, ld, V, ld, N, p, q, tol, atol) == 2) b = 1;
                    wave_order();
                }
            if (b) {
                if (one) big1 = 1;
                else big2 = 1;
            }
        }
        __syncthreads();
    }
}

// Stages one block for the Jacobi sweeps: G = W (cold, V = I) or G = W V_prev (warm), W symmetric
// (column j of W = row j), read from the packed lower triangle vs.  Warm, with at most kMfmaHold
// 16 x 16 tiles of G per wavefront, W is staged where G goes and each wavefront keeps its tiles of
// W V in registers until every read of W is done; otherwise W is staged in the global scratch Tm.
// Returns |W|_F^2 (every thread).
template <typename T, int NT, typename GP, typename VP>
__device__ __forceinline__ double stage_block(T *__restrict__ vs, int N, T *__restrict__ Vs, bool warm, GP G, VP V,
                                              int ld, T *__restrict__ Tm, const EigScratch &sc) {
    const int tid = threadIdx.x;
    constexpr int NW = NT / 64;
    const int nt16 = (N + 15) >> 4;
    const bool wreg = warm && nt16 * nt16 <= NW * kMfmaHold;
    // four entries per thread and pass, their global reads issued together
    double fro2 = 0.0, dummy = 0.0;
    for (int base = 0; base < N * N; base += 4 * NT) {
        int ii[4], jj[4];
        T xs[4], vv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = base + q * NT + tid;
            jj[q] = idx / N;
            ii[q] = idx - jj[q] * N;   // column jj, row ii
            if (idx < N * N) {
                const int a = ii[q] > jj[q] ? ii[q] : jj[q], bb = ii[q] > jj[q] ? jj[q] : ii[q];
                xs[q] = vs[svec_idx(a, bb, N)];
                vv[q] = warm ? Vs[jj[q] * N + ii[q]] : (ii[q] == jj[q] ? (T)1 : (T)0);
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (base + q * NT + tid >= N * N) continue;
            const int i = ii[q], j = jj[q];
            const T x = xs[q];
            fro2 += (double)x * (double)x;
            if (warm && !wreg)
                Tm[j * N + i] = x;
            else
                G[j * ld + i] = x;
            V[j * ld + i] = vv[q];
        }
    }
    __syncthreads();
    if (warm) {
        // G = W V_prev on the matrix cores; W read from G's storage (held tiles) or from Tm
        constexpr bool g_lds = std::is_same<GP, typename Lds<T>::type *>::value;
        if (wreg) mfma_wv<T, NT>(G, ld, !g_lds, V, ld, G, ld, N, true);
        else mfma_wv<T, NT>(Tm, N, true, V, ld, G, ld, N, false);
        __syncthreads();
    }
    block_sum2<NT>(fro2, dummy, sc.s_red);
    return fro2;
}

// One Jacobi sweep of one block (see project_block); returns 1 (in the threads that saw one) if a
// rotation had relative coupling above sqrt(tol).
template <typename T, int NT, typename GP, typename VP>
__device__ __forceinline__ int sweep_block(GP G, VP V, int ld, int N, T tol, T atol, int gs, int jblock) {
    const int tid = threadIdx.x;
    const int M = N + (N & 1);
    const int H = M / 2;
    int big = 0;
    constexpr bool kBothLds = std::is_same<GP, typename Lds<T>::type *>::value && std::is_same<VP, GP>::value;
    // lanes per column pair: a tile choice per block-size bucket (autotuned), or the
    // block-cyclic order (G and V in LDS)
    if (kBothLds && jblock == 8) {
        if constexpr (kBothLds) big = block_cyclic_sweep<T, NT>(G, V, ld, N, tol, atol);
    } else if (gs == 8) {
        const int grp = tid / 8;
        for (int r = 0; r < M - 1; ++r) {
            for (int kk = grp; kk < H; kk += NT / 8) {
                int p, q;
                rr_pair(r, kk, M, p, q);
                if (q < N && os_rotate_pair<T, 8, GP, VP>(G, ld, V, ld, N, p, q, tol, atol) == 2) big = 1;
            }
            __syncthreads();
        }
    } else if (gs == 32) {
        const int grp = tid / 32;
        for (int r = 0; r < M - 1; ++r) {
            for (int kk = grp; kk < H; kk += NT / 32) {
                int p, q;
                rr_pair(r, kk, M, p, q);
                if (q < N && os_rotate_pair<T, 32, GP, VP>(G, ld, V, ld, N, p, q, tol, atol) == 2) big = 1;
            }
            __syncthreads();
        }
    } else {
        const int grp = tid / 16;
        for (int r = 0; r < M - 1; ++r) {
            for (int kk = grp; kk < H; kk += NT / 16) {
                int p, q;
                rr_pair(r, kk, M, p, q);
                if (q < N && os_rotate_pair<T, 16, GP, VP>(G, ld, V, ld, N, p, q, tol, atol) == 2) big = 1;
            }
            __syncthreads();
        }
    }
    return big;
}

// sigma_j = |g_j|, then u = lower((W + V Sigma V^T) / 2), v = u - w on the matrix cores, and the
// eigenvectors into the warm-start cache Vs.
template <typename T, int NT, typename GP, typename VP>
__device__ __forceinline__ void finish_block(T *__restrict__ vs, T *__restrict__ us, int N, T *__restrict__ Vs, GP G,
                                             VP V, int ld, typename Lds<T>::type *s_sig) {
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    constexpr int NW = NT / 64;
    for (int j = wid; j < N; j += NW) {
        T s = 0;
        for (int i = lane; i < N; i += 64) s += G[j * ld + i] * G[j * ld + i];
        s = wave_allsum(s);
        if (lane == 0) s_sig[j] = sqrt(s);
    }
    __syncthreads();
    mfma_rebuild<T, NT>(V, ld, s_sig, N, vs, us);
    if (Vs)
        for (int idx = tid; idx < N * N; idx += NT) {
            const int j = idx / N, i = idx - (idx / N) * N;
            Vs[j * N + i] = V[j * ld + i];
        }
    __syncthreads();
}

template <typename T, int NT, typename GP, typename VP>
__device__ __noinline__ void project_block(T *__restrict__ vs, T *__restrict__ us, int N, T *__restrict__ Vs, bool warm, GP G,
                              VP V, int ld, T *__restrict__ Tm, typename Lds<T>::type *s_sig, const EigScratch &sc,
                              int max_sweeps, int gs = 16, int jblock = 0) {
    const int tid = threadIdx.x;
    if (N == 1) {
        if (tid == 0) {
            const T w = vs[0];
            const T x = w > (T)0 ? w : (T)0;
            us[0] = x;
            vs[0] = x - w;
            if (Vs) Vs[0] = (T)1;
        }
        __syncthreads();
        return;
    }
    const double fro2 = stage_block<T, NT>(vs, N, Vs, warm, G, V, ld, Tm, sc);
    // a pair is rotated while it is coupled beyond rounding, relative to both columns
    // (16 eps) and absolutely (eps |W|_F times the larger column): below that, the pair's
    // contribution to |W| is under the rounding error of W itself, and columns of
    // near-zero eigenvalues stop trading noise
    const T tol = jacobi_tol<T>(sc.jtol);
    const T atol = (T)(jacobi_atol_factor(N) * TS<T>::eps * sqrt(fro2));
    int nsw = 0;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        if (tid == 0) *sc.s_flag = 0;
        __syncthreads();
        // big: some rotation of the sweep had relative coupling above sqrt(tol).  Without one
        // the sweep is the last: cyclic Jacobi converges quadratically, so what such a sweep
        // leaves is coupling of order tol, which the next sweep would not rotate
        const int big = sweep_block<T, NT>(G, V, ld, N, tol, atol, gs, jblock);
        if (big) *sc.s_flag = 1;
        __syncthreads();
        const int any = *sc.s_flag;
        __syncthreads();
        ++nsw;
        if (!any) break;
    }
    // counted after the loop: no thread-0 block ends the body next to the one that begins it
    if (tid == 0) *sc.s_sweeps += nsw;
    finish_block<T, NT>(vs, us, N, Vs, G, V, ld, s_sig);
}

// stage_block for two blocks at once (project_two): one staging pass over both blocks' entries,
// one pass of warm products over both blocks' 16 x 16 tiles (each wavefront holding its tiles of
// both until every read of W is done), so the smaller block fills slots the larger leaves idle.
// Falls back to two stage_block calls when a wavefront would hold more than kMfmaHold tiles.
// Returns |W_1|_F^2 and |W_2|_F^2 (every thread).
template <typename T, int NT, typename LP>
__device__ __forceinline__ void stage_pair(T *__restrict__ vs1, int N1, T *__restrict__ Vs1, LP G1, LP V1, int ld1,
                                           T *__restrict__ vs2, int N2, T *__restrict__ Vs2, LP G2, LP V2, int ld2,
                                           bool warm, T *__restrict__ Tm, const EigScratch &sc, double &fro1,
                                           double &fro2) {
    typedef typename Mma<T>::acc AC;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    constexpr int NW = NT / 64;
    const int nt1 = (N1 + 15) >> 4, nt2 = (N2 + 15) >> 4;
    const int ntt1 = nt1 * nt1, ntt2 = nt2 * nt2;
    if (warm && ntt1 + ntt2 > NW * kMfmaHold) {
        fro1 = stage_block<T, NT>(vs1, N1, Vs1, warm, G1, V1, ld1, Tm, sc);
        fro2 = stage_block<T, NT>(vs2, N2, Vs2, warm, G2, V2, ld2, Tm, sc);
        return;
    }
    double f1 = 0.0, f2 = 0.0;
    const int e1 = N1 * N1, etot = e1 + N2 * N2;
    for (int idx = tid; idx < etot; idx += NT) {
        const bool one = idx < e1;
        const int N = one ? N1 : N2, ld = one ? ld1 : ld2, id = one ? idx : idx - e1;
        const int j = id / N, i = id - j * N;
        const int a = i > j ? i : j, bb = i > j ? j : i;
        const T x = (one ? vs1 : vs2)[svec_idx(a, bb, N)];
        const T vv = warm ? (one ? Vs1 : Vs2)[j * N + i] : (i == j ? (T)1 : (T)0);
        (one ? G1 : G2)[j * ld + i] = x;   // W where G goes (warm: read back by the products below)
        (one ? V1 : V2)[j * ld + i] = vv;
        if (one) f1 += (double)x * (double)x;
        else f2 += (double)x * (double)x;
    }
    __syncthreads();
    if (warm) {
        // G = W V_prev: tile c of the combined list (block 1's ntt1 tiles, then block 2's) to
        // wavefront c mod NW, W read from G's storage, written after the barrier
        const int li = lane & 15, lg = lane >> 4;
        AC acc[kMfmaHold];
#pragma unroll
        for (int q = 0; q < kMfmaHold; ++q) {
            acc[q] = (AC)(T)0;
            const int c = q * NW + wid;
            if (c >= ntt1 + ntt2) continue;
            const bool one = c < ntt1;
            const int nt = one ? nt1 : nt2, tl = one ? c : c - ntt1, N = one ? N1 : N2, ld = one ? ld1 : ld2;
            LP W = one ? G1 : G2;
            LP V = one ? V1 : V2;
            const int i = (tl % nt) * 16 + li, j = (tl / nt) * 16 + li;
            const bool iok = i < N, jok = j < N;
            for (int k0 = 0; k0 < N; k0 += 16) {
                const int kb = k0 + 4 * lg;
                T a[4], b[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const bool kok = kb + t < N;
                    a[t] = (iok && kok) ? W[(long long)i * ld + kb + t] : (T)0;
                    b[t] = (jok && kok) ? V[(long long)j * ld + kb + t] : (T)0;
                }
#pragma unroll
                for (int t = 0; t < 4; ++t) acc[q] = Mma<T>::step(a[t], b[t], acc[q]);
            }
        }
        __syncthreads();   // every read of W done before G, its storage, is written
#pragma unroll
        for (int q = 0; q < kMfmaHold; ++q) {
            const int c = q * NW + wid;
            if (c >= ntt1 + ntt2) continue;
            const bool one = c < ntt1;
            const int nt = one ? nt1 : nt2, tl = one ? c : c - ntt1, N = one ? N1 : N2, ld = one ? ld1 : ld2;
            LP G = one ? G1 : G2;
            const int i0 = (tl % nt) * 16, j = (tl / nt) * 16 + li;
            if (j >= N) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + Mma<T>::row(lg, r);
                if (i < N) G[(long long)j * ld + i] = acc[q][r];
            }
        }
        __syncthreads();
    }
    block_sum2<NT>(f1, f2, sc.s_red);
    fro1 = f1;
    fro2 = f2;
}

// finish_block for two blocks at once: both blocks' sigma in one pass (block 2's after its V), the
// two rebuilds' tiles spread as one list over the wavefronts, both caches written, one barrier.
template <typename T, int NT, typename LP>
__device__ __forceinline__ void finish_pair(T *__restrict__ vs1, T *__restrict__ us1, int N1, T *__restrict__ Vs1, LP G1,
                                            LP V1, int ld1, LP sig1, T *__restrict__ vs2, T *__restrict__ us2, int N2,
                                            T *__restrict__ Vs2, LP G2, LP V2, int ld2, LP sig2) {
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    constexpr int NW = NT / 64;
    for (int c = wid; c < N1 + N2; c += NW) {
        const bool one = c < N1;
        const int j = one ? c : c - N1, ld = one ? ld1 : ld2, N = one ? N1 : N2;
        LP G = one ? G1 : G2;
        T sum = 0;
        for (int i = lane; i < N; i += 64) sum += G[j * ld + i] * G[j * ld + i];
        sum = wave_allsum(sum);
        if (lane == 0) (one ? sig1 : sig2)[j] = sqrt(sum);
    }
    __syncthreads();
    const int nt1 = (N1 + 15) >> 4, ntri1 = nt1 * (nt1 + 1) / 2;
    mfma_rebuild<T, NT>(V1, ld1, sig1, N1, vs1, us1, wid, NW);
    mfma_rebuild<T, NT>(V2, ld2, sig2, N2, vs2, us2, ((wid - ntri1) % NW + NW) % NW, NW);
    const int e1 = N1 * N1, etot = e1 + N2 * N2;
    for (int idx = tid; idx < etot; idx += NT) {
        const bool one = idx < e1;
        T *Vs = one ? Vs1 : Vs2;
        if (!Vs) continue;
        const int N = one ? N1 : N2, ld = one ? ld1 : ld2, id = one ? idx : idx - e1;
        const int j = id / N, i = id - j * N;
        Vs[j * N + i] = (one ? V1 : V2)[j * ld + i];
    }
    __syncthreads();
}

// Projects the two blocks of a problem together (both at least 2 x 2, G and V of both in LDS from
// s_mat on, columns padded to lds_ld): each staged as project_block stages it, then sweeps of both
// at once (block_cyclic_sweep2) until each has had a sweep without a rotation of relative coupling
// above sqrt(tol) (or max_sweeps), each block's sweeps counted and stopped as project_block's, then
// each finished as project_block finishes it.  Every block's arithmetic is the same as projecting
// it alone; the smaller block's sweeps run on wavefronts the larger one leaves idle.
template <typename T, int NT>
__device__ __noinline__ void project_two(T *__restrict__ vs1, T *__restrict__ us1, int N1, T *__restrict__ Vs1,
                                         T *__restrict__ vs2, T *__restrict__ us2, int N2, T *__restrict__ Vs2, bool warm,
                                         typename Lds<T>::type *s_mat, T *__restrict__ Tm, typename Lds<T>::type *s_sig,
                                         const EigScratch &sc, int max_sweeps) {
    typedef typename Lds<T>::type *LP;
    __shared__ int s_vote[2];
    const int tid = threadIdx.x;
    const int ld1 = lds_ld(N1), ld2 = lds_ld(N2);
    LP G1 = s_mat, V1 = G1 + (long long)N1 * ld1, G2 = V1 + (long long)N1 * ld1, V2 = G2 + (long long)N2 * ld2;
    LP sig2 = V2 + (long long)N2 * ld2;   // block 2's sigma (s_sig holds block 1's)
    double fro1, fro2;
    stage_pair<T, NT, LP>(vs1, N1, Vs1, G1, V1, ld1, vs2, N2, Vs2, G2, V2, ld2, warm, Tm, sc, fro1, fro2);
    const T tol = jacobi_tol<T>(sc.jtol);
    const T atol1 = (T)(jacobi_atol_factor(N1) * TS<T>::eps * sqrt(fro1));
    const T atol2 = (T)(jacobi_atol_factor(N2) * TS<T>::eps * sqrt(fro2));
    bool act1 = true, act2 = true;
    int nsw1 = 0, nsw2 = 0;
    for (int sweep = 0; sweep < max_sweeps && (act1 || act2); ++sweep) {
        if (tid == 0) s_vote[0] = s_vote[1] = 0;
        __syncthreads();
        int b1, b2;
        block_cyclic_sweep2<T, NT, LP>(G1, V1, ld1, N1, tol, atol1, act1, G2, V2, ld2, N2, tol, atol2, act2, b1, b2);
        if (b1) s_vote[0] = 1;
        if (b2) s_vote[1] = 1;
        __syncthreads();
        const int any1 = s_vote[0], any2 = s_vote[1];
        __syncthreads();
        if (act1) {
            ++nsw1;
            if (!any1) act1 = false;
        }
        if (act2) {
            ++nsw2;
            if (!any2) act2 = false;
        }
    }
    if (tid == 0) *sc.s_sweeps += nsw1 + nsw2;
    finish_pair<T, NT, LP>(vs1, us1, N1, Vs1, G1, V1, ld1, s_sig, vs2, us2, N2, Vs2, G2, V2, ld2, sig2);
}

// ----------------------------------------------------------------------------- PSD projection, helpers
// 16-byte vector of T, in LDS
template <typename T> struct V16;
template <> struct V16<float> {
    typedef float v __attribute__((ext_vector_type(4)));
    static constexpr int n = 4;
};
template <> struct V16<double> {
    typedef double v __attribute__((ext_vector_type(2)));
    static constexpr int n = 2;
};
template <typename T> __device__ __forceinline__ T hsum(typename V16<T>::v x);
template <> __device__ __forceinline__ float hsum<float>(V16<float>::v x) { return (x.x + x.y) + (x.z + x.w); }
template <> __device__ __forceinline__ double hsum<double>(V16<double>::v x) { return x.x + x.y; }

// ----------------------------------------------------------------------------- PSD projection, rows per wavefront
// Same projection again, with the rows of the column-major N x N matrices G and V split
// over the NW wavefronts of the workgroup: wavefront w owns rows [w R, (w + 1) R) of every
// column (R a multiple of the 16-byte vector width; rows N..NW R - 1 are zero).  Lane kk
// of every wavefront takes column pair kk of the round: each wavefront forms partial inner
// products over its rows, the partials meet in LDS (one workgroup barrier per round),
// every wavefront sums them in the same order, so all take bitwise-equal rotation
// decisions, and each rotates its own rows.  No wavefront touches another's rows of G or
// V; the barrier only guards the partials, which alternate between two buffers by round
// parity (a wavefront can only be one round ahead of the slowest).
// Wavefronts that own rows: among the counts up to nw with the fewest rows per wavefront
// (the latency of a round), the one that pads the fewest rows in total (the LDS traffic);
// ties keep more wavefronts.  The others only join the barriers.
__host__ __device__ __forceinline__ int rows_nwe(int N, int elem_bytes, int nw) {
    const int vw = 16 / elem_bytes;
    int best = nw, best_r = 1 << 30, best_np = 1 << 30;
    for (int e = nw; e >= 1; --e) {
        const int r = ((N + e - 1) / e + vw - 1) / vw * vw;
        if (r < best_r || (r == best_r && e * r < best_np)) {
            best_r = r;
            best_np = e * r;
            best = e;
        }
    }
    return best;
}
__host__ __device__ __forceinline__ int rows_R(int N, int elem_bytes, int nw) {
    const int vw = 16 / elem_bytes;
    const int e = rows_nwe(N, elem_bytes, nw);
    return ((N + e - 1) / e + vw - 1) / vw * vw;
}
// leading dimension: at least nwe R, and 16 bytes (mod 128): lanes on consecutive columns
// read distinct 4-bank groups
__host__ __device__ __forceinline__ int rows_ld(int N, int elem_bytes, int nw) {
    const int q = 128 / elem_bytes, r = 16 / elem_bytes;
    const int np = rows_nwe(N, elem_bytes, nw) * rows_R(N, elem_bytes, nw);
    return q * ((np - r + q - 1) / q) + r;
}
// column pairs per round
__host__ __device__ __forceinline__ int rows_hp(int N) { return (N + (N & 1)) / 2; }
// partial sums (al, be, ga) of one pair and one wavefront: one 16-byte record in FP32,
// two in FP64; records of a pair padded to nw + 1, so lanes on consecutive pairs read
// distinct bank groups
__host__ __device__ __forceinline__ int rows_rec(int elem_bytes) { return elem_bytes == 4 ? 1 : 2; }
// LDS elements of one block: G, V, two buffers of partial records, sigma
__host__ __device__ __forceinline__ long long rows_region(int N, int elem_bytes, int nw) {
    const int vw = 16 / elem_bytes;
    return 2LL * N * rows_ld(N, elem_bytes, nw) + 2LL * rows_hp(N) * (nw + 1) * rows_rec(elem_bytes) * vw +
           ((N + 3) & ~3);
}
// most 16-byte vectors per column and wavefront held in registers through a round
template <typename T> struct RowsCache { static constexpr int n = 6; };

template <typename T, int NT>
__device__ __noinline__ void project_block_rows(T *__restrict__ vs, T *__restrict__ us, int N, T *__restrict__ Vs,
                                                bool warm, typename Lds<T>::type *G, T *__restrict__ Tm,
                                                const EigScratch &sc, int max_sweeps) {
    typedef typename Lds<T>::type LT;
    typedef typename V16<T>::v VT;
    typedef __attribute__((address_space(3))) VT LVT;
    constexpr int NW = NT / 64;
    constexpr int VW = V16<T>::n;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (N == 1) {
        if (tid == 0) {
            const T x0 = vs[0];
            const T x = x0 > (T)0 ? x0 : (T)0;
            us[0] = x;
            vs[0] = x - x0;
            if (Vs) Vs[0] = (T)1;
        }
        __syncthreads();
        return;
    }
    const int NWE = rows_nwe(N, (int)sizeof(T), NW);   // wavefronts owning rows
    const int R = rows_R(N, (int)sizeof(T), NW);
    const int ld = rows_ld(N, (int)sizeof(T), NW);
    const int HP = rows_hp(N);
    const int Np = NWE * R;
    constexpr int REC = sizeof(T) == 4 ? 1 : 2;   // 16-byte records per partial (al, be, ga)
    LT *V = G + (long long)N * ld;
    LT *part = V + (long long)N * ld;   // [2][HP][NW + 1][REC] records
    LT *sig = part + 2LL * HP * (NW + 1) * REC * VW;
    double fro2 = 0.0, dummy = 0.0;
    for (int idx = tid; idx < N * N; idx += NT) {
        const int j = idx / N, i = idx - (idx / N) * N;
        const int a = i > j ? i : j, bb = i > j ? j : i;
        const T x = vs[svec_idx(a, bb, N)];
        fro2 += (double)x * (double)x;
        if (warm) {
            Tm[j * N + i] = x;
            V[j * ld + i] = Vs[j * N + i];
        } else {
            G[j * ld + i] = x;
            V[j * ld + i] = (i == j) ? (T)1 : (T)0;
        }
    }
    for (int idx = tid; idx < (Np - N) * N; idx += NT) {
        const int j = idx / (Np - N), i = N + idx - (idx / (Np - N)) * (Np - N);
        G[j * ld + i] = (T)0;
        V[j * ld + i] = (T)0;
    }
    block_sum2<NT>(fro2, dummy, sc.s_red);   // its barriers also publish G, V, Tm
    if (warm) {
        // G = W V_prev on the matrix cores (W in Tm; rows N.. of G stay zero)
        mfma_wv<T, NT>(Tm, N, true, V, ld, G, ld, N, false);
        __syncthreads();
    }
    const T tol = jacobi_tol<T>(sc.jtol);
    const T atol = (T)(jacobi_atol_factor(N) * TS<T>::eps * sqrt(fro2));
    const T tol2 = tol * tol, atol2 = atol * atol;
    const int M = N + (N & 1);
    const int H = M / 2;
    const int nvw = R / VW;              // vectors per column in this wavefront's rows
    const int row0 = w * R;
    const bool owner = w < NWE;          // wavefronts past NWE own no rows: barriers only
    constexpr int NC = RowsCache<T>::n;
    const bool cache = nvw <= NC;        // columns of the lane's first pair stay in registers
    LVT *const partv = (LVT *)part;
    int nsw = 0, round = 0;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        int rotated = 0, big = 0;   // big: some rotation of the sweep had coupling above sqrt(tol)
        for (int r = 0; r < M - 1; ++r, ++round) {
            LVT *pb = partv + (long long)(round & 1) * HP * (NW + 1) * REC;
            // pair kk of the round (no ordering p < q needed): lanes on consecutive kk touch
            // consecutive columns r + kk and r - kk
            VT cA[NC], cB[NC], cC[NC], cD[NC];   // this wavefront's rows of g_p, g_q, v_p, v_q (first pair)
            for (int kk = owner ? lane : H; kk < H; kk += 64) {
                int p, q;
                if (kk == 0) {
                    p = r;
                    q = M - 1;
                } else {
                    p = r + kk;
                    if (p >= M - 1) p -= M - 1;
                    q = r - kk;
                    if (q < 0) q += M - 1;
                }
                T al = 0, be = 0, ga = 0;
                if (p < N && q < N) {
                    const LVT *gp = (const LVT *)(G + p * ld + row0), *gq = (const LVT *)(G + q * ld + row0);
                    VT sa = (VT)(T)0, sb = (VT)(T)0, sg = (VT)(T)0;
                    if (cache && kk < 64) {
                        // all of this wavefront's rows of the four columns in one burst of reads
                        const LVT *vp = (const LVT *)(V + p * ld + row0), *vq = (const LVT *)(V + q * ld + row0);
#pragma unroll
                        for (int c = 0; c < NC; ++c)
                            if (c < nvw) {
                                cA[c] = gp[c];
                                cB[c] = gq[c];
                                cC[c] = vp[c];
                                cD[c] = vq[c];
                            }
#pragma unroll
                        for (int c = 0; c < NC; ++c)
                            if (c < nvw) {
                                sa += cA[c] * cA[c];
                                sb += cB[c] * cB[c];
                                sg += cA[c] * cB[c];
                            }
                    } else {
#pragma unroll 2
                        for (int c = 0; c < nvw; ++c) {
                            const VT a = gp[c], b = gq[c];
                            sa += a * a;
                            sb += b * b;
                            sg += a * b;
                        }
                    }
                    al = hsum<T>(sa);
                    be = hsum<T>(sb);
                    ga = hsum<T>(sg);
                }
                LVT *rec = pb + ((long long)kk * (NW + 1) + w) * REC;
                if constexpr (REC == 1) {
                    VT x;
                    x[0] = al;
                    x[1] = be;
                    x[2] = ga;
                    x[3] = (T)0;
                    rec[0] = x;
                } else {
                    VT x0, x1;
                    x0[0] = al;
                    x0[1] = be;
                    x1[0] = ga;
                    x1[1] = (T)0;
                    rec[0] = x0;
                    rec[1] = x1;
                }
            }
            __syncthreads();
            // every wavefront (owner or not) takes the rotation decisions, so the
            // convergence vote below is the same in all of them
            for (int kk = lane; kk < H; kk += 64) {
                int p, q;
                if (kk == 0) {
                    p = r;
                    q = M - 1;
                } else {
                    p = r + kk;
                    if (p >= M - 1) p -= M - 1;
                    q = r - kk;
                    if (q < 0) q += M - 1;
                }
                if (p >= N || q >= N) continue;
                // the NWE partial records of pair kk, summed in wavefront order (all wavefronts alike)
                const LVT *rk = pb + (long long)kk * (NW + 1) * REC;
                T al = 0, be = 0, ga = 0;
                if constexpr (REC == 1) {
                    VT x[NW];
#pragma unroll
                    for (int y = 0; y < NW; ++y)
                        if (y < NWE) x[y] = rk[y];
#pragma unroll
                    for (int y = 0; y < NW; ++y)
                        if (y < NWE) {
                            al += x[y][0];
                            be += x[y][1];
                            ga += x[y][2];
                        }
                } else {
                    VT x[2 * NW];
#pragma unroll
                    for (int y = 0; y < NW; ++y)
                        if (y < NWE) {
                            x[2 * y] = rk[2 * y];
                            x[2 * y + 1] = rk[2 * y + 1];
                        }
#pragma unroll
                    for (int y = 0; y < NW; ++y)
                        if (y < NWE) {
                            al += x[2 * y][0];
                            be += x[2 * y][1];
                            ga += x[2 * y + 1][0];
                        }
                }
                T cc, ss;
                if (!jacobi_rot<T>(al, be, ga, tol2, atol2, cc, ss)) continue;
                if (ga * ga > tol * (al * be)) big = 1;
                rotated = 1;
                if (!owner) continue;
                LVT *gp = (LVT *)(G + p * ld + row0), *gq = (LVT *)(G + q * ld + row0);
                LVT *vp = (LVT *)(V + p * ld + row0), *vq = (LVT *)(V + q * ld + row0);
                if (cache && kk < 64) {
#pragma unroll
                    for (int c = 0; c < NC; ++c)
                        if (c < nvw) {
                            gp[c] = cc * cA[c] - ss * cB[c];
                            gq[c] = ss * cA[c] + cc * cB[c];
                            vp[c] = cc * cC[c] - ss * cD[c];
                            vq[c] = ss * cC[c] + cc * cD[c];
                        }
                } else {
                    // one 16-byte vector per column at a time, the next one read before the
                    // current one is written (columns p and q are distinct, so they never overlap)
                    VT A = gp[0], Bv = gq[0], C = vp[0], D = vq[0];
                    for (int c = 0; c < nvw; ++c) {
                        VT nA, nB, nC, nD;
                        const bool more = c + 1 < nvw;
                        if (more) {
                            nA = gp[c + 1];
                            nB = gq[c + 1];
                            nC = vp[c + 1];
                            nD = vq[c + 1];
                        }
                        gp[c] = cc * A - ss * Bv;
                        gq[c] = ss * A + cc * Bv;
                        vp[c] = cc * C - ss * D;
                        vq[c] = ss * C + cc * D;
                        if (more) {
                            A = nA;
                            Bv = nB;
                            C = nC;
                            D = nD;
                        }
                    }
                }
            }
            // this wavefront's next partials read rows its own lanes just rotated
            wave_order();
        }
        ++nsw;
        // every wavefront took the same decisions, so the vote needs no exchange.  Converged:
        // no rotation, or every rotation of the sweep was small (relative coupling at most
        // sqrt(tol)); cyclic Jacobi converges quadratically, so such a sweep leaves coupling
        // of order tol, which the next sweep would not rotate
        if (!__any(rotated) || !__any(big)) break;
    }
    if (tid == 0) *sc.s_sweeps += nsw;
    __syncthreads();
    for (int j = tid; j < N; j += NT) {
        const LVT *gj = (const LVT *)(G + j * ld);
        VT s = (VT)(T)0;
        for (int c = 0; c < Np / VW; ++c) s += gj[c] * gj[c];
        sig[j] = sqrt(hsum<T>(s));
    }
    __syncthreads();
    // u = lower((W + V Sigma V^T) / 2), v = u - w, on the matrix cores
    mfma_rebuild<T, NT>(V, ld, sig, N, vs, us);
    if (Vs)
        for (int idx = tid; idx < N * N; idx += NT) {
            const int j = idx / N, i = idx - (idx / N) * N;
            Vs[j * N + i] = V[j * ld + i];
        }
    __syncthreads();
}

// ----------------------------------------------------------------------------- residuals (FP64)
template <typename T, int NT>
__device__ __noinline__ int residual_phase(const ProbDesc &P, double tol, double *s_red, int iters_done, double *res_max = nullptr) {
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
        acc[2] += P.b64[a] * (double)u[nx + a];
        double rp = ax - P.b64[a] * tau;
        if (P.rsc64) {   // equilibrated: rows back in the original units
            rp *= P.rsc64[a];
            ax *= P.rsc64[a];
        }
        acc[0] += rp * rp;
        acc[1] += ax * ax;
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
        double g = aty + (double)v[e];
        double rd = g - P.c64[e] * tau;
        if (P.csc64) {   // equilibrated: columns back in the original units
            rd *= P.csc64[e];
            g *= P.csc64[e];
        }
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
    if (res_max) {
        // progress measures: the largest residual, and (once tau has collapsed) the smaller
        // relative error of the two infeasibility certificates
        double ce = INFINITY;
        if (by > 0.0) ce = fmin(ce, sqrt(saty) / by);
        if (cx < 0.0) ce = fmin(ce, sqrt(sax) / (-cx));
        res_max[0] = mx;
        res_max[1] = ce;
    }
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
// launch bounds: at least 2 waves per SIMD (the second argument is waves per execution
// unit), i.e. at most 256 VGPRs, so that two or more workgroups (problems) can share a CU
// and hide each other's latency
// One solve phase of one problem (RUN_STEP: exactly rp.iters iterations; RUN_SOLVE: to tol,
// a certificate, the budget, or a stall) by the whole workgroup, in precision T.  Returns
// the status the phase ended with (0: stalled or out of budget).
template <typename T, int NT>
__device__ __noinline__ int run_phase(const ProbDesc &P, const RunParams &rp, char *wbase, char *ebase, char *dyn_lds,
                                      const EigScratch &sc) {
    // dynamic LDS: sigma (eig_ld values), then the eigensolver's matrices (layout by the
    // launcher for this T); the affine step's k-vector and the small solve's partial sums
    // share the eigen region, the two phases being separated by barriers
    typename Lds<T>::type *s_sig = as_lds<T>(dyn_lds);
    typename Lds<T>::type *s_mat = as_lds<T>(dyn_lds + rp.lds_mat_off);
    double *s_z = reinterpret_cast<double *>(dyn_lds + rp.lds_mat_off);
    // the affine step's LDS past its k-vector and partial sums (2 SOS_KMAX_LDS doubles)
    char *aff_lds = dyn_lds + rp.lds_mat_off + sizeof(double) * 2 * SOS_KMAX_LDS;
    const long long aff_cap = (long long)rp.lds_bytes - rp.lds_mat_off - (long long)sizeof(double) * 2 * SOS_KMAX_LDS;
    double *s_red = sc.s_red;
    T *wy = reinterpret_cast<T *>(wbase);
    T *wx = wy + ((P.m + 63) & ~63);
    T *Tm = reinterpret_cast<T *>(ebase);
    T *u = TS<T>::u(P);
    T *v = TS<T>::v(P);
    T *vstore = TS<T>::vstore(P);
    bool warm = P.tk[2] != 0.0;
    if (threadIdx.x == 0) *sc.s_sweeps = 0;

    int it = 0;
    int status = 0;
    unsigned long long t_aff = 0, t_eig = 0, t_res = 0, t0 = 0;   // wall-clock ticks by phase
    // iteration budget: in an accumulating (second) phase, what the first phase left over
    int cap = rp.iters;
    if (rp.accumulate) {
        cap = rp.iters + (int)P.out[SOS_OUT_WARM] - (int)P.out[SOS_OUT_TOTAL];
        if (cap < rp.min_iters) cap = rp.min_iters;
    }
    // a warm start under judgement (first launch of a solve only)
    bool trying = rp.mode == RUN_SOLVE && !rp.accumulate && rp.warm_budget > 0 && P.tk[3] != 0.0;
    int it_warm = 0;   // iterations of an abandoned warm attempt
    double best = INFINITY, best_ce = INFINITY;
    bool was_cert = false;
    int since_best = 0;
    bool stalled = false;
    while (it < cap) {
        t0 = wall_clock64();
        affine_phase<T, NT, T>(P, rp, wy, wx, s_z, s_red, aff_lds, aff_cap);
        const unsigned long long t1 = wall_clock64();
        t_aff += t1 - t0;
        long long voff = 0;
        // two blocks that both take the lane-group form with G and V in LDS, in the block-cyclic
        // order, and fit in LDS together: projected at once
        const bool two = P.nblk == 2 && rp.jac_block == 8 && rp.lds_pair > 0 && [&] {
            for (int bk = 0; bk < 2; ++bk) {
                const int N = P.blk_N[bk];
                if (N < 2 || N > rp.lds_nmax || (N <= rp.rows_nmax && N >= rp.rows_nmin)) return false;
            }
            return sos_pair_need(P.blk_N[0], P.blk_N[1]) <= rp.lds_pair;
        }();
        if (two) {
            const int N0 = P.blk_N[0], N1 = P.blk_N[1];
            project_two<T, NT>(v + P.blk_off[0], u + P.blk_off[0], N0, rp.warm_eig ? vstore : nullptr, v + P.blk_off[1],
                               u + P.blk_off[1], N1, rp.warm_eig ? vstore + (long long)N0 * N0 : nullptr,
                               rp.warm_eig && warm, s_mat, Tm, s_sig, sc, rp.max_sweeps);
        }
        for (int bk = 0; bk < (two ? 0 : P.nblk); ++bk) {
            const int off = P.blk_off[bk];
            const int N = P.blk_N[bk];
            if (N <= rp.rows_nmax && N >= rp.rows_nmin) {
                // rows split over the wavefronts, G, V and partial sums in LDS
                project_block_rows<T, NT>(v + off, u + off, N, rp.warm_eig ? vstore + voff : nullptr,
                                          rp.warm_eig && warm, s_mat, Tm, sc, rp.max_sweeps);
                voff += (long long)N * N;
                continue;
            }
            const int ld = N;
            T *vc = rp.warm_eig ? vstore + voff : nullptr;
            const bool wm = rp.warm_eig && warm;
            const int gs = lanes_per_pair(rp, N);
            T *g1 = Tm + (long long)P.nmax * P.nmax, *g2 = g1 + (long long)P.nmax * P.nmax;
            if (N <= rp.lds_nmax)        // G and V in LDS, columns padded (lds_ld)
                project_block<T, NT>(v + off, u + off, N, vc, wm, s_mat, s_mat + (long long)N * lds_ld(N), lds_ld(N),
                                     Tm, s_sig, sc, rp.max_sweeps, gs, rp.jac_block);
            else if (N <= rp.lds_nmax_g)  // G in LDS, V in global scratch
                project_block<T, NT>(v + off, u + off, N, vc, wm, s_mat, g1, ld, Tm, s_sig, sc, rp.max_sweeps, gs);
            else                          // both in global scratch
                project_block<T, NT>(v + off, u + off, N, vc, wm, g1, g2, ld, Tm, s_sig, sc, rp.max_sweeps, gs);
            voff += (long long)N * N;
        }
        warm = rp.warm_eig != 0;
        ++it;
        const unsigned long long t2 = wall_clock64();
        t_eig += t2 - t1;
        if (rp.mode == RUN_SOLVE && it >= rp.min_iters &&
            (it % rp.check_every == 0 || it == cap || it == rp.min_iters)) {
            double pm[2] = {INFINITY, INFINITY};
            status = residual_phase<T, NT>(P, rp.tol, s_red, it_warm + it, pm);
            t_res += wall_clock64() - t2;
            if (status) break;
            if (trying && (!(P.tk[0] > 0.0) || it >= rp.warm_budget)) {
                // the warm start failed its trial: restart from the cold start u = v = (0, 0, 1)
                // with the full budget (the cold method as the fallback)
                __syncthreads();
                const int nu = P.nx + P.m;
                for (int e = threadIdx.x; e < nu; e += NT) {
                    u[e] = (T)0;
                    if (e < P.nx) v[e] = (T)0;
                }
                if (threadIdx.x == 0) {
                    P.tk[0] = 1.0;
                    P.tk[1] = 1.0;
                    P.tk[2] = 0.0;
                    P.tk[3] = 0.0;
                }
                __syncthreads();
                trying = false;
                warm = false;
                it_warm += it;
                it = 0;
                cap = rp.iters;
                best = INFINITY;
                best_ce = INFINITY;
                was_cert = false;
                since_best = 0;
                continue;
            }
            // a phase that stops improving hands over (the FP32 phase of the mixed form):
            // stalled once stall_checks checks in a row (three times as many while
            // tau = 0) missed 0.99 x the best value of the measure of the current
            // regime: the largest residual while tau > 0, the certificate error while
            // tau = 0 (each best kept per regime; a change of regime restarts the count)
            if (rp.stall_checks > 0) {
                const bool cert = !isfinite(pm[0]);
                bool better;
                if (!cert) {
                    better = pm[0] < 0.99 * best;
                    best = fmin(best, pm[0]);
                } else {
                    better = !isfinite(pm[1]) || pm[1] < 0.99 * best_ce;
                    best_ce = fmin(best_ce, pm[1]);
                }
                if (cert != was_cert) better = true;
                was_cert = cert;
                // the certificate error decays like 1/k with bumps, and the FP32
                // iterate carries it down to about 5 tol: a longer window there
                if (better) {
                    since_best = 0;
                } else if (++since_best >= (cert ? 3 * rp.stall_checks : rp.stall_checks)) {
                    stalled = true;
                    break;
                }
            }
        }
    }
    if (rp.mode == RUN_STEP || status == 0) {
        status = residual_phase<T, NT>(P, rp.tol, s_red, it_warm + it);
        if (rp.mode == RUN_SOLVE && status == 0 && !stalled && threadIdx.x == 0) P.out[SOS_OUT_STATUS] = 4;
    }
    if (threadIdx.x == 0) {
        P.out[SOS_OUT_T_AFFINE] = (double)t_aff;
        P.out[SOS_OUT_T_EIG] = (double)t_eig;
        P.out[SOS_OUT_T_RES] = (double)t_res;
        P.out[SOS_OUT_SWEEPS] = (it > 0 && P.nblk > 0) ? (double)(*sc.s_sweeps) / ((double)it * P.nblk) : 0.0;
        P.out[SOS_OUT_TOTAL] = (rp.accumulate ? P.out[SOS_OUT_TOTAL] : 0.0) + it_warm + it;
        if (!rp.accumulate) P.out[SOS_OUT_WARM] = it_warm;
        if (it > 0) P.tk[2] = rp.warm_eig ? 1.0 : 0.0;
        if (rp.mode == RUN_SOLVE) P.tk[3] = 0.0;   // judged (or never under judgement)
    }
    __syncthreads();
    return status;
}

template <typename T, int NT>
__global__ __launch_bounds__(NT, 2) void admm_persistent(RunParams rp) {
    __shared__ int s_idx;
    __shared__ int s_flag;
    __shared__ int s_sweeps;
    __shared__ double s_red[4 * (NT / 64)];
    extern __shared__ __attribute__((aligned(16))) char dyn_lds[];
    char *wbase = reinterpret_cast<char *>(rp.work) + (long long)blockIdx.x * rp.work_stride;
    char *ebase = reinterpret_cast<char *>(rp.eig) + (long long)blockIdx.x * rp.eig_stride;
    EigScratch sc;
    sc.s_flag = as_lds<int>((void *)&s_flag);
    sc.s_sweeps = as_lds<int>((void *)&s_sweeps);
    sc.s_red = s_red;
    sc.jtol = rp.jacobi_tol;
    if (rp.ts && threadIdx.x == 0) atomicMin(&rp.ts[0], (unsigned long long)wall_clock64());
    int prev = -1;
    for (;;) {
        // one thread-0 block per pass: it stamps the end of the previous problem and takes the
        // next one.  (A second thread-0 block at the end of the body, with only the back edge
        // between it and this one, lets the compiler merge the two into a path that reaches
        // the barrier below with part of wavefront 0 still outside it.)
        if (threadIdx.x == 0) {
            if (prev >= 0) rp.probs[prev].out[SOS_OUT_T_END] = (double)wall_clock64();
            s_idx = atomicAdd(rp.counter, 1);
        }
        __syncthreads();
        const int idx = __builtin_amdgcn_readfirstlane(s_idx);
        __syncthreads();
        if (idx >= rp.count) break;
        const int pid = __builtin_amdgcn_readfirstlane(rp.order[idx]);
        if (threadIdx.x == 0 && !rp.accumulate) rp.probs[pid].out[SOS_OUT_T_START] = (double)wall_clock64();
        run_phase<T, NT>(rp.probs[pid], rp, wbase, ebase, dyn_lds, sc);
        prev = pid;
    }
    if (rp.ts && threadIdx.x == 0) atomicMax(&rp.ts[1], (unsigned long long)wall_clock64());
}

// The mixed form in one launch: each problem runs its FP32 phase (rp32: to tol, a
// certificate, a stall or the budget), its iterate is widened to FP64 in place, and the
// same workgroup continues at once with the FP64 phase (rp64: the rest of the budget, at
// least the polish iterations).  No problem waits for another's FP32 phase to end.
template <int NT>
__global__ __launch_bounds__(NT, 2) void admm_mixed(RunParams rp32, RunParams rp64) {
    __shared__ int s_idx;
    __shared__ int s_flag;
    __shared__ int s_sweeps;
    __shared__ double s_red[4 * (NT / 64)];
    extern __shared__ __attribute__((aligned(16))) char dyn_lds[];
    char *wbase = reinterpret_cast<char *>(rp32.work) + (long long)blockIdx.x * rp32.work_stride;
    char *ebase = reinterpret_cast<char *>(rp32.eig) + (long long)blockIdx.x * rp32.eig_stride;
    EigScratch sc;
    sc.s_flag = as_lds<int>((void *)&s_flag);
    sc.s_sweeps = as_lds<int>((void *)&s_sweeps);
    sc.s_red = s_red;
    if (rp32.ts && threadIdx.x == 0) atomicMin(&rp32.ts[0], (unsigned long long)wall_clock64());
    int prev = -1;
    for (;;) {
        // one thread-0 block per pass (see admm_persistent)
        if (threadIdx.x == 0) {
            if (prev >= 0) rp32.probs[prev].out[SOS_OUT_T_END] = (double)wall_clock64();
            s_idx = atomicAdd(rp32.counter, 1);
        }
        __syncthreads();
        const int idx = __builtin_amdgcn_readfirstlane(s_idx);
        __syncthreads();
        if (idx >= rp32.count) break;
        const int pid = __builtin_amdgcn_readfirstlane(rp32.order[idx]);
        const ProbDesc &P = rp32.probs[pid];
        sc.jtol = rp32.jacobi_tol;
        if (threadIdx.x == 0) P.out[SOS_OUT_T_START] = (double)wall_clock64();
        run_phase<float, NT>(P, rp32, wbase, ebase, dyn_lds, sc);
        // widen the iterate; the cached FP64 eigenvectors are stale
        const int nu = P.nx + P.m;
        for (int e = threadIdx.x; e < nu; e += NT) {
            P.u64[e] = (double)P.u32[e];
            if (e < P.nx) P.v64[e] = (double)P.v32[e];
        }
        if (threadIdx.x == 0) P.tk[2] = 0.0;
        __syncthreads();
        sc.jtol = rp64.jacobi_tol;
        run_phase<double, NT>(P, rp64, wbase, ebase, dyn_lds, sc);
        prev = pid;
    }
    if (rp32.ts && threadIdx.x == 0) atomicMax(&rp32.ts[1], (unsigned long long)wall_clock64());
}

// ----------------------------------------------------------------------------- multi-workgroup path
// One problem spread over a cooperative grid: a software barrier over all workgroups (they are
// co-resident under a cooperative launch), with a bounded wait so that a missing workgroup
// ends the launch with an error flag instead of a hang.
__device__ __forceinline__ void grid_sync(CoopCtl *ctl) {
    __syncthreads();   // the workgroup's writes are ordered before thread 0's arrival
    if (threadIdx.x == 0) {
        const unsigned int g = __hip_atomic_load(&ctl->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // arrival: an agent-scope release (publishes the workgroup's writes) and acquire
        const unsigned int arrived = __hip_atomic_fetch_add(&ctl->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == gridDim.x - 1) {
            __hip_atomic_store(&ctl->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&ctl->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            // bounded wait (about a second, far beyond any barrier of a working launch); once a wait
            // has timed out, later barriers do not wait at all, so a broken launch still ends soon.
            // Polls are relaxed; one acquire fence after the release of the generation is seen
            long long spins = 0;
            while (__hip_atomic_load(&ctl->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g &&
                   !__hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > (1LL << 25)) {
                    __hip_atomic_store(&ctl->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
    }
    __syncthreads();
}

// Sum of one double per workgroup in workgroup order (the same bits in every workgroup): each
// workgroup writes its partial into parts[blockIdx.x], then the grid barrier, then all read.
__device__ __forceinline__ double grid_sum(double x, double *parts, CoopCtl *ctl, double *s_red1) {
    if (threadIdx.x == 0) parts[blockIdx.x] = x;
    grid_sync(ctl);
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int g = 0; g < (int)gridDim.x; ++g) t += __hip_atomic_load(&parts[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *s_red1 = t;
    }
    __syncthreads();
    const double t = *s_red1;
    grid_sync(ctl);   // parts may be reused right after
    return t;
}

// Rotation of the local columns p, q (G and V in LDS, leading dimension ld) by one wavefront.
template <typename T>
__device__ __forceinline__ int wave_rotate_pair(typename Lds<T>::type *gp, typename Lds<T>::type *gq,
                                                typename Lds<T>::type *vp, typename Lds<T>::type *vq, int N, T tol,
                                                T atol) {
    const int lane = threadIdx.x & 63;
    T al = 0, be = 0, ga = 0;
    for (int i = lane; i < N; i += 64) {
        const T a = gp[i], b = gq[i];
        al += a * a;
        be += b * b;
        ga += a * b;
    }
    al = wave_allsum(al);
    be = wave_allsum(be);
    ga = wave_allsum(ga);
    T c, s;
    if (!jacobi_rot<T>(al, be, ga, tol * tol, atol * atol, c, s)) return 0;
    for (int i = lane; i < N; i += 64) {
        const T a = gp[i], b = gq[i];
        gp[i] = c * a - s * b;
        gq[i] = s * a + c * b;
        const T x = vp[i], y = vq[i];
        vp[i] = c * x - s * y;
        vq[i] = s * x + c * y;
    }
    return ga * ga > tol * (al * be) ? 2 : 1;
}

// Dynamic LDS of gram_block_round for NT threads: NT / 64 partial Gram tiles, the Gram matrix C
// and the accumulated rotation Z (16 x 16 each), two flags.
__host__ __device__ constexpr size_t gram_round_lds_bytes(int nt) {
    return sizeof(double) * ((size_t)(nt / 64) * 256 + 2 * 256) + sizeof(int) * 2;
}

// One cyclic sweep of two-sided Jacobi on the 16 x 16 symmetric C (row-major, LDS) by one
// wavefront, accumulating the rotations in Z (set to I here): round-robin order, 8 disjoint
// rotations per round (rows, then columns of C, then columns of Z); lane l applies the rotations
// of pairs l / 16 and 4 + l / 16 to row or column l % 16 and computes their angles itself.  Since C = G_b^T G_b, rotating C
// on both sides by the rotation of columns p, q is that column rotation seen through the Gram
// matrix: the sweep is the one-sided sweep over the 16 columns, done on 16 x 16 numbers instead of
// on N-long columns.  A pair is rotated by jacobi_rot (same thresholds and angle as a column pair
// of the one-sided form).
__device__ __forceinline__ void small_jacobi16(double *C, double *Z, double tol2, double atol2) {
    const int lane = threadIdx.x & 63;
    for (int e = lane; e < 256; e += 64) Z[e] = (e >> 4) == (e & 15) ? 1.0 : 0.0;
    wave_order();
    const int j = lane & 15;   // this lane's column (row phase) and row (column phase)
    for (int r = 0; r < 15; ++r) {
        // the two pairs this lane works on, k = lane / 16 and 4 + lane / 16, each rotation computed
        // by the 16 lanes that apply it (no exchange of angles)
        int p[2], q[2];
        double c[2], sn[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            rr_pair(r, (lane >> 4) + 4 * h, 16, p[h], q[h]);
            if (!jacobi_rot<double>(C[p[h] * 16 + p[h]], C[q[h] * 16 + q[h]], C[p[h] * 16 + q[h]], tol2, atol2, c[h],
                                    sn[h])) {
                c[h] = 1.0;
                sn[h] = 0.0;
            }
        }
        wave_order();
#pragma unroll
        for (int h = 0; h < 2; ++h) {   // rows p, q of C: J^T C
            if (sn[h] != 0.0) {
                const double x = C[p[h] * 16 + j], y = C[q[h] * 16 + j];
                C[p[h] * 16 + j] = c[h] * x - sn[h] * y;
                C[q[h] * 16 + j] = sn[h] * x + c[h] * y;
            }
        }
        wave_order();
#pragma unroll
        for (int h = 0; h < 2; ++h) {   // columns p, q of C and Z: C J, Z J
            if (sn[h] != 0.0) {
                const double x = C[j * 16 + p[h]], y = C[j * 16 + q[h]];
                C[j * 16 + p[h]] = c[h] * x - sn[h] * y;
                C[j * 16 + q[h]] = sn[h] * x + c[h] * y;
                const double zx = Z[j * 16 + p[h]], zy = Z[j * 16 + q[h]];
                Z[j * 16 + p[h]] = c[h] * zx - sn[h] * zy;
                Z[j * 16 + q[h]] = sn[h] * zx + c[h] * zy;
            }
        }
        wave_order();
    }
}

// One block round of the multi-workgroup one-sided Jacobi, by one workgroup: the 16 columns of
// blocks P0 and Q0 (8 columns each, Q0 < 0 for none; columns at or past N are zero) of G and V
// (column-major, ld N, global).  Their Gram matrix C = G_b^T G_b on the matrix cores (FP64 MFMA,
// rows split over the wavefronts, partial tiles summed in wavefront order), its eigenvectors Z by
// small_jacobi16 on one wavefront, then G_b <- G_b Z and V_b <- V_b Z on the matrix cores (a
// wavefront per 16-row tile, in place): the same sweep over the 16 columns as rotating them pair
// by pair, in 15 short rounds on 16 x 16 numbers and one product instead of 15 dependent rounds
// over all N rows.  The update is skipped when no pair is
// coupled above the rotation thresholds.  Returns 1 (to every thread) if a pair had relative
// coupling above sqrt(tol), the sweep vote.
template <int NT>
__device__ __forceinline__ int gram_block_round(double *__restrict__ G, double *__restrict__ V, int N, int P0, int Q0,
                                                double tol, double atol, char *dyn_lds) {
    typedef Mma<double>::acc AC;
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    double *part = reinterpret_cast<double *>(dyn_lds);   // [NW][256]
    double *C = part + NW * 256, *Z = C + 256;
    int *flag = reinterpret_cast<int *>(Z + 256);
    // local column c (0..15) -> global column, -1 if absent
    auto gcol = [&](int c) -> int {
        const int g = c < 8 ? P0 * 8 + c : (Q0 >= 0 ? Q0 * 8 + c - 8 : N);
        return g < N ? g : -1;
    };
    const int myc = gcol(li);
    // C = G_b^T G_b: chunk of 16 rows per 4 MFMA steps, lane group lg taking rows k0 + 4 lg + t;
    // four chunks' loads in flight before their steps (the columns were last written by other
    // workgroups, so each load waits on the memory side)
    AC acc = (AC)0.0;
    for (int base = wid * 16; base < N; base += NW * 64) {
        double a[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int k = base + u * NW * 16 + 4 * lg + t;
                a[u][t] = (myc >= 0 && k < N) ? G[(long long)myc * N + k] : 0.0;
            }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc = Mma<double>::step(a[u][t], a[u][t], acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) part[wid * 256 + Mma<double>::row(lg, r) * 16 + li] = acc[r];
    __syncthreads();
    if (tid < 256) {
        double c = 0.0;
        for (int w = 0; w < NW; ++w) c += part[w * 256 + tid];
        C[tid] = c;
    }
    __syncthreads();
    const double tol2 = tol * tol, atol2 = atol * atol;
    if (wid == 0) {
        // the pairs' couplings before the round: the sweep vote and whether to rotate at all
        int big = 0, need = 0;
        for (int e = lane; e < 256; e += 64) {
            const int p = e >> 4, q = e & 15;
            if (p < q) {
                const double app = C[p * 16 + p], aqq = C[q * 16 + q], apq = C[e];
                const double g2 = apq * apq;
                if (g2 > atol2 * (app > aqq ? app : aqq)) {
                    if (g2 > tol2 * (app * aqq)) need = 1;
                    if (g2 > tol * (app * aqq)) big = 1;
                }
            }
        }
        need = __any(need);
        big = __any(big);
        if (lane == 0) {
            flag[0] = need;
            flag[1] = big;
        }
    }
    __syncthreads();
    const int need = flag[0], big = flag[1];
    if (need) {
        // G_b <- G_b Z and V_b <- V_b Z: a 16-row tile per wavefront at a time, lane group lg taking
        // Z's rows 4 lg + t in step t; output row lg + 4 r, column li.  Wavefront 0 computes Z (one
        // inner sweep) while the others load their first four tiles; then four tiles' loads in
        // flight at a time
        const int nt = (N + 15) >> 4;
        int cols[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) cols[t] = gcol(4 * lg + t);
        double a[4][4];
        auto load_batch = [&](int base) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int tile = base + u * NW;
                const double *M = tile < nt ? G : V;
                const int row = (tile < nt ? tile : tile - nt) * 16 + li;
                const bool ok = tile < 2 * nt && row < N;
#pragma unroll
                for (int t = 0; t < 4; ++t) a[u][t] = (ok && cols[t] >= 0) ? M[(long long)cols[t] * N + row] : 0.0;
            }
        };
        if (wid == 0) small_jacobi16(C, Z, tol2, atol2);
        else load_batch(wid);
        __syncthreads();
        double b[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) b[t] = Z[(4 * lg + t) * 16 + li];
        for (int base = wid; base < 2 * nt; base += 4 * NW) {
            if (wid == 0 || base != wid) load_batch(base);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int tile = base + u * NW;
                if (tile >= 2 * nt) break;
                double *M = tile < nt ? G : V;
                const int r0 = (tile < nt ? tile : tile - nt) * 16;
                AC d = (AC)0.0;
#pragma unroll
                for (int t = 0; t < 4; ++t) d = Mma<double>::step(a[u][t], b[t], d);
                if (myc >= 0) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = r0 + Mma<double>::row(lg, r);
                        if (i < N) M[(long long)myc * N + i] = d[r];
                    }
                }
            }
        }
    }
    __syncthreads();
    return big;
}

// P_{S+} of one block over the whole grid: G, V, W (N x N, column-major, ld N) and sigma (N) in
// global scratch.  Block one-sided Jacobi: the columns form blocks of 8; in each block round
// (round-robin over the blocks, as the scalar form pairs columns) a workgroup orthogonalises the
// 16 columns of a pair of blocks at once (gram_block_round); a grid barrier ends the round.  Every
// pair of columns meets once per sweep of block rounds; sweeps stop as in the single-workgroup
// forms (a sweep whose pairs all had relative coupling at most sqrt(tol)), the vote collected in
// global memory.  Every workgroup passes the same barriers: the same block rounds per sweep, and
// the same vote after the last.
template <typename T, int NT>
__device__ __noinline__ void coop_project_block(T *__restrict__ vs, T *__restrict__ us, int N, T *__restrict__ Vs,
                                                bool warm, T *__restrict__ G, T *__restrict__ V, T *__restrict__ W,
                                                T *__restrict__ sig, double *parts, CoopCtl *ctl,
                                                int max_sweeps, double jtol, char *dyn_lds, double *s_red,
                                                double *s_red1, int *nsweeps, int &gsw) {
    typedef typename Lds<T>::type LT;
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int wg = blockIdx.x, nwg = gridDim.x;
    const long long gt = (long long)wg * NT + tid, gstride = (long long)nwg * NT;
    const int w0 = wg * NW + wid, nw = nwg * NW;
    // stage: G = W and V = I (cold), or W and V = V_prev (warm); |W|_F^2 from the packed triangle
    double fro2 = 0.0;
    for (long long idx = gt; idx < (long long)N * N; idx += gstride) {
        const int j = (int)(idx / N), i = (int)(idx - (long long)j * N);
        const int a = i > j ? i : j, b = i > j ? j : i;
        const T x = vs[svec_idx(a, b, N)];
        if (warm) {
            W[idx] = x;
            V[idx] = Vs[idx];
        } else {
            G[idx] = x;
            V[idx] = (i == j) ? (T)1 : (T)0;
        }
        fro2 += (double)x * (double)x;
    }
    {
        double d = 0.0;
        block_sum2<NT>(fro2, d, s_red);   // every thread: this workgroup's part
    }
    fro2 = grid_sum(fro2, parts, ctl, s_red1);   // its barriers also publish G, V, W
    if (warm) {
        mfma_wv<T, NT>(W, N, true, V, N, G, N, N, false, w0, nw);
        grid_sync(ctl);
    }
    const T tol = jacobi_tol<T>(jtol);
    const T atol = (T)(jacobi_atol_factor(N) * TS<T>::eps * sqrt(fro2));
    const int nb = (N + 7) / 8, nbp = nb + (nb & 1);
    __shared__ int s_big;
    int sweep = 0;
    while (sweep < max_sweeps) {
        // vote flags by the launch's running sweep count gsw (a projection's first sweep continues
        // where the last one stopped, so no flag is read before it was reset for its sweep)
        const int fl = gsw % 3;
        if (wg == 0 && tid == 0) __hip_atomic_store(&ctl->big[(gsw + 1) % 3], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (tid == 0) s_big = 0;
        __syncthreads();
        for (int R = 0; R < nbp - 1; ++R) {
            for (int pk = wg; pk < nbp / 2; pk += nwg) {
                int P0, Q0;
                rr_pair(R, pk, nbp, P0, Q0);
                if (gram_block_round<NT>(G, V, N, P0, Q0 < nb ? Q0 : -1, tol, atol, dyn_lds) && tid == 0) s_big = 1;
            }
            __syncthreads();
            if (R == nbp - 2 && tid == 0 && s_big)
                __hip_atomic_store(&ctl->big[fl], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            grid_sync(ctl);
        }
        const int any = __hip_atomic_load(&ctl->big[fl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ++sweep;
        ++gsw;
        if (!any) break;
    }
    if (wg == 0 && tid == 0) *nsweeps += sweep;
    // sigma_j = |g_j|, one wavefront per column
    for (int j = w0; j < N; j += nw) {
        T sacc = 0;
        for (int i = lane; i < N; i += 64) sacc += G[(long long)j * N + i] * G[(long long)j * N + i];
        sacc = wave_allsum(sacc);
        if (lane == 0) sig[j] = sqrt(sacc);
    }
    grid_sync(ctl);
    mfma_rebuild<T, NT>(V, N, sig, N, vs, us, w0, nw);
    if (Vs)
        for (long long idx = gt; idx < (long long)N * N; idx += gstride) Vs[idx] = V[idx];
    grid_sync(ctl);
}

// The affine step (Section IV-A, the projection onto the embedding's subspace, with the
// inverse of Section IV-B) of one FP64 problem spread over the cooperative grid: the same phases
// and per-row arithmetic as affine_phase, each phase over all workgroups with a grid barrier
// after it.  A^T_f x and S^{-1} (A^T_f x) live in global scratch (kq, kz, k entries each); the
// product with S^{-1} takes whole rows per wavefront (S^{-1} is symmetric, so a row is a
// contiguous column), each workgroup always the same rows; the two inner products that give
// theta are summed in workgroup order (parts, two per workgroup), so every workgroup computes the
// same theta.  Ends without a barrier: the caller's next grid barrier publishes u, v and tau.
template <int NT>
__device__ __noinline__ void coop_affine_phase(const ProbDesc &P, const RunParams &rp, double *__restrict__ wy,
                                               double *__restrict__ wx, double *__restrict__ kq,
                                               double *__restrict__ kz, double *parts, CoopCtl *ctl,
                                               double *s_red) {
    typedef double T;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    constexpr int NW = NT / 64;
    const int wg = blockIdx.x, nwg = gridDim.x;
    const long long gt = (long long)wg * NT + tid, gstride = (long long)nwg * NT;
    const long long ggrp = gt >> 3, ngrp = gstride >> 3;
    const int gw = wg * NW + wid, ngw = nwg * NW;
    const int m = P.m, nx = P.nx, k = P.k, nfree = P.nfree;
    T *__restrict__ u = P.u64;
    T *__restrict__ v = P.v64;
    const T *__restrict__ val = P.val64;
    const T *__restrict__ colval = P.colval64;
    const T *__restrict__ fval = P.fval64;
    const T *__restrict__ frval = P.frval64;
    const T *__restrict__ dinv = P.dinv64;
    const T *__restrict__ h = P.h64;
    const T *__restrict__ b = P.b64;
    const T *__restrict__ c = P.c64;
    const T *__restrict__ cw = P.cw64;
    const int *__restrict__ rowptr = P.rowptr;
    const int *__restrict__ colidx = P.colidx;
    const int *__restrict__ colrow = P.colrow;
    const double tau = P.tk[0], kap = P.tk[1];
    const double wt = tau + kap;
    const T *__restrict__ uy = u + nx;
    const int gl = tid & 7;

    // P1: x = (w2 - A w1) / d, rows over the grid
    for (long long a = gt; a < m; a += gstride) {
        T acc = uy[a] + b[a] * wt;
        T acc1 = 0, acc2 = 0, acc3 = 0;
        const int e1 = rowptr[a + 1];
        int e = rowptr[a];
        for (; e + 4 <= e1; e += 4) {
            const int j0 = colidx[e], j1 = colidx[e + 1], j2 = colidx[e + 2], j3 = colidx[e + 3];
            acc -= val[e] * (u[j0] + v[j0] - c[j0] * wt);
            acc1 -= val[e + 1] * (u[j1] + v[j1] - c[j1] * wt);
            acc2 -= val[e + 2] * (u[j2] + v[j2] - c[j2] * wt);
            acc3 -= val[e + 3] * (u[j3] + v[j3] - c[j3] * wt);
        }
        for (; e < e1; ++e) {
            const int j = colidx[e];
            acc -= val[e] * (u[j] + v[j] - c[j] * wt);
        }
        wy[a] = (acc + acc1 + (acc2 + acc3)) * dinv[a];
    }
    grid_sync(ctl);

    if (k > 0) {
        // P2: q = A_f^T x (a group of 8 lanes per column), then z = S^{-1} q (a wavefront per row)
        const int *__restrict__ fptr = P.fptr;
        const int *__restrict__ frow = P.frow;
        for (long long j = ggrp; j < k; j += ngrp) {
            double s = 0.0;
            const int e1 = fptr[j + 1];
            for (int e = fptr[j] + gl; e < e1; e += 8) s += fval[e] * wy[frow[e]];
            s = group_allsum<8>(s);
            if (gl == 0) kq[j] = s;
        }
        grid_sync(ctl);
        const double *__restrict__ Sinv = P.Sinv;
        for (int i = gw; i < k; i += ngw) {
            const double *__restrict__ row = Sinv + (long long)i * k;
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            int j = lane;
            for (; j + 192 < k; j += 256) {
                a0 += row[j] * kq[j];
                a1 += row[j + 64] * kq[j + 64];
                a2 += row[j + 128] * kq[j + 128];
                a3 += row[j + 192] * kq[j + 192];
            }
            for (; j < k; j += 64) a0 += row[j] * kq[j];
            const double t = wave_allsum((a0 + a1) + (a2 + a3));
            if (lane == 0) kz[i] = t;
        }
        grid_sync(ctl);
    }

    // P3: sigma_2 = x - D^{-1} A_f z ; partial b^T sigma_2
    double bs = 0.0;
    {
        const int *__restrict__ frptr = P.frptr;
        const int *__restrict__ frcol = P.frcol;
        for (long long a = gt; a < m; a += gstride) {
            T s2 = wy[a];
            if (k > 0) {
                double acc = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
                const int e1 = frptr[a + 1];
                int e = frptr[a];
                for (; e + 4 <= e1; e += 4) {
                    acc += frval[e] * kz[frcol[e]];
                    acc1 += frval[e + 1] * kz[frcol[e + 1]];
                    acc2 += frval[e + 2] * kz[frcol[e + 2]];
                    acc3 += frval[e + 3] * kz[frcol[e + 3]];
                }
                for (; e < e1; ++e) acc += frval[e] * kz[frcol[e]];
                s2 = s2 - ((acc + acc1) + (acc2 + acc3)) * dinv[a];
            }
            wy[a] = s2;
            bs += b[a] * s2;
        }
    }
    grid_sync(ctl);

    // P4: sigma_1 = w1 + A^T sigma_2 ; partial c^T sigma_1
    double cs = 0.0;
    {
        for (long long e = gt; e < nx; e += gstride) {
            const int r = colrow[e];
            if (r <= -2) continue;
            const T w1 = u[e] + v[e] - c[e] * wt;
            const T s1 = r >= 0 ? w1 + colval[e] * wy[r] : w1;
            wx[e] = s1;
            cs += cw[e] * s1;
        }
        const int *__restrict__ fptr = P.fptr;
        const int *__restrict__ frow = P.frow;
        const int *__restrict__ fcol = P.fcol;
        for (long long j = ggrp; j < k; j += ngrp) {
            T acc = 0;
            const int i1 = fptr[j + 1];
            for (int i = fptr[j] + gl; i < i1; i += 8) acc += fval[i] * wy[frow[i]];
            acc = group_allsum<8>(acc);
            if (gl == 0) {
                const int e = fcol[j];
                const T s1 = u[e] + v[e] - c[e] * wt + acc;
                wx[e] = s1;
                cs += cw[e] * s1;
            }
        }
    }
    block_sum2<NT>(cs, bs, s_red);
    if (tid == 0) {
        parts[2 * wg] = cs;
        parts[2 * wg + 1] = bs;
    }
    grid_sync(ctl);
    if (tid == 0) {
        double tc = 0.0, tb = 0.0;
        for (int g = 0; g < nwg; ++g) {
            tc += __hip_atomic_load(&parts[2 * g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            tb += __hip_atomic_load(&parts[2 * g + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        s_red[0] = tc;
        s_red[1] = tb;
    }
    __syncthreads();
    const double theta = (s_red[0] - s_red[1]) / P.eta;
    const double al = rp.alpha;
    const bool relax = rp.alpha != 1.0;

    // P5: u_hat, w = u_hat - v, direct updates of the free, y and tau parts
    for (long long e = gt; e < nx; e += gstride) {
        T uh = wx[e] - theta * h[e];
        if (relax) uh = al * uh + (1.0 - al) * u[e];
        const T w = uh - v[e];
        if (e < nfree) {
            u[e] = w;
            v[e] = 0.0;
        } else {
            v[e] = w;
        }
    }
    for (long long a = gt; a < m; a += gstride) {
        T uh = wy[a] - theta * h[nx + a];
        if (relax) uh = al * uh + (1.0 - al) * u[nx + a];
        u[nx + a] = uh;
    }
    if (wg == 0 && tid == 0) {
        double uht = wt + theta;
        if (relax) uht = al * uht + (1.0 - al) * tau;
        const double wtt = uht - kap;
        const double tn = wtt > 0.0 ? wtt : 0.0;
        P.tk[0] = tn;
        P.tk[1] = tn - wtt;
    }
}

// Whole FP64 iterations of one problem over a cooperative grid (see sos_launch_admm_coop).
template <int NT>
__global__ __launch_bounds__(NT) void admm_coop(RunParams rp, CoopCtl *ctl, double *scr) {
    typedef double T;
    __shared__ double s_red[4 * (NT / 64)];
    __shared__ double s_red1;
    __shared__ int s_sweeps;
    extern __shared__ __attribute__((aligned(16))) char dyn_lds[];
    const ProbDesc &P = rp.probs[0];
    const int wg = blockIdx.x, tid = threadIdx.x;
    const int nm = P.nmax;
    T *G = scr, *V = G + (long long)nm * nm, *W = V + (long long)nm * nm, *sig = W + (long long)nm * nm;
    double *parts = sig + nm;                            // 2 per workgroup
    double *kq = parts + 2 * SOS_COOP_MAX_WG, *kz = kq + ((P.k + 63) & ~63);
    T *wy = reinterpret_cast<T *>(rp.work);
    T *wx = wy + ((P.m + 63) & ~63);
    T *u = P.u64, *v = P.v64, *vstore = P.vs64;
    bool warm = P.tk[2] != 0.0;
    if (tid == 0) s_sweeps = 0;
    int it = 0, status = 0, gsw = 0;
    unsigned long long t_aff = 0, t_eig = 0, t_res = 0;
    const int cap = rp.iters;
    while (it < cap) {
        const unsigned long long t0 = wall_clock64();
        coop_affine_phase<NT>(P, rp, wy, wx, kq, kz, parts, ctl, s_red);
        grid_sync(ctl);
        const unsigned long long t1 = wall_clock64();
        t_aff += t1 - t0;
        long long voff = 0;
        for (int bk = 0; bk < P.nblk; ++bk) {
            const int off = P.blk_off[bk], N = P.blk_N[bk];
            coop_project_block<T, NT>(v + off, u + off, N, rp.warm_eig ? vstore + voff : nullptr, rp.warm_eig && warm, G, V,
                                      W, sig, parts, ctl, rp.max_sweeps, rp.jacobi_tol, dyn_lds, s_red, &s_red1,
                                      &s_sweeps, gsw);
            voff += (long long)N * N;
        }
        warm = rp.warm_eig != 0;
        ++it;
        const unsigned long long t2 = wall_clock64();
        t_eig += t2 - t1;
        if (rp.mode == RUN_SOLVE && (it % rp.check_every == 0 || it == cap)) {
            if (wg == 0) {
                const int st = residual_phase<T, NT>(P, rp.tol, s_red, it);
                if (tid == 0) __hip_atomic_store(&ctl->status, st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            grid_sync(ctl);
            status = __hip_atomic_load(&ctl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            t_res += wall_clock64() - t2;
            if (status) break;
        }
    }
    if (wg == 0) {
        if (rp.mode == RUN_STEP || status == 0) {
            status = residual_phase<T, NT>(P, rp.tol, s_red, it);
            if (rp.mode == RUN_SOLVE && status == 0 && tid == 0) P.out[SOS_OUT_STATUS] = 4;
        }
        if (tid == 0) {
            P.out[SOS_OUT_T_AFFINE] = (double)t_aff;
            P.out[SOS_OUT_T_EIG] = (double)t_eig;
            P.out[SOS_OUT_T_RES] = (double)t_res;
            P.out[SOS_OUT_SWEEPS] = (it > 0 && P.nblk > 0) ? (double)s_sweeps / ((double)it * P.nblk) : 0.0;
            P.out[SOS_OUT_TOTAL] = it;
            P.out[SOS_OUT_WARM] = 0;
            if (it > 0) P.tk[2] = rp.warm_eig ? 1.0 : 0.0;
            if (rp.mode == RUN_SOLVE) P.tk[3] = 0.0;
        }
    }
}

__global__ void reset_coop(CoopCtl *ctl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->count = 0;
        ctl->gen = 0;
        ctl->err = 0;
        ctl->status = 0;
        ctl->big[0] = ctl->big[1] = ctl->big[2] = 0;
    }
}

// Learned warm start: from a predicted (xi, y) (FP32 rows, internal layout), set
//   u = (P_K(xi), y, 1),  v = (P_{K*}(c - A^T y), 0, 0)
// for every problem of a batch.  Launched on the batch's persistent grid (whose
// per-workgroup scratch areas exist), each workgroup takes problems blockIdx.x,
// blockIdx.x + gridDim.x, ...
template <typename T, int NT>
__global__ __launch_bounds__(NT) void warm_start_kernel(RunParams rp, const float *__restrict__ pred, long long ld) {
    __shared__ int s_flag;
    __shared__ int s_sweeps;
    __shared__ double s_red[4 * (NT / 64)];
    extern __shared__ __attribute__((aligned(16))) char dyn_lds[];
    typename Lds<T>::type *s_sig = as_lds<T>(dyn_lds);
    typename Lds<T>::type *s_mat = as_lds<T>(dyn_lds + rp.lds_mat_off);
    char *wbase = reinterpret_cast<char *>(rp.work) + (long long)blockIdx.x * rp.work_stride;
    char *ebase = reinterpret_cast<char *>(rp.eig) + (long long)blockIdx.x * rp.eig_stride;
    T *wx = reinterpret_cast<T *>(wbase);
    T *Tm = reinterpret_cast<T *>(ebase);
    EigScratch sc;
    sc.s_flag = as_lds<int>((void *)&s_flag);
    sc.s_sweeps = as_lds<int>((void *)&s_sweeps);
    sc.s_red = s_red;
    sc.jtol = 0.0;
    for (int p = blockIdx.x; p < rp.count; p += gridDim.x) {
    const ProbDesc &P = rp.probs[p];
    T *u = TS<T>::u(P);
    T *v = TS<T>::v(P);
    const float *xs = pred + (long long)p * ld;
    const float *ys = xs + P.nx;
    const int tid = threadIdx.x;
    for (int i = tid; i < P.m; i += NT) u[P.nx + i] = (T)ys[i];
    for (int e = tid; e < P.nx; e += NT) {
        u[e] = (T)xs[e];
        double aty = 0.0;
        const int r = P.colrow[e];
        if (r >= 0) {
            aty = P.colval64[e] * (double)ys[r];
        } else if (r <= -2) {
            const int j = -2 - r;
            for (int i = P.fptr[j]; i < P.fptr[j + 1]; ++i) aty += P.fval64[i] * (double)ys[P.frow[i]];
        }
        v[e] = e < P.nfree ? (T)0 : (T)(P.c64[e] - aty);
    }
    __syncthreads();
    for (int bk = 0; bk < P.nblk; ++bk) {
        const int off = P.blk_off[bk];
        const int N = P.blk_N[bk];
        const int ns = N * (N + 1) / 2;
        T *g1 = Tm + (long long)P.nmax * P.nmax, *g2 = g1 + (long long)P.nmax * P.nmax;
        for (int pass = 0; pass < 2; ++pass) {
            T *blk = (pass == 0 ? u : v) + off;   // projected in place via the scratch wx
            if (N <= rp.rows_nmax && N >= rp.rows_nmin) {
                project_block_rows<T, NT>(blk, wx, N, nullptr, false, s_mat, Tm, sc, rp.max_sweeps);
            } else if (N <= rp.lds_nmax) {
                project_block<T, NT>(blk, wx, N, nullptr, false, s_mat, s_mat + (long long)N * lds_ld(N), lds_ld(N), Tm,
                                     s_sig, sc, rp.max_sweeps, lanes_per_pair(rp, N));
            } else if (N <= rp.lds_nmax_g) {
                project_block<T, NT>(blk, wx, N, nullptr, false, s_mat, g1, N, Tm, s_sig, sc, rp.max_sweeps,
                                     lanes_per_pair(rp, N));
            } else {
                project_block<T, NT>(blk, wx, N, nullptr, false, g1, g2, N, Tm, s_sig, sc, rp.max_sweeps,
                                     lanes_per_pair(rp, N));
            }
            for (int s = tid; s < ns; s += NT) blk[s] = wx[s];
            __syncthreads();
        }
    }
    if (tid == 0) {
        P.tk[0] = 1.0;
        P.tk[1] = 0.0;
        P.tk[2] = 0.0;
        P.tk[3] = 1.0;   // a warm start, to be judged by the next solve
    }
    __syncthreads();
    }
}

// Eigen-decomposition of one PSD block of the current solution, X = xi / tau (dual = 0) or
// Z = z / tau (dual = 1), by the projection's own Jacobi eigensolver (cold start, FP64, full
// accuracy): eigenvectors column-major into evecs (N x N), eigenvalues as Rayleigh quotients
// v_j^T W v_j (signed) into evals.  One workgroup on problem 0 of rp.  W is staged in the
// eigensolver scratch Tm, which a cold projection does not use; the projection's own output
// goes to the work area.
template <int NT>
__global__ __launch_bounds__(NT) void psd_factor_kernel(RunParams rp, int blk, int dual, double *__restrict__ evals,
                                                      double *__restrict__ evecs) {
    __shared__ int s_flag;
    __shared__ int s_sweeps;
    __shared__ double s_red[4 * (NT / 64)];
    extern __shared__ __attribute__((aligned(16))) char dyn_lds[];
    typename Lds<double>::type *s_sig = as_lds<double>(dyn_lds);
    typename Lds<double>::type *s_mat = as_lds<double>(dyn_lds + rp.lds_mat_off);
    EigScratch sc;
    sc.s_flag = as_lds<int>((void *)&s_flag);
    sc.s_sweeps = as_lds<int>((void *)&s_sweeps);
    sc.s_red = s_red;
    sc.jtol = 0.0;
    if (threadIdx.x == 0) s_sweeps = 0;
    const ProbDesc &P = rp.probs[0];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    constexpr int NW = NT / 64;
    const int off = P.blk_off[blk], N = P.blk_N[blk], ns = N * (N + 1) / 2;
    const double inv_tau = 1.0 / P.tk[0];
    const double *src = (dual ? P.v64 : P.u64) + off;
    double *Tm = reinterpret_cast<double *>(rp.eig);
    double *wout = reinterpret_cast<double *>(rp.work);
    for (int e = tid; e < ns; e += NT) Tm[e] = src[e] * inv_tau;
    __syncthreads();
    double *g1 = Tm + (long long)P.nmax * P.nmax, *g2 = g1 + (long long)P.nmax * P.nmax;
    if (N <= rp.rows_nmax && N >= rp.rows_nmin)
        project_block_rows<double, NT>(Tm, wout, N, evecs, false, s_mat, Tm, sc, rp.max_sweeps);
    else if (N <= rp.lds_nmax)
        project_block<double, NT>(Tm, wout, N, evecs, false, s_mat, s_mat + (long long)N * lds_ld(N), lds_ld(N), Tm,
                                  s_sig, sc, rp.max_sweeps, lanes_per_pair(rp, N));
    else if (N <= rp.lds_nmax_g)
        project_block<double, NT>(Tm, wout, N, evecs, false, s_mat, g1, N, Tm, s_sig, sc, rp.max_sweeps,
                                  lanes_per_pair(rp, N));
    else
        project_block<double, NT>(Tm, wout, N, evecs, false, g1, g2, N, Tm, s_sig, sc, rp.max_sweeps,
                                  lanes_per_pair(rp, N));
    // Rayleigh quotients with W read from the iterate (the staged copy was overwritten)
    for (int j = wid; j < N; j += NW) {
        const double *vj = evecs + (long long)j * N;
        double acc = 0.0;
        for (int i = lane; i < N; i += 64) {
            double wv = 0.0;
            for (int k = 0; k < N; ++k) {
                const int a = i > k ? i : k, b = i > k ? k : i;
                wv += src[svec_idx(a, b, N)] * vj[k];
            }
            acc += vj[i] * wv;
        }
        acc = wave_allsum(acc);
        if (lane == 0) evals[j] = acc * inv_tau;
    }
}

// rows of out (ld apart): [xi / tau (nx) | y / tau (m)] of every problem, FP32, internal layout
template <typename T>
__global__ void export_solution(const ProbDesc *probs, int count, float *out, long long ld) {
    const int p = blockIdx.y;
    if (p >= count) return;
    const ProbDesc &P = probs[p];
    const T *u = TS<T>::u(P);
    const double tau = P.tk[0];
    const double s = tau > 0.0 ? 1.0 / tau : 0.0;
    const int n = P.nx + P.m;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        out[(long long)p * ld + i] = (float)((double)u[i] * s);
}

__global__ void reset_counter(int *c, unsigned long long *ts) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *c = 0;
        if (ts) {
            ts[0] = ~0ull;
            ts[1] = 0ull;
        }
    }
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
    if (blockIdx.x == 0 && threadIdx.x == 0) P.tk[2] = 0.0;   // the other precision's eigenvectors are stale
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
        P.tk[2] = 0.0;
        P.tk[3] = 0.0;
    }
}

// Launch diagnostics: an error an earlier asynchronous call left pending is reported (not
// cleared silently) before a launch, and a failed launch leaves its HIP error string.
thread_local char g_launch_msg[256] = "";
bool launch_precheck() {
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return true;
    snprintf(g_launch_msg, sizeof(g_launch_msg), "HIP error pending from an earlier call: %s", hipGetErrorString(e));
    return false;
}
int launch_result() {
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess) return 0;
    snprintf(g_launch_msg, sizeof(g_launch_msg), "kernel launch: %s", hipGetErrorString(e));
    return -4;
}

// Dynamic LDS layout for element type T: sigma, then the eigen region: the rows form's G, V,
// partial records and sigma for blocks up to rows_nmax (eig_wave 2); for the lane-group form,
// G and V (both N x N) up to lds_nmax, or G alone up to lds_nmax_g (larger blocks work in
// global scratch).  The affine step's k-vector and partial sums alias the eigen region.
template <typename T>
void lds_layout(int eig_ld, int lds_budget, int nw, int &mat_off, int &lds_nmax, int &lds_nmax_g, size_t &bytes,
                int eig_wave, int &rows_nmax) {
    size_t off = sizeof(T) * (size_t)(eig_ld + 1);
    off = (off + 15) & ~(size_t)15;
    mat_off = (int)off;
    lds_nmax = lds_nmax_g = 0;
    for (int N = eig_ld; N >= 2 && !lds_nmax; --N)
        if ((long long)(off + sizeof(T) * 2 * (size_t)N * lds_ld(N)) <= lds_budget) lds_nmax = N;
    for (int N = eig_ld; N >= 2 && !lds_nmax_g; --N)
        if ((long long)(off + sizeof(T) * (size_t)N * N) <= lds_budget) lds_nmax_g = N;
    const size_t need2 = lds_nmax ? off + sizeof(T) * 2 * (size_t)lds_nmax * lds_ld(lds_nmax) : off;
    const size_t need1 = lds_nmax_g ? off + sizeof(T) * (size_t)lds_nmax_g * lds_nmax_g : off;
    bytes = need2 > need1 ? need2 : need1;
    // rows-per-wavefront form (eig_wave 2): G, V, partial records and sigma of one block
    rows_nmax = 0;
    size_t need3 = off;
    if (eig_wave == 2) {
        for (int N = eig_ld; N >= 1 && !rows_nmax; --N)
            if ((long long)(off + sizeof(T) * (size_t)rows_region(N, (int)sizeof(T), nw)) <= lds_budget) rows_nmax = N;
        if (rows_nmax) need3 = off + sizeof(T) * (size_t)rows_region(rows_nmax, (int)sizeof(T), nw);
    }
    if (need3 > bytes) bytes = need3;
    // the affine step's k-vector and partial sums alias the eigen region
    const size_t need_z = off + sizeof(double) * 2 * SOS_KMAX_LDS;
    if (need_z > bytes) bytes = need_z;
}

// LDS for projecting a two-block problem's blocks at once (project_two): enlarges the launch's
// dynamic LDS to hold both blocks' G and V after the sigma area when the budget allows.
template <typename T>
void pair_layout(RunParams &rp, size_t &bytes) {
    rp.lds_pair = 0;
    if (rp.pair_need <= 0) return;
    const size_t need = (size_t)rp.lds_mat_off + sizeof(T) * (size_t)rp.pair_need;
    if (need > (size_t)rp.lds_budget) return;
    rp.lds_pair = rp.pair_need;
    if (need > bytes) bytes = need;
}

template <typename T, int NT>
int launch_t(int grid, const RunParams &rp_in, hipStream_t st) {
    RunParams rp = rp_in;
    size_t lds = 0;
    lds_layout<T>(rp.eig_ld, rp.lds_budget, NT / 64, rp.lds_mat_off, rp.lds_nmax, rp.lds_nmax_g, lds, rp.eig_wave,
                  rp.rows_nmax);
    pair_layout<T>(rp, lds);
    rp.lds_bytes = (long long)lds;
    if (lds > 64 * 1024) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&admm_persistent<T, NT>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipGetLastError();   // not every runtime needs (or accepts during capture) the attribute
    }
    hipLaunchKernelGGL((admm_persistent<T, NT>), dim3(grid), dim3(NT), lds, st, rp);
    return launch_result();
}

template <int NT>
int launch_mixed(int grid, const RunParams &rp32_in, const RunParams &rp64_in, hipStream_t st) {
    RunParams rp32 = rp32_in, rp64 = rp64_in;
    size_t lds32 = 0, lds64 = 0;
    lds_layout<float>(rp32.eig_ld, rp32.lds_budget, NT / 64, rp32.lds_mat_off, rp32.lds_nmax, rp32.lds_nmax_g, lds32,
                      rp32.eig_wave, rp32.rows_nmax);
    lds_layout<double>(rp64.eig_ld, rp64.lds_budget, NT / 64, rp64.lds_mat_off, rp64.lds_nmax, rp64.lds_nmax_g, lds64,
                       rp64.eig_wave, rp64.rows_nmax);
    pair_layout<float>(rp32, lds32);
    pair_layout<double>(rp64, lds64);
    const size_t lds = lds32 > lds64 ? lds32 : lds64;
    rp32.lds_bytes = rp64.lds_bytes = (long long)lds;   // one allocation serves both phases
    if (lds > 64 * 1024) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&admm_mixed<NT>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipGetLastError();
    }
    hipLaunchKernelGGL((admm_mixed<NT>), dim3(grid), dim3(NT), lds, st, rp32, rp64);
    return launch_result();
}

}   // namespace

const char *sos_launch_message() { return g_launch_msg; }

int sos_launch_admm_mixed(int threads, int grid, const RunParams &rp32, const RunParams &rp64, void *stream) {
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    switch (threads) {
        case 256: return launch_mixed<256>(grid, rp32, rp64, st);
        case 512: return launch_mixed<512>(grid, rp32, rp64, st);
    }
    return -1;   // other widths: the caller uses the two-launch form
}

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

int sos_launch_reset(int *counter, void *stream, unsigned long long *ts) {
    if (!launch_precheck()) return -4;
    hipLaunchKernelGGL(reset_counter, dim3(1), dim3(64), 0, reinterpret_cast<hipStream_t>(stream), counter, ts);
    return launch_result();
}

int sos_launch_cast_state(const ProbDesc *probs_dev, const int *ids, int count, int to64, void *stream,
                          int max_len) {
    if (count <= 0) return 0;
    int gx = (max_len + 255) / 256;
    if (gx > 64) gx = 64;
    if (gx < 1) gx = 1;
    if (!launch_precheck()) return -4;
    hipLaunchKernelGGL(cast_state, dim3(gx, count), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), probs_dev,
                       ids, count, to64);
    return launch_result();
}

int sos_launch_reset_state(const ProbDesc *probs_dev, int count, int max_len, void *stream) {
    if (count <= 0) return 0;
    int gx = (max_len + 255) / 256;
    if (gx > 64) gx = 64;
    if (gx < 1) gx = 1;
    if (!launch_precheck()) return -4;
    hipLaunchKernelGGL(reset_state, dim3(gx, count), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), probs_dev,
                       count);
    return launch_result();
}

int sos_launch_warm_start(int fp64, int threads, int grid, const RunParams &rp_in, const float *pred, long long ld,
                          void *stream) {
    RunParams rp = rp_in;
    if (grid < 1) return -1;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    size_t lds = 0;
    if (!launch_precheck()) return -4;
#define SOS_WS(TT, NTT)                                                                                          \
    {                                                                                                           \
        lds_layout<TT>(rp.eig_ld, rp.lds_budget, NTT / 64, rp.lds_mat_off, rp.lds_nmax, rp.lds_nmax_g, lds,      \
                       rp.eig_wave,                                                                             \
                       rp.rows_nmax);                                                                            \
        if (lds > 64 * 1024) {                                                                                  \
            (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&warm_start_kernel<TT, NTT>),               \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                    \
            (void)hipGetLastError();                                                                            \
        }                                                                                                       \
        hipLaunchKernelGGL((warm_start_kernel<TT, NTT>), dim3(grid), dim3(NTT), lds, st, rp, pred, ld);          \
    }
    if (fp64) {
        if (threads == 256) SOS_WS(double, 256) else if (threads == 512) SOS_WS(double, 512) else if (threads == 128) SOS_WS(double, 128) else SOS_WS(double, 64)
    } else {
        if (threads == 256) SOS_WS(float, 256) else if (threads == 512) SOS_WS(float, 512) else if (threads == 128) SOS_WS(float, 128) else SOS_WS(float, 64)
    }
#undef SOS_WS
    return launch_result();
}

int sos_static_scratch(void **ptr) {
    // one lookup per device, made with that device current, kept for the process
    constexpr int kMaxDev = 64;
    static std::mutex mu;
    static void *addr[kMaxDev] = {};
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return -4;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return -4;
        }
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return 0;
}

// dynamic LDS of admm_coop: the block round's Gram tiles and rotations (the affine step keeps its
// k-vectors in global scratch)
static size_t coop_lds_bytes(int threads) {
    return gram_round_lds_bytes(threads);
}

int sos_coop_max_grid(int threads, const RunParams &rp) {
    const size_t lds = coop_lds_bytes(threads);
    if (lds > (size_t)rp.lds_budget) return 0;
    int dev = 0, coop = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const void *f = nullptr;
    switch (threads) {
        case 256: f = reinterpret_cast<const void *>(&admm_coop<256>); break;
        case 512: f = reinterpret_cast<const void *>(&admm_coop<512>); break;
        default: return 0;
    }
    if (lds > 64 * 1024) {
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipGetLastError();
    }
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, threads, lds) != hipSuccess || per < 1) {
        (void)hipGetLastError();
        return 0;
    }
    const int g = cus * per;
    return g < SOS_COOP_MAX_WG ? g : SOS_COOP_MAX_WG;
}

int sos_launch_admm_coop(int threads, int grid, const RunParams &rp_in, CoopCtl *ctl, double *scratch, void *stream) {
    RunParams rp = rp_in;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (grid < 1 || grid > SOS_COOP_MAX_WG) return -1;
    const size_t lds = coop_lds_bytes(threads);
    if (!launch_precheck()) return -4;
    hipLaunchKernelGGL(reset_coop, dim3(1), dim3(64), 0, st, ctl);
    void *args[] = {&rp, &ctl, &scratch};
    hipError_t e;
    switch (threads) {
        case 256:
            e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&admm_coop<256>), dim3(grid), dim3(256), args,
                                           (unsigned)lds, st);
            break;
        case 512:
            e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&admm_coop<512>), dim3(grid), dim3(512), args,
                                           (unsigned)lds, st);
            break;
        default: return -1;
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        snprintf(g_launch_msg, sizeof(g_launch_msg), "cooperative launch: %s", hipGetErrorString(e));
        return -4;
    }
    return 0;
}

int sos_launch_psd_factor(int threads, const RunParams &rp_in, int blk, int dual, double *evals, double *evecs,
                          void *stream) {
    RunParams rp = rp_in;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    size_t lds = 0;
    if (!launch_precheck()) return -4;
#define SOS_PF(NTT)                                                                                               \
    {                                                                                                            \
        lds_layout<double>(rp.eig_ld, rp.lds_budget, NTT / 64, rp.lds_mat_off, rp.lds_nmax, rp.lds_nmax_g, lds,   \
                           rp.eig_wave, rp.rows_nmax);                                                           \
        if (lds > 64 * 1024) {                                                                                   \
            (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&psd_factor_kernel<NTT>),                    \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                     \
            (void)hipGetLastError();                                                                             \
        }                                                                                                        \
        hipLaunchKernelGGL((psd_factor_kernel<NTT>), dim3(1), dim3(NTT), lds, st, rp, blk, dual, evals, evecs);   \
    }
    switch (threads) {
        case 64: SOS_PF(64) break;
        case 128: SOS_PF(128) break;
        case 256: SOS_PF(256) break;
        case 512: SOS_PF(512) break;
        case 1024: SOS_PF(1024) break;
        default: return -1;
    }
#undef SOS_PF
    return launch_result();
}

int sos_launch_export(int fp64, const ProbDesc *probs, int count, float *out, long long ld, int max_len, void *stream) {
    if (count <= 0) return 0;
    int gx = (max_len + 255) / 256;
    if (gx > 64) gx = 64;
    if (gx < 1) gx = 1;
    if (!launch_precheck()) return -4;
    if (fp64)
        hipLaunchKernelGGL(export_solution<double>, dim3(gx, count), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                           probs, count, out, ld);
    else
        hipLaunchKernelGGL(export_solution<float>, dim3(gx, count), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                           probs, count, out, ld);
    return launch_result();
}
