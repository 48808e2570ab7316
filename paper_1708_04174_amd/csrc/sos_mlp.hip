// Learned warm start: a small MLP (input -> H -> H -> output, GELU) in FP32, with
// hand-written forward, backward and Adam kernels.  It maps features of a parametric SOS
// family to the solver's converged (xi, y), which then seeds the ADMM iteration; the cold
// start stays the fallback.  Parameters live in one device buffer:
//   [W1 (in x H) | b1 (H) | W2 (H x H) | b2 (H) | W3 (H x out) | b3 (out)],  row-major W,
// so a layer is Z = X W + b for a row-major batch X.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/sos.h"

namespace {

constexpr int TM = 64, TN = 64, TK = 16;   // GEMM tile

// C (M x N) = op(A) (M x K) * op(B) (K x N) [+ C if accumulate]; row-major, leading dims given.
// op(A)[i][k] = TA ? A[k*lda + i] : A[i*lda + k];  op(B)[k][j] = TB ? B[j*ldb + k] : B[k*ldb + j].
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_f32(int M, int N, int K, const float *__restrict__ A, int lda,
                                                const float *__restrict__ B, int ldb, float *__restrict__ C, int ldc,
                                                int accumulate) {
    __shared__ float sA[TK][TM + 4];
    __shared__ float sB[TK][TN + 4];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i0 = blockIdx.y * TM, j0 = blockIdx.x * TN;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += TK) {
        // 64 x 16 tile of op(A) and 16 x 64 tile of op(B): 1024 values each, 4 per thread
        for (int l = threadIdx.x; l < TM * TK; l += 256) {
            int ii, kk;
            if (TA) {   // contiguous along i
                ii = l % TM;
                kk = l / TM;
            } else {    // contiguous along k
                kk = l % TK;
                ii = l / TK;
            }
            const int gi = i0 + ii, gk = k0 + kk;
            float a = 0.f;
            if (gi < M && gk < K) a = TA ? A[(long long)gk * lda + gi] : A[(long long)gi * lda + gk];
            sA[kk][ii] = a;
        }
        for (int l = threadIdx.x; l < TK * TN; l += 256) {
            int kk, jj;
            if (TB) {   // contiguous along k
                kk = l % TK;
                jj = l / TK;
            } else {    // contiguous along j
                jj = l % TN;
                kk = l / TN;
            }
            const int gk = k0 + kk, gj = j0 + jj;
            float b = 0.f;
            if (gk < K && gj < N) b = TB ? B[(long long)gj * ldb + gk] : B[(long long)gk * ldb + gj];
            sB[kk][jj] = b;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = sA[kk][ty * 4 + r];
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = sB[kk][tx * 4 + c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] += a[r] * b[c];
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int gi = i0 + ty * 4 + r, gj = j0 + tx * 4 + c;
            if (gi < M && gj < N) {
                float *p = C + (long long)gi * ldc + gj;
                *p = accumulate ? *p + acc[r][c] : acc[r][c];
            }
        }
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// Z += b (row broadcast); H = gelu(Z) if act, else H = Z
__global__ void bias_act(int M, int N, float *__restrict__ Z, const float *__restrict__ b, float *__restrict__ H,
                         int act) {
    const long long total = (long long)M * N;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
        const float z = Z[i] + b[i % N];
        Z[i] = z;
        if (H) H[i] = act ? gelu(z) : z;
    }
}

// dY = 2 (Y - T) / (M N); per-block partial sums of (Y - T)^2 into part[blockIdx.x]
__global__ void mse_grad(int M, int N, const float *__restrict__ Y, const float *__restrict__ T, float *__restrict__ dY,
                         double *__restrict__ part) {
    __shared__ double red[256];
    const long long total = (long long)M * N;
    const float sc = 2.0f / (float)total;
    double s = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
        const float d = Y[i] - T[i];
        dY[i] = sc * d;
        s += (double)d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void sum_parts(int n, const double *__restrict__ part, double *__restrict__ out, double scale) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += part[i];
        *out = s * scale;
    }
}

// dZ = dH * gelu'(Z)
__global__ void gelu_back(long long total, const float *__restrict__ Z, const float *__restrict__ dH, float *__restrict__ dZ) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x)
        dZ[i] = dH[i] * gelu_grad(Z[i]);
}

// db[j] = sum_i dZ[i][j] (one thread per column, fixed order)
__global__ void col_sum(int M, int N, const float *__restrict__ dZ, float *__restrict__ db) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    float s = 0.f;
    for (int i = 0; i < M; ++i) s += dZ[(long long)i * N + j];
    db[j] = s;
}

__global__ void adam_step(long long n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                          float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// Y = Y * scale[j] + shift[j]
// dst[r][:] = src[rows[r]][:] for r < nrows (row-major, cols columns): a mini-batch gather
__global__ void gather_rows(const float *__restrict__ src, int cols, const int *__restrict__ rows, int nrows,
                            float *__restrict__ dst) {
    const long long total = (long long)nrows * cols;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
        const long long r = i / cols, c = i - r * cols;
        dst[i] = src[(long long)rows[r] * cols + c];
    }
}

__global__ void affine_cols(int M, int N, float *__restrict__ Y, const float *__restrict__ scale,
                            const float *__restrict__ shift) {
    const long long total = (long long)M * N;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(i % N);
        Y[i] = Y[i] * scale[j] + shift[j];
    }
}

int grid_for(long long n) {
    long long g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

}   // namespace

struct sos_mlp {
    int nin = 0, nh = 0, nout = 0, cap = 0;
    long long np = 0;
    hipStream_t st = nullptr;
    float *P = nullptr, *G = nullptr, *Mm = nullptr, *Vv = nullptr;   // params, grads, Adam moments
    float *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr, *Y = nullptr;
    float *dY = nullptr, *dH = nullptr, *dZ = nullptr;
    float *oscale = nullptr, *oshift = nullptr;
    float *Xg = nullptr, *Tg = nullptr;                                 // gathered mini-batch (train_step_rows)
    double *part = nullptr, *loss = nullptr;
    long long step = 0;
    std::string err;
    float *W1() const { return P; }
    float *B1() const { return P + (long long)nin * nh; }
    float *W2() const { return B1() + nh; }
    float *B2() const { return W2() + (long long)nh * nh; }
    float *W3() const { return B2() + nh; }
    float *B3() const { return W3() + (long long)nh * nout; }
    float *gW1() const { return G; }
    float *gB1() const { return G + (long long)nin * nh; }
    float *gW2() const { return gB1() + nh; }
    float *gB2() const { return gW2() + (long long)nh * nh; }
    float *gW3() const { return gB2() + nh; }
    float *gB3() const { return gW3() + (long long)nh * nout; }
};

namespace {

bool ok(hipError_t e) { return e == hipSuccess; }

template <bool TA, bool TB>
void gemm(hipStream_t st, int M, int N, int K, const float *A, int lda, const float *B, int ldb, float *C, int ldc,
          int accumulate) {
    dim3 grid((N + TN - 1) / TN, (M + TM - 1) / TM);
    hipLaunchKernelGGL((gemm_f32<TA, TB>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, accumulate);
}

void forward(sos_mlp *m, const float *X, int Bn) {
    hipStream_t st = m->st;
    gemm<false, false>(st, Bn, m->nh, m->nin, X, m->nin, m->W1(), m->nh, m->Z1, m->nh, 0);
    hipLaunchKernelGGL(bias_act, dim3(grid_for((long long)Bn * m->nh)), dim3(256), 0, st, Bn, m->nh, m->Z1, m->B1(), m->H1, 1);
    gemm<false, false>(st, Bn, m->nh, m->nh, m->H1, m->nh, m->W2(), m->nh, m->Z2, m->nh, 0);
    hipLaunchKernelGGL(bias_act, dim3(grid_for((long long)Bn * m->nh)), dim3(256), 0, st, Bn, m->nh, m->Z2, m->B2(), m->H2, 1);
    gemm<false, false>(st, Bn, m->nout, m->nh, m->H2, m->nh, m->W3(), m->nout, m->Y, m->nout, 0);
    hipLaunchKernelGGL(bias_act, dim3(grid_for((long long)Bn * m->nout)), dim3(256), 0, st, Bn, m->nout, m->Y, m->B3(),
                       (float *)nullptr, 0);
}

// gradients of the mean squared error into G, loss into m->loss (device)
void backward(sos_mlp *m, const float *X, const float *T, int Bn) {
    hipStream_t st = m->st;
    const long long ny = (long long)Bn * m->nout, nh = (long long)Bn * m->nh;
    const int gp = 256;
    hipLaunchKernelGGL(mse_grad, dim3(gp), dim3(256), 0, st, Bn, m->nout, m->Y, T, m->dY, m->part);
    hipLaunchKernelGGL(sum_parts, dim3(1), dim3(64), 0, st, gp, m->part, m->loss, 1.0 / (double)ny);
    // layer 3
    gemm<true, false>(st, m->nh, m->nout, Bn, m->H2, m->nh, m->dY, m->nout, m->gW3(), m->nout, 0);
    hipLaunchKernelGGL(col_sum, dim3((m->nout + 255) / 256), dim3(256), 0, st, Bn, m->nout, m->dY, m->gB3());
    gemm<false, true>(st, Bn, m->nh, m->nout, m->dY, m->nout, m->W3(), m->nout, m->dH, m->nh, 0);
    hipLaunchKernelGGL(gelu_back, dim3(grid_for(nh)), dim3(256), 0, st, nh, m->Z2, m->dH, m->dZ);
    // layer 2
    gemm<true, false>(st, m->nh, m->nh, Bn, m->H1, m->nh, m->dZ, m->nh, m->gW2(), m->nh, 0);
    hipLaunchKernelGGL(col_sum, dim3((m->nh + 255) / 256), dim3(256), 0, st, Bn, m->nh, m->dZ, m->gB2());
    gemm<false, true>(st, Bn, m->nh, m->nh, m->dZ, m->nh, m->W2(), m->nh, m->dH, m->nh, 0);
    hipLaunchKernelGGL(gelu_back, dim3(grid_for(nh)), dim3(256), 0, st, nh, m->Z1, m->dH, m->dZ);
    // layer 1
    gemm<true, false>(st, m->nin, m->nh, Bn, X, m->nin, m->dZ, m->nh, m->gW1(), m->nh, 0);
    hipLaunchKernelGGL(col_sum, dim3((m->nh + 255) / 256), dim3(256), 0, st, Bn, m->nh, m->dZ, m->gB1());
}

template <typename F>
int guard(sos_mlp *m, F &&f) {
    (void)hipGetLastError();
    const int rc = f();
    if (rc != SOS_OK) return rc;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        if (m) m->err = hipGetErrorString(e);
        return SOS_E_HIP;
    }
    return SOS_OK;
}

}   // namespace

extern "C" {

int sos_mlp_create(int32_t n_in, int32_t n_hidden, int32_t n_out, int32_t max_batch, void *hip_stream, sos_mlp **out) {
    if (!out || n_in < 1 || n_hidden < 1 || n_out < 1 || max_batch < 1) return SOS_E_INVAL;
    *out = nullptr;
    sos_mlp *m = new (std::nothrow) sos_mlp();
    if (!m) return SOS_E_NOMEM;
    m->nin = n_in;
    m->nh = n_hidden;
    m->nout = n_out;
    m->cap = max_batch;
    m->st = reinterpret_cast<hipStream_t>(hip_stream);
    m->np = (long long)n_in * n_hidden + n_hidden + (long long)n_hidden * n_hidden + n_hidden +
            (long long)n_hidden * n_out + n_out;
    const long long bh = (long long)max_batch * n_hidden, bo = (long long)max_batch * n_out;
    bool good = ok(hipMalloc(&m->P, m->np * 4)) && ok(hipMalloc(&m->G, m->np * 4)) &&
                ok(hipMalloc(&m->Mm, m->np * 4)) && ok(hipMalloc(&m->Vv, m->np * 4)) &&
                ok(hipMalloc(&m->Z1, bh * 4)) && ok(hipMalloc(&m->H1, bh * 4)) && ok(hipMalloc(&m->Z2, bh * 4)) &&
                ok(hipMalloc(&m->H2, bh * 4)) && ok(hipMalloc(&m->Y, bo * 4)) && ok(hipMalloc(&m->dY, bo * 4)) &&
                ok(hipMalloc(&m->dH, bh * 4)) && ok(hipMalloc(&m->dZ, bh * 4)) &&
                ok(hipMalloc(&m->oscale, (long long)n_out * 4)) && ok(hipMalloc(&m->oshift, (long long)n_out * 4)) &&
                ok(hipMalloc(&m->part, 256 * 8)) && ok(hipMalloc(&m->loss, 8)) &&
                ok(hipMalloc(&m->Xg, (long long)max_batch * n_in * 4)) && ok(hipMalloc(&m->Tg, bo * 4));
    if (!good) {
        sos_mlp_free(m);
        return SOS_E_NOMEM;
    }
    std::vector<float> ones(n_out, 1.f), zeros(n_out, 0.f);
    good = ok(hipMemset(m->P, 0, m->np * 4)) && ok(hipMemset(m->Mm, 0, m->np * 4)) && ok(hipMemset(m->Vv, 0, m->np * 4)) &&
           ok(hipMemcpy(m->oscale, ones.data(), n_out * 4, hipMemcpyHostToDevice)) &&
           ok(hipMemcpy(m->oshift, zeros.data(), n_out * 4, hipMemcpyHostToDevice));
    if (!good) {
        sos_mlp_free(m);
        return SOS_E_HIP;
    }
    *out = m;
    return SOS_OK;
}

int64_t sos_mlp_num_params(const sos_mlp *m) { return m ? m->np : 0; }

int sos_mlp_set_params(sos_mlp *m, const float *host_params) {
    if (!m || !host_params) return SOS_E_INVAL;
    if (!ok(hipMemcpy(m->P, host_params, m->np * 4, hipMemcpyHostToDevice))) return SOS_E_HIP;
    if (!ok(hipMemset(m->Mm, 0, m->np * 4)) || !ok(hipMemset(m->Vv, 0, m->np * 4))) return SOS_E_HIP;
    m->step = 0;
    return SOS_OK;
}

int sos_mlp_get_params(const sos_mlp *m, float *host_params) {
    if (!m || !host_params) return SOS_E_INVAL;
    return ok(hipMemcpy(host_params, m->P, m->np * 4, hipMemcpyDeviceToHost)) ? SOS_OK : SOS_E_HIP;
}

int sos_mlp_set_output_affine(sos_mlp *m, const float *host_scale, const float *host_shift) {
    if (!m || !host_scale || !host_shift) return SOS_E_INVAL;
    return ok(hipMemcpy(m->oscale, host_scale, m->nout * 4, hipMemcpyHostToDevice)) &&
                   ok(hipMemcpy(m->oshift, host_shift, m->nout * 4, hipMemcpyHostToDevice))
               ? SOS_OK
               : SOS_E_HIP;
}

int sos_mlp_forward(sos_mlp *m, const float *X_dev, int32_t batch, float *Y_dev, int32_t apply_output_affine) {
    if (!m || !X_dev || !Y_dev || batch < 1 || batch > m->cap) return SOS_E_INVAL;
    return guard(m, [&] {
        forward(m, X_dev, batch);
        if (apply_output_affine)
            hipLaunchKernelGGL(affine_cols, dim3(grid_for((long long)batch * m->nout)), dim3(256), 0, m->st, batch,
                               m->nout, m->Y, m->oscale, m->oshift);
        if (!ok(hipMemcpyAsync(Y_dev, m->Y, (long long)batch * m->nout * 4, hipMemcpyDeviceToDevice, m->st)))
            return SOS_E_HIP;
        return SOS_OK;
    });
}

int sos_mlp_gradient(sos_mlp *m, const float *X_dev, const float *T_dev, int32_t batch, float *grad_host,
                     double *loss_host) {
    if (!m || !X_dev || !T_dev || batch < 1 || batch > m->cap) return SOS_E_INVAL;
    return guard(m, [&] {
        forward(m, X_dev, batch);
        backward(m, X_dev, T_dev, batch);
        if (grad_host && !ok(hipMemcpyAsync(grad_host, m->G, m->np * 4, hipMemcpyDeviceToHost, m->st))) return SOS_E_HIP;
        if (loss_host && !ok(hipMemcpyAsync(loss_host, m->loss, 8, hipMemcpyDeviceToHost, m->st))) return SOS_E_HIP;
        return ok(hipStreamSynchronize(m->st)) ? SOS_OK : SOS_E_HIP;
    });
}

int sos_mlp_train_step_rows(sos_mlp *m, const float *X_dev, const float *T_dev, const int32_t *rows_dev, int32_t batch,
                            float lr, double *loss_host) {
    if (!m || !X_dev || !T_dev || !rows_dev || batch < 1 || batch > m->cap || !(lr > 0.f)) return SOS_E_INVAL;
    const int rc = guard(m, [&] {
        hipLaunchKernelGGL(gather_rows, dim3(grid_for((long long)batch * m->nin)), dim3(256), 0, m->st, X_dev, m->nin,
                           rows_dev, batch, m->Xg);
        hipLaunchKernelGGL(gather_rows, dim3(grid_for((long long)batch * m->nout)), dim3(256), 0, m->st, T_dev, m->nout,
                           rows_dev, batch, m->Tg);
        return SOS_OK;
    });
    if (rc != SOS_OK) return rc;
    return sos_mlp_train_step(m, m->Xg, m->Tg, batch, lr, loss_host);
}

int sos_mlp_train_step(sos_mlp *m, const float *X_dev, const float *T_dev, int32_t batch, float lr, double *loss_host) {
    if (!m || !X_dev || !T_dev || batch < 1 || batch > m->cap || !(lr > 0.f)) return SOS_E_INVAL;
    return guard(m, [&] {
        forward(m, X_dev, batch);
        backward(m, X_dev, T_dev, batch);
        m->step += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.f - powf(b1, (float)m->step), c2 = 1.f - powf(b2, (float)m->step);
        hipLaunchKernelGGL(adam_step, dim3(grid_for(m->np)), dim3(256), 0, m->st, m->np, m->P, m->G, m->Mm, m->Vv, lr,
                           b1, b2, 1e-8f, c1, c2);
        if (loss_host) {
            if (!ok(hipMemcpyAsync(loss_host, m->loss, 8, hipMemcpyDeviceToHost, m->st))) return SOS_E_HIP;
            if (!ok(hipStreamSynchronize(m->st))) return SOS_E_HIP;
        }
        return SOS_OK;
    });
}

void sos_mlp_free(sos_mlp *m) {
    if (!m) return;
    if (m->st) (void)hipStreamSynchronize(m->st);
    for (void *p : {(void *)m->P, (void *)m->G, (void *)m->Mm, (void *)m->Vv, (void *)m->Z1, (void *)m->H1,
                    (void *)m->Z2, (void *)m->H2, (void *)m->Y, (void *)m->dY, (void *)m->dH, (void *)m->dZ,
                    (void *)m->oscale, (void *)m->oshift, (void *)m->part, (void *)m->loss, (void *)m->Xg,
                    (void *)m->Tg})
        if (p) (void)hipFree(p);
    delete m;
}

}   // extern "C"
