// lrr.hip -- the elementwise and reduction steps of the low-rank
// representation host (Type A of Table 6, its inexact ALM): linear
// combinations of matrices, the column-wise l2,1 shrinkage, the multiplier
// updates with their max-norm residuals, and the infinity norm that starts
// the Newton-Schulz inverse of I + X^T X.  The products run on the matrix
// cores (launch_gemm_f64_mfma) and the J step through the FRSVT path.
#include "device_common.h"
#include "internal.h"

namespace frk {

constexpr int kLrrThreads = 256;

// out = a A + b B + c C + g I (m x n; a null operand contributes nothing;
// out may alias A).
__global__ void __launch_bounds__(kLrrThreads) k_lrr_comb(int64_t m, int64_t n, double a, const double *A,
                                                          int64_t lda, double b, const double *B, int64_t ldb,
                                                          double c, const double *C, int64_t ldc, double g,
                                                          double *out, int64_t ldo)
{
    const int64_t total = m * n;
    for (int64_t t = (int64_t)blockIdx.x * kLrrThreads + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * kLrrThreads) {
        const int64_t i = t % m, j = t / m;
        double v = (i == j) ? g : 0.0;
        if (A) v += a * A[i + j * lda];
        if (B) v += b * B[i + j * ldb];
        if (C) v += c * C[i + j * ldc];
        out[i + j * ldo] = v;
    }
}

hipError_t launch_lrr_comb(int64_t m, int64_t n, double a, const double *A, int64_t lda, double b,
                           const double *B, int64_t ldb, double c, const double *C, int64_t ldc, double g,
                           double *out, int64_t ldo, hipStream_t s)
{
    if (m < 1 || n < 1) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((m * n + kLrrThreads - 1) / kLrrThreads, 4096);
    hipLaunchKernelGGL(k_lrr_comb, dim3((unsigned)blocks), dim3(kLrrThreads), 0, s, m, n, a, A, lda, b, B, ldb,
                       c, C, ldc, g, out, ldo);
    return hipGetLastError();
}

// out[0] = max_i sum_j |A(i, j)| (one workgroup, rows over threads).
__global__ void __launch_bounds__(kLrrThreads) k_lrr_norm_inf(int64_t n, const double *A, int64_t lda, double *out)
{
    __shared__ double red[kLrrThreads / kWave];
    double mx = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kLrrThreads) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j) s += fabs(A[i + j * lda]);
        mx = fmax(mx, s);
    }
    mx = wave_max(mx);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kLrrThreads / kWave; ++w) t = fmax(t, red[w]);
        out[0] = t;
    }
}

hipError_t launch_lrr_norm_inf(int64_t n, const double *A, int64_t lda, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_lrr_norm_inf, dim3(1), dim3(kLrrThreads), 0, s, n, A, lda, out);
    return hipGetLastError();
}

// E(:, j) = max(0, 1 - thr / ||v||) v with v = X(:, j) - XZ(:, j) + Y1(:, j) / mu
// (one workgroup per column; the norm added in a fixed order).
__global__ void __launch_bounds__(kLrrThreads) k_lrr_colshrink(int64_t d, const double *X, int64_t ldx,
                                                               const double *XZ, const double *Y1, double inv_mu,
                                                               double thr, double *E, int64_t lde)
{
    __shared__ double red[kLrrThreads / kWave];
    __shared__ double scale;
    const int64_t j = blockIdx.x;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < d; i += kLrrThreads) {
        const double v = X[i + j * ldx] - XZ[i + j * d] + Y1[i + j * d] * inv_mu;
        s += v * v;
    }
    s = wave_sum(s);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kLrrThreads / kWave; ++w) t += red[w];
        const double nrm = sqrt(t);
        scale = nrm > thr ? (nrm - thr) / nrm : 0.0;
    }
    __syncthreads();
    const double f = scale;
    for (int64_t i = threadIdx.x; i < d; i += kLrrThreads)
        E[i + j * lde] = f * (X[i + j * ldx] - XZ[i + j * d] + Y1[i + j * d] * inv_mu);
}

hipError_t launch_lrr_colshrink(int64_t d, int64_t n, const double *X, int64_t ldx, const double *XZ,
                                const double *Y1, double inv_mu, double thr, double *E, int64_t lde, hipStream_t s)
{
    hipLaunchKernelGGL(k_lrr_colshrink, dim3((unsigned)n), dim3(kLrrThreads), 0, s, d, X, ldx, XZ, Y1, inv_mu, thr,
                       E, lde);
    return hipGetLastError();
}

// Y += mu (P - Q - R) (R optional), part[block] = max |P - Q - R| over the
// block's elements.
__global__ void __launch_bounds__(kLrrThreads) k_lrr_dual(int64_t m, int64_t n, double mu, const double *P,
                                                          int64_t ldp, const double *Q, int64_t ldq,
                                                          const double *R, int64_t ldr, double *Y, double *part)
{
    __shared__ double red[kLrrThreads / kWave];
    const int64_t total = m * n;
    double mx = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * kLrrThreads + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * kLrrThreads) {
        const int64_t i = t % m, j = t / m;
        double z = P[i + j * ldp] - Q[i + j * ldq];
        if (R) z -= R[i + j * ldr];
        Y[i + j * m] += mu * z;
        mx = fmax(mx, fabs(z));
    }
    mx = wave_max(mx);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kLrrThreads / kWave; ++w) t = fmax(t, red[w]);
        part[blockIdx.x] = t;
    }
}

// out[k] = max over parts of block k's slice (one workgroup per k)
__global__ void __launch_bounds__(kLrrThreads) k_lrr_max_parts(const double *part, int nparts, double *out)
{
    __shared__ double red[kLrrThreads / kWave];
    double mx = 0.0;
    for (int g = threadIdx.x; g < nparts; g += kLrrThreads) mx = fmax(mx, part[(int64_t)blockIdx.x * nparts + g]);
    mx = wave_max(mx);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kLrrThreads / kWave; ++w) t = fmax(t, red[w]);
        out[blockIdx.x] = t;
    }
}

int lrr_dual_parts() { return 512; }

hipError_t launch_lrr_dual(int64_t m, int64_t n, double mu, const double *P, int64_t ldp, const double *Q,
                           int64_t ldq, const double *R, int64_t ldr, double *Y, double *part, hipStream_t s)
{
    hipLaunchKernelGGL(k_lrr_dual, dim3((unsigned)lrr_dual_parts()), dim3(kLrrThreads), 0, s, m, n, mu, P, ldp, Q,
                       ldq, R, ldr, Y, part);
    return hipGetLastError();
}

hipError_t launch_lrr_max_parts(const double *part, int nparts, int count, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_lrr_max_parts, dim3((unsigned)count), dim3(kLrrThreads), 0, s, part, nparts, out);
    return hipGetLastError();
}

}  // namespace frk
