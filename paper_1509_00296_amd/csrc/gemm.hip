// gemm.hip -- generic tiled GEMM, materialised Gaussian matrix and the large-path CholeskyQR pieces.
#include "device_common.h"
#include "internal.h"
#include "block_dense.h"

#include <algorithm>

namespace frk {

// ===========================================================================
// Generic tiled GEMM with arbitrary strides: 64 x 64 output tile, k-step 16,
// 256 threads, 4 x 4 outputs per thread (rows tm + 16 i, columns tn + 16 j so
// that neighbouring lanes read neighbouring LDS words).
// ===========================================================================
constexpr int GB = 64, GK = 16;

template <typename TI, typename TA, typename TO, bool DIRECT>
__global__ void __launch_bounds__(kThreads) k_gemm(int64_t M, int64_t N, int64_t K, const TI *A, int64_t sam, int64_t sak, const TI *B, int64_t sbk, int64_t sbn, TO *C, int64_t scm, int64_t scn, int64_t kchunk, TA *part)
{
    __shared__ TA sA[GK][GB + 1];
    __shared__ TA sB[GK][GB + 1];
    const int tid = threadIdx.x;
    const int tm = tid % 16, tn = tid / 16;
    const int64_t m0 = (int64_t)blockIdx.x * GB, n0 = (int64_t)blockIdx.y * GB;
    const int64_t kb = (int64_t)blockIdx.z * kchunk;
    const int64_t ke = min(K, kb + kchunk);
    TA acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = TA(0);
    const bool a_m_contig = (sam == 1);
    const bool b_n_contig = (sbn == 1);
    for (int64_t k0 = kb; k0 < ke; k0 += GK) {
        for (int idx = tid; idx < GB * GK; idx += kThreads) {
            int mm, kk;
            if (a_m_contig) { mm = idx % GB; kk = idx / GB; }
            else { kk = idx % GK; mm = idx / GK; }
            const int64_t gm = m0 + mm, gk = k0 + kk;
            sA[kk][mm] = (gm < M && gk < ke) ? (TA)A[gm * sam + gk * sak] : TA(0);
        }
        for (int idx = tid; idx < GB * GK; idx += kThreads) {
            int nn, kk;
            if (b_n_contig) { nn = idx % GB; kk = idx / GB; }
            else { kk = idx % GK; nn = idx / GK; }
            const int64_t gn = n0 + nn, gk = k0 + kk;
            sB[kk][nn] = (gn < N && gk < ke) ? (TA)B[gk * sbk + gn * sbn] : TA(0);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK; ++kk) {
            TA av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = sA[kk][tm + 16 * i];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = sB[kk][tn + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] += av[i] * bv[j];
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t gm = m0 + tm + 16 * i, gn = n0 + tn + 16 * j;
            if (gm < M && gn < N) {
                if (DIRECT) C[gm * scm + gn * scn] = (TO)acc[i][j];
                else part[(int64_t)blockIdx.z * M * N + gm + gn * M] = acc[i][j];
            }
        }
}

template <typename TA, typename TO>
__global__ void __launch_bounds__(kThreads) k_gemm_store(int64_t M, int64_t N, int splitk, const TA *part, TO *C, int64_t scm, int64_t scn)
{
    const int64_t total = M * N;
    for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kThreads) {
        TA s = TA(0);
        for (int z = 0; z < splitk; ++z) s += part[(int64_t)z * total + idx];
        const int64_t gm = idx % M, gn = idx / M;
        C[gm * scm + gn * scn] = (TO)s;
    }
}

template <typename TI, typename TA, typename TO>
hipError_t launch_gemm(int64_t M, int64_t N, int64_t K, const TI *A, int64_t sam, int64_t sak, const TI *B, int64_t sbk, int64_t sbn, TO *C, int64_t scm, int64_t scn, int splitk, TA *part, hipStream_t s)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    if (splitk < 1) splitk = 1;
    int64_t kchunk = (K + splitk - 1) / splitk;
    kchunk = ((kchunk + GK - 1) / GK) * GK;
    if (kchunk < GK) kchunk = GK;
    const int sk = (int)std::max<int64_t>(1, (K + kchunk - 1) / kchunk);
    dim3 grid((unsigned)((M + GB - 1) / GB), (unsigned)((N + GB - 1) / GB), (unsigned)sk);
    if (sk == 1) {
        hipLaunchKernelGGL((k_gemm<TI, TA, TO, true>), grid, dim3(kThreads), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, C, scm, scn, kchunk, part);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_gemm<TI, TA, TO, false>), grid, dim3(kThreads), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, C, scm, scn, kchunk, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t total = M * N;
    const int g2 = (int)std::min<int64_t>(4096, (total + kThreads - 1) / kThreads);
    hipLaunchKernelGGL((k_gemm_store<TA, TO>), dim3(g2), dim3(kThreads), 0, s, M, N, sk, part, C, scm, scn);
    return hipGetLastError();
}
template hipError_t launch_gemm<double, double, double>(int64_t, int64_t, int64_t, const double *, int64_t, int64_t, const double *, int64_t, int64_t, double *, int64_t, int64_t, int, double *, hipStream_t);
template hipError_t launch_gemm<float, float, float>(int64_t, int64_t, int64_t, const float *, int64_t, int64_t, const float *, int64_t, int64_t, float *, int64_t, int64_t, int, float *, hipStream_t);
template hipError_t launch_gemm<float, double, double>(int64_t, int64_t, int64_t, const float *, int64_t, int64_t, const float *, int64_t, int64_t, double *, int64_t, int64_t, int, double *, hipStream_t);

// Omega materialised (large path).
template <typename T>
__global__ void __launch_bounds__(kThreads) k_omega(int64_t rows, int cols, uint64_t seed, uint64_t counter, T *Om, int64_t ld)
{
    const int npair = (cols + 1) / 2;
    const int64_t total = rows * npair;
    for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kThreads) {
        const int64_t k = idx % rows;
        const int j = (int)(idx / rows);
        double z0, z1;
        gaussian_pair(seed, counter, (uint32_t)k, (uint32_t)j, z0, z1);
        Om[k + (int64_t)(2 * j) * ld] = (T)z0;
        if (2 * j + 1 < cols) Om[k + (int64_t)(2 * j + 1) * ld] = (T)z1;
    }
}

template <typename T>
hipError_t launch_omega(int64_t rows, int cols, uint64_t seed, uint64_t counter, T *Om, int64_t ld, hipStream_t s)
{
    hipLaunchKernelGGL((k_omega<T>), dim3(2048), dim3(kThreads), 0, s, rows, cols, seed, counter, Om, ld);
    return hipGetLastError();
}
template hipError_t launch_omega<double>(int64_t, int, uint64_t, uint64_t, double *, int64_t, hipStream_t);
template hipError_t launch_omega<float>(int64_t, int, uint64_t, uint64_t, float *, int64_t, hipStream_t);

// ===========================================================================
// Large-path CholeskyQR pieces.
// ===========================================================================
__global__ void __launch_bounds__(kThreads) k_chol(int l, const double *G, double shift_factor, double null_tol, double *R, int *null_cols, int *flags)
{
    // G staged in LDS; the factor is formed directly in the output R
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *sG = reinterpret_cast<double *>(smem_raw);
    double *sR = R;
    __shared__ double shift, tolabs;
    for (int idx = threadIdx.x; idx < l * l; idx += kThreads) sG[idx] = G[idx];
    __syncthreads();
    if (threadIdx.x == 0) {
        double tr = 0.0, mx = 0.0;
        for (int j = 0; j < l; ++j) {
            tr += sG[j * l + j];
            mx = fmax(mx, sG[j * l + j]);
        }
        shift = shift_factor * tr;
        tolabs = null_tol > 0.0 ? null_tol * fmax(mx, 1e-300) : 0.0;
    }
    __syncthreads();
    const CholInfo ci = block_chol(sG, l, shift, tolabs, sR, null_cols);
    if (threadIdx.x == 0 && flags) {
        flags[1] = ci.nnull;
        if (null_tol <= 0.0 && ci.nnull > 0) flags[2] |= 1;
    }
}

hipError_t launch_chol(int l, const double *G, double shift_factor, double null_tol, double *R, int *null_cols, int *flags, hipStream_t s)
{
    const size_t lds = (size_t)l * l * sizeof(double);
    if (l > 128) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_chol, dim3(1), dim3(kThreads), lds, s, l, G, shift_factor, null_tol, R, null_cols, flags);
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_trsm(int64_t rows, int l, T *Y, int64_t ldy, const double *R)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const double *sR = R;
    if (l <= 90) {
        double *t = reinterpret_cast<double *>(smem_raw);
        for (int idx = threadIdx.x; idx < l * l; idx += kThreads) t[idx] = R[idx];
        sR = t;
        __syncthreads();
    }
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= rows) return;
    double y[128];
    for (int j = 0; j < l; ++j) {
        double v = (double)Y[i + (int64_t)j * ldy];
        for (int t = 0; t < j; ++t) v -= y[t] * sR[t * l + j];
        y[j] = v / sR[j * l + j];
    }
    for (int j = 0; j < l; ++j) Y[i + (int64_t)j * ldy] = (T)y[j];
}

template <typename T>
hipError_t launch_trsm(int64_t rows, int l, T *Y, int64_t ldy, const double *R, hipStream_t s)
{
    if (l > 128) return hipErrorInvalidValue;
    const size_t lds = l <= 90 ? (size_t)l * l * sizeof(double) : 0;
    hipLaunchKernelGGL((k_trsm<T>), dim3((unsigned)((rows + kThreads - 1) / kThreads)), dim3(kThreads), lds, s, rows, l, Y, ldy, R);
    return hipGetLastError();
}
template hipError_t launch_trsm<double>(int64_t, int, double *, int64_t, const double *, hipStream_t);
template hipError_t launch_trsm<float>(int64_t, int, float *, int64_t, const double *, hipStream_t);

template <typename T>
__global__ void __launch_bounds__(kThreads) k_refill(int64_t rows, int l, T *Y, int64_t ldy, const int *null_cols, uint64_t seed, uint64_t counter, int attempt)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= rows) return;
    for (int j = 0; j < l; ++j) {
        if (!null_cols[j]) continue;
        double z0, z1;
        gaussian_pair(seed, counter, (uint32_t)i, kRefillTag | (uint32_t)(attempt * 1024 + j), z0, z1);
        Y[i + (int64_t)j * ldy] = (T)z0;
    }
}

template <typename T>
hipError_t launch_refill(int64_t rows, int l, T *Y, int64_t ldy, const int *null_cols, uint64_t seed, uint64_t counter, int attempt, hipStream_t s)
{
    hipLaunchKernelGGL((k_refill<T>), dim3((unsigned)((rows + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, rows, l, Y, ldy, null_cols, seed, counter, attempt);
    return hipGetLastError();
}
template hipError_t launch_refill<double>(int64_t, int, double *, int64_t, const int *, uint64_t, uint64_t, int, hipStream_t);
template hipError_t launch_refill<float>(int64_t, int, float *, int64_t, const int *, uint64_t, uint64_t, int, hipStream_t);

template <typename T>
__global__ void __launch_bounds__(kThreads) k_col_scale(int64_t rows, int l, T *Y, int64_t ldy, const double *G)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= rows) return;
    for (int j = 0; j < l; ++j) {
        const double g = G[j * l + j];
        const double sc = g > 0.0 ? 1.0 / sqrt(g) : 0.0;
        Y[i + (int64_t)j * ldy] = (T)((double)Y[i + (int64_t)j * ldy] * sc);
    }
}

template <typename T>
hipError_t launch_col_scale(int64_t rows, int l, T *Y, int64_t ldy, const double *G, hipStream_t s)
{
    hipLaunchKernelGGL((k_col_scale<T>), dim3((unsigned)((rows + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, rows, l, Y, ldy, G);
    return hipGetLastError();
}
template hipError_t launch_col_scale<double>(int64_t, int, double *, int64_t, const double *, hipStream_t);
template hipError_t launch_col_scale<float>(int64_t, int, float *, int64_t, const double *, hipStream_t);

template <typename T>
__global__ void __launch_bounds__(kThreads) k_cast(int64_t m, int64_t n, const void *src, int src_is_double, int64_t lds, T *dst, int64_t ldd)
{
    const int64_t total = m * n;
    for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kThreads) {
        const int64_t i = idx % m, j = idx / m;
        const double v = src_is_double ? ((const double *)src)[i + j * lds] : (double)((const float *)src)[i + j * lds];
        dst[i + j * ldd] = (T)v;
    }
}

template <typename T>
hipError_t launch_cast(int64_t m, int64_t n, const void *src, int src_is_double, int64_t lds, T *dst, int64_t ldd, hipStream_t s)
{
    hipLaunchKernelGGL((k_cast<T>), dim3(2048), dim3(kThreads), 0, s, m, n, src, src_is_double, lds, dst, ldd);
    return hipGetLastError();
}
template hipError_t launch_cast<double>(int64_t, int64_t, const void *, int, int64_t, double *, int64_t, hipStream_t);
template hipError_t launch_cast<float>(int64_t, int64_t, const void *, int, int64_t, float *, int64_t, hipStream_t);

}  // namespace frk
