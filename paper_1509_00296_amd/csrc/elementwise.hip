// elementwise.hip -- rank-l shrink-and-reconstruct, the RPCA epilogue and elementwise helpers (Alg. 1's thresholded reconstruction and the iALM updates).
#include "device_common.h"
#include "internal.h"

#include <algorithm>

namespace frk {

// ===========================================================================
// Rank-l reconstruct / RPCA epilogue.  A workgroup owns 256 consecutive
// physical rows (coalesced) and kReconCols physical columns; each thread keeps
// its row of FR in registers and reads the column factors from LDS.
// ===========================================================================
constexpr int kReconCols = 16;
bool recon_ok(int c) { return c >= 0 && c <= 32; }

template <typename T, int MODE, int CM>
__global__ void __launch_bounds__(kThreads) k_recon(ReconArgs<T> a)
{
    __shared__ T sFC[kReconCols][CM];
    __shared__ double sred[kThreads / kWave];
    const int64_t pr = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t pc0 = (int64_t)blockIdx.y * kReconCols;
    const int c = a.c;
    for (int idx = threadIdx.x; idx < kReconCols * CM; idx += kThreads) {
        const int j = idx / CM, cc = idx % CM;
        const int64_t pc = pc0 + j;
        sFC[j][cc] = (cc < c && pc < a.cols && a.FC) ? a.FC[pc + (int64_t)cc * a.ldfc] : T(0);
    }
    T fr[CM];
#pragma unroll
    for (int cc = 0; cc < CM; ++cc) fr[cc] = (cc < c && pr < a.rows && a.FR) ? a.FR[pr + (int64_t)cc * a.ldfr] : T(0);
    __syncthreads();
    double zz = 0.0;
    if (pr < a.rows) {
        const T mu = (T)a.mu, inv_mu = (T)(1.0 / a.mu), inv_mu_next = (T)(1.0 / a.mu_next);
        const T thr = (T)(a.lam / a.mu);
        for (int j = 0; j < kReconCols; ++j) {
            const int64_t pc = pc0 + j;
            if (pc >= a.cols) break;
            T L = T(0);
            if (a.Lin) {
                L = a.Lin[pr + pc * a.ldlin];
            } else {
#pragma unroll
                for (int cc = 0; cc < CM; ++cc) L += fr[cc] * sFC[j][cc];
            }
            if (MODE == kRecon) {
                a.X[pr + pc * a.ldx] = L;
            } else {
                const T o = a.O[pr + pc * a.ldo];
                const T y = a.Y[pr + pc * a.ldy];
                const T sv = soft_shrink(o - L + y * inv_mu, thr);
                if (MODE == kEpi) {
                    const T z = o - L - sv;
                    const T yn = y + mu * z;
                    a.Ynext[pr + pc * a.ldyn] = yn;
                    a.Anext[pr + pc * a.ldan] = o - sv + yn * inv_mu_next;
                    zz += (double)z * (double)z;
                } else {
                    a.X[pr + pc * a.ldx] = L;
                    a.S[pr + pc * a.lds] = sv;
                }
            }
        }
    }
    if (MODE == kEpi) {
        zz = wave_sum(zz);
        if (threadIdx.x % kWave == 0) sred[threadIdx.x / kWave] = zz;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < kThreads / kWave; ++w) s += sred[w];
            a.zpart[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = s;
        }
    }
}

template <typename T, int MODE>
static hipError_t launch_recon_cm(const ReconArgs<T> &a, dim3 grid, hipStream_t s)
{
    if (a.c <= 8) hipLaunchKernelGGL((k_recon<T, MODE, 8>), grid, dim3(kThreads), 0, s, a);
    else if (a.c <= 16) hipLaunchKernelGGL((k_recon<T, MODE, 16>), grid, dim3(kThreads), 0, s, a);
    else hipLaunchKernelGGL((k_recon<T, MODE, 32>), grid, dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_recon(int mode, const ReconArgs<T> &a, int *nparts, hipStream_t s)
{
    if (!recon_ok(a.c)) return hipErrorInvalidValue;
    dim3 grid((unsigned)((a.rows + kThreads - 1) / kThreads), (unsigned)((a.cols + kReconCols - 1) / kReconCols));
    if (nparts) *nparts = (int)(grid.x * grid.y);
    if (mode == kRecon) return launch_recon_cm<T, kRecon>(a, grid, s);
    if (mode == kEpi) return launch_recon_cm<T, kEpi>(a, grid, s);
    return launch_recon_cm<T, kFinal>(a, grid, s);
}
template hipError_t launch_recon<double>(int, const ReconArgs<double> &, int *, hipStream_t);
template hipError_t launch_recon<float>(int, const ReconArgs<float> &, int *, hipStream_t);

// ===========================================================================
// Elementwise helpers.
// ===========================================================================
template <typename T>
__global__ void __launch_bounds__(kThreads) k_norms(int64_t m, int64_t n, const T *A, int64_t lda, double *parts)
{
    __shared__ double s1[kThreads / kWave], s2[kThreads / kWave];
    double ss = 0.0, mx = 0.0;
    const int64_t total = m * n;
    for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kThreads) {
        const int64_t i = idx % m, j = idx / m;
        const double v = (double)A[i + j * lda];
        ss += v * v;
        mx = fmax(mx, fabs(v));
    }
    ss = wave_sum(ss);
    mx = wave_max(mx);
    if (threadIdx.x % kWave == 0) {
        s1[threadIdx.x / kWave] = ss;
        s2[threadIdx.x / kWave] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < kThreads / kWave; ++w) {
            a += s1[w];
            b = fmax(b, s2[w]);
        }
        parts[2 * blockIdx.x] = a;
        parts[2 * blockIdx.x + 1] = b;
    }
}

template <typename T>
hipError_t launch_norms(int64_t m, int64_t n, const T *A, int64_t lda, double *parts, int *nparts, hipStream_t s)
{
    const int grid = 1024;
    *nparts = grid;
    hipLaunchKernelGGL((k_norms<T>), dim3(grid), dim3(kThreads), 0, s, m, n, A, lda, parts);
    return hipGetLastError();
}
template hipError_t launch_norms<double>(int64_t, int64_t, const double *, int64_t, double *, int *, hipStream_t);
template hipError_t launch_norms<float>(int64_t, int64_t, const float *, int64_t, double *, int *, hipStream_t);

template <typename T>
__global__ void __launch_bounds__(kThreads) k_rpca_init(int64_t m, int64_t n, const T *O, int64_t ldo, double invJ, double inv_mu, T *Y, int64_t ldy, T *A, int64_t lda)
{
    const int64_t total = m * n;
    for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kThreads) {
        const int64_t i = idx % m, j = idx / m;
        const T o = O[i + j * ldo];
        const T y = o * (T)invJ;
        Y[i + j * ldy] = y;
        A[i + j * lda] = o + y * (T)inv_mu;
    }
}

template <typename T>
hipError_t launch_rpca_init(int64_t m, int64_t n, const T *O, int64_t ldo, double invJ, double inv_mu, T *Y, int64_t ldy, T *A, int64_t lda, hipStream_t s)
{
    hipLaunchKernelGGL((k_rpca_init<T>), dim3(2048), dim3(kThreads), 0, s, m, n, O, ldo, invJ, inv_mu, Y, ldy, A, lda);
    return hipGetLastError();
}
template hipError_t launch_rpca_init<double>(int64_t, int64_t, const double *, int64_t, double, double, double *, int64_t, double *, int64_t, hipStream_t);
template hipError_t launch_rpca_init<float>(int64_t, int64_t, const float *, int64_t, double, double, float *, int64_t, float *, int64_t, hipStream_t);

template <typename T>
__global__ void __launch_bounds__(kThreads) k_finite(int64_t m, int64_t n, const T *A, int64_t lda, int *flag)
{
    int bad = 0;
    const int64_t total = m * n;
    for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kThreads) {
        const int64_t i = idx % m, j = idx / m;
        const double v = (double)A[i + j * lda];
        bad |= !isfinite(v);
    }
    if (__any(bad) && threadIdx.x % kWave == 0) atomicOr(flag, 1);
}

template <typename T>
hipError_t launch_finite_check(int64_t m, int64_t n, const T *A, int64_t lda, int *flag, hipStream_t s)
{
    hipLaunchKernelGGL((k_finite<T>), dim3(1024), dim3(kThreads), 0, s, m, n, A, lda, flag);
    return hipGetLastError();
}
template hipError_t launch_finite_check<double>(int64_t, int64_t, const double *, int64_t, int *, hipStream_t);
template hipError_t launch_finite_check<float>(int64_t, int64_t, const float *, int64_t, int *, hipStream_t);

// Power method on a symmetric PSD l x l matrix (global memory, one workgroup).
__global__ void __launch_bounds__(1024) k_power_eig(int l, const double *G, double *x, double *out)
{
    __shared__ double red[16];
    __shared__ double lam_sh, nrm_sh;
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    double *y = x + l;
    for (int i = tid; i < l; i += 1024) x[i] = 1.0 / sqrt((double)l) * (1.0 + 0.01 * (i % 7));
    __syncthreads();
    double lam_old = -1.0;
    for (int it = 0; it < 20000; ++it) {
        // y = G x
        for (int i = tid; i < l; i += 1024) {
            double s = 0.0;
            for (int j = 0; j < l; ++j) s += G[i + (size_t)j * l] * x[j];
            y[i] = s;
        }
        __syncthreads();
        // lambda = x^T y, ||y||
        double a = 0.0, b = 0.0;
        for (int i = tid; i < l; i += 1024) {
            a += x[i] * y[i];
            b += y[i] * y[i];
        }
        a = wave_sum(a);
        b = wave_sum(b);
        if (lane == 0) {
            red[wave] = a;
        }
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < 16; ++w) s += red[w];
            lam_sh = s;
        }
        __syncthreads();
        if (lane == 0) red[wave] = b;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < 16; ++w) s += red[w];
            nrm_sh = sqrt(s);
        }
        __syncthreads();
        const double lam = lam_sh, nrm = nrm_sh;
        if (!(nrm > 0.0)) {
            if (tid == 0) out[0] = 0.0;
            return;
        }
        for (int i = tid; i < l; i += 1024) x[i] = y[i] / nrm;
        __syncthreads();
        if (fabs(lam - lam_old) <= 1e-15 * lam && it > 3) break;
        lam_old = lam;
    }
    // final Rayleigh quotient with the normalised x
    for (int i = tid; i < l; i += 1024) {
        double s = 0.0;
        for (int j = 0; j < l; ++j) s += G[i + (size_t)j * l] * x[j];
        y[i] = s;
    }
    __syncthreads();
    double a = 0.0;
    for (int i = tid; i < l; i += 1024) a += x[i] * y[i];
    a = wave_sum(a);
    if (lane == 0) red[wave] = a;
    __syncthreads();
    if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < 16; ++w) s += red[w];
        out[0] = s;
    }
}

hipError_t launch_power_eig(int l, const double *G, double *work, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_power_eig, dim3(1), dim3(1024), 0, s, l, G, work, out);
    return hipGetLastError();
}

}  // namespace frk
