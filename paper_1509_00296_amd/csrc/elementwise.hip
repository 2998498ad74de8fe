// elementwise.hip -- rank-l shrink-and-reconstruct, the RPCA epilogue and elementwise helpers (Alg. 1's thresholded reconstruction and the iALM updates).
#include "device_common.h"
#include "internal.h"

#include <algorithm>
#include <type_traits>

namespace frk {

// ===========================================================================
// Rank-l reconstruct / RPCA epilogue.  A workgroup owns 256 consecutive
// physical rows (coalesced) and kReconCols physical columns; each thread keeps
// its row of FR in registers and reads the column factors from LDS.
// ===========================================================================
constexpr int kReconCols = 16;
bool recon_ok(int c) { return c >= 0 && c <= 32; }
int64_t recon_row_blocks(int64_t rows) { return (rows + kThreads - 1) / kThreads; }

// With SK (kEpi, double), the workgroup also forms its part of the next
// iteration's sketch Y = Ahat Omega (Ahat = A^T, so a row of A is a long
// index k): for its 16 columns i and j < csk, the sum over its rows k of
// Anext(k, i) Omega(k, j).  Per wavefront that is Omega^T (16 x 64, rows of
// Omega past csk zero) times Anext (64 x 16) on the matrix cores, both
// operands moved through LDS from the lane-per-row layout of the epilogue to
// the 16-lanes-per-row operand layout; the four wavefronts' products are
// added in a fixed order.
__device__ __forceinline__ void sketch_rows(const ReconArgs<double> &a, int64_t pr, double (&an)[16], double *sW)
{
    const int lane = threadIdx.x % kWave;
    // Omega row pr, columns j < csk (the sketch pass's draw: pair p of row k
    // gives columns 2p and 2p + 1)
    double om[8];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        double z0 = 0.0, z1 = 0.0;
        if (2 * p < a.csk && pr < a.rows) gaussian_pair(a.seed, a.counter, (uint32_t)pr, (uint32_t)p, z0, z1);
        om[2 * p] = z0;
        om[2 * p + 1] = (2 * p + 1 < a.csk) ? z1 : 0.0;
    }
    constexpr int LDW = 17;
#pragma unroll
    for (int j = 0; j < 8; ++j) sW[lane * LDW + j] = om[j];
    __syncthreads();
    const int ro = lane >> 4, co = lane & 15;
    double aop[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) aop[s] = co < 8 ? sW[(4 * s + ro) * LDW + co] : 0.0;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) sW[lane * LDW + j] = an[j];
    __syncthreads();
    typedef __attribute__((__vector_size__(4 * sizeof(double)))) double d4;
    d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 16; ++s)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(aop[s], sW[(4 * s + ro) * LDW + co], acc, 0, 0, 0);
    __syncthreads();
    // D(j, i): lane holds j = ro + 4 r, i = co; rows j < 8 kept
    double *sC = sW - (threadIdx.x / kWave) * 64 * LDW;   // start of the workgroup's area
    const int w = threadIdx.x / kWave;
    sC[(w * 8 + ro) * 16 + co] = acc[0];
    sC[(w * 8 + ro + 4) * 16 + co] = acc[1];
    __syncthreads();
    if (threadIdx.x < 128) {
        const int j = threadIdx.x >> 4, i = threadIdx.x & 15;
        const int64_t pc = (int64_t)blockIdx.y * kReconCols + i;
        const double t = ((sC[(0 * 8 + j) * 16 + i] + sC[(1 * 8 + j) * 16 + i]) + sC[(2 * 8 + j) * 16 + i]) +
                         sC[(3 * 8 + j) * 16 + i];
        if (j < a.csk && pc < a.cols) a.ysk[(int64_t)blockIdx.x * a.cols * a.csk + pc + (int64_t)j * a.cols] = t;
    }
}

template <typename T, int MODE, int CM, bool SK = false>
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
    T anv[SK ? kReconCols : 1];
#pragma unroll
    for (int j = 0; j < (SK ? kReconCols : 1); ++j) anv[j] = T(0);
    if (pr < a.rows) {
        const T mu = (T)a.mu, inv_mu = (T)(1.0 / a.mu), inv_mu_next = (T)(1.0 / a.mu_next);
        const T thr = (T)(a.lam / a.mu);
        const int ncol = (int)min((int64_t)kReconCols, a.cols - pc0);
        // the loads of all the columns are issued first, so that their
        // latencies overlap; then the arithmetic and the stores.  O, Y and
        // the next multiplier are streamed (non-temporal: they are not read
        // again before the next epilogue), so that the caches keep the next
        // A for the passes that read it
        // (columns past the end load the last column again: unconditional
        // loads, nothing stored for them)
        T lv[kReconCols], ov[kReconCols], yv[kReconCols];
        if (MODE != kRecon) {
#pragma unroll
            for (int j = 0; j < kReconCols; ++j) {
                const int64_t pc = pc0 + min(j, ncol - 1);
                ov[j] = __builtin_nontemporal_load(&a.O[pr + pc * a.ldo]);
                yv[j] = __builtin_nontemporal_load(&a.Y[pr + pc * a.ldy]);
            }
        }
        if (a.Lin) {
#pragma unroll
            for (int j = 0; j < kReconCols; ++j) lv[j] = a.Lin[pr + (pc0 + min(j, ncol - 1)) * a.ldlin];
        } else {
#pragma unroll
            for (int j = 0; j < kReconCols; ++j) {
                T L = T(0);
#pragma unroll
                for (int cc = 0; cc < CM; ++cc) L += fr[cc] * sFC[j][cc];
                lv[j] = L;
            }
        }
#pragma unroll
        for (int j = 0; j < kReconCols; ++j) {
            if (j >= ncol) break;
            const int64_t pc = pc0 + j;
            const T L = lv[j];
            if (MODE == kRecon) {
                a.X[pr + pc * a.ldx] = L;
            } else {
                const T o = ov[j];
                const T y = yv[j];
                const T sv = soft_shrink(o - L + y * inv_mu, thr);
                if (MODE == kEpi) {
                    const T z = o - L - sv;
                    const T yn = y + mu * z;
                    __builtin_nontemporal_store(yn, &a.Ynext[pr + pc * a.ldyn]);
                    const T an = o - sv + yn * inv_mu_next;
                    a.Anext[pr + pc * a.ldan] = an;
                    if constexpr (SK) anv[j] = an;
                    zz += (double)z * (double)z;
                } else {
                    a.X[pr + pc * a.ldx] = L;
                    a.S[pr + pc * a.lds] = sv;
                }
            }
        }
    }
    if constexpr (SK) {
        __shared__ double sW[kThreads / kWave][64 * 17];
        sketch_rows(a, pr, anv, sW[threadIdx.x / kWave]);
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
    if constexpr (MODE == kEpi && std::is_same<T, double>::value) {
        if (a.ysk) {
            if (a.c <= 8) hipLaunchKernelGGL((k_recon<T, MODE, 8, true>), grid, dim3(kThreads), 0, s, a);
            else if (a.c <= 16) hipLaunchKernelGGL((k_recon<T, MODE, 16, true>), grid, dim3(kThreads), 0, s, a);
            else hipLaunchKernelGGL((k_recon<T, MODE, 32, true>), grid, dim3(kThreads), 0, s, a);
            return hipGetLastError();
        }
    } else {
        if (a.ysk) return hipErrorInvalidValue;
    }
    if (a.c <= 8) hipLaunchKernelGGL((k_recon<T, MODE, 8>), grid, dim3(kThreads), 0, s, a);
    else if (a.c <= 16) hipLaunchKernelGGL((k_recon<T, MODE, 16>), grid, dim3(kThreads), 0, s, a);
    else hipLaunchKernelGGL((k_recon<T, MODE, 32>), grid, dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_recon(int mode, const ReconArgs<T> &a, int *nparts, hipStream_t s)
{
    if (!recon_ok(a.c)) return hipErrorInvalidValue;
    if (a.ysk && (mode != kEpi || a.csk < 1 || a.csk > 8)) return hipErrorInvalidValue;
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
