// elementwise.hip -- rank-l shrink-and-reconstruct, the RPCA epilogue and elementwise helpers (Alg. 1's thresholded reconstruction and the iALM updates).
#include "block_dense.h"
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
// (ncol_blk: the workgroup's column count, 8 or 16; an[] holds zeros past it)
template <bool PRE>
__device__ __forceinline__ void sketch_rows(const ReconArgs<double> &a, int64_t pr, int rb, int cb, int ncol_blk,
                                            double (&an)[16], double *sW)
{
    const int lane = threadIdx.x % kWave;
    // Omega row pr, columns j < csk (the sketch pass's draw: pair p of row k
    // gives columns 2p and 2p + 1)
    double om[8];
    if (PRE) {
        // drawn beforehand (k_omega_rows), eight per row
#pragma unroll
        for (int j = 0; j < 8; ++j) om[j] = pr < a.rows ? a.om[pr * 8 + j] : 0.0;
    } else {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            double z0 = 0.0, z1 = 0.0;
            if (2 * p < a.csk && pr < a.rows) gaussian_pair(a.seed, a.counter, (uint32_t)pr, (uint32_t)p, z0, z1);
            om[2 * p] = z0;
            om[2 * p + 1] = (2 * p + 1 < a.csk) ? z1 : 0.0;
        }
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
        const int64_t pc = (int64_t)cb * ncol_blk + i;
        const double t = ((sC[(0 * 8 + j) * 16 + i] + sC[(1 * 8 + j) * 16 + i]) + sC[(2 * 8 + j) * 16 + i]) +
                         sC[(3 * 8 + j) * 16 + i];
        if (j < a.csk && i < ncol_blk && pc < a.cols) a.ysk[(int64_t)rb * a.cols * a.csk + pc + (int64_t)j * a.cols] = t;
    }
}

// Omega(k, j) for rows k < rows and j < csk <= 8 (zeros up to eight per
// row), exactly as the sketch draws it (pair p of row k gives columns 2p and
// 2p + 1): the epilogue's sketch reads these rows instead of drawing them in
// each of its column blocks.
__global__ void __launch_bounds__(kThreads) k_omega_rows(int64_t rows, int csk, uint64_t seed, uint64_t counter,
                                                         double *om)
{
    const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t k = idx >> 2;
    const int p = (int)(idx & 3);
    if (k >= rows) return;
    double z0 = 0.0, z1 = 0.0;
    if (2 * p < csk) gaussian_pair(seed, counter, (uint32_t)k, (uint32_t)p, z0, z1);
    om[k * 8 + 2 * p] = z0;
    om[k * 8 + 2 * p + 1] = (2 * p + 1 < csk) ? z1 : 0.0;
}

hipError_t launch_omega_rows(int64_t rows, int csk, uint64_t seed, uint64_t counter, double *om, hipStream_t s)
{
    if (rows < 1 || csk < 1 || csk > 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_omega_rows, dim3((unsigned)((4 * rows + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                       rows, csk, seed, counter, om);
    return hipGetLastError();
}

// SK: 0 no sketch, 1 the sketch with Omega drawn here, 2 with Omega's rows
// read from a.om
template <typename T, int MODE, int CM, int SK = 0, int NC = kReconCols>
__global__ void __launch_bounds__(kThreads, (SK == 2 && CM <= 16) ? 3 : 1) k_recon(ReconArgs<T> a)
{
    constexpr int kReconCols = NC;   // this instantiation's columns per workgroup
    __shared__ T sFC[kReconCols][CM];
    __shared__ double sred[kThreads / kWave];
    // XCD-aware tile order: workgroups are dealt to the eight XCDs in turn
    // (w mod 8), so workgroup w takes row block 8 (i / nb) + w mod 8 and
    // column block i mod nb, i = w / 8, nb column blocks: every column block
    // of a row block runs on one XCD, one after the other, and the row
    // factors (and the sketch's Omega rows) they all read stay in its L2
    const int xcd = (int)(blockIdx.x & 7), wi = (int)(blockIdx.x >> 3);
    const int rb = (wi / a.ncb) * 8 + xcd, cb = wi % a.ncb;
    if (rb >= a.nrb) return;
    const int64_t pr = (int64_t)rb * kThreads + threadIdx.x;
    const int64_t pc0 = (int64_t)cb * kReconCols;
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
    T anv[SK ? 16 : 1];
#pragma unroll
    for (int j = 0; j < (SK ? 16 : 1); ++j) anv[j] = T(0);
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
        T ov[kReconCols], yv[kReconCols];
        if (MODE != kRecon) {
#pragma unroll
            for (int j = 0; j < kReconCols; ++j) {
                const int64_t pc = pc0 + min(j, ncol - 1);
                ov[j] = __builtin_nontemporal_load(&a.O[pr + pc * a.ldo]);
                yv[j] = __builtin_nontemporal_load(&a.Y[pr + pc * a.ldy]);
            }
        }
        // L of each column formed where it is used (from the factors, or read)
        T lin[kReconCols];
        if (a.Lin) {
#pragma unroll
            for (int j = 0; j < kReconCols; ++j) lin[j] = a.Lin[pr + (pc0 + min(j, ncol - 1)) * a.ldlin];
        }
#pragma unroll
        for (int j = 0; j < kReconCols; ++j) {
            if (j >= ncol) continue;
            const int64_t pc = pc0 + j;
            T L = T(0);
            if (a.Lin) {
                L = lin[j];
            } else {
#pragma unroll
                for (int cc = 0; cc < CM; ++cc) L += fr[cc] * sFC[j][cc];
            }
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
    if constexpr (SK != 0) {
        __shared__ double sW[kThreads / kWave][64 * 17];
        sketch_rows<SK == 2>(a, pr, rb, cb, kReconCols, anv, sW[threadIdx.x / kWave]);
    }
    if (MODE == kEpi) {
        zz = wave_sum(zz);
        if (threadIdx.x % kWave == 0) sred[threadIdx.x / kWave] = zz;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < kThreads / kWave; ++w) s += sred[w];
            a.zpart[(int64_t)cb * a.nrb + rb] = s;
        }
    }
}

template <typename T, int MODE>
static hipError_t launch_recon_cm(const ReconArgs<T> &a, dim3 grid, hipStream_t s)
{
    // (a carries nrb, ncb; the grid is 8 ceil(nrb / 8) ncb workgroups)
    if constexpr (MODE == kEpi && std::is_same<T, double>::value) {
        if (a.ysk && a.om) {
            if (a.c <= 8) hipLaunchKernelGGL((k_recon<T, MODE, 8, 2>), grid, dim3(kThreads), 0, s, a);
            else if (a.c <= 16) hipLaunchKernelGGL((k_recon<T, MODE, 16, 2>), grid, dim3(kThreads), 0, s, a);
            else hipLaunchKernelGGL((k_recon<T, MODE, 32, 2>), grid, dim3(kThreads), 0, s, a);
            return hipGetLastError();
        }
        if (a.ysk) {
            if (a.c <= 8) hipLaunchKernelGGL((k_recon<T, MODE, 8, 1>), grid, dim3(kThreads), 0, s, a);
            else if (a.c <= 16) hipLaunchKernelGGL((k_recon<T, MODE, 16, 1>), grid, dim3(kThreads), 0, s, a);
            else hipLaunchKernelGGL((k_recon<T, MODE, 32, 1>), grid, dim3(kThreads), 0, s, a);
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
    ReconArgs<T> b = a;
    const int ncol = kReconCols;
    const int64_t nrb = (a.rows + kThreads - 1) / kThreads, ncb = (a.cols + ncol - 1) / ncol;
    if (nrb < 1 || ncb < 1 || 8 * ((nrb + 7) / 8) * ncb > (int64_t)0x7fffffff) return hipErrorInvalidValue;
    b.nrb = (int)nrb;
    b.ncb = (int)ncb;
    dim3 grid((unsigned)(8 * ((nrb + 7) / 8) * ncb));
    if (nparts) *nparts = (int)(nrb * ncb);
    if (mode == kRecon) return launch_recon_cm<T, kRecon>(b, grid, s);
    if (mode == kEpi) return launch_recon_cm<T, kEpi>(b, grid, s);
    return launch_recon_cm<T, kFinal>(b, grid, s);
}
template hipError_t launch_recon<double>(int, const ReconArgs<double> &, int *, hipStream_t);
template hipError_t launch_recon<float>(int, const ReconArgs<float> &, int *, hipStream_t);

// ===========================================================================
// Elementwise helpers.
// ===========================================================================
// Per-workgroup sum of squares and largest magnitude of A (m x n, ld lda),
// and, when flag is set, *flag |= 1 for a NaN or infinite entry (the same
// pass).  A dense A (lda == m) is read as one flat array.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_norms(int64_t m, int64_t n, const T *A, int64_t lda, double *parts,
                                                    int *flag)
{
    __shared__ double s1[kThreads / kWave], s2[kThreads / kWave];
    double ss = 0.0, mx = 0.0;
    int bad = 0;
    const int64_t total = m * n;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    if (lda == m) {
        for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < total; idx += stride) {
            const double v = (double)A[idx];
            ss += v * v;
            mx = fmax(mx, fabs(v));
            bad |= !isfinite(v);
        }
    } else {
        for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < total; idx += stride) {
            const int64_t i = idx % m, j = idx / m;
            const double v = (double)A[i + j * lda];
            ss += v * v;
            mx = fmax(mx, fabs(v));
            bad |= !isfinite(v);
        }
    }
    if (flag && __any(bad) && threadIdx.x % kWave == 0) atomicOr(flag, 1);
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
hipError_t launch_norms(int64_t m, int64_t n, const T *A, int64_t lda, double *parts, int *nparts, hipStream_t s,
                        int *flag)
{
    const int grid = 1024;
    *nparts = grid;
    hipLaunchKernelGGL((k_norms<T>), dim3(grid), dim3(kThreads), 0, s, m, n, A, lda, parts, flag);
    return hipGetLastError();
}
template hipError_t launch_norms<double>(int64_t, int64_t, const double *, int64_t, double *, int *, hipStream_t,
                                         int *);
template hipError_t launch_norms<float>(int64_t, int64_t, const float *, int64_t, double *, int *, hipStream_t, int *);

template <typename T>
__global__ void __launch_bounds__(kThreads) k_rpca_init(int64_t m, int64_t n, const T *O, int64_t ldo, double invJ, double inv_mu, T *Y, int64_t ldy, T *A, int64_t lda)
{
    const int64_t total = m * n;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    if (ldo == m && ldy == m && lda == m) {
        // dense: one flat index (no division per element)
        for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < total; idx += stride) {
            const T o = O[idx];
            const T y = o * (T)invJ;
            Y[idx] = y;
            A[idx] = o + y * (T)inv_mu;
        }
        return;
    }
    for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < total; idx += stride) {
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


// Largest eigenvalue of a symmetric positive semidefinite n x n matrix G
// (the Gram A A^T; 8 <= n <= 1024, global memory, one workgroup) by subspace
// iteration with a block of kEigB vectors and Rayleigh-Ritz: from a Gaussian
// start block (Philox), each outer step forms W = G V and the Rayleigh matrix
// H = V^T W of the orthonormal V; its eigenvalues are the squared singular
// values of the Cholesky factor of H, found by the lane-grid one-sided Jacobi
// of one wavefront; theta_1 is the estimate.  V then advances by kEigQ
// products with G (scaled by 1 / theta_1) and two Cholesky-QR passes.  The
// error of theta_1 contracts by (lambda_{kEigB+1} / lambda_1)^2 per product,
// whatever the gaps inside the top kEigB (close or equal top eigenvalues do
// not slow it); the smallest Ritz value theta_kEigB (<= lambda_kEigB) over
// theta_1 bounds that ratio from above once the block has settled.  Stops
// when theta_1 moved by at most 16 n u of itself (the rounding level of the
// Rayleigh matrix) and (theta_kEigB / theta_1)^(2 m) <= 1e-16, m the
// products behind the current V plus one, or after max_it outer steps.
// out[0] = theta_1, out[1] = 1 when the test was met (else 0: the caller
// takes another method), out[2] = the outer steps taken.
constexpr int kEigB = 8;
constexpr int kEigNP = kEigB * (kEigB + 1) / 2;   // packed symmetric entries
constexpr int kEigThreads = 256;
constexpr int kEigQ = 4;   // products with G per outer step

__device__ __forceinline__ void eig_pair(int p, int &a, int &b)
{
    a = 0;
    while (p >= kEigB - a) {
        p -= kEigB - a;
        ++a;
    }
    b = a + p;
}

// packed index of (a, b), a <= b (rows of the upper triangle in order)
__host__ __device__ constexpr int eig_idx(int a, int b) { return a * kEigB - a * (a - 1) / 2 + (b - a); }

// Packed symmetric sums over the block's rows: red[k] = sum_i x_i[a] y_i[b]
// for the kEigNP pairs (a <= b), in a fixed order (wavefront shuffles, then
// the wavefronts in order).
__device__ __forceinline__ void eig_block_gram(int n, const double *X, const double *Y, double *part,
                                               double *red)
{
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    constexpr int nw = kEigThreads / kWave;
    double acc[kEigNP];
#pragma unroll
    for (int p = 0; p < kEigNP; ++p) acc[p] = 0.0;
    for (int i = tid; i < n; i += kEigThreads) {
        double x[kEigB], y[kEigB];
#pragma unroll
        for (int c = 0; c < kEigB; ++c) {
            x[c] = X[i * kEigB + c];
            y[c] = Y[i * kEigB + c];
        }
#pragma unroll
        for (int a = 0; a < kEigB; ++a)
#pragma unroll
            for (int b = a; b < kEigB; ++b) acc[eig_idx(a, b)] += x[a] * y[b];
    }
#pragma unroll
    for (int p = 0; p < kEigNP; ++p) {
        const double v = wave_sum(acc[p]);
        if (lane == 0) part[p * nw + wave] = v;
    }
    __syncthreads();
    if (tid < kEigNP) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += part[tid * nw + w];
        red[tid] = s;
    }
    __syncthreads();
}

// Semidefinite upper Cholesky factor of the packed Gram (one thread, all in
// registers): a pivot at or below 64 u times the largest diagonal entry
// gives a zero row (the block has lost that direction: G has smaller rank
// than the block, and the remaining columns already span its range); false
// for a non-finite Gram.
__device__ bool eig_chol(const double *gp, double *R)
{
    double M[kEigB][kEigB];
    double mx = 0.0;
#pragma unroll
    for (int a = 0; a < kEigB; ++a)
#pragma unroll
        for (int b = 0; b < kEigB; ++b) {
            M[a][b] = b >= a ? gp[eig_idx(a, b)] : 0.0;
            if (a == b) mx = fmax(mx, M[a][b]);
        }
    if (!(mx < 1e300)) return false;
    const double tol = 64.0 * kU * mx;
#pragma unroll
    for (int j = 0; j < kEigB; ++j) {
        double d = M[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) d -= M[k][j] * M[k][j];
        const bool null = !(d > tol);
        const double r = null ? 0.0 : sqrt(d);
        const double inv = null ? 0.0 : 1.0 / r;
        M[j][j] = r;
#pragma unroll
        for (int c = j + 1; c < kEigB; ++c) {
            double v = M[j][c];
#pragma unroll
            for (int k = 0; k < j; ++k) v -= M[k][j] * M[k][c];
            M[j][c] = v * inv;
        }
    }
#pragma unroll
    for (int a = 0; a < kEigB; ++a)
#pragma unroll
        for (int b = 0; b < kEigB; ++b) R[a * kEigB + b] = b >= a ? M[a][b] : 0.0;
    return true;
}

__global__ void __launch_bounds__(kEigThreads) k_power_eig(int n, const double *G, double *out, int max_it)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *V = reinterpret_cast<double *>(smem_raw);          // n x kEigB, row-major
    double *W = V + (size_t)n * kEigB;                          // n x kEigB
    __shared__ double part[kEigNP * (kEigThreads / kWave)];
    __shared__ double red[kEigNP];
    __shared__ double R[kEigB * kEigB];
    __shared__ double est_sh;
    __shared__ int stop_sh, ok_sh;
    const int tid = threadIdx.x;
    // Gaussian start block (a fixed Philox stream)
    for (int i = tid; i < n; i += kEigThreads)
        for (int c = 0; c < kEigB; c += 2) {
            double z0, z1;
            gaussian_pair(0x6e6f726d32ull, 0, (uint32_t)i, 0x40000000u | (uint32_t)c, z0, z1);
            V[i * kEigB + c] = z0;
            V[i * kEigB + c + 1] = z1;
        }
    if (tid == 0) {
        est_sh = 0.0;
        stop_sh = 0;
        ok_sh = 0;
    }
    __syncthreads();
    // X <- X R^-1 for the rows of X (zero pivots give zero columns)
    auto right_solve = [&](double *X) {
        for (int i = tid; i < n; i += kEigThreads) {
            double x[kEigB];
#pragma unroll
            for (int c = 0; c < kEigB; ++c) x[c] = X[i * kEigB + c];
#pragma unroll
            for (int c = 0; c < kEigB; ++c) {
                double v = x[c];
#pragma unroll
                for (int k = 0; k < c; ++k) v -= x[k] * R[k * kEigB + c];
                const double rc = R[c * kEigB + c];
                x[c] = rc > 0.0 ? v / rc : 0.0;
            }
#pragma unroll
            for (int c = 0; c < kEigB; ++c) V[i * kEigB + c] = x[c];
        }
        __syncthreads();
    };
    // V = orth(X): two Cholesky-QR passes
    auto orth = [&](double *X) {
        for (int pass = 0; pass < 2; ++pass) {
            double *Xp = pass == 0 ? X : V;
            eig_block_gram(n, Xp, Xp, part, red);
            if (tid == 0 && !eig_chol(red, R)) stop_sh = 2;
            __syncthreads();
            if (stop_sh == 2) return;
            right_solve(Xp);
        }
    };
    // Y = scale G X (G symmetric: row i read as column i, coalesced across
    // threads; 32 loads in flight per thread)
    auto matvec = [&](const double *X, double *Y, double scale) {
        for (int i = tid; i < n; i += kEigThreads) {
            double w[kEigB];
#pragma unroll
            for (int c = 0; c < kEigB; ++c) w[c] = 0.0;
            for (int j0 = 0; j0 < n; j0 += 32) {
                double gv[32];
#pragma unroll
                for (int u = 0; u < 32; ++u) gv[u] = j0 + u < n ? G[i + (size_t)(j0 + u) * n] : 0.0;
#pragma unroll
                for (int u = 0; u < 32; ++u) {
                    if (j0 + u < n) {
#pragma unroll
                        for (int c = 0; c < kEigB; ++c) w[c] += gv[u] * X[(j0 + u) * kEigB + c];
                    }
                }
            }
#pragma unroll
            for (int c = 0; c < kEigB; ++c) Y[i * kEigB + c] = w[c] * scale;
        }
        __syncthreads();
    };
    orth(V);
    int m = 0, it = 0;
    for (it = 0; it < max_it && stop_sh == 0; ++it) {
        matvec(V, W, 1.0);
        // Rayleigh matrix of V; its extreme eigenvalues from wavefront 0
        eig_block_gram(n, V, W, part, red);
        if (tid < kWave) {
            double g[8][8];
#pragma unroll
            for (int a = 0; a < 8; ++a)
#pragma unroll
                for (int b = 0; b < 8; ++b) g[a][b] = b >= a ? red[eig_idx(a, b)] : 0.0;
            double x = wave8_factor(g, kEigB);
            wave8_jacobi(x, kEigB, 60);
            const double s2 = seg8_sum(x * x);
            double est = 0.0, tmin = 0.0;
#pragma unroll
            for (int b = 0; b < kEigB; ++b) {
                const double t = read_lane(s2, b * 8);
                est = b ? fmax(est, t) : t;
                tmin = b ? fmin(tmin, t) : t;
            }
            if (tid == 0) {
                const double d = est - est_sh;
                const double ratio = est > 0.0 ? fmax(tmin, 0.0) / est : 1.0;
                // the Rayleigh matrix carries rounding of order n u lambda_1: a
                // step that moves the estimate by less than 16 n u of it has
                // converged
                if (it >= 1 && fabs(d) <= 16.0 * (double)n * kU * fabs(est) && pow(ratio, 2.0 * (m + 1)) <= 1e-16) {
                    stop_sh = 1;
                    ok_sh = 1;
                }
                if (!(est > 0.0)) {  // G = 0
                    stop_sh = 1;
                    ok_sh = 1;
                }
                est_sh = fmax(est, est_sh);
            }
        }
        __syncthreads();
        if (stop_sh) break;
        // V <- orth(G^kEigQ V), the products scaled by 1 / theta_1
        const double sc = 1.0 / est_sh;
        for (int q = 1; q < kEigQ; ++q) {
            if (q & 1) matvec(W, V, sc);
            else matvec(V, W, sc);
        }
        orth((kEigQ - 1) & 1 ? V : W);
        m += kEigQ;
    }
    if (tid == 0) {
        out[0] = est_sh;
        out[1] = ok_sh ? 1.0 : 0.0;
        out[2] = (double)it;
    }
}

// Largest eigenvalue of a symmetric positive semidefinite n x n matrix G
// (n <= 256, one workgroup, thread i owns row i) when it dominates: single
// vector power iteration y = G x (x unit, from a fixed Philox start) with
// the Rayleigh quotient theta = x^T y and the residual eps^2 = ||y||^2 -
// theta^2 = ||G x - theta x||^2.  All eigenvalues are >= 0, so lambda_2 <=
// trace(G) - lambda_1 <= trace(G) - theta; once theta > trace(G) / 2 that
// leaves lambda_1 as the only eigenvalue above trace(G) - theta, and the
// Kato-Temple inequality bounds lambda_1 - theta <= eps^2 / (2 theta -
// trace(G)).  eps^2 is formed with an absolute rounding error below 4 u
// ||y||^2, which the test adds.  Stops when that bound is at most 1e-15
// theta: out[0] = theta, out[1] = 1; after max_it steps (no dominant
// eigenvalue, or too slow) out[1] = 0 and the caller takes the block method.
// NG > 0: n <= NG and thread i keeps row i of G in registers for the whole
// iteration (one read of G); NG = 0: each product streams G again.
template <int NG>
__global__ void __launch_bounds__(kEigThreads) k_power_dom(int n, const double *G, double *out, int max_it)
{
    __shared__ double sx[256];
    __shared__ double part[2 * (kEigThreads / kWave)];
    __shared__ double tr_sh;
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    constexpr int nw = kEigThreads / kWave;
    // start vector and trace
    double xi = 0.0, gii = 0.0;
    if (tid < n) {
        double z0, z1;
        gaussian_pair(0x646f6d6e74ull, 0, (uint32_t)tid, 0x40000000u, z0, z1);
        xi = z0;
        gii = G[tid + (size_t)tid * n];
    }
    {
        const double a = wave_sum(xi * xi), t = wave_sum(gii);
        if (lane == 0) {
            part[wave] = a;
            part[nw + wave] = t;
        }
        __syncthreads();
        if (tid == 0) {
            double s2 = 0.0, tr = 0.0;
            for (int w = 0; w < nw; ++w) {
                s2 += part[w];
                tr += part[nw + w];
            }
            part[0] = s2;
            tr_sh = tr;
        }
        __syncthreads();
        const double inv = part[0] > 0.0 ? 1.0 / sqrt(part[0]) : 0.0;
        sx[tid] = tid < n ? xi * inv : 0.0;   // zeros past n (read by the register form)
        __syncthreads();
    }
    const double tr = tr_sh;
    double grow[NG > 0 ? NG : 1];
    if constexpr (NG > 0) {
        // row i of G (= column i: G is symmetric), all loads issued at once
#pragma unroll
        for (int j = 0; j < NG; ++j) grow[j] = (tid < n && j < n) ? G[(size_t)tid * n + j] : 0.0;
    }
    double theta = 0.0;
    int ok = 0;
    if (!(tr > 0.0)) {
        // G = 0 (a PSD matrix with zero trace)
        ok = 1;
    } else {
        for (int it = 0; it < max_it; ++it) {
            // y_i = sum_j G(i, j) x_j (column j read across the threads)
            double yi = 0.0, xo = 0.0;
            if (NG > 0 && tid < n) {
                xo = sx[tid];
                // two chains, x read from LDS two entries at a time
                double y0 = 0.0, y1 = 0.0;
#pragma unroll
                for (int j = 0; j < (NG > 0 ? NG : 2); j += 2) {
                    y0 += grow[j] * sx[j];
                    y1 += grow[j + 1] * sx[j + 1];
                }
                yi = y0 + y1;
            } else if (tid < n) {
                xo = sx[tid];
                for (int j0 = 0; j0 < n; j0 += 32) {
                    double gv[32];
#pragma unroll
                    for (int u = 0; u < 32; ++u) gv[u] = j0 + u < n ? G[tid + (size_t)(j0 + u) * n] : 0.0;
#pragma unroll
                    for (int u = 0; u < 32; ++u)
                        if (j0 + u < n) yi += gv[u] * sx[j0 + u];
                }
            }
            const double a = wave_sum(xo * yi), b = wave_sum(yi * yi);
            if (lane == 0) {
                part[wave] = a;
                part[nw + wave] = b;
            }
            __syncthreads();
            double th = 0.0, yy = 0.0;
            for (int w = 0; w < nw; ++w) {
                th += part[w];
                yy += part[nw + w];
            }
            theta = th;
            const double eps2 = fmax(yy - th * th, 0.0) + 4.0 * kU * yy;
            const double gap = 2.0 * th - tr;
            if (gap > 0.0 && eps2 <= 1e-15 * th * gap) {
                ok = 1;
                break;
            }
            __syncthreads();  // every read of sx and part is done
            if (tid < n) sx[tid] = yy > 0.0 ? yi / sqrt(yy) : 0.0;
            __syncthreads();
        }
    }
    if (tid == 0) {
        out[0] = theta;
        out[1] = ok ? 1.0 : 0.0;
    }
}

hipError_t launch_power_dom(int n, const double *G, double *out, hipStream_t s)
{
    if (n < 1 || n > 256) return hipErrorInvalidValue;
    if (n <= 208)
        hipLaunchKernelGGL(k_power_dom<208>, dim3(1), dim3(kEigThreads), 0, s, n, G, out, 60);
    else
        hipLaunchKernelGGL(k_power_dom<0>, dim3(1), dim3(kEigThreads), 0, s, n, G, out, 60);
    return hipGetLastError();
}

hipError_t launch_power_eig(int n, const double *G, double *out, hipStream_t s)
{
    if (n < kEigB || n > 1024) return hipErrorInvalidValue;
    const size_t lds = 2 * (size_t)n * kEigB * sizeof(double);
    hipLaunchKernelGGL(k_power_eig, dim3(1), dim3(kEigThreads), lds, s, n, G, out, 100);
    return hipGetLastError();
}

}  // namespace frk
