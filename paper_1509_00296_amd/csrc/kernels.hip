// kernels.hip -- gfx950 kernels of the FRSVT library.
//
// Steps of Alg. 1 of "Fast Randomized Singular Value Thresholding for
// Low-rank Optimization" (arXiv:1509.00296) and of the inexact-ALM RPCA host:
//   long pass (sketch Y = Ahat Omega, fused power step Y = Ahat Ahat^T Q,
//   projection B^T = Ahat^T Q with its Gram B B^T), the split-K reduction,
//   CholeskyQR re-orthonormalisation, the small SVD of B through the Cholesky
//   factor of B B^T and a one-sided Jacobi SVD, the rank-l
//   shrink-and-reconstruct / RPCA epilogue, a generic tiled GEMM for shapes
//   beyond the one-workgroup paths.
#include "device_common.h"
#include "internal.h"

#include <algorithm>

namespace frk {

constexpr int kThreads = 256;
constexpr double kU = 1.1102230246251565e-16;  // unit roundoff of double

// ===========================================================================
// Long pass: one workgroup owns a tile of `kt` long-dimension indices and the
// whole short dimension.  The tile of Ahat is staged in LDS as
// sTile[kk * mhp + i] (i contiguous, odd stride so that column reads across
// lanes avoid bank conflicts) whatever the global layout; loads are coalesced
// along whichever dimension is contiguous in memory.
// ===========================================================================
bool long_path_ok(int mh, int c) { return mh >= 1 && mh <= 1024 && c >= 1 && c <= 32 && (mh | 1) * c <= 6144; }

static int pow2_floor(int v)
{
    int p = 1;
    while (p * 2 <= v) p *= 2;
    return p;
}

LongPlan long_plan(int mh, int64_t nh, int c, int elem_bytes, int mode, int num_cu)
{
    LongPlan p{};
    p.mhp = mh | 1;
    p.cm = c <= 8 ? 8 : (c <= 16 ? 16 : 32);
    p.rpt = (mh + kThreads - 1) / kThreads;
    // tile + V tile + (Q) within 64 KB of LDS
    size_t qbytes = (mode == kPower || mode == kProject) ? (size_t)c * p.mhp * elem_bytes : 0;
    size_t budget = qbytes < 48 * 1024 ? 64 * 1024 - qbytes : 16 * 1024;
    int kt = (int)(budget / ((size_t)p.mhp * elem_bytes + (size_t)p.cm * elem_bytes));
    kt = std::max(4, std::min(64, pow2_floor(std::max(kt, 4))));
    p.kt = kt;
    p.ntiles = (int)((nh + kt - 1) / kt);
    int target = 2 * num_cu;
    p.grid = std::max(1, std::min(p.ntiles, target));
    p.lds = (size_t)kt * p.mhp * elem_bytes + (size_t)kt * p.cm * elem_bytes + qbytes;
    return p;
}

template <typename T, bool TR, int MODE, int CM, int RPT>
__global__ void __launch_bounds__(kThreads) k_long(LongArgs<T> a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *sTile = reinterpret_cast<T *>(smem_raw);
    T *sV = sTile + (size_t)a.kt * a.mhp;
    T *sQ = sV + (size_t)a.kt * CM;
    const int tid = threadIdx.x;
    const int mh = a.mh, c = a.c, kt = a.kt, mhp = a.mhp;

    for (int idx = tid; idx < kt * CM; idx += kThreads) sV[idx] = T(0);
    if (MODE == kPower || MODE == kProject) {
        for (int idx = tid; idx < mh * c; idx += kThreads) {
            const int i = idx % mh, cc = idx / mh;
            sQ[cc * mhp + i] = a.Q[i + (int64_t)cc * a.ldq];
        }
    }
    T acc[RPT][CM];
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int cc = 0; cc < CM; ++cc) acc[r][cc] = T(0);
    double gacc[4] = {0.0, 0.0, 0.0, 0.0};

    for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
        const int64_t k0 = (int64_t)tile * kt;
        const int kval = (int)min((int64_t)kt, a.nh - k0);
        if (TR) {
            for (int idx = tid; idx < kt * mh; idx += kThreads) {
                const int kk = idx % kt, i = idx / kt;
                sTile[kk * mhp + i] = kk < kval ? a.A[(k0 + kk) + (int64_t)i * a.lda] : T(0);
            }
        } else {
            for (int idx = tid; idx < kt * mh; idx += kThreads) {
                const int i = idx % mh, kk = idx / mh;
                sTile[kk * mhp + i] = kk < kval ? a.A[i + (k0 + kk) * a.lda] : T(0);
            }
        }
        if (MODE == kSketch) {
            const int npair = (c + 1) / 2;
            for (int idx = tid; idx < kt * npair; idx += kThreads) {
                const int kk = idx % kt, j = idx / kt;
                double z0 = 0.0, z1 = 0.0;
                if (kk < kval) gaussian_pair(a.seed, a.counter, (uint32_t)(k0 + kk), (uint32_t)j, z0, z1);
                sV[kk * CM + 2 * j] = T(z0);
                if (2 * j + 1 < c) sV[kk * CM + 2 * j + 1] = T(z1);
            }
        } else if (MODE == kVecMul) {
            for (int idx = tid; idx < kt * c; idx += kThreads) {
                const int kk = idx % kt, cc = idx / kt;
                sV[kk * CM + cc] = kk < kval ? a.V[(k0 + kk) + (int64_t)cc * a.ldv] : T(0);
            }
        }
        __syncthreads();
        if (MODE == kPower || MODE == kProject) {
            for (int idx = tid; idx < kt * c; idx += kThreads) {
                const int cc = idx % c, kk = idx / c;
                const T *tr = sTile + kk * mhp;
                const T *qr = sQ + cc * mhp;
                T s0 = T(0), s1 = T(0);
                int i = 0;
                for (; i + 1 < mh; i += 2) {
                    s0 += tr[i] * qr[i];
                    s1 += tr[i + 1] * qr[i + 1];
                }
                if (i < mh) s0 += tr[i] * qr[i];
                sV[kk * CM + cc] = s0 + s1;
            }
            __syncthreads();
        }
        if (MODE == kProject) {
            for (int idx = tid; idx < kt * c; idx += kThreads) {
                const int kk = idx % kt, cc = idx / kt;
                if (kk < kval) a.Z[(k0 + kk) + (int64_t)cc * a.ldz] = sV[kk * CM + cc];
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int p = tid + e * kThreads;
                if (p < c * c) {
                    const int x = p % c, y = p / c;
                    double s = 0.0;
                    for (int kk = 0; kk < kt; ++kk)
                        s += (double)sV[kk * CM + x] * (double)sV[kk * CM + y];
                    gacc[e] += s;
                }
            }
        } else {
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int i = tid + r * kThreads;
                if (i < mh) {
                    for (int kk = 0; kk < kt; ++kk) {
                        const T av = sTile[kk * mhp + i];
                        const T *vr = sV + kk * CM;
#pragma unroll
                        for (int cc = 0; cc < CM; ++cc) acc[r][cc] += av * vr[cc];
                    }
                }
            }
        }
        __syncthreads();
    }
    if (MODE == kProject) {
        double *gp = a.Gpart + (size_t)blockIdx.x * c * c;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int p = tid + e * kThreads;
            if (p < c * c) gp[p] = gacc[e];
        }
    } else {
        T *yp = a.Ypart + (size_t)blockIdx.x * mh * c;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int i = tid + r * kThreads;
            if (i < mh)
#pragma unroll
                for (int cc = 0; cc < CM; ++cc)
                    if (cc < c) yp[i + (size_t)cc * mh] = acc[r][cc];
        }
    }
}

template <typename T, bool TR, int MODE, int CM>
static hipError_t launch_long_rpt(const LongPlan &p, const LongArgs<T> &a, hipStream_t s)
{
    switch (p.rpt) {
    case 1: hipLaunchKernelGGL((k_long<T, TR, MODE, CM, 1>), dim3(p.grid), dim3(kThreads), p.lds, s, a); break;
    case 2: hipLaunchKernelGGL((k_long<T, TR, MODE, CM, 2>), dim3(p.grid), dim3(kThreads), p.lds, s, a); break;
    default: hipLaunchKernelGGL((k_long<T, TR, MODE, CM, 4>), dim3(p.grid), dim3(kThreads), p.lds, s, a); break;
    }
    return hipGetLastError();
}

template <typename T, bool TR, int MODE>
static hipError_t launch_long_cm(const LongPlan &p, const LongArgs<T> &a, hipStream_t s)
{
    if (p.cm == 8) return launch_long_rpt<T, TR, MODE, 8>(p, a, s);
    if (p.cm == 16) return launch_long_rpt<T, TR, MODE, 16>(p, a, s);
    return launch_long_rpt<T, TR, MODE, 32>(p, a, s);
}

template <typename T, bool TR>
static hipError_t launch_long_mode(const LongPlan &p, int mode, const LongArgs<T> &a, hipStream_t s)
{
    switch (mode) {
    case kSketch: return launch_long_cm<T, TR, kSketch>(p, a, s);
    case kVecMul: return launch_long_cm<T, TR, kVecMul>(p, a, s);
    case kPower: return launch_long_cm<T, TR, kPower>(p, a, s);
    default: return launch_long_cm<T, TR, kProject>(p, a, s);
    }
}

template <typename T>
hipError_t launch_long(const LongPlan &p, int mode, const LongArgs<T> &a0, hipStream_t s)
{
    LongArgs<T> a = a0;
    a.kt = p.kt;
    a.mhp = p.mhp;
    a.ntiles = p.ntiles;
    if (p.rpt > 4) return hipErrorInvalidValue;
    if (a.trans) return launch_long_mode<T, true>(p, mode, a, s);
    return launch_long_mode<T, false>(p, mode, a, s);
}
template hipError_t launch_long<double>(const LongPlan &, int, const LongArgs<double> &, hipStream_t);
template hipError_t launch_long<float>(const LongPlan &, int, const LongArgs<float> &, hipStream_t);

// ===========================================================================
// Split-K reduction in a fixed order (bitwise reproducible).
// ===========================================================================
template <typename T>
__global__ void __launch_bounds__(kThreads) k_reduce(const T *part, int64_t count, int nparts, T *out)
{
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j >= count) return;
    T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
    int g = 0;
    for (; g + 3 < nparts; g += 4) {
        s0 += part[(int64_t)g * count + j];
        s1 += part[(int64_t)(g + 1) * count + j];
        s2 += part[(int64_t)(g + 2) * count + j];
        s3 += part[(int64_t)(g + 3) * count + j];
    }
    for (; g < nparts; ++g) s0 += part[(int64_t)g * count + j];
    out[j] = (s0 + s1) + (s2 + s3);
}

template <typename T>
hipError_t launch_reduce(const T *part, int64_t count, int nparts, T *out, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    const int grid = (int)((count + kThreads - 1) / kThreads);
    hipLaunchKernelGGL((k_reduce<T>), dim3(grid), dim3(kThreads), 0, s, part, count, nparts, out);
    return hipGetLastError();
}
template hipError_t launch_reduce<double>(const double *, int64_t, int, double *, hipStream_t);
template hipError_t launch_reduce<float>(const float *, int64_t, int, float *, hipStream_t);

// ===========================================================================
// Block-level dense helpers on LDS-resident column-major matrices (double).
// W: l columns of length mh at W[j * mhp + i].  G, R: l x l at [a * l + b].
// ===========================================================================

// G = W^T W (full symmetric), one wavefront per (a, b) pair, lanes over rows.
__device__ void block_gram(const double *W, int mh, int mhp, int l, double *G)
{
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    const int npairs = l * (l + 1) / 2;
    for (int p = wave; p < npairs; p += nw) {
        int a = 0, rem = p;
        while (rem >= l - a) {
            rem -= l - a;
            ++a;
        }
        const int b = a + rem;
        const double *wa = W + (size_t)a * mhp, *wb = W + (size_t)b * mhp;
        double s = 0.0;
        for (int i = lane; i < mh; i += kWave) s += wa[i] * wb[i];
        s = wave_sum(s);
        if (lane == 0) {
            G[a * l + b] = s;
            G[b * l + a] = s;
        }
    }
    __syncthreads();
}

// Cholesky of (G + shift I) into the upper triangle of R (row-major R[j*l+k]).
// Pivots <= null_tol are treated as numerically null: R_jj = 1 and a zero row,
// and null[j] = 1.  Returns (through sh_count) the number of null pivots.
__device__ void block_chol(const double *G, int l, double shift, double null_tol, double *R,
                           int *null_flags, int *sh_count)
{
    const int tid = threadIdx.x;
    if (tid == 0) *sh_count = 0;
    for (int idx = tid; idx < l * l; idx += blockDim.x) R[idx] = 0.0;
    __syncthreads();
    for (int j = 0; j < l; ++j) {
        __shared__ double piv;
        __shared__ int isnull;
        if (tid == 0) {
            double d = G[j * l + j] + shift;
            for (int t = 0; t < j; ++t) d -= R[t * l + j] * R[t * l + j];
            isnull = !(d > null_tol);
            if (isnull) {
                R[j * l + j] = 1.0;
                (*sh_count)++;
                if (null_flags) null_flags[j] = 1;
            } else {
                R[j * l + j] = sqrt(d);
                if (null_flags) null_flags[j] = 0;
            }
            piv = R[j * l + j];
        }
        __syncthreads();
        if (!isnull) {
            for (int k = j + 1 + tid; k < l; k += blockDim.x) {
                double v = G[j * l + k];
                for (int t = 0; t < j; ++t) v -= R[t * l + j] * R[t * l + k];
                R[j * l + k] = v / piv;
            }
        }
        __syncthreads();
    }
}

// W <- W R^{-1} (R upper, row-major), each thread owns rows.
__device__ void block_trsm(double *W, int mh, int mhp, int l, const double *R)
{
    for (int i = threadIdx.x; i < mh; i += blockDim.x) {
        for (int j = 0; j < l; ++j) {
            double v = W[(size_t)j * mhp + i];
            for (int t = 0; t < j; ++t) v -= W[(size_t)t * mhp + i] * R[t * l + j];
            W[(size_t)j * mhp + i] = v / R[j * l + j];
        }
    }
    __syncthreads();
}

// ===========================================================================
// One-workgroup orthonormalisation of [Qt, Y] (mh x l, l = rp + c), all in LDS.
//   1. CGS2: Y <- Y - Qt (Qt^T Y), twice (the partial orthogonalisation of
//      range propagation, Alg. 1 line 10).
//   2. Column equilibration (the span is what matters).
//   3. Shifted CholeskyQR: R = chol(W^T W + s I), s = 11 (mh l + l(l+1)) u
//      trace(W^T W), W <- W R^{-1}  (shifted CholeskyQR3 of Fukaya et al.).
//   4. CholeskyQR with null detection; null columns are replaced by fresh
//      Gaussian directions and the pass is repeated (any orthonormal
//      completion leaves the thresholded result unchanged).
//   5. A final CholeskyQR pass.
// ===========================================================================
bool small_orth_ok(int mh, int l) { return l >= 1 && l <= 64 && (size_t)(mh | 1) * l * 8 + (size_t)l * l * 16 <= 60 * 1024; }

template <typename T>
__global__ void __launch_bounds__(kThreads) k_small_orth(int mh, const T *Qt, int64_t ldqt, int rp,
                                                         const T *Y, int64_t ldy, int c, T *Q,
                                                         int64_t ldq, uint64_t seed,
                                                         uint64_t counter, int *flags)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int l = rp + c;
    const int mhp = mh | 1;
    double *W = reinterpret_cast<double *>(smem_raw);
    double *G = W + (size_t)l * mhp;
    double *R = G + (size_t)l * l;
    __shared__ int null_flags[64];
    __shared__ int nnull;
    __shared__ double scal[64];
    const int tid = threadIdx.x;
    const int lane = tid % kWave, wave = tid / kWave, nw = kThreads / kWave;

    for (int idx = tid; idx < mh * rp; idx += kThreads) {
        const int i = idx % mh, j = idx / mh;
        W[(size_t)j * mhp + i] = (double)Qt[i + (int64_t)j * ldqt];
    }
    for (int idx = tid; idx < mh * c; idx += kThreads) {
        const int i = idx % mh, j = idx / mh;
        W[(size_t)(rp + j) * mhp + i] = (double)Y[i + (int64_t)j * ldy];
    }
    __syncthreads();

    // 1. CGS2 against the propagated basis
    if (rp > 0 && c > 0) {
        for (int pass = 0; pass < 2; ++pass) {
            // coefficients C(t, j) = Qt(:,t)^T Y(:,j) into G (rp x c)
            for (int p = wave; p < rp * c; p += nw) {
                const int t = p % rp, j = p / rp;
                const double *qa = W + (size_t)t * mhp, *ya = W + (size_t)(rp + j) * mhp;
                double s = 0.0;
                for (int i = lane; i < mh; i += kWave) s += qa[i] * ya[i];
                s = wave_sum(s);
                if (lane == 0) G[t * c + j] = s;
            }
            __syncthreads();
            for (int idx = tid; idx < mh * c; idx += kThreads) {
                const int i = idx % mh, j = idx / mh;
                double v = W[(size_t)(rp + j) * mhp + i];
                for (int t = 0; t < rp; ++t) v -= W[(size_t)t * mhp + i] * G[t * c + j];
                W[(size_t)(rp + j) * mhp + i] = v;
            }
            __syncthreads();
        }
    }
    // 2. column equilibration
    for (int j = wave; j < l; j += nw) {
        const double *wj = W + (size_t)j * mhp;
        double s = 0.0;
        for (int i = lane; i < mh; i += kWave) s += wj[i] * wj[i];
        s = wave_sum(s);
        if (lane == 0) scal[j] = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    }
    __syncthreads();
    for (int idx = tid; idx < mh * l; idx += kThreads) {
        const int i = idx % mh, j = idx / mh;
        W[(size_t)j * mhp + i] *= scal[j];
    }
    __syncthreads();

    // 3. shifted CholeskyQR
    block_gram(W, mh, mhp, l, G);
    __shared__ double shift;
    if (tid == 0) {
        double tr = 0.0;
        for (int j = 0; j < l; ++j) tr += G[j * l + j];
        shift = 11.0 * ((double)mh * l + (double)l * (l + 1)) * kU * tr;
        if (!(shift > 0.0)) shift = kU;
    }
    __syncthreads();
    block_chol(G, l, shift, 0.0, R, nullptr, &nnull);
    block_trsm(W, mh, mhp, l, R);

    // 4. CholeskyQR with refill of numerically null columns
    int refilled = 0;
    for (int attempt = 0; attempt < 4; ++attempt) {
        block_gram(W, mh, mhp, l, G);
        __shared__ double tol;
        if (tid == 0) {
            double mx = 0.0;
            for (int j = 0; j < l; ++j) mx = fmax(mx, G[j * l + j]);
            tol = 16.0 * l * kU * fmax(mx, 1e-300);
        }
        __syncthreads();
        block_chol(G, l, 0.0, tol, R, null_flags, &nnull);
        if (nnull == 0 || attempt == 3) break;
        // replace null columns by Gaussian directions, unit norm
        for (int j = 0; j < l; ++j) {
            if (!null_flags[j]) continue;
            for (int i = tid; i < mh; i += kThreads) {
                double z0, z1;
                gaussian_pair(seed, counter, (uint32_t)i,
                              kRefillTag | (uint32_t)(attempt * 64 + j), z0, z1);
                W[(size_t)j * mhp + i] = z0;
            }
        }
        __syncthreads();
        for (int j = wave; j < l; j += nw) {
            if (!null_flags[j]) continue;
            double *wj = W + (size_t)j * mhp;
            double s = 0.0;
            for (int i = lane; i < mh; i += kWave) s += wj[i] * wj[i];
            s = wave_sum(s);
            const double inv = 1.0 / sqrt(s);
            for (int i = lane; i < mh; i += kWave) wj[i] *= inv;
        }
        __syncthreads();
        refilled += nnull;
    }
    block_trsm(W, mh, mhp, l, R);
    // 5. final pass
    block_gram(W, mh, mhp, l, G);
    block_chol(G, l, 0.0, 0.0, R, nullptr, &nnull);
    const int final_fail = nnull;
    block_trsm(W, mh, mhp, l, R);

    for (int idx = tid; idx < mh * l; idx += kThreads) {
        const int i = idx % mh, j = idx / mh;
        Q[i + (int64_t)j * ldq] = (T)W[(size_t)j * mhp + i];
    }
    if (tid == 0 && flags) {
        flags[0] = 1;
        flags[1] = refilled;
        flags[2] = final_fail;
    }
}

template <typename T>
hipError_t launch_small_orth(int mh, const T *Qt, int64_t ldqt, int rp, const T *Y, int64_t ldy,
                             int c, T *Q, int64_t ldq, uint64_t seed, uint64_t counter, int *flags,
                             hipStream_t s)
{
    const int l = rp + c;
    const size_t lds = ((size_t)l * (mh | 1) + 2 * (size_t)l * l) * sizeof(double);
    hipLaunchKernelGGL((k_small_orth<T>), dim3(1), dim3(kThreads), lds, s, mh, Qt, ldqt, rp, Y,
                       ldy, c, Q, ldq, seed, counter, flags);
    return hipGetLastError();
}
template hipError_t launch_small_orth<double>(int, const double *, int64_t, int, const double *, int64_t, int, double *, int64_t, uint64_t, uint64_t, int *, hipStream_t);
template hipError_t launch_small_orth<float>(int, const float *, int64_t, int, const float *, int64_t, int, float *, int64_t, uint64_t, uint64_t, int *, hipStream_t);

// ===========================================================================
// Small SVD of B from G = B B^T (Alg. 1 lines 16-18 reformulated):
//   G = R^T R (semidefinite Cholesky), one-sided Jacobi on M = R^T: M V = W S,
//   then B = R^T H^T has left singular vectors U_B = W S^{-1} (the normalised
//   columns) and singular values S.  Round-robin (circle method) pair order;
//   each wavefront rotates one column pair with lane-level dot products
//   reduced across the wavefront.
// ===========================================================================
bool small_svd_fuse_q_ok(int mh, int l) { return (int64_t)mh * l * l <= (int64_t)4 << 20; }

template <int NT>
__device__ int block_jacobi_cols(double *M, int rows, int ld, int n, int max_sweeps, int *sh_rot)
{
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    constexpr int nw = NT / kWave;
    const int n2 = n + (n & 1);  // pad with a dummy column
    const double tol = (double)(rows > 1 ? rows : 1) * 2.0 * kU;
    int sweep;
    for (sweep = 1; sweep <= max_sweeps; ++sweep) {
        if (threadIdx.x == 0) *sh_rot = 0;
        __syncthreads();
        for (int round = 0; round < n2 - 1; ++round) {
            for (int t = wave; t < n2 / 2; t += nw) {
                int p, q;
                if (t == 0) {
                    p = n2 - 1;
                    q = round;
                } else {
                    p = (round + t) % (n2 - 1);
                    q = (round - t + n2 - 1) % (n2 - 1);
                }
                if (p >= n || q >= n) continue;
                if (p > q) {
                    const int tmp = p;
                    p = q;
                    q = tmp;
                }
                double *mp = M + (size_t)p * ld, *mq = M + (size_t)q * ld;
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int i = lane; i < rows; i += kWave) {
                    const double x = mp[i], y = mq[i];
                    al += x * x;
                    be += y * y;
                    ga += x * y;
                }
                al = wave_sum(al);
                be = wave_sum(be);
                ga = wave_sum(ga);
                if (fabs(ga) > tol * sqrt(al * be)) {
                    const double zeta = (be - al) / (2.0 * ga);
                    const double t1 = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
                    const double cs = 1.0 / sqrt(1.0 + t1 * t1);
                    const double sn = cs * t1;
                    for (int i = lane; i < rows; i += kWave) {
                        const double x = mp[i], y = mq[i];
                        mp[i] = cs * x - sn * y;
                        mq[i] = sn * x + cs * y;
                    }
                    if (lane == 0) *sh_rot = 1;
                }
            }
            __syncthreads();
        }
        const int rot = *sh_rot;
        __syncthreads();
        if (!rot) break;
    }
    return sweep;
}

template <typename T, int NT>
__global__ void __launch_bounds__(NT) k_small_svd(int l, const double *Gin, double tau,
                                                  const double *w, const T *Q, int64_t ldq, int mh,
                                                  T *QM, int64_t ldqm, T *Qout, int64_t ldqo,
                                                  SmallSvdOut out, double *work, int fuse_q)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *M = (l <= 80) ? reinterpret_cast<double *>(smem_raw) : work;
    __shared__ int sh_rot;
    __shared__ int order[1024];
    __shared__ double sig[1024];
    const int tid = threadIdx.x;
    const int lane = tid % kWave, wave = tid / kWave;
    constexpr int nw = NT / kWave;

    // Row-major in-place Cholesky: M[j*l + k] = R(j, k), k >= j.  Read as
    // column-major, column j of M is row j of R, i.e. M = R^T.
    for (int idx = tid; idx < l * l; idx += NT) M[idx] = Gin[idx];
    __syncthreads();
    __shared__ double maxdiag;
    if (tid == 0) {
        double mx = 0.0;
        for (int j = 0; j < l; ++j) mx = fmax(mx, M[j * l + j]);
        maxdiag = mx;
    }
    __syncthreads();
    const double ptol = 4.0 * l * kU * maxdiag;
    for (int j = 0; j < l; ++j) {
        __shared__ double piv;
        if (tid == 0) {
            double d = M[j * l + j];
            for (int t = 0; t < j; ++t) d -= M[t * l + j] * M[t * l + j];
            piv = d > ptol ? sqrt(d) : 0.0;
            M[j * l + j] = piv;
        }
        __syncthreads();
        for (int k = j + 1 + tid; k < l; k += NT) {
            double v = 0.0;
            if (piv > 0.0) {
                v = M[j * l + k];
                for (int t = 0; t < j; ++t) v -= M[t * l + j] * M[t * l + k];
                v /= piv;
            }
            M[j * l + k] = v;
        }
        __syncthreads();
    }
    for (int idx = tid; idx < l * l; idx += NT) {
        const int j = idx / l, k = idx % l;
        if (k < j) M[idx] = 0.0;
    }
    __syncthreads();

    const int sweeps = block_jacobi_cols<NT>(M, l, l, l, 60, &sh_rot);

    for (int j = wave; j < l; j += nw) {
        const double *mj = M + (size_t)j * l;
        double s = 0.0;
        for (int i = lane; i < l; i += kWave) s += mj[i] * mj[i];
        s = wave_sum(s);
        if (lane == 0) sig[j] = sqrt(s);
    }
    __syncthreads();
    __shared__ int rank;
    if (tid == 0) {
        for (int j = 0; j < l; ++j) order[j] = j;
        for (int a = 0; a < l; ++a) {
            int best = a;
            for (int b = a + 1; b < l; ++b)
                if (sig[order[b]] > sig[order[best]]) best = b;
            const int tmp = order[a];
            order[a] = order[best];
            order[best] = tmp;
        }
        int r = 0;
        for (int a = 0; a < l; ++a) {
            const double sa = sig[order[a]];
            const double th = w ? w[a] : tau;
            if (sa - th > 0.0) ++r;
        }
        rank = r;
    }
    __syncthreads();
    // U(:, a) = M(:, order[a]) / sigma; sigma sorted
    for (int idx = tid; idx < l * l; idx += NT) {
        const int a = idx / l, i = idx % l;
        const double sa = sig[order[a]];
        out.U[i + (size_t)a * l] = sa > 0.0 ? M[(size_t)order[a] * l + i] / sa : 0.0;
    }
    for (int a = tid; a < l; a += NT) out.sigma[a] = sig[order[a]];
    __syncthreads();
    // Mm = sum_a coef_a u_a u_a^T, coef = f(s)/s
    for (int idx = tid; idx < l * l; idx += NT) {
        const int i = idx % l, j = idx / l;
        double v = 0.0;
        for (int a = 0; a < l; ++a) {
            const double sa = out.sigma[a];
            const double th = w ? w[a] : tau;
            const double f = sa - th;
            if (f > 0.0) v += (f / sa) * out.U[i + (size_t)a * l] * out.U[j + (size_t)a * l];
        }
        out.Mm[i + (size_t)j * l] = v;
    }
    if (tid == 0) {
        out.status[0] = rank;
        out.status[1] = sweeps;
        out.status[2] = sweeps <= 60 ? 1 : 0;
    }
    __syncthreads();
    if (fuse_q && Q) {
        const int r = rank;
        for (int idx = tid; idx < mh * l; idx += NT) {
            const int i = idx % mh, j = idx / mh;
            double v = 0.0;
            for (int t = 0; t < l; ++t) v += (double)Q[i + (int64_t)t * ldq] * out.Mm[t + (size_t)j * l];
            QM[i + (int64_t)j * ldqm] = (T)v;
        }
        if (Qout) {
            for (int idx = tid; idx < mh * r; idx += NT) {
                const int i = idx % mh, j = idx / mh;
                double v = 0.0;
                for (int t = 0; t < l; ++t) v += (double)Q[i + (int64_t)t * ldq] * out.U[t + (size_t)j * l];
                Qout[i + (int64_t)j * ldqo] = (T)v;
            }
        }
    }
}

template <typename T>
hipError_t launch_small_svd(int l, const double *G, double tau, const double *w, const T *Q,
                            int64_t ldq, int mh, T *QM, int64_t ldqm, T *Qout, int64_t ldqo,
                            const SmallSvdOut &out, double *work, int fuse_q, hipStream_t s)
{
    if (l < 1 || l > 1024) return hipErrorInvalidValue;
    const size_t lds = l <= 80 ? (size_t)l * l * sizeof(double) : 0;
    if (l <= 64)
        hipLaunchKernelGGL((k_small_svd<T, 256>), dim3(1), dim3(256), lds, s, l, G, tau, w, Q, ldq, mh, QM, ldqm, Qout, ldqo, out, work, fuse_q);
    else
        hipLaunchKernelGGL((k_small_svd<T, 1024>), dim3(1), dim3(1024), lds, s, l, G, tau, w, Q, ldq, mh, QM, ldqm, Qout, ldqo, out, work, fuse_q);
    return hipGetLastError();
}
template hipError_t launch_small_svd<double>(int, const double *, double, const double *, const double *, int64_t, int, double *, int64_t, double *, int64_t, const SmallSvdOut &, double *, int, hipStream_t);
template hipError_t launch_small_svd<float>(int, const double *, double, const double *, const float *, int64_t, int, float *, int64_t, float *, int64_t, const SmallSvdOut &, double *, int, hipStream_t);

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
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *sG = reinterpret_cast<double *>(smem_raw);
    double *sR = sG + (size_t)l * l;
    __shared__ int nnull;
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
    block_chol(sG, l, shift, tolabs, sR, null_cols, &nnull);
    for (int idx = threadIdx.x; idx < l * l; idx += kThreads) R[idx] = sR[idx];
    if (threadIdx.x == 0 && flags) {
        flags[1] = nnull;
        if (null_tol <= 0.0 && nnull > 0) flags[2] |= 1;
    }
}

hipError_t launch_chol(int l, const double *G, double shift_factor, double null_tol, double *R, int *null_cols, int *flags, hipStream_t s)
{
    const size_t lds = 2 * (size_t)l * l * sizeof(double);
    if (lds > 64 * 1024) return hipErrorInvalidValue;
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
