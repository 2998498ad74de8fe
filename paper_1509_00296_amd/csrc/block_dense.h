// block_dense.h -- workgroup-level dense helpers on LDS-resident matrices
// (Gram, Cholesky with null-pivot detection, triangular solve).
#pragma once
#include "device_common.h"

namespace frk {

// W: l columns of length mh at W[j * mhp + i] (double).  G, R: l x l at
// [a * l + b] (R upper triangular, row-major).

// G = W^T W (full symmetric), one wavefront per (a, b) pair, lanes over rows.
__device__ inline void block_gram(const double *W, int mh, int mhp, int l, double *G)
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

struct CholInfo {
    int nnull;         // pivots treated as numerically null
    double min_ratio;  // min over non-null columns of pivot / (G_jj + shift)
};

// Cholesky of (G + shift I) into the upper triangle of R.  Every thread
// forms the pivot itself from LDS (no broadcast step), so each column costs
// one barrier.  Pivots <= null_tol are numerically null: R_jj = 1, zero row,
// null_flags[j] = 1.
__device__ inline CholInfo block_chol(const double *G, int l, double shift, double null_tol,
                                      double *R, int *null_flags)
{
    const int tid = threadIdx.x;
    for (int idx = tid; idx < l * l; idx += blockDim.x) R[idx] = 0.0;
    __syncthreads();
    CholInfo info{0, 1.0};
    for (int j = 0; j < l; ++j) {
        const double gjj = G[j * l + j] + shift;
        double d = gjj;
        for (int t = 0; t < j; ++t) d -= R[t * l + j] * R[t * l + j];
        const bool isnull = !(d > null_tol);
        const double piv = isnull ? 1.0 : sqrt(d);
        if (isnull) ++info.nnull;
        else if (gjj > 0.0) info.min_ratio = fmin(info.min_ratio, d / gjj);
        if (tid == 0) {
            R[j * l + j] = piv;
            if (null_flags) null_flags[j] = isnull ? 1 : 0;
        }
        if (!isnull) {
            for (int k = j + 1 + tid; k < l; k += blockDim.x) {
                double v = G[j * l + k];
                for (int t = 0; t < j; ++t) v -= R[t * l + j] * R[t * l + k];
                R[j * l + k] = v / piv;
            }
        }
        __syncthreads();
    }
    return info;
}

// W <- W R^{-1} (R upper, row-major), each thread owns rows; for l <= 16 a
// row is held in registers while it is solved.
__device__ inline void block_trsm(double *W, int mh, int mhp, int l, const double *R)
{
    if (l <= 16) {
        for (int i = threadIdx.x; i < mh; i += blockDim.x) {
            double w[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) w[j] = j < l ? W[(size_t)j * mhp + i] : 0.0;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                if (j < l) {
                    double v = w[j];
#pragma unroll
                    for (int t = 0; t < j; ++t) v -= w[t] * R[t * l + j];
                    w[j] = v / R[j * l + j];
                }
            }
#pragma unroll
            for (int j = 0; j < 16; ++j)
                if (j < l) W[(size_t)j * mhp + i] = w[j];
        }
    } else {
        for (int i = threadIdx.x; i < mh; i += blockDim.x) {
            for (int j = 0; j < l; ++j) {
                double v = W[(size_t)j * mhp + i];
                for (int t = 0; t < j; ++t) v -= W[(size_t)t * mhp + i] * R[t * l + j];
                W[(size_t)j * mhp + i] = v / R[j * l + j];
            }
        }
    }
    __syncthreads();
}


// ---------------------------------------------------------------------------
// Fast forms for l <= 16 columns (blockDim = 256, four wavefronts).
// ---------------------------------------------------------------------------
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double bd_doublex4;

// G = W^T W (l <= 16, G row-major [a * l + b]) on the matrix cores: K = rows,
// wavefront w takes the 4-row steps 4w, 4w + 16, ...; A and B operands are
// the same element W(i, a) with a = lane % 16, i = step + lane / 16.  The
// four partial 16 x 16 blocks are added in a fixed order.  part: 4 * 256
// doubles of LDS.  Ends with a barrier.
__device__ inline void gram16_mfma(const double *W, int mh, int mhp, int l, double *G, double *part)
{
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int a = lane & 15, ko = lane >> 4;
    bd_doublex4 z0 = {0, 0, 0, 0}, z1 = {0, 0, 0, 0};
    int i0 = 4 * wave;
    for (; i0 + 16 < mh; i0 += 32) {
        const int i = i0 + ko, i2 = i0 + 16 + ko;
        const double x = (a < l) ? W[(size_t)a * mhp + i] : 0.0;
        const double y = (a < l && i2 < mh) ? W[(size_t)a * mhp + i2] : 0.0;
        z0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x, x, z0, 0, 0, 0);
        z1 = __builtin_amdgcn_mfma_f64_16x16x4f64(y, y, z1, 0, 0, 0);
    }
    if (i0 < mh) {
        const int i = i0 + ko;
        const double x = (a < l && i < mh) ? W[(size_t)a * mhp + i] : 0.0;
        z0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x, x, z0, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) part[wave * 256 + ((lane >> 4) + 4 * r) * 16 + a] = z0[r] + z1[r];
    __syncthreads();
    for (int idx = threadIdx.x; idx < l * l; idx += blockDim.x) {
        const int x = idx / l, y = idx % l;
        const int e = x * 16 + y;
        G[idx] = ((part[e] + part[256 + e]) + part[512 + e]) + part[768 + e];
    }
    __syncthreads();
}

// Cholesky of (G + shift I), l <= 16, by ONE wavefront: lane k holds column
// k of the trailing matrix in registers; each pivot and each row of R is
// broadcast with readlane.  Writes R (upper, row-major [j * l + k], the
// strict lower triangle set to zero) and null_flags; pivots <= null_tol are
// numerically null: a zero row with R_jj = 1 (null_pivot_one) or 0.  G may
// alias R (it is read into registers first).  No barrier inside: call from
// one wavefront, synchronise afterwards.
__device__ inline CholInfo wave_chol16(const double *G, int l, double shift, double null_tol,
                                       double *R, int *null_flags, bool null_pivot_one = true)
{
    const int k = threadIdx.x % kWave;
    double g[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) g[i] = (i < l && k < l) ? G[i * l + k] + (i == k ? shift : 0.0) : 0.0;
    double gkk = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i)
        if (i == k) gkk = g[i];
    CholInfo info{0, 1.0};
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if (j >= l) break;
        double gj = 0.0;   // this lane's element j of its column: G'(j, k)
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (i == j) gj = g[i];
        const double d = read_lane(gj, j);
        const double ojj = read_lane(gkk, j);
        const bool isnull = !(d > null_tol);
        const double piv = isnull ? (null_pivot_one ? 1.0 : 0.0) : sqrt(d);
        if (isnull) ++info.nnull;
        else if (ojj > 0.0) info.min_ratio = fmin(info.min_ratio, d / ojj);
        const double inv = isnull ? 0.0 : 1.0 / piv;
        double rjk = 0.0;
        if (k == j) rjk = piv;
        else if (k > j && k < l && !isnull) rjk = gj * inv;
        if (k < l) R[j * l + k] = rjk;
        if (k == 0 && null_flags) null_flags[j] = isnull ? 1 : 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (i > j && i < l) {
                const double rji = read_lane(rjk, i);
                if (k > j) g[i] -= rji * rjk;
            }
        }
    }
    return info;
}

}  // namespace frk
