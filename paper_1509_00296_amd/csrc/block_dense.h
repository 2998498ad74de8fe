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

}  // namespace frk
