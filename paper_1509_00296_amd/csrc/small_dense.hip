// small_dense.hip -- one-workgroup dense kernels: CholeskyQR
// re-orthonormalisation of the sampled basis (Alg. 1: the fresh sketch's QR,
// range propagation's partial orthogonalisation, the power-iteration QR) and
// the small SVD of B with thresholds and reconstruction factors (its
// projection, polar/eigen and reconstruction steps).
#include "block_dense.h"
#include "device_common.h"
#include "internal.h"

#include <algorithm>

namespace frk {

// ===========================================================================
// Orthonormalisation of W = [Qt, Y] (mh x l, l = rp + c), all in LDS:
//   1. CGS2: Y <- Y - Qt (Qt^T Y), twice (the partial orthogonalisation of
//      range propagation's partial orthogonalisation in Alg. 1).
//   2. Column equilibration (only the span matters).
//   3. Fast path: CholeskyQR2.  The first Cholesky must see no null pivot
//      and a smallest pivot ratio >= 1e-8; the second must have every pivot
//      within 1e-6 of 1 (W^T W ~ I).  Otherwise:
//   4. Fallback from the saved equilibrated W: shifted CholeskyQR with
//      shift 11 (mh l + l(l+1)) u trace(W^T W) (shifted CholeskyQR3 of
//      Fukaya et al.), then CholeskyQR passes in which numerically null
//      columns are replaced by fresh Gaussian directions (any orthonormal
//      completion leaves the thresholded result unchanged), then a final
//      CholeskyQR pass.
// flags: [0] 1 = fast path, 2 = fallback; [1] refilled columns; [2] final
// pass failures.
// ===========================================================================
bool small_orth_ok(int mh, int l)
{
    // W, its saved copy, G, R and the matrix-core Gram partials (4 x 256
    // doubles, 4 x 768 for 16 < l <= 32)
    return l >= 1 && l <= 64 &&
           (size_t)(mh | 1) * l * 16 + (size_t)l * l * 16 + (l > 16 && l <= 32 ? 24576 : 8192) <= 96 * 1024;
}

// Step 4 of the orthonormalisation, from the equilibrated basis in W (LDS,
// all NT threads): shifted CholeskyQR, refill of numerically null columns,
// and a final CholeskyQR pass.  Ends with a barrier.
__device__ __forceinline__ void orth_fallback(double *W, double *G, double *R, int *null_flags, int mh, int mhp,
                                              int l, uint64_t seed, uint64_t counter, int &refilled,
                                              int &final_fail)
{
    const int tid = threadIdx.x, NT = blockDim.x;
    const int lane = tid % kWave, wave = tid / kWave, nw = NT / kWave;
    block_gram(W, mh, mhp, l, G);
    double tr = 0.0;
    for (int j = 0; j < l; ++j) tr += G[j * l + j];
    double shift = 11.0 * ((double)mh * l + (double)l * (l + 1)) * kU * tr;
    if (!(shift > 0.0)) shift = kU;
    block_chol(G, l, shift, 0.0, R, nullptr);
    block_trsm(W, mh, mhp, l, R);
    for (int attempt = 0; attempt < 4; ++attempt) {
        block_gram(W, mh, mhp, l, G);
        double mxd = 0.0;
        for (int j = 0; j < l; ++j) mxd = fmax(mxd, G[j * l + j]);
        const CholInfo ci = block_chol(G, l, 0.0, 16.0 * l * kU * fmax(mxd, 1e-300), R, null_flags);
        if (ci.nnull == 0 || attempt == 3) break;
        for (int j = 0; j < l; ++j) {
            if (!null_flags[j]) continue;
            for (int i = tid; i < mh; i += NT) {
                double z0, z1;
                gaussian_pair(seed, counter, (uint32_t)i, kRefillTag | (uint32_t)(attempt * 64 + j), z0, z1);
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
        refilled += ci.nnull;
    }
    block_trsm(W, mh, mhp, l, R);
    block_gram(W, mh, mhp, l, G);
    final_fail = block_chol(G, l, 0.0, 0.0, R, nullptr).nnull;
    block_trsm(W, mh, mhp, l, R);
}

// LC > 0 fixes the width l = rp + c at compile time (see k_small_orth8).
template <typename T, int NT, int LM, int LC = 0>
__global__ void __launch_bounds__(NT) k_small_orth(int mh, const T *Qt, int64_t ldqt, int rp,
                                                   const T *Y, int64_t ldy, int c, T *Q,
                                                   int64_t ldq, uint64_t seed, uint64_t counter,
                                                   int *flags, double *resid2)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int l = LC > 0 ? LC : rp + c;
    const int mhp = mh | 1;
    double *W = reinterpret_cast<double *>(smem_raw);
    double *W0 = W + (size_t)l * mhp;
    double *G = W0 + (size_t)l * mhp;
    double *R = G + (size_t)l * l;
    __shared__ int null_flags[64];
    __shared__ double scal[64];
    const int tid = threadIdx.x;
    const int lane = tid % kWave, wave = tid / kWave;
    constexpr int nw = NT / kWave;

    for (int idx = tid; idx < mh * rp; idx += NT) {
        const int i = idx % mh, j = idx / mh;
        W[(size_t)j * mhp + i] = (double)Qt[i + (int64_t)j * ldqt];
    }
    for (int idx = tid; idx < mh * c; idx += NT) {
        const int i = idx % mh, j = idx / mh;
        W[(size_t)(rp + j) * mhp + i] = (double)Y[i + (int64_t)j * ldy];
    }
    __syncthreads();

    __shared__ int sh_info[2];
    __shared__ double sh_ratio[2];
    bool fast = true;
    if (l <= LM && NT == 256) {
        // ---- l <= LM (8, 16 or 32): Grams on the matrix cores, Cholesky in one wavefront
        double *part = R + (size_t)l * l;
        // 1. CGS2: coefficients from the Qt-Y block of the Gram of [Qt, Y]
        if (rp > 0 && c > 0) {
            for (int pass = 0; pass < 2; ++pass) {
                gram_mfma<LM>(W, mh, mhp, l, G, part);
                for (int i = tid; i < mh; i += NT) {
                    double qt[LM];
#pragma unroll
                    for (int t = 0; t < LM; ++t) qt[t] = t < rp ? W[(size_t)t * mhp + i] : 0.0;
                    for (int j = 0; j < c; ++j) {
                        double v = W[(size_t)(rp + j) * mhp + i];
#pragma unroll
                        for (int t = 0; t < LM; ++t)
                            if (t < rp) v -= qt[t] * G[t * l + rp + j];
                        W[(size_t)(rp + j) * mhp + i] = v;
                    }
                }
                __syncthreads();
            }
        }
        // 2. equilibration from the Gram's diagonal; the Gram of the scaled
        //    basis is the scaled Gram
        gram_mfma<LM>(W, mh, mhp, l, G, part);
        // the first new column's squared residual against Qt (its norm when
        // nothing is propagated): Prop. 4's by-product
        if (resid2 && tid == 0) *resid2 = c > 0 ? G[rp * l + rp] : -1.0;
        for (int j = tid; j < l; j += NT) {
            const double d = G[j * l + j];
            scal[j] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
        }
        __syncthreads();
        for (int idx = tid; idx < mh * l; idx += NT) {
            const int i = idx % mh, j = idx / mh;
            const double v = W[(size_t)j * mhp + i] * scal[j];
            W[(size_t)j * mhp + i] = v;
            W0[(size_t)j * mhp + i] = v;
        }
        for (int idx = tid; idx < l * l; idx += NT) G[idx] *= scal[idx / l] * scal[idx % l];
        __syncthreads();
        // 3. CholeskyQR2
        double mx = 0.0;
        for (int j = 0; j < l; ++j) mx = fmax(mx, G[j * l + j]);
        if (wave == 0) {
            const CholInfo c1 = wave_chol16<LM>(G, l, 0.0, 16.0 * l * kU * fmax(mx, 1e-300), R, nullptr);
            if (lane == 0) {
                sh_info[0] = c1.nnull;
                sh_ratio[0] = c1.min_ratio;
            }
        }
        __syncthreads();
        if (sh_info[0] > 0 || sh_ratio[0] < 1e-8) fast = false;
        if (fast) {
            block_trsm<LM>(W, mh, mhp, l, R);
            gram_mfma<LM>(W, mh, mhp, l, G, part);
            if (wave == 0) {
                const CholInfo c2 = wave_chol16<LM>(G, l, 0.0, 0.5, R, nullptr);
                if (lane == 0) sh_info[1] = c2.nnull;
            }
            __syncthreads();
            bool near_one = sh_info[1] == 0;
            for (int j = 0; j < l && near_one; ++j) near_one = fabs(R[j * l + j] - 1.0) <= 1e-6;
            if (near_one) block_trsm<LM>(W, mh, mhp, l, R);
            else fast = false;
        }
    } else {
        // 1. CGS2 against the propagated basis
        if (rp > 0 && c > 0) {
            for (int pass = 0; pass < 2; ++pass) {
                for (int p = wave; p < rp * c; p += nw) {
                    const int t = p % rp, j = p / rp;
                    const double *qa = W + (size_t)t * mhp, *ya = W + (size_t)(rp + j) * mhp;
                    double s = 0.0;
                    for (int i = lane; i < mh; i += kWave) s += qa[i] * ya[i];
                    s = wave_sum(s);
                    if (lane == 0) G[t * c + j] = s;
                }
                __syncthreads();
                for (int idx = tid; idx < mh * c; idx += NT) {
                    const int i = idx % mh, j = idx / mh;
                    double v = W[(size_t)(rp + j) * mhp + i];
                    for (int t = 0; t < rp; ++t) v -= W[(size_t)t * mhp + i] * G[t * c + j];
                    W[(size_t)(rp + j) * mhp + i] = v;
                }
                __syncthreads();
            }
        }
        // 2. column equilibration, and a saved copy for the fallback
        for (int j = wave; j < l; j += nw) {
            const double *wj = W + (size_t)j * mhp;
            double s = 0.0;
            for (int i = lane; i < mh; i += kWave) s += wj[i] * wj[i];
            s = wave_sum(s);
            if (lane == 0) {
                scal[j] = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
                if (resid2 && j == rp) *resid2 = s;
            }
        }
        if (resid2 && c == 0 && tid == 0) *resid2 = -1.0;
        __syncthreads();
        for (int idx = tid; idx < mh * l; idx += NT) {
            const int i = idx % mh, j = idx / mh;
            const double v = W[(size_t)j * mhp + i] * scal[j];
            W[(size_t)j * mhp + i] = v;
            W0[(size_t)j * mhp + i] = v;
        }
        __syncthreads();

        // 3. fast path: CholeskyQR2
        block_gram(W, mh, mhp, l, G);
        double mx = 0.0;
        for (int j = 0; j < l; ++j) mx = fmax(mx, G[j * l + j]);
        const CholInfo c1 = block_chol(G, l, 0.0, 16.0 * l * kU * fmax(mx, 1e-300), R, nullptr);
        if (c1.nnull > 0 || c1.min_ratio < 1e-8) fast = false;
        if (fast) {
            block_trsm(W, mh, mhp, l, R);
            block_gram(W, mh, mhp, l, G);
            const CholInfo c2 = block_chol(G, l, 0.0, 0.5, R, nullptr);
            bool near_one = c2.nnull == 0;
            for (int j = 0; j < l && near_one; ++j) near_one = fabs(R[j * l + j] - 1.0) <= 1e-6;
            if (near_one) block_trsm(W, mh, mhp, l, R);
            else fast = false;
        }
    }
    int refilled = 0, final_fail = 0;
    if (!fast) {
        // 4. fallback from the saved equilibrated basis
        for (int idx = tid; idx < mh * l; idx += NT) {
            const int i = idx % mh, j = idx / mh;
            W[(size_t)j * mhp + i] = W0[(size_t)j * mhp + i];
        }
        __syncthreads();
        orth_fallback(W, G, R, null_flags, mh, mhp, l, seed, counter, refilled, final_fail);
    }

    for (int idx = tid; idx < mh * l; idx += NT) {
        const int i = idx % mh, j = idx / mh;
        Q[i + (int64_t)j * ldq] = (T)W[(size_t)j * mhp + i];
    }
    if (tid == 0 && flags) {
        flags[0] = fast ? 1 : 2;
        flags[1] = refilled;
        flags[2] = final_fail;
    }
}

// l <= 8 and mh <= 256 RPT: the same steps with the rows of W in registers
// (thread t owns rows t + 256 k, k < RPT).  The Grams run on the matrix cores
// from an LDS copy of W (gram16_mfma); every thread then reads the l x l Gram
// and factors it itself (reg_chol: the same arithmetic in every thread, so
// no broadcast step and no barrier for the factor), and solves its own rows
// with the reciprocal pivots.  The fallback (step 4) runs from LDS.  LC > 0
// fixes the width l = rp + c at compile time: the kernel runs once per launch
// from a cold instruction cache, and a fixed width removes the guards and
// address arithmetic of the unrolled loops from the straight-line code.
template <typename T, int RPT, int LC = 0>
__global__ void __launch_bounds__(256) k_small_orth8(int mh, const T *Qt, int64_t ldqt, int rp, const T *Y,
                                                     int64_t ldy, int c, T *Q, int64_t ldq, uint64_t seed,
                                                     uint64_t counter, int *flags, double *resid2)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int l = LC > 0 ? LC : rp + c;
    const int mhp = mh | 1;
    double *W = reinterpret_cast<double *>(smem_raw);
    double *W0 = W + (size_t)l * mhp;
    double *G = W0 + (size_t)l * mhp;
    double *R = G + (size_t)l * l;
    double *part = R + (size_t)l * l;
    __shared__ int null_flags[64];
    const int tid = threadIdx.x;

    // every load of the thread's rows issued before the first use
    double w[RPT][8];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int i = tid + 256 * k;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            double v = 0.0;
            if (i < mh && j < l) v = j < rp ? (double)Qt[i + (int64_t)j * ldqt] : (double)Y[i + (int64_t)(j - rp) * ldy];
            w[k][j] = v;
        }
    }
    auto put = [&](int j0) {
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int i = tid + 256 * k;
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (i < mh && j >= j0 && j < l) W[(size_t)j * mhp + i] = w[k][j];
        }
    };
    put(0);
    __syncthreads();

    // 1. CGS2 against the propagated basis: Y <- Y - Qt C, C = Qt^T Y (the
    //    Qt-Y block of the Gram of [Qt, Y])
    if (rp > 0 && c > 0) {
        for (int pass = 0; pass < 2; ++pass) {
            gram16_mfma(W, mh, mhp, l, G, part);
            double cf[8][8];
#pragma unroll
            for (int t = 0; t < 8; ++t)
#pragma unroll
                for (int j = 0; j < 8; ++j) cf[t][j] = (t < rp && j >= rp && j < l) ? G[t * l + j] : 0.0;
#pragma unroll
            for (int k = 0; k < RPT; ++k)
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    if (j >= rp && j < l) {
                        double v = w[k][j];
#pragma unroll
                        for (int t = 0; t < 8; ++t)
                            if (t < rp) v -= w[k][t] * cf[t][j];
                        w[k][j] = v;
                    }
                }
            put(rp);
            __syncthreads();
        }
    }
    // 2. equilibration from the Gram's diagonal; the Gram of the scaled basis
    //    is the scaled Gram
    gram16_mfma(W, mh, mhp, l, G, part);
    if (resid2 && tid == 0) *resid2 = c > 0 ? G[rp * l + rp] : -1.0;
    double sc[8], g[8][8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const double d = j < l ? G[j * l + j] : 0.0;
        sc[j] = d > 0.0 ? rsqrt_pos(d) : 0.0;
    }
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b) g[a][b] = (b >= a && b < l) ? G[a * l + b] * (sc[a] * sc[b]) : 0.0;
    double w0[RPT][8];
#pragma unroll
    for (int k = 0; k < RPT; ++k)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            w[k][j] *= sc[j];
            w0[k][j] = w[k][j];
        }
    // 3. CholeskyQR2
    double mx = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (j < l) mx = fmax(mx, g[j][j]);
    double rinv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) rinv[j] = 0.0;
    const CholInfo c1 = reg_chol<8>(g, l, 16.0 * l * kU * fmax(mx, 1e-300), 1.0, 1e-8, rinv);
    bool fast = c1.nnull == 0 && c1.min_ratio > 0.0;
    if (fast) {
#pragma unroll
        for (int k = 0; k < RPT; ++k) reg_trsm_row<8>(w[k], g, rinv, l);
        put(0);
        __syncthreads();
        gram16_mfma(W, mh, mhp, l, G, part);
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int b = 0; b < 8; ++b) g[a][b] = (b >= a && b < l) ? G[a * l + b] : 0.0;
        const CholInfo c2 = reg_chol<8>(g, l, 0.5, 1.0, 0.0, rinv);
        bool near_one = c2.nnull == 0;
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (j < l) near_one = near_one && fabs(g[j][j] - 1.0) <= 1e-6;
        if (near_one) {
#pragma unroll
            for (int k = 0; k < RPT; ++k) reg_trsm_row<8>(w[k], g, rinv, l);
        } else {
            fast = false;
        }
    }
    int refilled = 0, final_fail = 0;
    if (!fast) {
        // 4. fallback from the saved equilibrated basis, in LDS
        __syncthreads();
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int i = tid + 256 * k;
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (i < mh && j < l) W[(size_t)j * mhp + i] = w0[k][j];
        }
        __syncthreads();
        orth_fallback(W, G, R, null_flags, mh, mhp, l, seed, counter, refilled, final_fail);
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int i = tid + 256 * k;
#pragma unroll
            for (int j = 0; j < 8; ++j) w[k][j] = (i < mh && j < l) ? W[(size_t)j * mhp + i] : 0.0;
        }
    }
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        const int i = tid + 256 * k;
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (i < mh && j < l) Q[i + (int64_t)j * ldq] = (T)w[k][j];
    }
    if (tid == 0 && flags) {
        flags[0] = fast ? 1 : 2;
        flags[1] = refilled;
        flags[2] = final_fail;
    }
}

template <typename T>
hipError_t launch_small_orth(int mh, const T *Qt, int64_t ldqt, int rp, const T *Y, int64_t ldy,
                             int c, T *Q, int64_t ldq, uint64_t seed, uint64_t counter, int *flags,
                             double *resid2, hipStream_t s)
{
    const int l = rp + c;
    if (!small_orth_ok(mh, l)) return hipErrorInvalidValue;
    const size_t lds =
        (2 * (size_t)l * (mh | 1) + 2 * (size_t)l * l + (l > 16 && l <= 32 ? 4 * 768 : 4 * 256)) * sizeof(double);
    if (l <= 8 && mh <= 256) {
        switch (l) {
#define FRK_ORTH8_CASE(L)                                                                                    \
    case L:                                                                                                  \
        hipLaunchKernelGGL((k_small_orth8<T, 1, L>), dim3(1), dim3(256), lds, s, mh, Qt, ldqt, rp, Y, ldy, c, \
                           Q, ldq, seed, counter, flags, resid2);                                            \
        break;
            FRK_ORTH8_CASE(1) FRK_ORTH8_CASE(2) FRK_ORTH8_CASE(3) FRK_ORTH8_CASE(4)
            FRK_ORTH8_CASE(5) FRK_ORTH8_CASE(6) FRK_ORTH8_CASE(7) FRK_ORTH8_CASE(8)
#undef FRK_ORTH8_CASE
        default: return hipErrorInvalidValue;
        }
    } else if (l <= 8 && mh <= 512)
        hipLaunchKernelGGL((k_small_orth8<T, 2>), dim3(1), dim3(256), lds, s, mh, Qt, ldqt, rp, Y, ldy, c, Q,
                           ldq, seed, counter, flags, resid2);
    else if (l <= 8)
        hipLaunchKernelGGL((k_small_orth<T, 256, 8>), dim3(1), dim3(256), lds, s, mh, Qt, ldqt, rp, Y,
                           ldy, c, Q, ldq, seed, counter, flags, resid2);
    else if (l <= 16) {
        switch (l) {
#define FRK_ORTH16_CASE(L)                                                                                    \
    case L:                                                                                                   \
        hipLaunchKernelGGL((k_small_orth<T, 256, 16, L>), dim3(1), dim3(256), lds, s, mh, Qt, ldqt, rp, Y, ldy, \
                           c, Q, ldq, seed, counter, flags, resid2);                                          \
        break;
            FRK_ORTH16_CASE(9) FRK_ORTH16_CASE(10) FRK_ORTH16_CASE(11) FRK_ORTH16_CASE(12)
            FRK_ORTH16_CASE(13) FRK_ORTH16_CASE(14) FRK_ORTH16_CASE(15) FRK_ORTH16_CASE(16)
#undef FRK_ORTH16_CASE
        }
    }
    else {
        switch (l) {
#define FRK_ORTH32_CASE(L)                                                                                    \
    case L:                                                                                                   \
        hipLaunchKernelGGL((k_small_orth<T, 256, 32, L>), dim3(1), dim3(256), lds, s, mh, Qt, ldqt, rp, Y, ldy, \
                           c, Q, ldq, seed, counter, flags, resid2);                                          \
        break;
            FRK_ORTH32_CASE(17) FRK_ORTH32_CASE(18) FRK_ORTH32_CASE(19) FRK_ORTH32_CASE(20)
            FRK_ORTH32_CASE(21) FRK_ORTH32_CASE(22) FRK_ORTH32_CASE(23) FRK_ORTH32_CASE(24)
            FRK_ORTH32_CASE(25) FRK_ORTH32_CASE(26) FRK_ORTH32_CASE(27) FRK_ORTH32_CASE(28)
            FRK_ORTH32_CASE(29) FRK_ORTH32_CASE(30) FRK_ORTH32_CASE(31) FRK_ORTH32_CASE(32)
#undef FRK_ORTH32_CASE
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}
template hipError_t launch_small_orth<double>(int, const double *, int64_t, int, const double *, int64_t, int, double *, int64_t, uint64_t, uint64_t, int *, double *, hipStream_t);
template hipError_t launch_small_orth<float>(int, const float *, int64_t, int, const float *, int64_t, int, float *, int64_t, uint64_t, uint64_t, int *, double *, hipStream_t);

// ---------------------------------------------------------------------------
// Prop. 4's residual where the basis is orthonormalised without an explicit
// Gram-Schmidt step (the large path): column rp of Q (the first new sample)
// against columns 0 .. rp-1 (the propagated basis), two classical
// Gram-Schmidt passes; the squared norm goes to out, -1 without a new
// sample.  Wavefront w forms the inner products of columns w, w + 4, ...
// (lanes over rows), then every thread updates its rows.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_resid_est(int mh, const T *Q, int64_t ldq, int rp, int c, double *out)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *y = reinterpret_cast<double *>(smem_raw);
    double *d = y + mh;
    __shared__ double red[4];
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    if (c <= 0) {
        if (tid == 0) *out = -1.0;
        return;
    }
    for (int i = tid; i < mh; i += 256) y[i] = (double)Q[i + (int64_t)rp * ldq];
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
        for (int t = wave; t < rp; t += 4) {
            double s = 0.0;
            for (int i = lane; i < mh; i += kWave) s += (double)Q[i + (int64_t)t * ldq] * y[i];
            s = wave_sum(s);
            if (lane == 0) d[t] = s;
        }
        __syncthreads();
        for (int i = tid; i < mh; i += 256) {
            double v = y[i];
            for (int t = 0; t < rp; ++t) v -= (double)Q[i + (int64_t)t * ldq] * d[t];
            y[i] = v;
        }
        __syncthreads();
    }
    double s = 0.0;
    for (int i = tid; i < mh; i += 256) s += y[i] * y[i];
    s = wave_sum(s);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    if (tid == 0) *out = ((red[0] + red[1]) + red[2]) + red[3];
}

template <typename T>
hipError_t launch_resid_est(int mh, const T *Q, int64_t ldq, int rp, int c, double *out, hipStream_t s)
{
    const size_t lds = ((size_t)mh + (size_t)std::max(rp, 1)) * sizeof(double);
    if (mh < 1 || rp < 0 || ldq < mh || lds > 64 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_resid_est<T>), dim3(1), dim3(256), lds, s, mh, Q, ldq, rp, c, out);
    return hipGetLastError();
}
template hipError_t launch_resid_est<double>(int, const double *, int64_t, int, int, double *, hipStream_t);
template hipError_t launch_resid_est<float>(int, const float *, int64_t, int, int, double *, hipStream_t);

// ===========================================================================
// Sequential residual check (Sec. 3.2 after Prop. 4): the new samples
// y_1..y_c (columns of Y) taken in order, each projected off the basis it
// would extend, [Qt, q_1, ..., q_{j-1}] (Qt: rp orthonormal columns; q_i the
// normalised residuals of the earlier samples), by classical Gram-Schmidt
// applied twice.  out[j] = ||residual of y_{j+1}||^2; a zero residual adds
// no basis column.  One workgroup; the new basis columns stay in LDS.
// ===========================================================================
template <typename T>
__global__ void __launch_bounds__(256) k_resid_seq(int mh, const T *Qt, int64_t ldqt, int rp, const T *Y,
                                                   int64_t ldy, int c, double *out)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *y = reinterpret_cast<double *>(smem_raw);
    double *B = y + mh;                       // mh x c new basis columns
    double *d = B + (size_t)mh * c;           // rp + c coefficients
    __shared__ double red[4];
    __shared__ int nb_sh;
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    if (tid == 0) nb_sh = 0;
    for (int j = 0; j < c; ++j) {
        __syncthreads();
        const int nb = nb_sh;
        for (int i = tid; i < mh; i += 256) y[i] = (double)Y[i + (int64_t)j * ldy];
        __syncthreads();
        for (int pass = 0; pass < 2; ++pass) {
            // all coefficients of this pass from the same y (classical Gram-Schmidt)
            for (int t = wave; t < rp + nb; t += 4) {
                double s = 0.0;
                if (t < rp)
                    for (int i = lane; i < mh; i += kWave) s += (double)Qt[i + (int64_t)t * ldqt] * y[i];
                else
                    for (int i = lane; i < mh; i += kWave) s += B[(size_t)(t - rp) * mh + i] * y[i];
                s = wave_sum(s);
                if (lane == 0) d[t] = s;
            }
            __syncthreads();
            for (int i = tid; i < mh; i += 256) {
                double v = y[i];
                for (int t = 0; t < rp; ++t) v -= (double)Qt[i + (int64_t)t * ldqt] * d[t];
                for (int t = 0; t < nb; ++t) v -= B[(size_t)t * mh + i] * d[rp + t];
                y[i] = v;
            }
            __syncthreads();
        }
        double s = 0.0;
        for (int i = tid; i < mh; i += 256) s += y[i] * y[i];
        s = wave_sum(s);
        if (lane == 0) red[wave] = s;
        __syncthreads();
        const double nrm2 = ((red[0] + red[1]) + red[2]) + red[3];
        if (tid == 0) out[j] = nrm2;
        if (nrm2 > 0.0) {
            const double inv = 1.0 / sqrt(nrm2);
            for (int i = tid; i < mh; i += 256) B[(size_t)nb * mh + i] = y[i] * inv;
            if (tid == 0) nb_sh = nb + 1;
        }
    }
}

bool resid_seq_ok(int mh, int rp, int c)
{
    return mh >= 1 && rp >= 0 && c >= 1 &&
           ((size_t)mh * (c + 1) + (size_t)(rp + c + 1)) * sizeof(double) <= 64 * 1024;
}

template <typename T>
hipError_t launch_resid_seq(int mh, const T *Qt, int64_t ldqt, int rp, const T *Y, int64_t ldy, int c,
                            double *out, hipStream_t s)
{
    const size_t lds = ((size_t)mh * (c + 1) + (size_t)(rp + c + 1)) * sizeof(double);
    if (!resid_seq_ok(mh, rp, c) || ldy < mh || (rp > 0 && ldqt < mh)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_resid_seq<T>), dim3(1), dim3(256), lds, s, mh, Qt, ldqt, rp, Y, ldy, c, out);
    return hipGetLastError();
}
template hipError_t launch_resid_seq<double>(int, const double *, int64_t, int, const double *, int64_t, int,
                                             double *, hipStream_t);
template hipError_t launch_resid_seq<float>(int, const float *, int64_t, int, const float *, int64_t, int,
                                            double *, hipStream_t);

// ===========================================================================
// Rank truncation of a fresh sketch by QR with column pivoting (Alg. 1's
// QR_CP of the sampled matrix; Sec. 2.1's real sampling rate s = min(l, r)):
// Householder QR of Y (mh x c) where step j moves the remaining column of
// largest norm (recomputed from the rows j.. of the reduced matrix) to
// position j.  s = the number of leading |R_jj| above tol_factor |R_00|;
// the first s pivoted columns of Y (whose span is that of QR_CP's Q_s) are
// written to Yout in pivot order, and s to *s_out.  One workgroup, Y in LDS.
// ===========================================================================
template <typename T>
__global__ void __launch_bounds__(256) k_qrcp_trunc(int mh, int c, const T *Y, int64_t ldy, double tol_factor,
                                                    T *Yout, int64_t ldo, int *s_out)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int mhp = mh | 1;
    double *W = reinterpret_cast<double *>(smem_raw);   // mh x c, ld mhp
    __shared__ double cn[64];
    __shared__ double rdiag[64];
    __shared__ int perm[64];
    __shared__ double sh_beta, sh_scale;
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    for (int idx = tid; idx < mh * c; idx += 256) {
        const int i = idx % mh, j = idx / mh;
        W[(size_t)j * mhp + i] = (double)Y[i + (int64_t)j * ldy];
    }
    for (int j = tid; j < c; j += 256) perm[j] = j;
    __syncthreads();
    const int kmax = mh < c ? mh : c;
    for (int j = 0; j < kmax; ++j) {
        // norms of the remaining parts of columns j..c-1
        for (int col = j + wave; col < c; col += 4) {
            double s = 0.0;
            for (int i = j + lane; i < mh; i += kWave) {
                const double v = W[(size_t)col * mhp + i];
                s += v * v;
            }
            s = wave_sum(s);
            if (lane == 0) cn[col] = s;
        }
        __syncthreads();
        int best = j;
        double bn = cn[j];
        for (int col = j + 1; col < c; ++col)
            if (cn[col] > bn) {
                bn = cn[col];
                best = col;
            }
        if (best != j) {
            for (int i = tid; i < mh; i += 256) {
                const double t = W[(size_t)j * mhp + i];
                W[(size_t)j * mhp + i] = W[(size_t)best * mhp + i];
                W[(size_t)best * mhp + i] = t;
            }
            if (tid == 0) {
                const int t = perm[j];
                perm[j] = perm[best];
                perm[best] = t;
            }
        }
        __syncthreads();
        // Householder reflector of W(j:, j): v = x - alpha e1, alpha = -sign(x0) ||x||
        if (tid == 0) {
            const double nrm = sqrt(bn);
            const double x0 = W[(size_t)j * mhp + j];
            const double alpha = x0 >= 0.0 ? -nrm : nrm;
            const double v0 = x0 - alpha;
            // v scaled so that v0 = 1; beta = -v0 / alpha
            sh_beta = nrm > 0.0 ? -v0 / alpha : 0.0;
            sh_scale = (nrm > 0.0 && v0 != 0.0) ? 1.0 / v0 : 0.0;
            rdiag[j] = nrm > 0.0 ? alpha : 0.0;
        }
        __syncthreads();
        const double beta = sh_beta, scale = sh_scale;
        for (int i = j + 1 + tid; i < mh; i += 256) W[(size_t)j * mhp + i] *= scale;
        __syncthreads();
        // apply (I - beta v v^T) to columns j+1..c-1, v = [1, W(j+1:, j)]
        for (int col = j + 1 + wave; col < c; col += 4) {
            double s = lane == 0 ? W[(size_t)col * mhp + j] : 0.0;
            for (int i = j + 1 + lane; i < mh; i += kWave) s += W[(size_t)j * mhp + i] * W[(size_t)col * mhp + i];
            s = wave_sum(s);
            const double f = beta * s;
            if (lane == 0) W[(size_t)col * mhp + j] -= f;
            for (int i = j + 1 + lane; i < mh; i += kWave) W[(size_t)col * mhp + i] -= f * W[(size_t)j * mhp + i];
        }
        __syncthreads();
    }
    __shared__ int s_sh;
    if (tid == 0) {
        const double r00 = kmax > 0 ? fabs(rdiag[0]) : 0.0;
        const double tol = tol_factor * r00;
        int s = 0;
        while (s < kmax && fabs(rdiag[s]) > tol) ++s;
        s_sh = s;
        *s_out = s;
    }
    __syncthreads();
    const int s = s_sh;
    for (int idx = tid; idx < mh * s; idx += 256) {
        const int i = idx % mh, j = idx / mh;
        Yout[i + (int64_t)j * ldo] = Y[i + (int64_t)perm[j] * ldy];
    }
}

bool qrcp_trunc_ok(int mh, int c) { return c >= 1 && c <= 64 && (size_t)(mh | 1) * c * sizeof(double) <= 128 * 1024; }

template <typename T>
hipError_t launch_qrcp_trunc(int mh, int c, const T *Y, int64_t ldy, double tol_factor, T *Yout, int64_t ldo,
                             int *s_out, hipStream_t s)
{
    if (!qrcp_trunc_ok(mh, c) || ldy < mh || ldo < mh) return hipErrorInvalidValue;
    const size_t lds = (size_t)(mh | 1) * c * sizeof(double);
    hipLaunchKernelGGL((k_qrcp_trunc<T>), dim3(1), dim3(256), lds, s, mh, c, Y, ldy, tol_factor, Yout, ldo, s_out);
    return hipGetLastError();
}
template hipError_t launch_qrcp_trunc<double>(int, int, const double *, int64_t, double, double *, int64_t, int *,
                                              hipStream_t);
template hipError_t launch_qrcp_trunc<float>(int, int, const float *, int64_t, double, float *, int64_t, int *,
                                             hipStream_t);


// ===========================================================================
// Small SVD of B from G = B B^T (Alg. 1's QR of A^T Q, polar and eigen steps reformulated):
//   G = R^T R (semidefinite Cholesky), one-sided Jacobi on M = R^T: M V = W S.
//   B = R^T H^T has left singular vectors U_B = W S^{-1} (the normalised
//   columns of the converged M) and singular values S.
// Pairs follow the circle method (n - 1 rounds of n/2 disjoint pairs).  A
// pair is rotated when |m_p.m_q| > rows u' sqrt(|m_p|^2 |m_q|^2).
//
// Two Jacobi engines:
//   l <= 16: one wavefront; four groups of 16 lanes each rotate one pair,
//            lane = row, with 16-lane shuffle reductions (no barriers
//            between the rotations of a step beyond the wavefront's own).
//   l > 16 : groups of 16 lanes (64 beyond l = 256), one pair per group,
//            rows in registers, one block barrier per round.
// ===========================================================================
bool small_svd_fuse_q_ok(int mh, int l) { return mh >= 1 && l >= 1 && 2 * (size_t)l * l * sizeof(double) <= 96 * 1024; }

// Orders this wavefront's LDS accesses around a point (DS instructions of one
// wavefront execute in order); used where a single wavefront works alone.
__device__ __forceinline__ void wave_sync()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// One wavefront, l <= 16, run by a single wavefront of the workgroup (no
// block barrier inside).  M column-major with ld = l.
__device__ __forceinline__ int jacobi_wave16(double *M, int l, int max_sweeps)
{
    const int lane = threadIdx.x % kWave;
    const int g = lane / 16, row = lane % 16;
    const int n2 = l + (l & 1);
    const int npairs = n2 / 2;
    const double tol = (double)l * 2.0 * kU;
    int sweep;
    for (sweep = 1; sweep <= max_sweeps; ++sweep) {
        int rot = 0;
        for (int round = 0; round < n2 - 1; ++round) {
            for (int t0 = 0; t0 < npairs; t0 += 4) {
                const int t = t0 + g;
                int p = 0, q = 0;
                bool live = false;
                if (t < npairs) {
                    circle_pair(n2, round, t, p, q);
                    live = q < l;
                }
                double x = 0.0, y = 0.0;
                if (live && row < l) {
                    x = M[p * l + row];
                    y = M[q * l + row];
                }
                double al = x * x, be = y * y, ga = x * y;
                al = seg16_sum(al);
                be = seg16_sum(be);
                ga = seg16_sum(ga);
                const bool doit = live && jacobi_needed(al, be, ga, tol);
                if (doit) {
                    double cs, sn;
                    jacobi_rotation(al, be, ga, cs, sn);
                    if (row < l) {
                        M[p * l + row] = cs * x - sn * y;
                        M[q * l + row] = sn * x + cs * y;
                    }
                }
                rot |= __any(doit && jacobi_needed(al, be, ga, kJacobiQuadStop)) ? 1 : 0;
                wave_sync();
            }
        }
        if (!rot) break;
    }
    return sweep;
}

// Row capacity of the Jacobi groups for 16 < l <= 128 (16 lanes x 2, 4, 6,
// 7 or 8 rows each): the column stride of M, rows past l held at zero.
__host__ __device__ __forceinline__ int svd_row_capacity(int l)
{
    return l <= 32 ? 32 : (l <= 64 ? 64 : (l <= 96 ? 96 : (l <= 112 ? 112 : 128)));
}

// The body of k_small_svd with the Jacobi storage M either in LDS or in
// global memory (inlined once for each, so LDS accesses compile to LDS
// instructions); smem is the dynamic LDS block.
template <typename T, int NT, int LM>
__device__ __forceinline__ void small_svd_body(double *M, double *smem, int l, const double *Gin,
                                               double tau, const double *w, int keep, const T *Q,
                                               int64_t ldq, int mh, T *QM, int64_t ldqm, T *Qout,
                                               int64_t ldqo, const SmallSvdOut &out, int fuse_q,
                                               int &sh_rot, int &rank, int *order, double *sig,
                                               double *coef, double *wc, int in_factor)
{
    const int tid = threadIdx.x;
    const int wave = tid / kWave;

    // l <= 16 with fused products: this thread's first row of Q is loaded
    // now, so that its latency passes during the factorisation
    constexpr int kPre = NT <= 256 ? LM : 1;  // the l <= LM path runs with 256 threads
    double qpre[kPre];
    const bool pre = NT <= 256 && fuse_q && Q && l <= LM && tid < mh;
#pragma unroll
    for (int t = 0; t < kPre; ++t) qpre[t] = (pre && t < l) ? (double)Q[tid + (int64_t)t * ldq] : 0.0;

    // Row-major in-place semidefinite Cholesky: M[j*l + k] = R(j, k), k >= j.
    // Read column-major, column j of M is row j of R, i.e. M = R^T.
    int sweeps = 0;
    // column stride of M after the factorisation: l, or for 16 < l <= 128
    // (M in LDS) the Jacobi groups' row capacity 32, 64, 96, 112 or 128, the rows past
    // l held at zero
    const int ldm = (l > LM && l <= 128) ? svd_row_capacity(l) : l;
    if (in_factor) {
        // the input is already an upper triangular factor C with B^T = H C
        // (column-major): M takes it in the factorisation's layout and the
        // Cholesky step is skipped
        const int ldf = (NT >= 256 && l <= LM) ? l : ldm;
        for (int idx = tid; idx < l * ldf; idx += NT) {
            const int j = idx / ldf, k = idx % ldf;
            M[idx] = (k >= j && k < l) ? Gin[j + (size_t)k * l] : 0.0;
        }
        __syncthreads();
    } else {
        for (int idx = tid; idx < l * l; idx += NT) M[idx] = Gin[idx];
        __syncthreads();
    }
    if (NT >= 256 && l <= LM) {
        // wavefront 0 alone: register Cholesky, then the Jacobi
        if (wave == 0) {
            double maxdiag = 0.0;
            for (int j = 0; j < l; ++j) maxdiag = fmax(maxdiag, M[j * l + j]);
            if (!in_factor) wave_chol16<LM>(M, l, 0.0, 4.0 * l * kU * maxdiag, M, nullptr, false);
            wave_sync();
            sweeps = jacobi_wave16(M, l, 60);
        }
        __syncthreads();
    } else {
        // semidefinite Cholesky: pivots at or below ptol give a zero row
        double maxdiag = 0.0;
        for (int j = 0; j < l; ++j) maxdiag = fmax(maxdiag, M[j * l + j]);
        const double ptol = 4.0 * l * kU * maxdiag;
        if (l <= 128) {
            // sig and coef serve as the step buffers here; R comes back with
            // row stride ldm (zeros past column l - 1)
            if (!in_factor) chol_blk4<NT>(M, l, ptol, 0.0, coef, sig, nullptr, ldm);
            __syncthreads();
            // the nested ordering (one LDS column move per group and step)
            // where the workgroup has the groups for it, else the circle
            if (NT / 16 >= jacobi_nested_groups(l)) {
                if (ldm == 32) sweeps = jacobi_nested<NT, 16, 2>(M, l, ldm, l, 60, &sh_rot);
                else if (ldm == 64) sweeps = jacobi_nested<NT, 16, 4>(M, l, ldm, l, 60, &sh_rot);
                else if (ldm == 96) sweeps = jacobi_nested<NT, 16, 6>(M, l, ldm, l, 60, &sh_rot);
                else if (ldm == 112) sweeps = jacobi_nested<NT, 16, 7>(M, l, ldm, l, 60, &sh_rot);
                else sweeps = jacobi_nested<NT, 16, 8>(M, l, ldm, l, 60, &sh_rot);
            } else if (ldm == 32) sweeps = jacobi_groups<NT, 16, 2, true>(M, l, ldm, l, 60, &sh_rot);
            else if (ldm == 64) sweeps = jacobi_groups<NT, 16, 4, true>(M, l, ldm, l, 60, &sh_rot);
            else if (ldm == 96) sweeps = jacobi_groups<NT, 16, 6, true>(M, l, ldm, l, 60, &sh_rot);
            else if (ldm == 112) sweeps = jacobi_groups<NT, 16, 7, true>(M, l, ldm, l, 60, &sh_rot);
            else sweeps = jacobi_groups<NT, 16, 8, true>(M, l, ldm, l, 60, &sh_rot);
        } else {
            // right-looking in place: row j of R is scaled, then the trailing
            // upper triangle takes its rank-one update
            for (int j = 0; j < l && !in_factor; ++j) {
                const double d = M[j * l + j];
                const double piv = d > ptol ? sqrt(d) : 0.0;
                const double inv = piv > 0.0 ? 1.0 / piv : 0.0;
                for (int k = j + 1 + tid; k < l; k += NT) M[j * l + k] = piv > 0.0 ? M[j * l + k] * inv : 0.0;
                __syncthreads();
                if (tid == 0) M[j * l + j] = piv;
                const int m = l - j - 1;
                for (int idx = tid; idx < m * m; idx += NT) {
                    const int a = idx / m, b = idx - a * m;
                    if (b >= a) M[(j + 1 + a) * l + (j + 1 + b)] -= M[j * l + j + 1 + a] * M[j * l + j + 1 + b];
                }
                __syncthreads();
            }
            for (int idx = tid; idx < l * l; idx += NT) {
                const int j = idx / l, k = idx % l;
                if (k < j) M[idx] = 0.0;
            }
            __syncthreads();
            if (l <= 256) sweeps = jacobi_groups<NT, 16, 16>(M, l, l, l, 60, &sh_rot);
            else sweeps = jacobi_groups<NT, 64, 16>(M, l, l, l, 60, &sh_rot);
        }
        __syncthreads();
    }

    // singular values: column norms of the converged M, one 16-lane group
    // per column
    for (int j = tid / 16; j < l; j += NT / 16) {
        const double *mj = M + (size_t)j * ldm;
        double s = 0.0;
        for (int i = tid % 16; i < l; i += 16) s += mj[i] * mj[i];
        s = seg16_sum(s);
        if (tid % 16 == 0) sig[j] = sqrt(s);
    }
    if (tid == 0) rank = 0;
    __syncthreads();
    // descending order by counting (ties by column index)
    for (int a = tid; a < l; a += NT) {
        const double sa = sig[a];
        int pos = 0;
        for (int b = 0; b < l; ++b) {
            const double sb = sig[b];
            pos += (sb > sa || (sb == sa && b < a)) ? 1 : 0;
        }
        order[pos] = a;
    }
    __syncthreads();
    int rloc = 0;
    for (int a = tid; a < l; a += NT) {
        const double sa = sig[order[a]];
        // the first keep values pass unshrunk (partial SVT), the rest by
        // tau, or by their own thresholds w
        const double th = w ? w[a] : (a < keep ? 0.0 : tau);
        const double f = sa - th;
        coef[a] = (f > 0.0 && sa > 0.0) ? f / sa : 0.0;
        if (f > 0.0) ++rloc;
    }
    if (rloc) atomicAdd(&rank, rloc);
    __syncthreads();
    for (int idx = tid; idx < l * l; idx += NT) {
        const int a = idx / l, i = idx % l;
        const double sa = sig[order[a]];
        out.U[i + (size_t)a * l] = sa > 0.0 ? M[(size_t)order[a] * ldm + i] / sa : 0.0;
    }
    for (int a = tid; a < l; a += NT) out.sigma[a] = sig[order[a]];
    // Mm = sum_a coef_a u_a u_a^T = sum_c wc_c m_c m_c^T over the unsorted
    // columns m_c of M, wc = coef(position of c) / sigma_c^2; 4 x 4 output
    // blocks per thread
    {
        for (int p = tid; p < l; p += NT) {
            const int c = order[p];
            const double sc = sig[c];
            wc[c] = sc > 0.0 ? coef[p] / (sc * sc) : 0.0;
        }
        __syncthreads();
        const int nb = (l + 3) / 4;
        for (int blk = tid; blk < nb * nb; blk += NT) {
            const int bi = 4 * (blk % nb), bj = 4 * (blk / nb);
            double acc[4][4] = {};
            for (int c = 0; c < l; ++c) {
                const double wcc = wc[c];
                if (wcc == 0.0) continue;
                const double *mc = M + (size_t)c * ldm;
                double xi[4], xj[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    xi[e] = bi + e < l ? mc[bi + e] : 0.0;
                    xj[e] = bj + e < l ? wcc * mc[bj + e] : 0.0;
                }
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int f = 0; f < 4; ++f) acc[e][f] += xi[e] * xj[f];
            }
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int f = 0; f < 4; ++f)
                    if (bi + e < l && bj + f < l) out.Mm[(bi + e) + (size_t)(bj + f) * l] = acc[e][f];
        }
    }
    if (tid == 0) {
        out.status[0] = rank;
        out.status[1] = sweeps;
        out.status[2] = sweeps <= 60 ? 1 : 0;
    }
    __syncthreads();
    if (fuse_q && Q) {
        // QM = Q Mm and Qout = Q U(:, 1:r): one row of Q per thread in
        // registers, Mm and U broadcast from LDS (the Jacobi storage M is free).
        double *sU = smem;
        double *sMm = sU + (size_t)l * l;
        const int r = rank;
        for (int idx = tid; idx < l * l; idx += NT) {
            sU[idx] = out.U[idx];
            sMm[idx] = out.Mm[idx];
        }
        __syncthreads();
        if (l <= LM) {
            for (int i = tid; i < mh; i += NT) {
                double q[LM];
                if (kPre == LM && i == tid) {
#pragma unroll
                    for (int t = 0; t < LM; ++t) q[t] = qpre[t < kPre ? t : 0];
                } else {
#pragma unroll
                    for (int t = 0; t < LM; ++t) q[t] = t < l ? (double)Q[i + (int64_t)t * ldq] : 0.0;
                }
#pragma unroll
                for (int j = 0; j < LM; ++j) {
                    if (j < l) {
                        double v = 0.0, u = 0.0;
#pragma unroll
                        for (int t = 0; t < LM; ++t)
                            if (t < l) {
                                v += q[t] * sMm[t + j * l];
                                u += q[t] * sU[t + j * l];
                            }
                        QM[i + (int64_t)j * ldqm] = (T)v;
                        if (Qout && j < r) Qout[i + (int64_t)j * ldqo] = (T)u;
                    }
                }
            }
        } else {
            for (int idx = tid; idx < mh * l; idx += NT) {
                const int i = idx % mh, j = idx / mh;
                double v = 0.0, u = 0.0;
                for (int t = 0; t < l; ++t) {
                    const double qt = (double)Q[i + (int64_t)t * ldq];
                    v += qt * sMm[t + (size_t)j * l];
                    u += qt * sU[t + (size_t)j * l];
                }
                QM[i + (int64_t)j * ldqm] = (T)v;
                if (Qout && j < r) Qout[i + (int64_t)j * ldqo] = (T)u;
            }
        }
    }
}

// LC > 0 fixes l at compile time (see k_small_orth8).
template <typename T, int NT, int LM, int LC = 0>
__global__ void __launch_bounds__(NT) k_small_svd(int l_in, const double *Gin, double tau, int keep,
                                                  const double *w, const T *Q, int64_t ldq, int mh,
                                                  T *QM, int64_t ldqm, T *Qout, int64_t ldqo,
                                                  SmallSvdOut out, double *work, int fuse_q, int in_factor)
{
    const int l = LC > 0 ? LC : l_in;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int sh_rot, rank;
    __shared__ int order[1024];
    __shared__ __align__(16) double coef[1024];
    __shared__ double sig[1024], wc[1024];
    double *smem = reinterpret_cast<double *>(smem_raw);
    if (l <= 128)
        small_svd_body<T, NT, LM>(smem, smem, l, Gin, tau, w, keep, Q, ldq, mh, QM, ldqm, Qout, ldqo, out, fuse_q,
                              sh_rot, rank, order, sig, coef, wc, in_factor);
    else
        small_svd_body<T, NT, LM>(work, smem, l, Gin, tau, w, keep, Q, ldq, mh, QM, ldqm, Qout, ldqo, out, fuse_q,
                              sh_rot, rank, order, sig, coef, wc, in_factor);
}

// l <= 8: the whole small SVD in one wavefront's registers.  Every lane of
// wavefront 0 factors G = R^T R itself (reg_chol), then lane (r, c) =
// (lane % 8, lane / 8) keeps element (r, c) of M = R^T, so that a column of
// M is one 8-lane DPP segment.  Round `rd` of the circle ordering pairs column
// c with d = 2 rd - c mod (n2 - 1) (column rd with the fixed column n2 - 1);
// the partner's element arrives through one lane permute, and the three
// inner products are segment sums that both columns of a pair form over the
// same values in the same order, so both lanes compute the same rotation.
// No LDS access or barrier inside the sweeps.  The other wavefronts load
// their rows of Q meanwhile and join for the products with Q.
// LC > 0 fixes l at compile time (as for k_small_orth8).
template <typename T, int LC>
__global__ void __launch_bounds__(256) k_small_svd8(int l_in, const double *Gin, double tau, int keep,
                                                    const double *w, const T *Q, int64_t ldq, int mh, T *QM,
                                                    int64_t ldqm, T *Qout, int64_t ldqo, SmallSvdOut out,
                                                    int fuse_q, int in_factor)
{
    const int l = LC > 0 ? LC : l_in;
    __shared__ double sM[64], sU[64], sMm[64], swc[8];
    __shared__ int sh_rank;
    const int tid = threadIdx.x;
    const bool fq = fuse_q && Q;
    double qpre[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) qpre[t] = (fq && tid < mh && t < l) ? (double)Q[tid + (int64_t)t * ldq] : 0.0;

    if (tid < kWave) {
        const int lane = tid, r = lane & 7, c = lane >> 3;
        double x = 0.0;
        if (in_factor) {
            // the input is already the upper triangular factor C (column-major)
            if (r < l && c < l && r >= c) x = Gin[c + (size_t)r * l];
        } else {
            double g[8][8];
#pragma unroll
            for (int a = 0; a < 8; ++a)
#pragma unroll
                for (int b = 0; b < 8; ++b) g[a][b] = (b >= a && b < l) ? Gin[a * l + b] : 0.0;
            x = wave8_factor(g, l);
        }
        const int sweeps = wave8_jacobi(x, l, 60);
        // singular values (column norms), their descending order by counting
        // (ties by column index), thresholds and the factors
        const double sg = sqrt(seg8_sum(x * x));
        int pos = 0;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const double sb = read_lane(sg, b * 8);
            pos += (b < l && (sb > sg || (sb == sg && b < c))) ? 1 : 0;
        }
        const bool col = c < l;
        double coef = 0.0, f = -1.0;
        if (col) {
            const double th = w ? w[pos] : (pos < keep ? 0.0 : tau);
            f = sg - th;
            coef = (f > 0.0 && sg > 0.0) ? f / sg : 0.0;
        }
        const int rank = __popcll(__ballot(col && r == 0 && f > 0.0));
        const double u = sg > 0.0 ? x / sg : 0.0;
        if (col && r < l) {
            out.U[r + (size_t)pos * l] = u;
            sU[r + pos * 8] = u;
        }
        if (col && r == 0) {
            out.sigma[pos] = sg;
            swc[c] = sg > 0.0 ? coef / (sg * sg) : 0.0;
        }
        sM[lane] = x;
        wave_sync();
        // Mm(r, c) = sum_b wc_b M(r, b) M(c, b)
        double acc = 0.0;
        for (int b = 0; b < l; ++b) acc += sM[b * 8 + r] * (swc[b] * sM[b * 8 + c]);
        if (r < l && c < l) out.Mm[r + (size_t)c * l] = acc;
        sMm[r + c * 8] = acc;
        if (lane == 0) {
            out.status[0] = rank;
            out.status[1] = sweeps;
            out.status[2] = sweeps <= 60 ? 1 : 0;
            sh_rank = rank;
        }
    }
    __syncthreads();
    if (fq) {
        // QM = Q Mm and Qout = Q U(:, 1:r), one row of Q per thread
        const int rk = sh_rank;
        for (int i = tid; i < mh; i += 256) {
            double q[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) q[t] = (i == tid) ? qpre[t] : (t < l ? (double)Q[i + (int64_t)t * ldq] : 0.0);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (j < l) {
                    double v = 0.0, uu = 0.0;
#pragma unroll
                    for (int t = 0; t < 8; ++t)
                        if (t < l) {
                            v += q[t] * sMm[t + j * 8];
                            uu += q[t] * sU[t + j * 8];
                        }
                    QM[i + (int64_t)j * ldqm] = (T)v;
                    if (Qout && j < rk) Qout[i + (int64_t)j * ldqo] = (T)uu;
                }
            }
        }
    }
}

template <typename T>
hipError_t launch_small_svd(int l, const double *G, double tau, const double *w, int keep, const T *Q,
                            int64_t ldq, int mh, T *QM, int64_t ldqm, T *Qout, int64_t ldqo,
                            const SmallSvdOut &out, double *work, int fuse_q, hipStream_t s, int in_factor)
{
    if (l < 1 || l > 1024) return hipErrorInvalidValue;
    // M in LDS up to l = 128, columns padded to svd_row_capacity(l) rows past l = LM
    const int lm = l <= 8 ? 8 : 16;
    const int ldm = (l > lm && l <= 128) ? svd_row_capacity(l) : l;
    size_t lds = l <= 128 ? (size_t)l * std::max(l, ldm) * sizeof(double) : 0;
    if (fuse_q && Q) lds = std::max(lds, 2 * (size_t)l * l * sizeof(double));
    if (l <= 8) {
        switch (l) {
#define FRK_SVD8_CASE(L)                                                                                      \
    case L:                                                                                                   \
        hipLaunchKernelGGL((k_small_svd8<T, L>), dim3(1), dim3(256), 0, s, l, G, tau, keep, w, Q, ldq, mh, QM, \
                           ldqm, Qout, ldqo, out, fuse_q, in_factor);                                         \
        break;
            FRK_SVD8_CASE(1) FRK_SVD8_CASE(2) FRK_SVD8_CASE(3) FRK_SVD8_CASE(4)
            FRK_SVD8_CASE(5) FRK_SVD8_CASE(6) FRK_SVD8_CASE(7) FRK_SVD8_CASE(8)
#undef FRK_SVD8_CASE
        }
    } else if (l <= 32) {
        switch (l) {
#define FRK_SVD16_CASE(L)                                                                                     \
    case L:                                                                                                   \
        hipLaunchKernelGGL((k_small_svd<T, 256, 16, L>), dim3(1), dim3(256), lds, s, l, G, tau, keep, w, Q, ldq, \
                           mh, QM, ldqm, Qout, ldqo, out, work, fuse_q, in_factor);                           \
        break;
            FRK_SVD16_CASE(9) FRK_SVD16_CASE(10) FRK_SVD16_CASE(11) FRK_SVD16_CASE(12)
            FRK_SVD16_CASE(13) FRK_SVD16_CASE(14) FRK_SVD16_CASE(15) FRK_SVD16_CASE(16)
            FRK_SVD16_CASE(17) FRK_SVD16_CASE(18) FRK_SVD16_CASE(19) FRK_SVD16_CASE(20)
            FRK_SVD16_CASE(21) FRK_SVD16_CASE(22) FRK_SVD16_CASE(23) FRK_SVD16_CASE(24)
            FRK_SVD16_CASE(25) FRK_SVD16_CASE(26) FRK_SVD16_CASE(27) FRK_SVD16_CASE(28)
            FRK_SVD16_CASE(29) FRK_SVD16_CASE(30) FRK_SVD16_CASE(31) FRK_SVD16_CASE(32)
#undef FRK_SVD16_CASE
        }
    }
    else
        hipLaunchKernelGGL((k_small_svd<T, 1024, 16>), dim3(1), dim3(1024), lds, s, l, G, tau, keep, w, Q, ldq, mh, QM, ldqm, Qout, ldqo, out, work, fuse_q, in_factor);
    return hipGetLastError();
}
template hipError_t launch_small_svd<double>(int, const double *, double, const double *, int, const double *, int64_t, int, double *, int64_t, double *, int64_t, const SmallSvdOut &, double *, int, hipStream_t, int);
template hipError_t launch_small_svd<float>(int, const double *, double, const double *, int, const float *, int64_t, int, float *, int64_t, float *, int64_t, const SmallSvdOut &, double *, int, hipStream_t, int);

}  // namespace frk
