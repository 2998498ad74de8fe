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
// Large-path CholeskyQR pieces (l <= 128 columns).
// ===========================================================================
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double gd_doublex4;

// Partial Grams of a tall rows x l matrix Y (column-major, ld) on the
// matrix cores: workgroup g takes rows [g rpw, (g + 1) rpw) and writes
// the full l x l partial Gram to part + g l^2 ([a * l + b]).  The 16 x 16
// blocks (bi <= bj) of the upper triangle are dealt round-robin to the four
// wavefronts; a step takes 8 rows as two 16x16x4 products, k-slot s of the
// first holding row 2s and of the second row 2s + 1.
template <typename T>
__global__ void __launch_bounds__(kThreads) k_gram_tall(int64_t rows, int l, const T *__restrict__ Y,
                                                        int64_t ldy, int64_t rpw, double *part, const int *gate)
{
    if (gate && *gate == 0) return;  // the partials are still current
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int c = lane & 15, s = lane >> 4;
    const int nb = (l + 15) / 16;
    const int64_t r0 = (int64_t)blockIdx.x * rpw, r1 = min(rows, r0 + rpw);
    gd_doublex4 acc[9];
#pragma unroll
    for (int p = 0; p < 9; ++p) acc[p] = gd_doublex4{0.0, 0.0, 0.0, 0.0};
    for (int64_t i0 = r0; i0 < r1; i0 += 8) {
        const int64_t ia = i0 + 2 * s, ib = ia + 1;
        double v0[8], v1[8];
#pragma unroll
        for (int bk = 0; bk < 8; ++bk) {
            const int col = 16 * bk + c;
            const bool okc = bk < nb && col < l;
            const T *yc = Y + (int64_t)col * ldy;
            v0[bk] = (okc && ia < r1) ? (double)yc[ia] : 0.0;
            v1[bk] = (okc && ib < r1) ? (double)yc[ib] : 0.0;
        }
        int idx = 0;
#pragma unroll
        for (int bi = 0; bi < 8; ++bi)
#pragma unroll
            for (int bj = bi; bj < 8; ++bj, ++idx) {
                if ((idx & 3) == wave && bj < nb) {
                    acc[idx >> 2] = __builtin_amdgcn_mfma_f64_16x16x4f64(v0[bi], v0[bj], acc[idx >> 2], 0, 0, 0);
                    acc[idx >> 2] = __builtin_amdgcn_mfma_f64_16x16x4f64(v1[bi], v1[bj], acc[idx >> 2], 0, 0, 0);
                }
            }
    }
    double *pg = part + (int64_t)blockIdx.x * l * l;
    int idx = 0;
#pragma unroll
    for (int bi = 0; bi < 8; ++bi)
#pragma unroll
        for (int bj = bi; bj < 8; ++bj, ++idx) {
            if ((idx & 3) == wave && bj < nb) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int a = 16 * bi + s + 4 * e, b = 16 * bj + c;
                    if (a < l && b < l) {
                        pg[a * l + b] = acc[idx >> 2][e];
                        pg[b * l + a] = acc[idx >> 2][e];
                    }
                }
            }
        }
}

template <typename T>
hipError_t launch_gram_tall(int64_t rows, int l, const T *Y, int64_t ldy, double *part, double *G,
                            hipStream_t s, const int *gate)
{
    if (l < 1 || l > 128) return hipErrorInvalidValue;
    int64_t rpw = std::max<int64_t>(64, (rows + 63) / 64);
    rpw = (rpw + 7) / 8 * 8;
    const int nparts = (int)std::max<int64_t>(1, (rows + rpw - 1) / rpw);
    hipLaunchKernelGGL((k_gram_tall<T>), dim3(nparts), dim3(kThreads), 0, s, rows, l, Y, ldy, rpw, part, gate);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_reduce<double>(part, (int64_t)l * l, nparts, G, s);
}
template hipError_t launch_gram_tall<double>(int64_t, int, const double *, int64_t, double *, double *, hipStream_t, const int *);
template hipError_t launch_gram_tall<float>(int64_t, int, const float *, int64_t, double *, double *, hipStream_t, const int *);

// Cholesky of (G + shift I), shift = shift_factor trace(G), l <= 128, by one
// workgroup on the matrix in LDS (row-major, upper triangle used), blocked
// in panels of 16 rows (right-looking):
//   1. wavefront 0 factors the 16 x 16 diagonal block in registers (lane k
//      holds column k; pivots and rows broadcast with readlane);
//   2. the panel's rows right of the block, R_JJ^{-T} A(J, k), one column k
//      per thread;
//   3. the trailing upper triangle takes the rank-16 update in 4 x 4 blocks.
// Three barriers per panel.  Pivots <= null_tol max_j G_jj are numerically
// null: R_jj = 1 and a zero row (null_cols[j] = 1).  R is written whole
// (upper, row-major [j * l + k], zeros below the diagonal).
constexpr int kCholThreads = 512;
// near_one > 0: a pivot further than near_one from 1 is also counted (and
// treated) as null (the second CholeskyQR pass's check that the Gram is
// near the identity).
__global__ void __launch_bounds__(kCholThreads) k_chol(int l, const double *G, double shift_factor, double null_tol, double *R, int *null_cols, int *flags, const int *gate, int *nn_out, double near_one)
{
    if (gate && *gate == 0) return;  // the factor in R is still current
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *M = reinterpret_cast<double *>(smem_raw);
    __shared__ double shift, tolabs;
    __shared__ double srinv[128];
    __shared__ int snull[128];
    __shared__ int sh_nn;
    const int tid = threadIdx.x, lane = tid % kWave;
    for (int idx = tid; idx < l * l; idx += kCholThreads) M[idx] = G[idx];
    __syncthreads();
    if (tid == 0) {
        double tr = 0.0, mx = 0.0;
        for (int j = 0; j < l; ++j) {
            tr += M[j * l + j];
            mx = fmax(mx, M[j * l + j]);
        }
        shift = shift_factor * tr;
        tolabs = null_tol > 0.0 ? null_tol * fmax(mx, 1e-300) : 0.0;
        sh_nn = 0;
    }
    __syncthreads();
    for (int j = tid; j < l; j += kCholThreads) M[j * l + j] += shift;
    __syncthreads();
    const double tol = tolabs;
    for (int J = 0; J < l; J += 16) {
        const int nb = min(16, l - J);
        // 1. the diagonal block (upper entries read; the lower ones are stale)
        if (tid < kWave) {
            double g[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) g[i] = (i < nb && lane < nb) ? M[(J + i) * l + J + lane] : 0.0;
            int nn = 0;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                if (j < nb) {
                    double gj = 0.0;
#pragma unroll
                    for (int i = 0; i < 16; ++i)
                        if (i == j) gj = g[i];
                    const double d = read_lane(gj, j);
                    bool isnull = !(d > tol);
                    if (near_one > 0.0 && !isnull) isnull = !(fabs(sqrt(d) - 1.0) <= near_one);
                    const double rs = rsqrt(isnull ? 1.0 : d);
                    const double piv = isnull ? 1.0 : d * rs;
                    nn += isnull ? 1 : 0;
                    double rjk = 0.0;
                    if (lane == j) rjk = piv;
                    else if (lane > j && lane < nb && !isnull) rjk = gj * rs;
                    if (lane < nb) M[(J + j) * l + J + lane] = rjk;
                    if (lane == 0) {
                        snull[J + j] = isnull ? 1 : 0;
                        srinv[J + j] = isnull ? 0.0 : rs;
                        if (null_cols) null_cols[J + j] = isnull ? 1 : 0;
                    }
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        if (i > j) {
                            const double rji = read_lane(rjk, i);
                            g[i] = lane > j ? g[i] - rji * rjk : g[i];
                        }
                    }
                }
            }
            if (lane == 0) sh_nn += nn;
        }
        __syncthreads();
        // 2. R(J : J + nb, k) = R_JJ^{-T} A(J : J + nb, k), k >= J + nb (null
        //    rows zero)
        for (int k = J + nb + tid; k < l; k += kCholThreads) {
            double x[16];
#pragma unroll
            for (int a = 0; a < 16; ++a) x[a] = a < nb ? M[(J + a) * l + k] : 0.0;
#pragma unroll
            for (int a = 0; a < 16; ++a) {
                if (a < nb) {
                    double v = x[a];
#pragma unroll
                    for (int t = 0; t < a; ++t) v -= M[(J + t) * l + J + a] * x[t];
                    x[a] = v * srinv[J + a];
                }
            }
#pragma unroll
            for (int a = 0; a < 16; ++a)
                if (a < nb) M[(J + a) * l + k] = x[a];
        }
        __syncthreads();
        // 3. trailing update of the upper triangle, rows and columns >= J + nb
        const int base = J + nb, nt = l - base;
        if (nt > 0) {
            const int nbk = (nt + 3) / 4;
            const int nblk = nbk * (nbk + 1) / 2;
            for (int blk = tid; blk < nblk; blk += kCholThreads) {
                int bi = 0, rem = blk;
                while (rem >= nbk - bi) {
                    rem -= nbk - bi;
                    ++bi;
                }
                const int bj = bi + rem;
                const int a0 = base + 4 * bi, k0 = base + 4 * bj;
                double acc[4][4];
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int f = 0; f < 4; ++f)
                        acc[e][f] = (a0 + e < l && k0 + f < l) ? M[(a0 + e) * l + k0 + f] : 0.0;
                for (int t = 0; t < nb; ++t) {
                    const double *row = M + (J + t) * l;
                    double ra[4], rk[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        ra[e] = a0 + e < l ? row[a0 + e] : 0.0;
                        rk[e] = k0 + e < l ? row[k0 + e] : 0.0;
                    }
#pragma unroll
                    for (int e = 0; e < 4; ++e)
#pragma unroll
                        for (int f = 0; f < 4; ++f) acc[e][f] -= ra[e] * rk[f];
                }
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int f = 0; f < 4; ++f)
                        if (a0 + e < l && k0 + f < l) M[(a0 + e) * l + k0 + f] = acc[e][f];
            }
        }
        __syncthreads();
    }
    for (int idx = tid; idx < l * l; idx += kCholThreads) {
        const int j = idx / l, k = idx % l;
        R[idx] = k >= j ? M[idx] : 0.0;
    }
    if (tid == 0) {
        const int nn = sh_nn;
        if (flags) {
            // null checks report the columns they flag; the final pass (no
            // shift, no null tolerance) records whether its factor still failed
            if (null_tol > 0.0) flags[1] = nn;
            if (null_tol <= 0.0 && shift_factor == 0.0) flags[2] = nn > 0 ? 1 : 0;
        }
        if (nn_out) *nn_out = nn;
    }
}

hipError_t launch_chol(int l, const double *G, double shift_factor, double null_tol, double *R, int *null_cols, int *flags, hipStream_t s, const int *gate, int *nn_out, double near_one)
{
    const size_t lds = (size_t)l * l * sizeof(double);
    if (l < 1 || l > 128) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_chol, dim3(1), dim3(kCholThreads), lds, s, l, G, shift_factor, null_tol, R, null_cols, flags, gate, nn_out, near_one);
    return hipGetLastError();
}

// G_out(a, b) = G(a, b) / sqrt(G(a, a) G(b, b)) (zero where a diagonal entry
// is not positive): the Gram of the columns scaled as k_col_scale scales them.
__global__ void __launch_bounds__(kThreads) k_scale_gram(int l, const double *G, double *Gout)
{
    for (int idx = blockIdx.x * kThreads + threadIdx.x; idx < l * l; idx += gridDim.x * kThreads) {
        const int a = idx / l, b = idx % l;
        const double ga = G[a * l + a], gb = G[b * l + b];
        const double sa = ga > 0.0 ? 1.0 / sqrt(ga) : 0.0, sb = gb > 0.0 ? 1.0 / sqrt(gb) : 0.0;
        Gout[idx] = G[idx] * (sa * sb);
    }
}

hipError_t launch_scale_gram(int l, const double *G, double *Gout, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale_gram, dim3((unsigned)((l * l + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, l, G, Gout);
    return hipGetLastError();
}

// Y <- Y R^{-1} (R upper, row-major, l <= 128).  A workgroup of four
// wavefronts takes 64 rows, one row per lane, and solves blocks of 16
// columns: for block J the four wavefronts split the update by the
// already-solved column t (t = w mod 4), their partial sums are added in
// wavefront order, and wavefront 0 solves the 16 x 16 diagonal block with
// the reciprocals of R's diagonal.  Solved columns stay in LDS (column t at
// sY[t * 64 + lane]); the panel R(0 : J + 16, J : J + 16) is staged in LDS
// (zero off the diagonal and unit diagonal past column l) and read by
// broadcast.
constexpr int kTrsmThreads = 256;
template <typename T>
__global__ void __launch_bounds__(kTrsmThreads) k_trsm(int64_t rows, int l, T *Y, int64_t ldy, const double *__restrict__ R)
{
    __shared__ double sY[128 * kWave];
    __shared__ __align__(16) double sR[128 * 16];
    __shared__ double sRinv[16];
    __shared__ double sPart[3 * 16 * kWave];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int64_t i = (int64_t)blockIdx.x * kWave + lane;
    const bool live = i < rows;
    for (int J = 0; J < l; J += 16) {
        const int ne = (J + 16) * 16;
        for (int e = threadIdx.x; e < ne; e += kTrsmThreads) {
            const int t = e / 16, c = J + e % 16;
            sR[e] = (t < l && c < l) ? R[(int64_t)t * l + c] : (t == c ? 1.0 : 0.0);
        }
        if (threadIdx.x < 16) {
            const int c = J + threadIdx.x;
            sRinv[threadIdx.x] = c < l ? 1.0 / R[(int64_t)c * l + c] : 1.0;
        }
        double acc[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj)
            acc[jj] = (wave == 0 && live && J + jj < l) ? (double)Y[i + (int64_t)(J + jj) * ldy] : 0.0;
        __syncthreads();
#pragma unroll 2
        for (int t = wave; t < J; t += 4) {
            const double yt = sY[t * kWave + lane];
            const double2 *rt = reinterpret_cast<const double2 *>(sR + t * 16);
#pragma unroll
            for (int h = 0; h < 8; ++h) {
                const double2 r = rt[h];
                acc[2 * h] -= yt * r.x;
                acc[2 * h + 1] -= yt * r.y;
            }
        }
        if (J > 0) {
            if (wave > 0) {
#pragma unroll
                for (int jj = 0; jj < 16; ++jj) sPart[((wave - 1) * 16 + jj) * kWave + lane] = acc[jj];
            }
            __syncthreads();
        }
        if (wave == 0) {
            if (J > 0) {
#pragma unroll
                for (int jj = 0; jj < 16; ++jj)
                    acc[jj] = ((acc[jj] + sPart[jj * kWave + lane]) + sPart[(16 + jj) * kWave + lane]) +
                              sPart[(32 + jj) * kWave + lane];
            }
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) {
                double v = acc[jj];
#pragma unroll
                for (int tt = 0; tt < jj; ++tt) v -= acc[tt] * sR[(J + tt) * 16 + jj];
                acc[jj] = v * sRinv[jj];
            }
            // stores after the block's solves: a global store ahead of a
            // later load's first use would make that use wait for the store
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) {
                sY[(J + jj) * kWave + lane] = acc[jj];
                if (live && J + jj < l) Y[i + (int64_t)(J + jj) * ldy] = (T)acc[jj];
            }
        }
        __syncthreads();
    }
}

template <typename T>
hipError_t launch_trsm(int64_t rows, int l, T *Y, int64_t ldy, const double *R, hipStream_t s)
{
    if (l > 128) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_trsm<T>), dim3((unsigned)((rows + kWave - 1) / kWave)), dim3(kTrsmThreads), 0, s, rows, l, Y, ldy, R);
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
    const int64_t total = rows * l;
    for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kThreads) {
        const int64_t i = idx % rows;
        const int j = (int)(idx / rows);
        const double g = G[j * l + j];
        const double sc = g > 0.0 ? 1.0 / sqrt(g) : 0.0;
        Y[i + (int64_t)j * ldy] = (T)((double)Y[i + (int64_t)j * ldy] * sc);
    }
}

template <typename T>
hipError_t launch_col_scale(int64_t rows, int l, T *Y, int64_t ldy, const double *G, hipStream_t s)
{
    const int64_t total = rows * l;
    const unsigned g = (unsigned)std::min<int64_t>(2048, std::max<int64_t>(1, (total + kThreads - 1) / kThreads));
    hipLaunchKernelGGL((k_col_scale<T>), dim3(g), dim3(kThreads), 0, s, rows, l, Y, ldy, G);
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
