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

// Cholesky of (G + shift I), shift = shift_factor trace(G), l <= 256, by one
// workgroup of four wavefronts on the matrix in LDS (l <= 128; beyond, by
// sixteen wavefronts on a global workspace gwork of lp x lp doubles, which
// stays in the caches) (row-major, rows and columns padded to a multiple of
// 16 with zeros; upper triangle used),
// blocked in panels of 16 rows (right-looking):
//   1. wavefront 0 factors the 16 x 16 diagonal block in registers (lane k
//      holds column k; pivots and rows broadcast with readlane; one lean
//      reciprocal square root per pivot);
//   2. the panel's rows right of the block, R_JJ^{-T} A(J, k), one column k
//      per thread; meanwhile wavefront 3 inverts the diagonal block (dinv,
//      when requested: the operand of the matrix-core triangular solve);
//   3. the trailing upper triangle takes the rank-16 update as 16 x 16 tiles
//      on the matrix cores (four 16x16x4 FP64 products per tile).
// Three barriers per panel.  Pivots <= null_tol max_j G_jj are numerically
// null, and with near_one > 0 so is a pivot further than near_one from 1
// (the second CholeskyQR pass's check that the Gram is near the identity):
// R_jj = 1 and a zero row (null_cols[j] = 1).  R is written whole (upper,
// row-major [j * l + k], zeros below the diagonal).
// GM: the matrix in a global workspace (l > 128, where it does not fit in
// LDS) instead of LDS, NT threads (1024 there: more wavefronts for the
// trailing tiles, whose operands then come from the caches).
template <bool GM, int NT>
__global__ void __launch_bounds__(NT) k_chol(int l, const double *G, double shift_factor, double null_tol, double *R, int *null_cols, int *flags, const int *gate, int *nn_out, double near_one, double *dinv, double *gwork)
{
    constexpr int kCholThreads = NT;
    if (gate && *gate == 0) return;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *M = GM ? gwork : reinterpret_cast<double *>(smem_raw);   // lp x lp, row-major
    __shared__ double sRd[16 * 16];
    __shared__ double srinv[16];
    __shared__ double sdiag[2];
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    const int lp = (l + 15) & ~15;
    for (int idx = tid; idx < lp * lp; idx += kCholThreads) {
        const int j = idx / lp, k = idx - j * lp;
        M[idx] = (j < l && k < l) ? G[(size_t)j * l + k] : 0.0;
    }
    __syncthreads();
    if (wave == 0) {
        double tr = 0.0, mx = 0.0;
        for (int j = lane; j < l; j += kWave) {
            const double d = M[j * lp + j];
            tr += d;
            mx = fmax(mx, d);
        }
        tr = wave_sum(tr);
        mx = wave_max(mx);
        if (lane == 0) {
            sdiag[0] = shift_factor * tr;
            sdiag[1] = null_tol > 0.0 ? null_tol * fmax(mx, 1e-300) : 0.0;
        }
    }
    __syncthreads();
    const double shift = sdiag[0], tol = sdiag[1];
    if (shift != 0.0) {
        for (int j = tid; j < l; j += kCholThreads) M[j * lp + j] += shift;
        __syncthreads();
    }
    int nn = 0;
    for (int J = 0; J < l; J += 16) {
        const int nb = min(16, l - J);
        if (wave == 0) {
            double g[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) g[i] = (lane < nb && i <= lane) ? M[(J + i) * lp + J + lane] : 0.0;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                double r = 0.0, rs = 0.0;
                if (j < nb) {
                    const double d = read_lane(g[j], j);
                    bool isnull = !(d > tol);
                    const double rq = rsqrt_pos(isnull ? 1.0 : d);
                    const double piv = d * rq;
                    if (near_one > 0.0 && !isnull) isnull = !(fabs(piv - 1.0) <= near_one);
                    rs = isnull ? 0.0 : rq;
                    nn += isnull ? 1 : 0;
                    if (lane == j) r = isnull ? 1.0 : piv;
                    else if (lane > j && lane < nb) r = g[j] * rs;
                    if (lane == 0 && null_cols) null_cols[J + j] = isnull ? 1 : 0;
                    // every lane updates (lanes below i change entries below
                    // the diagonal, which are never read)
#pragma unroll
                    for (int i = j + 1; i < 16; ++i) g[i] -= read_lane(r, i) * r;
                }
                if (lane < 16) sRd[j * 16 + lane] = r;
                if (lane == 0) srinv[j] = rs;
            }
        }
        __syncthreads();
        if (dinv && wave == kCholThreads / kWave - 1) {
            // the inverse of this 16 x 16 diagonal block (identity past l):
            // lane c forms column c by back substitution
            const int c = lane & 15;
            double x[16];
#pragma unroll
            for (int i = 15; i >= 0; --i) {
                double v = (i == c) ? 1.0 : 0.0;
                if (i < nb) {
#pragma unroll
                    for (int t = i + 1; t < 16; ++t) v -= sRd[i * 16 + t] * x[t];
                    v /= sRd[i * 16 + i];
                }
                x[i] = v;
            }
            if (lane < 16)
#pragma unroll
                for (int i = 0; i < 16; ++i) dinv[(J >> 4) * 256 + i * 16 + c] = x[i];
        }
        for (int k = J + 16 + tid; k < l; k += kCholThreads) {
            double x[16];
#pragma unroll
            for (int a = 0; a < 16; ++a) x[a] = M[(J + a) * lp + k];
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                x[t] *= srinv[t];
#pragma unroll
                for (int a = t + 1; a < 16; ++a) x[a] -= sRd[t * 16 + a] * x[t];
            }
#pragma unroll
            for (int a = 0; a < 16; ++a) M[(J + a) * lp + k] = x[a];
        }
        for (int e = tid; e < 256; e += kCholThreads) M[(J + e / 16) * lp + J + e % 16] = sRd[e];
        __syncthreads();
        const int K0 = J + 16;
        const int nrem = (lp - K0) / 16;
        const int ntiles = nrem * (nrem + 1) / 2;
        for (int tile = wave; tile < ntiles; tile += kCholThreads / kWave) {
            int bi = 0, rem = tile;
            while (rem >= nrem - bi) {
                rem -= nrem - bi;
                ++bi;
            }
            const int K = K0 + 16 * bi, L = K0 + 16 * (bi + rem);
            bd_doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int t = J + 4 * s + (lane >> 4);
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(M[t * lp + K + (lane & 15)], M[t * lp + L + (lane & 15)],
                                                           acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) M[(K + (lane >> 4) + 4 * r) * lp + L + (lane & 15)] -= acc[r];
        }
        __syncthreads();
    }
    for (int idx = tid; idx < l * l; idx += kCholThreads) {
        const int j = idx / l, k = idx - j * l;
        R[idx] = k >= j ? M[j * lp + k] : 0.0;
    }
    if (tid == 0) {
        if (flags) {
            if (null_tol > 0.0) flags[1] = nn;
            if (null_tol <= 0.0 && shift_factor == 0.0) flags[2] = nn > 0 ? 1 : 0;
        }
        if (nn_out) *nn_out = nn;
    }
}

hipError_t launch_chol(int l, const double *G, double shift_factor, double null_tol, double *R, int *null_cols, int *flags, hipStream_t s, const int *gate, int *nn_out, double near_one, double *dinv, double *gwork)
{
    if (l < 1 || l > 256 || (l > 128 && !gwork)) return hipErrorInvalidValue;
    const int lp = (l + 15) & ~15;
    if (l > 128) {
        hipLaunchKernelGGL((k_chol<true, 1024>), dim3(1), dim3(1024), 0, s, l, G, shift_factor, null_tol, R, null_cols,
                           flags, gate, nn_out, near_one, dinv, gwork);
    } else {
        const size_t lds = (size_t)lp * lp * sizeof(double);
        hipLaunchKernelGGL((k_chol<false, 256>), dim3(1), dim3(256), lds, s, l, G, shift_factor, null_tol, R, null_cols,
                           flags, gate, nn_out, near_one, dinv, gwork);
    }
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

// Orders one wavefront's LDS accesses around a point (its DS instructions
// execute in order); for kernels whose workgroup is a single wavefront.
__device__ __forceinline__ void wave_lds_sync()
{
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_wave_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// Y <- Y R^{-1} on the matrix cores, given the inverses Dinv of R's 16 x 16
// diagonal blocks (k_chol writes them; identity past l).  One wavefront per
// 16 rows of Y; for column block J:
//   X_J = (Y_J - sum_{K < J} X_K R_KJ) Dinv_J,
// the sum as 16x16x4 FP64 products in two interleaved accumulation chains
// (A operand: the solved blocks X_K from LDS; B operand: R from memory,
// shared by every wavefront through the caches), the block Y_J - sum moved
// to operand layout through LDS and multiplied by Dinv_J.
// LDX: the row stride of the solved block in LDS, odd (the operand reads of
// 16 rows hit distinct banks) and above l: 129 for l <= 128, 257 for l <= 256.
template <typename T, int LDX>
__global__ void __launch_bounds__(kWave) k_trsm_mfma(int64_t rows, int l, T *Y, int64_t ldy,
                                                     const double *__restrict__ R, const double *__restrict__ Dinv,
                                                     const int *gate)
{
    if (gate && *gate == 0) return;   // the solve is not wanted this time
    __shared__ double sX[16 * LDX];
    __shared__ double sT[16 * 17];
    const int lane = threadIdx.x;
    const int nb = (l + 15) >> 4;
    const int64_t i0 = (int64_t)blockIdx.x * 16;
    const int ar = lane & 15, ak = lane >> 4;   // operand row / column within 16 and k within 4
    for (int J = 0; J < nb; ++J) {
        const int cj = J * 16 + ar;
        double y[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t i = i0 + ak + 4 * r;
            y[r] = (i < rows && cj < l) ? (double)Y[i + (int64_t)cj * ldy] : 0.0;
        }
        bd_doublex4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
        for (int K = 0; K < J; ++K) {
            double b[4], a[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int t = K * 16 + 4 * q + ak;   // < J * 16 < l
                b[q] = cj < l ? R[(int64_t)t * l + cj] : 0.0;
                a[q] = sX[ar * LDX + t];
            }
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], b[1], acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[2], b[2], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[3], b[3], acc1, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) sT[(ak + 4 * r) * 17 + ar] = y[r] - (acc0[r] + acc1[r]);
        wave_lds_sync();
        bd_doublex4 x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < 4; ++q)
            x = __builtin_amdgcn_mfma_f64_16x16x4f64(sT[ar * 17 + 4 * q + ak], Dinv[J * 256 + (4 * q + ak) * 16 + ar], x,
                                                     0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = ak + 4 * r;
            sX[row * LDX + cj] = x[r];
            const int64_t i = i0 + row;
            if (i < rows && cj < l) Y[i + (int64_t)cj * ldy] = (T)x[r];
        }
        wave_lds_sync();
    }
}

template <typename T>
hipError_t launch_trsm(int64_t rows, int l, T *Y, int64_t ldy, const double *R, hipStream_t s, const double *dinv,
                       const int *gate)
{
    if (l > 256 || (l > 128 && !dinv) || (gate && !dinv)) return hipErrorInvalidValue;
    if (dinv && l > 128)
        hipLaunchKernelGGL((k_trsm_mfma<T, 257>), dim3((unsigned)((rows + 15) / 16)), dim3(kWave), 0, s, rows, l, Y, ldy,
                           R, dinv, gate);
    else if (dinv)
        hipLaunchKernelGGL((k_trsm_mfma<T, 129>), dim3((unsigned)((rows + 15) / 16)), dim3(kWave), 0, s, rows, l, Y, ldy,
                           R, dinv, gate);
    else
        hipLaunchKernelGGL((k_trsm<T>), dim3((unsigned)((rows + kWave - 1) / kWave)), dim3(kTrsmThreads), 0, s, rows, l,
                           Y, ldy, R);
    return hipGetLastError();
}
template hipError_t launch_trsm<double>(int64_t, int, double *, int64_t, const double *, hipStream_t, const double *,
                                        const int *);
template hipError_t launch_trsm<float>(int64_t, int, float *, int64_t, const double *, hipStream_t, const double *,
                                       const int *);

// Y <- Y U for an upper triangular U (row-major, l <= 128) on the matrix
// cores: one wavefront per 16 rows, the rows of Y staged in LDS first, then
// every column block Y_J' = sum_{K <= J} Y_K U_KJ.
template <typename T, int LDX>
__global__ void __launch_bounds__(kWave) k_trmm_mfma(int64_t rows, int l, T *Y, int64_t ldy, const double *__restrict__ U,
                                                     const int *skip)
{
    if (skip && *skip != 0) return;   // the product is not wanted this time
    __shared__ double sX[16 * LDX];
    const int lane = threadIdx.x;
    const int nb = (l + 15) >> 4;
    const int64_t i0 = (int64_t)blockIdx.x * 16;
    const int ar = lane & 15, ak = lane >> 4;
    for (int J = 0; J < nb; ++J) {
        const int cj = J * 16 + ar;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t i = i0 + ak + 4 * r;
            sX[(ak + 4 * r) * LDX + cj] = (i < rows && cj < l) ? (double)Y[i + (int64_t)cj * ldy] : 0.0;
        }
    }
    wave_lds_sync();
    for (int J = 0; J < nb; ++J) {
        const int cj = J * 16 + ar;
        bd_doublex4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
        for (int K = 0; K <= J; ++K) {
            double b[4], a[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int t = K * 16 + 4 * q + ak;
                b[q] = (t < l && cj < l) ? U[(int64_t)t * l + cj] : 0.0;
                a[q] = sX[ar * LDX + t];
            }
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], b[1], acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[2], b[2], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[3], b[3], acc1, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t i = i0 + ak + 4 * r;
            if (i < rows && cj < l) Y[i + (int64_t)cj * ldy] = (T)(acc0[r] + acc1[r]);
        }
    }
}

template <typename T>
hipError_t launch_trmm(int64_t rows, int l, T *Y, int64_t ldy, const double *U, hipStream_t s, const int *skip)
{
    if (l < 1 || l > 256) return hipErrorInvalidValue;
    if (l > 128)
        hipLaunchKernelGGL((k_trmm_mfma<T, 257>), dim3((unsigned)((rows + 15) / 16)), dim3(kWave), 0, s, rows, l, Y, ldy,
                           U, skip);
    else
        hipLaunchKernelGGL((k_trmm_mfma<T, 129>), dim3((unsigned)((rows + 15) / 16)), dim3(kWave), 0, s, rows, l, Y, ldy,
                           U, skip);
    return hipGetLastError();
}
template hipError_t launch_trmm<double>(int64_t, int, double *, int64_t, const double *, hipStream_t, const int *);
template hipError_t launch_trmm<float>(int64_t, int, float *, int64_t, const double *, hipStream_t, const int *);

// The second CholeskyQR pass when the Gram G = I + E of the once
// orthonormalised basis is close to the identity: its Cholesky factor is
// R = I + S + O(|E|^2), S the upper triangle of E with half its diagonal
// (so that S + S^T = E), and R^{-1} = I - S + O(|E|^2).  Writes U = I - S
// (upper, row-major), *full = 1 when ||E||_F exceeds tol (the first-order
// factor would not be accurate to working precision: the full Cholesky
// pass is wanted) else 0, and clears *nn (the null count of that pass).
__global__ void __launch_bounds__(kThreads) k_near_identity(int l, const double *G, double *U, int *full, int *nn,
                                                            double tol)
{
    __shared__ double sred[kThreads / kWave];
    double ss = 0.0;
    for (int idx = threadIdx.x; idx < l * l; idx += kThreads) {
        const int i = idx / l, j = idx - i * l;
        const double e = G[idx] - (i == j ? 1.0 : 0.0);
        ss += e * e;
        U[idx] = j > i ? -e : (j == i ? 1.0 - 0.5 * e : 0.0);
    }
    ss = wave_sum(ss);
    if (threadIdx.x % kWave == 0) sred[threadIdx.x / kWave] = ss;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kThreads / kWave; ++w) t += sred[w];
        *full = !(sqrt(t) <= tol) ? 1 : 0;
        *nn = 0;
    }
}

hipError_t launch_near_identity(int l, const double *G, double *U, int *full, int *nn, double tol, hipStream_t s)
{
    hipLaunchKernelGGL(k_near_identity, dim3(1), dim3(kThreads), 0, s, l, G, U, full, nn, tol);
    return hipGetLastError();
}

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
