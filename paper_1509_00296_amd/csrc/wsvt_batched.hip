// wsvt_batched.hip -- weighted SVT of many small matrices of uneven shapes
// in one persistent launch (the WSVT of weighted nuclear norm minimisation,
// Sec. 1 / footnote 1 of arXiv:1509.00296, applied to patch groups).
//
// Each workgroup pops matrix indices from an atomic queue (longest first) and
// for matrix j (rows x cols, column-major, float), with s = min(rows, cols)
// and W the long-by-short view of A (W = A when cols <= rows, else A^T):
//   1. G = W^T W in double on the matrix cores, straight from A in memory
//      (the upper 16 x 16 blocks dealt to the wavefronts);
//   2. semidefinite Cholesky G = R^T R in LDS (4 x 4 register blocks);
//   3. one-sided Jacobi on M = R^T by groups of gs lanes, one pair per group:
//      the normalised columns of M are the eigenvectors of G (the singular
//      vectors of A on the short side), its column norms the singular values;
//   4. thresholds w_i from the weight rule (or a constant), coef = f / s^3;
//   5. X = A P (or P A) with P = sum coef_c m_c m_c^T as a rank-r update:
//      Z = A m_c (or A^T m_c) for the kept columns, four at a time, then
//      X += coef_c Z m_c^T.
// LDS holds M (and the four Z columns) only, so two workgroups share a
// compute unit.  gs (8, 16 or 32 lanes per pair) is chosen per size bucket
// by the host autotuner and read from a table.
#include "device_common.h"
#include "internal.h"
#include "block_dense.h"

#include <algorithm>

namespace frk {

constexpr int kWB = 256;          // threads per workgroup (four wavefronts, one per SIMD)
constexpr int kWMaxLong = 128;    // longest side
constexpr int kWMaxShort = 96;    // shortest side
constexpr int kWZ = 4;            // kept singular vectors per update chunk

size_t wsvt_batched_lds()
{
    return (size_t)kWMaxShort * kWMaxShort * sizeof(double) + (size_t)kWZ * kWMaxLong * sizeof(double);
}

// G = W^T W (s x s, row-major into M), W(i, x) = A[i * wsi + x * wsx],
// i < L, x < s <= 96.  Step: 8 rows as two 16x16x4 products (k-slot q of
// the first holds row 2q, of the second row 2q + 1).
__device__ __forceinline__ void wsvt_gram(const float *__restrict__ A, int64_t wsi, int64_t wsx, int L, int s,
                                          double *M)
{
    constexpr int NW = kWB / kWave;
    constexpr int NP = (21 + NW - 1) / NW;  // block pairs per wavefront
    typedef __attribute__((__vector_size__(4 * sizeof(double)))) double dx4;
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int c = lane & 15, q = lane >> 4;
    const int nb = (s + 15) / 16;
    dx4 acc[NP];
#pragma unroll
    for (int t = 0; t < NP; ++t) acc[t] = dx4{0.0, 0.0, 0.0, 0.0};
    for (int i0 = 0; i0 < L; i0 += 8) {
        const int ia = i0 + 2 * q, ib = ia + 1;
        double v0[6], v1[6];
#pragma unroll
        for (int bk = 0; bk < 6; ++bk) {
            const int x = 16 * bk + c;
            const bool ok = bk < nb && x < s;
            v0[bk] = (ok && ia < L) ? (double)A[ia * wsi + x * wsx] : 0.0;
            v1[bk] = (ok && ib < L) ? (double)A[ib * wsi + x * wsx] : 0.0;
        }
        int idx = 0;
#pragma unroll
        for (int bi = 0; bi < 6; ++bi)
#pragma unroll
            for (int bj = bi; bj < 6; ++bj, ++idx) {
                if (idx % NW == wave && bj < nb) {
                    acc[idx / NW] = __builtin_amdgcn_mfma_f64_16x16x4f64(v0[bi], v0[bj], acc[idx / NW], 0, 0, 0);
                    acc[idx / NW] = __builtin_amdgcn_mfma_f64_16x16x4f64(v1[bi], v1[bj], acc[idx / NW], 0, 0, 0);
                }
            }
    }
    int idx = 0;
#pragma unroll
    for (int bi = 0; bi < 6; ++bi)
#pragma unroll
        for (int bj = bi; bj < 6; ++bj, ++idx) {
            if (idx % NW == wave && bj < nb) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int x = 16 * bi + q + 4 * e, y = 16 * bj + c;
                    if (x < s && y < s) {
                        M[x * s + y] = acc[idx / NW][e];
                        M[y * s + x] = acc[idx / NW][e];
                    }
                }
            }
        }
}

__global__ void __launch_bounds__(kWB, 2) k_wsvt_batched(WsvtBatchArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *M = reinterpret_cast<double *>(smem_raw);
    double *Z = M + kWMaxShort * kWMaxShort;  // [kWZ][kWMaxLong]
    __shared__ int sh_idx, sh_rot, sh_rank, sh_nz;
    // the workgroup's count of the Jacobi work (added to a.work at the end)
    __shared__ unsigned long long sh_work[3];
    unsigned long long *const wk = a.work ? sh_work : nullptr;
    __shared__ __align__(16) double coef[kWMaxShort];
    __shared__ double sig[kWMaxShort];
    __shared__ int nzc[kWMaxShort];
    const int tid = threadIdx.x;
    if (tid < 3) sh_work[tid] = 0;
    for (;;) {
        if (tid == 0) sh_idx = atomicAdd(a.queue, 1);
        __syncthreads();
        const int64_t qi = sh_idx;
        if (qi >= a.count) break;
        const int j = a.order ? a.order[qi] : (int)qi;
        const int m = a.rows[j], n = a.cols[j];
        if (m < 1 || n < 1 || m > kWMaxLong || n > kWMaxLong || min(m, n) > kWMaxShort) {
            // shapes are read on the device at every launch: one outside the
            // bounds (e.g. rewritten after the graph was captured) is skipped
            // and reported instead of overrunning the local memory
            if (tid == 0) {
                atomicOr(a.queue + 1, 1);
                if (a.ranks) a.ranks[j] = -1;
            }
            __syncthreads();
            continue;
        }
        const int64_t off = a.offsets[j];
        const float *Aj = a.A + off;
        const bool tall = n <= m;
        const int s = tall ? n : m, L = tall ? m : n;
        const int bucket = s <= 48 ? 0 : (s <= 64 ? 1 : 2);
        const int gs = a.group_size[bucket];

        // 1. Gram of the short side (W(i, x) = A(i, x) tall, A(x, i) wide)
        wsvt_gram(Aj, tall ? 1 : m, tall ? m : 1, L, s, M);
        __syncthreads();
        // 2. semidefinite Cholesky (coef and sig serve as its step buffers)
        double maxdiag = 0.0;
        for (int d = 0; d < s; ++d) maxdiag = fmax(maxdiag, M[d * s + d]);
        // column stride of the factor: the Jacobi groups' row capacity
        // (gs x rows per lane), the rows past s held at zero
        const int ldm = bucket == 0 ? (gs == 32 ? 64 : 48) : (bucket == 1 ? 64 : 96);
        chol_blk4<kWB, 2>(M, s, 4.0 * s * kU * maxdiag, 0.0, coef, sig, nullptr, ldm);
        // 3. one-sided Jacobi on M = R^T
        //    (rows per lane E = ceil(bucket bound / gs), so no lane reads past
        //    its bucket)
        int sweeps;
        if (bucket == 0) {
            if (gs == 8) sweeps = jacobi_groups<kWB, 8, 6, true>(M, s, ldm, s, 40, &sh_rot, wk);
            else if (gs == 32) sweeps = jacobi_groups<kWB, 32, 2, true>(M, s, ldm, s, 40, &sh_rot, wk);
            else sweeps = jacobi_groups<kWB, 16, 3, true>(M, s, ldm, s, 40, &sh_rot, wk);
        } else if (bucket == 1) {
            if (gs == 8) sweeps = jacobi_groups<kWB, 8, 8, true>(M, s, ldm, s, 40, &sh_rot, wk);
            else if (gs == 32) sweeps = jacobi_groups<kWB, 32, 2, true>(M, s, ldm, s, 40, &sh_rot, wk);
            else sweeps = jacobi_groups<kWB, 16, 4, true>(M, s, ldm, s, 40, &sh_rot, wk);
        } else {
            if (gs == 8) sweeps = jacobi_groups<kWB, 8, 12, true>(M, s, ldm, s, 40, &sh_rot, wk);
            else if (gs == 32) sweeps = jacobi_groups<kWB, 32, 3, true>(M, s, ldm, s, 40, &sh_rot, wk);
            else sweeps = jacobi_groups<kWB, 16, 6, true>(M, s, ldm, s, 40, &sh_rot, wk);
        }
        // 4. singular values, thresholds: P = sum_c (f_c / s_c) v_c v_c^T with
        //    v_c = m_c / s_c, i.e. coef_c = f_c / s_c^3 on the columns m_c
        for (int cc = tid / 16; cc < s; cc += kWB / 16) {
            const double *mc = M + (size_t)cc * ldm;
            double ss = 0.0;
            for (int i = tid % 16; i < s; i += 16) ss += mc[i] * mc[i];
            ss = seg16_sum(ss);
            if (tid % 16 == 0) {
                const double sv = sqrt(ss);
                double w = a.tau;
                if (a.c > 0.0) {
                    const double e = sv * sv - (double)n * a.noise_var;
                    w = a.c * sqrt((double)n) / ((e > 0.0 ? sqrt(e) : 0.0) + a.eps);
                }
                const double f = sv - w;
                sig[cc] = sv;
                coef[cc] = (f > 0.0 && sv > 0.0) ? f / (sv * sv * sv) : 0.0;
            }
        }
        __syncthreads();
        if (tid == 0) {
            int r = 0;
            for (int cc = 0; cc < s; ++cc)
                if (coef[cc] != 0.0) nzc[r++] = cc;
            sh_rank = r;
            sh_nz = r;
        }
        __syncthreads();
        // 5. X = sum_c coef_c Z_c m_c^T (tall) or coef_c m_c Z_c^T (wide); a
        //    chunk after the first adds to what the same thread stored
        const int nz = sh_nz;
        if (nz == 0)
            for (int idx = tid; idx < m * n; idx += kWB) a.X[off + idx] = 0.0f;
        for (int c0 = 0; c0 < nz; c0 += kWZ) {
            const int cn = min(kWZ, nz - c0);
            for (int idx = tid; idx < cn * L; idx += kWB) {
                const int cc = idx / L, i = idx - cc * L;
                const double *mc = M + (size_t)nzc[c0 + cc] * ldm;
                double z = 0.0;
                if (tall) {
#pragma unroll 8
                    for (int t = 0; t < s; ++t) z += (double)Aj[i + (int64_t)t * m] * mc[t];
                } else {
#pragma unroll 8
                    for (int t = 0; t < s; ++t) z += mc[t] * (double)Aj[t + (int64_t)i * m];
                }
                Z[cc * kWMaxLong + i] = z;
            }
            __syncthreads();
            for (int idx = tid; idx < m * n; idx += kWB) {
                const int i = idx % m, k = idx / m;
                double v = c0 ? (double)a.X[off + idx] : 0.0;
                for (int cc = 0; cc < cn; ++cc) {
                    const int col = nzc[c0 + cc];
                    const double *mc = M + (size_t)col * ldm;
                    v += tall ? coef[col] * Z[cc * kWMaxLong + i] * mc[k] : coef[col] * mc[i] * Z[cc * kWMaxLong + k];
                }
                a.X[off + idx] = (float)v;
            }
            __syncthreads();
        }
        if (tid == 0) {
            if (a.ranks) a.ranks[j] = sh_rank;
            if (a.sweeps) a.sweeps[j] = sweeps;
        }
        __syncthreads();
    }
    if (a.work && tid < 3 && sh_work[tid]) atomicAdd(&a.work[tid], sh_work[tid]);
}

// q[0]: the work counter; q[1]: set when a matrix's shape is outside the
// bounds the kernel's local memory holds (that matrix is skipped); the Jacobi
// work counters (three 64-bit words at byte 64 of the queue block)
__global__ void k_queue_reset(int *q)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        q[0] = 0;
        q[1] = 0;
        unsigned long long *w = reinterpret_cast<unsigned long long *>(q + 16);
        w[0] = 0;
        w[1] = 0;
        w[2] = 0;
    }
}

hipError_t launch_wsvt_batched(const WsvtBatchArgs &a, int grid, hipStream_t s)
{
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, s, a.queue);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wsvt_batched, dim3(grid), dim3(kWB), wsvt_batched_lds(), s, a);
    return hipGetLastError();
}

}  // namespace frk
