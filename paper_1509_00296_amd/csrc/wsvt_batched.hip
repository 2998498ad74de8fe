// wsvt_batched.hip -- weighted SVT of many small matrices of uneven shapes
// in one persistent launch (the WSVT of weighted nuclear norm minimisation,
// Sec. 1 / footnote 1 of arXiv:1509.00296, applied to patch groups).
//
// Each workgroup pops matrix indices from an atomic queue (longest first) and
// for matrix j (rows x cols, column-major, float):
//   1. stages A in LDS (float), forms the Gram G of its short side in double
//      (A^T A when cols <= rows, else A A^T), s = min(rows, cols);
//   2. semidefinite Cholesky G = R^T R in place;
//   3. one-sided Jacobi on M = R^T: its normalised columns are the
//      eigenvectors V of G (the singular vectors of A on the short side) and
//      its column norms the singular values of A;
//   4. thresholds w_i from the weight rule (or a constant), coef = f/s;
//   5. P = V diag(coef) V^T (float) and X = A P (or P A), written as float.
// Jacobi pairs (circle method) are spread over groups of `gs` lanes; gs is
// chosen per size bucket by the host autotuner and read from a table.
#include "device_common.h"
#include "internal.h"

#include <algorithm>

namespace frk {

constexpr int kWB = 512;          // threads per workgroup
constexpr int kWMaxLong = 128;    // longest side
constexpr int kWMaxShort = 96;    // shortest side

size_t wsvt_batched_lds() { return (size_t)kWMaxLong * kWMaxShort * 4 + (size_t)kWMaxShort * kWMaxShort * 8 + (size_t)kWMaxShort * kWMaxShort * 4; }

// sum over the aligned group of gs lanes (gs = 8, 16 or 32), in every lane
__device__ __forceinline__ double seg_sum(double v, int gs)
{
    if (gs == 8) return seg8_sum(v);
    if (gs == 16) return seg16_sum(v);
    return seg32_sum(v);
}

__global__ void __launch_bounds__(kWB) k_wsvt_batched(WsvtBatchArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float *sA = reinterpret_cast<float *>(smem_raw);                               // rows x cols
    double *sM = reinterpret_cast<double *>(smem_raw + (size_t)kWMaxLong * kWMaxShort * 4);
    float *sP = reinterpret_cast<float *>(smem_raw + (size_t)kWMaxLong * kWMaxShort * 4 +
                                          (size_t)kWMaxShort * kWMaxShort * 8);
    __shared__ int sh_idx, sh_rot, sh_rank;
    __shared__ double sig[kWMaxShort], coef[kWMaxShort];
    const int tid = threadIdx.x;
    const int64_t nrot_local = 0;
    (void)nrot_local;
    for (;;) {
        if (tid == 0) sh_idx = atomicAdd(a.queue, 1);
        __syncthreads();
        const int64_t qi = sh_idx;
        if (qi >= a.count) break;
        const int j = a.order ? a.order[qi] : (int)qi;
        const int m = a.rows[j], n = a.cols[j];
        const int64_t off = a.offsets[j];
        const bool tall = n <= m;
        const int s = tall ? n : m, L = tall ? m : n;
        const int bucket = s <= 48 ? 0 : (s <= 64 ? 1 : 2);
        const int gs = a.group_size[bucket];
        const int ngroups = kWB / gs;

        for (int idx = tid; idx < m * n; idx += kWB) sA[idx] = a.A[off + idx];
        __syncthreads();
        // 1. Gram of the short side, double
        const int npairs = s * (s + 1) / 2;
        for (int p = tid; p < npairs; p += kWB) {
            int x = 0, rem = p;
            while (rem >= s - x) {
                rem -= s - x;
                ++x;
            }
            const int y = x + rem;
            double acc = 0.0;
            if (tall) {
                const float *ca = sA + (size_t)x * m, *cb = sA + (size_t)y * m;
                for (int i = 0; i < m; ++i) acc += (double)ca[i] * (double)cb[i];
            } else {
                for (int k = 0; k < n; ++k) acc += (double)sA[x + (size_t)k * m] * (double)sA[y + (size_t)k * m];
            }
            sM[x * s + y] = acc;
            sM[y * s + x] = acc;
        }
        __syncthreads();
        // 2. semidefinite Cholesky, row-major in place (sM[r*s + c] = R(r, c))
        double maxdiag = 0.0;
        for (int d = 0; d < s; ++d) maxdiag = fmax(maxdiag, sM[d * s + d]);
        const double ptol = 4.0 * s * kU * maxdiag;
        for (int c0 = 0; c0 < s; ++c0) {
            double d = sM[c0 * s + c0];
            for (int t = 0; t < c0; ++t) d -= sM[t * s + c0] * sM[t * s + c0];
            const double piv = d > ptol ? sqrt(d) : 0.0;
            __syncthreads();
            if (tid == 0) sM[c0 * s + c0] = piv;
            for (int k = c0 + 1 + tid; k < s; k += kWB) {
                double v = 0.0;
                if (piv > 0.0) {
                    v = sM[c0 * s + k];
                    for (int t = 0; t < c0; ++t) v -= sM[t * s + c0] * sM[t * s + k];
                    v /= piv;
                }
                sM[c0 * s + k] = v;
            }
            __syncthreads();
        }
        for (int idx = tid; idx < s * s; idx += kWB)
            if (idx % s < idx / s) sM[idx] = 0.0;
        __syncthreads();
        // 3. one-sided Jacobi on M = R^T (column c of M = row c of R)
        const int n2 = s + (s & 1);
        const int pairs = n2 / 2;
        const int g = tid / gs, gl = tid % gs;
        const double tol = (double)s * 2.0 * kU;
        int sweeps = 0;
        for (int sweep = 0; sweep < 40; ++sweep) {
            if (tid == 0) sh_rot = 0;
            __syncthreads();
            for (int round = 0; round < n2 - 1; ++round) {
                for (int t0 = 0; t0 < pairs; t0 += ngroups) {
                    const int t = t0 + g;
                    int p = 0, q = 0;
                    bool live = false;
                    if (t < pairs) {
                        if (t == 0) {
                            p = n2 - 1;
                            q = round;
                        } else {
                            p = (round + t) % (n2 - 1);
                            q = (round - t + n2 - 1) % (n2 - 1);
                        }
                        if (p > q) {
                            const int tmp = p;
                            p = q;
                            q = tmp;
                        }
                        live = q < s;
                    }
                    double al = 0.0, be = 0.0, ga = 0.0;
                    if (live)
                        for (int i = gl; i < s; i += gs) {
                            const double x = sM[p * s + i], y = sM[q * s + i];
                            al += x * x;
                            be += y * y;
                            ga += x * y;
                        }
                    al = seg_sum(al, gs);
                    be = seg_sum(be, gs);
                    ga = seg_sum(ga, gs);
                    if (live && fabs(ga) > tol * sqrt(al * be)) {
                        const double zeta = (be - al) / (2.0 * ga);
                        const double t1 = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
                        const double cs = 1.0 / sqrt(1.0 + t1 * t1), sn = cs * t1;
                        for (int i = gl; i < s; i += gs) {
                            const double x = sM[p * s + i], y = sM[q * s + i];
                            sM[p * s + i] = cs * x - sn * y;
                            sM[q * s + i] = sn * x + cs * y;
                        }
                        if (gl == 0) sh_rot = 1;
                    }
                    __syncthreads();
                }
            }
            sweeps = sweep + 1;
            const int rot = sh_rot;
            __syncthreads();
            if (!rot) break;
        }
        // 4. singular values, thresholds
        for (int c = tid; c < s; c += kWB) {
            double ss = 0.0;
            for (int i = 0; i < s; ++i) ss += sM[c * s + i] * sM[c * s + i];
            const double sv = sqrt(ss);
            double w = a.tau;
            if (a.c > 0.0) {
                const double e = sv * sv - (double)n * a.noise_var;
                w = a.c * sqrt((double)n) / ((e > 0.0 ? sqrt(e) : 0.0) + a.eps);
            }
            const double f = sv - w;
            sig[c] = sv;
            // P = sum_c (f_c / s_c) v_c v_c^T with v_c = m_c / s_c
            coef[c] = (f > 0.0 && sv > 0.0) ? f / (sv * sv * sv) : 0.0;
        }
        __syncthreads();
        if (tid == 0) {
            int r = 0;
            for (int c = 0; c < s; ++c) r += coef[c] > 0.0 ? 1 : 0;
            sh_rank = r;
        }
        // 5. P = sum_c coef_c m_c m_c^T
        for (int idx = tid; idx < s * s; idx += kWB) {
            const int x = idx % s, y = idx / s;
            double v = 0.0;
            for (int c = 0; c < s; ++c)
                if (coef[c] != 0.0) v += coef[c] * sM[c * s + x] * sM[c * s + y];
            sP[idx] = (float)v;
        }
        __syncthreads();
        for (int idx = tid; idx < m * n; idx += kWB) {
            const int i = idx % m, k = idx / m;
            float v = 0.0f;
            if (tall)
                for (int t = 0; t < n; ++t) v += sA[i + t * m] * sP[t + k * s];
            else
                for (int t = 0; t < m; ++t) v += sP[i + t * s] * sA[t + k * m];
            a.X[off + idx] = v;
        }
        if (tid == 0) {
            if (a.ranks) a.ranks[j] = sh_rank;
            if (a.sweeps) a.sweeps[j] = sweeps;
        }
        __syncthreads();
    }
}

__global__ void k_queue_reset(int *q)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) q[0] = 0;
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
