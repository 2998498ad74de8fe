// long_pass.hip -- passes over Ahat along its long dimension: the Gaussian
// sketch Y = Ahat Omega (Alg. 1 lines 5 and 9), the fused power step
// Y = Ahat (Ahat^T Q) (line 14) and the projection B^T = Ahat^T Q with the
// Gram B B^T (line 16); plus the fixed-order split-K reductions.
#include "device_common.h"
#include "internal.h"

#include <algorithm>

namespace frk {

// ===========================================================================
// One workgroup (256 threads) walks tiles of kKT long-dimension indices; each
// tile holds the whole short dimension (mh <= 512) in LDS as
// sTile[kk * mhp + i] with an odd row stride.  The next tile is prefetched
// into registers while the current one is processed.
//
//  phase 1 (power / projection): z(kk, :) = sum_i Ahat(i, k0+kk) Q(i, :).
//    Thread (kk, column group cg, slice s) sums the rows i = s, s+S, ...;
//    the S slices are combined in a fixed order through LDS.
//  phase 2 (sketch / power): Y(i, :) += sum_kk Ahat(i, k0+kk) v(kk, :), one
//    thread per short index i, v broadcast from LDS (no cross-lane sums).
//  projection: B^T rows written out, Gram B B^T accumulated in double.
// ===========================================================================
constexpr int kKT = 16;
constexpr int kMaxMh = 512;

bool long_path_ok(int mh, int c) { return mh >= 1 && mh <= kMaxMh && c >= 1 && c <= 32; }

LongPlan long_plan(int mh, int64_t nh, int c, int elem_bytes, int mode, int num_cu)
{
    LongPlan p{};
    p.mhp = mh | 1;
    p.cm = c <= 8 ? 8 : (c <= 16 ? 16 : 32);
    p.rpt = (mh + kThreads - 1) / kThreads;
    p.kt = kKT;
    p.ntiles = (int)((nh + kKT - 1) / kKT);
    p.grid = std::max(1, std::min(p.ntiles, 2 * num_cu));
    const bool needs_q = (mode == kPower || mode == kProject);
    const int cg = p.cm / 8, slices = 16 / cg;
    p.lds = (size_t)kKT * p.mhp * elem_bytes + (size_t)kKT * p.cm * elem_bytes +
            (needs_q ? (size_t)mh * p.cm * elem_bytes + (size_t)slices * kKT * p.cm * elem_bytes : 0);
    return p;
}

template <typename T, bool TR, int MODE, int CM, int RPT>
__global__ void __launch_bounds__(kThreads) k_long(LongArgs<T> a)
{
    constexpr bool kNeedQ = (MODE == kPower || MODE == kProject);
    constexpr int kCG = CM / 8;          // groups of 8 columns
    constexpr int kS = 16 / kCG;         // row slices of phase 1
    constexpr int kPF = kKT * RPT;       // prefetch registers per thread (mh <= 256 RPT)
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tid = threadIdx.x;
    const int mh = a.mh, c = a.c, mhp = a.mhp;
    T *sTile = reinterpret_cast<T *>(smem_raw);
    T *sV = sTile + (size_t)kKT * mhp;
    T *sQ = sV + (size_t)kKT * CM;
    T *sZp = sQ + (size_t)mh * CM;

    for (int idx = tid; idx < kKT * CM; idx += kThreads) sV[idx] = T(0);
    if (kNeedQ) {
        for (int idx = tid; idx < mh * CM; idx += kThreads) {
            const int i = idx / CM, cc = idx % CM;
            sQ[idx] = cc < c ? a.Q[i + (int64_t)cc * a.ldq] : T(0);
        }
    }
    T acc[RPT][CM];
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int cc = 0; cc < CM; ++cc) acc[r][cc] = T(0);
    double gacc[4] = {0.0, 0.0, 0.0, 0.0};

    const int per_tile = kKT * mh;
    T pre[kPF];
    auto load_tile = [&](int tile) {
        const int64_t k0 = (int64_t)tile * kKT;
        const int64_t kval = min((int64_t)kKT, a.nh - k0);
#pragma unroll
        for (int j = 0; j < kPF; ++j) {
            const int e = tid + j * kThreads;
            T v = T(0);
            if (e < per_tile) {
                int kk, i;
                if (TR) {
                    kk = e % kKT;
                    i = e / kKT;
                } else {
                    i = e % mh;
                    kk = e / mh;
                }
                if (kk < kval) v = TR ? a.A[(k0 + kk) + (int64_t)i * a.lda] : a.A[i + (k0 + kk) * a.lda];
            }
            pre[j] = v;
        }
    };
    if ((int)blockIdx.x < a.ntiles) load_tile(blockIdx.x);

    for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x) {
        const int64_t k0 = (int64_t)tile * kKT;
        const int kval = (int)min((int64_t)kKT, a.nh - k0);
#pragma unroll
        for (int j = 0; j < kPF; ++j) {
            const int e = tid + j * kThreads;
            if (e < per_tile) {
                int kk, i;
                if (TR) {
                    kk = e % kKT;
                    i = e / kKT;
                } else {
                    i = e % mh;
                    kk = e / mh;
                }
                sTile[kk * mhp + i] = pre[j];
            }
        }
        if (MODE == kSketch) {
            const int npair = (c + 1) / 2;
            for (int idx = tid; idx < kKT * npair; idx += kThreads) {
                const int kk = idx % kKT, j = idx / kKT;
                double z0 = 0.0, z1 = 0.0;
                if (kk < kval) gaussian_pair(a.seed, a.counter, (uint32_t)(k0 + kk), (uint32_t)j, z0, z1);
                sV[kk * CM + 2 * j] = T(z0);
                if (2 * j + 1 < c) sV[kk * CM + 2 * j + 1] = T(z1);
            }
        } else if (MODE == kVecMul) {
            for (int idx = tid; idx < kKT * c; idx += kThreads) {
                const int kk = idx % kKT, cc = idx / kKT;
                sV[kk * CM + cc] = kk < kval ? a.V[(k0 + kk) + (int64_t)cc * a.ldv] : T(0);
            }
        }
        __syncthreads();
        if (tile + (int)gridDim.x < a.ntiles) load_tile(tile + gridDim.x);

        if (kNeedQ) {
            // phase 1
            const int kk = tid % kKT;
            const int cg = (tid / kKT) % kCG;
            const int s = tid / (kKT * kCG);
            T z[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) z[u] = T(0);
            const T *trow = sTile + kk * mhp;
            for (int i = s; i < mh; i += kS) {
                const T av = trow[i];
                const T *qr = sQ + i * CM + cg * 8;
#pragma unroll
                for (int u = 0; u < 8; ++u) z[u] += av * qr[u];
            }
            T *zp = sZp + ((size_t)s * kKT + kk) * CM + cg * 8;
#pragma unroll
            for (int u = 0; u < 8; ++u) zp[u] = z[u];
            __syncthreads();
            for (int idx = tid; idx < kKT * CM; idx += kThreads) {
                T t = T(0);
                for (int ss = 0; ss < kS; ++ss) t += sZp[(size_t)ss * kKT * CM + idx];
                sV[idx] = t;
            }
            __syncthreads();
        }
        if (MODE == kProject) {
            for (int idx = tid; idx < kKT * c; idx += kThreads) {
                const int kk = idx % kKT, cc = idx / kKT;
                if (kk < kval) a.Z[(k0 + kk) + (int64_t)cc * a.ldz] = sV[kk * CM + cc];
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int p = tid + e * kThreads;
                if (p < c * c) {
                    const int x = p % c, y = p / c;
                    double sum = 0.0;
#pragma unroll
                    for (int kk = 0; kk < kKT; ++kk) sum += (double)sV[kk * CM + x] * (double)sV[kk * CM + y];
                    gacc[e] += sum;
                }
            }
        } else {
            // phase 2
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int i = tid + r * kThreads;
                if (i < mh) {
#pragma unroll 4
                    for (int kk = 0; kk < kKT; ++kk) {
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
    if (p.rpt == 1)
        hipLaunchKernelGGL((k_long<T, TR, MODE, CM, 1>), dim3(p.grid), dim3(kThreads), p.lds, s, a);
    else
        hipLaunchKernelGGL((k_long<T, TR, MODE, CM, 2>), dim3(p.grid), dim3(kThreads), p.lds, s, a);
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
    if (!long_path_ok(a0.mh, a0.c) || p.rpt > 2) return hipErrorInvalidValue;
    LongArgs<T> a = a0;
    a.kt = p.kt;
    a.mhp = p.mhp;
    a.ntiles = p.ntiles;
    if (a.trans) return launch_long_mode<T, true>(p, mode, a, s);
    return launch_long_mode<T, false>(p, mode, a, s);
}
template hipError_t launch_long<double>(const LongPlan &, int, const LongArgs<double> &, hipStream_t);
template hipError_t launch_long<float>(const LongPlan &, int, const LongArgs<float> &, hipStream_t);

// ===========================================================================
// Fixed-order reductions: out[j] = sum_g part[g * count + j].
//   Columns: a 64 x 16 thread block; thread (x, y) sums the parts g = y,
//   y + 16, ... of output x; the 16 slices are then added in order.
//   Scalars (count small): all 1024 threads stride over the parts, then a
//   fixed tree.  Both orders are independent of timing, so results repeat
//   bit for bit.
// ===========================================================================
template <typename T>
__global__ void __launch_bounds__(1024) k_reduce_cols(const T *part, int64_t count, int nparts, T *out)
{
    __shared__ T red[16][65];
    const int x = threadIdx.x % 64, y = threadIdx.x / 64;
    const int64_t j = (int64_t)blockIdx.x * 64 + x;
    T s0 = T(0), s1 = T(0);
    if (j < count) {
        int g = y;
        for (; g + 16 < nparts; g += 32) {
            s0 += part[(int64_t)g * count + j];
            s1 += part[(int64_t)(g + 16) * count + j];
        }
        if (g < nparts) s0 += part[(int64_t)g * count + j];
    }
    red[y][x] = s0 + s1;
    __syncthreads();
    if (y == 0 && j < count) {
        T t = T(0);
        for (int yy = 0; yy < 16; ++yy) t += red[yy][x];
        out[j] = t;
    }
}

template <typename T>
__global__ void __launch_bounds__(1024) k_reduce_scalar(const T *part, int64_t count, int nparts, T *out)
{
    __shared__ double red[16];
    const int64_t j = blockIdx.x;
    double s = 0.0;
    for (int g = threadIdx.x; g < nparts; g += 1024) s += (double)part[(int64_t)g * count + j];
    s = wave_sum(s);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < 16; ++w) t += red[w];
        out[j] = (T)t;
    }
}

template <typename T>
hipError_t launch_reduce(const T *part, int64_t count, int nparts, T *out, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (count <= 8)
        hipLaunchKernelGGL((k_reduce_scalar<T>), dim3((unsigned)count), dim3(1024), 0, s, part, count, nparts, out);
    else
        hipLaunchKernelGGL((k_reduce_cols<T>), dim3((unsigned)((count + 63) / 64)), dim3(1024), 0, s, part, count, nparts, out);
    return hipGetLastError();
}
template hipError_t launch_reduce<double>(const double *, int64_t, int, double *, hipStream_t);
template hipError_t launch_reduce<float>(const float *, int64_t, int, float *, hipStream_t);

}  // namespace frk
