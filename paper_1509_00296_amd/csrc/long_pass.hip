// long_pass.hip -- passes over Ahat along its long dimension: the Gaussian
// sketch Y = Ahat Omega (Alg. 1's sampling steps), the fused power step
// Y = Ahat (Ahat^T Q) (its power iteration) and the projection B^T = Ahat^T Q
// with the Gram B B^T (its QR of A^T Q); plus the fixed-order split-K
// reductions.
#include "device_common.h"
#include "internal.h"

#include <algorithm>

namespace frk {

// ===========================================================================
// One workgroup (256 threads, 4 wavefronts) walks tiles of kKT = 16
// long-dimension indices; a tile holds the whole short dimension (mh <= 512,
// padded to whole 16-row blocks) in LDS as sT[i * LD + kk] (k contiguous per
// row).  The next tile is prefetched into registers while the current one is
// processed.  Both contractions run on the matrix cores (16x16x4 f64 / f32):
//
//  phase 1 (power, projection): Z(kk, j) = sum_i Ahat(i, k0+kk) Q(i, j).
//    Wavefront w takes the 4-row steps i0 = 4w, 4w + 16, ...; the four
//    partial 16 x 16 blocks are added in a fixed order through LDS.
//  phase 2 (sketch, power):     Y(i, j) += sum_kk Ahat(i, k0+kk) V(kk, j),
//    wavefront w owns the row blocks w, w + 4, ... and keeps their
//    accumulators in registers for the whole pass.
//  projection: B^T rows written out, the Gram B B^T accumulated in double.
// Columns beyond c and rows beyond mh are zero in LDS, so they contribute
// nothing; the output is written for i < mh, j < c only.
// ===========================================================================
constexpr int kKT = 16;
constexpr int kMaxMh = 512;

typedef __attribute__((__vector_size__(4 * sizeof(float)))) float lp_floatx4;
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double lp_doublex4;

template <typename T>
struct LpMfma;
template <>
struct LpMfma<double> {
    using V4 = lp_doublex4;
    static constexpr int kLD = 18;  // LDS row stride of the tile (144 bytes)
    __device__ static V4 mma(double a, double b, V4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    // row of D element r held by lane l
    __device__ static int drow(int l, int r) { return (l >> 4) + 4 * r; }
};
template <>
struct LpMfma<float> {
    using V4 = lp_floatx4;
    static constexpr int kLD = 20;  // 80 bytes
    __device__ static V4 mma(float a, float b, V4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int drow(int l, int r) { return 4 * (l >> 4) + r; }
};

bool long_path_ok(int mh, int c) { return mh >= 1 && mh <= kMaxMh && c >= 1 && c <= 32; }

int long_grid_cap(int num_cu) { return 3 * num_cu; }

LongPlan long_plan(int mh, int64_t nh, int c, int elem_bytes, int mode, int num_cu, bool trans)
{
    LongPlan p{};
    const int nrb = (mh + 15) / 16;
    p.mhp = nrb * 16;                      // padded rows
    p.cm = c <= 16 ? 16 : 32;              // padded columns (VLD)
    p.rpt = nrb <= 16 ? 4 : 8;             // row blocks per wavefront (phase 2)
    p.kt = kKT;
    p.ntiles = (int)((nh + kKT - 1) / kKT);
    // two workgroups per compute unit (three, where the registers allow it,
    // measured no faster on the transposed power and projection passes)
    (void)trans;
    p.grid = std::max(1, std::min(p.ntiles, 2 * num_cu));
    const bool needs_q = (mode == kPower || mode == kProject);
    const int ld = elem_bytes == 8 ? LpMfma<double>::kLD : LpMfma<float>::kLD;
    p.lds = (size_t)p.mhp * ld * elem_bytes + (size_t)kKT * p.cm * elem_bytes +
            (needs_q ? (size_t)p.mhp * p.cm * elem_bytes + (size_t)4 * kKT * p.cm * elem_bytes : 0);
    // vector-FMA form
    p.cmv = c <= 8 ? 8 : (c <= 16 ? 16 : 32);
    p.rptv = mh <= kThreads ? 1 : 2;
    const int gch = 96 / p.cmv, slices = 16 / (p.cmv / 8);
    p.ldsv = (size_t)p.mhp * ld * elem_bytes +
             (size_t)(mode == kSketch ? gch : 1) * kKT * p.cmv * elem_bytes +
             (needs_q ? (size_t)mh * p.cmv * elem_bytes + (size_t)slices * kKT * p.cmv * elem_bytes : 0);
    p.vec = 0;
    // transposed fast form: LDS = tile + V (or the Gaussian chunk) + phase-1 partials
    p.ldst = (size_t)(p.mhp + 1) * ld * elem_bytes +
             (size_t)(mode == kSketch ? 12 : 1) * kKT * p.cm * elem_bytes +
             (needs_q ? (size_t)4 * kKT * p.cm * elem_bytes : 0);
    return p;
}

template <typename T, bool TR, int MODE, int NB, int MAXRB>
__global__ void __launch_bounds__(kThreads) k_long(LongArgs<T> a)
{
    using M = LpMfma<T>;
    using V4 = typename M::V4;
    constexpr bool kNeedQ = (MODE == kPower || MODE == kProject);
    constexpr bool kPhase2 = (MODE != kProject);
    constexpr int LD = M::kLD;
    constexpr int VLD = 16 * NB;
    constexpr int kPF = kKT * 64 * MAXRB / kThreads;   // prefetch registers (>= 16 mh / 256)
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int mh = a.mh, c = a.c, mhp = a.mhp;
    const int nrb = mhp >> 4;
    T *sT = reinterpret_cast<T *>(smem_raw);
    T *sV = sT + (size_t)mhp * LD;
    T *sQ = sV + (size_t)kKT * VLD;
    T *sZp = sQ + (size_t)mhp * VLD;

    // padding rows of the tile stay zero; Q padded with zeros
    for (int idx = tid; idx < (mhp - mh) * LD; idx += kThreads) sT[(size_t)mh * LD + idx] = T(0);
    if (kNeedQ)
        for (int idx = tid; idx < mhp * VLD; idx += kThreads) {
            const int i = idx / VLD, j = idx % VLD;
            sQ[idx] = (i < mh && j < c) ? a.Q[i + (int64_t)j * a.ldq] : T(0);
        }
    V4 acc[MAXRB][NB];
#pragma unroll
    for (int r = 0; r < MAXRB; ++r)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[r][b] = V4{0, 0, 0, 0};
    double gacc[4] = {0.0, 0.0, 0.0, 0.0};

    const int per_tile = kKT * mh;
    const int npf = (per_tile + kThreads - 1) / kThreads;
    T pre[kPF];
    auto load_tile = [&](int tile) {
        const int64_t k0 = (int64_t)tile * kKT;
        const int64_t kval = min((int64_t)kKT, a.nh - k0);
#pragma unroll
        for (int j = 0; j < kPF; ++j) {
            T v = T(0);
            if (j < npf) {
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
                    if (kk < kval) v = TR ? a.A[(k0 + kk) + (int64_t)i * a.lda] : a.A[i + (k0 + kk) * a.lda];
                }
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
            if (j < npf) {
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
                    sT[i * LD + kk] = pre[j];
                }
            }
        }
        if (MODE == kSketch) {
            // pairs spread over the four wavefronts
            const int npair = (c + 1) / 2;
            for (int p = (tid & 3) * 64 + (tid >> 2); p < kKT * (VLD / 2); p += kThreads) {
                const int kk = p % kKT, j = p / kKT;
                double z0 = 0.0, z1 = 0.0;
                if (kk < kval && j < npair) gaussian_pair(a.seed, a.counter, (uint32_t)(k0 + kk), (uint32_t)j, z0, z1);
                sV[kk * VLD + 2 * j] = T(z0);
                sV[kk * VLD + 2 * j + 1] = (2 * j + 1 < c) ? T(z1) : T(0);
            }
        } else if (MODE == kVecMul) {
            for (int idx = tid; idx < kKT * VLD; idx += kThreads) {
                const int kk = idx % kKT, j = idx / kKT;
                sV[kk * VLD + j] = (kk < kval && j < c) ? a.V[(k0 + kk) + (int64_t)j * a.ldv] : T(0);
            }
        }
        __syncthreads();
        if (tile + (int)gridDim.x < a.ntiles) load_tile(tile + gridDim.x);

        if (kNeedQ) {
            // phase 1: Z = Ahat(:, tile)^T Q over this wavefront's 4-row steps
            V4 z[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) z[b] = V4{0, 0, 0, 0};
            const int kk = lane & 15, ko = lane >> 4;
            for (int i0 = 4 * wave; i0 < mhp; i0 += 16) {
                const T av = sT[(i0 + ko) * LD + kk];
#pragma unroll
                for (int b = 0; b < NB; ++b) z[b] = M::mma(av, sQ[(i0 + ko) * VLD + b * 16 + kk], z[b]);
            }
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    sZp[((size_t)wave * kKT + M::drow(lane, r)) * VLD + b * 16 + (lane & 15)] = z[b][r];
            __syncthreads();
            for (int idx = tid; idx < kKT * VLD; idx += kThreads) {
                const size_t st = (size_t)kKT * VLD;
                sV[idx] = ((sZp[idx] + sZp[st + idx]) + sZp[2 * st + idx]) + sZp[3 * st + idx];
            }
            __syncthreads();
        }
        if (MODE == kProject) {
            for (int idx = tid; idx < kKT * c; idx += kThreads) {
                const int kk = idx % kKT, j = idx / kKT;
                if (kk < kval) a.Z[(k0 + kk) + (int64_t)j * a.ldz] = sV[kk * VLD + j];
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int p = tid + e * kThreads;
                if (p < c * c) {
                    const int x = p % c, y = p / c;
                    double sum = 0.0;
#pragma unroll
                    for (int kk = 0; kk < kKT; ++kk) sum += (double)sV[kk * VLD + x] * (double)sV[kk * VLD + y];
                    gacc[e] += sum;
                }
            }
        }
        if (kPhase2) {
            // phase 2: Y(block rows) += Ahat(:, tile) V
#pragma unroll
            for (int r = 0; r < MAXRB; ++r) {
                const int rb = wave + 4 * r;
                if (rb < nrb) {
                    const int i = rb * 16 + (lane & 15);
#pragma unroll
                    for (int ks = 0; ks < kKT / 4; ++ks) {
                        const int kk = ks * 4 + (lane >> 4);
                        const T av = sT[i * LD + kk];
#pragma unroll
                        for (int b = 0; b < NB; ++b)
                            acc[r][b] = M::mma(av, sV[kk * VLD + b * 16 + (lane & 15)], acc[r][b]);
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
        for (int r = 0; r < MAXRB; ++r) {
            const int rb = wave + 4 * r;
            if (rb < nrb) {
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const int j = b * 16 + (lane & 15);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int i = rb * 16 + M::drow(lane, q);
                        if (i < mh && j < c) yp[i + (size_t)j * mh] = acc[r][b][q];
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Vector-FMA form of the same passes for narrow column counts (c <= 8 or
// 16), where the 16-column matrix-core tiles would waste half their work:
//  phase 1: thread (kk, column group of 8, row slice) sums its rows, four
//    rows per batch of LDS reads; the slices are added in a fixed order;
//  phase 2: one thread per short index i (RPT of them), KB long-dimension
//    indices per batch of LDS reads.
// The sketch draws the Gaussian columns of the workgroup's next GCH tiles in
// one go (overlapping the first tile's load) into LDS.
// ---------------------------------------------------------------------------
template <typename T, bool TR, int MODE, int CM, int RPT>
__global__ void __launch_bounds__(kThreads) k_long_v(LongArgs<T> a)
{
    constexpr bool kNeedQ = (MODE == kPower || MODE == kProject);
    constexpr bool kPhase2 = (MODE != kProject);
    constexpr int LD = LpMfma<T>::kLD;
    constexpr int kCG = CM / 8;
    constexpr int kS = 16 / kCG;
    constexpr int KB = CM == 8 ? 4 : (CM == 16 ? 2 : 1);
    constexpr int GCH = 96 / CM;
    constexpr int kPF = kKT * kThreads * RPT / kThreads;   // 16 RPT >= 16 mh / 256
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tid = threadIdx.x;
    const int mh = a.mh, c = a.c;
    T *sT = reinterpret_cast<T *>(smem_raw);
    T *sV = sT + (size_t)a.mhp * LD;                      // kKT x CM (or GCH x kKT x CM)
    T *sQ = sV + (size_t)(MODE == kSketch ? GCH : 1) * kKT * CM;
    T *sZp = sQ + (size_t)mh * CM;

    if (kNeedQ)
        for (int idx = tid; idx < mh * CM; idx += kThreads) {
            const int i = idx / CM, j = idx % CM;
            sQ[idx] = j < c ? a.Q[i + (int64_t)j * a.ldq] : T(0);
        }
    T acc[RPT][CM];
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
        for (int cc = 0; cc < CM; ++cc) acc[r][cc] = T(0);
    double gacc[4] = {0.0, 0.0, 0.0, 0.0};

    const int per_tile = kKT * mh;
    const int npf = (per_tile + kThreads - 1) / kThreads;
    T pre[kPF];
    auto load_tile = [&](int tile) {
        const int64_t k0 = (int64_t)tile * kKT;
        const int64_t kval = min((int64_t)kKT, a.nh - k0);
#pragma unroll
        for (int j = 0; j < kPF; ++j) {
            T v = T(0);
            if (j < npf) {
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
                    if (kk < kval) v = TR ? a.A[(k0 + kk) + (int64_t)i * a.lda] : a.A[i + (k0 + kk) * a.lda];
                }
            }
            pre[j] = v;
        }
    };
    // Gaussian columns of the tiles blockIdx + (t0 + g) gridDim, g < GCH
    auto draw = [&](int t0) {
        const int npair = (c + 1) / 2;
        for (int p = tid; p < GCH * kKT * (CM / 2); p += kThreads) {
            const int g = p / (kKT * (CM / 2)), rem = p % (kKT * (CM / 2));
            const int kk = rem % kKT, j = rem / kKT;
            const int64_t tile = (int64_t)blockIdx.x + (int64_t)(t0 + g) * gridDim.x;
            const int64_t k = tile * kKT + kk;
            double z0 = 0.0, z1 = 0.0;
            if (tile < a.ntiles && k < a.nh && j < npair)
                gaussian_pair(a.seed, a.counter, (uint32_t)k, (uint32_t)j, z0, z1);
            T *dst = sV + ((size_t)g * kKT + kk) * CM + 2 * j;
            dst[0] = T(z0);
            dst[1] = (2 * j + 1 < c) ? T(z1) : T(0);
        }
    };
    if ((int)blockIdx.x < a.ntiles) load_tile(blockIdx.x);
    if (MODE == kSketch) draw(0);

    int it = 0;
    for (int tile = blockIdx.x; tile < a.ntiles; tile += gridDim.x, ++it) {
        const int64_t k0 = (int64_t)tile * kKT;
        const int kval = (int)min((int64_t)kKT, a.nh - k0);
        if (MODE == kSketch && it > 0 && it % GCH == 0) draw(it);
#pragma unroll
        for (int j = 0; j < kPF; ++j) {
            if (j < npf) {
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
                    sT[i * LD + kk] = pre[j];
                }
            }
        }
        if (MODE == kVecMul) {
            for (int idx = tid; idx < kKT * CM; idx += kThreads) {
                const int kk = idx % kKT, j = idx / kKT;
                sV[kk * CM + j] = (kk < kval && j < c) ? a.V[(k0 + kk) + (int64_t)j * a.ldv] : T(0);
            }
        }
        __syncthreads();
        if (tile + (int)gridDim.x < a.ntiles) load_tile(tile + gridDim.x);

        if (kNeedQ) {
            const int kk = tid % kKT, cg = (tid / kKT) % kCG, sl = tid / (kKT * kCG);
            T z[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) z[u] = T(0);
            for (int i0 = sl; i0 < mh; i0 += 4 * kS) {
                T av[4], qv[4][8];
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int i = i0 + b * kS;
                    const bool ok = i < mh;
                    av[b] = ok ? sT[i * LD + kk] : T(0);
#pragma unroll
                    for (int u = 0; u < 8; ++u) qv[b][u] = ok ? sQ[i * CM + cg * 8 + u] : T(0);
                }
#pragma unroll
                for (int b = 0; b < 4; ++b)
#pragma unroll
                    for (int u = 0; u < 8; ++u) z[u] += av[b] * qv[b][u];
            }
            T *zp = sZp + ((size_t)sl * kKT + kk) * CM + cg * 8;
#pragma unroll
            for (int u = 0; u < 8; ++u) zp[u] = z[u];
            __syncthreads();
            for (int idx = tid; idx < kKT * CM; idx += kThreads) {
                T t[kS];
#pragma unroll
                for (int q = 0; q < kS; ++q) t[q] = sZp[(size_t)q * kKT * CM + idx];
                T sum = T(0);
#pragma unroll
                for (int q = 0; q < kS; ++q) sum += t[q];
                sV[idx] = sum;
            }
            __syncthreads();
        }
        if (MODE == kProject) {
            for (int idx = tid; idx < kKT * c; idx += kThreads) {
                const int kk = idx % kKT, j = idx / kKT;
                if (kk < kval) a.Z[(k0 + kk) + (int64_t)j * a.ldz] = sV[kk * CM + j];
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
        }
        if (kPhase2) {
            const T *vbase = sV + (MODE == kSketch ? (size_t)(it % GCH) * kKT * CM : 0);
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const int i = tid + r * kThreads;
                if (i < mh) {
                    const T *arow = sT + i * LD;
#pragma unroll
                    for (int k0b = 0; k0b < kKT; k0b += KB) {
                        T av[KB], vv[KB][CM];
#pragma unroll
                        for (int b = 0; b < KB; ++b) {
                            av[b] = arow[k0b + b];
#pragma unroll
                            for (int cc = 0; cc < CM; ++cc) vv[b][cc] = vbase[(k0b + b) * CM + cc];
                        }
#pragma unroll
                        for (int b = 0; b < KB; ++b)
#pragma unroll
                            for (int cc = 0; cc < CM; ++cc) acc[r][cc] += av[b] * vv[b][cc];
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

// ---------------------------------------------------------------------------
// Transposed orientation (Ahat = A^T, the long dimension contiguous in
// memory), mh <= 256.  The coalesced load of a tile -- 16 lanes over 16
// consecutive long indices of one column, four columns per instruction --
// is exactly the A-operand layout of phase 1 (M = kk, K = i), so phase 1 runs
// from the prefetch registers with Q's B-operand held in registers for the
// whole pass; the registers are also written to LDS for phase 2.  Loads are
// buffer loads with one per-thread offset and a per-tile offset; lanes past
// the end of the long dimension (or rows past mh) use an offset outside the
// buffer, which the hardware returns as zero.
// ---------------------------------------------------------------------------
constexpr uint32_t kOob = 0x80000000u;

template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

template <typename T, int MODE, int NB, int RING, int NJ>
__global__ void __launch_bounds__(kThreads) k_long_tr(LongArgs<T> a, uint32_t span_bytes)
{
    using M = LpMfma<T>;
    using V4 = typename M::V4;
    constexpr bool kNeedQ = (MODE == kPower || MODE == kProject);
    constexpr bool kPhase2 = (MODE != kProject);
    constexpr int LD = M::kLD;
    constexpr int VLD = 16 * NB;
    constexpr int GCH = 12;           // tiles per Gaussian chunk (sketch)
    constexpr uint32_t ESZ = sizeof(T);
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int mh = a.mh, c = a.c, mhp = a.mhp;
    const int nrb = mhp >> 4;
    const int nj = nrb;               // row groups present (i_j = (tid >> 4) + 16 j < mhp)
    T *sT = reinterpret_cast<T *>(smem_raw);
    // row mhp of the tile takes the stores of row groups past mhp
    T *sV = sT + (size_t)(mhp + 1) * LD;
    T *sZp = sV + (size_t)(MODE == kSketch ? GCH : 1) * kKT * VLD;

    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc((void *)a.A, (short)0, (int)span_bytes, 0x00020000);
    const int kk_l = tid & 15, r0 = tid >> 4;
    const uint32_t v0 = ((uint32_t)kk_l + (uint32_t)r0 * (uint32_t)a.lda) * ESZ;
    const uint32_t rowstep = 16u * (uint32_t)a.lda * ESZ;   // bytes between row groups
    // Q as the phase-1 B operand: row i_j, column b*16 + (lane & 15)
    T qreg[NJ][NB];
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int i = r0 + 16 * j, col = b * 16 + (lane & 15);
            qreg[j][b] = (kNeedQ && j < nj && i < mh && col < c) ? a.Q[i + (int64_t)col * a.ldq] : T(0);
        }
    V4 acc[4][NB];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[r][b] = V4{0, 0, 0, 0};
    double gacc[4] = {0.0, 0.0, 0.0, 0.0};

    // Register ring of RING tiles: while one is consumed, the loads of the
    // next RING - 1 are in flight.
    T pa[NJ], pb[NJ];
    auto load_tile = [&](T (&pre)[NJ], int tile) {
        const int64_t k0 = (int64_t)tile * kKT;
        const bool kin = k0 + kk_l < a.nh;
        const uint32_t vt = kin ? v0 + (uint32_t)k0 * ESZ : kOob;
        // every row group is loaded, groups past mhp and tiles past the end
        // through the out-of-range offset, so that the loads are
        // unconditional and the waits for them exact
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const bool jin = j < nj;
            const uint32_t vo = (jin && r0 + 16 * j < mh) ? vt : kOob;
            pre[j] = buf_load<T>(rsrc, vo, jin ? (uint32_t)j * rowstep : 0u);
        }
    };
    auto draw = [&](int t0) {
        const int npair = (c + 1) / 2;
        for (int p = tid; p < GCH * kKT * (VLD / 2); p += kThreads) {
            const int g = p / (kKT * (VLD / 2)), rem = p % (kKT * (VLD / 2));
            const int kk = rem % kKT, j = rem / kKT;
            const int64_t tile = (int64_t)blockIdx.x + (int64_t)(t0 + g) * gridDim.x;
            const int64_t k = tile * kKT + kk;
            double z0 = 0.0, z1 = 0.0;
            if (tile < a.ntiles && k < a.nh && j < npair)
                gaussian_pair(a.seed, a.counter, (uint32_t)k, (uint32_t)j, z0, z1);
            T *dst = sV + ((size_t)g * kKT + kk) * VLD + 2 * j;
            dst[0] = T(z0);
            dst[1] = (2 * j + 1 < c) ? T(z1) : T(0);
        }
    };
    load_tile(pa, blockIdx.x);
    // issue order pa, pb kept (the waits in the loop count on it)
    __builtin_amdgcn_sched_barrier(0);
    if (RING > 1) load_tile(pb, blockIdx.x + gridDim.x);
    if (MODE == kSketch) draw(0);
    if (MODE == kProject && a.om) {
        // Omega's rows for the next sketch, spread over the whole grid while
        // the first tiles load: item g is pair g % 4 of row g / 4
        for (int64_t g = (int64_t)blockIdx.x * kThreads + tid; g < 4 * a.nh; g += (int64_t)gridDim.x * kThreads) {
            const int64_t k = g >> 2;
            const int pp = (int)(g & 3);
            double z0 = 0.0, z1 = 0.0;
            if (2 * pp < a.om_c) gaussian_pair(a.seed, a.om_counter, (uint32_t)k, (uint32_t)pp, z0, z1);
            a.om[k * 8 + 2 * pp] = z0;
            a.om[k * 8 + 2 * pp + 1] = (2 * pp + 1 < a.om_c) ? z1 : 0.0;
        }
    }

    auto process = [&](T (&pre)[NJ], int tile, int it) {
        const int64_t k0 = (int64_t)tile * kKT;
        const int kval = (int)min((int64_t)kKT, a.nh - k0);
        if (MODE == kSketch && it > 0 && it % GCH == 0) draw(it);
        // branch-free over the NJ row groups (groups past nj hold zeros)
#pragma unroll
        for (int j = 0; j < NJ; ++j) sT[(j < nj ? r0 + 16 * j : mhp) * LD + kk_l] = pre[j];
        if (MODE == kVecMul) {
            for (int idx = tid; idx < kKT * VLD; idx += kThreads) {
                const int kk = idx % kKT, j = idx / kKT;
                sV[kk * VLD + j] = (kk < kval && j < c) ? a.V[(k0 + kk) + (int64_t)j * a.ldv] : T(0);
            }
        }
        if (!kNeedQ) load_tile(pre, tile + RING * gridDim.x);

        if (kNeedQ) {
            // phase 1 from registers: rows r0 + 16 j, two accumulation chains
            V4 z0[NB], z1[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                z0[b] = V4{0, 0, 0, 0};
                z1[b] = V4{0, 0, 0, 0};
            }
#pragma unroll
            for (int j = 0; j < NJ; j += 2) {
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    z0[b] = M::mma(pre[j], qreg[j][b], z0[b]);
                    if (j + 1 < NJ) z1[b] = M::mma(pre[j + 1], qreg[j + 1][b], z1[b]);
                }
            }
            // the registers are free once phase 1 has read them
            load_tile(pre, tile + RING * gridDim.x);
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    sZp[((size_t)wave * kKT + M::drow(lane, r)) * VLD + b * 16 + (lane & 15)] = z0[b][r] + z1[b][r];
            __syncthreads();
            for (int idx = tid; idx < kKT * VLD; idx += kThreads) {
                const size_t st = (size_t)kKT * VLD;
                sV[idx] = ((sZp[idx] + sZp[st + idx]) + sZp[2 * st + idx]) + sZp[3 * st + idx];
            }
        }
        __syncthreads();
        if (MODE == kProject) {
            for (int idx = tid; idx < kKT * c; idx += kThreads) {
                const int kk = idx % kKT, j = idx / kKT;
                if (kk < kval) a.Z[(k0 + kk) + (int64_t)j * a.ldz] = sV[kk * VLD + j];
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int p = tid + e * kThreads;
                if (p < c * c) {
                    const int x = p % c, y = p / c;
                    double sum = 0.0;
#pragma unroll
                    for (int kk = 0; kk < kKT; ++kk) sum += (double)sV[kk * VLD + x] * (double)sV[kk * VLD + y];
                    gacc[e] += sum;
                }
            }
        }
        if (kPhase2) {
            const T *vb = sV + (MODE == kSketch ? (size_t)(it % GCH) * kKT * VLD : 0);
            T bv[4][NB];
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                for (int b = 0; b < NB; ++b) bv[ks][b] = vb[(ks * 4 + (lane >> 4)) * VLD + b * 16 + (lane & 15)];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int rb = wave + 4 * r;
                if (rb < nrb) {
                    const int i = rb * 16 + (lane & 15);
#pragma unroll
                    for (int ks = 0; ks < 4; ++ks) {
                        const T av = sT[i * LD + ks * 4 + (lane >> 4)];
#pragma unroll
                        for (int b = 0; b < NB; ++b) acc[r][b] = M::mma(av, bv[ks][b], acc[r][b]);
                    }
                }
            }
        }
        __syncthreads();
    };
    // One exit: the second tile of a pair is processed even past the end
    // (its loads return zeros, its outputs are masked), so that every
    // iteration leaves the loads in the same order.
    int it = 0;
    for (int tile = blockIdx.x; tile < a.ntiles; tile += RING * gridDim.x) {
        process(pa, tile, it++);
        if (RING > 1) process(pb, tile + gridDim.x, it++);
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
        for (int r = 0; r < 4; ++r) {
            const int rb = wave + 4 * r;
            if (rb < nrb) {
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const int j = b * 16 + (lane & 15);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int i = rb * 16 + M::drow(lane, q);
                        if (i < mh && j < c) yp[i + (size_t)j * mh] = acc[r][b][q];
                    }
                }
            }
        }
    }
}

template <typename T, bool TR, int MODE, int NB>
static hipError_t launch_long_rb(const LongPlan &p, const LongArgs<T> &a, hipStream_t s)
{
    if (p.rpt == 4)
        hipLaunchKernelGGL((k_long<T, TR, MODE, NB, 4>), dim3(p.grid), dim3(kThreads), p.lds, s, a);
    else
        hipLaunchKernelGGL((k_long<T, TR, MODE, NB, 8>), dim3(p.grid), dim3(kThreads), p.lds, s, a);
    return hipGetLastError();
}

template <typename T, bool TR, int MODE, int CM>
static hipError_t launch_long_v(const LongPlan &p, const LongArgs<T> &a, hipStream_t s)
{
    if (p.rptv == 1)
        hipLaunchKernelGGL((k_long_v<T, TR, MODE, CM, 1>), dim3(p.grid), dim3(kThreads), p.ldsv, s, a);
    else
        hipLaunchKernelGGL((k_long_v<T, TR, MODE, CM, 2>), dim3(p.grid), dim3(kThreads), p.ldsv, s, a);
    return hipGetLastError();
}

template <typename T, bool TR, int MODE>
static hipError_t launch_long_cm(const LongPlan &p, const LongArgs<T> &a, hipStream_t s)
{
    if (p.vec) {
        if (p.cmv == 8) return launch_long_v<T, TR, MODE, 8>(p, a, s);
        if (p.cmv == 16) return launch_long_v<T, TR, MODE, 16>(p, a, s);
        return launch_long_v<T, TR, MODE, 32>(p, a, s);
    }
    if (p.cm == 16) return launch_long_rb<T, TR, MODE, 1>(p, a, s);
    return launch_long_rb<T, TR, MODE, 2>(p, a, s);
}

template <typename T, int MODE>
static hipError_t launch_long_tr(const LongPlan &p, const LongArgs<T> &a, uint32_t span, hipStream_t s)
{
    // NJ row groups of 16 per thread: 8 for mhp <= 128, 13 for mhp <= 208
    // (no phase-1 products of empty row groups), else 16
    const bool nj8 = p.mhp <= 128;
    if (p.cm == 16 && nj8)
        hipLaunchKernelGGL((k_long_tr<T, MODE, 1, 2, 8>), dim3(p.grid), dim3(kThreads), p.ldst, s, a, span);
    else if (p.cm == 16 && p.mhp <= 208)
        hipLaunchKernelGGL((k_long_tr<T, MODE, 1, 2, 13>), dim3(p.grid), dim3(kThreads), p.ldst, s, a, span);
    else if (p.cm == 16)
        hipLaunchKernelGGL((k_long_tr<T, MODE, 1, 2, 16>), dim3(p.grid), dim3(kThreads), p.ldst, s, a, span);
    else if (nj8)
        hipLaunchKernelGGL((k_long_tr<T, MODE, 2, 1, 8>), dim3(p.grid), dim3(kThreads), p.ldst, s, a, span);
    else
        hipLaunchKernelGGL((k_long_tr<T, MODE, 2, 1, 16>), dim3(p.grid), dim3(kThreads), p.ldst, s, a, span);
    return hipGetLastError();
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
    if (!long_path_ok(a0.mh, a0.c) || p.mhp < a0.mh || p.mhp > kMaxMh || p.cm < a0.c ||
        (p.rpt != 4 && p.rpt != 8) || 4 * p.rpt * 16 < p.mhp)
        return hipErrorInvalidValue;
    if (p.vec && (p.cmv < a0.c || (p.cmv != 8 && p.cmv != 16 && p.cmv != 32) || p.rptv < 1 ||
                  p.rptv > 2 || p.rptv * kThreads < a0.mh))
        return hipErrorInvalidValue;
    LongArgs<T> a = a0;
    a.kt = p.kt;
    a.mhp = p.mhp;
    a.ntiles = p.ntiles;
    if (a.trans && p.mhp <= 256 && !p.vec) {
        // byte span of A touched: rows (long index) < nh of columns < mh
        const uint64_t span = ((uint64_t)(a.nh - 1) + (uint64_t)(a.mh - 1) * (uint64_t)a.lda + 1) * sizeof(T);
        const uint64_t rows16 = (uint64_t)16 * (uint64_t)a.lda * sizeof(T) * (uint64_t)(p.mhp / 16);
        if (span < kOob && rows16 < kOob) {
            switch (mode) {
            case kSketch: return launch_long_tr<T, kSketch>(p, a, (uint32_t)span, s);
            case kVecMul: return launch_long_tr<T, kVecMul>(p, a, (uint32_t)span, s);
            case kPower: return launch_long_tr<T, kPower>(p, a, (uint32_t)span, s);
            default: return launch_long_tr<T, kProject>(p, a, (uint32_t)span, s);
            }
        }
    }
    hipError_t e = a.trans ? launch_long_mode<T, true>(p, mode, a, s) : launch_long_mode<T, false>(p, mode, a, s);
    // the other forms leave Omega's rows to a pass of their own
    if (e == hipSuccess && mode == kProject && a.om)
        e = launch_omega_rows(a.nh, a.om_c, a.seed, a.om_counter, a.om, s);
    return e;
}
template hipError_t launch_long<double>(const LongPlan &, int, const LongArgs<double> &, hipStream_t);
template hipError_t launch_long<float>(const LongPlan &, int, const LongArgs<float> &, hipStream_t);

// ===========================================================================
// Gram G = Ahat Ahat^T (mh x mh, double) in the transposed orientation (the
// long dimension contiguous), mh <= 16 NRB <= 256: the Gram behind ||O||_2.
// One workgroup per compute unit streams tiles of 16 long indices x mh rows
// with buffer loads (the next tile in registers while the current one is
// used; rows past mh and indices past nh read as zero), stores the tile to
// LDS and accumulates the upper 16 x 16 blocks (I <= J) on the matrix cores:
// wavefront w owns the blocks w, w + 4, ... for the whole pass, four
// 16x16x4 steps per tile (K = the tile's long indices).  Each workgroup
// writes its blocks as one partial (block b, MFMA register r, lane l at
// (b * 4 + r) * 64 + l); the fixed-order reduction adds the partials and
// k_gram_scatter places the sum in both triangles of G.
// ===========================================================================
__host__ __device__ constexpr int gram_nblk(int nrb) { return nrb * (nrb + 1) / 2; }

template <typename T, int NRB>
__global__ void __launch_bounds__(kThreads) k_gram_tr(const T *A, int64_t lda, int mh, int64_t nh, int ntiles,
                                                      uint32_t span_bytes, double *part)
{
    constexpr int NBLK = gram_nblk(NRB);
    constexpr int NPW = (NBLK + 3) / 4;
    constexpr int LD = 17;  // LDS row stride in doubles (odd: operand reads spread over the banks)
    constexpr uint32_t ESZ = sizeof(T);
    typedef __attribute__((__vector_size__(4 * sizeof(double)))) double d4;
    __shared__ double sT[16 * NRB * LD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc((void *)A, (short)0, (int)span_bytes, 0x00020000);
    const int kk_l = tid & 15, r0 = tid >> 4;
    const uint32_t v0 = ((uint32_t)kk_l + (uint32_t)r0 * (uint32_t)lda) * ESZ;
    const uint32_t rowstep = 16u * (uint32_t)lda * ESZ;
    // this wavefront's blocks (I, J), I <= J, in row-major order of the
    // upper block triangle
    int bi[NPW], bj[NPW];
#pragma unroll
    for (int q = 0; q < NPW; ++q) {
        int b = wave + 4 * q, I = 0;
        if (b >= NBLK) b = 0;
        while (b >= NRB - I) {
            b -= NRB - I;
            ++I;
        }
        bi[q] = I;
        bj[q] = I + b;
    }
    d4 acc[NPW];
#pragma unroll
    for (int q = 0; q < NPW; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
    T pre[NRB];
    auto load_tile = [&](int tile) {
        const int64_t k0 = (int64_t)tile * kKT;
        const uint32_t vt = (k0 + kk_l < nh) ? v0 + (uint32_t)k0 * ESZ : kOob;
#pragma unroll
        for (int j = 0; j < NRB; ++j) pre[j] = buf_load<T>(rsrc, (r0 + 16 * j < mh) ? vt : kOob, (uint32_t)j * rowstep);
    };
    if ((int)blockIdx.x < ntiles) load_tile(blockIdx.x);
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
#pragma unroll
        for (int j = 0; j < NRB; ++j) sT[(r0 + 16 * j) * LD + kk_l] = (double)pre[j];
        __syncthreads();
        if (tile + (int)gridDim.x < ntiles) load_tile(tile + gridDim.x);
#pragma unroll
        for (int q = 0; q < NPW; ++q) {
            if (wave + 4 * q < NBLK) {
                const double *ra = sT + (bi[q] * 16 + (lane & 15)) * LD + (lane >> 4);
                const double *rb = sT + (bj[q] * 16 + (lane & 15)) * LD + (lane >> 4);
#pragma unroll
                for (int k4 = 0; k4 < kKT; k4 += 4)
                    acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(ra[k4], rb[k4], acc[q], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    double *pp = part + (size_t)blockIdx.x * NBLK * 256;
#pragma unroll
    for (int q = 0; q < NPW; ++q) {
        const int b = wave + 4 * q;
        if (b < NBLK)
#pragma unroll
            for (int r = 0; r < 4; ++r) pp[(size_t)(b * 4 + r) * 64 + lane] = acc[q][r];
    }
}

// G (mh x mh, column-major) from the summed blocks of k_gram_tr: entry
// (b, r, l) is row 16 I + (l >> 4) + 4 r, column 16 J + (l & 15) of block
// b = (I, J), and its mirror.
__global__ void k_gram_scatter(const double *sum, int nrb, int mh, double *G)
{
    const int nblk = gram_nblk(nrb);
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nblk * 256) return;
    int b = idx / 256, I = 0;
    const int r = (idx / 64) % 4, l = idx % 64;
    while (b >= nrb - I) {
        b -= nrb - I;
        ++I;
    }
    const int J = I + b;
    const int row = 16 * I + (l >> 4) + 4 * r, col = 16 * J + (l & 15);
    if (row < mh && col < mh) {
        const double v = sum[idx];
        G[row + (size_t)col * mh] = v;
        G[col + (size_t)row * mh] = v;
    }
}

bool gram_tr_ok(int mh, int64_t nh, int64_t lda, int elem_bytes)
{
    if (mh < 1 || mh > 256 || nh < 1 || lda < nh) return false;
    const uint64_t span = ((uint64_t)(nh - 1) + (uint64_t)(mh - 1) * (uint64_t)lda + 1) * (uint64_t)elem_bytes;
    const uint64_t rows = (uint64_t)16 * (uint64_t)lda * (uint64_t)elem_bytes * 16;
    return span < kOob && rows < kOob;
}

size_t gram_tr_part_doubles(int mh, int grid) { return (size_t)grid * gram_nblk((mh + 15) / 16) * 256; }

template <typename T, int NRB>
static hipError_t launch_gram_tr_nrb(const T *A, int64_t lda, int mh, int64_t nh, int grid, double *part,
                                     double *sum, double *G, hipStream_t s)
{
    const int ntiles = (int)((nh + kKT - 1) / kKT);
    const uint32_t span = (uint32_t)(((uint64_t)(nh - 1) + (uint64_t)(mh - 1) * (uint64_t)lda + 1) * sizeof(T));
    hipLaunchKernelGGL((k_gram_tr<T, NRB>), dim3(grid), dim3(kThreads), 0, s, A, lda, mh, nh, ntiles, span, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int count = gram_nblk(NRB) * 256;
    if ((e = launch_reduce<double>(part, count, grid, sum, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_gram_scatter, dim3((count + 255) / 256), dim3(256), 0, s, sum, NRB, mh, G);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gram_tr(const T *A, int64_t lda, int mh, int64_t nh, int grid, double *part, double *sum,
                          double *G, hipStream_t s)
{
    if (!gram_tr_ok(mh, nh, lda, sizeof(T)) || grid < 1) return hipErrorInvalidValue;
    const int nrb = (mh + 15) / 16;
    if (nrb <= 4) return launch_gram_tr_nrb<T, 4>(A, lda, mh, nh, grid, part, sum, G, s);
    if (nrb <= 8) return launch_gram_tr_nrb<T, 8>(A, lda, mh, nh, grid, part, sum, G, s);
    if (nrb <= 13) return launch_gram_tr_nrb<T, 13>(A, lda, mh, nh, grid, part, sum, G, s);
    return launch_gram_tr_nrb<T, 16>(A, lda, mh, nh, grid, part, sum, G, s);
}
template hipError_t launch_gram_tr<double>(const double *, int64_t, int, int64_t, int, double *, double *, double *,
                                           hipStream_t);
template hipError_t launch_gram_tr<float>(const float *, int64_t, int, int64_t, int, double *, double *, double *,
                                          hipStream_t);

// ===========================================================================
// Fixed-order reductions: out[j] = sum_g part[g * count + j].
//   Columns: a W x (1024 / W) thread block; thread (x, y) sums the parts
//   g = y, y + S, ... (S = 1024 / W) of output x in eight interleaved partial
//   sums (added in a fixed tree); the S slices are then added by a pairwise
//   tree in LDS.  W is 64, 16 or 4 by the output count, so that narrow
//   outputs over many parts still spread over enough workgroups and each
//   thread issues only a batch or two of loads.
//   Scalars (count small): all 1024 threads stride over the parts, then a
//   fixed tree.  Both orders are independent of timing, so results repeat
//   bit for bit.
// ===========================================================================
template <typename T, int W>
__global__ void __launch_bounds__(1024) k_reduce_cols(const T *part, int64_t count, int nparts, T *out)
{
    constexpr int S = 1024 / W;
    __shared__ T red[S][W + 1];
    const int x = threadIdx.x % W, y = threadIdx.x / W;
    const int64_t j = (int64_t)blockIdx.x * W + x;
    // eight independent partial sums (parts g + S k), their loads issued
    // together
    T acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = T(0);
    if (j < count) {
        int g = y;
        for (; g + 7 * S < nparts; g += 8 * S) {
            T v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = part[(int64_t)(g + S * k) * count + j];
#pragma unroll
            for (int k = 0; k < 8; ++k) acc[k] += v[k];
        }
        for (; g < nparts; g += S) acc[0] += part[(int64_t)g * count + j];
    }
    red[y][x] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    __syncthreads();
#pragma unroll
    for (int h = S / 2; h > 0; h >>= 1) {
        if (y < h) red[y][x] += red[y + h][x];
        __syncthreads();
    }
    if (y == 0 && j < count) out[j] = red[0][x];
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

// The RPCA iteration's last step: the residual partials summed as
// k_reduce_scalar does (same order, same result), written with the first
// nstatus status words straight to mapped host memory, so that the host
// reads them after an event without a copy on the stream.
__global__ void __launch_bounds__(1024) k_finish_iter(const double *part, int nparts, const int *status,
                                                      int nstatus, int *host_status, double *host_z,
                                                      const double *res, double *host_res, int *host_seq,
                                                      int seq)
{
    __shared__ double red[16];
    double s = 0.0;
    for (int g = threadIdx.x; g < nparts; g += 1024) s += part[g];
    s = wave_sum(s);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < 16; ++w) t += red[w];
        for (int i = 0; i < nstatus; ++i) host_status[i] = status[i];
        *host_z = t;
        if (host_res) *host_res = res ? *res : -1.0;
        __threadfence_system();
        // the sequence number last: a host that sees it sees the words above
        if (host_seq) {
            *(volatile int *)host_seq = seq;
            __threadfence_system();
        }
    }
}

hipError_t launch_finish_iter(const double *part, int nparts, const int *status, int nstatus,
                              int *host_status, double *host_z, const double *res, double *host_res,
                              hipStream_t s, int *host_seq, int seq)
{
    hipLaunchKernelGGL(k_finish_iter, dim3(1), dim3(1024), 0, s, part, nparts, status, nstatus, host_status, host_z,
                       res, host_res, host_seq, seq);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_reduce(const T *part, int64_t count, int nparts, T *out, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    if (count <= 8)
        hipLaunchKernelGGL((k_reduce_scalar<T>), dim3((unsigned)count), dim3(1024), 0, s, part, count, nparts, out);
    else if (count >= 64 * 256)
        hipLaunchKernelGGL((k_reduce_cols<T, 64>), dim3((unsigned)((count + 63) / 64)), dim3(1024), 0, s, part, count,
                           nparts, out);
    else if (count >= 16 * 64)
        hipLaunchKernelGGL((k_reduce_cols<T, 16>), dim3((unsigned)((count + 15) / 16)), dim3(1024), 0, s, part, count,
                           nparts, out);
    else
        hipLaunchKernelGGL((k_reduce_cols<T, 4>), dim3((unsigned)((count + 3) / 4)), dim3(1024), 0, s, part, count,
                           nparts, out);
    return hipGetLastError();
}
template hipError_t launch_reduce<double>(const double *, int64_t, int, double *, hipStream_t);
template hipError_t launch_reduce<float>(const float *, int64_t, int, float *, hipStream_t);

}  // namespace frk
