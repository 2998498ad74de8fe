// gemm_mfma.hip -- matrix-core GEMMs for the large path: the bfloat16 sketch
// and power products of the precision form (float accumulation), float
// projection/reconstruction, and double products, all as
//   C(m, n) = sum_k A(m, k) B(k, n)
// with arbitrary element strides (one of each operand's strides must be 1).
//
// gfx950 matrix instructions (lane layouts checked on the device):
//   v_mfma_f32_16x16x32_bf16 : A lane l = row l%16, k 8(l/16)..+7 (8 bf16);
//                              B lane l = col l%16, same k; D lane l = col l%16,
//                              rows 4(l/16)+i.
//   v_mfma_f32_16x16x4f32    : A row l%16, k l/16; B col l%16, k l/16;
//                              D col l%16, rows 4(l/16)+i.
//   v_mfma_f64_16x16x4f64    : as f32 for A and B; D col l%16, rows (l/16)+4i.
// Workgroup tile BM x BN, 4 wavefronts in a 2 x 2 arrangement; operand tiles
// are staged in LDS with k contiguous (As[m][k], Bs[n][k]); a tile whose
// global layout is not k-contiguous is transposed on its way into LDS.
#include "device_common.h"
#include "internal.h"

#include <algorithm>

namespace frk {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4_t;
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double doublex4_t;

template <typename TI>
struct MfmaTraits;
template <>
struct MfmaTraits<uint16_t> {  // bfloat16 bits
    using Acc = float;
    using AccV = floatx4_t;
    static constexpr int kVec = 8;     // elements per 16-byte vector
    static constexpr int kBK = 32;     // k per LDS stage
    static constexpr int kKStep = 32;  // k per instruction
    static constexpr int kPad = 8;
    static constexpr bool kRowsInterleaved = false;
};
template <>
struct MfmaTraits<float> {
    using Acc = float;
    using AccV = floatx4_t;
    static constexpr int kVec = 4;
    static constexpr int kBK = 16;
    static constexpr int kKStep = 4;
    static constexpr int kPad = 4;
    static constexpr bool kRowsInterleaved = false;
};
template <>
struct MfmaTraits<double> {
    using Acc = double;
    using AccV = doublex4_t;
    static constexpr int kVec = 2;
    static constexpr int kBK = 16;
    static constexpr int kKStep = 4;
    static constexpr int kPad = 2;
    static constexpr bool kRowsInterleaved = true;
};

template <typename TI>
struct Vec16 {
    TI v[16 / sizeof(TI)];
};

// Stage a rows x kBK operand tile (global element (r, k) at P[r*sr + k*sk])
// into LDS T[r * ldt + k], zero outside [0, rmax) x [k0, kend).
template <typename TI, int ROWS>
__device__ __forceinline__ void stage_tile(const TI *__restrict__ P, int64_t sr, int64_t sk,
                                           int64_t r0, int64_t rmax, int64_t k0, int64_t kend,
                                           TI *T, int ldt)
{
    constexpr int V = MfmaTraits<TI>::kVec, BK = MfmaTraits<TI>::kBK;
    if (sk == 1) {
        constexpr int slots = ROWS * (BK / V);
        for (int s = threadIdx.x; s < slots; s += kThreads) {
            const int r = s / (BK / V), kv = (s % (BK / V)) * V;
            const int64_t gr = r0 + r, gk = k0 + kv;
            TI *dst = T + r * ldt + kv;
            const TI *src = P + gr * sr + gk;
            if (gr < rmax && gk + V <= kend && ((uintptr_t)src % 16) == 0) {
                *reinterpret_cast<Vec16<TI> *>(dst) = *reinterpret_cast<const Vec16<TI> *>(src);
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e) dst[e] = (gr < rmax && gk + e < kend) ? P[gr * sr + gk + e] : TI(0);
            }
        }
    } else {
        // rows contiguous (sr == 1): vectors along r, transposed into LDS
        constexpr int slots = (ROWS / V) * BK;
        for (int s = threadIdx.x; s < slots; s += kThreads) {
            const int rv = (s % (ROWS / V)) * V, k = s / (ROWS / V);
            const int64_t gr = r0 + rv, gk = k0 + k;
            const TI *src = P + gr + gk * sk;
            TI tmp[V];
            if (gk < kend && gr + V <= rmax && ((uintptr_t)src % 16) == 0) {
                const Vec16<TI> v = *reinterpret_cast<const Vec16<TI> *>(src);
#pragma unroll
                for (int e = 0; e < V; ++e) tmp[e] = v.v[e];
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e) tmp[e] = (gk < kend && gr + e < rmax) ? P[(gr + e) + gk * sk] : TI(0);
            }
#pragma unroll
            for (int e = 0; e < V; ++e) T[(rv + e) * ldt + k] = tmp[e];
        }
    }
}

template <typename TI>
__device__ __forceinline__ typename MfmaTraits<TI>::AccV mfma_step(const TI *As, const TI *Bs, int ldt,
                                                                   int arow, int bcol, int kk,
                                                                   typename MfmaTraits<TI>::AccV acc);

template <>
__device__ __forceinline__ floatx4_t mfma_step<uint16_t>(const uint16_t *As, const uint16_t *Bs, int ldt,
                                                         int arow, int bcol, int kk, floatx4_t acc)
{
    const int lane = threadIdx.x % kWave;
    const int ko = kk + 8 * (lane / 16);
    const bf16x8_t a = *reinterpret_cast<const bf16x8_t *>(As + (arow + lane % 16) * ldt + ko);
    const bf16x8_t b = *reinterpret_cast<const bf16x8_t *>(Bs + (bcol + lane % 16) * ldt + ko);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
}

template <>
__device__ __forceinline__ floatx4_t mfma_step<float>(const float *As, const float *Bs, int ldt, int arow,
                                                      int bcol, int kk, floatx4_t acc)
{
    const int lane = threadIdx.x % kWave;
    const int ko = kk + lane / 16;
    return __builtin_amdgcn_mfma_f32_16x16x4f32(As[(arow + lane % 16) * ldt + ko],
                                                Bs[(bcol + lane % 16) * ldt + ko], acc, 0, 0, 0);
}

template <>
__device__ __forceinline__ doublex4_t mfma_step<double>(const double *As, const double *Bs, int ldt,
                                                        int arow, int bcol, int kk, doublex4_t acc)
{
    const int lane = threadIdx.x % kWave;
    const int ko = kk + lane / 16;
    return __builtin_amdgcn_mfma_f64_16x16x4f64(As[(arow + lane % 16) * ldt + ko],
                                                Bs[(bcol + lane % 16) * ldt + ko], acc, 0, 0, 0);
}

template <typename TI, typename TO, int BM, int BN, bool DIRECT>
__global__ void __launch_bounds__(kThreads) k_mfma_gemm(int64_t M, int64_t N, int64_t K, const TI *A,
                                                        int64_t sam, int64_t sak, const TI *B,
                                                        int64_t sbk, int64_t sbn, TO *C, int64_t scm,
                                                        int64_t scn, int64_t kchunk,
                                                        typename MfmaTraits<TI>::Acc *part)
{
    using Tr = MfmaTraits<TI>;
    using Acc = typename Tr::Acc;
    using AccV = typename Tr::AccV;
    constexpr int BK = Tr::kBK, LDT = BK + Tr::kPad;
    constexpr int WM = BM / 2, WN = BN / 2;        // wavefront sub-tile
    constexpr int FM = WM / 16, FN = WN / 16;      // 16 x 16 blocks per wavefront
    __shared__ __align__(16) TI As[BM * LDT];
    __shared__ __align__(16) TI Bs[BN * LDT];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int wm = (wave % 2) * WM, wn = (wave / 2) * WN;
    const int64_t m0 = (int64_t)blockIdx.x * BM, n0 = (int64_t)blockIdx.y * BN;
    const int64_t kb = (int64_t)blockIdx.z * kchunk, ke = min(K, kb + kchunk);
    AccV acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[i][j][e] = Acc(0);

    for (int64_t k0 = kb; k0 < ke; k0 += BK) {
        stage_tile<TI, BM>(A, sam, sak, m0, M, k0, ke, As, LDT);
        // B(k, n) = B[k*sbk + n*sbn]: rows of the staged tile are n
        stage_tile<TI, BN>(B, sbn, sbk, n0, N, k0, ke, Bs, LDT);
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; kk += Tr::kKStep)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = mfma_step<TI>(As, Bs, LDT, wm + 16 * i, wn + 16 * j, kk, acc[i][j]);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = Tr::kRowsInterleaved ? (lane / 16) + 4 * e : 4 * (lane / 16) + e;
                const int64_t gm = m0 + wm + 16 * i + row, gn = n0 + wn + 16 * j + lane % 16;
                if (gm < M && gn < N) {
                    if (DIRECT) C[gm * scm + gn * scn] = (TO)acc[i][j][e];
                    else part[(int64_t)blockIdx.z * M * N + gm + gn * M] = acc[i][j][e];
                }
            }
}

template <typename TA, typename TO>
__global__ void __launch_bounds__(kThreads) k_mfma_store(int64_t M, int64_t N, int splitk, const TA *part,
                                                         TO *C, int64_t scm, int64_t scn)
{
    const int64_t total = M * N;
    for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * kThreads) {
        TA s = TA(0);
        for (int z = 0; z < splitk; ++z) s += part[(int64_t)z * total + idx];
        C[(idx % M) * scm + (idx / M) * scn] = (TO)s;
    }
}

template <typename TI, typename TO, int BM, int BN>
static hipError_t launch_tiles(int64_t M, int64_t N, int64_t K, const TI *A, int64_t sam, int64_t sak,
                               const TI *B, int64_t sbk, int64_t sbn, TO *C, int64_t scm, int64_t scn,
                               int splitk, typename MfmaTraits<TI>::Acc *part, hipStream_t s)
{
    using Acc = typename MfmaTraits<TI>::Acc;
    constexpr int BK = MfmaTraits<TI>::kBK;
    int64_t kchunk = (K + splitk - 1) / splitk;
    kchunk = std::max<int64_t>(BK, ((kchunk + BK - 1) / BK) * BK);
    const int sk = (int)std::max<int64_t>(1, (K + kchunk - 1) / kchunk);
    dim3 grid((unsigned)((M + BM - 1) / BM), (unsigned)((N + BN - 1) / BN), (unsigned)sk);
    if (sk == 1 || part == nullptr) {
        if (sk != 1) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_mfma_gemm<TI, TO, BM, BN, true>), grid, dim3(kThreads), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, C, scm, scn, kchunk, part);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((k_mfma_gemm<TI, TO, BM, BN, false>), grid, dim3(kThreads), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, C, scm, scn, kchunk, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t total = M * N;
    const int g2 = (int)std::min<int64_t>(8192, (total + kThreads - 1) / kThreads);
    hipLaunchKernelGGL((k_mfma_store<Acc, TO>), dim3(g2), dim3(kThreads), 0, s, M, N, sk, part, C, scm, scn);
    return hipGetLastError();
}

bool mfma_operand_ok(int64_t s_row, int64_t s_k) { return s_row == 1 || s_k == 1; }

template <typename TI, typename TO>
hipError_t launch_mfma_gemm(int64_t M, int64_t N, int64_t K, const TI *A, int64_t sam, int64_t sak,
                            const TI *B, int64_t sbk, int64_t sbn, TO *C, int64_t scm, int64_t scn,
                            int splitk, typename MfmaTraits<TI>::Acc *part, hipStream_t s)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    if (!mfma_operand_ok(sam, sak) || !mfma_operand_ok(sbn, sbk)) return hipErrorInvalidValue;
    if (N <= 32) return launch_tiles<TI, TO, 64, 32>(M, N, K, A, sam, sak, B, sbk, sbn, C, scm, scn, splitk, part, s);
    if (N <= 128 && M >= 4 * N) return launch_tiles<TI, TO, 32, 128>(M, N, K, A, sam, sak, B, sbk, sbn, C, scm, scn, splitk, part, s);
    return launch_tiles<TI, TO, 64, 64>(M, N, K, A, sam, sak, B, sbk, sbn, C, scm, scn, splitk, part, s);
}

// explicit instantiations used by the host code
hipError_t launch_gemm_bf16(int64_t M, int64_t N, int64_t K, const uint16_t *A, int64_t sam,
                            int64_t sak, const uint16_t *B, int64_t sbk, int64_t sbn, float *C,
                            int64_t scm, int64_t scn, int splitk, float *part, hipStream_t s)
{
    return launch_mfma_gemm<uint16_t, float>(M, N, K, A, sam, sak, B, sbk, sbn, C, scm, scn, splitk, part, s);
}
hipError_t launch_gemm_f32_mfma(int64_t M, int64_t N, int64_t K, const float *A, int64_t sam,
                                int64_t sak, const float *B, int64_t sbk, int64_t sbn, float *C,
                                int64_t scm, int64_t scn, int splitk, float *part, hipStream_t s)
{
    return launch_mfma_gemm<float, float>(M, N, K, A, sam, sak, B, sbk, sbn, C, scm, scn, splitk, part, s);
}
hipError_t launch_gemm_f64_mfma(int64_t M, int64_t N, int64_t K, const double *A, int64_t sam,
                                int64_t sak, const double *B, int64_t sbk, int64_t sbn, double *C,
                                int64_t scm, int64_t scn, int splitk, double *part, hipStream_t s)
{
    return launch_mfma_gemm<double, double>(M, N, K, A, sam, sak, B, sbk, sbn, C, scm, scn, splitk, part, s);
}

// ---------------------------------------------------------------------------
// Tall-skinny products C (M x N) = A (M x K) B (K x N) with N <= 128 and M,
// K large (the sketch, power and projection products of the large path).
// A workgroup of four wavefronts owns 64 FM rows and all N columns of a
// K-chunk (split K, partial sums reduced in a fixed order afterwards).  B's
// chunk is staged in LDS in buffers of KB values of k (double-buffered,
// rows n with k contiguous, padded by 16 bytes), A streams from memory
// straight into the matrix-core operand registers.  Four matrix steps form a
// group; within a group, lane slot s (lane / 16) and step j take
//   k = g0 + s (4 P) + j P + e,  e < P
// (P values per lane per step: 8 for bfloat16, 1 for float and double), so
// a lane's A values of a group are 4 P consecutive k of one row when A is
// k-contiguous (one to four 16-byte loads), and one element per step when A
// is row-contiguous (16 rows of one column per 128 bytes).  B's operand
// uses the same k for each column n = 16 nb + lane % 16.
// ---------------------------------------------------------------------------
template <typename TI>
struct TsTraits;
template <>
struct TsTraits<uint16_t> {
    using Acc = float;
    using AccV = floatx4_t;
    static constexpr int P = 8, KB = 128;
    static constexpr bool kRowsInterleaved = false;
};
template <>
struct TsTraits<float> {
    using Acc = float;
    using AccV = floatx4_t;
    static constexpr int P = 1, KB = 64;
    static constexpr bool kRowsInterleaved = false;
};
template <>
struct TsTraits<double> {
    using Acc = double;
    using AccV = doublex4_t;
    static constexpr int P = 1, KB = 32;
    static constexpr bool kRowsInterleaved = true;
};

template <typename TI>
struct TsOp;  // one lane's operand of one matrix step
template <>
struct TsOp<uint16_t> {
    bf16x8_t v;
};
template <>
struct TsOp<float> {
    float v;
};
template <>
struct TsOp<double> {
    double v;
};

__device__ __forceinline__ floatx4_t ts_mfma(const TsOp<uint16_t> &a, const TsOp<uint16_t> &b, floatx4_t c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4_t ts_mfma(const TsOp<float> &a, const TsOp<float> &b, floatx4_t c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a.v, b.v, c, 0, 0, 0);
}
__device__ __forceinline__ doublex4_t ts_mfma(const TsOp<double> &a, const TsOp<double> &b, doublex4_t c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a.v, b.v, c, 0, 0, 0);
}

constexpr int kTsMaxN = 128;

// A operands of one group (four steps) for row m, k from kg (= g0 + s 4 P).
// full: the group lies inside [0, kend) and the row inside [0, M).
template <typename TI, bool AKC>
__device__ __forceinline__ void ts_load_a(const TI *__restrict__ A, int64_t lda, int64_t m, bool mok,
                                          int64_t kg, int64_t kend, bool full, TsOp<TI> (&a)[4])
{
    constexpr int P = TsTraits<TI>::P;
    if (AKC) {
        const TI *src = A + m * lda + kg;
        if (full && mok) {
            if (P == 8) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    a[j] = *reinterpret_cast<const TsOp<TI> *>(src + 8 * j);
            } else if (sizeof(TI) == 4) {
                const float4 v = *reinterpret_cast<const float4 *>(src);
                const float t[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int j = 0; j < 4; ++j) a[j] = *reinterpret_cast<const TsOp<TI> *>(&t[j]);
            } else {
                const double2 v0 = *reinterpret_cast<const double2 *>(src);
                const double2 v1 = *reinterpret_cast<const double2 *>(src + 2);
                const double t[4] = {v0.x, v0.y, v1.x, v1.y};
#pragma unroll
                for (int j = 0; j < 4; ++j) a[j] = *reinterpret_cast<const TsOp<TI> *>(&t[j]);
            }
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                TI t[P];
#pragma unroll
                for (int e = 0; e < P; ++e) {
                    const int64_t k = kg + j * P + e;
                    t[e] = (mok && k < kend) ? src[j * P + e] : TI(0);
                }
                a[j] = *reinterpret_cast<const TsOp<TI> *>(t);
            }
        }
    } else if constexpr (P == 1) {
        // row-contiguous A (float or double only): element (m, k) at m + k lda
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t k = kg + j;
            a[j].v = (mok && (full || k < kend)) ? A[m + k * lda] : TI(0);
        }
    }
}

template <typename TI, bool AKC, int FM>
__global__ void __launch_bounds__(kThreads, FM >= 4 ? 1 : 2) k_ts_gemm(int64_t M, int N, int64_t K, const TI *__restrict__ A,
                                                         int64_t lda, const TI *__restrict__ B, int64_t ldb,
                                                         int64_t kchunk, int bvec,
                                                         typename TsTraits<TI>::Acc *part, void *Cv,
                                                         int64_t scm, int64_t scn, int direct, int c_is_double)
{
    using Tr = TsTraits<TI>;
    using Acc = typename Tr::Acc;
    using AccV = typename Tr::AccV;
    constexpr int P = Tr::P, KB = Tr::KB, GK = 16 * P;
    constexpr int LDB = KB + 16 / (int)sizeof(TI);
    constexpr int VPR = KB * (int)sizeof(TI) / 16;  // 16-byte vectors per staged row
    constexpr int NVEC = kTsMaxN * VPR / kThreads;   // per thread
    __shared__ __align__(16) TI Bs[2][kTsMaxN * LDB];
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int r = lane & 15, s = lane >> 4;
    const int nbn = (N + 15) / 16;
    const int64_t mw = (int64_t)blockIdx.x * (64 * FM) + wave * (16 * FM);
    const int64_t kb = (int64_t)blockIdx.y * kchunk, ke = min(K, kb + kchunk);
    const int nbuf = (int)((ke - kb + KB - 1) / KB);

    AccV acc[FM][8];
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int nb = 0; nb < 8; ++nb)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[f][nb][e] = Acc(0);

    // B staging: thread t covers vectors t, t + 256, ... of the [128][VPR] grid
    Vec16<TI> stg[NVEC];
    auto stage_load = [&](int ib) {
        const int64_t k0 = kb + (int64_t)ib * KB;
#pragma unroll
        for (int q = 0; q < NVEC; ++q) {
            const int vi = threadIdx.x + q * kThreads;
            const int n = vi / VPR, kv = (vi % VPR) * (16 / (int)sizeof(TI));
            const int64_t k = k0 + kv;
            constexpr int V = 16 / (int)sizeof(TI);
            if (n < N && bvec && k + V <= ke) {
                stg[q] = *reinterpret_cast<const Vec16<TI> *>(B + k + (int64_t)n * ldb);
            } else {
#pragma unroll
                for (int e = 0; e < V; ++e) stg[q].v[e] = (n < N && k + e < ke) ? B[k + e + (int64_t)n * ldb] : TI(0);
            }
        }
    };
    auto stage_store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < NVEC; ++q) {
            const int vi = threadIdx.x + q * kThreads;
            const int n = vi / VPR, kv = (vi % VPR) * (16 / (int)sizeof(TI));
            *reinterpret_cast<Vec16<TI> *>(&Bs[buf][n * LDB + kv]) = stg[q];
        }
    };

    // groups run in order; A of group g + 1 is loaded while group g computes
    constexpr int GPB = KB / GK;
    const int ng = (int)((ke - kb + GK - 1) / GK);
    auto load_group = [&](int g, TsOp<TI>(&a)[FM][4]) {
        const int64_t g0 = kb + (int64_t)g * GK;
        const bool full = g0 + GK <= ke;
        const int64_t kg = g0 + s * 4 * P;
#pragma unroll
        for (int f = 0; f < FM; ++f) {
            const int64_t m = mw + 16 * f + r;
            const bool mok = m < M;
            ts_load_a<TI, AKC>(A, lda, mok ? m : 0, mok, kg, ke, full, a[f]);
        }
    };
    TsOp<TI> acur[FM][4], anext[FM][4];
    stage_load(0);
    load_group(0, acur);
    stage_store(0);
    __syncthreads();
    for (int g = 0; g < ng; ++g) {
        const int ib = g / GPB, gi = g - ib * GPB;
        if (g + 1 < ng) load_group(g + 1, anext);
        const TI *bs = Bs[ib & 1];
#pragma unroll
        for (int nb = 0; nb < 8; ++nb) {
            if (nb < nbn) {
                TsOp<TI> b[4];
                const TI *src = bs + (16 * nb + r) * LDB + gi * GK + s * 4 * P;
                if (P == 8) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) b[j] = *reinterpret_cast<const TsOp<TI> *>(src + 8 * j);
                } else {
#pragma unroll
                    for (int j = 0; j < 4; ++j) b[j] = *reinterpret_cast<const TsOp<TI> *>(src + j);
                }
#pragma unroll
                for (int f = 0; f < FM; ++f)
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[f][nb] = ts_mfma(acur[f][j], b[j], acc[f][nb]);
            }
        }
#pragma unroll
        for (int f = 0; f < FM; ++f)
#pragma unroll
            for (int j = 0; j < 4; ++j) acur[f][j] = anext[f][j];
        if (gi == GPB - 1 || g == ng - 1) {
            // B's next buffer (from L2): loaded and stored here, so that its
            // staging registers are not live during the products
            if (ib + 1 < nbuf) {
                stage_load(ib + 1);
                stage_store((ib + 1) & 1);
            }
            __syncthreads();
        }
    }

    // epilogue: partial sums (split K) or the result directly.  In the float
    // layout a lane holds rows 4 s .. 4 s + 3 of one column: one 16-byte
    // store per column block where M allows.
    if constexpr (!Tr::kRowsInterleaved) {
      if (!direct && (M & 3) == 0) {
#pragma unroll
        for (int f = 0; f < FM; ++f) {
            const int64_t gm = mw + 16 * f + 4 * s;
#pragma unroll
            for (int nb = 0; nb < 8; ++nb) {
                const int gn = 16 * nb + r;
                if (nb < nbn && gm < M && gn < N) {
                    float4 v;
                    v.x = (float)acc[f][nb][0];
                    v.y = (float)acc[f][nb][1];
                    v.z = (float)acc[f][nb][2];
                    v.w = (float)acc[f][nb][3];
                    *reinterpret_cast<float4 *>(part + (int64_t)blockIdx.y * M * N + gm + (int64_t)gn * M) = v;
                }
            }
        }
        return;
      }
    }
#pragma unroll
    for (int f = 0; f < FM; ++f)
#pragma unroll
        for (int nb = 0; nb < 8; ++nb) {
            if (nb < nbn) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int row = Tr::kRowsInterleaved ? s + 4 * e : 4 * s + e;
                    const int64_t gm = mw + 16 * f + row;
                    const int gn = 16 * nb + r;
                    if (gm < M && gn < N) {
                        const Acc v = acc[f][nb][e];
                        if (!direct) part[(int64_t)blockIdx.y * M * N + gm + (int64_t)gn * M] = v;
                        else if (c_is_double) ((double *)Cv)[gm * scm + gn * scn] = (double)v;
                        else ((float *)Cv)[gm * scm + gn * scn] = (float)v;
                    }
                }
            }
        }
}

bool ts_gemm_ok(int64_t N, int64_t sam, int64_t sak, const void *A, int esize)
{
    if (N < 1 || N > kTsMaxN) return false;
    if (sak == 1) return ((uintptr_t)A % 16) == 0 && (sam * esize) % 16 == 0;
    return sam == 1 && esize != 2;
}

template <typename TI, typename TO>
hipError_t launch_ts_gemm(int64_t M, int64_t N, int64_t K, const TI *A, int64_t sam, int64_t sak,
                          const TI *B, int64_t ldb, TO *C, int64_t scm, int64_t scn,
                          typename TsTraits<TI>::Acc *part, int64_t part_cap, int num_cu, hipStream_t s)
{
    using Acc = typename TsTraits<TI>::Acc;
    constexpr int KB = TsTraits<TI>::KB;
    constexpr int FM = 2;
    if (M <= 0 || N <= 0) return hipSuccess;
    if (!ts_gemm_ok(N, sam, sak, A, (int)sizeof(TI))) return hipErrorNotSupported;
    const bool akc = sak == 1;
    const int64_t lda = akc ? sam : sak;
    const int bvec = ((uintptr_t)B % 16) == 0 && (ldb * (int64_t)sizeof(TI)) % 16 == 0;
    const int64_t mt = (M + 64 * FM - 1) / (64 * FM);
    // split K until the grid fills the compute units (per_cu workgroups each),
    // with chunks of at least 4 staging buffers and partials within part_cap
    const int per_cu = 2;
    int64_t sk = std::max<int64_t>(1, (per_cu * (int64_t)num_cu + mt - 1) / mt);
    sk = std::min<int64_t>(sk, std::max<int64_t>(1, K / (4 * KB)));
    if (part) sk = std::min<int64_t>(sk, std::max<int64_t>(1, part_cap / (M * N)));
    else sk = 1;
    int64_t kchunk = (K + sk - 1) / sk;
    kchunk = (kchunk + KB - 1) / KB * KB;
    sk = (K + kchunk - 1) / kchunk;
    const int direct = sk == 1;
    const int cd = sizeof(TO) == 8;
    dim3 grid((unsigned)mt, (unsigned)sk);
    if (akc) {
        hipLaunchKernelGGL((k_ts_gemm<TI, true, FM>), grid, dim3(kThreads), 0, s, M, (int)N, K, A, lda, B, ldb, kchunk, bvec, part, (void *)C, scm, scn, direct, cd);
    } else {
        if constexpr (TsTraits<TI>::P == 1)
            hipLaunchKernelGGL((k_ts_gemm<TI, false, FM>), grid, dim3(kThreads), 0, s, M, (int)N, K, A, lda, B, ldb, kchunk, bvec, part, (void *)C, scm, scn, direct, cd);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || direct) return e;
    const int64_t total = M * N;
    const int g2 = (int)std::min<int64_t>(8192, (total + kThreads - 1) / kThreads);
    hipLaunchKernelGGL((k_mfma_store<Acc, TO>), dim3(g2), dim3(kThreads), 0, s, M, N, (int)sk, part, C, scm, scn);
    return hipGetLastError();
}

hipError_t launch_ts_gemm_bf16(int64_t M, int64_t N, int64_t K, const uint16_t *A, int64_t sam, int64_t sak,
                               const uint16_t *B, int64_t ldb, float *C, int64_t scm, int64_t scn,
                               float *part, int64_t part_cap, int num_cu, hipStream_t s)
{
    return launch_ts_gemm<uint16_t, float>(M, N, K, A, sam, sak, B, ldb, C, scm, scn, part, part_cap, num_cu, s);
}
hipError_t launch_ts_gemm_f32(int64_t M, int64_t N, int64_t K, const float *A, int64_t sam, int64_t sak,
                              const float *B, int64_t ldb, float *C, int64_t scm, int64_t scn,
                              float *part, int64_t part_cap, int num_cu, hipStream_t s)
{
    return launch_ts_gemm<float, float>(M, N, K, A, sam, sak, B, ldb, C, scm, scn, part, part_cap, num_cu, s);
}
hipError_t launch_ts_gemm_f64(int64_t M, int64_t N, int64_t K, const double *A, int64_t sam, int64_t sak,
                              const double *B, int64_t ldb, double *C, int64_t scm, int64_t scn,
                              double *part, int64_t part_cap, int num_cu, hipStream_t s)
{
    return launch_ts_gemm<double, double>(M, N, K, A, sam, sak, B, ldb, C, scm, scn, part, part_cap, num_cu, s);
}

// ---------------------------------------------------------------------------
// Round-to-nearest-even conversion to bfloat16 (NaN kept quiet).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t to_bf16(float x)
{
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <typename TS>
__global__ void __launch_bounds__(kThreads) k_to_bf16(int64_t m, int64_t n, const TS *src, int64_t lds,
                                                      uint16_t *dst, int64_t ldd)
{
    const int64_t total = m * n;
    for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * kThreads) {
        const int64_t i = idx % m, j = idx / m;
        dst[i + j * ldd] = to_bf16((float)src[i + j * lds]);
    }
}

// Both bfloat16 copies of an m x n column-major float matrix: dst (m x n,
// ld m) and dstT (its transpose, n x m, ld n), through 64 x 64 LDS tiles.
__global__ void __launch_bounds__(kThreads) k_to_bf16_pair(int64_t m, int64_t n, const float *src, int64_t lds,
                                                           uint16_t *dst, uint16_t *dstT)
{
    __shared__ uint16_t t[64][65];
    const int64_t tm = (m + 63) / 64, tn = (n + 63) / 64;
    for (int64_t tile = blockIdx.x; tile < tm * tn; tile += gridDim.x) {
        const int64_t i0 = (tile % tm) * 64, j0 = (tile / tm) * 64;
        for (int e = threadIdx.x; e < 64 * 64; e += kThreads) {
            const int di = e % 64, dj = e / 64;
            const int64_t i = i0 + di, j = j0 + dj;
            uint16_t b = 0;
            if (i < m && j < n) {
                b = to_bf16(src[i + j * lds]);
                dst[i + j * m] = b;
            }
            t[dj][di] = b;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 64 * 64; e += kThreads) {
            const int dj = e % 64, di = e / 64;
            const int64_t i = i0 + di, j = j0 + dj;
            if (i < m && j < n) dstT[j + i * n] = t[dj][di];
        }
        __syncthreads();
    }
}

hipError_t launch_to_bf16_pair(int64_t m, int64_t n, const float *src, int64_t lds, uint16_t *dst,
                               uint16_t *dstT, hipStream_t s)
{
    const int64_t tiles = ((m + 63) / 64) * ((n + 63) / 64);
    hipLaunchKernelGGL(k_to_bf16_pair, dim3((unsigned)std::min<int64_t>(tiles, 4096)), dim3(kThreads), 0, s, m, n, src, lds, dst, dstT);
    return hipGetLastError();
}

hipError_t launch_to_bf16(int64_t m, int64_t n, const float *src, int64_t lds, uint16_t *dst,
                          int64_t ldd, hipStream_t s)
{
    hipLaunchKernelGGL((k_to_bf16<float>), dim3(4096), dim3(kThreads), 0, s, m, n, src, lds, dst, ldd);
    return hipGetLastError();
}

// Omega in bfloat16: the double Box-Muller outputs rounded to float, then to
// bfloat16 (the same values the oracle is fed for the precision form).
__global__ void __launch_bounds__(kThreads) k_omega_bf16(int64_t rows, int cols, uint64_t seed,
                                                         uint64_t counter, uint16_t *Om, int64_t ld)
{
    const int npair = (cols + 1) / 2;
    const int64_t total = rows * npair;
    for (int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * kThreads) {
        const int64_t k = idx % rows;
        const int j = (int)(idx / rows);
        double z0, z1;
        gaussian_pair(seed, counter, (uint32_t)k, (uint32_t)j, z0, z1);
        Om[k + (int64_t)(2 * j) * ld] = to_bf16((float)z0);
        if (2 * j + 1 < cols) Om[k + (int64_t)(2 * j + 1) * ld] = to_bf16((float)z1);
    }
}

hipError_t launch_omega_bf16(int64_t rows, int cols, uint64_t seed, uint64_t counter, uint16_t *Om,
                             int64_t ld, hipStream_t s)
{
    hipLaunchKernelGGL(k_omega_bf16, dim3(2048), dim3(kThreads), 0, s, rows, cols, seed, counter, Om, ld);
    return hipGetLastError();
}

}  // namespace frk
