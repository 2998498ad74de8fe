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
