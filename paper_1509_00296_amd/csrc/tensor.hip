// tensor.hip -- the elementwise steps of the 3-way tensor host (Type C of
// Table 6, the low-rank + sparse decomposition with the alignment fixed):
// the shrinkage of the mean of the three modes' estimates, the three
// multiplier updates with their residual sums, and the three SVT inputs of
// the next iteration, in one pass.  The tensor is column-major
// (i1 + I1 i2 + I1 I2 i3).  The unfoldings of modes 1 and 3 are strided views
// of that layout; mode 2's unfolding (rows i2, columns i1 + I1 i3) is kept in
// a buffer of its own, which this pass reads and writes at the permuted index.
#include "device_common.h"
#include "internal.h"

namespace frk {

constexpr int kTenThreads = 256;
constexpr int kTenBlocks = 1024;
constexpr int64_t kTenSlice = 8192;   // frontal slices up to this size go whole to one workgroup

__device__ __forceinline__ int64_t mode2_index(int64_t t, int64_t I1, int64_t I2)
{
    const int64_t i1 = t % I1, r = t / I1;
    const int64_t i2 = r % I2, i3 = r / I2;
    return i2 + I2 * (i1 + I1 * i3);
}

// A2p = mode-2 unfolding of O.
__global__ void __launch_bounds__(kTenThreads) k_ten_perm(int64_t N, int64_t I1, int64_t I2, const double *O,
                                                          double *A2p)
{
    for (int64_t t = (int64_t)blockIdx.x * kTenThreads + threadIdx.x; t < N; t += (int64_t)gridDim.x * kTenThreads)
        A2p[mode2_index(t, I1, I2)] = O[t];
}

// With L_1, L_2 (mode-2 layout), L_3 from the SVT steps:
//   E = shrink_thr(mean_i(O - L_i + Y_i / mu)),
//   Y_i += mu (O - L_i - E)  (part[i * gridDim + block] = its squares' sum),
//   A_i = O - E + Y_i / mu_next  (the next SVT inputs; A_2 in mode-2 layout).
__global__ void __launch_bounds__(kTenThreads)
    k_ten_update(int64_t N, int64_t I1, int64_t I2, const double *O, const double *L1, const double *L2p,
                 const double *L3, double *Y1, double *Y2, double *Y3, double *E, double *A1, double *A2p,
                 double *A3, double mu, double inv_mu, double thr, double inv_mu_next, double *part)
{
    __shared__ double red[3][kTenThreads / kWave];
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
    auto step = [&](int64_t t) {
        const int64_t tp = mode2_index(t, I1, I2);
        const double o = O[t];
        const double l1 = L1[t], l2 = L2p[tp], l3 = L3[t];
        double y1 = Y1[t], y2 = Y2[t], y3 = Y3[t];
        const double v = ((o - l1 + y1 * inv_mu) + (o - l2 + y2 * inv_mu) + (o - l3 + y3 * inv_mu)) / 3.0;
        const double av = fabs(v) - thr;
        const double e = av > 0.0 ? copysign(av, v) : 0.0;
        const double z1 = o - l1 - e, z2 = o - l2 - e, z3 = o - l3 - e;
        y1 += mu * z1;
        y2 += mu * z2;
        y3 += mu * z3;
        s1 += z1 * z1;
        s2 += z2 * z2;
        s3 += z3 * z3;
        Y1[t] = y1;
        Y2[t] = y2;
        Y3[t] = y3;
        E[t] = e;
        const double oe = o - e;
        A1[t] = oe + y1 * inv_mu_next;
        A2p[tp] = oe + y2 * inv_mu_next;
        A3[t] = oe + y3 * inv_mu_next;
    };
    // Small frontal slices go whole to one workgroup, so that a slice's
    // region of the mode-2 buffer (its I1 I2 values, consecutive there) is
    // read and written by one workgroup and its cache lines are completed in
    // one L2; larger slices are dealt out element by element.
    const int64_t S = I1 * I2;
    if (S <= kTenSlice) {
        const int64_t nslice = N / S;
        for (int64_t sl = blockIdx.x; sl < nslice; sl += gridDim.x)
            for (int64_t e = threadIdx.x; e < S; e += kTenThreads) step(sl * S + e);
    } else {
        for (int64_t t = (int64_t)blockIdx.x * kTenThreads + threadIdx.x; t < N;
             t += (int64_t)gridDim.x * kTenThreads)
            step(t);
    }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    s3 = wave_sum(s3);
    if (threadIdx.x % kWave == 0) {
        red[0][threadIdx.x / kWave] = s1;
        red[1][threadIdx.x / kWave] = s2;
        red[2][threadIdx.x / kWave] = s3;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        double a = 0.0;
        for (int w = 0; w < kTenThreads / kWave; ++w) a += red[threadIdx.x][w];
        part[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = a;
    }
}

// out[k] = sum_g part[k * nparts + g] for k < 3, added in a fixed order
__global__ void __launch_bounds__(kTenThreads) k_ten_sum_parts(const double *part, int nparts, double *out)
{
    __shared__ double red[kTenThreads / kWave];
    double a = 0.0;
    for (int g = threadIdx.x; g < nparts; g += kTenThreads) a += part[(int64_t)blockIdx.x * nparts + g];
    a = wave_sum(a);
    if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kTenThreads / kWave; ++w) t += red[w];
        out[blockIdx.x] = t;
    }
}

// L = (L_1 + L_2 + L_3) / 3 (L_2 in mode-2 layout; L may alias L_1)
__global__ void __launch_bounds__(kTenThreads) k_ten_mean(int64_t N, int64_t I1, int64_t I2, const double *L1,
                                                          const double *L2p, const double *L3, double *L)
{
    for (int64_t t = (int64_t)blockIdx.x * kTenThreads + threadIdx.x; t < N; t += (int64_t)gridDim.x * kTenThreads)
        L[t] = (L1[t] + L2p[mode2_index(t, I1, I2)] + L3[t]) / 3.0;
}

static unsigned ten_grid(int64_t N)
{
    return (unsigned)std::min<int64_t>((N + kTenThreads - 1) / kTenThreads, kTenBlocks);
}

int ten_parts() { return kTenBlocks; }

hipError_t launch_ten_perm(int64_t I1, int64_t I2, int64_t I3, const double *O, double *A2p, hipStream_t s)
{
    const int64_t N = I1 * I2 * I3;
    hipLaunchKernelGGL(k_ten_perm, dim3(ten_grid(N)), dim3(kTenThreads), 0, s, N, I1, I2, O, A2p);
    return hipGetLastError();
}

hipError_t launch_ten_update(int64_t I1, int64_t I2, int64_t I3, const double *O, const double *L1,
                             const double *L2p, const double *L3, double *Y1, double *Y2, double *Y3, double *E,
                             double *A1, double *A2p, double *A3, double mu, double thr, double mu_next,
                             double *part, double *sums, hipStream_t s)
{
    const int64_t N = I1 * I2 * I3;
    const unsigned g = ten_grid(N);
    hipLaunchKernelGGL(k_ten_update, dim3(g), dim3(kTenThreads), 0, s, N, I1, I2, O, L1, L2p, L3, Y1, Y2, Y3, E,
                       A1, A2p, A3, mu, 1.0 / mu, thr, 1.0 / mu_next, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ten_sum_parts, dim3(3), dim3(kTenThreads), 0, s, (const double *)part, (int)g, sums);
    return hipGetLastError();
}

hipError_t launch_ten_mean(int64_t I1, int64_t I2, int64_t I3, const double *L1, const double *L2p,
                           const double *L3, double *L, hipStream_t s)
{
    const int64_t N = I1 * I2 * I3;
    hipLaunchKernelGGL(k_ten_mean, dim3(ten_grid(N)), dim3(kTenThreads), 0, s, N, I1, I2, L1, L2p, L3, L);
    return hipGetLastError();
}

}  // namespace frk
