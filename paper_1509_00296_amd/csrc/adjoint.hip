// adjoint.hip -- kernels of the vector-Jacobian product (VJP) of FRSVT and of
// the unrolled inexact-ALM step.  The method of arXiv:1509.00296 is not
// differentiated in the paper; the derivative here is that of the map its
// Alg. 1 computes for a fixed Gaussian sketch,
//   X = Q S_tau(Q^T Ahat),  Q = qr((Ahat Ahat^T)^q Ahat Omega)  (Prop. 1),
// taken step by step backwards.
//
// Small factors.  With B = Q^T Ahat (l x nhat), B B^T = U diag(s^2) U^T and
// D = diag(f(s)/s), f(s) = max(s - tau, 0), the SVT of B is S = M2 B with
// M2 = U D U^T.  For an upstream gradient Sbar (l x nhat) the gradient of B
// is
//   Bbar = M1 B + M2 Sbar,   M1 = U N U^T,   N_ij = c_ij (G_ij + G_ji),
//   G = U^T (Sbar B^T) U,
// where c is symmetric and bounded (the spectral-function derivative written
// with W s = B^T U so that no 1/s_j of a small singular value appears):
//   both s_i, s_j > tau : c = tau / (s_i s_j (s_i + s_j))
//   one above (a), one not (d): c = g / (s_a (s_a + s_d)),
//        g = f(s_a) / (s_a - s_d) in [0, 1], set to 1/2 when
//        s_a - s_d <= 1e-12 s_a (the near-degenerate guard)
//   both <= tau          : c = 0.
// d/dtau of S is -U_r W_r^T, so taubar = -sum_{s_i > tau} G_ii / s_i.
#include "device_common.h"
#include "internal.h"

#include <algorithm>

namespace frk {

constexpr int kAdjT = 256;

// Columns of U (l x l, column-major) with s_j == 0 carry no direction after
// the semidefinite Cholesky; they are completed to an orthonormal basis of
// the null space (the derivative needs the whole of U).
__device__ void complete_basis(double *sU, const double *sig, int l, double *tmp)
{
    const int tid = threadIdx.x;
    for (int j = 0; j < l; ++j) {
        if (sig[j] > 0.0) continue;
        // candidate e_k with the least weight on the columns kept so far
        __shared__ int best_k;
        if (tid == 0) {
            double bw = 1e300;
            int bk = 0;
            for (int k = 0; k < l; ++k) {
                double w = 0.0;
                for (int c = 0; c < l; ++c)
                    if (c != j && (sig[c] > 0.0 || c < j)) w += sU[k + c * l] * sU[k + c * l];
                if (w < bw) {
                    bw = w;
                    bk = k;
                }
            }
            best_k = bk;
        }
        __syncthreads();
        for (int i = tid; i < l; i += blockDim.x) sU[i + j * l] = (i == best_k) ? 1.0 : 0.0;
        __syncthreads();
        for (int pass = 0; pass < 2; ++pass) {
            // coefficients against every other kept column, then the update
            for (int c = tid; c < l; c += blockDim.x) {
                double d = 0.0;
                if (c != j && (sig[c] > 0.0 || c < j))
                    for (int i = 0; i < l; ++i) d += sU[i + c * l] * sU[i + j * l];
                tmp[c] = d;
            }
            __syncthreads();
            for (int i = tid; i < l; i += blockDim.x) {
                double v = sU[i + j * l];
                for (int c = 0; c < l; ++c) v -= tmp[c] * sU[i + c * l];
                tmp[l + i] = v;
            }
            __syncthreads();
            if (tid == 0) {
                double nn = 0.0;
                for (int i = 0; i < l; ++i) nn += tmp[l + i] * tmp[l + i];
                tmp[2 * l] = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
            }
            __syncthreads();
            for (int i = tid; i < l; i += blockDim.x) sU[i + j * l] = tmp[l + i] * tmp[2 * l];
            __syncthreads();
        }
    }
}

__global__ void __launch_bounds__(kAdjT) k_svt_vjp_small(int l, const double *sigma, const double *U,
                                                         const double *H, double tau, double *M1,
                                                         double *M2, double *tau_bar)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *sU = reinterpret_cast<double *>(smem_raw);
    double *sA = sU + (size_t)l * l;
    double *sB = sA + (size_t)l * l;
    double *sig = sB + (size_t)l * l;
    double *tmp = sig + l;  // 2 l + 1
    const int tid = threadIdx.x;
    const int ll = l * l;
    for (int i = tid; i < ll; i += kAdjT) {
        sU[i] = U[i];
        sB[i] = H[i];
    }
    for (int i = tid; i < l; i += kAdjT) sig[i] = sigma[i];
    __syncthreads();
    complete_basis(sU, sig, l, tmp);
    // sA = H U ; sB = U^T sA = G
    for (int idx = tid; idx < ll; idx += kAdjT) {
        const int i = idx % l, j = idx / l;
        double v = 0.0;
        for (int t = 0; t < l; ++t) v += sB[i + t * l] * sU[t + j * l];
        sA[idx] = v;
    }
    __syncthreads();
    for (int idx = tid; idx < ll; idx += kAdjT) {
        const int i = idx % l, j = idx / l;
        double v = 0.0;
        for (int t = 0; t < l; ++t) v += sU[t + i * l] * sA[t + j * l];
        sB[idx] = v;
    }
    __syncthreads();
    if (tid == 0 && tau_bar) {
        double tb = 0.0;
        for (int i = 0; i < l; ++i)
            if (sig[i] > tau) tb -= sB[i + i * l] / sig[i];
        tau_bar[0] = tb;
    }
    // sA = N
    for (int idx = tid; idx < ll; idx += kAdjT) {
        const int i = idx % l, j = idx / l;
        const double si = sig[i], sj = sig[j];
        const bool ai = si > tau, aj = sj > tau;
        double c = 0.0;
        if (ai && aj) {
            c = tau / (si * sj * (si + sj));
        } else if (ai != aj) {
            const double sa = ai ? si : sj, sd = ai ? sj : si;
            const double gap = sa - sd;
            const double g = gap <= 1e-12 * sa ? 0.5 : (sa - tau) / gap;
            c = g / (sa * (sa + sd));
        }
        sA[idx] = c * (sB[idx] + sB[j + i * l]);
    }
    __syncthreads();
    // sB = U N ; M1 = sB U^T ; M2 = U D U^T
    for (int idx = tid; idx < ll; idx += kAdjT) {
        const int i = idx % l, j = idx / l;
        double v = 0.0;
        for (int t = 0; t < l; ++t) v += sU[i + t * l] * sA[t + j * l];
        sB[idx] = v;
    }
    __syncthreads();
    for (int idx = tid; idx < ll; idx += kAdjT) {
        const int i = idx % l, j = idx / l;
        double v1 = 0.0, v2 = 0.0;
        for (int t = 0; t < l; ++t) {
            v1 += sB[i + t * l] * sU[j + t * l];
            const double st = sig[t];
            if (st > tau) v2 += (st - tau) / st * sU[i + t * l] * sU[j + t * l];
        }
        M1[idx] = v1;
        M2[idx] = v2;
    }
}

hipError_t launch_svt_vjp_small(int l, const double *sigma, const double *U, const double *H,
                                double tau, double *M1, double *M2, double *tau_bar, hipStream_t s)
{
    if (l < 1 || l > 64) return hipErrorInvalidValue;
    const size_t lds = (3 * (size_t)l * l + 3 * (size_t)l + 1) * sizeof(double);
    hipLaunchKernelGGL(k_svt_vjp_small, dim3(1), dim3(kAdjT), lds, s, l, sigma, U, H, tau, M1, M2,
                       tau_bar);
    return hipGetLastError();
}

// QR step Y = Q R (R upper triangular): with K = Qbar^T Q and
// S = copyltu(-K) (lower triangle mirrored), Ybar = Qbar R^{-T} + Q S R^{-T}.
// Writes CA = R^{-T} and CB = S R^{-T} (l x l, column-major); flags[0] |= 1
// when a diagonal entry of R is not positive.
__global__ void __launch_bounds__(kAdjT) k_qr_vjp_small(int l, const double *K, const double *R,
                                                        double *CA, double *CB, int *flags)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *sRi = reinterpret_cast<double *>(smem_raw);  // R^{-1}, upper
    double *sS = sRi + (size_t)l * l;
    const int tid = threadIdx.x;
    const int ll = l * l;
    // column j of R^{-1}: back substitution of R x = e_j (one thread per column)
    for (int j = tid; j < l; j += kAdjT) {
        for (int i = l - 1; i >= 0; --i) {
            if (i > j) {
                sRi[i + j * l] = 0.0;
                continue;
            }
            double v = (i == j) ? 1.0 : 0.0;
            for (int t = i + 1; t <= j; ++t) v -= R[i + t * l] * sRi[t + j * l];
            const double d = R[i + i * l];
            sRi[i + j * l] = d > 0.0 ? v / d : 0.0;
        }
    }
    for (int idx = tid; idx < ll; idx += kAdjT) {
        const int i = idx % l, j = idx / l;
        // S(i, j) = -K(max, min) taken from the lower triangle
        sS[idx] = i >= j ? -K[i + j * l] : -K[j + i * l];
    }
    if (tid == 0 && flags) {
        int bad = 0;
        for (int i = 0; i < l; ++i) bad |= !(R[i + i * l] > 0.0);
        if (bad) flags[0] |= 1;
    }
    __syncthreads();
    for (int idx = tid; idx < ll; idx += kAdjT) {
        const int i = idx % l, j = idx / l;
        CA[idx] = sRi[j + i * l];
        double v = 0.0;
        for (int t = 0; t < l; ++t) v += sS[i + t * l] * sRi[j + t * l];
        CB[idx] = v;
    }
}

hipError_t launch_qr_vjp_small(int l, const double *K, const double *R, double *CA, double *CB,
                               int *flags, hipStream_t s)
{
    if (l < 1 || l > 64) return hipErrorInvalidValue;
    const size_t lds = 2 * (size_t)l * l * sizeof(double);
    hipLaunchKernelGGL(k_qr_vjp_small, dim3(1), dim3(kAdjT), lds, s, l, K, R, CA, CB, flags);
    return hipGetLastError();
}

// Out (rows x c) = sum_b In_b (rows x w_b) Coef_b (w_b x c), Coef_b in double
// (nullptr = identity, w_b = c), accumulated in double.  Block (x, y) owns
// 256 rows of column y; the coefficient column sits in LDS.
template <typename T>
__global__ void __launch_bounds__(kAdjT) k_combine(CombineArgs<T> a)
{
    __shared__ double sc[kCombineMaxIn][64];
    const int j = blockIdx.y;
    for (int b = 0; b < a.nin; ++b)
        for (int k = threadIdx.x; k < a.w[b]; k += kAdjT)
            sc[b][k] = a.coef[b] ? a.coef[b][k + (int64_t)j * a.w[b]] : (k == j ? 1.0 : 0.0);
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kAdjT + threadIdx.x;
    if (i >= a.rows) return;
    double v = 0.0;
    for (int b = 0; b < a.nin; ++b) {
        const T *in = a.in[b];
        const int64_t ld = a.ldin[b];
        for (int k = 0; k < a.w[b]; ++k) v += (double)in[i + k * ld] * sc[b][k];
    }
    a.out[i + (int64_t)j * a.ldout] = (T)v;
}

template <typename T>
hipError_t launch_combine(const CombineArgs<T> &a, hipStream_t s)
{
    if (a.nin < 1 || a.nin > kCombineMaxIn || a.c < 1 || a.c > 64) return hipErrorInvalidValue;
    for (int b = 0; b < a.nin; ++b)
        if (a.w[b] < 1 || a.w[b] > 64 || (!a.coef[b] && a.w[b] != a.c)) return hipErrorInvalidValue;
    if (a.rows <= 0) return hipSuccess;
    dim3 grid((unsigned)((a.rows + kAdjT - 1) / kAdjT), (unsigned)a.c);
    hipLaunchKernelGGL((k_combine<T>), grid, dim3(kAdjT), 0, s, a);
    return hipGetLastError();
}
template hipError_t launch_combine<double>(const CombineArgs<double> &, hipStream_t);
template hipError_t launch_combine<float>(const CombineArgs<float> &, hipStream_t);

// ---------------------------------------------------------------------------
// One unrolled inexact-ALM step after the thresholding (the S- and
// multiplier updates of the iALM loop, with learnable shrink threshold lam):
//   V = O - L + Y/mu,  S = shrink(V, lam),  Y' = Y + mu (O - L - S),
//   A' = O - S + Y'/mu'   (the input of the next thresholding).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kAdjT) k_dual_step(DualStepArgs<T> a)
{
    const int64_t total = a.m * a.n;
    const T mu = (T)a.mu, inv_mu = (T)(1.0 / a.mu), inv_mu_next = (T)(1.0 / a.mu_next);
    const T lam = (T)a.lam;
    for (int64_t idx = (int64_t)blockIdx.x * kAdjT + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * kAdjT) {
        const int64_t i = idx % a.m, j = idx / a.m;
        const T o = a.O[i + j * a.ldo], L = a.L[i + j * a.ldl], y = a.Y[i + j * a.ldy];
        const T sv = soft_shrink(o - L + y * inv_mu, lam);
        const T yn = y + mu * (o - L - sv);
        if (a.S) a.S[i + j * a.lds] = sv;
        if (a.Yn) a.Yn[i + j * a.ldyn] = yn;
        if (a.An) a.An[i + j * a.ldan] = o - sv + yn * inv_mu_next;
    }
}

// Reverse of k_dual_step for upstream gradients Sb, Ynb, Anb (each optional):
//   Yt = Ynb + Anb/mu',  St = Sb - Anb - mu Yt,  Vb = St [|V| > lam],
//   Lb = -mu Yt - Vb,  Yb = Yt + Vb/mu,  lambar = -sum St sgn(V) [|V| > lam].
template <typename T>
__global__ void __launch_bounds__(kAdjT) k_dual_step_vjp(DualStepArgs<T> a)
{
    __shared__ double sred[kAdjT / kWave];
    const int64_t total = a.m * a.n;
    const T mu = (T)a.mu, inv_mu = (T)(1.0 / a.mu), inv_mu_next = (T)(1.0 / a.mu_next);
    const T lam = (T)a.lam;
    double lb = 0.0;
    for (int64_t idx = (int64_t)blockIdx.x * kAdjT + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * kAdjT) {
        const int64_t i = idx % a.m, j = idx / a.m;
        const T o = a.O[i + j * a.ldo], L = a.L[i + j * a.ldl], y = a.Y[i + j * a.ldy];
        const T v = o - L + y * inv_mu;
        const T anb = a.Anb ? a.Anb[i + j * a.ldanb] : T(0);
        const T yt = (a.Ynb ? a.Ynb[i + j * a.ldynb] : T(0)) + anb * inv_mu_next;
        const T st = (a.Sb ? a.Sb[i + j * a.ldsb] : T(0)) - anb - mu * yt;
        const bool pass = (v > T(0) ? v : -v) > lam;
        const T vb = pass ? st : T(0);
        if (pass) lb -= (double)(v > T(0) ? st : -st);
        a.Lb[i + j * a.ldlb] = -mu * yt - vb;
        a.Yb[i + j * a.ldyb] = yt + vb * inv_mu;
    }
    lb = wave_sum(lb);
    if (threadIdx.x % kWave == 0) sred[threadIdx.x / kWave] = lb;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kAdjT / kWave; ++w) s += sred[w];
        a.part[blockIdx.x] = s;
    }
}

template <typename T>
hipError_t launch_dual_step(const DualStepArgs<T> &a, bool vjp, int *nparts, hipStream_t s)
{
    const int64_t total = a.m * a.n;
    int grid = (int)std::min<int64_t>((total + kAdjT - 1) / kAdjT, kDualGrid);
    if (grid < 1) grid = 1;
    if (nparts) *nparts = grid;
    if (vjp) hipLaunchKernelGGL((k_dual_step_vjp<T>), dim3(grid), dim3(kAdjT), 0, s, a);
    else hipLaunchKernelGGL((k_dual_step<T>), dim3(grid), dim3(kAdjT), 0, s, a);
    return hipGetLastError();
}
template hipError_t launch_dual_step<double>(const DualStepArgs<double> &, bool, int *, hipStream_t);
template hipError_t launch_dual_step<float>(const DualStepArgs<float> &, bool, int *, hipStream_t);

// p[0..count) = value (a kernel, so that the call stays capturable in a graph)
__global__ void k_fill_int(int *p, int count, int value)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

hipError_t launch_fill_int(int *p, int count, int value, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_int, dim3((count + 255) / 256), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}

}  // namespace frk
