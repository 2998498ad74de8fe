// block_dense.h -- workgroup-level dense helpers on LDS-resident matrices
// (Gram, Cholesky with null-pivot detection, triangular solve).
#pragma once
#include "device_common.h"

namespace frk {

// W: l columns of length mh at W[j * mhp + i] (double).  G, R: l x l at
// [a * l + b] (R upper triangular, row-major).

// G = W^T W (full symmetric), one wavefront per (a, b) pair, lanes over rows.
__device__ __forceinline__ void block_gram(const double *W, int mh, int mhp, int l, double *G)
{
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    const int npairs = l * (l + 1) / 2;
    for (int p = wave; p < npairs; p += nw) {
        int a = 0, rem = p;
        while (rem >= l - a) {
            rem -= l - a;
            ++a;
        }
        const int b = a + rem;
        const double *wa = W + (size_t)a * mhp, *wb = W + (size_t)b * mhp;
        double s = 0.0;
        for (int i = lane; i < mh; i += kWave) s += wa[i] * wb[i];
        s = wave_sum(s);
        if (lane == 0) {
            G[a * l + b] = s;
            G[b * l + a] = s;
        }
    }
    __syncthreads();
}

struct CholInfo {
    int nnull;         // pivots treated as numerically null
    double min_ratio;  // min over non-null columns of pivot / (G_jj + shift)
};

// Cholesky of (G + shift I) into the upper triangle of R.  Every thread
// forms the pivot itself from LDS (no broadcast step), so each column costs
// one barrier.  Pivots <= null_tol are numerically null: R_jj = 1, zero row,
// null_flags[j] = 1.
__device__ __forceinline__ CholInfo block_chol(const double *G, int l, double shift, double null_tol,
                                      double *R, int *null_flags)
{
    const int tid = threadIdx.x;
    for (int idx = tid; idx < l * l; idx += blockDim.x) R[idx] = 0.0;
    __syncthreads();
    CholInfo info{0, 1.0};
    for (int j = 0; j < l; ++j) {
        const double gjj = G[j * l + j] + shift;
        double d = gjj;
        for (int t = 0; t < j; ++t) d -= R[t * l + j] * R[t * l + j];
        const bool isnull = !(d > null_tol);
        const double piv = isnull ? 1.0 : sqrt(d);
        if (isnull) ++info.nnull;
        else if (gjj > 0.0) info.min_ratio = fmin(info.min_ratio, d / gjj);
        if (tid == 0) {
            R[j * l + j] = piv;
            if (null_flags) null_flags[j] = isnull ? 1 : 0;
        }
        if (!isnull) {
            for (int k = j + 1 + tid; k < l; k += blockDim.x) {
                double v = G[j * l + k];
                for (int t = 0; t < j; ++t) v -= R[t * l + j] * R[t * l + k];
                R[j * l + k] = v / piv;
            }
        }
        __syncthreads();
    }
    return info;
}

// W <- W R^{-1} (R upper, row-major), each thread owns rows; for l <= LM
// (LM <= 16, a compile-time bound) a row is held in registers while it is
// solved.
template <int LM = 16>
__device__ __forceinline__ void block_trsm(double *W, int mh, int mhp, int l, const double *R)
{
    if (l <= LM) {
        for (int i = threadIdx.x; i < mh; i += blockDim.x) {
            double w[LM];
#pragma unroll
            for (int j = 0; j < LM; ++j) w[j] = j < l ? W[(size_t)j * mhp + i] : 0.0;
#pragma unroll
            for (int j = 0; j < LM; ++j) {
                if (j < l) {
                    double v = w[j];
#pragma unroll
                    for (int t = 0; t < j; ++t) v -= w[t] * R[t * l + j];
                    w[j] = v / R[j * l + j];
                }
            }
#pragma unroll
            for (int j = 0; j < LM; ++j)
                if (j < l) W[(size_t)j * mhp + i] = w[j];
        }
    } else {
        for (int i = threadIdx.x; i < mh; i += blockDim.x) {
            for (int j = 0; j < l; ++j) {
                double v = W[(size_t)j * mhp + i];
                for (int t = 0; t < j; ++t) v -= W[(size_t)t * mhp + i] * R[t * l + j];
                W[(size_t)j * mhp + i] = v / R[j * l + j];
            }
        }
    }
    __syncthreads();
}


// ---------------------------------------------------------------------------
// Fast forms for l <= 16 columns (blockDim = 256, four wavefronts).
// ---------------------------------------------------------------------------
typedef __attribute__((__vector_size__(4 * sizeof(double)))) double bd_doublex4;

// G = W^T W (l <= 16, G row-major [a * l + b]) on the matrix cores: K = rows,
// wavefront w takes the 4-row steps 4w, 4w + 16, ... (four chains); A and B operands are
// the same element W(i, a) with a = lane % 16, i = step + lane / 16.  The
// four partial 16 x 16 blocks are added in a fixed order.  part: 4 * 256
// doubles of LDS.  Ends with a barrier.
__device__ __forceinline__ void gram16_mfma(const double *W, int mh, int mhp, int l, double *G, double *part)
{
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int a = lane & 15, ko = lane >> 4;
    bd_doublex4 z0 = {0, 0, 0, 0}, z1 = {0, 0, 0, 0}, z2 = {0, 0, 0, 0}, z3 = {0, 0, 0, 0};
    // four independent accumulation chains over row steps 4 w + 16 t; all
    // loads of an iteration are issued before its products
    const double *wa = W + (size_t)(a < l ? a : 0) * mhp;
    for (int i0 = 4 * wave; i0 < mh; i0 += 64) {
        double x[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int i = i0 + 16 * t + ko;
            x[t] = (a < l && i < mh) ? wa[i < mh ? i : 0] : 0.0;
        }
        z0 = __builtin_amdgcn_mfma_f64_16x16x4f64(x[0], x[0], z0, 0, 0, 0);
        z1 = __builtin_amdgcn_mfma_f64_16x16x4f64(x[1], x[1], z1, 0, 0, 0);
        z2 = __builtin_amdgcn_mfma_f64_16x16x4f64(x[2], x[2], z2, 0, 0, 0);
        z3 = __builtin_amdgcn_mfma_f64_16x16x4f64(x[3], x[3], z3, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
        part[wave * 256 + ((lane >> 4) + 4 * r) * 16 + a] = (z0[r] + z1[r]) + (z2[r] + z3[r]);
    __syncthreads();
    for (int idx = threadIdx.x; idx < l * l; idx += blockDim.x) {
        const int x = idx / l, y = idx % l;
        const int e = x * 16 + y;
        G[idx] = ((part[e] + part[256 + e]) + part[512 + e]) + part[768 + e];
    }
    __syncthreads();
}

// G = W^T W for 16 < l <= 32 on the matrix cores: the three distinct 16 x 16
// blocks (columns 0-15 with 0-15, 0-15 with 16-31, 16-31 with 16-31), each
// wavefront over the 4-row steps 4 w, 4 w + 16, ... as gram16_mfma; the four
// wavefronts' partial blocks added in a fixed order.  part: 4 * 768 doubles
// of LDS.  Ends with a barrier.
__device__ __forceinline__ void gram32_mfma(const double *W, int mh, int mhp, int l, double *G, double *part)
{
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const int a = lane & 15, ko = lane >> 4;
    bd_doublex4 z00 = {0, 0, 0, 0}, z01 = {0, 0, 0, 0}, z11 = {0, 0, 0, 0};
    const double *w0 = W + (size_t)a * mhp;
    const double *w1 = W + (size_t)(16 + a < l ? 16 + a : 0) * mhp;
    for (int i0 = 4 * wave; i0 < mh; i0 += 16) {
        const int i = i0 + ko;
        const double x0 = i < mh ? w0[i] : 0.0;
        const double x1 = (i < mh && 16 + a < l) ? w1[i] : 0.0;
        z00 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, x0, z00, 0, 0, 0);
        z01 = __builtin_amdgcn_mfma_f64_16x16x4f64(x0, x1, z01, 0, 0, 0);
        z11 = __builtin_amdgcn_mfma_f64_16x16x4f64(x1, x1, z11, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int e = ((lane >> 4) + 4 * r) * 16 + a;
        part[wave * 768 + e] = z00[r];
        part[wave * 768 + 256 + e] = z01[r];
        part[wave * 768 + 512 + e] = z11[r];
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < l * l; idx += blockDim.x) {
        const int x = idx / l, y = idx % l;
        int e;
        if (x < 16 && y < 16) e = x * 16 + y;
        else if (x < 16) e = 256 + x * 16 + (y - 16);
        else if (y < 16) e = 256 + y * 16 + (x - 16);
        else e = 512 + (x - 16) * 16 + (y - 16);
        G[idx] = ((part[e] + part[768 + e]) + part[1536 + e]) + part[2304 + e];
    }
    __syncthreads();
}

// The Gram of an l <= LM column basis in LDS on the matrix cores.
template <int LM>
__device__ __forceinline__ void gram_mfma(const double *W, int mh, int mhp, int l, double *G, double *part)
{
    if (LM <= 16) gram16_mfma(W, mh, mhp, l, G, part);
    else gram32_mfma(W, mh, mhp, l, G, part);
}

// Cholesky of (G + shift I), l <= LM <= 16 (LM a compile-time bound), by
// ONE wavefront: lane k holds column
// k of the trailing matrix in registers; each pivot and each row of R is
// broadcast with readlane.  Writes R (upper, row-major [j * l + k], the
// strict lower triangle set to zero) and null_flags; pivots <= null_tol are
// numerically null: a zero row with R_jj = 1 (null_pivot_one) or 0.  G may
// alias R (it is read into registers first).  No barrier inside: call from
// one wavefront, synchronise afterwards.
template <int LM = 16>
__device__ __forceinline__ CholInfo wave_chol16(const double *G, int l, double shift, double null_tol,
                                       double *R, int *null_flags, bool null_pivot_one = true)
{
    const int k = threadIdx.x % kWave;
    double g[LM];
#pragma unroll
    for (int i = 0; i < LM; ++i) g[i] = (i < l && k < l) ? G[i * l + k] + (i == k ? shift : 0.0) : 0.0;
    double gkk = 0.0;
#pragma unroll
    for (int i = 0; i < LM; ++i)
        if (i == k) gkk = g[i];
    CholInfo info{0, 1.0};
#pragma unroll
    for (int j = 0; j < LM; ++j) {
        if (j >= l) break;
        double gj = 0.0;   // this lane's element j of its column: G'(j, k)
#pragma unroll
        for (int i = 0; i < LM; ++i)
            if (i == j) gj = g[i];
        const double d = read_lane(gj, j);
        const double ojj = read_lane(gkk, j);
        const bool isnull = !(d > null_tol);
        // pivot and its reciprocal from one reciprocal square root
        const double rs = rsqrt(isnull ? 1.0 : d);
        const double piv = isnull ? (null_pivot_one ? 1.0 : 0.0) : d * rs;
        if (isnull) ++info.nnull;
        else if (ojj > 0.0) info.min_ratio = fmin(info.min_ratio, d / ojj);
        const double inv = isnull ? 0.0 : rs;
        double rjk = 0.0;
        if (k == j) rjk = piv;
        else if (k > j && k < l && !isnull) rjk = gj * inv;
        if (k < l) R[j * l + k] = rjk;
        if (k == 0 && null_flags) null_flags[j] = isnull ? 1 : 0;
        // rows i >= l take zero updates (lanes k >= l hold rjk = 0), so the
        // loop needs no runtime bound
#pragma unroll
        for (int i = 0; i < LM; ++i) {
            if (i > j) {
                const double rji = read_lane(rjk, i);
                g[i] = (k > j) ? g[i] - rji * rjk : g[i];
            }
        }
    }
    return info;
}

// 1/sqrt(x) for x > 0: the lean form where x is normal, the library's
// below (a denormal x).
__device__ __forceinline__ double rsqrt_pos(double x) { return x >= 1e-300 ? rsqrt_nr(x) : rsqrt(x); }

// Cholesky of the upper triangle of g (l <= N), done by the calling thread on
// its own copy in registers: every thread that calls it with the same g gets
// the same R, so a workgroup needs no broadcast of the factor.  Row j of R
// overwrites row j of g (entries past column l - 1 set to zero); pivots <=
// null_tol are numerically null: R_jj = null_piv and a zero row.  min_ratio
// is 0 when a non-null pivot fell below ratio_tol times its original
// diagonal entry, else 1 (a comparison, no division).
// rinv (optional) receives 1 / R_jj from the same reciprocal square root
// (0 for a null pivot).
template <int N>
__device__ __forceinline__ CholInfo reg_chol(double (&g)[N][N], int l, double null_tol, double null_piv,
                                             double ratio_tol = 0.0, double *rinv = nullptr)
{
    CholInfo info{0, 1.0};
    double od[N];
#pragma unroll
    for (int j = 0; j < N; ++j) od[j] = g[j][j];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        if (j < l) {
            const double d = g[j][j];
            const bool isnull = !(d > null_tol);
            const double rs = rsqrt_pos(isnull ? 1.0 : d);
            if (isnull) ++info.nnull;
            else if (d < ratio_tol * od[j]) info.min_ratio = 0.0;
            g[j][j] = isnull ? null_piv : d * rs;
            const double inv = isnull ? 0.0 : rs;
            if (rinv) rinv[j] = inv;
#pragma unroll
            for (int k = j + 1; k < N; ++k) g[j][k] = k < l ? g[j][k] * inv : 0.0;
#pragma unroll
            for (int i = j + 1; i < N; ++i)
#pragma unroll
                for (int k = i; k < N; ++k) g[i][k] -= g[j][i] * g[j][k];
        }
    }
    return info;
}

// w <- w R^{-1} for one row w (length l <= N) and R upper in registers (the
// reciprocals of the diagonal formed once).
template <int N>
__device__ __forceinline__ void reg_trsm_row(double (&w)[N], const double (&R)[N][N], const double (&rinv)[N], int l)
{
#pragma unroll
    for (int j = 0; j < N; ++j) {
        if (j < l) {
            double v = w[j];
#pragma unroll
            for (int t = 0; t < j; ++t) v -= w[t] * R[t][j];
            w[j] = v * rinv[j];
        }
    }
}

// Cholesky of the symmetric l x l matrix M (row-major; the upper triangle
// is read) by NT threads: thread t owns the 4 x 4 blocks t, t + NT, ...
// (BPT of them; blocks bi <= bj dealt in row-major order over the block
// triangle, nb (nb + 1) / 2 <= BPT NT, nb = ceil(l / 4)) in registers.
// Step j: the owner of (j, j) has published the updated diagonal d_j in
// sh_d[j]; every thread forms the pivot from it (d_j <= tol: numerically
// null, pivot null_piv and a zero row); the owners of row j scale it and
// publish it in rowbuf (16-byte aligned, at least 4 nb doubles); the trailing
// triangle takes the rank-one update (eight reads of rowbuf for sixteen
// products per block) and the owner of (j + 1, j + 1) publishes d_{j+1}.
// Two barriers per step.  R is written back into M (upper, row-major with
// row stride ldo or l, zeros below and past column l - 1).  Returns the
// number of null pivots; null_flags[j] (if given) marks them.
template <int NT, int BPT = 1>
__device__ __forceinline__ int chol_blk4(double *M, int l, double tol, double null_piv, double *rowbuf,
                                         double *sh_d, int *null_flags, int ldo = 0)
{
    // R goes back with row stride ld (ldo if given, else l); entries past
    // column l - 1 of a row are zero
    const int ld = ldo > 0 ? ldo : l;
    const int tid = threadIdx.x;
    const int nb = (l + 3) / 4;
    int bi[BPT], bj[BPT];
    bool owner[BPT];
    double v[BPT][4][4];
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
        bi[q] = nb;
        bj[q] = nb;
        int rem = tid + q * NT, r = 0;
        while (r < nb && rem >= nb - r) {
            rem -= nb - r;
            ++r;
        }
        if (r < nb) {
            bi[q] = r;
            bj[q] = r + rem;
        }
        owner[q] = bi[q] < nb;
#pragma unroll
        for (int r2 = 0; r2 < 4; ++r2)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int aa = 4 * bi[q] + r2, bb = 4 * bj[q] + c;
                v[q][r2][c] = (owner[q] && aa < l && bb < l && bb >= aa) ? M[aa * l + bb] : 0.0;
            }
        if (owner[q] && bi[q] == 0 && bj[q] == 0) sh_d[0] = v[q][0][0];
    }
    __syncthreads();
    int nnull = 0;
    for (int j = 0; j < l; ++j) {
        const double d = sh_d[j];
        const bool isnull = !(d > tol);
        // pivot and its reciprocal from one reciprocal square root
        const double rs = rsqrt(isnull ? 1.0 : d);
        const double piv = isnull ? null_piv : d * rs;
        const double inv = isnull ? 0.0 : rs;
        nnull += isnull ? 1 : 0;
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
            if (owner[q] && bi[q] == (j >> 2)) {
                const int rj = j & 3;
                const int b0 = 4 * bj[q];
#pragma unroll
                for (int r2 = 0; r2 < 4; ++r2) {
                    if (r2 == rj) {
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            const int bb = b0 + c;
                            v[q][r2][c] = bb == j ? piv : (bb > j ? v[q][r2][c] * inv : v[q][r2][c]);
                            if (bb > j && bb < l) rowbuf[bb] = v[q][r2][c];
                        }
                    }
                }
            }
        }
        __syncthreads();
        if (!isnull) {
#pragma unroll
            for (int q = 0; q < BPT; ++q) {
                const int a0 = 4 * bi[q], b0 = 4 * bj[q];
                if (owner[q] && b0 + 3 > j) {
                    const double2 *ra2 = reinterpret_cast<const double2 *>(rowbuf + a0);
                    const double2 *rb2 = reinterpret_cast<const double2 *>(rowbuf + b0);
                    const double2 x0 = ra2[0], x1 = ra2[1], y0 = rb2[0], y1 = rb2[1];
                    const double xa[4] = {x0.x, x0.y, x1.x, x1.y}, yb[4] = {y0.x, y0.y, y1.x, y1.y};
#pragma unroll
                    for (int r2 = 0; r2 < 4; ++r2)
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            const int aa = a0 + r2, bb = b0 + c;
                            const double nv = v[q][r2][c] - xa[r2] * yb[c];
                            v[q][r2][c] = (aa > j && bb >= aa) ? nv : v[q][r2][c];
                        }
                }
            }
        }
        const int j1 = j + 1;
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
            if (owner[q] && j1 < l && bi[q] == (j1 >> 2) && bj[q] == bi[q]) {
#pragma unroll
                for (int r2 = 0; r2 < 4; ++r2)
                    if (r2 == (j1 & 3)) sh_d[j1] = v[q][r2][r2];
            }
        }
        __syncthreads();
    }
    for (int idx = tid; idx < l * ld; idx += NT) {
        const int aa = idx / ld, bb = idx - aa * ld;
        if (bb < aa || bb >= l) M[idx] = 0.0;
    }
#pragma unroll
    for (int q = 0; q < BPT; ++q)
#pragma unroll
        for (int r2 = 0; r2 < 4; ++r2)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int aa = 4 * bi[q] + r2, bb = 4 * bj[q] + c;
                if (owner[q] && aa < l && bb < l && bb >= aa) M[aa * ld + bb] = v[q][r2][c];
            }
    // the published diagonals decide the null flags (no global store inside
    // the step loop, whose barriers would wait for it)
    if (null_flags)
        for (int j = tid; j < l; j += NT) null_flags[j] = (sh_d[j] > tol) ? 0 : 1;
    __syncthreads();
    return nnull;
}

// ---------------------------------------------------------------------------
// One-sided Jacobi pieces: the circle ordering, the rotation, its test and
// the group engine (shared by the small SVD and the batched WSVT).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void circle_pair(int n2, int round, int t, int &p, int &q)
{
    // 0 <= round, t < n2 - 1: both sums lie in [0, 2 (n2 - 1))
    if (t == 0) {
        p = n2 - 1;
        q = round;
    } else {
        p = round + t;
        q = round - t + n2 - 1;
        if (p >= n2 - 1) p -= n2 - 1;
        if (q >= n2 - 1) q -= n2 - 1;
    }
    if (p > q) {
        const int tmp = p;
        p = q;
        q = tmp;
    }
}

// Rotation of the pair with squared norms al, be and inner product ga.
// With d = be - al, g2 = 2 ga and h = sqrt(d^2 + g2^2), the angle theta
// (|theta| <= pi/4) has cos 2theta = |d| / h and sin 2theta = sgn(d) g2 / h,
// and the half-angle formulas give cs = sqrt((1 + cos 2theta) / 2),
// sn = sin 2theta / (2 cs): two dependent reciprocal square roots (1/h and
// 1/cs) instead of a square root, a division and a reciprocal square root.
// Operands whose squares would overflow or underflow take the tangent form
// t = sgn(zeta) / (|zeta| + sqrt(1 + zeta^2)), zeta = d / g2.
__device__ __forceinline__ void jacobi_rotation(double al, double be, double ga, double &cs, double &sn)
{
    const double d = be - al, g2 = 2.0 * ga;
    const double h2 = d * d + g2 * g2;
    if (h2 > 1e-290 && h2 < 1e290) {
        // both arguments normal (hc lies in [1/2, 1]): the lean reciprocal
        // square root
        const double rh = rsqrt_nr(h2);
        const double c2 = fabs(d) * rh;
        const double s2 = (d >= 0.0 ? g2 : -g2) * rh;
        const double hc = 0.5 * (1.0 + c2);
        const double rc = rsqrt_nr(hc);
        cs = hc * rc;
        sn = 0.5 * s2 * rc;
    } else {
        const double zeta = d / g2;
        const double t1 = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
        cs = rsqrt(1.0 + t1 * t1);
        sn = cs * t1;
    }
}

// The rotation test |ga| > tol sqrt(al be), squared where al be is finite
// and far from overflow (no square root on the common path).
__device__ __forceinline__ bool jacobi_needed(double al, double be, double ga, double tol)
{
    const double ab = al * be;
    return ab < 1e300 ? ga * ga > (tol * tol) * ab : fabs(ga) > tol * sqrt(ab);
}

// Stopping rule of the cyclic Jacobi sweeps: a pair is rotated while its
// cosine |m_p.m_q| / (|m_p| |m_q|) exceeds rows 2u, and the sweeps stop after
// one in which no applied rotation had a cosine above kJacobiQuadStop.  Near
// convergence each sweep squares the largest cosine (the quadratic
// convergence of cyclic Jacobi), so the sweep that would follow would find
// cosines near 1e-16, below the rotation threshold: stopping here saves that
// confirming sweep and leaves the columns orthogonal to working precision.
constexpr double kJacobiQuadStop = 1e-8;

// ---------------------------------------------------------------------------
// One wavefront, l <= 8: the lane grid (r, c) = (lane % 8, lane / 8), lane
// (r, c) holding element (r, c) of an 8 x 8 matrix M (zeros past l), so that
// a column of M is one 8-lane DPP segment.
// ---------------------------------------------------------------------------
// M = R^T for the semidefinite upper Cholesky factor R of the symmetric g
// (upper triangle read; pivots at or below 4 l u max_j g_jj give zero rows).
// Every lane factors g itself (reg_chol) and keeps its element.
__device__ __forceinline__ double wave8_factor(double (&g)[8][8], int l)
{
    const int lane = threadIdx.x % kWave, r = lane & 7, c = lane >> 3;
    double maxdiag = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (j < l) maxdiag = fmax(maxdiag, g[j][j]);
    reg_chol<8>(g, l, 4.0 * l * kU * maxdiag, 0.0);
    double x = 0.0;
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = a; b < 8; ++b)
            if (a == c && b == r) x = g[a][b];
    return x;
}

// One-sided Jacobi on the columns of M in the lane grid.  Round rd of the
// circle ordering pairs column c with d = 2 rd - c mod (n2 - 1) (column rd
// with the fixed column n2 - 1); the partner's element arrives through one
// lane permute, and the three inner products are segment sums that both
// columns of a pair form over the same values in the same order, so both
// lanes compute the same rotation.  No LDS access or barrier.  Returns the
// sweeps taken (max_sweeps + 1 when the limit was hit).
__device__ __forceinline__ int wave8_jacobi(double &x, int l, int max_sweeps)
{
    const int lane = threadIdx.x % kWave, r = lane & 7, c = lane >> 3;
    const int n2 = l + (l & 1);
    const double tol = (double)l * 2.0 * kU;
    const bool live = c < n2;
    int sweeps;
    for (sweeps = 1; sweeps <= max_sweeps; ++sweeps) {
        int rot = 0;
        for (int rd = 0; rd < n2 - 1; ++rd) {
            // the partner, without branches
            int d2 = 2 * rd - c;
            d2 += d2 < 0 ? n2 - 1 : 0;
            d2 -= d2 >= n2 - 1 ? n2 - 1 : 0;
            int d = c == n2 - 1 ? rd : (c == rd ? n2 - 1 : d2);
            d = live ? d : c;
            const double y = __shfl(x, (d << 3) | r, kWave);
            double o2 = x * x, p2 = y * y, cr = x * y;
            seg8_sum3(o2, p2, cr);
            const bool isp = c < d;
            const double al = isp ? o2 : p2, be = isp ? p2 : o2;
            const bool doit = live && d != c && jacobi_needed(al, be, cr, tol);
            if (doit) {
                double cs, sn;
                jacobi_rotation(al, be, cr, cs, sn);
                x = isp ? cs * x - sn * y : sn * y + cs * x;
            }
            rot |= __any(doit && jacobi_needed(al, be, cr, kJacobiQuadStop)) ? 1 : 0;
        }
        if (!rot) break;
    }
    return sweeps;
}

// One-sided Jacobi on the n columns (length rows, stride ld) of M by groups
// of G lanes (G = 8, 16, 32 or 64): a group rotates one pair of the round,
// lane i of the group holding rows i, i + G, ..., i + (E - 1) G in
// registers.  With PAD the caller keeps ld >= G E and zeros in rows
// [rows, G E) of every column, so loads and stores need no bounds.  Rounds
// with more pairs than groups take several passes (their pairs are
// disjoint); one block barrier per round.  M may be in LDS or global memory.
//
// work (optional, LDS): the group leaders add the pairs they examined times
// rows to work[0], the rotations they applied times rows to work[1] and the
// rotations to work[2] (the floating-point work of the sweeps: 6 rows per
// examined pair for the three inner products, 6 rows per rotation for the
// update, and the rotation's angle).
template <int NT, int G, int E, bool PAD = false>
__device__ __forceinline__ int jacobi_groups(double *M, int rows, int ld, int n, int max_sweeps, int *sh_rot,
                                             unsigned long long *work = nullptr)
{
    unsigned npair = 0, nrot = 0;
    constexpr int ngroups = NT / G;
    const int gl = threadIdx.x % G, gid = threadIdx.x / G;
    const int n2 = n + (n & 1), npairs = n2 / 2;
    const double tol = (double)(rows > 1 ? rows : 1) * 2.0 * kU;
    int sweep;
    for (sweep = 1; sweep <= max_sweeps; ++sweep) {
        if (threadIdx.x == 0) *sh_rot = 0;
        __syncthreads();
        for (int round = 0; round < n2 - 1; ++round) {
            for (int t0 = 0; t0 < npairs; t0 += ngroups) {
                const int t = t0 + gid;
                int p = 0, q = 0;
                bool live = false;
                if (t < npairs) {
                    circle_pair(n2, round, t, p, q);
                    live = q < n;
                }
                if (!live) p = q = 0;  // a group without a pair reads column 0
                double *mp = M + (size_t)p * ld, *mq = M + (size_t)q * ld;
                double x[E], y[E];
                double al = 0.0, be = 0.0, ga = 0.0;
                if (PAD) {
                    // rows [rows, G E) hold zeros: plain loads
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        x[e] = mp[gl + G * e];
                        y[e] = mq[gl + G * e];
                    }
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        al += x[e] * x[e];
                        be += y[e] * y[e];
                        ga += x[e] * y[e];
                    }
                } else {
                    // loads at clamped addresses, masked afterwards (no
                    // branch per element)
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        const int i = gl + G * e;
                        const int ic = i < rows ? i : 0;
                        x[e] = mp[ic];
                        y[e] = mq[ic];
                    }
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        const bool in = live && gl + G * e < rows;
                        x[e] = in ? x[e] : 0.0;
                        y[e] = in ? y[e] : 0.0;
                        al += x[e] * x[e];
                        be += y[e] * y[e];
                        ga += x[e] * y[e];
                    }
                }
                if (G == 8) {
                    al = seg8_sum(al);
                    be = seg8_sum(be);
                    ga = seg8_sum(ga);
                } else if (G == 16) {
                    al = seg16_sum(al);
                    be = seg16_sum(be);
                    ga = seg16_sum(ga);
                } else if (G == 32) {
                    al = seg32_sum(al);
                    be = seg32_sum(be);
                    ga = seg32_sum(ga);
                } else {
                    al = wave_sum(al);
                    be = wave_sum(be);
                    ga = wave_sum(ga);
                }
                const bool doit = live && jacobi_needed(al, be, ga, tol);
                if (doit) {
                    double cs, sn;
                    jacobi_rotation(al, be, ga, cs, sn);
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        const int i = gl + G * e;
                        if (PAD || i < rows) {
                            mp[i] = cs * x[e] - sn * y[e];
                            mq[i] = sn * x[e] + cs * y[e];
                        }
                    }
                    if (gl == 0 && jacobi_needed(al, be, ga, kJacobiQuadStop)) *sh_rot = 1;
                }
                npair += live ? 1u : 0u;
                nrot += doit ? 1u : 0u;
            }
            __syncthreads();
        }
        const int rot = *sh_rot;
        __syncthreads();
        if (!rot) break;
    }
    if (work && gl == 0 && npair) {
        atomicAdd(&work[0], (unsigned long long)npair * (unsigned)rows);
        atomicAdd(&work[1], (unsigned long long)nrot * (unsigned)rows);
        atomicAdd(&work[2], (unsigned long long)nrot);
    }
    return sweep;
}

// Groups of G lanes a cyclic sweep of one-sided Jacobi needs with the
// nested ordering below (n columns): 2^L ceil(n / 2^(L+1)) at its widest
// level, at most n rounded up to a power of two, halved.
__host__ __device__ __forceinline__ int jacobi_nested_groups(int n)
{
    int need = 1, s = n, lv = 0;
    while (s >= 2) {
        const int h = (s + 1) / 2;
        need = (1 << lv) * h > need ? (1 << lv) * h : need;
        s = h;
        ++lv;
    }
    return need;
}

// One-sided Jacobi as jacobi_groups (PAD layout: ld >= G E, zeros in rows
// [rows, G E)), with a nested ordering in which each group keeps one column
// of its pair in registers for many steps, so that a step moves one column
// per group through LDS instead of two.  Level 0 pairs every column of the
// first half of [0, n) (padded to even length; the pad is a column that
// never exists) with every column of the second half: group q keeps column
// q and meets second-half column hs + (q + st) mod hs at step st.  Each half
// is then split the same way (level 1, its pairs all disjoint from the
// other half's), and so on down to halves of one column: every pair exactly
// once per sweep, in sum_l ceil(s_l / 2) steps (s_0 = n, s_{l+1} =
// ceil(s_l / 2); 111 steps for n = 110, against 109 rounds of the circle
// ordering).  The moving column of a step was written back by the
// neighbouring group in the step before; one block barrier per step.
// Requires NT / G >= jacobi_nested_groups(n); returns the sweeps as
// jacobi_groups does (the same rotation test and stopping rule).
template <int NT, int G, int E>
__device__ __forceinline__ int jacobi_nested(double *M, int rows, int ld, int n, int max_sweeps, int *sh_rot)
{
    const int gl = threadIdx.x % G, gid = threadIdx.x / G;
    const double tol = (double)(rows > 1 ? rows : 1) * 2.0 * kU;
    int sweep;
    for (sweep = 1; sweep <= max_sweeps; ++sweep) {
        if (threadIdx.x == 0) *sh_rot = 0;
        __syncthreads();
        for (int lv = 0, s = n; s >= 2; ++lv, s = (s + 1) / 2) {
            const int h = (s + 1) / 2;
            const int k = gid / h, q = gid % h;
            // this group's set [a, b): node k of depth lv of the halving tree
            int a = 0, b = n;
            for (int d = lv - 1; d >= 0; --d) {
                const int m = b - a, mid = a + (m + 1) / 2;
                if ((k >> d) & 1) a = mid;
                else b = mid;
            }
            const int hs = (b - a + 1) / 2;
            const bool grp = k < (1 << lv) && q < hs && b - a >= 2;
            const int f = a + q;
            double xf[E], ym[E];
            double *mf = M + (size_t)(grp ? f : 0) * ld;
#pragma unroll
            for (int e = 0; e < E; ++e) xf[e] = mf[gl + G * e];
            for (int st = 0; st < h; ++st) {
                const int c = a + hs + (q + st) % (hs > 0 ? hs : 1);
                const bool live = grp && st < hs && c < b;
                double *mc = M + (size_t)(live ? c : 0) * ld;
                double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    ym[e] = mc[gl + G * e];
                    al += xf[e] * xf[e];
                    be += ym[e] * ym[e];
                    ga += xf[e] * ym[e];
                }
                if (G == 8) {
                    al = seg8_sum(al);
                    be = seg8_sum(be);
                    ga = seg8_sum(ga);
                } else if (G == 16) {
                    al = seg16_sum(al);
                    be = seg16_sum(be);
                    ga = seg16_sum(ga);
                } else if (G == 32) {
                    al = seg32_sum(al);
                    be = seg32_sum(be);
                    ga = seg32_sum(ga);
                } else {
                    al = wave_sum(al);
                    be = wave_sum(be);
                    ga = wave_sum(ga);
                }
                if (live && jacobi_needed(al, be, ga, tol)) {
                    double cs, sn;
                    jacobi_rotation(al, be, ga, cs, sn);
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        const double x = xf[e], y = ym[e];
                        xf[e] = cs * x - sn * y;
                        mc[gl + G * e] = sn * x + cs * y;
                    }
                    if (gl == 0 && jacobi_needed(al, be, ga, kJacobiQuadStop)) *sh_rot = 1;
                }
                __syncthreads();
            }
            if (grp) {
#pragma unroll
                for (int e = 0; e < E; ++e) mf[gl + G * e] = xf[e];
            }
            __syncthreads();
        }
        const int rot = *sh_rot;
        __syncthreads();
        if (!rot) break;
    }
    return sweep;
}

}  // namespace frk
