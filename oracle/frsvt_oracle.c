/*
 * frsvt_oracle.c -- plain, slow, obviously-correct FP64 CPU reference for
 * fast randomized singular value thresholding (FRSVT) and the inexact-ALM
 * RPCA loop that hosts it (Oh, Matsushita, Tai, Kweon, arXiv:1509.00296).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the GPU product path.  No BLAS,
 * no LAPACK, no blocking, no fusion: every step is the textbook definition or
 * the paper's algorithm step, in the paper's order.
 *
 * Storage: column-major double, AT(M, ld, i, j) = M[i + j*ld].
 */
#include "frsvt_oracle.h"

#ifdef _OPENMP
#include <omp.h>
#endif

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define AT(M, ld, i, j) (M)[(size_t)(i) + (size_t)(j) * (size_t)(ld)]

static double *dalloc(int64_t count)
{
    if (count < 1) count = 1;
    return (double *)calloc((size_t)count, sizeof(double));
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11, Sec. 4): ten rounds of two 32x32->64
 * multiplies, the key bumped by the Weyl constants between rounds.         */
/* ------------------------------------------------------------------------ */

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 27 high bits of a and 26 high bits of b give a 53-bit integer c; the value
 * (c + 1/2) 2^-53 lies in (0, 1] (the top code rounds to 1.0), so the
 * logarithm taken of it below is always finite. */
double orc_uniform53(uint32_t a, uint32_t b)
{
    double hi = (double)(a >> 5);
    double lo = (double)(b >> 6);
    return (hi * 67108864.0 + lo + 0.5) * (1.0 / 9007199254740992.0);
}

/* Omega of Alg. 1 (both sampling steps): Sec. 2.4 takes a dense test matrix
 * with iid N(0,1) entries.  Box-Muller turns each Philox output into two
 * normals.  */
void orc_gaussian_matrix(uint64_t seed, uint64_t counter, int64_t rows, int64_t cols,
                         double *Om, int64_t ld)
{
    const double two_pi = 6.283185307179586476925286766559;
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t k = 0; k < rows; ++k) {
        for (int64_t j = 0; 2 * j < cols; ++j) {
            uint32_t ctr[4] = {(uint32_t)k, (uint32_t)j, (uint32_t)counter,
                               (uint32_t)(counter >> 32)};
            uint32_t x[4];
            orc_philox4x32_10(ctr, key, x);
            double u1 = orc_uniform53(x[0], x[1]);
            double u2 = orc_uniform53(x[2], x[3]);
            double radius = sqrt(-2.0 * log(u1));
            double angle = two_pi * u2;
            AT(Om, ld, k, 2 * j) = radius * cos(angle);
            if (2 * j + 1 < cols) AT(Om, ld, k, 2 * j + 1) = radius * sin(angle);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Small dense helpers (textbook loops)                                      */
/* ------------------------------------------------------------------------ */

/* C (m x n) = A (m x k) * B (k x n) */
static void mat_mul(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda,
                    const double *B, int64_t ldb, double *C, int64_t ldc)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) AT(C, ldc, i, j) = 0.0;
        for (int64_t p = 0; p < k; ++p) {
            double b = AT(B, ldb, p, j);
            if (b == 0.0) continue;
            for (int64_t i = 0; i < m; ++i) AT(C, ldc, i, j) += AT(A, lda, i, p) * b;
        }
    }
}

/* C (m x n) = A^T B with A (k x m), B (k x n) */
static void mat_mul_tn(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda,
                       const double *B, int64_t ldb, double *C, int64_t ldc)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0;
            for (int64_t p = 0; p < k; ++p) s += AT(A, lda, p, i) * AT(B, ldb, p, j);
            AT(C, ldc, i, j) = s;
        }
}

static void mat_transpose(int64_t m, int64_t n, const double *A, int64_t lda, double *T,
                          int64_t ldt)
{
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) AT(T, ldt, j, i) = AT(A, lda, i, j);
}

static void mat_copy(int64_t m, int64_t n, const double *A, int64_t lda, double *B, int64_t ldb)
{
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) AT(B, ldb, i, j) = AT(A, lda, i, j);
}

static double col_dot(int64_t m, const double *x, const double *y)
{
    double s = 0.0;
    for (int64_t i = 0; i < m; ++i) s += x[i] * y[i];
    return s;
}

static double col_norm(int64_t m, const double *x)
{
    return sqrt(col_dot(m, x, x));
}

/* ------------------------------------------------------------------------ */
/* Householder reflector: for x (length len) find v (v[0] = 1) and beta with */
/* (I - beta v v^T) x = alpha e_1.  Golub & Van Loan, Matrix Computations,   */
/* Alg. 5.1.1.  v overwrites x[1..]; returns alpha, writes beta.             */
/* ------------------------------------------------------------------------ */
static double householder(int64_t len, double *x, double *beta)
{
    double nrm = col_norm(len, x);
    if (nrm == 0.0) {
        *beta = 0.0;
        return 0.0;
    }
    double x0 = x[0];
    double alpha = (x0 >= 0.0) ? -nrm : nrm;
    double v0 = x0 - alpha;
    for (int64_t i = 1; i < len; ++i) x[i] /= v0;
    *beta = -v0 / alpha;
    x[0] = alpha;
    return alpha;
}

/* Apply (I - beta v v^T), v = [1; W(j+1:m, j)], to columns c0..c1-1 of W. */
static void apply_reflector(int64_t m, int64_t j, double beta, double *W, int64_t ldw,
                            int64_t c0, int64_t c1)
{
    if (beta == 0.0) return;
#pragma omp parallel for schedule(static)
    for (int64_t c = c0; c < c1; ++c) {
        double s = AT(W, ldw, j, c);
        for (int64_t i = j + 1; i < m; ++i) s += AT(W, ldw, i, j) * AT(W, ldw, i, c);
        s *= beta;
        AT(W, ldw, j, c) -= s;
        for (int64_t i = j + 1; i < m; ++i) AT(W, ldw, i, c) -= s * AT(W, ldw, i, j);
    }
}

/* Form the first ncols columns of H_0 H_1 ... H_{nref-1}, reflectors stored
 * below the diagonal of W (m x nref), by backward accumulation. */
static void form_q(int64_t m, int64_t nref, int64_t ncols, const double *W, int64_t ldw,
                   const double *beta, double *Q, int64_t ldq)
{
    for (int64_t j = 0; j < ncols; ++j)
        for (int64_t i = 0; i < m; ++i) AT(Q, ldq, i, j) = (i == j) ? 1.0 : 0.0;
    for (int64_t j = nref - 1; j >= 0; --j) {
        if (beta[j] == 0.0) continue;
        for (int64_t c = j; c < ncols; ++c) {
            double s = AT(Q, ldq, j, c);
            for (int64_t i = j + 1; i < m; ++i) s += AT(W, ldw, i, j) * AT(Q, ldq, i, c);
            s *= beta[j];
            AT(Q, ldq, j, c) -= s;
            for (int64_t i = j + 1; i < m; ++i) AT(Q, ldq, i, c) -= s * AT(W, ldw, i, j);
        }
    }
}

int orc_qr(int64_t m, int64_t n, const double *A, int64_t lda, double *Q, int64_t ldq,
           double *R, int64_t ldr)
{
    if (m < 0) return -1;
    if (n < 0 || n > m) return -2;
    if (lda < (m > 1 ? m : 1)) return -4;
    double *W = dalloc(m * n);
    double *beta = dalloc(n);
    mat_copy(m, n, A, lda, W, m);
    for (int64_t j = 0; j < n; ++j) {
        householder(m - j, &AT(W, m, j, j), &beta[j]);
        apply_reflector(m, j, beta[j], W, m, j + 1, n);
    }
    if (R)
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i) AT(R, ldr, i, j) = (i <= j) ? AT(W, m, i, j) : 0.0;
    if (Q) form_q(m, n, n, W, m, beta, Q, ldq);
    free(W);
    free(beta);
    return 0;
}

/* QR with column pivoting (Businger & Golub): at step j the remaining column
 * of largest norm is moved to position j.  Column norms are recomputed from
 * scratch at each step (slow and plain).  This is the QR_CP of Alg. 1's fresh sketch
 * and Sec. 2.1, which also yields the real sampling rate s = min(l, r). */
int64_t orc_qrcp_basis(int64_t m, int64_t n, const double *A, int64_t lda, double *Q,
                       int64_t ldq)
{
    int64_t kmax = m < n ? m : n;
    double *W = dalloc(m * n);
    double *beta = dalloc(n);
    double *tmp = dalloc(m);
    mat_copy(m, n, A, lda, W, m);
    for (int64_t j = 0; j < kmax; ++j) {
        int64_t best = j;
        double best_norm = -1.0;
        for (int64_t c = j; c < n; ++c) {
            double nc = col_norm(m - j, &AT(W, m, j, c));
            if (nc > best_norm) {
                best_norm = nc;
                best = c;
            }
        }
        if (best != j) {
            memcpy(tmp, &AT(W, m, 0, j), (size_t)m * sizeof(double));
            memcpy(&AT(W, m, 0, j), &AT(W, m, 0, best), (size_t)m * sizeof(double));
            memcpy(&AT(W, m, 0, best), tmp, (size_t)m * sizeof(double));
        }
        householder(m - j, &AT(W, m, j, j), &beta[j]);
        apply_reflector(m, j, beta[j], W, m, j + 1, n);
    }
    double r00 = kmax > 0 ? fabs(AT(W, m, 0, 0)) : 0.0;
    double tol = (double)(m > n ? m : n) * DBL_EPSILON * r00;
    int64_t s = 0;
    while (s < kmax && fabs(AT(W, m, s, s)) > tol) ++s;
    if (Q && s > 0) form_q(m, s, s, W, m, beta, Q, ldq);
    free(W);
    free(beta);
    free(tmp);
    return s;
}

/* ------------------------------------------------------------------------ */
/* One-sided Jacobi (Hestenes) SVD.                                          */
/* ------------------------------------------------------------------------ */

/* Orthogonalise the n columns of G (m x n, m >= n) by plane rotations
 * G <- G J, accumulating V <- V J (V starts as I).  Pairs are visited in
 * cyclic-by-row order; a pair is rotated when its cosine |g_p.g_q| /
 * (|g_p| |g_q|) exceeds m * 2^-52.  Returns the number of sweeps, or -1. */
static int jacobi_orthogonalise(int64_t m, int64_t n, double *G, int64_t ldg, double *V,
                                int64_t ldv, int max_sweeps)
{
    const double tol = (double)(m > 1 ? m : 1) * DBL_EPSILON;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) AT(V, ldv, i, j) = (i == j) ? 1.0 : 0.0;
    for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
        int rotated = 0;
        for (int64_t p = 0; p + 1 < n; ++p) {
            for (int64_t q = p + 1; q < n; ++q) {
                double *gp = &AT(G, ldg, 0, p), *gq = &AT(G, ldg, 0, q);
                double alpha = col_dot(m, gp, gp);
                double beta = col_dot(m, gq, gq);
                double gamma = col_dot(m, gp, gq);
                if (fabs(gamma) <= tol * sqrt(alpha * beta)) continue;
                /* rotation that zeroes the (p,q) entry of G^T G */
                double zeta = (beta - alpha) / (2.0 * gamma);
                double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + hypot(1.0, zeta));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = c * t;
                for (int64_t i = 0; i < m; ++i) {
                    double a = gp[i], b = gq[i];
                    gp[i] = c * a - s * b;
                    gq[i] = s * a + c * b;
                }
                double *vp = &AT(V, ldv, 0, p), *vq = &AT(V, ldv, 0, q);
                for (int64_t i = 0; i < n; ++i) {
                    double a = vp[i], b = vq[i];
                    vp[i] = c * a - s * b;
                    vq[i] = s * a + c * b;
                }
                rotated = 1;
            }
        }
        if (!rotated) return sweep;
    }
    return -1;
}

/* Replace the columns of U (m x k) flagged in `missing` by an orthonormal
 * completion of the others, built from standard basis vectors (classical
 * Gram-Schmidt applied twice). */
static void complete_orthonormal(int64_t m, int64_t k, double *U, int64_t ldu,
                                 const int *missing)
{
    double *u = dalloc(m);
    int64_t next_e = 0;
    for (int64_t j = 0; j < k; ++j) {
        if (!missing[j]) continue;
        for (; next_e < m; ++next_e) {
            for (int64_t i = 0; i < m; ++i) u[i] = (i == next_e) ? 1.0 : 0.0;
            for (int pass = 0; pass < 2; ++pass)
                for (int64_t c = 0; c < k; ++c) {
                    if (missing[c] && c >= j) continue;
                    double d = col_dot(m, &AT(U, ldu, 0, c), u);
                    for (int64_t i = 0; i < m; ++i) u[i] -= d * AT(U, ldu, i, c);
                }
            double nu = col_norm(m, u);
            if (nu > 0.5) {
                for (int64_t i = 0; i < m; ++i) AT(U, ldu, i, j) = u[i] / nu;
                ++next_e;
                break;
            }
        }
    }
    free(u);
}

int orc_svd(int64_t m, int64_t n, const double *A, int64_t lda, double *U, int64_t ldu,
            double *S, double *V, int64_t ldv)
{
    if (m < 1) return -1;
    if (n < 1) return -2;
    if (lda < m) return -4;
    if (m < n) {
        /* SVD of A^T = V S U^T */
        double *At = dalloc(n * m);
        mat_transpose(m, n, A, lda, At, n);
        int rc = orc_svd(n, m, At, n, V, ldv, S, U, ldu);
        free(At);
        return rc;
    }
    /* m >= n: A = Q R (Householder), then Jacobi on R: R V = U_R Sigma. */
    double *Q = dalloc(m * n), *R = dalloc(n * n), *VR = dalloc(n * n);
    orc_qr(m, n, A, lda, Q, m, R, n);
    int sweeps = jacobi_orthogonalise(n, n, R, n, VR, n, 80);
    double *sig = dalloc(n);
    int64_t *order = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    for (int64_t j = 0; j < n; ++j) {
        sig[j] = col_norm(n, &AT(R, n, 0, j));
        order[j] = j;
    }
    /* sort descending (selection sort on an index array) */
    for (int64_t a = 0; a < n; ++a) {
        int64_t best = a;
        for (int64_t b = a + 1; b < n; ++b)
            if (sig[order[b]] > sig[order[best]]) best = b;
        int64_t t = order[a];
        order[a] = order[best];
        order[best] = t;
    }
    double *UR = dalloc(n * n);
    int *missing = (int *)calloc((size_t)n, sizeof(int));
    for (int64_t a = 0; a < n; ++a) {
        int64_t j = order[a];
        S[a] = sig[j];
        for (int64_t i = 0; i < n; ++i) {
            AT(V, ldv, i, a) = AT(VR, n, i, j);
            AT(UR, n, i, a) = sig[j] > 0.0 ? AT(R, n, i, j) / sig[j] : 0.0;
        }
        missing[a] = !(sig[j] > 0.0);
    }
    complete_orthonormal(n, n, UR, n, missing);
    mat_mul(m, n, n, Q, m, UR, n, U, ldu);
    free(Q); free(R); free(VR); free(sig); free(order); free(UR); free(missing);
    return sweeps < 0 ? 1080 : sweeps;
}

/* ------------------------------------------------------------------------ */
/* Exact SVT, Def. 1, Eq. (3); soft shrinkage S_tau(x) = sgn(x)max(|x|-tau,0) */
/* ------------------------------------------------------------------------ */

static double soft_shrink(double x, double tau)
{
    double a = fabs(x) - tau;
    if (a <= 0.0) return 0.0;
    return x > 0.0 ? a : -a;
}

/* X = sum_i shrunk_i u_i v_i^T over the first `count` singular triplets. */
static void rank_sum(int64_t m, int64_t n, int64_t count, const double *U, int64_t ldu,
                     const double *shrunk, const double *V, int64_t ldv, double *X, int64_t ldx)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        for (int64_t i = 0; i < m; ++i) AT(X, ldx, i, j) = 0.0;
        for (int64_t c = 0; c < count; ++c) {
            double coef = shrunk[c] * AT(V, ldv, j, c);
            if (coef == 0.0) continue;
            for (int64_t i = 0; i < m; ++i) AT(X, ldx, i, j) += coef * AT(U, ldu, i, c);
        }
    }
}

int orc_svt(int64_t m, int64_t n, const double *A, int64_t lda, double tau, double *X,
            int64_t ldx, int64_t *rank)
{
    if (m < 1) return -1;
    if (n < 1) return -2;
    if (lda < m) return -4;
    if (!(tau >= 0.0)) return -5;
    if (ldx < m) return -7;
    int64_t k = m < n ? m : n;
    double *U = dalloc(m * k), *S = dalloc(k), *V = dalloc(n * k), *shr = dalloc(k);
    int sweeps = orc_svd(m, n, A, lda, U, m, S, V, n);
    int64_t r = 0;
    for (int64_t i = 0; i < k; ++i) {
        shr[i] = soft_shrink(S[i], tau);
        if (S[i] > tau) ++r;
    }
    rank_sum(m, n, r, U, m, shr, V, n, X, ldx);
    if (rank) *rank = r;
    free(U); free(S); free(V); free(shr);
    return sweeps >= 1000 ? 1 : 0;
}

/* Partial SVT (the proximal step of the truncated nuclear norm, Type B of
 * Table 6): the keep largest singular values pass unshrunk, the others are
 * soft-thresholded by tau; rank counts the nonzero results. */
int orc_psvt(int64_t m, int64_t n, const double *A, int64_t lda, double tau, int64_t keep,
             double *X, int64_t ldx, int64_t *rank)
{
    if (m < 1) return -1;
    if (n < 1) return -2;
    if (lda < m) return -4;
    if (!(tau >= 0.0)) return -5;
    if (keep < 0) return -6;
    if (ldx < m) return -8;
    int64_t k = m < n ? m : n;
    double *U = dalloc(m * k), *S = dalloc(k), *V = dalloc(n * k), *shr = dalloc(k);
    int sweeps = orc_svd(m, n, A, lda, U, m, S, V, n);
    int64_t r = 0;
    for (int64_t i = 0; i < k; ++i) {
        shr[i] = i < keep ? S[i] : soft_shrink(S[i], tau);
        if (shr[i] > 0.0) ++r;
    }
    rank_sum(m, n, r, U, m, shr, V, n, X, ldx);
    if (rank) *rank = r;
    free(U); free(S); free(V); free(shr);
    return sweeps >= 1000 ? 1 : 0;
}

/* Weighted SVT (the WSVT of the weighted nuclear norm named in Sec. 1 and
 * footnote 1): threshold the i-th largest singular value by w_i. */
int orc_wsvt(int64_t m, int64_t n, const double *A, int64_t lda, const double *w, double *X,
             int64_t ldx, int64_t *rank)
{
    if (m < 1) return -1;
    if (n < 1) return -2;
    if (lda < m) return -4;
    if (!w) return -5;
    if (ldx < m) return -7;
    int64_t k = m < n ? m : n;
    double *U = dalloc(m * k), *S = dalloc(k), *V = dalloc(n * k), *shr = dalloc(k);
    int sweeps = orc_svd(m, n, A, lda, U, m, S, V, n);
    int64_t r = 0;
    for (int64_t i = 0; i < k; ++i) {
        double d = S[i] - w[i];
        shr[i] = d > 0.0 ? d : 0.0;
        if (d > 0.0) ++r;
    }
    rank_sum(m, n, k, U, m, shr, V, n, X, ldx);
    if (rank) *rank = r;
    free(U); free(S); free(V); free(shr);
    return sweeps >= 1000 ? 1 : 0;
}

/* Weighted SVT under the patch-group weight rule (the weights are a
 * function of each singular value; the noise level enters through the
 * column count n and the per-entry noise variance). */
int orc_wsvt_rule(int64_t m, int64_t n, const double *A, int64_t lda, double c,
                  double noise_var, double eps, double tau, double *X, int64_t ldx,
                  int64_t *rank)
{
    if (m < 1) return -1;
    if (n < 1) return -2;
    if (lda < m) return -4;
    if (ldx < m) return -10;
    int64_t k = m < n ? m : n;
    double *U = dalloc(m * k), *S = dalloc(k), *V = dalloc(n * k), *shr = dalloc(k);
    int sweeps = orc_svd(m, n, A, lda, U, m, S, V, n);
    int64_t r = 0;
    for (int64_t i = 0; i < k; ++i) {
        double w = tau;
        if (c > 0.0) {
            double e = S[i] * S[i] - (double)n * noise_var;
            double sh = e > 0.0 ? sqrt(e) : 0.0;
            w = c * sqrt((double)n) / (sh + eps);
        }
        double d = S[i] - w;
        shr[i] = d > 0.0 ? d : 0.0;
        if (d > 0.0) ++r;
    }
    rank_sum(m, n, k, U, m, shr, V, n, X, ldx);
    if (rank) *rank = r;
    free(U); free(S); free(V); free(shr);
    return sweeps >= 1000 ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* FRSVT, Alg. 1                                                            */
/* ------------------------------------------------------------------------ */

/* PartialOrthogonalization of Alg. 1 (Sec. 2.1, "Range Propagation"):
 * modified Gram-Schmidt of each new sample y_j against the propagated basis
 * and the new vectors accepted before it, the projection pass done twice,
 * then normalisation.  Q holds `have` orthonormal columns on entry; the
 * normalised y_j are appended as columns have..have+p-1. */
static void partial_orthogonalisation(int64_t m, double *Q, int64_t ldq, int64_t have,
                                      const double *Y, int64_t ldy, int64_t p)
{
    double *y = dalloc(m);
    int *missing = (int *)calloc((size_t)(have + p), sizeof(int));
    for (int64_t j = 0; j < p; ++j) {
        memcpy(y, &AT(Y, ldy, 0, j), (size_t)m * sizeof(double));
        for (int pass = 0; pass < 2; ++pass)
            for (int64_t c = 0; c < have + j; ++c) {
                if (missing[c]) continue;
                double d = col_dot(m, &AT(Q, ldq, 0, c), y);
                for (int64_t i = 0; i < m; ++i) y[i] -= d * AT(Q, ldq, i, c);
            }
        double after = col_norm(m, y);
        if (after > 0.0) {
            for (int64_t i = 0; i < m; ++i) AT(Q, ldq, i, have + j) = y[i] / after;
        } else {
            missing[have + j] = 1;
        }
    }
    complete_orthonormal(m, have + p, Q, ldq, missing);
    free(y);
    free(missing);
}

int orc_frsvt_keep(int64_t m, int64_t n, const double *A, int64_t lda, double tau, int64_t keep,
                   int q, const double *Om, int64_t ldom, int64_t nomega, const double *Qt,
                   int64_t ldqt, int64_t r_prev, double *X, int64_t ldx, double *Qout,
                   int64_t ldqo, int64_t *r_out, double *sigma, int64_t *s_out)
{
    if (m < 1) return -1;
    if (n < 1) return -2;
    if (lda < m) return -4;
    if (!(tau >= 0.0)) return -5;
    if (q < 0) return -6;
    /* Orientation (Sec. 2.5): work on Ahat with mhat = min(m,n) rows so that
     * the power iteration acts on the short side. */
    const int transposed = m > n;
    const int64_t mh = transposed ? n : m, nh = transposed ? m : n;
    if (!Om || ldom < nh) return -8;
    if (nomega < 0 || (nomega < 1 && !(Qt && r_prev > 0))) return -9;
    if (Qt && (r_prev < 0 || r_prev > mh || ldqt < mh)) return -12;
    if (ldx < m) return -14;

    double *Ah = dalloc(mh * nh);
    if (transposed) mat_transpose(m, n, A, lda, Ah, mh);
    else mat_copy(m, n, A, lda, Ah, mh);

    /* Alg. 1, the initial basis Q (mhat x s). */
    int64_t lmax = (Qt ? r_prev : 0) + nomega;
    if (lmax > mh) lmax = mh;
    double *Q = dalloc(mh * lmax);
    int64_t s;
    if (!Qt || r_prev == 0) {
        int64_t l = nomega < mh ? nomega : mh;
        double *Y = dalloc(mh * l);
        mat_mul(mh, l, nh, Ah, mh, Om, ldom, Y, mh);  /* Y = A Omega */
        s = orc_qrcp_basis(mh, l, Y, mh, Q, mh);      /* Q = QR_CP(Y) */
        free(Y);
        if (s == 0) { /* A Omega == 0: keep one arbitrary direction */
            int miss = 1;
            complete_orthonormal(mh, 1, Q, mh, &miss);
            s = 1;
        }
    } else {
        int64_t p = lmax - r_prev;
        mat_copy(mh, r_prev, Qt, ldqt, Q, mh);
        if (p > 0) {
            double *Y = dalloc(mh * p);
            mat_mul(mh, p, nh, Ah, mh, Om, ldom, Y, mh);      /* Y = A Omega_p */
            partial_orthogonalisation(mh, Q, mh, r_prev, Y, mh, p); /* Q = [Q~, Q_Y] */
            free(Y);
        }
        s = lmax;
    }

    /* Power iterations: Q = QR(A A^T Q), q times. */
    double *Z = dalloc(nh * s), *Y = dalloc(mh * s), *Rtmp = dalloc(s * s);
    for (int it = 0; it < q; ++it) {
        mat_mul_tn(nh, s, mh, Ah, mh, Q, mh, Z, nh); /* Z = A^T Q */
        mat_mul(mh, s, nh, Ah, mh, Z, nh, Y, mh);    /* Y = A Z   */
        orc_qr(mh, s, Y, mh, Q, mh, Rtmp, s);
    }

    /* [H, C] = QR(A^T Q), Bt = A^T Q is nhat x s. */
    double *Bt = Z;
    mat_mul_tn(nh, s, mh, Ah, mh, Q, mh, Bt, nh);
    double *H = dalloc(nh * s), *C = dalloc(s * s);
    orc_qr(nh, s, Bt, nh, H, nh, C, s);

    /* The polar and eigen steps compute C = (W V) D V^T, an SVD of the core matrix C.  The
     * oracle obtains the same factorisation directly with the Jacobi SVD:
     * C = UC diag(D) VC^T, so V = VC and W V = UC. */
    double *UC = dalloc(s * s), *VC = dalloc(s * s), *D = dalloc(s);
    int sweeps = orc_svd(s, s, C, s, UC, s, D, VC, s);

    /* Reconstruction, Eq. (6): S_tau(A) ~ (Q V) S_tau(D) (H W V)^T, keeping the r
     * singular values above tau (Sec. 2.3 defines r this way); with keep > 0
     * the keep largest pass unshrunk (partial SVT). */
    int64_t r = 0;
    double *shr = dalloc(s);
    for (int64_t i = 0; i < s; ++i) {
        shr[i] = i < keep ? D[i] : soft_shrink(D[i], tau);
        if (shr[i] > 0.0) ++r;
    }
    double *QV = dalloc(mh * s), *HWV = dalloc(nh * s), *Xh = dalloc(mh * nh);
    mat_mul(mh, s, s, Q, mh, VC, s, QV, mh);
    mat_mul(nh, s, s, H, nh, UC, s, HWV, nh);
    rank_sum(mh, nh, r, QV, mh, shr, HWV, nh, Xh, mh);
    if (transposed) mat_transpose(mh, nh, Xh, mh, X, ldx);
    else mat_copy(mh, nh, Xh, mh, X, ldx);

    /* Output: the propagated basis Q~ = Q V, its first r columns (Sec. 2.3). */
    if (Qout) mat_copy(mh, r, QV, mh, Qout, ldqo);
    if (r_out) *r_out = r;
    if (sigma) for (int64_t i = 0; i < s; ++i) sigma[i] = D[i];
    if (s_out) *s_out = s;

    free(Ah); free(Q); free(Z); free(Y); free(Rtmp); free(H); free(C);
    free(UC); free(VC); free(D); free(shr); free(QV); free(HWV); free(Xh);
    return sweeps >= 1000 ? 1 : 0;
}

int orc_frsvt(int64_t m, int64_t n, const double *A, int64_t lda, double tau, int q,
              const double *Om, int64_t ldom, int64_t nomega, const double *Qt,
              int64_t ldqt, int64_t r_prev, double *X, int64_t ldx, double *Qout,
              int64_t ldqo, int64_t *r_out, double *sigma, int64_t *s_out)
{
    return orc_frsvt_keep(m, n, A, lda, tau, 0, q, Om, ldom, nomega, Qt, ldqt, r_prev, X, ldx, Qout,
                          ldqo, r_out, sigma, s_out);
}

/* ------------------------------------------------------------------------ */
/* Residual singular-value estimate (Prop. 4 with Lemma 3): for Q~ (mhat x r, */
/* orthonormal columns) and one standard Gaussian vector omega (length nhat), */
/*   est = alpha sqrt(2/pi) ||(I - Q~ Q~^T) Ahat omega||_2                    */
/* bounds sigma_{r+1}(Ahat) from above with probability >= 1 - 1/alpha.  The  */
/* projection is applied twice (classical Gram-Schmidt, two passes), as the   */
/* range propagation's partial orthogonalisation forms it.                    */
/* ------------------------------------------------------------------------ */
double orc_residual_estimate(int64_t m, int64_t n, const double *A, int64_t lda, const double *Qt,
                             int64_t ldq, int64_t r, const double *omega, double alpha)
{
    const int transposed = m > n;
    const int64_t mh = transposed ? n : m;
    double *y = dalloc(mh);
    if (transposed) mat_mul_tn(mh, 1, m, A, lda, omega, m, y, mh);   /* y = A^T omega */
    else mat_mul(mh, 1, n, A, lda, omega, n, y, mh);                  /* y = A omega   */
    for (int pass = 0; pass < 2; ++pass)
        for (int64_t c = 0; c < r; ++c) {
            const double d = col_dot(mh, &AT(Qt, ldq, 0, c), y);
            for (int64_t i = 0; i < mh; ++i) y[i] -= d * AT(Qt, ldq, i, c);
        }
    const double pi = 3.14159265358979323846;
    const double est = alpha * sqrt(2.0 / pi) * col_norm(mh, y);
    free(y);
    return est;
}

/* ------------------------------------------------------------------------ */
/* Residual check that steers sampling (Sec. 3.2 after Prop. 4): the new     */
/* samples y_j = Ahat omega_j are taken in order; each is compared with the  */
/* basis it would extend, Q_j = [Q~, y_1, ..., y_{j-1}] orthonormalised, by  */
/*   s_j = alpha sqrt(2/pi) ||(I - Q_j Q_j^T) y_j||_2,                       */
/* an upper bound on sigma_{k+1}(Ahat) (k = columns of Q_j) with probability */
/* >= 1 - 1/alpha.  Once s_j <= tau no direction above the threshold is left */
/* outside [Q_j, y_j] (with that probability): sampling stops and y_j is the  */
/* last sample kept.  Returns the number of samples kept, j (all nomega when */
/* no check passes).  The projection is applied twice (classical Gram-       */
/* Schmidt, two passes).  est_out[j-1] = s_j for the samples checked.        */
/* ------------------------------------------------------------------------ */
int64_t orc_residual_check(int64_t m, int64_t n, const double *A, int64_t lda, const double *Qt,
                           int64_t ldq, int64_t r, const double *Om, int64_t ldom, int64_t nomega,
                           double tau, double alpha, double *est_out)
{
    const int transposed = m > n;
    const int64_t mh = transposed ? n : m;
    const double pi = 3.14159265358979323846;
    double *B = dalloc(mh * (r + nomega + 1));   /* the growing orthonormal basis */
    double *y = dalloc(mh);
    if (r > 0) mat_copy(mh, r, Qt, ldq, B, mh);
    int64_t k = r, kept = nomega;
    for (int64_t j = 0; j < nomega; ++j) {
        const double *om = &AT(Om, ldom, 0, j);
        if (transposed) mat_mul_tn(mh, 1, m, A, lda, om, m, y, mh);  /* y = A^T omega */
        else mat_mul(mh, 1, n, A, lda, om, n, y, mh);                 /* y = A omega   */
        for (int pass = 0; pass < 2; ++pass)
            for (int64_t c = 0; c < k; ++c) {
                const double d = col_dot(mh, &AT(B, mh, 0, c), y);
                for (int64_t i = 0; i < mh; ++i) y[i] -= d * AT(B, mh, i, c);
            }
        const double nrm = col_norm(mh, y);
        const double est = alpha * sqrt(2.0 / pi) * nrm;
        if (est_out) est_out[j] = est;
        if (est <= tau) {
            kept = j + 1;
            break;
        }
        if (nrm > 0.0) {
            for (int64_t i = 0; i < mh; ++i) AT(B, mh, i, k) = y[i] / nrm;
            ++k;
        }
    }
    free(B);
    free(y);
    return kept;
}

/* ------------------------------------------------------------------------ */
/* Inexact augmented Lagrange multiplier RPCA (the iALM host of Sec. 4.1,    */
/* "Robust PCA test"; lambda = 1/sqrt(max(m,n)) there).  The paper cites the */
/* method without formulas; this is its standard form: an SVT step on L, a   */
/* soft-shrinkage step on S, a dual ascent step on Y, mu grown by rho.      */
/* ------------------------------------------------------------------------ */
/* Sketch widths (Sec. 2.1, 2.3).  Fixed rule: first call l0 = ceil(0.1 mhat),
 * then p new samples beside the r propagated columns.  Adaptive rank
 * prediction (Eq. 7, ap != 0), with n of Eq. 7 the short side mhat:
 *   p_{i+1} = a             if r_i < l_i,
 *             ceil(rho mhat) otherwise,
 *   l_{i+1} = min(r_i + p_{i+1}, b),  b = ceil(gamma mhat),  l_0 = ceil(0.1 b);
 * the propagated basis holds r_i columns, so l_{i+1} - r_i samples are new
 * (none once r_i = b: the propagated basis alone, power iterations still
 * applied).  widths[i] = l_i. */
int orc_rpca_ialm_ap(int64_t m, int64_t n, const double *O, int64_t ldo, double lambda,
                     int svt_mode, int64_t p, int q, uint64_t seed, double tol, int max_iter,
                     double mu0, double rho, double mu_bar_factor, int ap, int64_t ap_a,
                     double ap_rho, double ap_gamma, int64_t keep, const double *Qinit,
                     int64_t r_init, double *Qfinal, int64_t *r_final, double *L, int64_t ldl,
                     double *S, int64_t lds, int64_t *ranks, int64_t *widths, double *resid_est,
                     double *resid, int *iters)
{
    return orc_rpca_ialm_rc(m, n, O, ldo, lambda, svt_mode, p, q, seed, tol, max_iter, mu0, rho,
                            mu_bar_factor, ap, ap_a, ap_rho, ap_gamma, keep, Qinit, r_init, Qfinal,
                            r_final, 0, L, ldl, S, lds, ranks, widths, resid_est, resid, iters);
}

int orc_rpca_ialm_rc(int64_t m, int64_t n, const double *O, int64_t ldo, double lambda,
                     int svt_mode, int64_t p, int q, uint64_t seed, double tol, int max_iter,
                     double mu0, double rho, double mu_bar_factor, int ap, int64_t ap_a,
                     double ap_rho, double ap_gamma, int64_t keep, const double *Qinit,
                     int64_t r_init, double *Qfinal, int64_t *r_final, int resid_check, double *L,
                     int64_t ldl, double *S, int64_t lds, int64_t *ranks, int64_t *widths,
                     double *resid_est, double *resid, int *iters)
{
    if (m < 1) return -1;
    if (n < 1) return -2;
    if (ldo < m) return -4;
    if (!(lambda > 0.0)) return -5;
    if (svt_mode != 0 && svt_mode != 1) return -6;
    if (svt_mode == 1 && p < 1 && !ap) return -7;
    if (max_iter < 1) return -11;
    if (ap && (ap_a < 1 || !(ap_rho > 0.0) || !(ap_gamma > 0.0) || ap_gamma > 1.0)) return -15;
    if (keep < 0) return -19;
    const int64_t mn = m * n;
    const int64_t mh = m < n ? m : n, nh = m < n ? n : m;

    /* ||O||_2 from the SVD, ||O||_inf = max |O_ij|, ||O||_F. */
    int64_t k = mh;
    double *U1 = dalloc(m * k), *S1 = dalloc(k), *V1 = dalloc(n * k);
    orc_svd(m, n, O, ldo, U1, m, S1, V1, n);
    double norm2 = S1[0];
    free(U1); free(S1); free(V1);
    double norm_inf = 0.0, norm_fro = 0.0;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) {
            double v = AT(O, ldo, i, j);
            if (fabs(v) > norm_inf) norm_inf = fabs(v);
            norm_fro += v * v;
        }
    norm_fro = sqrt(norm_fro);

    double *Y = dalloc(mn), *A = dalloc(mn), *Lk = dalloc(mn), *Sk = dalloc(mn);
    double J = norm2 > norm_inf / lambda ? norm2 : norm_inf / lambda;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) AT(Y, m, i, j) = AT(O, ldo, i, j) / J;
    double mu = mu0 > 0.0 ? mu0 : 1.25 / norm2;
    double mu_bar = mu * mu_bar_factor;

    double *Qt = dalloc(mh * mh), *Qnew = dalloc(mh * mh);
    int64_t r_prev = -1; /* -1: no propagated basis yet */
    if (svt_mode == 1 && Qinit && r_init > 0) {
        /* semi-online: the caller's basis is the first call's propagated basis */
        if (r_init > mh) { free(Qt); free(Qnew); free(Y); free(A); free(Lk); free(Sk); return -20; }
        mat_copy(mh, r_init, Qinit, mh, Qt, mh);
        r_prev = r_init;
    }
    int64_t bmax = mh, l_prev = r_prev > 0 ? r_prev : 0;
    if (ap) {
        bmax = (int64_t)ceil(ap_gamma * (double)mh);
        if (bmax < 1) bmax = 1;
        if (bmax > mh) bmax = mh;
    }
    int64_t l0 = (int64_t)ceil(0.1 * (double)bmax);
    if (l0 < 1) l0 = 1;
    int status = 2;
    int it;
    for (it = 0; it < max_iter; ++it) {
        /* L-step: L = SVT_{1/mu}(O - S + Y/mu) */
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < m; ++i)
                AT(A, m, i, j) = AT(O, ldo, i, j) - AT(Sk, m, i, j) + AT(Y, m, i, j) / mu;
        int64_t r = 0;
        if (svt_mode == 0) {
            orc_psvt(m, n, A, m, 1.0 / mu, keep, Lk, m, &r);
        } else {
            int64_t nomega;
            const double *Qprop = NULL;
            if (r_prev < 0) {
                nomega = l0;                         /* first call: l0 = 0.1 b */
            } else if (ap) {
                const int64_t pn = r_prev < l_prev ? ap_a : (int64_t)ceil(ap_rho * (double)mh);
                const int64_t ln = r_prev + pn < bmax ? r_prev + pn : bmax;
                if (r_prev == 0) nomega = ln;        /* nothing to propagate */
                else {
                    Qprop = Qt;
                    nomega = ln - r_prev;            /* may be 0 once r = b */
                }
            } else if (r_prev == 0) {
                nomega = p;                          /* nothing to propagate */
            } else {                                 /* range propagation */
                Qprop = Qt;
                nomega = p;
                if (r_prev + nomega > mh) nomega = mh - r_prev;
            }
            if (nomega < 1 && !Qprop) nomega = 1;
            if (nomega < 0) nomega = 0;
            double *Om = dalloc(nh * (nomega > 0 ? nomega : 1));
            if (nomega > 0) orc_gaussian_matrix(seed, (uint64_t)it, nh, nomega, Om, nh);
            /* Sec. 3.2: stop sampling once the residual estimate is below
             * this iteration's threshold */
            if (resid_check && nomega > 0)
                nomega = orc_residual_check(m, n, A, m, Qt, mh, Qprop ? r_prev : 0, Om, nh, nomega,
                                            1.0 / mu, 20.0, NULL);
            const int64_t lw = (Qprop ? r_prev : 0) + nomega;
            l_prev = lw < mh ? lw : mh;
            if (widths) widths[it] = l_prev;
            /* Prop. 4 with the first new sample (alpha = 20); -1: no sample */
            if (resid_est)
                resid_est[it] = nomega > 0 ? orc_residual_estimate(m, n, A, m, Qt, mh, Qprop ? r_prev : 0,
                                                                   Om, 20.0)
                                           : -1.0;
            orc_frsvt_keep(m, n, A, m, 1.0 / mu, keep, q, Om, nh, nomega, Qprop, mh,
                           Qprop ? r_prev : 0, Lk, m, Qnew, mh, &r, NULL, NULL);
            free(Om);
            mat_copy(mh, r, Qnew, mh, Qt, mh);
            r_prev = r;
        }
        if (ranks) ranks[it] = r;
        /* S-step: S = shrink_{lambda/mu}(O - L + Y/mu) */
        double zz = 0.0;
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < m; ++i) {
                double o = AT(O, ldo, i, j), l = AT(Lk, m, i, j);
                double s = soft_shrink(o - l + AT(Y, m, i, j) / mu, lambda / mu);
                AT(Sk, m, i, j) = s;
                double z = o - l - s;          /* primal residual */
                AT(Y, m, i, j) += mu * z;      /* dual ascent */
                zz += z * z;
            }
        double res = sqrt(zz) / norm_fro;
        if (resid) resid[it] = res;
        mu = rho * mu < mu_bar ? rho * mu : mu_bar;
        if (res < tol) {
            status = 0;
            ++it;
            break;
        }
    }
    if (iters) *iters = it;
    if (r_final) *r_final = svt_mode == 1 && r_prev > 0 ? r_prev : 0;
    if (Qfinal && svt_mode == 1 && r_prev > 0) mat_copy(mh, r_prev, Qt, mh, Qfinal, mh);
    mat_copy(m, n, Lk, m, L, ldl);
    mat_copy(m, n, Sk, m, S, lds);
    free(Y); free(A); free(Lk); free(Sk); free(Qt); free(Qnew);
    return status;
}

int orc_rpca_ialm(int64_t m, int64_t n, const double *O, int64_t ldo, double lambda,
                  int svt_mode, int64_t p, int q, uint64_t seed, double tol, int max_iter,
                  double mu0, double rho, double mu_bar_factor, double *L, int64_t ldl,
                  double *S, int64_t lds, int64_t *ranks, double *resid, int *iters)
{
    return orc_rpca_ialm_ap(m, n, O, ldo, lambda, svt_mode, p, q, seed, tol, max_iter, mu0, rho,
                            mu_bar_factor, 0, 0, 0.0, 0.0, 0, NULL, 0, NULL, NULL, L, ldl, S, lds,
                            ranks, NULL, NULL, resid, iters);
}

/* ------------------------------------------------------------------------ */
/* VJP of exact SVT.  For A = U diag(sigma) V^T (thin, m >= n, V square) and  */
/* f(s) = max(s - tau, 0), X = U f(Sigma) V^T; a perturbation dA gives       */
/*   dX = U [Gs o sym(P) + Ga o skew(P)] V^T + (I - UU^T) dA V diag(f/s) V^T, */
/* P = U^T dA V, Gs_ij = (f_i - f_j)/(s_i - s_j) (f'(s_i) on the diagonal),  */
/* Ga_ij = (f_i + f_j)/(s_i + s_j).  The adjoint follows by transposition.   */
/* ------------------------------------------------------------------------ */
int orc_svt_vjp(int64_t m, int64_t n, const double *A, int64_t lda, double tau,
                const double *Xbar, int64_t ldxb, double *Abar, int64_t ldab, double *taubar)
{
    if (m < 1) return -1;
    if (n < 1) return -2;
    if (lda < m) return -4;
    if (!(tau >= 0.0)) return -5;
    if (m < n) {
        /* SVT(A^T) = SVT(A)^T */
        double *At = dalloc(n * m), *XbT = dalloc(n * m), *AbT = dalloc(n * m);
        mat_transpose(m, n, A, lda, At, n);
        mat_transpose(m, n, Xbar, ldxb, XbT, n);
        int rc = orc_svt_vjp(n, m, At, n, tau, XbT, n, AbT, n, taubar);
        mat_transpose(n, m, AbT, n, Abar, ldab);
        free(At); free(XbT); free(AbT);
        return rc;
    }
    double *U = dalloc(m * n), *sg = dalloc(n), *V = dalloc(n * n);
    int sweeps = orc_svd(m, n, A, lda, U, m, sg, V, n);
    double *f = dalloc(n);
    for (int64_t i = 0; i < n; ++i) f[i] = sg[i] > tau ? sg[i] - tau : 0.0;

    double *XV = dalloc(m * n), *Xp = dalloc(n * n), *Pb = dalloc(n * n);
    mat_mul(m, n, n, Xbar, ldxb, V, n, XV, m);  /* Xbar V */
    mat_mul_tn(n, n, m, U, m, XV, m, Xp, n);    /* U^T Xbar V */
    double tb = 0.0;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) {
            int above_i = sg[i] > tau, above_j = sg[j] > tau;
            double gs, ga;
            if (i == j) gs = above_i ? 1.0 : 0.0;
            else if (above_i && above_j) gs = 1.0;
            else if (!above_i && !above_j) gs = 0.0;
            else if (fabs(sg[i] - sg[j]) <= 1e-12 * fmax(sg[i], sg[j])) gs = 0.5;  /* straddling pair, guard */
            else gs = (f[i] - f[j]) / (sg[i] - sg[j]);
            ga = (sg[i] + sg[j] > 0.0) ? (f[i] + f[j]) / (sg[i] + sg[j]) : 0.0;
            double xij = AT(Xp, n, i, j), xji = AT(Xp, n, j, i);
            AT(Pb, n, i, j) = gs * 0.5 * (xij + xji) + ga * 0.5 * (xij - xji);
        }
    for (int64_t i = 0; i < n; ++i)
        if (sg[i] > tau) tb -= AT(Xp, n, i, i);

    /* Abar = U Pb V^T + (I - U U^T) Xbar V diag(f/s) V^T */
    double *T = dalloc(m * n), *UtT = dalloc(n * n), *M2 = dalloc(m * n);
    for (int64_t j = 0; j < n; ++j) {
        double d = sg[j] > tau ? f[j] / sg[j] : 0.0;
        for (int64_t i = 0; i < m; ++i) AT(T, m, i, j) = AT(XV, m, i, j) * d;
    }
    mat_mul_tn(n, n, m, U, m, T, m, UtT, n);
    mat_mul(m, n, n, U, m, UtT, n, M2, m);
    double *UPb = dalloc(m * n);
    mat_mul(m, n, n, U, m, Pb, n, UPb, m);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i)
            AT(T, m, i, j) = AT(UPb, m, i, j) + AT(T, m, i, j) - AT(M2, m, i, j);
    /* Abar = T V^T */
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) {
            double s = 0.0;
            for (int64_t c = 0; c < n; ++c) s += AT(T, m, i, c) * AT(V, n, j, c);
            AT(Abar, ldab, i, j) = s;
        }
    if (taubar) *taubar = tb;
    free(U); free(sg); free(V); free(f); free(XV); free(Xp); free(Pb);
    free(T); free(UtT); free(M2); free(UPb);
    return sweeps >= 1000 ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Low-rank representation (Type A of Table 6), solved by the inexact ALM of */
/* the LRR method the paper hosts FRSVT in:                                  */
/*   min ||J||_* + lambda ||E||_{2,1}  s.t.  X = X Z + E,  Z = J,            */
/* from Z = J = E = Y1 = Y2 = 0 and mu = mu0, each iteration                */
/*   J  = SVT_{1/mu}(Z + Y2/mu)   (exact, or FRSVT + range propagation with  */
/*                                 the widths of the RPCA host, counter = k) */
/*   Z  = (I + X^T X)^{-1} (X^T (X - E) + J + (X^T Y1 - Y2)/mu)              */
/*   E  = column-wise shrink_{lambda/mu}(X - X Z + Y1/mu)                    */
/*   Y1 += mu (X - X Z - E),  Y2 += mu (Z - J),  mu = min(rho mu, mu_max)    */
/* until max|X - X Z - E| < tol and max|Z - J| < tol.                        */
/* ------------------------------------------------------------------------ */

/* In-place Cholesky A = L L^T of an SPD n x n matrix (lower triangle). */
static void chol_lower(int64_t n, double *A, int64_t lda)
{
    for (int64_t j = 0; j < n; ++j) {
        double d = AT(A, lda, j, j);
        for (int64_t k = 0; k < j; ++k) d -= AT(A, lda, j, k) * AT(A, lda, j, k);
        d = sqrt(d);
        AT(A, lda, j, j) = d;
        for (int64_t i = j + 1; i < n; ++i) {
            double s = AT(A, lda, i, j);
            for (int64_t k = 0; k < j; ++k) s -= AT(A, lda, i, k) * AT(A, lda, j, k);
            AT(A, lda, i, j) = s / d;
        }
    }
}

/* B <- (L L^T)^{-1} B for n x m B (forward then backward substitution). */
static void chol_solve(int64_t n, const double *L, int64_t ldl, int64_t m, double *B, int64_t ldb)
{
    for (int64_t c = 0; c < m; ++c) {
        double *b = &AT(B, ldb, 0, c);
        for (int64_t i = 0; i < n; ++i) {
            double s = b[i];
            for (int64_t k = 0; k < i; ++k) s -= AT(L, ldl, i, k) * b[k];
            b[i] = s / AT(L, ldl, i, i);
        }
        for (int64_t i = n - 1; i >= 0; --i) {
            double s = b[i];
            for (int64_t k = i + 1; k < n; ++k) s -= AT(L, ldl, k, i) * b[k];
            b[i] = s / AT(L, ldl, i, i);
        }
    }
}

int orc_lrr_ialm(int64_t d, int64_t n, const double *X, int64_t ldx, double lambda, int svt_mode,
                 int64_t p, int q, uint64_t seed, double tol, int max_iter, double mu0, double rho,
                 double mu_max, double *Z, int64_t ldz, double *E, int64_t lde, int64_t *ranks,
                 int *iters)
{
    if (d < 1) return -1;
    if (n < 1) return -2;
    if (ldx < d) return -4;
    if (!(lambda > 0.0)) return -5;
    if (svt_mode != 0 && svt_mode != 1) return -6;
    if (svt_mode == 1 && p < 1) return -7;
    if (max_iter < 1) return -11;
    if (!(mu0 > 0.0) || !(rho >= 1.0) || !(mu_max >= mu0)) return -12;

    double *Lc = dalloc(n * n);                    /* I + X^T X, then its Cholesky factor */
    mat_mul_tn(n, n, d, X, ldx, X, ldx, Lc, n);
    for (int64_t i = 0; i < n; ++i) AT(Lc, n, i, i) += 1.0;
    chol_lower(n, Lc, n);

    double *Zk = dalloc(n * n), *J = dalloc(n * n), *Ek = dalloc(d * n);
    double *Y1 = dalloc(d * n), *Y2 = dalloc(n * n), *XZ = dalloc(d * n);
    double *T = dalloc(n * n), *W = dalloc(d * n), *R = dalloc(n * n);
    double *Qt = dalloc(n * n), *Qnew = dalloc(n * n);
    const int64_t l0 = (int64_t)ceil(0.1 * (double)n) > 0 ? (int64_t)ceil(0.1 * (double)n) : 1;
    int64_t r_prev = -1;
    double mu = mu0;
    int status = 2, it;
    for (it = 0; it < max_iter; ++it) {
        /* J = SVT_{1/mu}(Z + Y2/mu) */
        for (int64_t i = 0; i < n * n; ++i) T[i] = Zk[i] + Y2[i] / mu;
        int64_t r = 0;
        if (svt_mode == 0) {
            orc_svt(n, n, T, n, 1.0 / mu, J, n, &r);
        } else {
            int64_t nomega = r_prev < 0 ? l0 : p;
            const double *Qprop = NULL;
            if (r_prev > 0) {
                Qprop = Qt;
                if (r_prev + nomega > n) nomega = n - r_prev;
            }
            if (nomega < 1 && !Qprop) nomega = 1;
            if (nomega < 0) nomega = 0;
            double *Om = dalloc(n * (nomega > 0 ? nomega : 1));
            if (nomega > 0) orc_gaussian_matrix(seed, (uint64_t)it, n, nomega, Om, n);
            orc_frsvt(n, n, T, n, 1.0 / mu, q, Om, n, nomega, Qprop, n, Qprop ? r_prev : 0, J, n,
                      Qnew, n, &r, NULL, NULL);
            free(Om);
            mat_copy(n, r, Qnew, n, Qt, n);
            r_prev = r;
        }
        if (ranks) ranks[it] = r;
        /* Z = (I + X^T X)^{-1} (X^T (X - E + Y1/mu) + J - Y2/mu) */
        for (int64_t i = 0; i < d * n; ++i) W[i] = 0.0;
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < d; ++i)
                AT(W, d, i, j) = AT(X, ldx, i, j) - AT(Ek, d, i, j) + AT(Y1, d, i, j) / mu;
        mat_mul_tn(n, n, d, X, ldx, W, d, R, n);
        for (int64_t i = 0; i < n * n; ++i) R[i] += J[i] - Y2[i] / mu;
        chol_solve(n, Lc, n, n, R, n);
        memcpy(Zk, R, (size_t)(n * n) * sizeof(double));
        /* E = column shrink_{lambda/mu}(X - X Z + Y1/mu) */
        mat_mul(d, n, n, X, ldx, Zk, n, XZ, d);
        const double thr = lambda / mu;
        for (int64_t j = 0; j < n; ++j) {
            double nrm = 0.0;
            for (int64_t i = 0; i < d; ++i) {
                const double v = AT(X, ldx, i, j) - AT(XZ, d, i, j) + AT(Y1, d, i, j) / mu;
                AT(W, d, i, j) = v;
                nrm += v * v;
            }
            nrm = sqrt(nrm);
            const double f = nrm > thr ? (nrm - thr) / nrm : 0.0;
            for (int64_t i = 0; i < d; ++i) AT(Ek, d, i, j) = f * AT(W, d, i, j);
        }
        /* multipliers, penalty, stopping test */
        double r1 = 0.0, r2 = 0.0;
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < d; ++i) {
                const double z = AT(X, ldx, i, j) - AT(XZ, d, i, j) - AT(Ek, d, i, j);
                AT(Y1, d, i, j) += mu * z;
                if (fabs(z) > r1) r1 = fabs(z);
            }
        for (int64_t i = 0; i < n * n; ++i) {
            const double z = Zk[i] - J[i];
            Y2[i] += mu * z;
            if (fabs(z) > r2) r2 = fabs(z);
        }
        mu = rho * mu < mu_max ? rho * mu : mu_max;
        if (r1 < tol && r2 < tol) {
            status = 0;
            ++it;
            break;
        }
    }
    if (iters) *iters = it;
    mat_copy(n, n, Zk, n, Z, ldz);
    mat_copy(d, n, Ek, d, E, lde);
    free(Lc); free(Zk); free(J); free(Ek); free(Y1); free(Y2); free(XZ); free(T); free(W);
    free(R); free(Qt); free(Qnew);
    return status;
}

/* Threads the oracle's loops use: 1 in the plain build; in the OpenMP build
 * (-fopenmp, for the all-core CPU baseline) the OpenMP thread count.  The
 * parallel loops split independent output columns (or reflector target
 * columns), so both builds compute every value in the same order. */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
