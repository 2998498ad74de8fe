/*
 * frsvt_oracle.h -- plain FP64 CPU reference ("oracle") for fast randomized
 * singular value thresholding (FRSVT), arXiv:1509.00296 (Oh, Matsushita, Tai,
 * Kweon).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library.
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no source, header, table or helper with
 * the GPU library, and it never calls it.
 *
 * Conventions: every matrix is column-major double with an explicit leading
 * dimension (element (i,j) of M is M[i + j*ld]).  Sizes are int64_t.  Return
 * value 0 = success, a negative value -i = the i-th argument is invalid, a
 * positive value = an iteration limit was hit (the result is still written).
 */
#ifndef FRSVT_ORACLE_H
#define FRSVT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- Random numbers: counter-based Gaussian test matrix Omega (Alg. 1) ---- */

/* Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* 53-bit uniform in (0,1) from two 32-bit words. */
double orc_uniform53(uint32_t a, uint32_t b);

/* Fill Om (rows x cols) with iid N(0,1): Om(k, 2j+e) is the e-th Box-Muller
 * output of Philox(ctr = {k, j, counter lo, counter hi}, key = seed). */
void orc_gaussian_matrix(uint64_t seed, uint64_t counter, int64_t rows, int64_t cols,
                         double *Om, int64_t ld);

/* ---- Dense factorizations ---- */

/* Thin Householder QR of a tall m x n matrix (m >= n): Q (m x n), R (n x n). */
int orc_qr(int64_t m, int64_t n, const double *A, int64_t lda,
           double *Q, int64_t ldq, double *R, int64_t ldr);

/* Householder QR with column pivoting; writes the first s columns of Q, where
 * s is the numerical rank (|R_jj| > max(m,n) * 2^-52 * |R_00|).  Returns s. */
int64_t orc_qrcp_basis(int64_t m, int64_t n, const double *A, int64_t lda,
                       double *Q, int64_t ldq);

/* Thin SVD by one-sided Jacobi (after a Householder QR): A = U diag(S) V^T
 * with k = min(m,n), U m x k, V n x k, S descending.  Returns the number of
 * Jacobi sweeps, or 1000+sweeps when the sweep limit was hit. */
int orc_svd(int64_t m, int64_t n, const double *A, int64_t lda,
            double *U, int64_t ldu, double *S, double *V, int64_t ldv);

/* ---- Proximal operators ---- */

/* Exact SVT, Def. 1 / Eq. (3): X = U S_tau(Sigma) V^T.  rank = #{sigma > tau}. */
int orc_svt(int64_t m, int64_t n, const double *A, int64_t lda, double tau,
            double *X, int64_t ldx, int64_t *rank);

/* Weighted SVT: X = U diag(max(sigma_i - w_i, 0)) V^T, w indexed by
 * descending sigma (length min(m,n)).  rank = #{sigma_i > w_i}. */
int orc_wsvt(int64_t m, int64_t n, const double *A, int64_t lda, const double *w,
             double *X, int64_t ldx, int64_t *rank);

/* Weighted SVT with the patch-group weight rule of weighted nuclear norm
 * denoising: w_i = c sqrt(n) / (sigma_hat_i + eps), sigma_hat_i =
 * sqrt(max(sigma_i^2 - n noise_var, 0)), n = the number of columns.  With
 * c <= 0 every threshold is tau (plain SVT).  rank = #{sigma_i > w_i}. */
int orc_wsvt_rule(int64_t m, int64_t n, const double *A, int64_t lda, double c,
                  double noise_var, double eps, double tau, double *X, int64_t ldx,
                  int64_t *rank);

/* FRSVT, Alg. 1.  Works on the oriented matrix Ahat = A (m <= n) or A^T
 * (m > n), mhat = min(m,n), nhat = max(m,n).
 *   Qt == NULL : fresh sketch, Omega is nhat x nomega, l = nomega.
 *   Qt != NULL : range propagation, Qt is mhat x r_prev with orthonormal
 *                columns, Omega is nhat x nomega (the p new samples).
 * q power iterations.  Outputs X (m x n), Qout (mhat x r, optional),
 * r_out, sigma (the s singular values of B, optional, length >= l), s_out. */
int orc_frsvt(int64_t m, int64_t n, const double *A, int64_t lda, double tau,
              int q, const double *Om, int64_t ldom, int64_t nomega,
              const double *Qt, int64_t ldqt, int64_t r_prev,
              double *X, int64_t ldx, double *Qout, int64_t ldqo,
              int64_t *r_out, double *sigma, int64_t *s_out);

/* Inexact-ALM RPCA, min ||L||_* + lambda ||S||_1 s.t. O = L + S.
 * svt_mode 0: exact SVT; 1: FRSVT with range propagation (l0 = ceil(0.1 mhat),
 * then l = r_prev + p; q power iterations; Omega of iteration k drawn with
 * counter k).  mu0 <= 0 selects 1.25/||O||_2.  Per-iteration ranks[] and
 * resid[] (length max_iter) are optional. */
int orc_rpca_ialm(int64_t m, int64_t n, const double *O, int64_t ldo, double lambda,
                  int svt_mode, int64_t p, int q, uint64_t seed,
                  double tol, int max_iter, double mu0, double rho, double mu_bar_factor,
                  double *L, int64_t ldl, double *S, int64_t lds,
                  int64_t *ranks, double *resid, int *iters);

/* The same with the sketch widths of adaptive rank prediction (Sec. 2.3,
 * Eq. 7) when ap != 0: after a call of width l_i and rank r_i the next width
 * is l_{i+1} = min(r_i + (r_i < l_i ? a : ceil(rho mhat)), b), b =
 * ceil(gamma mhat), l_0 = ceil(0.1 b); the propagated basis holds r_i of
 * them (no new sample once r_i = b).  p is unused then.  widths[] (length
 * max_iter, optional) receives l_i, resid_est[] the estimate below; returns -15 for a < 1, rho <= 0 or gamma
 * outside (0, 1]. */
/* Sequential residual check of Sec. 3.2 (Prop. 4 with Lemma 3): number of
 * the nomega samples Ahat Om(:, j) kept before (and including) the first
 * whose residual estimate against the basis it extends is <= tau. */
int64_t orc_residual_check(int64_t m, int64_t n, const double *A, int64_t lda, const double *Qt,
                           int64_t ldq, int64_t r, const double *Om, int64_t ldom, int64_t nomega,
                           double tau, double alpha, double *est_out);

/* orc_rpca_ialm_ap with the residual check steering the number of new
 * samples per iteration (resid_check != 0). */
int orc_rpca_ialm_rc(int64_t m, int64_t n, const double *O, int64_t ldo, double lambda,
                     int svt_mode, int64_t p, int q, uint64_t seed, double tol, int max_iter,
                     double mu0, double rho, double mu_bar_factor, int ap, int64_t ap_a,
                     double ap_rho, double ap_gamma, int64_t keep, const double *Qinit,
                     int64_t r_init, double *Qfinal, int64_t *r_final, int resid_check, double *L,
                     int64_t ldl, double *S, int64_t lds, int64_t *ranks, int64_t *widths,
                     double *resid_est, double *resid, int *iters);

int orc_rpca_ialm_ap(int64_t m, int64_t n, const double *O, int64_t ldo, double lambda,
                     int svt_mode, int64_t p, int q, uint64_t seed, double tol, int max_iter,
                     double mu0, double rho, double mu_bar_factor, int ap, int64_t ap_a,
                     double ap_rho, double ap_gamma, int64_t keep, const double *Qinit,
                     int64_t r_init, double *Qfinal, int64_t *r_final, double *L, int64_t ldl,
                     double *S, int64_t lds, int64_t *ranks, int64_t *widths, double *resid_est,
                     double *resid, int *iters);

/* Partial SVT: the keep largest singular values pass unshrunk, the others
 * are soft-thresholded by tau (the truncated nuclear norm's proximal step).
 * orc_frsvt_keep is orc_frsvt with that thresholding; orc_rpca_ialm_ap uses
 * it (and orc_psvt in the exact mode) with its keep argument, starts from
 * the propagated basis Qinit (mhat x r_init, ld mhat) when r_init > 0, and
 * returns the last propagated basis in Qfinal (mhat x *r_final, ld mhat). */
int orc_psvt(int64_t m, int64_t n, const double *A, int64_t lda, double tau, int64_t keep,
             double *X, int64_t ldx, int64_t *rank);
int orc_frsvt_keep(int64_t m, int64_t n, const double *A, int64_t lda, double tau, int64_t keep,
                   int q, const double *Om, int64_t ldom, int64_t nomega, const double *Qt,
                   int64_t ldqt, int64_t r_prev, double *X, int64_t ldx, double *Qout,
                   int64_t ldqo, int64_t *r_out, double *sigma, int64_t *s_out);

/* Prop. 4's residual singular-value estimate alpha sqrt(2/pi)
 * ||(I - Q~ Q~^T) Ahat omega||_2 (Ahat = A if m <= n, else A^T; Q~ mhat x r
 * orthonormal, omega of length nhat), an upper bound on sigma_{r+1}(Ahat)
 * with probability >= 1 - 1/alpha.  In orc_rpca_ialm_ap, resid_est[i] is
 * this estimate (alpha = 20) for the first new sample of iteration i, with
 * the propagated basis as Q~ (none for a fresh sketch), -1 when no sample is
 * drawn. */
double orc_residual_estimate(int64_t m, int64_t n, const double *A, int64_t lda, const double *Qt,
                             int64_t ldq, int64_t r, const double *omega, double alpha);

/* Low-rank representation (Type A of Table 6) by its inexact ALM:
 *   min ||J||_* + lambda ||E||_{2,1} s.t. X = X Z + E, Z = J
 * (X d x n; Z n x n; E d x n).  svt_mode 0: exact SVT for the J step; 1:
 * FRSVT with range propagation (l0 = ceil(0.1 n), then r + p; q power
 * iterations; counter = iteration).  mu0, rho, mu_max: the penalty
 * schedule; stops when max|X - XZ - E| < tol and max|Z - J| < tol.
 * ranks[] (length max_iter) optional.  Returns 0 when converged, 2 when
 * max_iter was reached. */
int orc_lrr_ialm(int64_t d, int64_t n, const double *X, int64_t ldx, double lambda, int svt_mode,
                 int64_t p, int q, uint64_t seed, double tol, int max_iter, double mu0, double rho,
                 double mu_max, double *Z, int64_t ldz, double *E, int64_t lde, int64_t *ranks,
                 int *iters);

/* Vector-Jacobian product of exact SVT from a full SVD: given Xbar,
 * Abar = (dX/dA)^T Xbar and taubar = <Xbar, dX/dtau>. */
int orc_svt_vjp(int64_t m, int64_t n, const double *A, int64_t lda, double tau,
                const double *Xbar, int64_t ldxb, double *Abar, int64_t ldab,
                double *taubar);

/* 1 in the plain build, the OpenMP thread count in the OpenMP build. */
int orc_threads(void);

#ifdef __cplusplus
}
#endif
#endif
