/*
 * frsvt.h -- C ABI of the MI355X (gfx950) library for fast randomized
 * singular value thresholding (FRSVT) and its hosts.
 *
 * Method: T.-H. Oh, Y. Matsushita, Y.-W. Tai, I.S. Kweon, "Fast Randomized
 * Singular Value Thresholding for Low-rank Optimization", arXiv:1509.00296.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are DEVICE pointers, column-major, with a leading dimension
 *   (element (i,j) of an m x n matrix M with leading dimension ld is at
 *   M[i + j*ld], ld >= max(1, m)).  A row-major tensor is passed as the
 *   column-major view of its transpose.
 * - The element type of every matrix argument is fixed by `prec`:
 *     FRSVT_F64        double everywhere;
 *     FRSVT_F32        float storage and float GEMMs, FP64 Gram/Cholesky and
 *                      small SVD;
 *     FRSVT_MIXED_BF16 float storage; the sketch and power-iteration products
 *                      run on a bfloat16 copy of A with float accumulation,
 *                      the projection and the reconstruction in float, the
 *                      Gram/Cholesky steps and the small SVD in double.
 * - Orientation (Sec. 2.5 of the paper): the method works on Ahat = A when
 *   m <= n and on Ahat = A^T when m > n, with mhat = min(m,n) rows and
 *   nhat = max(m,n) columns, so that the power iteration acts on the short
 *   side.  The sketch Omega is nhat x l; the propagated basis Q~ is mhat x r.
 * - Ownership: the caller owns every input and output buffer.  The library
 *   owns its workspace, held in the handle, grown on demand and freed by
 *   frsvt_destroy; lrr_ialm and tensor_rpca also allocate their iteration
 *   state for the duration of the call.  All work is enqueued on the handle's HIP stream in order;
 *   an entry point blocks the host only when it writes a HOST output pointer
 *   (ranks, statistics), which it documents.
 * - Status codes (LAPACK-like `info`): 0 success; -i the i-th argument is
 *   invalid (nothing is launched); FRSVT_NOT_CONVERGED (+1) a Jacobi sweep
 *   limit was reached (the result is still written); FRSVT_MAX_ITER (+2) an
 *   iterative host (rpca_ialm, lrr_ialm, tensor_rpca) stopped at max_iter; FRSVT_ERR_* below for runtime failures:
 *   -100 a HIP runtime error, -101 out of device memory, -102 non-finite
 *   input, -103 the final Cholesky factor of a re-orthonormalisation still
 *   failed after the shifted fallback and the refill of null columns
 *   (reported where the call reads its status words: frsvt/svt with a rank
 *   output, and every rpca_ialm iteration), -104 unsupported device or size,
 *   -105 invalid handle, -106 problem too large for frsvt_noalloc's scratch.
 *   No C++ exception crosses this interface.
 */
#ifndef FRSVT_H
#define FRSVT_H

#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define FRSVT_API __attribute__((visibility("default")))
#else
#define FRSVT_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct frsvt_context *frsvt_handle;

typedef enum {
    FRSVT_F64 = 0,
    FRSVT_F32 = 1,
    FRSVT_MIXED_BF16 = 2
} frsvt_precision;

#define FRSVT_OK 0
#define FRSVT_NOT_CONVERGED 1
#define FRSVT_MAX_ITER 2
#define FRSVT_ERR_HIP (-100)
#define FRSVT_ERR_OOM (-101)
#define FRSVT_ERR_NONFINITE (-102)
#define FRSVT_ERR_CHOLESKY (-103)
#define FRSVT_ERR_UNSUPPORTED (-104)
#define FRSVT_ERR_HANDLE (-105)
#define FRSVT_ERR_SCRATCH (-106)

/* Size of the fixed device scratch behind frsvt_noalloc (64 MiB per GPU). */
#define FRSVT_NOALLOC_SCRATCH_BYTES (64u << 20)

/* ------------------------------------------------------------------ handle */

/* Create a handle bound to HIP device `device` and the HIP stream
 * `hip_stream` (a hipStream_t; NULL selects the null stream).  The device
 * must be a gfx950 GPU; returns FRSVT_ERR_UNSUPPORTED otherwise. */
FRSVT_API int frsvt_create(frsvt_handle *handle, int device, void *hip_stream);

/* Release the workspace and the handle.  Waits for the handle's stream. */
FRSVT_API int frsvt_destroy(frsvt_handle handle);

/* Handle options (off by default):
 *   FRSVT_OPT_QRCP_TRUNCATE  value 1: a fresh sketch (frsvt / frsvt_noalloc
 *     without Q_prev) is truncated to its numerical rank before the power
 *     iterations, as Alg. 1's QR_CP step and Sec. 2.1's s = min(l, r) do:
 *     Householder QR with column pivoting of Y = Ahat Omega keeps the s
 *     leading pivoted samples with |R_jj| > mhat * 2^-52 * |R_11|.  The
 *     thresholded result does not depend on it (the dropped samples add no
 *     direction of Ahat's range); the small factors shrink to s.  One host
 *     wait per call; on the one-workgroup path (FP64/FP32, l <= 64 and
 *     mhat l within its local memory) only, elsewhere l samples are kept.
 *     frsvt_last_info word 3 reports s (l when nothing was dropped).
 * Returns -2 for an unknown option, -3 for an invalid value. */
#define FRSVT_OPT_QRCP_TRUNCATE 1
FRSVT_API int frsvt_set_option(frsvt_handle handle, int option, int value);

/* Rebind the handle to another stream of the same device. */
FRSVT_API int frsvt_set_stream(frsvt_handle handle, void *hip_stream);

/* Human-readable text of a status code (static storage). */
FRSVT_API const char *frsvt_status_string(int status);

/* Text of the last runtime error seen by this handle (static per handle). */
FRSVT_API const char *frsvt_last_error(frsvt_handle handle);

/* Device bytes currently held by the handle's workspace. */
FRSVT_API int64_t frsvt_workspace_bytes(frsvt_handle handle);

/* ------------------------------------------------------------------ tracing */

/* Kernel classes timed by the tracer. */
typedef enum {
    FRSVT_K_SKETCH = 0,   /* Y = Ahat Omega (Omega drawn in registers) */
    FRSVT_K_POWER = 1,    /* fused power step Y = Ahat (Ahat^T Q) */
    FRSVT_K_PROJECT = 2,  /* B^T = Ahat^T Q and the Gram B B^T */
    FRSVT_K_REDUCE = 3,   /* split-K reductions */
    FRSVT_K_ORTH = 4,     /* CholeskyQR re-orthonormalisation */
    FRSVT_K_SMALL_SVD = 5,/* Cholesky + one-sided Jacobi SVD of the small factor */
    FRSVT_K_RECON = 6,    /* shrink-and-reconstruct X = (Q Mm) B */
    FRSVT_K_EPILOGUE = 7, /* RPCA epilogue (L on the fly, S, multiplier, next A) */
    FRSVT_K_GEMM = 8,     /* generic tiled GEMM (large shapes, exact SVT) */
    FRSVT_K_OTHER = 9,
    FRSVT_K_GEMM_BF16 = 10, /* bfloat16 matrix-core sketch / power products */
    FRSVT_K_WSVT_BATCHED = 11, /* persistent batched weighted SVT */
    FRSVT_K_ADJOINT = 12, /* adjoint (vector-Jacobian product) kernels */
    FRSVT_K_COUNT = 13
} frsvt_kernel_class;

/* Start (enable != 0, clearing earlier records) or stop recording a pair of
 * HIP events around every kernel launch of this handle, on the handle's
 * stream.  Off by default. */
FRSVT_API int frsvt_trace_enable(frsvt_handle handle, int enable);

/* Waits for the recorded events and returns, for one kernel class, the total
 * GPU time in milliseconds and the number of launches recorded since
 * tracing was enabled. */
FRSVT_API int frsvt_trace_read(frsvt_handle handle, int kernel_class, double *total_ms,
                               int64_t *launches);

/* Name of a kernel class (static storage). */
FRSVT_API const char *frsvt_trace_name(int kernel_class);

/* Status words of the last thresholding step, copied to the host (waits for
 * the stream): info[0] rank r, info[1] Jacobi sweeps of the small SVD,
 * info[2] 1 when that Jacobi met its stopping test, info[3] the sketch width
 * s used by the last frsvt call (after the optional QR_CP truncation),
 * info[4] 1 when the last
 * re-orthonormalisation took the CholeskyQR2 fast path (2 = shifted
 * fallback), info[5] columns refilled, info[6] final Cholesky failures,
 * info[7] 1 when frsvt_vjp met a singular triangular factor.
 * `count` words (at most 8) are written. */
FRSVT_API int frsvt_last_info(frsvt_handle handle, int32_t *info, int count);

/* ---------------------------------------------------------- exact operator */

/*
 * svt: exact singular value thresholding, Def. 1 / Eq. (3) of the paper,
 *   X = U S_tau(Sigma) V^T,  S_tau(x) = sgn(x) max(|x| - tau, 0),
 * the minimiser of Problem (2): tau ||X||_* + 1/2 ||X - A||_F^2.
 *   A     [in]  m x n, leading dimension lda >= m.
 *   tau   [in]  threshold, tau >= 0.
 *   X     [out] m x n, leading dimension ldx >= m; must not alias A.
 *   rank  [out, HOST, optional] #{sigma_i > tau}; when non-NULL the call
 *         waits for the stream.
 * The full singular value decomposition is taken of the mhat x mhat Gram
 * matrix Ahat Ahat^T through its Cholesky factor and a one-sided Jacobi SVD.
 */
FRSVT_API int svt(frsvt_handle handle, frsvt_precision prec, int64_t m, int64_t n, const void *A,
        int64_t lda, double tau, void *X, int64_t ldx, int32_t *rank);

/* --------------------------------------------------------------- FRSVT */

/*
 * frsvt: fast randomized SVT, Alg. 1 of the paper.
 *   A, lda, tau  as for svt (tau >= 0; tau = 0 returns the projection P_Q A).
 *   k, p         target rank and oversampling (Table 1); l = k + p > 0.
 *   q            number of power iterations (eta in the paper), q >= 0.
 *   Q_prev       [in, optional] range propagation (Alg. 1, Sec. 2.1):
 *                mhat x r_prev orthonormal columns, leading dimension
 *                ldq_prev >= mhat.  When given, only p new Gaussian samples
 *                are drawn and l = r_prev + p; k is ignored.  NULL (or
 *                r_prev = 0) selects the fresh sketch.
 *   seed, counter  key and call counter of the Philox4x32-10 stream from
 *                which Omega(k, 2j+e) is drawn (e-th Box-Muller output of
 *                counter {k, j, counter lo, counter hi}); the same
 *                (seed, counter) always gives the same Omega.
 *   X            [out] m x n, ldx >= m; must not alias A or Q_prev.
 *   Q_out        [out, optional] Q~ = (Q V)_{:,1:r} of Alg. 1's output, mhat x r,
 *                leading dimension ldq_out >= mhat, capacity l columns; may
 *                alias Q_prev (it is written after Q_prev is consumed).
 *   r_out        [out, HOST, optional] r = #{sigma_i > tau}; non-NULL makes
 *                the call wait for the stream.
 * l is clamped to mhat; at l = mhat the result equals exact SVT.  A width
 * min(l, mhat) above 256 returns FRSVT_ERR_UNSUPPORTED (the
 * orthonormalisation's factor is formed for at most 256 columns).
 */
FRSVT_API int frsvt(frsvt_handle handle, frsvt_precision prec, int64_t m, int64_t n, const void *A,
          int64_t lda, double tau, int32_t k, int32_t p, int32_t q, const void *Q_prev,
          int32_t r_prev, int64_t ldq_prev, uint64_t seed, uint64_t counter, void *X,
          int64_t ldx, void *Q_out, int64_t ldq_out, int32_t *r_out);

/*
 * frsvt_noalloc: frsvt without any allocation, for callers that cannot
 * allocate device memory during the call (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Arguments,
 * results and status codes are those of frsvt, computed by the same kernels
 * in the same order (results equal frsvt's bit for bit).
 * Differences:
 *   - the workspace is a fixed device array of FRSVT_NOALLOC_SCRATCH_BYTES
 *     that each GPU holds until the process ends, not the handle's
 *     growable workspace; the call allocates and frees nothing;
 *   - a problem whose workspace exceeds it returns FRSVT_ERR_SCRATCH before
 *     anything is launched (frsvt_last_error states the bytes needed; the
 *     sketch's split-K partials dominate: about 4096 * mhat * l bytes in
 *     FP64, e.g. 18.4 MB for mhat = 300, l = 15);
 *   - every call on one GPU shares that GPU's array, which keeps the last
 *     call's contents: calls that overlap on one GPU (two streams or two
 *     host threads) race and must be serialised by the caller.  No part of
 *     the scratch needs to start at zero (every buffer carved from it is
 *     written before it is read).
 * The handle must come from frsvt_create, which looks up the array's device
 * address on its device; r_out (HOST) waits for the stream as in frsvt.
 */
FRSVT_API int frsvt_noalloc(frsvt_handle handle, frsvt_precision prec, int64_t m, int64_t n,
                            const void *A, int64_t lda, double tau, int32_t k, int32_t p, int32_t q,
                            const void *Q_prev, int32_t r_prev, int64_t ldq_prev, uint64_t seed,
                            uint64_t counter, void *X, int64_t ldx, void *Q_out, int64_t ldq_out,
                            int32_t *r_out);

/* ------------------------------------------------------------ adjoint */

/*
 * frsvt_fwd: the fresh-sketch FRSVT of Alg. 1 (no range
 * propagation) that also saves what its adjoint needs, without waiting:
 *   A, lda, tau, k, p, q, seed, counter, X, ldx  as for frsvt (l = min(k+p, mhat),
 *                l <= 64).
 *   Q        [out] the basis of the projection step (the Q of B = Q^T Ahat), mhat x l,
 *            leading dimension ldq >= mhat.
 *   factors  [out] DEVICE, l + l*l doubles: the singular values of B
 *            (descending), then its left singular vectors U_B (l x l,
 *            column-major; columns of zero singular values are zero).
 * FRSVT_F64 and FRSVT_F32 only.
 */
FRSVT_API int frsvt_fwd(frsvt_handle handle, frsvt_precision prec, int64_t m, int64_t n,
                        const void *A, int64_t lda, double tau, int32_t k, int32_t p, int32_t q,
                        uint64_t seed, uint64_t counter, void *X, int64_t ldx, void *Q,
                        int64_t ldq, double *factors);

/*
 * frsvt_vjp: vector-Jacobian product of the frsvt_fwd map A -> X for its
 * fixed Omega (the paper does not differentiate the method; this is the
 * derivative of X = Q S_tau(Q^T Ahat), Prop. 1, through the power
 * iterations and the QR steps).  Given the upstream gradient X_bar it
 * writes A_bar = (dX/dA)^T X_bar and tau_bar = <X_bar, dX/dtau>.
 *   A, tau, k, p, q, seed, counter  exactly as passed to frsvt_fwd.
 *   Q, ldq, factors  [in] saved by that frsvt_fwd call.
 *   X_bar    [in]  m x n, ldxb >= m.
 *   A_bar    [out] m x n, ldab >= m; must not alias A or X_bar.
 *   tau_bar  [out, DEVICE, optional] one double.
 * The sketch Y_0 = Ahat Omega and the power iterations are recomputed from
 * (seed, counter) and A; nothing of them is stored.  The small-SVT part is
 * the spectral-function derivative with bounded divided differences; a pair
 * of singular values straddling tau closer than 1e-12 of the larger uses the
 * value 1/2.  The QR steps assume full column rank: frsvt_last_info word 7
 * is set when a triangular factor had a non-positive diagonal entry.  No
 * host wait.  FRSVT_F64 and FRSVT_F32 only; l <= 64.
 */
FRSVT_API int frsvt_vjp(frsvt_handle handle, frsvt_precision prec, int64_t m, int64_t n,
                        const void *A, int64_t lda, double tau, int32_t k, int32_t p, int32_t q,
                        uint64_t seed, uint64_t counter, const void *Q, int64_t ldq,
                        const double *factors, const void *X_bar, int64_t ldxb, void *A_bar,
                        int64_t ldab, double *tau_bar);

/*
 * rpca_dual_step: the updates of one inexact-ALM iteration that follow the
 * thresholding (Sec. 4.1's RPCA host), with the shrink threshold given
 * directly so that it can be learned per unrolled step:
 *   V = O - L + Y/mu,  S = shrink(V, lam),  Y_next = Y + mu (O - L - S),
 *   A_next = O - S + Y_next / mu_next   (the next thresholding input).
 * O, L, Y [in] m x n.  S, Y_next, A_next [out, each optional].  lam >= 0,
 * mu, mu_next > 0.  No host wait.
 */
FRSVT_API int rpca_dual_step(frsvt_handle handle, frsvt_precision prec, int64_t m, int64_t n,
                             const void *O, int64_t ldo, const void *L, int64_t ldl, const void *Y,
                             int64_t ldy, double lam, double mu, double mu_next, void *S,
                             int64_t lds, void *Y_next, int64_t ldyn, void *A_next, int64_t ldan);

/*
 * rpca_dual_step_vjp: reverse of rpca_dual_step.  Upstream gradients
 * S_bar, Y_next_bar, A_next_bar (each optional, NULL = zero) give
 *   L_bar, Y_bar [out] m x n, and lam_bar [out, DEVICE, optional] one
 * double (sum over the entries, fixed reduction order).  No host wait.
 */
FRSVT_API int rpca_dual_step_vjp(frsvt_handle handle, frsvt_precision prec, int64_t m, int64_t n,
                                 const void *O, int64_t ldo, const void *L, int64_t ldl,
                                 const void *Y, int64_t ldy, double lam, double mu, double mu_next,
                                 const void *S_bar, int64_t ldsb, const void *Y_next_bar,
                                 int64_t ldynb, const void *A_next_bar, int64_t ldanb, void *L_bar,
                                 int64_t ldlb, void *Y_bar, int64_t ldyb, double *lam_bar);

/*
 * rpca_init: starting point of the inexact-ALM loop, S_0 = 0,
 *   Y0 = O / J,  J = max(||O||_2, ||O||_inf / lambda),  A0 = O + Y0 / mu0,
 * with mu0 = 1.25 / ||O||_2 when the given mu0 <= 0.
 *   out [out, HOST, optional] 3 doubles: ||O||_2, mu0, J.  Waits for the
 *   stream.  FRSVT_ERR_NONFINITE when O holds NaN or Inf.
 */
FRSVT_API int rpca_init(frsvt_handle handle, frsvt_precision prec, int64_t m, int64_t n,
                        const void *O, int64_t ldo, double lambda, double mu0, void *Y0,
                        int64_t ldy, void *A0, int64_t lda0, double *out);

/*
 * Unrolled inexact-ALM RPCA over a batch (the differentiation form): T steps
 * of Sec. 4.1's iALM with a learnable SVT threshold tau_t and shrink
 * threshold lam_t per step (they replace 1/mu_t and lambda/mu_t):
 *   (Y_0, A_0) = rpca_init(O_b),  mu_t = min(mu_0 rho^t, mu_bar_factor mu_0),
 *   mu_0 = 1.25 / ||O_b||_2,
 *   L_{t+1} = frsvt_fwd(A_t, tau_t, k, p, q, seed + b, counter t),
 *   (Y_{t+1}, A_{t+1}) = rpca_dual_step(O_b, L_{t+1}, Y_t, lam_t, mu_t, mu_{t+1}),
 * output L_T of every instance.  Instance b of a batched argument X is the
 * column-major matrix at X + b * strideX (elements) with its leading
 * dimension.  taus, lams are DEVICE arrays of `steps` doubles (read once,
 * waiting for the stream).  Instances run concurrently on side streams of
 * the handle that start after the work already enqueued on its stream; the
 * handle's stream waits for them before the call returns (the forward
 * waits for the host once per instance, for ||O_b||_2).
 *
 * rpca_unrolled_saved_bytes: bytes of the state the forward keeps for the
 * reverse sweep (per instance: mu_t, every A_t and Y_t, L_t for t < T - 1,
 * the bases Q_t and the small factors); -1 for invalid sizes.
 */
FRSVT_API int64_t rpca_unrolled_saved_bytes(frsvt_precision prec, int32_t batch, int32_t steps, int64_t m,
                                            int64_t n, int32_t k, int32_t p);

/* rpca_unrolled_schedule: the plain iALM schedule of one instance O,
 * tau_t = 1/mu_t and lam_t = lambda/mu_t for t < steps (mu_t as above), into
 * HOST arrays; the starting values of the learnable thresholds.  Waits. */
FRSVT_API int rpca_unrolled_schedule(frsvt_handle handle, frsvt_precision prec, int64_t m, int64_t n,
                                     const void *O, int64_t ldo, double lambda, double rho,
                                     double mu_bar_factor, int32_t steps, double *taus, double *lams);

/* rpca_unrolled_fwd: the forward pass.  L [out] batch of m x n results
 * (ldl, strideL); saved [out] caller-owned DEVICE buffer of at least
 * rpca_unrolled_saved_bytes bytes, passed unchanged to rpca_unrolled_bwd.
 * FRSVT_F64 and FRSVT_F32; l = min(k + p, mhat) <= 64. */
FRSVT_API int rpca_unrolled_fwd(frsvt_handle handle, frsvt_precision prec, int32_t batch, int32_t steps,
                                int64_t m, int64_t n, const void *O, int64_t ldo, int64_t strideO,
                                const double *taus, const double *lams, double lambda, double rho,
                                double mu_bar_factor, int32_t k, int32_t p, int32_t q, uint64_t seed,
                                void *L, int64_t ldl, int64_t strideL, void *saved, int64_t saved_bytes);

/* rpca_unrolled_bwd: the reverse sweep of the forward call with the same
 * arguments and `saved`: given the upstream gradient L_bar of the outputs
 * it writes tau_bar and lam_bar [out, DEVICE, `steps` doubles each], the
 * gradients of sum_b <L_bar_b, L_T(b)> in tau_t and lam_t, summed over the
 * batch in a fixed order (lam_bar[T-1] = 0: lam_{T-1} does not reach L_T).
 * Reverse of each step: rpca_dual_step_vjp, then frsvt_vjp. */
FRSVT_API int rpca_unrolled_bwd(frsvt_handle handle, frsvt_precision prec, int32_t batch, int32_t steps,
                                int64_t m, int64_t n, const void *O, int64_t ldo, int64_t strideO,
                                const double *taus, const double *lams, int32_t k, int32_t p, int32_t q,
                                uint64_t seed, const void *saved, int64_t saved_bytes, const void *L_bar,
                                int64_t ldlb, int64_t strideLb, double *tau_bar, double *lam_bar);

/* --------------------------------------------------------------- WSVT */

/*
 * wsvt: weighted SVT (the WSVT of weighted nuclear norm minimisation, named
 * in Sec. 1 and footnote 1 of the paper):
 *   X = U diag(max(sigma_i - w_i, 0)) V^T,
 * with w indexed by DESCENDING sigma.  It minimises
 * sum_i w_i sigma_i(X) + 1/2 ||X - A||_F^2 when w is non-descending; other
 * weights are applied as given.
 *   w     [in] DEVICE array of min(m,n) doubles.
 *   rank  [out, HOST, optional] #{sigma_i > w_i}.
 */
FRSVT_API int wsvt(frsvt_handle handle, frsvt_precision prec, int64_t m, int64_t n, const void *A,
         int64_t lda, const double *w, void *X, int64_t ldx, int32_t *rank);

/* Weight rule of a batched WSVT call.  With c > 0 the weights follow the
 * patch-group denoising rule w_i = c sqrt(cols) / (sigma_hat_i + eps),
 * sigma_hat_i = sqrt(max(sigma_i^2 - cols * noise_var, 0)).  With c <= 0 the
 * thresholds are the constant `tau` for every singular value (plain SVT). */
typedef struct {
    double c;
    double noise_var;
    double eps;
    double tau;
} frsvt_wsvt_rule;

/*
 * wsvt_batched: weighted SVT of `count` independent small matrices of
 * uneven shapes in one persistent launch.
 *   rows, cols   [in] DEVICE int32 arrays (count); 1 <= rows, cols <= 128,
 *                min(rows, cols) <= 96.
 *   offsets      [in] DEVICE int64 array (count): element offset of matrix
 *                j inside A_packed / X_packed; each matrix is column-major
 *                with leading dimension rows[j].
 *   A_packed     [in]  float, DEVICE.
 *   X_packed     [out] float, DEVICE; must not alias A_packed.
 *   ranks        [out, DEVICE, optional] int32 per matrix, #{sigma > w}.
 * The small SVD runs in double precision in the local data share.  The
 * first call with a given argument set reads the shapes to the host (it
 * waits for the stream), orders the matrices longest first, runs the
 * autotuner once per handle (group size of the Jacobi pair work per size
 * bucket, timed on the device) and captures the persistent launch in a HIP
 * graph; later calls with the same arguments (pointers, count and rule)
 * replay that graph.  The replay reads rows/cols anew: shapes rewritten in
 * place keep the first call's processing order and tuning, and a shape
 * outside the bounds above is skipped by the kernel (its rank set to -1)
 * and reported as FRSVT_ERR_UNSUPPORTED.  Every call waits for the stream
 * once, to read that check.
 */
FRSVT_API int wsvt_batched(frsvt_handle handle, int64_t count, const int32_t *rows,
                 const int32_t *cols, const int64_t *offsets, const float *A_packed,
                 float *X_packed, const frsvt_wsvt_rule *rule, int32_t *ranks);

/* Group sizes (lanes per Jacobi pair) chosen by the autotuner for the size
 * buckets min(rows, cols) <= 48, <= 64, <= 96; zeros before the first
 * batched call. */
FRSVT_API int frsvt_wsvt_tuning(frsvt_handle handle, int32_t group_size[3]);

/* The one-sided Jacobi work of the last wsvt_batched call on this handle
 * (waits for the handle's stream): work[0] = sum over examined pairs of the
 * column length, work[1] = the same sum over applied rotations, work[2] =
 * the number of applied rotations.  Each examined pair costs 6 column
 * lengths of floating-point operations (three inner products), each
 * rotation 6 more (the update) plus its angle.  Zeros before the first
 * batched call. */
FRSVT_API int frsvt_wsvt_work(frsvt_handle handle, int64_t work[3]);

/* ---------------------------------------------------------- RPCA host */

typedef struct {
    double tol;            /* stop when ||O - L - S||_F / ||O||_F < tol (1e-7) */
    int32_t max_iter;      /* iteration limit (60) */
    double mu0;            /* initial penalty; <= 0 selects 1.25 / ||O||_2 */
    double rho;            /* penalty growth (1.5) */
    double mu_bar_factor;  /* mu never exceeds mu0 * mu_bar_factor (1e7) */
    int32_t use_frsvt;     /* 1: FRSVT with range propagation; 0: exact svt */
    int32_t p;             /* oversampling of the propagated sketch (5) */
    int32_t q;             /* power iterations (1) */
    int32_t l0;            /* first sketch width; <= 0 selects ceil(0.1 b) (b = mhat
                              without adaptive prediction) */
    uint64_t seed;         /* Philox key; iteration i uses counter i */
    /* Adaptive rank prediction (Sec. 2.3, Eq. 7), with n of Eq. 7 the short
     * side mhat: after an iteration of sketch width l_i and rank r_i the next
     * width is l_{i+1} = min(r_i + p_{i+1}, b), p_{i+1} = ap_a if r_i < l_i,
     * else ceil(ap_rho mhat); b = ceil(ap_gamma mhat); the r_i propagated
     * columns are part of it (no new sample once r_i = b: the propagated
     * basis alone, power iterations still applied).  p is unused then. */
    int32_t ap;            /* 1: adaptive prediction; 0: p new samples (default) */
    int32_t ap_a;          /* a >= 1 (2) */
    double ap_rho;         /* rho in (0, 1] (0.05) */
    double ap_gamma;       /* gamma in (0, 1] (1.0) */
    /* Partial SVT (the truncated nuclear norm, Type B of Table 6): the
     * largest keep singular values pass unshrunk, the rest by 1/mu (0: SVT). */
    int32_t keep;
    /* Semi-online use over consecutive observations (Sec. 4, Type B): an
     * initial propagated basis for the first FRSVT call (DEVICE, mhat x
     * r_init, leading dimension mhat, orthonormal columns, same precision as
     * O; r_init = 0: a fresh first sketch), and optionally the propagated
     * basis of the last call (DEVICE, mhat x mhat capacity, leading dimension
     * mhat; its column count is stats->ranks of the last iteration). */
    const void *q_init;
    int32_t r_init;
    void *q_final;
    /* Residual check steering the sampling (Sec. 3.2 after Prop. 4): the
     * new samples y_j of an iteration are taken in order and each is
     * projected off the basis it would extend, [Q~, y_1, ..., y_{j-1}]
     * (classical Gram-Schmidt, two passes); sampling stops at the first
     * whose estimate 20 sqrt(2/pi) ||residual|| is at most the iteration's
     * threshold 1/mu (y_j itself is kept); otherwise every sample of the
     * width rule is taken.  1: on, 0: off (default).  FRSVT mode on the
     * one-workgroup path only (short side and widths small enough for it):
     * FRSVT_ERR_UNSUPPORTED otherwise.  Costs one host wait per iteration. */
    int32_t resid_check;
} frsvt_rpca_opts;

typedef struct {
    int32_t iters;         /* iterations run */
    int32_t converged;     /* 1 when the tolerance was met */
    double residual;       /* final ||O - L - S||_F / ||O||_F */
    double norm2;          /* ||O||_2 used for mu0 */
    double seconds;        /* wall time of the iteration loop */
    int32_t ranks[64];     /* r_i of the first 64 iterations */
    double residuals[64];  /* residual of the first 64 iterations */
    int32_t widths[64];    /* sketch width l_i of the first 64 iterations (FRSVT) */
    /* Prop. 4 (with Lemma 3, alpha = 20): 20 sqrt(2/pi) ||(I - Q~ Q~^T) y||_2
     * for the first new sample y = Ahat omega of iteration i, Q~ the
     * propagated basis (none for a fresh sketch) -- an upper bound on
     * sigma_{r+1} of that iteration's Ahat with probability >= 0.95, computed
     * from the orthonormalisation's by-products; -1 when no sample was drawn
     * (FRSVT) */
    double resid_est[64];
} frsvt_rpca_stats;

/* Fill `opts` with the defaults listed above. */
FRSVT_API void frsvt_rpca_default_opts(frsvt_rpca_opts *opts);

/*
 * rpca_ialm: robust PCA, min ||L||_* + lambda ||S||_1 s.t. O = L + S, by the
 * inexact augmented Lagrange multiplier method used in Sec. 4.1 of the paper
 * (lambda = 1/sqrt(max(m,n)) there).  Each iteration:
 *   L = SVT_{1/mu}(O - S + Y/mu)  (FRSVT + range propagation, or exact svt),
 *   S = shrink_{lambda/mu}(O - L + Y/mu),  Y += mu (O - L - S),
 *   mu = min(rho mu, mu_bar),
 * starting from S = 0, Y = O / max(||O||_2, ||O||_inf / lambda).
 *   O      [in]  m x n, ldo >= m.
 *   L, S   [out] m x n, leading dimensions ldl, lds >= m.
 *   opts   [in, optional] NULL selects frsvt_rpca_default_opts.
 *   stats  [out, HOST, optional].
 * The host reads one 16-byte status word per iteration (rank and residual)
 * to size the next sketch and test convergence; the call returns after the
 * last iteration has finished.  Returns FRSVT_MAX_ITER when max_iter was
 * reached before tol.
 * Sizes: min(m, n) <= 1024 with exact SVT; <= 8192 with FRSVT, whose sketch
 * widths are capped at 256 (fewer new samples beside a wider propagated
 * basis).  Beyond a short side of 1024, ||O||_2 for the
 * starting point is the top Ritz value of 40 steps of 16-vector block
 * power iteration on O O^T (relative error below (s_17 / s_1)^160).
 */
FRSVT_API int rpca_ialm(frsvt_handle handle, frsvt_precision prec, int64_t m, int64_t n, const void *O,
              int64_t ldo, double lambda, const frsvt_rpca_opts *opts, void *L, int64_t ldl,
              void *S, int64_t lds, frsvt_rpca_stats *stats);

/*
 * rpca_sliding: semi-online low-rank + sparse decomposition of a frame
 * sequence (Type B of Table 6, Sec. 4).  The columns of F (m x frames,
 * ldf) are split into consecutive windows of `window` frames; window w is
 * decomposed by rpca_ialm with FRSVT and partial SVT (the keep largest
 * singular values unshrunk), q power iterations, sketch widths by adaptive
 * prediction bounded by l (ap_a = l - keep, ap_gamma = l / window), seed +
 * w, and the previous window's last propagated basis as its initial basis
 * (q_init / r_init; none for the first window).  Frames past the last whole
 * window are left untouched in L and S.
 *   lambda   > 0, commonly 1/sqrt(max(m, window)).  1 <= keep < l <= window, l <= m.
 *   L, S     [out] m x frames (ldl, lds >= m).
 *   stats    [out, HOST, optional] frames / window entries, one per window.
 *   bases    [out, DEVICE, optional] frames / window blocks of mhat x l
 *            (mhat = min(m, window)): window w's last propagated basis at
 *            bases + w * mhat * l, leading dimension mhat, its width the
 *            last rank in stats[w] (the rest of the block is not written).
 * Returns FRSVT_OK when every window ran (a window stopped at max_iter
 * still counts; its stats say so); max_iter <= 64.  Waits for the stream.
 */
FRSVT_API int rpca_sliding(frsvt_handle handle, frsvt_precision prec, int64_t m, int64_t frames,
                           const void *F, int64_t ldf, int32_t window, double lambda, int32_t keep,
                           int32_t l, int32_t q, uint64_t seed, double tol, int32_t max_iter, double rho,
                           void *L, int64_t ldl, void *S, int64_t lds, frsvt_rpca_stats *stats,
                           void *bases);

/* ---------------------------------------------------------- LRR host */

typedef struct {
    double tol;            /* stop when max|X - XZ - E| and max|Z - J| fall below tol (1e-8) */
    int32_t max_iter;      /* iteration limit (1000) */
    double mu0;            /* initial penalty (1e-6) */
    double rho;            /* penalty growth (1.1) */
    double mu_max;         /* penalty cap (1e10) */
    int32_t use_frsvt;     /* 1: FRSVT with range propagation for the J step; 0: exact svt */
    int32_t p;             /* new samples beside the propagated basis (5) */
    int32_t q;             /* power iterations (1) */
    uint64_t seed;         /* Philox key; iteration i uses counter i */
} frsvt_lrr_opts;

typedef struct {
    int32_t iters;         /* iterations run */
    int32_t converged;     /* 1 when the tolerance was met */
    int32_t rank;          /* rank of J in the last iteration */
    double primal;         /* final max|X - XZ - E| */
    double dual;           /* final max|Z - J| */
    double seconds;        /* wall time of the iteration loop */
} frsvt_lrr_stats;

/* Fill `opts` with the defaults listed above. */
FRSVT_API void frsvt_lrr_default_opts(frsvt_lrr_opts *opts);

/*
 * lrr_ialm: low-rank representation (Type A of Table 6, the host of Sec. 4's
 * subspace-clustering experiments), min ||Z||_* + lambda ||E||_{2,1}
 * s.t. X = X Z + E, by the inexact ALM of the LRR method with the auxiliary
 * J = Z.  From Z = J = E = 0, Y1 = Y2 = 0, mu = mu0, each iteration
 *   J = SVT_{1/mu}(Z + Y2/mu)  (FRSVT + range propagation: first sketch
 *       ceil(0.1 n) wide, then r + p; or exact svt),
 *   Z = (I + X^T X)^{-1} (X^T (X - E + Y1/mu) + J - Y2/mu),
 *   E = column-wise shrink_{lambda/mu}(X - X Z + Y1/mu),
 *   Y1 += mu (X - X Z - E), Y2 += mu (Z - J), mu = min(rho mu, mu_max),
 * until both max-norm residuals fall below tol.  (I + X^T X)^{-1} is formed
 * once by Newton-Schulz iterations on the matrix cores.
 *   prec   FRSVT_F64 only (others: FRSVT_ERR_UNSUPPORTED).
 *   X      [in]  d x n, ldx >= d (DEVICE).  n <= 1024.
 *   Z      [out] n x n, ldz >= n;  E [out] d x n, lde >= d (DEVICE).
 *   opts   [in, optional] NULL selects frsvt_lrr_default_opts.
 *   stats  [out, HOST, optional].
 * The call allocates its iteration state (about 4 d n + 9 n^2 doubles) and
 * frees it before returning; the host reads two residuals per iteration.
 * Returns FRSVT_MAX_ITER when max_iter was reached before tol.
 */
FRSVT_API int lrr_ialm(frsvt_handle handle, frsvt_precision prec, int64_t d, int64_t n, const void *X,
                       int64_t ldx, double lambda, const frsvt_lrr_opts *opts, void *Z, int64_t ldz,
                       void *E, int64_t lde, frsvt_lrr_stats *stats);

/* ---------------------------------------------------------- 3-way tensor host */

typedef struct {
    double tol;            /* stop when max_i ||O - L_i - E||_F / ||O||_F < tol (1e-7) */
    int32_t max_iter;      /* iteration limit (100) */
    double mu0;            /* initial penalty; 0 selects 1.25 / ||O_(1)||_2 (0) */
    double rho;            /* penalty growth (1.5) */
    double mu_max;         /* penalty cap (1e10) */
    int32_t use_frsvt;     /* 1: FRSVT with range propagation per mode; 0: exact svt */
    int32_t p;             /* new samples beside the propagated basis (5) */
    int32_t q;             /* power iterations (1) */
    uint64_t seed;         /* Philox key of mode 1; mode i uses seed + i - 1, iteration t counter t */
} frsvt_tensor_opts;

typedef struct {
    int32_t iters;         /* iterations run */
    int32_t converged;     /* 1 when the tolerance was met */
    int32_t rank[3];       /* rank of each mode's SVT in the last iteration */
    double resid;          /* final max_i ||O - L_i - E||_F / ||O||_F */
    double mu0;            /* the initial penalty used */
    double seconds;        /* wall time of the iteration loop */
} frsvt_tensor_stats;

/* Fill `opts` with the defaults listed above. */
FRSVT_API void frsvt_tensor_default_opts(frsvt_tensor_opts *opts);

/*
 * tensor_rpca: low-rank + sparse decomposition of a 3-way tensor, the convex
 * program of Type C in Table 6 with the alignment fixed to the identity:
 * min sum_i alpha_i ||L_(i)||_* + lambda ||E||_1 s.t. O = L + E, where L_(i)
 * is the mode-i unfolding (rows indexed by mode i, columns by the other two
 * modes with the earlier one varying fastest).  Inexact ALM over one copy
 * L_i of L per mode, each with its own constraint O = L_i + E and
 * multiplier Y_i; from E = Y_i = 0, each iteration
 *   L_i = fold_i(SVT_{alpha_i/mu}(unfold_i(O - E + Y_i/mu)))  (FRSVT + range
 *         propagation per mode: first sketch ceil(0.1 mhat_i) wide, then
 *         r_i + p; or exact svt),
 *   E   = shrink_{lambda/(3 mu)}(mean_i(O - L_i + Y_i/mu)),
 *   Y_i += mu (O - L_i - E),  mu = min(rho mu, mu_max).
 *   prec   FRSVT_F64 only (others: FRSVT_ERR_UNSUPPORTED).
 *   O      [in]  I1 x I2 x I3, column-major, contiguous (DEVICE).  Each
 *          unfolding's short side must be <= 1024.
 *   alpha  [in, HOST] three weights >= 0 (Table 6 assumes they sum to 1).
 *   L      [out] the mean of the three copies L_i; E [out]; both
 *          contiguous like O and distinct from O and from each other (DEVICE).
 *   opts   [in, optional] NULL selects frsvt_tensor_default_opts.
 *   stats  [out, HOST, optional].
 * The call allocates its iteration state (8 tensors plus the three modes'
 * bases) and frees it before returning; the host reads three residuals per
 * iteration.  O = 0 returns L = E = 0 with no iteration.  Returns
 * FRSVT_MAX_ITER when max_iter was reached before tol.
 */
FRSVT_API int tensor_rpca(frsvt_handle handle, frsvt_precision prec, int64_t I1, int64_t I2, int64_t I3,
                          const void *O, const double *alpha, double lambda, const frsvt_tensor_opts *opts,
                          void *L, void *E, frsvt_tensor_stats *stats);

#ifdef __cplusplus
}
#endif
#endif /* FRSVT_H */
