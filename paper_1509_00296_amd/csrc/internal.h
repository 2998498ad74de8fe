// internal.h -- launch interface between the host orchestration (api.hip) and
// the gfx950 kernels (kernels.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace frk {

// ----------------------------------------------------------------- long pass
// One pass over Ahat (mhat x nhat) reducing over the long dimension, with the
// whole short dimension inside one workgroup:
//   kSketch : Ypart += Ahat * Omega(seed, counter)           (Omega in-register)
//   kVecMul : Ypart += Ahat * V                               (V nhat x c)
//   kPower  : z_k = Ahat(:,k)^T Q,  Ypart += Ahat(:,k) z_k^T   (one read of A)
//   kProject: z_k = Ahat(:,k)^T Q -> Bt(k,:),  Gpart += z_k z_k^T
enum LongMode { kSketch = 0, kVecMul = 1, kPower = 2, kProject = 3 };

template <typename T>
struct LongArgs {
    const T *A;
    int64_t lda;
    int trans;       // 1: Ahat = A^T (A is nhat x mhat), 0: Ahat = A
    int mh;
    int64_t nh;
    int c;
    int kt;          // tile width along the long dimension
    int mhp;         // rows padded to whole 16-row blocks
    int ntiles;
    uint64_t seed, counter;
    const T *V;
    int64_t ldv;
    const T *Q;
    int64_t ldq;
    T *Ypart;        // [grid][c][mh]
    T *Z;            // kProject: Bt, nhat x c
    int64_t ldz;
    double *Gpart;   // kProject: [grid][c][c]
    // kProject, optional: also draw Omega's rows for the next sketch,
    // om[k * 8 + j] for k < nh, j < om_c (zeros past om_c), with (seed,
    // om_counter) as launch_omega_rows does
    double *om = nullptr;
    int om_c = 0;
    uint64_t om_counter = 0;
};

struct LongPlan {
    int kt, mhp, ntiles, grid, cm, rpt;
    size_t lds;
    // vector-FMA form (narrow c): columns padded to cmv, rows per thread rptv
    int vec, cmv, rptv;
    size_t ldsv;
    size_t ldst;   // transposed fast form
};

bool long_path_ok(int mh, int c);
LongPlan long_plan(int mh, int64_t nh, int c, int elem_bytes, int mode, int num_cu, bool trans);
// the most workgroups a long pass launches (partial buffers are sized for it)
int long_grid_cap(int num_cu);
template <typename T>
hipError_t launch_long(const LongPlan &plan, int mode, const LongArgs<T> &args, hipStream_t s);

// out[j] = sum_{g < nparts} part[g * count + j], fixed order.
template <typename T>
hipError_t launch_reduce(const T *part, int64_t count, int nparts, T *out, hipStream_t s);
// G = Ahat Ahat^T (mh x mh, double, column-major) for the transposed
// orientation (Ahat(i, k) = A[k + i lda]), mh <= 256, on `grid` workgroups;
// part: gram_tr_part_doubles(mh, grid) doubles, sum: the same for grid = 1.
bool gram_tr_ok(int mh, int64_t nh, int64_t lda, int elem_bytes);
size_t gram_tr_part_doubles(int mh, int grid);
template <typename T>
hipError_t launch_gram_tr(const T *A, int64_t lda, int mh, int64_t nh, int grid, double *part, double *sum,
                          double *G, hipStream_t s);
// sum of nparts doubles (the order of launch_reduce with count 1), the
// first nstatus status words and the double *res (-1 when res is null),
// written to mapped host memory (device pointers host_status, host_z,
// host_res); then, if host_seq is set, seq to *host_seq (after the words,
// so that a host polling that word sees them)
hipError_t launch_finish_iter(const double *part, int nparts, const int *status, int nstatus,
                              int *host_status, double *host_z, const double *res, double *host_res,
                              hipStream_t s, int *host_seq = nullptr, int seq = 0);

// ------------------------------------------------------ one-workgroup CholeskyQR
// Q = orth([Qt, Y]) with Qt (mh x rp) orthonormal and Y (mh x c):
//  CGS2 of Y against Qt, column equilibration, shifted CholeskyQR, then
//  CholeskyQR2 with refill of numerically null columns.  mh * (rp + c) must
//  fit the LDS budget (small_orth_ok).  resid2 (optional, device) receives
//  the squared norm of the first new column after CGS2 (-1 when c = 0).
bool small_orth_ok(int mh, int l);
template <typename T>
hipError_t launch_small_orth(int mh, const T *Qt, int64_t ldqt, int rp, const T *Y, int64_t ldy,
                             int c, T *Q, int64_t ldq, uint64_t seed, uint64_t counter,
                             int *flags, double *resid2, hipStream_t s);
// The same squared residual for a basis block Q = [Qt (rp columns), samples
// (c columns)] (two classical Gram-Schmidt passes of column rp against the
// first rp columns); -1 when c = 0.  (mh + rp) doubles of LDS, at most 64 KB.
template <typename T>
hipError_t launch_resid_est(int mh, const T *Q, int64_t ldq, int rp, int c, double *out, hipStream_t s);
// Sequential residual check: out[j] = squared norm of column j of Y after
// classical Gram-Schmidt (two passes) against [Qt (rp columns), the
// normalised residuals of columns 0..j-1].  mh (c + 1) + rp + c + 1 doubles
// of LDS, at most 64 KiB.
template <typename T>
hipError_t launch_resid_seq(int mh, const T *Qt, int64_t ldqt, int rp, const T *Y, int64_t ldy, int c,
                            double *out, hipStream_t s);
bool resid_seq_ok(int mh, int rp, int c);
// Rank truncation of a fresh sketch Y (mh x c) by Householder QR with
// column pivoting: *s_out = #{leading |R_jj| > tol_factor |R_00|}; the first
// s pivoted columns of Y are written to Yout.  One workgroup, Y in LDS.
template <typename T>
hipError_t launch_qrcp_trunc(int mh, int c, const T *Y, int64_t ldy, double tol_factor, T *Yout, int64_t ldo,
                             int *s_out, hipStream_t s);
bool qrcp_trunc_ok(int mh, int c);

// ------------------------------------------------------------- small SVD
// From the l x l Gram G = B B^T (double): semidefinite Cholesky G = R^T R,
// one-sided Jacobi on R^T, U_B and sigma (descending), thresholds (tau, or
// per-index weights w when w != nullptr), r = #{f > 0}, Mm = U diag(f/s) U^T.
// With Q (mh x l) given and mh * l small, also QM = Q Mm (mh x l) and
// Qout = Q U(:, 1:r).  Jacobi storage: LDS when l <= 128, else work (l*l).
struct SmallSvdOut {
    double *sigma;   // l
    double *U;       // l x l
    double *Mm;      // l x l
    int *status;     // [0] r, [1] sweeps, [2] converged flag, [3] unused
};
//  Thresholds in descending order of sigma: w[a] when w is set, else 0 for
//  the first keep values (partial SVT: they pass unshrunk) and tau after.
template <typename T>
hipError_t launch_small_svd(int l, const double *G, double tau, const double *w, int keep, const T *Q,
                            int64_t ldq, int mh, T *QM, int64_t ldqm, T *Qout, int64_t ldqo,
                            const SmallSvdOut &out, double *work, int fuse_q, hipStream_t s, int in_factor = 0);
// (in_factor: G holds an upper triangular factor C, column-major, with B^T = H C
//  for some H with orthonormal columns; the Cholesky step is skipped)
bool small_svd_fuse_q_ok(int mh, int l);

// ------------------------------------------------ rank-l reconstruct family
// Physical element (pr, pc) of an m x n column-major output, with
// L(pr, pc) = sum_c FR(pr, c) FC(pc, c):
//   kRecon : X = L
//   kEpi   : t = O - L + Y/mu, S = shrink(t, lam/mu), z = O - L - S,
//            Ynext = Y + mu z, Anext = O - S + Ynext/mu_next, zpart += z^2
//   kFinal : L and S of the last iteration (Y = the multiplier it used).
enum ReconMode { kRecon = 0, kEpi = 1, kFinal = 2 };
template <typename T>
struct ReconArgs {
    int64_t rows, cols;   // physical
    int c;
    const T *FR;          // rows x c, ld ldfr
    int64_t ldfr;
    const T *FC;          // cols x c, ld ldfc
    int64_t ldfc;
    T *X;                 // kRecon output / kFinal L
    int64_t ldx;
    const T *O;
    int64_t ldo;
    const T *Y;           // multiplier in
    int64_t ldy;
    T *Ynext;
    int64_t ldyn;
    T *Anext;
    int64_t ldan;
    T *S;                 // kFinal S
    int64_t lds;
    double mu, mu_next, lam;
    double *zpart;        // [grid] partial sums of z^2
    const T *Lin;         // when set, L is read from here instead of FR FC^T
    int64_t ldlin;
    // kEpi, T = double, rows = the long index: when ysk is set, the Gaussian
    // sketch of Anext for the next iteration is accumulated alongside,
    // ysk[blockIdx.x][i + j * cols] = sum over the workgroup's rows k of
    // Anext(k, i) Omega(k, j), j < csk <= 8, Omega drawn from (seed, counter)
    // as the sketch pass draws it.
    T *ysk;
    int csk;
    uint64_t seed, counter;
    // optional: Omega's rows drawn beforehand by launch_omega_rows (8 per
    // row, the same values); nullptr: drawn in the epilogue
    const double *om = nullptr;
    // row and column block counts (set by launch_recon)
    int nrb = 0, ncb = 0;
};
bool recon_ok(int c);
int64_t recon_row_blocks(int64_t rows);   // grid.x of the epilogue launch
template <typename T>
hipError_t launch_recon(int mode, const ReconArgs<T> &a, int *nparts, hipStream_t s);

// ------------------------------------------------------------ elementwise
// Sum of squares and max |.| of an m x n matrix: parts[2*g] = sum, parts[2*g+1] = max;
// with flag, *flag |= 1 in the same pass when an entry is NaN or infinite.
template <typename T>
hipError_t launch_norms(int64_t m, int64_t n, const T *A, int64_t lda, double *parts,
                        int *nparts, hipStream_t s, int *flag = nullptr);
// Y = O / J ;  A = O + Y / mu
template <typename T>
hipError_t launch_rpca_init(int64_t m, int64_t n, const T *O, int64_t ldo, double invJ,
                            double inv_mu, T *Y, int64_t ldy, T *A, int64_t lda, hipStream_t s);

// Largest eigenvalue of a symmetric positive semidefinite l x l matrix by the
// power method (one workgroup); out[0] = lambda_max.
// Largest eigenvalue of a symmetric PSD n x n matrix (8 <= n <= 1024) by
// block subspace iteration: out[0] the estimate, out[1] 1 when certified.
// Largest eigenvalue of the PSD n x n G (n <= 256) by a single-vector power
// iteration certified through the Kato-Temple bound when it exceeds half the
// trace: out[0] the estimate, out[1] 1 when certified (else 0).
hipError_t launch_power_dom(int n, const double *G, double *out, hipStream_t s);
// Omega(k, 0..csk-1) of the sketch, rows k < rows, into om[k * 8 + j]
// (zeros past csk): the epilogue's fused sketch reads them.
hipError_t launch_omega_rows(int64_t rows, int csk, uint64_t seed, uint64_t counter, double *om, hipStream_t s);
hipError_t launch_power_eig(int n, const double *G, double *out, hipStream_t s);

// --------------------------------------------------------- generic GEMM
// C(m, n) = sum_k A(m, k) B(k, n) with arbitrary element strides:
//   A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn], C(m,n) = C[m*scm + n*scn].
// splitk > 1 writes TA partials to part ([splitk][N][M]) and a store pass sums
// them in order into C.
template <typename TI, typename TA, typename TO>
hipError_t launch_gemm(int64_t M, int64_t N, int64_t K, const TI *A, int64_t sam, int64_t sak,
                       const TI *B, int64_t sbk, int64_t sbn, TO *C, int64_t scm, int64_t scn,
                       int splitk, TA *part, hipStream_t s);

// Omega (rows x cols, ld) materialised in storage precision.
template <typename T>
hipError_t launch_omega(int64_t rows, int cols, uint64_t seed, uint64_t counter, T *Om,
                        int64_t ld, hipStream_t s);

// ----------------------------------------------------- large CholeskyQR pieces
// One Cholesky pass on the l x l Gram (double, one workgroup): R = chol(G + shift I)
// with shift = shift_factor * trace(G); pivots below null_tol * maxdiag are
// flagged (flags[1] counts them, null_cols[j] = 1) and get R_jj = 1 with a
// zero row.  flags[2] |= 1 when a pivot is not positive in a pass without
// null handling.
// G = Y^T Y (l x l, [a * l + b]) for a tall rows x l matrix, l <= 128:
// partial Grams on the matrix cores into part (at most 64 l^2 doubles), then
// their sum.
// A non-null gate with *gate == 0 skips the partial products (they are
// still current).
template <typename T>
hipError_t launch_gram_tall(int64_t rows, int l, const T *Y, int64_t ldy, double *part, double *G,
                            hipStream_t s, const int *gate = nullptr);
// gate: as for launch_gram_tall (R is still current); nn_out receives the
// number of null pivots; near_one > 0 also treats a pivot further than
// near_one from 1 as null; dinv (optional, 256 ceil(l / 16) doubles)
// receives the inverses of R's 16 x 16 diagonal blocks (identity past l);
// l <= 128, or l <= 256 with gwork (a workspace of lp^2 doubles, lp = l
// rounded up to 16).
hipError_t launch_chol(int l, const double *G, double shift_factor, double null_tol, double *R,
                       int *null_cols, int *flags, hipStream_t s, const int *gate = nullptr,
                       int *nn_out = nullptr, double near_one = 0.0, double *dinv = nullptr,
                       double *gwork = nullptr);
// G_out(a, b) = G(a, b) / sqrt(G(a, a) G(b, b)): the Gram after k_col_scale.
hipError_t launch_scale_gram(int l, const double *G, double *Gout, hipStream_t s);
// Y (rows x l) <- Y R^{-1} in place (R upper, double): with dinv (the
// inverses of R's 16 x 16 diagonal blocks, 256 doubles each, as launch_chol
// writes them) on the matrix cores, one wavefront per 16 rows (l <= 256);
// else one lane per row (l <= 128).
template <typename T>
hipError_t launch_trsm(int64_t rows, int l, T *Y, int64_t ldy, const double *R, hipStream_t s,
                       const double *dinv = nullptr, const int *gate = nullptr);
// Y (rows x l) <- Y U in place, U upper triangular (row-major, double),
// l <= 256; nothing when skip is set and *skip != 0.
template <typename T>
hipError_t launch_trmm(int64_t rows, int l, T *Y, int64_t ldy, const double *U, hipStream_t s,
                       const int *skip = nullptr);
// U = I - S, S the upper triangle of E = G - I with half its diagonal (the
// inverse of G's Cholesky factor to first order in E); *full = 1 when
// ||E||_F > tol, else 0; *nn = 0.
hipError_t launch_near_identity(int l, const double *G, double *U, int *full, int *nn, double tol, hipStream_t s);
// Y(:, j) <- Gaussian(refill stream) for null_cols[j] = 1; also scales
// columns to unit norm when normalize != 0 (norms from the Gram diagonal).
template <typename T>
hipError_t launch_refill(int64_t rows, int l, T *Y, int64_t ldy, const int *null_cols,
                         uint64_t seed, uint64_t counter, int attempt, hipStream_t s);
template <typename T>
hipError_t launch_col_scale(int64_t rows, int l, T *Y, int64_t ldy, const double *G,
                            hipStream_t s);
// Y <- Y - Qt (Qt^T Y): coefficients C (rp x c) = Qt^T Y then the update.
template <typename T>
hipError_t launch_cast(int64_t m, int64_t n, const void *src, int src_is_double, int64_t lds,
                       T *dst, int64_t ldd, hipStream_t s);

}  // namespace frk

namespace frk {
// Matrix-core GEMMs (gemm_mfma.hip), strides as launch_gemm; each operand
// needs one unit stride.  splitk > 1 needs `part` ([splitk][N][M]).
hipError_t launch_gemm_bf16(int64_t M, int64_t N, int64_t K, const uint16_t *A, int64_t sam,
                            int64_t sak, const uint16_t *B, int64_t sbk, int64_t sbn, float *C,
                            int64_t scm, int64_t scn, int splitk, float *part, hipStream_t s);
hipError_t launch_gemm_f32_mfma(int64_t M, int64_t N, int64_t K, const float *A, int64_t sam,
                                int64_t sak, const float *B, int64_t sbk, int64_t sbn, float *C,
                                int64_t scm, int64_t scn, int splitk, float *part, hipStream_t s);
hipError_t launch_gemm_f64_mfma(int64_t M, int64_t N, int64_t K, const double *A, int64_t sam,
                                int64_t sak, const double *B, int64_t sbk, int64_t sbn, double *C,
                                int64_t scm, int64_t scn, int splitk, double *part, hipStream_t s);
// Tall-skinny products C (M x N) = A (M x K) B (K x N), N <= 128, B
// k-contiguous (B(k, n) at B[k + n ldb]); A k-contiguous (sak = 1, rows
// 16-byte aligned) or, for float and double, row-contiguous (sam = 1).
// Split K into part (at most part_cap values), reduced into C in a fixed
// order.  hipErrorNotSupported for other shapes (the caller falls back).
// whether launch_ts_gemm_* takes these operands (esize: bytes per element;
// k-contiguous A needs 16-byte aligned rows; row-contiguous A is float or
// double only)
bool ts_gemm_ok(int64_t N, int64_t sam, int64_t sak, const void *A, int esize);
hipError_t launch_ts_gemm_bf16(int64_t M, int64_t N, int64_t K, const uint16_t *A, int64_t sam, int64_t sak,
                               const uint16_t *B, int64_t ldb, float *C, int64_t scm, int64_t scn,
                               float *part, int64_t part_cap, int num_cu, hipStream_t s);
hipError_t launch_ts_gemm_f32(int64_t M, int64_t N, int64_t K, const float *A, int64_t sam, int64_t sak,
                              const float *B, int64_t ldb, float *C, int64_t scm, int64_t scn,
                              float *part, int64_t part_cap, int num_cu, hipStream_t s);
hipError_t launch_ts_gemm_f64(int64_t M, int64_t N, int64_t K, const double *A, int64_t sam, int64_t sak,
                              const double *B, int64_t ldb, double *C, int64_t scm, int64_t scn,
                              double *part, int64_t part_cap, int num_cu, hipStream_t s);
// both bfloat16 copies of an m x n column-major float matrix: dst (m x n,
// ld m) and its transpose dstT (n x m, ld n)
hipError_t launch_to_bf16_pair(int64_t m, int64_t n, const float *src, int64_t lds, uint16_t *dst,
                               uint16_t *dstT, hipStream_t s);
// float -> bfloat16 (round to nearest even) of an m x n column-major matrix
hipError_t launch_to_bf16(int64_t m, int64_t n, const float *src, int64_t lds, uint16_t *dst,
                          int64_t ldd, hipStream_t s);
// Omega drawn as in the sketch kernels, rounded to float then to bfloat16
hipError_t launch_omega_bf16(int64_t rows, int cols, uint64_t seed, uint64_t counter, uint16_t *Om,
                             int64_t ld, hipStream_t s);
}  // namespace frk

namespace frk {
// Persistent batched weighted SVT (wsvt_batched.hip).
struct WsvtBatchArgs {
    int64_t count;
    const int32_t *rows, *cols;
    const int64_t *offsets;
    const float *A;
    float *X;
    double c, noise_var, eps, tau;
    int32_t *ranks;          // optional
    int32_t *sweeps;         // optional, Jacobi sweeps per matrix
    const int32_t *order;    // processing order or nullptr
    int *queue;              // work counter
    unsigned long long *work;   // optional: Jacobi work counters (pair rows, rotation rows, rotations)
    const int32_t *group_size;  // lanes per Jacobi pair group, per size bucket (3)
};
size_t wsvt_batched_lds();
hipError_t launch_wsvt_batched(const WsvtBatchArgs &a, int grid, hipStream_t s);
}  // namespace frk

namespace frk {
// Adjoint pieces (adjoint.hip).
// M1, M2 (l x l) of the SVT VJP on the small factors sigma, U of B and
// H = Sbar B^T; taubar (device, optional).  l <= 64.
hipError_t launch_svt_vjp_small(int l, const double *sigma, const double *U, const double *H,
                                double tau, double *M1, double *M2, double *tau_bar, hipStream_t s);
// CA = R^{-T}, CB = copyltu(-K) R^{-T} for the QR VJP; l <= 64.
hipError_t launch_qr_vjp_small(int l, const double *K, const double *R, double *CA, double *CB,
                               int *flags, hipStream_t s);

// p[0..count) = value.
hipError_t launch_fill_int(int *p, int count, int value, hipStream_t s);

constexpr int kCombineMaxIn = 3;
template <typename T>
struct CombineArgs {
    int64_t rows;
    int c;
    int nin;
    const T *in[kCombineMaxIn];
    int64_t ldin[kCombineMaxIn];
    int w[kCombineMaxIn];
    const double *coef[kCombineMaxIn];  // w_b x c, column-major; nullptr = identity
    T *out;
    int64_t ldout;
};
template <typename T>
hipError_t launch_combine(const CombineArgs<T> &a, hipStream_t s);

constexpr int kDualGrid = 1024;
template <typename T>
struct DualStepArgs {
    int64_t m, n;
    const T *O;
    int64_t ldo;
    const T *L;
    int64_t ldl;
    const T *Y;
    int64_t ldy;
    double lam, mu, mu_next;
    // forward outputs (each optional)
    T *S;
    int64_t lds;
    T *Yn;
    int64_t ldyn;
    T *An;
    int64_t ldan;
    // reverse: upstream gradients (optional), outputs, lambar partials
    const T *Sb;
    int64_t ldsb;
    const T *Ynb;
    int64_t ldynb;
    const T *Anb;
    int64_t ldanb;
    T *Lb;
    int64_t ldlb;
    T *Yb;
    int64_t ldyb;
    double *part;  // [grid]
};
template <typename T>
hipError_t launch_dual_step(const DualStepArgs<T> &a, bool vjp, int *nparts, hipStream_t s);
// ------------------------------------------------ low-rank representation host
// out = a A + b B + c C + g I (m x n, column-major; null operands skipped;
// out may alias A).
hipError_t launch_lrr_comb(int64_t m, int64_t n, double a, const double *A, int64_t lda, double b,
                           const double *B, int64_t ldb, double c, const double *C, int64_t ldc, double g,
                           double *out, int64_t ldo, hipStream_t s);
// out[0] = max_i sum_j |A(i, j)| (n x n)
hipError_t launch_lrr_norm_inf(int64_t n, const double *A, int64_t lda, double *out, hipStream_t s);
// E(:, j) = max(0, 1 - thr / ||v_j||) v_j, v = X - XZ + Y1 inv_mu (XZ, Y1 d x n, ld d)
hipError_t launch_lrr_colshrink(int64_t d, int64_t n, const double *X, int64_t ldx, const double *XZ,
                                const double *Y1, double inv_mu, double thr, double *E, int64_t lde, hipStream_t s);
// Y (ld m) += mu (P - Q - R), part[lrr_dual_parts()] = per-block max |P - Q - R|
int lrr_dual_parts();
hipError_t launch_lrr_dual(int64_t m, int64_t n, double mu, const double *P, int64_t ldp, const double *Q,
                           int64_t ldq, const double *R, int64_t ldr, double *Y, double *part, hipStream_t s);
// out[k] = max_g part[k * nparts + g], k < count
hipError_t launch_lrr_max_parts(const double *part, int nparts, int count, double *out, hipStream_t s);
// ------------------------------------------------ 3-way tensor host
// (column-major I1 x I2 x I3; "mode-2 layout" = the mode-2 unfolding,
// rows i2, columns i1 + I1 i3)
int ten_parts();
// A2p = O in mode-2 layout
hipError_t launch_ten_perm(int64_t I1, int64_t I2, int64_t I3, const double *O, double *A2p, hipStream_t s);
// E = shrink_thr(mean_i(O - L_i + Y_i/mu)), Y_i += mu (O - L_i - E),
// A_i = O - E + Y_i/mu_next; sums[i] = ||O - L_i - E||_F^2 (part: 3 ten_parts())
hipError_t launch_ten_update(int64_t I1, int64_t I2, int64_t I3, const double *O, const double *L1,
                             const double *L2p, const double *L3, double *Y1, double *Y2, double *Y3, double *E,
                             double *A1, double *A2p, double *A3, double mu, double thr, double mu_next,
                             double *part, double *sums, hipStream_t s);
// L = (L1 + L2 + L3) / 3 (L may alias L1)
hipError_t launch_ten_mean(int64_t I1, int64_t I2, int64_t I3, const double *L1, const double *L2p,
                           const double *L3, double *L, hipStream_t s);

}  // namespace frk
