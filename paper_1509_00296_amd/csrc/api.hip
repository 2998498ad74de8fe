// api.hip -- host orchestration behind the C ABI declared in include/frsvt.h.
//
// Argument validation, the handle and its workspace, and the order of the
// kernel launches for Alg. 1 (FRSVT), exact SVT, weighted SVT and the
// inexact-ALM RPCA loop of arXiv:1509.00296.
#include "frsvt.h"
#include "internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

using namespace frk;

struct frsvt_context {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cu = 256;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    int *dstatus = nullptr;      // small device status area (ints)
    double *dscalars = nullptr;  // small device scalar area (doubles)
    void *pinned = nullptr;      // host pinned status area
    void *scratch_dev = nullptr; // device address of this device's fixed scratch (frsvt_noalloc)
    int opt_truncate = 0;        // FRSVT_OPT_QRCP_TRUNCATE
    char last_error[256] = {0};
    // unrolled RPCA and other batch drivers: side contexts, each with its own
    // stream, workspace and status words, that run instances concurrently;
    // the fork/join events; a buffer for per-call state the drivers keep
    frsvt_context *side[4] = {nullptr, nullptr, nullptr, nullptr};
    bool owns_stream = false;
    hipEvent_t ev_fork = nullptr;
    hipEvent_t ev_join = nullptr;
    void *aux = nullptr;
    size_t aux_bytes = 0;
    // batched weighted SVT: tuned group sizes per size bucket, the queue and
    // order buffers, and the captured graph of the last argument set
    int wb_gs[3] = {0, 0, 0};
    bool wb_tuned = false;
    int *wb_queue = nullptr;
    int32_t *wb_gs_dev = nullptr;
    int32_t *wb_order = nullptr;
    int64_t wb_order_cap = 0;
    hipStream_t wb_capture = nullptr;
    hipGraphExec_t wb_exec = nullptr;
    std::vector<uint64_t> wb_key;
    // per-iteration status event of the RPCA host loop
    int iter_seq = 0;                // last sequence number of an RPCA iteration
    void *host_iter = nullptr;       // coherent mapped host words of the RPCA loop
    void *host_iter_dev = nullptr;   // its device address
    // tracing: event pairs around launches, aggregated per kernel class
    bool tracing = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> recs;
    std::vector<hipEvent_t> pool;
    double trace_ms[FRSVT_K_COUNT] = {0};
    int64_t trace_n[FRSVT_K_COUNT] = {0};
};

// Fixed scratch of frsvt_noalloc: a workspace that is never allocated at
// run time.  Each GPU the library runs on holds its own copy of this array
// until the process ends.  Host code never uses the array's name as an
// address: frsvt_create looks up the device address once per device (with
// that device current) and every launch takes that pointer.
static __device__ __align__(256) unsigned char scratch[FRSVT_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {nullptr};
bool g_scratch_done[kMaxDevices] = {false};

// Device address of `scratch` on the current device `device` (looked up
// once per device; nullptr when the lookup fails).
void *scratch_address(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[device]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_scratch_addr[device] = e == hipSuccess ? ptr : nullptr;
        g_scratch_done[device] = true;
    }
    return g_scratch_addr[device];
}

// A workspace supplied by the caller of an implementation instead of the
// handle's growable one.
struct FixedWs {
    void *base;
    size_t cap;
};

} // namespace

namespace {

constexpr double kU = 1.1102230246251565e-16;
constexpr size_t kStatusInts = 1024;
constexpr int kGateSlot = 12;  // status word: null pivots of the large path's first null check
constexpr int kResidSlot = 20; // status words 20-21: a double, Prop. 4's squared residual
constexpr size_t kScalarDoubles = 8192;
constexpr size_t kCheckSlot = 4096;  // device scalars 4096..4159: the residual check's squared norms

int fail(frsvt_context *h, hipError_t e, const char *what)
{
    if (h) snprintf(h->last_error, sizeof(h->last_error), "%s: %s", what, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? FRSVT_ERR_OOM : FRSVT_ERR_HIP;
}

#define CK(expr)                                                   \
    do {                                                           \
        hipError_t e_ = (expr);                                    \
        if (e_ != hipSuccess) return fail(h, e_, #expr);           \
    } while (0)

hipEvent_t ev_get(frsvt_context *h)
{
    if (!h->pool.empty()) {
        hipEvent_t e = h->pool.back();
        h->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records a HIP event pair on the handle's stream around one launch when
// tracing is on.
struct Span {
    frsvt_context *h;
    int id;
    hipEvent_t a = nullptr;
    Span(frsvt_context *hh, int kid) : h(hh), id(kid)
    {
        if (h->tracing) {
            a = ev_get(h);
            if (a) (void)hipEventRecord(a, h->stream);
        }
    }
    ~Span()
    {
        if (h->tracing && a) {
            hipEvent_t b = ev_get(h);
            if (b) {
                (void)hipEventRecord(b, h->stream);
                h->recs.push_back({id, {a, b}});
            }
        }
    }
};

#define CKT(kid, expr)                                             \
    do {                                                           \
        Span sp_(h, kid);                                          \
        hipError_t e_ = (expr);                                    \
        if (e_ != hipSuccess) return fail(h, e_, #expr);           \
    } while (0)

// Bump allocator over the handle's workspace; sizes are computed first with
// a dry run (base == nullptr), then the workspace is grown to fit.
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base((char *)b) {}
    template <typename T>
    T *take(size_t count)
    {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? (T *)(base + off) : nullptr;
        off += std::max<size_t>(count, 1) * sizeof(T);
        return p;
    }
};

int ensure_ws(frsvt_context *h, size_t bytes)
{
    if (bytes <= h->ws_bytes) return FRSVT_OK;
    if (h->ws) {
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return fail(h, e, "hipStreamSynchronize");
        (void)hipFree(h->ws);
        h->ws = nullptr;
        h->ws_bytes = 0;
    }
    size_t grow = std::max(bytes, (size_t)(h->ws_bytes * 3 / 2));
    hipError_t e = hipMalloc(&h->ws, grow);
    if (e != hipSuccess) {
        h->ws = nullptr;
        return fail(h, e, "hipMalloc(workspace)");
    }
    h->ws_bytes = grow;
    return FRSVT_OK;
}

template <typename T>
struct Prec;
template <>
struct Prec<double> {
    static constexpr int bytes = 8;
};
template <>
struct Prec<float> {
    static constexpr int bytes = 4;
};

// Strides of Ahat(i, k) = A[i * si + k * sk].
struct Orient {
    bool trans;
    int mh;
    int64_t nh;
    int64_t si, sk;
    int64_t si16, sk16;  // strides of the bfloat16 copy (leading dimension = rows of A)
};
Orient orient(int64_t m, int64_t n, int64_t lda)
{
    Orient o;
    o.trans = m > n;
    o.mh = (int)(o.trans ? n : m);
    o.nh = o.trans ? m : n;
    o.si = o.trans ? lda : 1;
    o.sk = o.trans ? 1 : lda;
    const int64_t rows = o.trans ? o.nh : o.mh;
    o.si16 = o.trans ? rows : 1;
    o.sk16 = o.trans ? 1 : rows;
    return o;
}

int gemm_splitk(int64_t M, int64_t N, int64_t K, int num_cu)
{
    const int64_t tiles = ((M + 63) / 64) * ((N + 63) / 64);
    int64_t want = (2 * num_cu + tiles - 1) / std::max<int64_t>(tiles, 1);
    want = std::min<int64_t>(want, std::max<int64_t>(1, K / 256));
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, 128));
}

// ---------------------------------------------------------------------------
// The FRSVT core: basis Q, projection B^T, the small SVD and the factors of
// the reconstruction X = (Q Mm) B, all in the workspace.
// ---------------------------------------------------------------------------
template <typename T>
struct Core {
    // inputs
    const T *A;
    int64_t lda;
    const uint16_t *A16;  // bfloat16 copy of A (precision form) or nullptr
    const uint16_t *A16T; // bfloat16 copy of A^T (precision form) or nullptr
    Orient o;
    double tau;
    const double *w;     // device weights (WSVT) or nullptr
    int q;
    const T *Qt;         // propagated basis (mh x rp) or nullptr
    int64_t ldqt;
    int rp;
    int cnew;            // new Gaussian samples
    uint64_t seed, counter;
    T *Qout;             // mh x l (ld ldqo); may alias Qt
    int64_t ldqo;
    bool sketch_ready;   // the sketch of this call is already in the buffers
    bool orth_ready = false;  // its orthonormalised basis [Qt, Y] too (b.Q, one-workgroup path)
    // optional: the projection pass also draws Omega's rows (counter
    // om_counter, om_c columns) into om for the next sketch; om_drawn is set
    // once they are enqueued
    double *om = nullptr;
    int om_c = 0;
    uint64_t om_counter = 0;
    bool om_drawn = false;
    // results (workspace)
    int l;
    T *Q, *Bt, *QM;
    double *G, *U, *Mm, *sigma;
    int *status;         // device: [0] r, [1] sweeps, [2] converged, [4..] orth flags
    double *resid_out = nullptr;   // device, optional: squared residual of the first new sample (Prop. 4)
    int keep = 0;        // partial SVT: the first keep singular values pass unshrunk
    const T *ysrc = nullptr;  // sketch columns to orthonormalise when not b.Y (after truncation)
};

template <typename T>
struct CoreBuffers {
    uint16_t *V16;   // bfloat16 scratch (nh x l) for the precision form
    T *Ypart, *Y, *Q, *Bt, *QM, *Om, *Z, *gpart_t, *Qtmp;
    double *Gpart, *G, *U, *Mm, *sigma, *R, *gpart_d, *jwork;
    double *dinv;    // inverses of R's 16 x 16 diagonal blocks (large path)
    double *cholw;   // the Cholesky's workspace beyond l = 128 (lp^2 doubles), else null
    int *nullc;
    size_t ypart_cap;   // elements of Ypart
};

template <typename T>
size_t carve_core(Carver &cv, const Orient &o, int l, int cnew, int num_cu, CoreBuffers<T> &b,
                  bool force_big = false)
{
    const int mh = o.mh;
    const int64_t nh = o.nh;
    const int grid = long_grid_cap(num_cu);
    const int cmax = std::max(l, 1);
    // the long passes' partials (they take at most 32 columns, and only
    // where the short side fits them)
    const size_t ypc = long_path_ok(mh, 1) ? (size_t)grid * mh * std::min(cmax, 32) : (size_t)mh;
    b.Ypart = cv.take<T>(ypc);
    b.ypart_cap = ypc;
    b.Y = cv.take<T>((size_t)mh * cmax);
    b.Q = cv.take<T>((size_t)mh * cmax);
    b.Qtmp = cv.take<T>((size_t)mh * cmax);
    b.Bt = cv.take<T>((size_t)nh * cmax);
    b.QM = cv.take<T>((size_t)mh * cmax);
    b.Gpart = cv.take<double>(long_path_ok(mh, 1) ? (size_t)grid * std::min(cmax, 32) * std::min(cmax, 32)
                                                  : (size_t)cmax * cmax);
    b.G = cv.take<double>((size_t)cmax * cmax);
    b.U = cv.take<double>((size_t)cmax * cmax);
    b.Mm = cv.take<double>((size_t)cmax * cmax);
    b.sigma = cv.take<double>((size_t)cmax);
    b.R = cv.take<double>((size_t)cmax * cmax);
    b.nullc = cv.take<int>((size_t)cmax);
    b.jwork = cv.take<double>((size_t)cmax * cmax);
    b.dinv = cv.take<double>((size_t)256 * ((cmax + 15) / 16));
    b.cholw = cmax > 128 ? cv.take<double>((size_t)((cmax + 15) / 16) * 256 * ((cmax + 15) / 16)) : nullptr;
    const bool big = force_big || !(long_path_ok(mh, std::max(l, 1)) && small_orth_ok(mh, l));
    b.V16 = nullptr;
    if (big) {
        b.V16 = cv.take<uint16_t>((size_t)nh * cmax);
        b.Om = cv.take<T>((size_t)nh * std::max(cnew, 1));
        b.Z = cv.take<T>((size_t)nh * cmax);
        // GEMM split-K partials: the largest of Y = Ahat V and Gram products
        const size_t p1 = (size_t)128 * mh * cmax;
        b.gpart_t = cv.take<T>(p1);
        b.gpart_d = cv.take<double>((size_t)std::max<int64_t>(128 * (int64_t)cmax * cmax, (int64_t)mh * cmax * 4));
    } else {
        b.Om = b.Z = b.gpart_t = nullptr;
        b.gpart_d = nullptr;
    }
    return cv.off;
}

// C = A B with arbitrary strides in storage precision: matrix cores when
// each operand has a unit stride, the generic tiled kernel otherwise.
template <typename T>
int mm(frsvt_context *h, int64_t M, int64_t N, int64_t K, const T *A, int64_t sam, int64_t sak,
       const T *B, int64_t sbk, int64_t sbn, T *C, int64_t scm, int64_t scn, int splitk, T *part)
{
    const bool unit = (sam == 1 || sak == 1) && (sbk == 1 || sbn == 1);
    if (splitk > 1 && part == nullptr) splitk = 1;
    if (unit && std::is_same<T, double>::value) {
        CKT(FRSVT_K_GEMM, launch_gemm_f64_mfma(M, N, K, (const double *)A, sam, sak, (const double *)B, sbk,
                                               sbn, (double *)C, scm, scn, splitk, (double *)part, h->stream));
    } else if (unit) {
        CKT(FRSVT_K_GEMM, launch_gemm_f32_mfma(M, N, K, (const float *)A, sam, sak, (const float *)B, sbk,
                                               sbn, (float *)C, scm, scn, splitk, (float *)part, h->stream));
    } else {
        CKT(FRSVT_K_GEMM, (launch_gemm<T, T, T>(M, N, K, A, sam, sak, B, sbk, sbn, C, scm, scn, splitk,
                                                part, h->stream)));
    }
    return FRSVT_OK;
}

// Tall-skinny product in storage precision (see launch_ts_gemm_*).
template <typename T>
hipError_t ts_gemm(int64_t M, int64_t N, int64_t K, const T *A, int64_t sam, int64_t sak, const T *B,
                   int64_t ldb, T *C, int64_t scm, int64_t scn, T *part, int64_t cap, frsvt_context *h)
{
    if (std::is_same<T, double>::value)
        return launch_ts_gemm_f64(M, N, K, (const double *)A, sam, sak, (const double *)B, ldb, (double *)C, scm,
                                  scn, (double *)part, cap, h->num_cu, h->stream);
    return launch_ts_gemm_f32(M, N, K, (const float *)A, sam, sak, (const float *)B, ldb, (float *)C, scm, scn,
                              (float *)part, cap, h->num_cu, h->stream);
}

// Ahat(mh x nh) times a tall matrix V (nh x c, ld ldv): Y (mh x c, ld mh).
// In the precision form (c.A16 set) the product runs on bfloat16 copies of
// Ahat and V with float accumulation; V16 is scratch for the copy of V.
template <typename T>
int ahat_times(frsvt_context *h, const Core<T> &c, const T *V, int64_t ldv, int cols, T *Y,
               T *part, uint16_t *V16 = nullptr, bool v_is_bf16 = false)
{
    const Orient &o = c.o;
    const int sk = gemm_splitk(o.mh, cols, o.nh, h->num_cu);
    // split-K partials: the workspace holds 128 mh cmax values
    const int64_t cap = (int64_t)128 * o.mh * cols;
    if (c.A16) {
        const uint16_t *v16 = (const uint16_t *)V;
        if (!v_is_bf16) {
            CKT(FRSVT_K_OTHER, launch_to_bf16(o.nh, cols, (const float *)V, ldv, V16, o.nh, h->stream));
            v16 = V16;
            ldv = o.nh;
        }
        // Ahat(i, j) with j contiguous: A^T's copy, or A's when Ahat = A^T
        const uint16_t *Ak = o.trans ? c.A16 : c.A16T;
        if (ts_gemm_ok(cols, o.nh, 1, Ak, 2))
            CKT(FRSVT_K_GEMM_BF16, launch_ts_gemm_bf16(o.mh, cols, o.nh, Ak, o.nh, 1, v16, ldv, (float *)Y, 1,
                                                       o.mh, (float *)part, cap, h->num_cu, h->stream));
        else
            CKT(FRSVT_K_GEMM_BF16, launch_gemm_bf16(o.mh, cols, o.nh, c.A16, o.si16, o.sk16, v16, 1, ldv,
                                                    (float *)Y, 1, o.mh, sk, (float *)part, h->stream));
        return FRSVT_OK;
    }
    if (ts_gemm_ok(cols, o.si, o.sk, c.A, (int)sizeof(T))) {
        CKT(FRSVT_K_GEMM, ts_gemm<T>(o.mh, cols, o.nh, c.A, o.si, o.sk, V, ldv, Y, 1, o.mh, part, cap, h));
        return FRSVT_OK;
    }
    return mm<T>(h, o.mh, cols, o.nh, c.A, o.si, o.sk, V, 1, ldv, Y, 1, o.mh, sk, part);
}

// Ahat^T (nh x mh) times Q (mh x c): Z (nh x c, ld nh).  With use16 the
// product runs on the bfloat16 copies (Q16 is scratch for the copy of Q).
template <typename T>
int ahat_t_times(frsvt_context *h, const Core<T> &c, const T *Qm, int64_t ldq, int cols, T *Z,
                 T *part, bool use16 = false, uint16_t *Q16 = nullptr)
{
    const Orient &o = c.o;
    const int64_t cap = (int64_t)128 * o.mh * cols;
    if (use16 && c.A16) {
        CKT(FRSVT_K_OTHER, launch_to_bf16(o.mh, cols, (const float *)Qm, ldq, Q16, o.mh, h->stream));
        // Ahat(i, j) with i contiguous: A's copy, or A^T's when Ahat = A^T
        const uint16_t *Ak = o.trans ? c.A16T : c.A16;
        if (ts_gemm_ok(cols, o.mh, 1, Ak, 2))
            CKT(FRSVT_K_GEMM_BF16, launch_ts_gemm_bf16(o.nh, cols, o.mh, Ak, o.mh, 1, Q16, o.mh, (float *)Z, 1,
                                                       o.nh, (float *)part, cap, h->num_cu, h->stream));
        else
            CKT(FRSVT_K_GEMM_BF16, launch_gemm_bf16(o.nh, cols, o.mh, c.A16, o.sk16, o.si16, Q16, 1, o.mh,
                                                    (float *)Z, 1, o.nh, 1, (float *)part, h->stream));
        return FRSVT_OK;
    }
    if (ts_gemm_ok(cols, o.sk, o.si, c.A, (int)sizeof(T))) {
        CKT(FRSVT_K_GEMM, ts_gemm<T>(o.nh, cols, o.mh, c.A, o.sk, o.si, Qm, ldq, Z, 1, o.nh, part, cap, h));
        return FRSVT_OK;
    }
    return mm<T>(h, o.nh, cols, o.mh, c.A, o.sk, o.si, Qm, 1, ldq, Z, 1, o.nh, 1, part);
}

// Gram G = Y^T Y (l x l, double) of a tall rows x l matrix.
template <typename T>
int gram(frsvt_context *h, int64_t rows, int l, const T *Y, int64_t ldy, double *G, double *part,
         const int *gate = nullptr)
{
    if (l <= 128) {
        CKT(FRSVT_K_GEMM, launch_gram_tall<T>(rows, l, Y, ldy, part, G, h->stream, gate));
        return FRSVT_OK;
    }
    const int sk = gemm_splitk(l, l, rows, h->num_cu);
    if (std::is_same<T, double>::value) {
        CKT(FRSVT_K_GEMM, (launch_gemm<double, double, double>(l, l, rows, (const double *)Y, ldy, 1,
                                                (const double *)Y, 1, ldy, G, 1, l, sk, part,
                                                h->stream)));
    } else {
        CKT(FRSVT_K_GEMM, (launch_gemm<float, double, double>(l, l, rows, (const float *)Y, ldy, 1,
                                               (const float *)Y, 1, ldy, G, 1, l, sk, part,
                                               h->stream)));
    }
    return FRSVT_OK;
}

// Large-path orthonormalisation of Y (rows x l) in place.  The fast path
// below (CholeskyQR2, one host read of its checks); where a check fails, or
// under graph capture, the robust sequence: column equilibration, shifted
// CholeskyQR, CholeskyQR with null refill, a final CholeskyQR pass (no host
// synchronisation).
template <typename T>
int big_orth(frsvt_context *h, int64_t rows, int l, T *Y, int64_t ldy, CoreBuffers<T> &b,
             uint64_t seed, uint64_t counter, int *flags)
{
    int rc;
    // Fast path (not under graph capture: it reads two status words on the
    // host): equilibration, one CholeskyQR pass in double precision, then
    // the second pass.  The first factor must have no pivot at or below
    // 1e-8 of the equilibrated diagonal.  The second Gram is I + E: while
    // ||E||_F <= 1e-8 its inverse Cholesky factor is I - S to working
    // precision (S the upper triangle of E, half diagonal), applied as a
    // triangular product on the matrix cores; otherwise the second factor is
    // computed (every pivot within 1e-6 of 1).  Both solves use the matrix
    // cores with the inverses of the factor's diagonal blocks.  A float
    // basis is orthonormalised on a double copy (written back at the end); a
    // double one in place, its equilibrated copy kept.  On a failed check
    // the robust sequence below runs from the basis as it came (float) or
    // from the equilibrated copy (double).
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    CK(hipStreamIsCapturing(h->stream, &cap));
    const bool dbl = std::is_same<T, double>::value;
    const size_t need_f = 2 * (size_t)rows * l * sizeof(double);   // float: double copy + spare
    if (cap == hipStreamCaptureStatusNone && (l <= 128 || (l <= 256 && b.cholw)) && b.jwork && b.dinv && ldy == rows &&
        (dbl ? b.Qtmp != nullptr : (b.gpart_t != nullptr && (size_t)128 * rows * l * sizeof(T) >= need_f))) {
        int *nn = h->dstatus + kGateSlot + 1;   // two words: null pivots of each pass
        int *full = h->dstatus + kGateSlot + 3;  // 1: the second pass needs its own factor
        double *Yd = dbl ? reinterpret_cast<double *>(Y) : reinterpret_cast<double *>(b.gpart_t);
        if (!dbl) CKT(FRSVT_K_ORTH, launch_cast<double>(rows, l, Y, 0, ldy, Yd, rows, h->stream));
        if ((rc = gram<double>(h, rows, l, Yd, rows, b.G, b.gpart_d))) return rc;
        CKT(FRSVT_K_ORTH, launch_col_scale<double>(rows, l, Yd, rows, b.G, h->stream));
        CKT(FRSVT_K_ORTH, launch_scale_gram(l, b.G, b.jwork, h->stream));
        if (dbl) CK(hipMemcpyAsync(b.Qtmp, Yd, (size_t)rows * l * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
        CKT(FRSVT_K_ORTH, launch_chol(l, b.jwork, 0.0, 1e-8, b.R, b.nullc, nullptr, h->stream, nullptr, nn, 0.0, b.dinv,
                                      b.cholw));
        CKT(FRSVT_K_ORTH, launch_trsm<double>(rows, l, Yd, rows, b.R, h->stream, b.dinv));
        if ((rc = gram<double>(h, rows, l, Yd, rows, b.G, b.gpart_d))) return rc;
        CKT(FRSVT_K_ORTH, launch_near_identity(l, b.G, b.jwork, full, nn + 1, 1e-8, h->stream));
        CKT(FRSVT_K_ORTH, launch_trmm<double>(rows, l, Yd, rows, b.jwork, h->stream, full));
        CKT(FRSVT_K_ORTH, launch_chol(l, b.G, 0.0, 0.5, b.R, b.nullc, nullptr, h->stream, full, nn + 1, 1e-6, b.dinv,
                                      b.cholw));
        CKT(FRSVT_K_ORTH, launch_trsm<double>(rows, l, Yd, rows, b.R, h->stream, b.dinv, full));
        CK(hipMemcpyAsync(h->pinned, nn, 2 * sizeof(int), hipMemcpyDeviceToHost, h->stream));
        CK(hipStreamSynchronize(h->stream));
        const int *hn = (const int *)h->pinned;
        if (hn[0] == 0 && hn[1] == 0) {
            if (!dbl) CKT(FRSVT_K_ORTH, launch_cast<T>(rows, l, Yd, 1, rows, Y, ldy, h->stream));
            if (flags) {
                CKT(FRSVT_K_OTHER, launch_fill_int(flags, 3, 0, h->stream));
                CKT(FRSVT_K_OTHER, launch_fill_int(flags, 1, 1, h->stream));
            }
            return FRSVT_OK;
        }
        if (dbl) CK(hipMemcpyAsync(Y, b.Qtmp, (size_t)rows * l * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    }
    if ((rc = gram(h, rows, l, Y, ldy, b.G, b.gpart_d))) return rc;
    CKT(FRSVT_K_ORTH, launch_col_scale<T>(rows, l, Y, ldy, b.G, h->stream));
    const double shift = 11.0 * ((double)rows * l + (double)l * (l + 1)) * kU;
    if ((rc = gram(h, rows, l, Y, ldy, b.G, b.gpart_d))) return rc;
    CKT(FRSVT_K_ORTH, launch_chol(l, b.G, shift, 0.0, b.R, nullptr, flags, h->stream, nullptr, nullptr, 0.0, b.dinv,
                                  b.cholw));
    CKT(FRSVT_K_ORTH, launch_trsm<T>(rows, l, Y, ldy, b.R, h->stream, b.dinv));
    // The first null check records its count in *gate; when it found no
    // null column nothing was refilled, so the Gram and factor of the second
    // check and of the next pass would repeat it: those launches return at
    // once (no host round trip) and the pass uses the first check's R.
    int *gate = h->dstatus + kGateSlot;
    for (int attempt = 0; attempt < 2; ++attempt) {
        const int *g = attempt ? gate : nullptr;
        if ((rc = gram(h, rows, l, Y, ldy, b.G, b.gpart_d, g))) return rc;
        CKT(FRSVT_K_ORTH, launch_chol(l, b.G, 0.0, 16.0 * l * kU, b.R, b.nullc, flags, h->stream, g,
                                      attempt ? nullptr : gate, 0.0, b.dinv, b.cholw));
        CKT(FRSVT_K_ORTH, launch_refill<T>(rows, l, Y, ldy, b.nullc, seed, counter, attempt, h->stream));
    }
    if ((rc = gram(h, rows, l, Y, ldy, b.G, b.gpart_d, gate))) return rc;
    CKT(FRSVT_K_ORTH, launch_chol(l, b.G, 0.0, 16.0 * l * kU, b.R, b.nullc, flags, h->stream, gate, nullptr, 0.0,
                                  b.dinv, b.cholw));
    CKT(FRSVT_K_ORTH, launch_trsm<T>(rows, l, Y, ldy, b.R, h->stream, b.dinv));
    if ((rc = gram(h, rows, l, Y, ldy, b.G, b.gpart_d))) return rc;
    CKT(FRSVT_K_ORTH, launch_chol(l, b.G, 0.0, 0.0, b.R, nullptr, flags, h->stream, nullptr, nullptr, 0.0, b.dinv,
                                  b.cholw));
    CKT(FRSVT_K_ORTH, launch_trsm<T>(rows, l, Y, ldy, b.R, h->stream, b.dinv));
    return FRSVT_OK;
}

// Alg. 1's sampling step (fresh or range-propagated) on the one-workgroup path: Y = Ahat Omega into b.Y.
// It depends only on A, the Philox stream and the number of new samples.
template <typename T>
int sketch_stage(frsvt_context *h, const Core<T> &c, CoreBuffers<T> &b)
{
    const Orient &o = c.o;
    const int mh = o.mh;
    if (c.cnew <= 0) return FRSVT_OK;
    LongArgs<T> la{};
    la.A = c.A;
    la.lda = c.lda;
    la.trans = o.trans ? 1 : 0;
    la.mh = mh;
    la.nh = o.nh;
    la.seed = c.seed;
    la.counter = c.counter;
    la.c = c.cnew;
    la.Ypart = b.Ypart;
    LongPlan p = long_plan(mh, o.nh, c.cnew, Prec<T>::bytes, kSketch, h->num_cu, o.trans);
    CKT(FRSVT_K_SKETCH, launch_long<T>(p, kSketch, la, h->stream));
    CKT(FRSVT_K_REDUCE, launch_reduce<T>(b.Ypart, (int64_t)mh * c.cnew, p.grid, b.Y, h->stream));
    return FRSVT_OK;
}

template <typename T>
bool core_small(const Core<T> &c, int l)
{
    return long_path_ok(c.o.mh, l) && small_orth_ok(c.o.mh, l);
}

template <typename T>
int run_core(frsvt_context *h, Core<T> &c, CoreBuffers<T> &b)
{
    const Orient &o = c.o;
    const int mh = o.mh;
    const int l = c.rp + c.cnew;
    c.l = l;
    c.Q = b.Q;
    c.Bt = b.Bt;
    c.QM = b.QM;
    c.G = b.G;
    c.U = b.U;
    c.Mm = b.Mm;
    c.sigma = b.sigma;
    const bool small = !c.A16 && long_path_ok(mh, l) && small_orth_ok(mh, l);
    int *oflags = c.status + 4;
    hipStream_t s = h->stream;
    int rc;

    LongArgs<T> la{};
    la.A = c.A;
    la.lda = c.lda;
    la.trans = o.trans ? 1 : 0;
    la.mh = mh;
    la.nh = o.nh;
    la.seed = c.seed;
    la.counter = c.counter;

    // Alg. 1, sketch and initial basis (fresh or range-propagated)
    if (small) {
        if (!c.sketch_ready && (rc = sketch_stage<T>(h, c, b))) return rc;
        if (!c.orth_ready)
            CKT(FRSVT_K_ORTH, launch_small_orth<T>(mh, c.Qt, c.ldqt, c.rp, c.ysrc ? c.ysrc : b.Y, mh, c.cnew, b.Q,
                                                   mh, c.seed, c.counter, oflags, c.resid_out, s));
    } else {
        if (c.rp > 0)
            CK(hipMemcpy2DAsync(b.Q, mh * sizeof(T), c.Qt, c.ldqt * sizeof(T), mh * sizeof(T),
                                c.rp, hipMemcpyDeviceToDevice, s));
        if (c.cnew > 0) {
            if (c.A16) {
                CKT(FRSVT_K_OTHER, launch_omega_bf16(o.nh, c.cnew, c.seed, c.counter, b.V16, o.nh, s));
                if ((rc = ahat_times<T>(h, c, (const T *)b.V16, o.nh, c.cnew, b.Q + (size_t)c.rp * mh,
                                        b.gpart_t, nullptr, true)))
                    return rc;
            } else {
                CKT(FRSVT_K_OTHER, launch_omega<T>(o.nh, c.cnew, c.seed, c.counter, b.Om, o.nh, s));
                if ((rc = ahat_times<T>(h, c, b.Om, o.nh, c.cnew, b.Q + (size_t)c.rp * mh, b.gpart_t)))
                    return rc;
            }
        }
        if (c.resid_out) CKT(FRSVT_K_ORTH, launch_resid_est<T>(mh, b.Q, mh, c.rp, c.cnew, c.resid_out, s));
        if ((rc = big_orth<T>(h, mh, l, b.Q, mh, b, c.seed, c.counter, oflags))) return rc;
    }

    // Alg. 1, power iterations Q = QR(Ahat Ahat^T Q)
    for (int it = 0; it < c.q; ++it) {
        const uint64_t ctr2 = c.counter ^ (0x5bd1e995ull << 32) ^ (uint64_t)(it + 1) << 56;
        if (small) {
            LongPlan p = long_plan(mh, o.nh, l, Prec<T>::bytes, kPower, h->num_cu, o.trans);
            la.c = l;
            la.Q = b.Q;
            la.ldq = mh;
            la.Ypart = b.Ypart;
            CKT(FRSVT_K_POWER, launch_long<T>(p, kPower, la, s));
            CKT(FRSVT_K_REDUCE, launch_reduce<T>(b.Ypart, (int64_t)mh * l, p.grid, b.Y, s));
            CKT(FRSVT_K_ORTH, launch_small_orth<T>(mh, (const T *)nullptr, mh, 0, b.Y, mh, l, b.Q, mh, c.seed,
                                    ctr2, oflags, (double *)nullptr, s));
        } else {
            if ((rc = ahat_t_times<T>(h, c, b.Q, mh, l, b.Z, b.gpart_t, true, b.V16))) return rc;
            if ((rc = ahat_times<T>(h, c, b.Z, o.nh, l, b.Q, b.gpart_t, b.V16))) return rc;
            if ((rc = big_orth<T>(h, mh, l, b.Q, mh, b, c.seed, ctr2, oflags))) return rc;
        }
    }

    // Alg. 1, QR of A^T Q: B^T = Ahat^T Q and its Gram B B^T
    if (small || (!c.A16 && long_path_ok(mh, l))) {
        LongPlan p = long_plan(mh, o.nh, l, Prec<T>::bytes, kProject, h->num_cu, o.trans);
        la.c = l;
        la.Q = b.Q;
        la.ldq = mh;
        la.Z = b.Bt;
        la.ldz = o.nh;
        la.Gpart = b.Gpart;
        if (c.om) {
            la.om = c.om;
            la.om_c = c.om_c;
            la.om_counter = c.om_counter;
        }
        CKT(FRSVT_K_PROJECT, launch_long<T>(p, kProject, la, s));
        c.om_drawn = c.om != nullptr;
        CKT(FRSVT_K_REDUCE, launch_reduce<double>(b.Gpart, (int64_t)l * l, p.grid, b.G, s));
    } else {
        if ((rc = ahat_t_times<T>(h, c, b.Q, mh, l, b.Bt, b.gpart_t))) return rc;
        if ((rc = gram<T>(h, o.nh, l, b.Bt, o.nh, b.G, b.gpart_d))) return rc;
    }

    // Alg. 1, polar/eigen and reconstruction: small SVD, thresholds, factors
    SmallSvdOut so{b.sigma, b.U, b.Mm, c.status};
    const int fuse = small_svd_fuse_q_ok(mh, l) ? 1 : 0;
    CKT(FRSVT_K_SMALL_SVD, launch_small_svd<T>(l, b.G, c.tau, c.w, c.keep, b.Q, mh, mh, b.QM, mh, c.Qout, c.ldqo, so, b.jwork,
                           fuse, s));
    if (!fuse) {
        // QM = Q Mm, Qout = Q U (double small factors cast through a copy)
        T *Mt = b.Qtmp;  // reuse: l x l in storage precision needs l*l <= mh*l
        CKT(FRSVT_K_OTHER, launch_cast<T>(l, l, b.Mm, 1, l, Mt, l, s));
        if ((rc = mm<T>(h, mh, l, l, b.Q, 1, mh, Mt, 1, l, b.QM, 1, mh, 1, b.gpart_t))) return rc;
        if (c.Qout) {
            CKT(FRSVT_K_OTHER, launch_cast<T>(l, l, b.U, 1, l, Mt, l, s));
            if ((rc = mm<T>(h, mh, l, l, b.Q, 1, mh, Mt, 1, l, c.Qout, 1, c.ldqo, 1, b.gpart_t)))
                return rc;
        }
    }
    return FRSVT_OK;
}

// X (physical m x n, ldx) = (QM) B.
template <typename T>
int write_x(frsvt_context *h, const Core<T> &c, T *X, int64_t ldx, T *part)
{
    const Orient &o = c.o;
    if (recon_ok(c.l)) {
        ReconArgs<T> ra{};
        ra.c = c.l;
        if (o.trans) {
            ra.rows = o.nh;
            ra.cols = o.mh;
            ra.FR = c.Bt;
            ra.ldfr = o.nh;
            ra.FC = c.QM;
            ra.ldfc = o.mh;
        } else {
            ra.rows = o.mh;
            ra.cols = o.nh;
            ra.FR = c.QM;
            ra.ldfr = o.mh;
            ra.FC = c.Bt;
            ra.ldfc = o.nh;
        }
        ra.X = X;
        ra.ldx = ldx;
        CKT(FRSVT_K_RECON, launch_recon<T>(kRecon, ra, nullptr, h->stream));
    } else {
        const int64_t scm = o.trans ? ldx : 1, scn = o.trans ? 1 : ldx;
        int rc = mm<T>(h, o.mh, o.nh, c.l, c.QM, 1, o.mh, c.Bt, o.nh, 1, X, scm, scn, 1, part);
        if (rc) return rc;
    }
    return FRSVT_OK;
}

// Exact SVT / WSVT: G = Ahat Ahat^T, small SVD of size mh, X = Mm Ahat.
template <typename T>
int exact_factors(frsvt_context *h, const T *A, int64_t lda, const Orient &o, double tau,
                  const double *w, Carver &cv, double **Mm_out, T **Mt_out, int keep = 0)
{
    const int mh = o.mh;
    const int sk = gemm_splitk(mh, mh, o.nh, h->num_cu);
    double *G = cv.take<double>((size_t)mh * mh);
    double *gp = cv.take<double>((size_t)sk * mh * mh);
    double *U = cv.take<double>((size_t)mh * mh);
    double *Mm = cv.take<double>((size_t)mh * mh);
    double *sig = cv.take<double>((size_t)mh);
    double *jw = cv.take<double>((size_t)mh * mh);
    T *Mt = cv.take<T>((size_t)mh * mh);
    if (!cv.base) return FRSVT_OK;
    if (std::is_same<T, double>::value) {
        // on the matrix cores (each operand has a unit stride)
        CKT(FRSVT_K_GEMM, launch_gemm_f64_mfma(mh, mh, o.nh, (const double *)A, o.si, o.sk, (const double *)A,
                                               o.sk, o.si, G, 1, mh, sk, gp, h->stream));
    } else {
        CKT(FRSVT_K_GEMM, (launch_gemm<float, double, double>(mh, mh, o.nh, (const float *)A, o.si, o.sk,
                                               (const float *)A, o.sk, o.si, G, 1, mh, sk, gp,
                                               h->stream)));
    }
    SmallSvdOut so{sig, U, Mm, h->dstatus};
    CKT(FRSVT_K_SMALL_SVD, launch_small_svd<T>(mh, G, tau, w, keep, (const T *)nullptr, 0, mh, (T *)nullptr, 0,
                           (T *)nullptr, 0, so, jw, 0, h->stream));
    CKT(FRSVT_K_OTHER, launch_cast<T>(mh, mh, Mm, 1, mh, Mt, mh, h->stream));
    *Mm_out = Mm;
    *Mt_out = Mt;
    return FRSVT_OK;
}

template <typename T>
int exact_svt_impl(frsvt_context *h, int64_t m, int64_t n, const T *A, int64_t lda, double tau,
                   const double *w, T *X, int64_t ldx, int32_t *rank)
{
    const Orient o = orient(m, n, lda);
    Carver dry(nullptr);
    double *Mm;
    T *Mt;
    exact_factors<T>(h, A, lda, o, tau, w, dry, &Mm, &Mt);
    int rc = ensure_ws(h, dry.off);
    if (rc) return rc;
    Carver cv(h->ws);
    if ((rc = exact_factors<T>(h, A, lda, o, tau, w, cv, &Mm, &Mt))) return rc;
    const int64_t scm = o.trans ? ldx : 1, scn = o.trans ? 1 : ldx;
    CKT(FRSVT_K_GEMM, (launch_gemm<T, T, T>(o.mh, o.nh, o.mh, Mt, 1, o.mh, A, o.si, o.sk, X, scm, scn, 1,
                             (T *)nullptr, h->stream)));
    if (rank) {
        CK(hipMemcpyAsync(h->pinned, h->dstatus, 4 * sizeof(int), hipMemcpyDeviceToHost, h->stream));
        CK(hipStreamSynchronize(h->stream));
        *rank = ((int *)h->pinned)[0];
        if (((int *)h->pinned)[2] == 0) return FRSVT_NOT_CONVERGED;
    }
    return FRSVT_OK;
}

template <typename T>
int frsvt_impl(frsvt_context *h, int64_t m, int64_t n, const T *A, int64_t lda, double tau,
               int k, int p, int q, const T *Qprev, int r_prev, int64_t ldqp, uint64_t seed,
               uint64_t counter, T *X, int64_t ldx, T *Qout, int64_t ldqo, int32_t *r_out,
               bool mixed = false, T *Qsave = nullptr, int64_t ldqs = 0, double *factors = nullptr,
               const FixedWs *fixed = nullptr)
{
    const Orient o = orient(m, n, lda);
    Core<T> c{};
    c.A = A;
    c.lda = lda;
    c.o = o;
    c.tau = tau;
    c.w = nullptr;
    c.q = q;
    c.seed = seed;
    c.counter = counter;
    if (Qprev && r_prev > 0) {
        c.Qt = Qprev;
        c.ldqt = ldqp;
        c.rp = std::min(r_prev, o.mh);
        c.cnew = std::max(0, std::min(p, o.mh - c.rp));
    } else {
        c.Qt = nullptr;
        c.ldqt = o.mh;
        c.rp = 0;
        c.cnew = std::max(1, std::min(k + p, o.mh));
    }
    c.Qout = Qout;
    c.ldqo = ldqo;
    c.status = h->dstatus;
    const int l = c.rp + c.cnew;
    CoreBuffers<T> b{};
    Carver dry(nullptr);
    if (mixed) {
        dry.take<uint16_t>((size_t)m * n);
        dry.take<uint16_t>((size_t)m * n);
    }
    carve_core<T>(dry, o, l, c.cnew, h->num_cu, b, mixed);
    int rc;
    void *base;
    if (fixed) {
        if (!fixed->base) {
            snprintf(h->last_error, sizeof(h->last_error), "device address of the fixed scratch unavailable");
            return FRSVT_ERR_HIP;
        }
        if (dry.off > fixed->cap) {
            snprintf(h->last_error, sizeof(h->last_error),
                     "frsvt_noalloc: this call needs %zu bytes of scratch, the fixed scratch holds %zu",
                     dry.off, fixed->cap);
            return FRSVT_ERR_SCRATCH;
        }
        base = fixed->base;
    } else {
        if ((rc = ensure_ws(h, dry.off))) return rc;
        base = h->ws;
    }
    Carver cv(base);
    c.A16 = c.A16T = nullptr;
    if (mixed) {
        // both orientations, so that every bfloat16 product reads its
        // operand along the reduction index
        uint16_t *A16 = cv.take<uint16_t>((size_t)m * n);
        uint16_t *A16T = cv.take<uint16_t>((size_t)m * n);
        CKT(FRSVT_K_OTHER, launch_to_bf16_pair(m, n, (const float *)A, lda, A16, A16T, h->stream));
        c.A16 = A16;
        c.A16T = A16T;
    }
    carve_core<T>(cv, o, l, c.cnew, h->num_cu, b, mixed);
    // Alg. 1's QR_CP of a fresh sketch (Sec. 2.1: s = min(l, r)): the
    // numerically null samples are dropped before the power iterations
    int s_used = l;
    if (h->opt_truncate && c.rp == 0 && c.cnew > 1 && !mixed && !Qsave && !factors &&
        core_small<T>(c, c.cnew) && qrcp_trunc_ok(o.mh, c.cnew)) {
        if ((rc = sketch_stage<T>(h, c, b))) return rc;
        CKT(FRSVT_K_ORTH, launch_qrcp_trunc<T>(o.mh, c.cnew, b.Y, o.mh, (double)o.mh * 2.220446049250313e-16,
                                               b.Qtmp, o.mh, h->dstatus + 3, h->stream));
        CK(hipMemcpyAsync(h->pinned, h->dstatus + 3, sizeof(int), hipMemcpyDeviceToHost, h->stream));
        CK(hipStreamSynchronize(h->stream));
        s_used = std::max(1, ((const int *)h->pinned)[0]);
        c.cnew = s_used;
        c.sketch_ready = true;
        c.ysrc = b.Qtmp;
    }
    if ((rc = run_core<T>(h, c, b))) return rc;
    CKT(FRSVT_K_OTHER, launch_fill_int(h->dstatus + 3, 1, s_used, h->stream));
    if (Qsave)
        CK(hipMemcpy2DAsync(Qsave, ldqs * sizeof(T), b.Q, o.mh * sizeof(T), o.mh * sizeof(T), l,
                            hipMemcpyDeviceToDevice, h->stream));
    if (factors) {
        CK(hipMemcpyAsync(factors, b.sigma, l * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
        CK(hipMemcpyAsync(factors + l, b.U, (size_t)l * l * sizeof(double), hipMemcpyDeviceToDevice,
                          h->stream));
    }
    if ((rc = write_x<T>(h, c, X, ldx, b.gpart_t))) return rc;
    if (r_out) {
        CK(hipMemcpyAsync(h->pinned, h->dstatus, 8 * sizeof(int), hipMemcpyDeviceToHost, h->stream));
        CK(hipStreamSynchronize(h->stream));
        *r_out = ((int *)h->pinned)[0];
        if (((int *)h->pinned)[6] != 0) {
            snprintf(h->last_error, sizeof(h->last_error),
                     "the last orthonormalisation's Cholesky factor failed after the shifted fallback and refill");
            return FRSVT_ERR_CHOLESKY;
        }
        if (((int *)h->pinned)[2] == 0) return FRSVT_NOT_CONVERGED;
    }
    return FRSVT_OK;
}

// ---------------------------------------------------------------------------
// Adjoint of the fresh-sketch FRSVT map X = Q S_tau(Q^T Ahat) of Alg. 1
// (fresh sketch, power iterations, projection, thresholding) for a fixed
// Omega.  The power iterations are recomputed from the seed, Q_q is the
// saved basis of the projection step and (sigma,
// U_B) the saved small factors.  With the blocks
//   Lf = [Q_q, Ybar_q, Q_{q-1}, ..., Ybar_1, Q_0, Ybar_0]   (mh x (2q+2) l)
//   Rf = [Bbar^T, Z_q, Zbar_q, ..., Z_1, Zbar_1, Omega]     (nh x (2q+2) l)
// the gradient is Abar_hat = Lf Rf^T, written in one product.
// ---------------------------------------------------------------------------
template <typename T>
int cross_gram(frsvt_context *h, int64_t rows, int l1, int l2, const T *X, int64_t ldx,
               const T *Y, int64_t ldy, double *G, double *part)
{
    const int sk = gemm_splitk(l1, l2, rows, h->num_cu);
    CKT(FRSVT_K_ADJOINT, (launch_gemm<T, double, double>(l1, l2, rows, X, ldx, 1, Y, 1, ldy, G, 1, l1,
                                                         sk, part, h->stream)));
    return FRSVT_OK;
}

// out = X1 C1 + X2 C2 (C = nullptr: identity), rows x l.
template <typename T>
int combine2(frsvt_context *h, int64_t rows, int l, const T *X1, int64_t ld1, const double *C1,
             const T *X2, int64_t ld2, const double *C2, T *out, int64_t ldout)
{
    CombineArgs<T> a{};
    a.rows = rows;
    a.c = l;
    a.nin = X2 ? 2 : 1;
    a.in[0] = X1;
    a.ldin[0] = ld1;
    a.w[0] = l;
    a.coef[0] = C1;
    if (X2) {
        a.in[1] = X2;
        a.ldin[1] = ld2;
        a.w[1] = l;
        a.coef[1] = C2;
    }
    a.out = out;
    a.ldout = ldout;
    CKT(FRSVT_K_ADJOINT, launch_combine<T>(a, h->stream));
    return FRSVT_OK;
}

template <typename T>
struct VjpBuffers {
    T *Lf, *Rf, *BC, *Ct, *Qb, *P, *Yt, *gpart_t;
    double *R, *H, *M1, *M2, *Kd, *CA, *CB, *gpart_d;
    CoreBuffers<T> ob;  // orthonormalisation scratch of the large path
};

template <typename T>
size_t carve_vjp(Carver &cv, int mh, int64_t nh, int l, int q, VjpBuffers<T> &b)
{
    const size_t K = (size_t)(2 * q + 2) * l;
    const size_t ll = (size_t)l * l;
    b.Lf = cv.take<T>((size_t)mh * K);
    b.Rf = cv.take<T>((size_t)nh * K);
    b.BC = cv.take<T>((size_t)nh * 2 * l);
    b.Ct = cv.take<T>((size_t)nh * l);
    b.Qb = cv.take<T>((size_t)mh * l);
    b.P = cv.take<T>((size_t)mh * 2 * l);
    b.Yt = cv.take<T>((size_t)mh * l);
    b.gpart_t = cv.take<T>((size_t)128 * mh * l);
    b.R = cv.take<double>((size_t)(q + 1) * ll);
    b.H = cv.take<double>(ll);
    b.M1 = cv.take<double>(ll);
    b.M2 = cv.take<double>(ll);
    b.Kd = cv.take<double>(ll);
    b.CA = cv.take<double>(ll);
    b.CB = cv.take<double>(ll);
    b.gpart_d = cv.take<double>((size_t)128 * ll);
    b.ob = CoreBuffers<T>{};
    b.ob.G = cv.take<double>(ll);
    b.ob.R = cv.take<double>(ll);
    b.ob.nullc = cv.take<int>((size_t)l);
    b.ob.gpart_d = b.gpart_d;
    return cv.off;
}

// Q = orth(Y) into Qdst (Y is kept): the one-workgroup CholeskyQR when it
// fits, else the large-path sequence on a copy.
template <typename T>
int orth_copy(frsvt_context *h, int mh, int l, const T *Y, T *Qdst, VjpBuffers<T> &b,
              uint64_t seed, uint64_t counter, int *flags)
{
    if (small_orth_ok(mh, l)) {
        CKT(FRSVT_K_ORTH, launch_small_orth<T>(mh, (const T *)nullptr, mh, 0, Y, mh, l, Qdst, mh, seed,
                                               counter, flags, (double *)nullptr, h->stream));
        return FRSVT_OK;
    }
    CK(hipMemcpyAsync(Qdst, Y, (size_t)mh * l * sizeof(T), hipMemcpyDeviceToDevice, h->stream));
    return big_orth<T>(h, mh, l, Qdst, mh, b.ob, seed, counter, flags);
}

template <typename T>
int frsvt_vjp_impl(frsvt_context *h, int64_t m, int64_t n, const T *A, int64_t lda, double tau,
                   int l, int q, uint64_t seed, uint64_t counter, const T *Qs, int64_t ldqs,
                   const double *factors, const T *Xb, int64_t ldxb, T *Ab, int64_t ldab,
                   double *tau_bar)
{
    const Orient o = orient(m, n, lda);
    const int mh = o.mh;
    const int64_t nh = o.nh;
    hipStream_t s = h->stream;
    VjpBuffers<T> b{};
    Carver dry(nullptr);
    carve_vjp<T>(dry, mh, nh, l, q, b);
    int rc = ensure_ws(h, dry.off);
    if (rc) return rc;
    Carver cv(h->ws);
    carve_vjp<T>(cv, mh, nh, l, q, b);

    Core<T> ca{};
    ca.A = A;
    ca.lda = lda;
    ca.o = o;
    Core<T> cx{};
    cx.A = Xb;
    cx.lda = ldxb;
    cx.o = orient(m, n, ldxb);
    auto Lb = [&](int j) { return b.Lf + (size_t)j * mh * l; };
    auto Rb = [&](int j) { return b.Rf + (size_t)j * nh * l; };
    auto Qi = [&](int i) { return i == q ? Lb(0) : Lb(2 * (q - i)); };
    auto Zi = [&](int i) { return Rb(2 * (q - i) + 1); };
    auto Zbar = [&](int i) { return Rb(2 * (q - i) + 2); };
    auto Ybar = [&](int i) { return i > 0 ? Lb(2 * (q - i) + 1) : Lb(2 * q + 1); };
    int *flags = h->dstatus + 4;
    CKT(FRSVT_K_OTHER, launch_fill_int(h->dstatus + 4, 4, 0, s));

    // forward recomputation: Omega, Y_0 = Ahat Omega, Q_i, Z_i = Ahat^T Q_{i-1},
    // Y_i = Ahat Z_i, R_i = Q_i^T Y_i
    CK(hipMemcpy2DAsync(Lb(0), mh * sizeof(T), Qs, ldqs * sizeof(T), mh * sizeof(T), l,
                        hipMemcpyDeviceToDevice, s));
    CKT(FRSVT_K_OTHER, launch_omega<T>(nh, l, seed, counter, Rb(2 * q + 1), nh, s));
    if ((rc = ahat_times<T>(h, ca, Rb(2 * q + 1), nh, l, b.Yt, b.gpart_t))) return rc;
    for (int i = 0; i <= q; ++i) {
        if (i > 0) {
            if ((rc = ahat_t_times<T>(h, ca, Qi(i - 1), mh, l, Zi(i), b.gpart_t))) return rc;
            if ((rc = ahat_times<T>(h, ca, Zi(i), nh, l, b.Yt, b.gpart_t))) return rc;
        }
        if (i < q && (rc = orth_copy<T>(h, mh, l, b.Yt, Qi(i), b, seed, counter, flags))) return rc;
        if ((rc = cross_gram<T>(h, mh, l, l, Qi(i), mh, b.Yt, mh, b.R + (size_t)i * l * l, b.gpart_d)))
            return rc;
    }

    // the projection again: B^T = Ahat^T Q; Sbar^T = Xbar_hat^T Q; H = Sbar B^T
    T *Bt = b.BC, *Sbt = b.BC + (size_t)nh * l;
    if ((rc = ahat_t_times<T>(h, ca, Lb(0), mh, l, Bt, b.gpart_t))) return rc;
    if ((rc = ahat_t_times<T>(h, cx, Lb(0), mh, l, Sbt, b.gpart_t))) return rc;
    if ((rc = cross_gram<T>(h, nh, l, l, Sbt, nh, Bt, nh, b.H, b.gpart_d))) return rc;
    CKT(FRSVT_K_ADJOINT, launch_svt_vjp_small(l, factors, factors + l, b.H, tau, b.M1, b.M2, tau_bar, s));
    // Bbar^T = B^T M1 + Sbar^T M2 (Rf block 0); C^T = B^T M2, the SVT of B
    if ((rc = combine2<T>(h, nh, l, Bt, nh, b.M1, Sbt, nh, b.M2, Rb(0), nh))) return rc;
    if ((rc = combine2<T>(h, nh, l, Bt, nh, b.M2, (const T *)nullptr, 0, nullptr, b.Ct, nh))) return rc;
    // Qbar_q = Xbar_hat C^T + Ahat Bbar^T
    T *P1 = b.P, *P2 = b.P + (size_t)mh * l;
    if ((rc = ahat_times<T>(h, cx, b.Ct, nh, l, P1, b.gpart_t))) return rc;
    if ((rc = ahat_times<T>(h, ca, Rb(0), nh, l, P2, b.gpart_t))) return rc;
    if ((rc = combine2<T>(h, mh, l, P1, mh, nullptr, P2, mh, nullptr, b.Qb, mh))) return rc;

    // back through the QR steps and the power iterations
    for (int i = q; i >= 0; --i) {
        if ((rc = cross_gram<T>(h, mh, l, l, b.Qb, mh, Qi(i), mh, b.Kd, b.gpart_d))) return rc;
        CKT(FRSVT_K_ADJOINT, launch_qr_vjp_small(l, b.Kd, b.R + (size_t)i * l * l, b.CA, b.CB,
                                                 h->dstatus + 7, s));
        if ((rc = combine2<T>(h, mh, l, b.Qb, mh, b.CA, Qi(i), mh, b.CB, Ybar(i), mh))) return rc;
        if (i > 0) {
            if ((rc = ahat_t_times<T>(h, ca, Ybar(i), mh, l, Zbar(i), b.gpart_t))) return rc;
            if ((rc = ahat_times<T>(h, ca, Zbar(i), nh, l, b.Qb, b.gpart_t))) return rc;
        }
    }

    const int K = (2 * q + 2) * l;
    const int64_t scm = o.trans ? ldab : 1, scn = o.trans ? 1 : ldab;
    return mm<T>(h, mh, nh, K, b.Lf, 1, mh, b.Rf, nh, 1, Ab, scm, scn, 1, (T *)nullptr);
}

// ---------------------------------------------------------------------------
// Unrolled inexact-ALM pieces: the step after the thresholding, its reverse,
// and the starting point.
// ---------------------------------------------------------------------------
template <typename T>
int dual_step_impl(frsvt_context *h, int64_t m, int64_t n, const T *O, int64_t ldo, const T *L,
                   int64_t ldl, const T *Y, int64_t ldy, double lam, double mu, double mu_next,
                   T *S, int64_t lds, T *Yn, int64_t ldyn, T *An, int64_t ldan)
{
    DualStepArgs<T> a{};
    a.m = m;
    a.n = n;
    a.O = O;
    a.ldo = ldo;
    a.L = L;
    a.ldl = ldl;
    a.Y = Y;
    a.ldy = ldy;
    a.lam = lam;
    a.mu = mu;
    a.mu_next = mu_next;
    a.S = S;
    a.lds = lds;
    a.Yn = Yn;
    a.ldyn = ldyn;
    a.An = An;
    a.ldan = ldan;
    CKT(FRSVT_K_EPILOGUE, launch_dual_step<T>(a, false, nullptr, h->stream));
    return FRSVT_OK;
}

template <typename T>
int dual_step_vjp_impl(frsvt_context *h, int64_t m, int64_t n, const T *O, int64_t ldo,
                       const T *L, int64_t ldl, const T *Y, int64_t ldy, double lam, double mu,
                       double mu_next, const T *Sb, int64_t ldsb, const T *Ynb, int64_t ldynb,
                       const T *Anb, int64_t ldanb, T *Lb, int64_t ldlb, T *Yb, int64_t ldyb,
                       double *lam_bar)
{
    int rc = ensure_ws(h, (size_t)kDualGrid * sizeof(double) + 256);
    if (rc) return rc;
    DualStepArgs<T> a{};
    a.m = m;
    a.n = n;
    a.O = O;
    a.ldo = ldo;
    a.L = L;
    a.ldl = ldl;
    a.Y = Y;
    a.ldy = ldy;
    a.lam = lam;
    a.mu = mu;
    a.mu_next = mu_next;
    a.Sb = Sb;
    a.ldsb = ldsb;
    a.Ynb = Ynb;
    a.ldynb = ldynb;
    a.Anb = Anb;
    a.ldanb = ldanb;
    a.Lb = Lb;
    a.ldlb = ldlb;
    a.Yb = Yb;
    a.ldyb = ldyb;
    a.part = (double *)h->ws;
    int np = 0;
    CKT(FRSVT_K_ADJOINT, launch_dual_step<T>(a, true, &np, h->stream));
    if (lam_bar) CKT(FRSVT_K_REDUCE, launch_reduce<double>(a.part, 1, np, lam_bar, h->stream));
    return FRSVT_OK;
}

// ||O||_F and ||O||_inf (host; waits), FRSVT_ERR_NONFINITE on NaN or Inf.
template <typename T>
int input_norms(frsvt_context *h, int64_t m, int64_t n, const T *O, int64_t ldo, double *normF,
                double *mx)
{
    hipStream_t s = h->stream;
    CKT(FRSVT_K_OTHER, launch_fill_int(h->dstatus + 16, 1, 0, s));
    int nparts = 0;
    CKT(FRSVT_K_OTHER, launch_norms<T>(m, n, O, ldo, h->dscalars + 16, &nparts, s, h->dstatus + 16));
    CK(hipMemcpyAsync(h->pinned, h->dstatus + 16, sizeof(int), hipMemcpyDeviceToHost, s));
    CK(hipMemcpyAsync((char *)h->pinned + 64, h->dscalars + 16, 2 * nparts * sizeof(double),
                      hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    if (((int *)h->pinned)[0]) return FRSVT_ERR_NONFINITE;
    double ss = 0.0, mxv = 0.0;
    const double *np = (const double *)((char *)h->pinned + 64);
    for (int g = 0; g < nparts; ++g) {
        ss += np[2 * g];
        mxv = std::max(mxv, np[2 * g + 1]);
    }
    *normF = std::sqrt(ss);
    *mx = mxv;
    return FRSVT_OK;
}

template <typename T>
int spectral_norm(frsvt_context *h, const T *A, int64_t lda, const Orient &o, double *out);

template <typename T>
int rpca_init_impl(frsvt_context *h, int64_t m, int64_t n, const T *O, int64_t ldo, double lambda,
                   double mu0, T *Y0, int64_t ldy, T *A0, int64_t lda0, double *out)
{
    double normF = 0.0, mx = 0.0, norm2 = 0.0;
    int rc = input_norms<T>(h, m, n, O, ldo, &normF, &mx);
    if (rc) return rc;
    if ((rc = spectral_norm<T>(h, O, ldo, orient(m, n, ldo), &norm2))) return rc;
    const double J = std::max(norm2, mx / lambda);
    const double mu = mu0 > 0.0 ? mu0 : (norm2 > 0.0 ? 1.25 / norm2 : 1.0);
    CKT(FRSVT_K_OTHER, launch_rpca_init<T>(m, n, O, ldo, J > 0.0 ? 1.0 / J : 0.0, 1.0 / mu, Y0, ldy, A0,
                                           lda0, h->stream));
    if (out) {
        out[0] = norm2;
        out[1] = mu;
        out[2] = J;
    }
    return FRSVT_OK;
}

// ---------------------------------------------------------------------------
// Inexact-ALM RPCA.
// ---------------------------------------------------------------------------
template <typename T>
int spectral_norm(frsvt_context *h, const T *A, int64_t lda, const Orient &o, double *out)
{
    // ||A||_2^2 = lambda_1(G), G = Ahat Ahat^T (mhat x mhat, FP64): block
    // subspace iteration with Rayleigh-Ritz; where it cannot certify its
    // estimate (more than eight top eigenvalues within a few per cent, or
    // mhat < 8) the full small SVD of G (Cholesky + one-sided Jacobi)
    const int mh = o.mh;
    const int sk = gemm_splitk(mh, mh, o.nh, h->num_cu);
    // the transposed orientation with mh <= 256 takes the dedicated Gram
    // kernel (one pass over A, upper blocks only)
    const bool gtr = o.trans && gram_tr_ok(mh, o.nh, lda, (int)sizeof(T));
    const size_t gpn = gtr ? gram_tr_part_doubles(mh, h->num_cu) + gram_tr_part_doubles(mh, 1)
                           : (size_t)sk * mh * mh;
    // (beyond mh = 1024: block power vectors and their small factors instead
    // of the small SVD's buffers)
    constexpr int kB = 16;
    const bool large = mh > 1024;
    const size_t svn = large ? (size_t)mh * kB * 2 + (size_t)64 * kB * kB + 4 * kB * kB + 512
                             : (size_t)mh * mh * 3 + mh;
    Carver dry(nullptr);
    dry.take<double>((size_t)mh * mh);
    dry.take<double>(gpn);
    dry.take<double>(svn);
    int rc = ensure_ws(h, dry.off);
    if (rc) return rc;
    Carver cv(h->ws);
    double *G = cv.take<double>((size_t)mh * mh);
    double *gp = cv.take<double>(gpn);
    double *sv = cv.take<double>(svn);
    if (gtr) {
        CKT(FRSVT_K_GEMM, launch_gram_tr<T>(A, lda, mh, o.nh, h->num_cu, gp,
                                            gp + gram_tr_part_doubles(mh, h->num_cu), G, h->stream));
    } else if (std::is_same<T, double>::value) {
        // on the matrix cores (each operand has a unit stride)
        CKT(FRSVT_K_GEMM, launch_gemm_f64_mfma(mh, mh, o.nh, (const double *)A, o.si, o.sk, (const double *)A,
                                               o.sk, o.si, G, 1, mh, sk, gp, h->stream));
    } else {
        CKT(FRSVT_K_GEMM, (launch_gemm<float, double, double>(mh, mh, o.nh, (const float *)A, o.si, o.sk,
                                               (const float *)A, o.sk, o.si, G, 1, mh, sk, gp,
                                               h->stream)));
    }
    if (large) {
        // beyond the one-workgroup eigen kernels: block power iteration on G
        // (16 vectors, 40 products, each block re-orthonormalised by
        // CholeskyQR), then the top Ritz value of V^T G V.  Its relative
        // error decays as (lambda_17 / lambda_1)^80; the RPCA host uses the
        // value only for its starting point (mu_0 and the dual scaling J).
        constexpr int kSteps = 40;
        double *V = sv, *W = V + (size_t)mh * kB, *pt = W + (size_t)mh * kB;
        double *H = pt + (size_t)64 * kB * kB, *R = H + kB * kB, *Ud = R + kB * kB, *Mmd = Ud + kB * kB;
        double *dv = Mmd + kB * kB, *sg = dv + 256;
        CKT(FRSVT_K_OTHER, launch_omega<double>(mh, kB, 0x5eed5eedull, 0x0c0ffee0ull, V, mh, h->stream));
        for (int t = 0; t < kSteps; ++t) {
            if ((rc = mm<double>(h, mh, kB, mh, G, 1, mh, V, 1, mh, W, 1, mh, 1, nullptr))) return rc;
            if ((rc = gram<double>(h, mh, kB, W, mh, H, pt))) return rc;
            CKT(FRSVT_K_ORTH, launch_col_scale<double>(mh, kB, W, mh, H, h->stream));
            if ((rc = gram<double>(h, mh, kB, W, mh, H, pt))) return rc;
            CKT(FRSVT_K_ORTH, launch_chol(kB, H, 0.0, 1e-14, R, nullptr, nullptr, h->stream, nullptr, nullptr, 0.0, dv));
            CKT(FRSVT_K_ORTH, launch_trsm<double>(mh, kB, W, mh, R, h->stream, dv));
            std::swap(V, W);
        }
        // H = V^T (G V)
        if ((rc = mm<double>(h, mh, kB, mh, G, 1, mh, V, 1, mh, W, 1, mh, 1, nullptr))) return rc;
        if ((rc = mm<double>(h, kB, kB, mh, V, mh, 1, W, 1, mh, H, 1, kB, 1, nullptr))) return rc;
        SmallSvdOut so{sg, Ud, Mmd, h->dstatus};
        CKT(FRSVT_K_SMALL_SVD, launch_small_svd<double>(kB, H, 0.0, nullptr, 0, (const double *)nullptr, 0, kB,
                                                        (double *)nullptr, 0, (double *)nullptr, 0, so, nullptr, 0,
                                                        h->stream));
        CK(hipMemcpyAsync(h->pinned, sg, sizeof(double), hipMemcpyDeviceToHost, h->stream));
        CK(hipStreamSynchronize(h->stream));
        // the small SVD takes H as a Gram: its singular values are sqrt(eig H)
        const double s1 = ((double *)h->pinned)[0];
        *out = s1 > 0.0 ? s1 : 0.0;
        return FRSVT_OK;
    }
    double lam = 0.0;
    bool ok = false;
    if (mh <= 256) {
        // a dominant top eigenvalue is certified by a few single-vector steps
        CKT(FRSVT_K_OTHER, launch_power_dom(mh, G, h->dscalars, h->stream));
        CK(hipMemcpyAsync(h->pinned, h->dscalars, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        CK(hipStreamSynchronize(h->stream));
        lam = ((double *)h->pinned)[0];
        ok = ((double *)h->pinned)[1] > 0.5;
    }
    if (!ok && mh >= 8) {
        CKT(FRSVT_K_OTHER, launch_power_eig(mh, G, h->dscalars, h->stream));
        CK(hipMemcpyAsync(h->pinned, h->dscalars, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        CK(hipStreamSynchronize(h->stream));
        lam = ((double *)h->pinned)[0];
        ok = ((double *)h->pinned)[1] > 0.5;
    }
    if (!ok) {
        double *sig = sv, *U = sv + mh, *Mm = U + (size_t)mh * mh, *jw = Mm + (size_t)mh * mh;
        SmallSvdOut so{sig, U, Mm, h->dstatus};
        CKT(FRSVT_K_SMALL_SVD, launch_small_svd<T>(mh, G, 0.0, nullptr, 0, (const T *)nullptr, 0, mh, (T *)nullptr,
                                                   0, (T *)nullptr, 0, so, jw, 0, h->stream));
        CK(hipMemcpyAsync(h->pinned, sig, sizeof(double), hipMemcpyDeviceToHost, h->stream));
        CK(hipStreamSynchronize(h->stream));
        const double s1 = ((double *)h->pinned)[0];
        *out = s1 > 0.0 ? s1 : 0.0;
        return FRSVT_OK;
    }
    *out = std::sqrt(std::max(0.0, lam));
    return FRSVT_OK;
}

// Int word of the mapped host block that carries an RPCA iteration's
// sequence number (after the status words 0-7, the residual sum 8-9 and the
// residual estimate 10-11).
constexpr int kIterSeqWord = 16;

// Waits for the last kernel of an RPCA iteration to have written its status
// words to mapped host memory: polls the sequence number it writes after
// them (an event on the stream would hold the next kernel back by a few
// microseconds), querying the stream now and then so that an error on it
// ends the wait.
int wait_iter_words(frsvt_context *h, hipStream_t s, volatile int *word, int seq)
{
    for (unsigned spin = 1;; ++spin) {
        if (*word == seq) {
            std::atomic_thread_fence(std::memory_order_acquire);
            return FRSVT_OK;
        }
        if ((spin & 65535u) == 0) {
            const hipError_t e = hipStreamQuery(s);
            if (e == hipSuccess) {
                // the stream has drained: the word is there or never comes
                std::atomic_thread_fence(std::memory_order_acquire);
                if (*word == seq) return FRSVT_OK;
                snprintf(h->last_error, sizeof(h->last_error),
                         "the RPCA iteration's status words did not reach mapped host memory");
                return FRSVT_ERR_HIP;
            }
            if (e != hipErrorNotReady) return fail(h, e, "hipStreamQuery (RPCA iteration)");
        }
        __builtin_ia32_pause();
    }
}

template <typename T>
int rpca_impl(frsvt_context *h, int64_t m, int64_t n, const T *O, int64_t ldo, double lambda,
              const frsvt_rpca_opts &op, T *L, int64_t ldl, T *S, int64_t lds,
              frsvt_rpca_stats *stats)
{
    const Orient o = orient(m, n, ldo);
    const int mh = o.mh;
    hipStream_t s = h->stream;
    int rc;

    double normF = 0.0, mx = 0.0;
    if ((rc = input_norms<T>(h, m, n, O, ldo, &normF, &mx))) return rc;
    double norm2 = 0.0;
    if ((rc = spectral_norm<T>(h, O, ldo, o, &norm2))) return rc;
    if (!(normF > 0.0) || !(norm2 > 0.0)) {
        // O = 0: L = S = 0
        CK(hipMemset2DAsync(L, ldl * sizeof(T), 0, m * sizeof(T), n, s));
        CK(hipMemset2DAsync(S, lds * sizeof(T), 0, m * sizeof(T), n, s));
        CK(hipStreamSynchronize(s));
        if (stats) {
            memset(stats, 0, sizeof(*stats));
            stats->converged = 1;
        }
        return FRSVT_OK;
    }
    const double J = std::max(norm2, mx / lambda);
    double mu = op.mu0 > 0.0 ? op.mu0 : 1.25 / norm2;
    const double mu_bar = mu * op.mu_bar_factor;
    // widest sketch: b = ceil(gamma mhat) under adaptive prediction, else mhat
    const int bmax = op.ap ? std::max(1, std::min(mh, (int)std::ceil(op.ap_gamma * mh))) : mh;
    const int l0 = op.l0 > 0 ? std::min(op.l0, bmax) : std::max(1, std::min(bmax, (int)std::ceil(0.1 * bmax)));

    // workspace: A, the FRSVT core at its largest width, exact factors, z partials
    // (the large path's orthonormalisation takes at most 256 columns)
    const int lmax = op.use_frsvt ? std::min(mh, 256) : mh;
    // residual partials: one per epilogue workgroup (256 x 16 elements)
    const size_t zcap = (size_t)((m + 255) / 256) * (size_t)((n + 15) / 16);
    // Omega's rows for the sketch fused into the epilogue (FP64, Ahat = A^T,
    // at most eight new samples): drawn one iteration ahead
    const int csk_fixed = std::min(op.ap ? op.ap_a : op.p, mh);
    const bool om_rows = op.use_frsvt && std::is_same<T, double>::value && o.trans && csk_fixed >= 1 && csk_fixed <= 8;
    auto layout = [&](Carver &cv, T **A, CoreBuffers<T> &b, T **Qt, double **zp, T **Lx,
                      double **zsum, double **om) {
        *A = cv.take<T>((size_t)m * n);
        *Qt = cv.take<T>((size_t)mh * mh);
        *zp = cv.take<double>(zcap);
        *zsum = cv.take<double>(4);
        *Lx = cv.take<T>((size_t)m * n);
        *om = om_rows ? cv.take<double>((size_t)o.nh * 8) : nullptr;
        if (op.use_frsvt) carve_core<T>(cv, o, lmax, lmax, h->num_cu, b);
        return cv.off;
    };
    T *A, *Qt, *Lx;
    double *zp, *zsum, *om;
    CoreBuffers<T> b{};
    Carver dry(nullptr);
    size_t need = layout(dry, &A, b, &Qt, &zp, &Lx, &zsum, &om);
    size_t exact_need = 0;
    if (!op.use_frsvt) {
        Carver d2(nullptr);
        d2.off = need;
        double *Mm;
        T *Mt;
        exact_factors<T>(h, O, ldo, o, 0.0, nullptr, d2, &Mm, &Mt);
        exact_need = d2.off;
    }
    if ((rc = ensure_ws(h, std::max(need, exact_need)))) return rc;
    Carver cv(h->ws);
    layout(cv, &A, b, &Qt, &zp, &Lx, &zsum, &om);
    const size_t exact_off = cv.off;


    T *Ybuf[2] = {L, S};
    const int64_t ldyb[2] = {ldl, lds};
    CKT(FRSVT_K_OTHER, launch_rpca_init<T>(m, n, O, ldo, 1.0 / J, 1.0 / mu, Ybuf[0], ldyb[0], A, m, s));

    auto t0 = std::chrono::steady_clock::now();
    int r_prev = -1, l_prev = 0;
    int spec_cnew = 0;
    // the next iteration's orthonormalisation enqueued before this
    // iteration's rank is read, for the rank of the previous one (-1: none)
    int spec_orth_rp = -1, spec_orth_cnew = 0;
    // semi-online: the caller's basis is the first call's propagated basis
    if (op.use_frsvt && op.r_init > 0) {
        if (op.r_init > mh) return -8;
        CK(hipMemcpy2DAsync(Qt, mh * sizeof(T), op.q_init, mh * sizeof(T), mh * sizeof(T), op.r_init,
                            hipMemcpyDeviceToDevice, s));
        r_prev = op.r_init;
        l_prev = op.r_init;
    }
    int it = 0;
    bool converged = false;
    double resid = 0.0, mu_last = mu;
    Core<T> c{};
    if (!h->host_iter) {
        CK(hipHostMalloc(&h->host_iter, 256, hipHostMallocCoherent | hipHostMallocMapped));
        CK(hipHostGetDevicePointer(&h->host_iter_dev, h->host_iter, 0));
    }
    volatile int *hst = (volatile int *)h->host_iter;
    for (it = 0; it < op.max_iter; ++it) {
        const double mu_next = std::min(op.rho * mu, mu_bar);
        const T *Yc = Ybuf[it & 1];
        T *Yn = Ybuf[(it + 1) & 1];
        ReconArgs<T> ra{};
        if (op.use_frsvt) {
            c = Core<T>{};
            c.A = A;
            c.lda = m;
            c.o = orient(m, n, m);
            c.tau = 1.0 / mu;
            c.keep = op.keep;
            c.w = nullptr;
            c.q = op.q;
            c.seed = op.seed;
            c.counter = (uint64_t)it;
            // new samples: p beside the propagated columns, or under
            // adaptive prediction (Eq. 7) l_{i+1} - r_i with
            // l_{i+1} = min(r_i + (r_i < l_i ? a : ceil(rho mhat)), b)
            auto ap_width = [&](int r, int lw) {
                const int pn = r < lw ? op.ap_a : (int)std::ceil(op.ap_rho * (double)mh);
                return std::min(r + pn, bmax);
            };
            if (r_prev > 0) {
                c.Qt = Qt;
                c.ldqt = mh;
                c.rp = r_prev;
                c.cnew = op.ap ? ap_width(r_prev, l_prev) - r_prev : std::max(0, std::min(op.p, mh - r_prev));
            } else {
                c.Qt = nullptr;
                c.ldqt = mh;
                c.rp = 0;
                c.cnew = r_prev < 0 ? l0 : (op.ap ? ap_width(0, l_prev) : std::min(op.p, mh));
            }
            // widths stay within the 256 columns the large path's
            // orthonormalisation takes: fewer new samples beside a wide
            // propagated basis (r_prev <= the previous width <= 256)
            if (c.rp + c.cnew > lmax) c.cnew = std::max(0, lmax - c.rp);
            // Sec. 3.2: the planned samples in order, sampling stopped at
            // the first whose residual estimate is at most 1/mu
            bool checked = false;
            if (op.resid_check && c.cnew > 0) {
                if (!core_small<T>(c, c.rp + c.cnew) || !resid_seq_ok(mh, c.rp, c.cnew) || c.cnew > 64) {
                    snprintf(h->last_error, sizeof(h->last_error),
                             "the residual check runs on the one-workgroup path only (short side %d, width %d)",
                             mh, c.rp + c.cnew);
                    CK(hipStreamSynchronize(s));
                    return FRSVT_ERR_UNSUPPORTED;
                }
                if (spec_cnew < c.cnew && (rc = sketch_stage<T>(h, c, b))) return rc;
                double *est2 = h->dscalars + kCheckSlot;
                CKT(FRSVT_K_ORTH, launch_resid_seq<T>(mh, c.Qt, c.ldqt, c.rp, b.Y, mh, c.cnew, est2, s));
                CK(hipMemcpyAsync(h->pinned, est2, (size_t)c.cnew * sizeof(double), hipMemcpyDeviceToHost, s));
                CK(hipStreamSynchronize(s));
                const double tau_it = 1.0 / mu;
                int kept = c.cnew;
                for (int j = 0; j < c.cnew; ++j) {
                    const double est = 20.0 * std::sqrt(2.0 / 3.14159265358979323846) *
                                       std::sqrt(((const double *)h->pinned)[j]);
                    if (est <= tau_it) {
                        kept = j + 1;
                        break;
                    }
                }
                c.cnew = kept;
                checked = true;
            }
            l_prev = std::min(mh, c.rp + c.cnew);
            if (stats && it < 64) stats->widths[it] = l_prev;
            // (the first c.cnew columns of a wider draw are the narrower draw)
            c.sketch_ready = checked || (spec_cnew > 0 && spec_cnew == c.cnew && core_small<T>(c, c.rp + c.cnew));
            c.orth_ready = !checked && c.sketch_ready && spec_orth_rp > 0 && spec_orth_rp == c.rp &&
                           spec_orth_cnew == c.cnew;
            c.Qout = Qt;
            c.ldqo = mh;
            c.status = h->dstatus;
            c.resid_out = reinterpret_cast<double *>(h->dstatus + kResidSlot);
            // the next epilogue's sketch rows (iteration it + 1), drawn by
            // this iteration's projection pass
            if (om && it + 1 < op.max_iter) {
                c.om = om;
                c.om_c = csk_fixed;
                c.om_counter = (uint64_t)(it + 1);
            }
            if ((rc = run_core<T>(h, c, b))) return rc;
            ra.c = c.l;
            if (o.trans) {
                ra.FR = c.Bt;
                ra.ldfr = o.nh;
                ra.FC = c.QM;
                ra.ldfc = o.mh;
            } else {
                ra.FR = c.QM;
                ra.ldfr = o.mh;
                ra.FC = c.Bt;
                ra.ldfc = o.nh;
            }
            if (!recon_ok(c.l)) {
                // wide basis: materialise L = (QM) B, then the epilogue reads it
                const int64_t scm = o.trans ? m : 1, scn = o.trans ? 1 : m;
                if ((rc = mm<T>(h, o.mh, o.nh, c.l, c.QM, 1, o.mh, c.Bt, o.nh, 1, Lx, scm, scn, 1, (T *)nullptr)))
                    return rc;
                ra.c = 0;
                ra.Lin = Lx;
                ra.ldlin = m;
            }
        } else {
            Carver ce(h->ws);
            ce.off = exact_off;
            double *Mm;
            T *Mt;
            if ((rc = exact_factors<T>(h, A, m, orient(m, n, m), 1.0 / mu, nullptr, ce, &Mm, &Mt, op.keep)))
                return rc;
            const Orient oa = orient(m, n, m);
            const int64_t scm = oa.trans ? m : 1, scn = oa.trans ? 1 : m;
            CKT(FRSVT_K_GEMM, (launch_gemm<T, T, T>(oa.mh, oa.nh, oa.mh, Mt, 1, oa.mh, A, oa.si, oa.sk, Lx, scm,
                                     scn, 1, (T *)nullptr, s)));
            ra.c = 0;
            ra.Lin = Lx;
            ra.ldlin = m;
        }
        ra.rows = m;
        ra.cols = n;
        ra.O = O;
        ra.ldo = ldo;
        ra.Y = Yc;
        ra.ldy = ldyb[it & 1];
        ra.Ynext = Yn;
        ra.ldyn = ldyb[(it + 1) & 1];
        ra.Anext = A;
        ra.ldan = m;
        ra.mu = mu;
        ra.mu_next = mu_next;
        ra.lam = lambda;
        ra.zpart = zp;
        // The next sketch needs only the next A and its Philox counter, with
        // p new samples (the width of every later sketch unless r + p > mh).
        // Where the rows of A are the long index, the epilogue forms it from
        // the values of A it writes (partials per row block); otherwise it
        // is a pass of its own below.
        Core<T> cn = c;
        cn.counter = (uint64_t)(it + 1);
        // (under adaptive prediction the width of the common case, r < l)
        cn.cnew = std::min(op.ap ? op.ap_a : op.p, mh);
        const bool next_sketch = op.use_frsvt && it + 1 < op.max_iter && cn.cnew > 0 && long_path_ok(mh, cn.cnew);
        const int64_t rblocks = recon_row_blocks(m);
        const bool fuse_sketch = next_sketch && std::is_same<T, double>::value && o.trans && cn.cnew <= 8 &&
                                 (size_t)rblocks * (size_t)n * (size_t)cn.cnew <= b.ypart_cap;
        if (fuse_sketch) {
            ra.ysk = b.Ypart;
            ra.csk = cn.cnew;
            ra.seed = cn.seed;
            ra.counter = cn.counter;
            if (om && c.om_drawn && cn.cnew == csk_fixed) ra.om = om;
        }
        int nz = 0;
        CKT(FRSVT_K_EPILOGUE, launch_recon<T>(kEpi, ra, &nz, s));
        // status words (rank, residual) written by the last kernel straight
        // to mapped host memory, then a sequence number; the host polls that
        // word only, so the GPU keeps working on the speculative sketch below
        // while the host reads them and enqueues the next iteration.
        int *hdev = (int *)h->host_iter_dev;
        const int seq = h->iter_seq = (h->iter_seq % 0x3fffffff) + 1;
        CKT(FRSVT_K_REDUCE, launch_finish_iter(zp, nz, h->dstatus, 8, hdev, (double *)(hdev + 8),
                                               op.use_frsvt ? reinterpret_cast<const double *>(h->dstatus + kResidSlot)
                                                            : nullptr,
                                               (double *)(hdev + 10), s, hdev + kIterSeqWord, seq));
        // the next sketch is completed (or run) before the host waits for
        // this iteration's rank
        spec_cnew = 0;
        if (fuse_sketch) {
            CKT(FRSVT_K_REDUCE, launch_reduce<T>(b.Ypart, (int64_t)mh * cn.cnew, (int)rblocks, b.Y, s));
            spec_cnew = cn.cnew;
        } else if (next_sketch) {
            if ((rc = sketch_stage<T>(h, cn, b))) return rc;
            spec_cnew = cn.cnew;
        }
        // and, for the rank of this iteration's own propagated basis (the
        // common case once the rank has settled), the next iteration's
        // orthonormalisation of [Qt, Y]; it is used only if the rank read
        // below matches (b.Q is free: this iteration is done with it)
        spec_orth_rp = -1;
        if (spec_cnew > 0 && !op.ap && !op.resid_check && r_prev > 0 &&
            spec_cnew == std::max(0, std::min(op.p, mh - r_prev))) {
            Core<T> cs = c;
            cs.rp = r_prev;
            cs.cnew = spec_cnew;
            if (core_small<T>(cs, r_prev + spec_cnew)) {
                CKT(FRSVT_K_ORTH, launch_small_orth<T>(mh, Qt, mh, r_prev, b.Y, mh, spec_cnew, b.Q, mh, op.seed,
                                                       (uint64_t)(it + 1), h->dstatus + 4,
                                                       reinterpret_cast<double *>(h->dstatus + kResidSlot), s));
                spec_orth_rp = r_prev;
                spec_orth_cnew = spec_cnew;
            }
        }

        if ((rc = wait_iter_words(h, s, hst + kIterSeqWord, seq))) return rc;
        const int r = hst[0];
        if (op.use_frsvt && hst[6] != 0) {
            snprintf(h->last_error, sizeof(h->last_error),
                     "iteration %d: the orthonormalisation's Cholesky factor failed after the shifted fallback", it);
            CK(hipStreamSynchronize(s));
            return FRSVT_ERR_CHOLESKY;
        }
        double zz;
        const int zw[2] = {hst[8], hst[9]};
        memcpy(&zz, zw, sizeof(double));
        (void)zsum;
        if (stats && it < 64 && op.use_frsvt) {
            // Prop. 4 with Lemma 3 (alpha = 20): an upper bound on
            // sigma_{r+1} of this iteration's A with probability >= 0.95
            const int rw[2] = {hst[10], hst[11]};
            double r2;
            memcpy(&r2, rw, sizeof(double));
            stats->resid_est[it] = r2 < 0.0 ? -1.0 : 20.0 * std::sqrt(2.0 / 3.14159265358979323846) * std::sqrt(r2);
        }
        resid = std::sqrt(zz) / normF;
        if (stats && it < 64) {
            stats->ranks[it] = r;
            stats->residuals[it] = resid;
        }
        r_prev = r;
        mu_last = mu;
        mu = mu_next;
        if (resid < op.tol) {
            converged = true;
            ++it;
            break;
        }
    }
    // the last propagated basis to the caller (semi-online use)
    if (op.use_frsvt && op.q_final && r_prev > 0)
        CK(hipMemcpy2DAsync(op.q_final, mh * sizeof(T), Qt, mh * sizeof(T), mh * sizeof(T), r_prev,
                            hipMemcpyDeviceToDevice, s));
    // L and S of the last iteration, from its factors and multiplier
    {
        const int last = it - 1;
        ReconArgs<T> ra{};
        if (op.use_frsvt && recon_ok(c.l)) {
            ra.c = c.l;
            if (o.trans) {
                ra.FR = c.Bt;
                ra.ldfr = o.nh;
                ra.FC = c.QM;
                ra.ldfc = o.mh;
            } else {
                ra.FR = c.QM;
                ra.ldfr = o.mh;
                ra.FC = c.Bt;
                ra.ldfc = o.nh;
            }
        } else {
            ra.c = 0;
            ra.Lin = Lx;
            ra.ldlin = m;
        }
        ra.rows = m;
        ra.cols = n;
        ra.O = O;
        ra.ldo = ldo;
        ra.Y = Ybuf[last & 1];
        ra.ldy = ldyb[last & 1];
        ra.X = L;
        ra.ldx = ldl;
        ra.S = S;
        ra.lds = lds;
        ra.mu = mu_last;
        ra.mu_next = mu_last;
        ra.lam = lambda;
        CKT(FRSVT_K_OTHER, launch_recon<T>(kFinal, ra, nullptr, s));
        CK(hipStreamSynchronize(s));
    }
    auto t1 = std::chrono::steady_clock::now();
    if (stats) {
        stats->iters = it;
        stats->converged = converged ? 1 : 0;
        stats->residual = resid;
        stats->norm2 = norm2;
        stats->seconds = std::chrono::duration<double>(t1 - t0).count();
    }
    return converged ? FRSVT_OK : FRSVT_MAX_ITER;
}

bool bad_ptr(const void *p) { return p == nullptr; }

// ---------------------------------------------------------------------------
// Batched weighted SVT: longest-first order, per-bucket autotuning of the
// Jacobi group size, one persistent launch captured in a HIP graph.
// ---------------------------------------------------------------------------
int wb_buffers(frsvt_context *h, int64_t count)
{
    if (!h->wb_queue) {
        hipError_t e = hipMalloc(&h->wb_queue, 256);
        if (e == hipSuccess) e = hipMalloc(&h->wb_gs_dev, 256);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->wb_capture, hipStreamNonBlocking);
        if (e != hipSuccess) return fail(h, e, "wsvt_batched buffers");
    }
    if (count > h->wb_order_cap) {
        if (h->wb_order) {
            (void)hipStreamSynchronize(h->stream);
            (void)hipFree(h->wb_order);
            h->wb_order = nullptr;
        }
        hipError_t e = hipMalloc(&h->wb_order, (size_t)count * sizeof(int32_t));
        if (e != hipSuccess) return fail(h, e, "wsvt_batched order");
        h->wb_order_cap = count;
    }
    return FRSVT_OK;
}

int wb_launch(frsvt_context *h, const WsvtBatchArgs &a, hipStream_t s)
{
    const int grid = 2 * h->num_cu;  // two persistent workgroups per compute unit
    CKT(FRSVT_K_WSVT_BATCHED, launch_wsvt_batched(a, grid, s));
    return FRSVT_OK;
}

int wsvt_batched_impl(frsvt_context *h, int64_t count, const int32_t *rows, const int32_t *cols,
                      const int64_t *offsets, const float *A, float *X,
                      const frsvt_wsvt_rule &rule, int32_t *ranks)
{
    int rc = wb_buffers(h, count);
    if (rc) return rc;
    std::vector<uint64_t> key = {(uint64_t)count, (uint64_t)(uintptr_t)rows, (uint64_t)(uintptr_t)cols,
                                 (uint64_t)(uintptr_t)offsets, (uint64_t)(uintptr_t)A,
                                 (uint64_t)(uintptr_t)X, (uint64_t)(uintptr_t)ranks};
    uint64_t bits[4];
    memcpy(bits, &rule, sizeof(bits));
    for (uint64_t b : bits) key.push_back(b);
    // the kernel checks every shape it reads and flags one outside the
    // bounds (the replay reads the shapes anew): the flag is read back after
    // every launch
    auto shape_flag = [&]() -> int {
        CK(hipMemcpyAsync(h->pinned, h->wb_queue + 1, sizeof(int), hipMemcpyDeviceToHost, h->stream));
        CK(hipStreamSynchronize(h->stream));
        if (((const int *)h->pinned)[0] != 0) {
            snprintf(h->last_error, sizeof(h->last_error),
                     "wsvt_batched: a matrix shape outside 1..128 (shorter side <= 96) was skipped "
                     "(shapes changed after the first call?); its rank is -1");
            return FRSVT_ERR_UNSUPPORTED;
        }
        return FRSVT_OK;
    };
    if (h->wb_exec && key == h->wb_key && !h->tracing) {
        CK(hipGraphLaunch(h->wb_exec, h->stream));
        return shape_flag();
    }
    // shapes to the host once per argument set: longest-first order and tuning
    std::vector<int32_t> hr(count), hc(count);
    CK(hipMemcpyAsync(hr.data(), rows, count * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    CK(hipMemcpyAsync(hc.data(), cols, count * sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    CK(hipStreamSynchronize(h->stream));
    for (int64_t j = 0; j < count; ++j) {
        if (hr[j] < 1 || hc[j] < 1 || hr[j] > 128 || hc[j] > 128 || std::min(hr[j], hc[j]) > 96)
            return FRSVT_ERR_UNSUPPORTED;
    }
    auto cost = [&](int64_t j) {
        const double s = std::min(hr[j], hc[j]), L = std::max(hr[j], hc[j]);
        return s * s * (L + 8.0 * s);
    };
    std::vector<int32_t> order(count);
    for (int64_t j = 0; j < count; ++j) order[j] = (int32_t)j;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return cost(x) > cost(y); });
    CK(hipMemcpyAsync(h->wb_order, order.data(), count * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));

    WsvtBatchArgs a{};
    a.count = count;
    a.rows = rows;
    a.cols = cols;
    a.offsets = offsets;
    a.A = A;
    a.X = X;
    a.c = rule.c;
    a.noise_var = rule.noise_var;
    a.eps = rule.eps;
    a.tau = rule.tau;
    a.ranks = ranks;
    a.sweeps = nullptr;
    a.order = h->wb_order;
    a.queue = h->wb_queue;
    a.work = reinterpret_cast<unsigned long long *>(h->wb_queue + 16);
    a.group_size = h->wb_gs_dev;

    if (!h->wb_tuned) {
        // Autotuner: for each size bucket with enough members, time the kernel
        // on (up to) 256 of its matrices with 8, 16 and 32 lanes per Jacobi
        // pair and keep the fastest.
        const int cand[3] = {8, 16, 32};
        for (int b = 0; b < 3; ++b) h->wb_gs[b] = 16;
        std::vector<int32_t> sample;
        hipEvent_t e0, e1;
        CK(hipEventCreate(&e0));
        CK(hipEventCreate(&e1));
        for (int b = 0; b < 3; ++b) {
            sample.clear();
            for (int64_t j = 0; j < count && (int64_t)sample.size() < 256; ++j) {
                const int s = std::min(hr[j], hc[j]);
                const int bb = s <= 48 ? 0 : (s <= 64 ? 1 : 2);
                if (bb == b) sample.push_back((int32_t)j);
            }
            if (sample.size() < 32) continue;
            CK(hipMemcpyAsync(h->wb_order, sample.data(), sample.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, h->stream));
            float best = 1e30f;
            for (int ci = 0; ci < 3; ++ci) {
                int32_t gs3[3] = {cand[ci], cand[ci], cand[ci]};
                CK(hipMemcpyAsync(h->wb_gs_dev, gs3, sizeof(gs3), hipMemcpyHostToDevice, h->stream));
                WsvtBatchArgs t = a;
                t.count = (int64_t)sample.size();
                t.ranks = nullptr;
                float ms = 0.0f, tot = 0.0f;
                for (int rep = 0; rep < 2; ++rep) {
                    CK(hipEventRecord(e0, h->stream));
                    if ((rc = wb_launch(h, t, h->stream))) return rc;
                    CK(hipEventRecord(e1, h->stream));
                    CK(hipEventSynchronize(e1));
                    CK(hipEventElapsedTime(&ms, e0, e1));
                    if (rep) tot += ms;
                }
                if (tot < best) {
                    best = tot;
                    h->wb_gs[b] = cand[ci];
                }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        h->wb_tuned = true;
        CK(hipMemcpyAsync(h->wb_order, order.data(), count * sizeof(int32_t), hipMemcpyHostToDevice,
                          h->stream));
    }
    int32_t gs3[3] = {h->wb_gs[0], h->wb_gs[1], h->wb_gs[2]};
    CK(hipMemcpyAsync(h->wb_gs_dev, gs3, sizeof(gs3), hipMemcpyHostToDevice, h->stream));
    CK(hipStreamSynchronize(h->stream));
    if (h->tracing) {
        if ((rc = wb_launch(h, a, h->stream))) return rc;
        return shape_flag();
    }
    // capture the persistent launch (queue reset kernel + kernel) once
    if (h->wb_exec) {
        (void)hipGraphExecDestroy(h->wb_exec);
        h->wb_exec = nullptr;
    }
    hipGraph_t graph = nullptr;
    CK(hipStreamBeginCapture(h->wb_capture, hipStreamCaptureModeThreadLocal));
    CK(launch_wsvt_batched(a, 2 * h->num_cu, h->wb_capture));
    CK(hipStreamEndCapture(h->wb_capture, &graph));
    hipError_t e = hipGraphInstantiate(&h->wb_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        h->wb_exec = nullptr;
        return fail(h, e, "hipGraphInstantiate");
    }
    h->wb_key = key;
    CK(hipGraphLaunch(h->wb_exec, h->stream));
    return shape_flag();
}



// ---------------------------------------------------------------------------
// Low-rank representation (Type A of Table 6) by its inexact ALM; the steps
// are listed with the lrr_ialm declaration.  The iteration state lives in
// one allocation of its own (the FRSVT calls of the J step grow and may move
// the handle's workspace).
// ---------------------------------------------------------------------------
struct DevBlock {
    void *p = nullptr;
    ~DevBlock()
    {
        if (p) (void)hipFree(p);
    }
};

int lrr_impl(frsvt_context *h, int64_t d, int64_t n, const double *X, int64_t ldx, double lambda,
             const frsvt_lrr_opts &op, double *Z, int64_t ldz, double *E, int64_t lde, frsvt_lrr_stats *stats)
{
    hipStream_t s = h->stream;
    if (stats) memset(stats, 0, sizeof(*stats));
    const int num_cu = h->num_cu;
    // split-K partials large enough for every product below
    const int sk1 = gemm_splitk(n, n, d, num_cu), sk2 = gemm_splitk(n, n, n, num_cu);
    const int sk3 = gemm_splitk(d, n, n, num_cu);
    const size_t part = std::max({(size_t)sk1 * n * n, (size_t)sk2 * n * n, (size_t)sk3 * d * n});
    const size_t nn = (size_t)n * n, dn = (size_t)d * n;
    const int np = lrr_dual_parts();
    const size_t total = 8 * nn + 3 * dn + part + 2 * (size_t)np + 8;
    DevBlock blk;
    CK(hipMalloc(&blk.p, total * sizeof(double)));
    double *J = (double *)blk.p, *Y2 = J + nn, *T = Y2 + nn, *R = T + nn, *Minv = R + nn;
    double *P1 = Minv + nn, *P2 = P1 + nn, *Qt = P2 + nn;
    double *Y1 = Qt + nn, *W = Y1 + dn, *XZ = W + dn, *gp = XZ + dn, *mparts = gp + part;
    double *dres = mparts + 2 * (size_t)np;
    auto gemm = [&](int64_t M, int64_t N, int64_t K, const double *A, int64_t sam, int64_t sak, const double *B,
                    int64_t sbk, int64_t sbn, double *C, int64_t ldc) -> int {
        const int sk = gemm_splitk(M, N, K, num_cu);
        CKT(FRSVT_K_GEMM, launch_gemm_f64_mfma(M, N, K, A, sam, sak, B, sbk, sbn, C, 1, ldc, sk, gp, s));
        return FRSVT_OK;
    };
    int rc;
    // state: Z = J = E = Y1 = Y2 = 0
    CK(launch_lrr_comb(n, n, 0, nullptr, 0, 0, nullptr, 0, 0, nullptr, 0, 0.0, Z, ldz, s));
    CK(launch_lrr_comb(d, n, 0, nullptr, 0, 0, nullptr, 0, 0, nullptr, 0, 0.0, E, lde, s));
    CK(launch_lrr_comb(n, n, 0, nullptr, 0, 0, nullptr, 0, 0, nullptr, 0, 0.0, Y2, n, s));
    CK(launch_lrr_comb(d, n, 0, nullptr, 0, 0, nullptr, 0, 0, nullptr, 0, 0.0, Y1, d, s));
    // (I + X^T X)^{-1} by Newton-Schulz: M <- 2 M - M (A M) from M = I / ||A||_inf;
    // the error I - A M squares each step from below 1 - 1 / ||A||_inf
    if ((rc = gemm(n, n, d, X, ldx, 1, X, 1, ldx, T, n))) return rc;
    CK(launch_lrr_comb(n, n, 1.0, T, n, 0, nullptr, 0, 0, nullptr, 0, 1.0, T, n, s));
    CK(launch_lrr_norm_inf(n, T, n, dres, s));
    double ninf = 1.0;
    CK(hipMemcpyAsync(&ninf, dres, sizeof(double), hipMemcpyDeviceToHost, s));
    CK(hipStreamSynchronize(s));
    if (!(ninf >= 1.0) || !std::isfinite(ninf)) return FRSVT_ERR_NONFINITE;
    // steps until (1 - 1/ninf)^(2^k) < 2^-60, plus two
    const int ns_steps = std::min(80, (int)std::ceil(std::log2(60.0 * std::log(2.0) * ninf + 1.0)) + 2);
    CK(launch_lrr_comb(n, n, 0, nullptr, 0, 0, nullptr, 0, 0, nullptr, 0, 1.0 / ninf, Minv, n, s));
    for (int k = 0; k < ns_steps; ++k) {
        if ((rc = gemm(n, n, n, T, 1, n, Minv, 1, n, P1, n))) return rc;       // A M
        if ((rc = gemm(n, n, n, Minv, 1, n, P1, 1, n, P2, n))) return rc;      // M A M
        CK(launch_lrr_comb(n, n, 2.0, Minv, n, -1.0, P2, n, 0, nullptr, 0, 0.0, Minv, n, s));
    }
    const int l0 = std::max(1, (int)std::ceil(0.1 * (double)n));
    int r_prev = -1, r = 0;
    double mu = op.mu0, primal = 0.0, dual = 0.0;
    bool converged = false;
    int it;
    const auto t0 = std::chrono::steady_clock::now();
    for (it = 0; it < op.max_iter; ++it) {
        // J = SVT_{1/mu}(Z + Y2/mu)
        CK(launch_lrr_comb(n, n, 1.0, Z, ldz, 1.0 / mu, Y2, n, 0, nullptr, 0, 0.0, T, n, s));
        int32_t rr = 0;
        if (op.use_frsvt) {
            const bool prop = r_prev > 0;
            const int kk = r_prev < 0 ? l0 : 0, pp = r_prev < 0 ? 0 : op.p;
            if ((rc = frsvt_impl<double>(h, n, n, T, n, 1.0 / mu, kk, pp, op.q, prop ? Qt : nullptr,
                                         prop ? r_prev : 0, n, op.seed, (uint64_t)it, J, n, Qt, n, &rr)))
                return rc;
            r_prev = rr;
        } else {
            if ((rc = exact_svt_impl<double>(h, n, n, T, n, 1.0 / mu, nullptr, J, n, &rr))) return rc;
        }
        r = rr;
        // Z = (I + X^T X)^{-1} (X^T (X - E + Y1/mu) + J - Y2/mu)
        CK(launch_lrr_comb(d, n, 1.0, X, ldx, -1.0, E, lde, 1.0 / mu, Y1, d, 0.0, W, d, s));
        if ((rc = gemm(n, n, d, X, ldx, 1, W, 1, d, R, n))) return rc;
        CK(launch_lrr_comb(n, n, 1.0, R, n, 1.0, J, n, -1.0 / mu, Y2, n, 0.0, R, n, s));
        if ((rc = gemm(n, n, n, Minv, 1, n, R, 1, n, Z, ldz))) return rc;
        // E = column shrink_{lambda/mu}(X - X Z + Y1/mu)
        if ((rc = gemm(d, n, n, X, 1, ldx, Z, 1, ldz, XZ, d))) return rc;
        CK(launch_lrr_colshrink(d, n, X, ldx, XZ, Y1, 1.0 / mu, lambda / mu, E, lde, s));
        // multipliers and the max-norm residuals
        CK(launch_lrr_dual(d, n, mu, X, ldx, XZ, d, E, lde, Y1, mparts, s));
        CK(launch_lrr_dual(n, n, mu, Z, ldz, J, n, nullptr, 0, Y2, mparts + np, s));
        CK(launch_lrr_max_parts(mparts, np, 2, dres, s));
        double res[2];
        CK(hipMemcpyAsync(res, dres, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        primal = res[0];
        dual = res[1];
        mu = std::min(op.rho * mu, op.mu_max);
        if (primal < op.tol && dual < op.tol) {
            converged = true;
            ++it;
            break;
        }
    }
    if (stats) {
        stats->iters = it;
        stats->converged = converged ? 1 : 0;
        stats->rank = r;
        stats->primal = primal;
        stats->dual = dual;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    CK(hipStreamSynchronize(s));
    return converged ? FRSVT_OK : FRSVT_MAX_ITER;
}


// 3-way tensor host: O (I1 x I2 x I3, column-major) = L + E with the
// weighted sum of the unfoldings' nuclear norms and lambda ||E||_1, by an
// inexact ALM over one copy L_i of L per mode (each with its own constraint
// O = L_i + E and multiplier Y_i).  Mode 1's unfolding is O itself (ld I1),
// mode 3's is the transpose of the (I1 I2) x I3 view (the SVT commutes with
// the transpose and the sketch sees the same short-by-long matrix), mode 2's
// lives in a permuted buffer.
int tensor_impl(frsvt_context *h, int64_t I1, int64_t I2, int64_t I3, const double *O, const double *alpha,
                double lambda, const frsvt_tensor_opts &op, double *L, double *E, frsvt_tensor_stats *stats)
{
    hipStream_t s = h->stream;
    if (stats) memset(stats, 0, sizeof(*stats));
    const int64_t N = I1 * I2 * I3;
    const int64_t vm[3] = {I1, I2, I1 * I2}, vn[3] = {I2 * I3, I1 * I3, I3};
    int64_t mh[3];
    for (int i = 0; i < 3; ++i) mh[i] = std::min(vm[i], vn[i]);
    double normF = 0.0, mx = 0.0, norm2 = 0.0;
    int rc = input_norms<double>(h, I1, I2 * I3, O, I1, &normF, &mx);
    if (rc) return rc;
    if (!(normF > 0.0)) {
        // O = 0: the minimiser is L = E = 0
        CK(launch_lrr_comb(N, 1, 0, nullptr, 0, 0, nullptr, 0, 0, nullptr, 0, 0.0, L, N, s));
        CK(launch_lrr_comb(N, 1, 0, nullptr, 0, 0, nullptr, 0, 0, nullptr, 0, 0.0, E, N, s));
        CK(hipStreamSynchronize(s));
        if (stats) stats->converged = 1;
        return FRSVT_OK;
    }
    double mu = op.mu0;
    if (!(mu > 0.0)) {
        if ((rc = spectral_norm<double>(h, O, I1, orient(I1, I2 * I3, I1), &norm2))) return rc;
        mu = 1.25 / norm2;
    }
    const double mu0 = mu;
    const int np = ten_parts();
    const size_t total = 8 * (size_t)N + (size_t)(mh[0] * mh[0] + mh[1] * mh[1] + mh[2] * mh[2]) + 3 * (size_t)np + 4;
    DevBlock blk;
    CK(hipMalloc(&blk.p, total * sizeof(double)));
    double *L2p = (double *)blk.p, *L3 = L2p + N, *Y1 = L3 + N, *Y2 = Y1 + N, *Y3 = Y2 + N;
    double *A1 = Y3 + N, *A2p = A1 + N, *A3 = A2p + N;
    double *Q[3];
    Q[0] = A3 + N;
    Q[1] = Q[0] + mh[0] * mh[0];
    Q[2] = Q[1] + mh[1] * mh[1];
    double *part = Q[2] + mh[2] * mh[2], *sums = part + 3 * (size_t)np;
    double *L1 = L;
    CK(launch_lrr_comb(N, 1, 0, nullptr, 0, 0, nullptr, 0, 0, nullptr, 0, 0.0, Y1, N, s));
    CK(launch_lrr_comb(N, 1, 0, nullptr, 0, 0, nullptr, 0, 0, nullptr, 0, 0.0, Y2, N, s));
    CK(launch_lrr_comb(N, 1, 0, nullptr, 0, 0, nullptr, 0, 0, nullptr, 0, 0.0, Y3, N, s));
    CK(launch_ten_perm(I1, I2, I3, O, A2p, s));
    double *X[3] = {L1, L2p, L3};
    int r_prev[3] = {-1, -1, -1}, r[3] = {0, 0, 0};
    double res = 0.0;
    bool converged = false;
    int it;
    const auto t0 = std::chrono::steady_clock::now();
    for (it = 0; it < op.max_iter; ++it) {
        // the iteration's SVT inputs O - E + Y_i / mu (O itself at the start)
        const double *A[3] = {it ? A1 : O, A2p, it ? A3 : O};
        for (int i = 0; i < 3; ++i) {
            int32_t rr = 0;
            const double tau = alpha[i] / mu;
            if (op.use_frsvt) {
                const int l0 = std::max(1, (int)std::ceil(0.1 * (double)mh[i]));
                const bool prop = r_prev[i] > 0;
                const int kk = r_prev[i] < 0 ? l0 : 0, pp = r_prev[i] < 0 ? 0 : op.p;
                if ((rc = frsvt_impl<double>(h, vm[i], vn[i], A[i], vm[i], tau, kk, pp, op.q, prop ? Q[i] : nullptr,
                                             prop ? r_prev[i] : 0, mh[i], op.seed + (uint64_t)i, (uint64_t)it,
                                             X[i], vm[i], Q[i], mh[i], &rr)))
                    return rc;
                r_prev[i] = rr;
            } else {
                if ((rc = exact_svt_impl<double>(h, vm[i], vn[i], A[i], vm[i], tau, nullptr, X[i], vm[i], &rr)))
                    return rc;
            }
            r[i] = rr;
        }
        const double mu_next = std::min(op.rho * mu, op.mu_max);
        CK(launch_ten_update(I1, I2, I3, O, L1, L2p, L3, Y1, Y2, Y3, E, A1, A2p, A3, mu, lambda / (3.0 * mu),
                             mu_next, part, sums, s));
        CK(hipMemcpyAsync(h->pinned, sums, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
        CK(hipStreamSynchronize(s));
        const double *hs = (const double *)h->pinned;
        res = std::sqrt(std::max({hs[0], hs[1], hs[2]})) / normF;
        mu = mu_next;
        if (res < op.tol) {
            converged = true;
            ++it;
            break;
        }
    }
    CK(launch_ten_mean(I1, I2, I3, L1, L2p, L3, L, s));
    CK(hipStreamSynchronize(s));
    if (stats) {
        stats->iters = it;
        stats->converged = converged ? 1 : 0;
        for (int i = 0; i < 3; ++i) stats->rank[i] = r[i];
        stats->resid = res;
        stats->mu0 = mu0;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return converged ? FRSVT_OK : FRSVT_MAX_ITER;
}


// ---------------------------------------------------------------------------
// Batch drivers: side contexts, fork/join, and the auxiliary buffer.
// ---------------------------------------------------------------------------
constexpr int kSides = 4;

int ensure_aux(frsvt_context *h, size_t bytes)
{
    if (bytes <= h->aux_bytes) return FRSVT_OK;
    if (h->aux) {
        CK(hipStreamSynchronize(h->stream));
        (void)hipFree(h->aux);
        h->aux = nullptr;
        h->aux_bytes = 0;
    }
    hipError_t e = hipMalloc(&h->aux, bytes);
    if (e != hipSuccess) {
        h->aux = nullptr;
        return fail(h, e, "hipMalloc(aux)");
    }
    h->aux_bytes = bytes;
    return FRSVT_OK;
}

// The side contexts of h (created on first use, each on a stream of its own
// at the default priority).
int ensure_sides(frsvt_context *h)
{
    if (h->side[0]) return FRSVT_OK;
    int dev_prev = 0;
    (void)hipGetDevice(&dev_prev);
    CK(hipSetDevice(h->device));
    int rc = FRSVT_OK;
    if (!h->ev_fork && hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) != hipSuccess)
        rc = FRSVT_ERR_HIP;
    for (int i = 0; i < kSides && rc == FRSVT_OK; ++i) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            rc = FRSVT_ERR_HIP;
            break;
        }
        frsvt_context *k = nullptr;
        rc = frsvt_create(&k, h->device, st);
        if (rc != FRSVT_OK) {
            (void)hipStreamDestroy(st);
            break;
        }
        k->owns_stream = true;
        if (hipEventCreateWithFlags(&k->ev_join, hipEventDisableTiming) != hipSuccess) rc = FRSVT_ERR_HIP;
        h->side[i] = k;
    }
    (void)hipSetDevice(dev_prev);
    if (rc != FRSVT_OK) snprintf(h->last_error, sizeof(h->last_error), "creating the side streams failed");
    return rc;
}

// The side streams wait for the work enqueued so far on h's stream.
int fork_sides(frsvt_context *h)
{
    CK(hipEventRecord(h->ev_fork, h->stream));
    for (int i = 0; i < kSides; ++i) CK(hipStreamWaitEvent(h->side[i]->stream, h->ev_fork, 0));
    return FRSVT_OK;
}

// h's stream waits for everything enqueued on the side streams.
int join_sides(frsvt_context *h)
{
    for (int i = 0; i < kSides; ++i) {
        CK(hipEventRecord(h->side[i]->ev_join, h->side[i]->stream));
        CK(hipStreamWaitEvent(h->stream, h->side[i]->ev_join, 0));
    }
    return FRSVT_OK;
}

// A side context's error text is copied to the caller's handle.
int side_rc(frsvt_context *h, frsvt_context *k, int rc)
{
    if (rc != FRSVT_OK && rc != FRSVT_NOT_CONVERGED) memcpy(h->last_error, k->last_error, sizeof(h->last_error));
    return rc;
}

// Reads n doubles of device memory (ordered on h's stream; waits).
int read_doubles(frsvt_context *h, const double *src, size_t n, std::vector<double> &dst)
{
    dst.resize(n);
    if (n == 0) return FRSVT_OK;
    if (n * sizeof(double) > (1u << 20)) return FRSVT_ERR_UNSUPPORTED;
    CK(hipMemcpyAsync(h->pinned, src, n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    CK(hipStreamSynchronize(h->stream));
    memcpy(dst.data(), h->pinned, n * sizeof(double));
    return FRSVT_OK;
}

// ---------------------------------------------------------------------------
// Unrolled inexact-ALM RPCA (differentiation form): T steps of
//   L_{t+1} = FRSVT_{tau_t}(A_t)  (fresh sketch, counter t, seed + b),
//   (Y_{t+1}, A_{t+1}) = dual step with lam_t, mu_t, mu_{t+1},
// from the iALM starting point of each instance; mu_t = min(mu_0 rho^t,
// mu_bar_factor mu_0), mu_0 = 1.25 / ||O_b||_2.  The forward keeps, per
// instance, mu, every A_t, Y_t, L_t (t < T - 1), the bases Q_t and the small
// factors in the caller's `saved` buffer; the reverse sweep reads them.
// ---------------------------------------------------------------------------
template <typename T>
struct UnrolledLayout {
    double *mus;
    std::vector<T *> A, Y, Lx, Q;
    std::vector<double *> fac;
};

template <typename T>
size_t carve_unrolled(Carver &cv, int steps, int64_t m, int64_t n, int l, UnrolledLayout<T> &u)
{
    const int64_t mh = std::min(m, n);
    u.A.assign(steps, nullptr);
    u.Y.assign(steps, nullptr);
    u.Lx.assign(std::max(steps - 1, 0), nullptr);
    u.Q.assign(steps, nullptr);
    u.fac.assign(steps, nullptr);
    u.mus = cv.take<double>((size_t)steps + 1);
    for (int t = 0; t < steps; ++t) {
        u.A[t] = cv.take<T>((size_t)m * n);
        u.Y[t] = cv.take<T>((size_t)m * n);
        if (t + 1 < steps) u.Lx[t] = cv.take<T>((size_t)m * n);
        u.Q[t] = cv.take<T>((size_t)mh * l);
        u.fac[t] = cv.take<double>((size_t)l + (size_t)l * l);
    }
    cv.off = (cv.off + 255) & ~(size_t)255;
    return cv.off;
}

template <typename T>
size_t unrolled_instance_bytes(int steps, int64_t m, int64_t n, int l)
{
    Carver dry(nullptr);
    UnrolledLayout<T> u;
    return carve_unrolled<T>(dry, steps, m, n, l, u);
}

// mu_t of the iALM schedule (capped at mu_bar_factor mu_0), t = 0..steps.
std::vector<double> mu_schedule(double mu0, double rho, double mu_bar_factor, int steps)
{
    std::vector<double> mus((size_t)steps + 1);
    double mu = mu0;
    const double mub = mu0 * mu_bar_factor;
    for (int t = 0; t <= steps; ++t) {
        mus[t] = std::min(mu, mub);
        mu *= rho;
    }
    return mus;
}

template <typename T>
int unrolled_fwd_impl(frsvt_context *h, int B, int steps, int64_t m, int64_t n, const T *O, int64_t ldo,
                      int64_t sO, const double *taus_d, const double *lams_d, double lambda, double rho,
                      double mu_bar_factor, int k, int p, int q, uint64_t seed, T *L, int64_t ldl,
                      int64_t sL, void *saved)
{
    const int64_t mh = std::min(m, n);
    const int l = (int)std::min<int64_t>(mh, (int64_t)k + p);
    std::vector<double> tv, lv;
    int rc;
    if ((rc = read_doubles(h, taus_d, steps, tv))) return rc;
    if ((rc = read_doubles(h, lams_d, steps, lv))) return rc;
    for (int t = 0; t < steps; ++t)
        if (!(tv[t] >= 0.0) || !std::isfinite(tv[t]) || !(lv[t] >= 0.0) || !std::isfinite(lv[t])) return -10;
    if ((rc = ensure_sides(h))) return rc;
    const size_t per = unrolled_instance_bytes<T>(steps, m, n, l);
    std::vector<UnrolledLayout<T>> lay(B);
    std::vector<std::vector<double>> mus(B);
    if ((rc = fork_sides(h))) return rc;
    // starting points (each waits for its side stream: ||O_b||_2 sets mu_0)
    for (int b = 0; b < B; ++b) {
        frsvt_context *k2 = h->side[b % kSides];
        Carver cv((char *)saved + (size_t)b * per);
        carve_unrolled<T>(cv, steps, m, n, l, lay[b]);
        double out[3];
        rc = rpca_init_impl<T>(k2, m, n, O + (size_t)b * sO, ldo, lambda, 0.0, lay[b].Y[0], m, lay[b].A[0], m, out);
        if (rc) return side_rc(h, k2, rc);
        mus[b] = mu_schedule(out[1], rho, mu_bar_factor, steps);
        CK(hipMemcpyAsync(lay[b].mus, mus[b].data(), mus[b].size() * sizeof(double), hipMemcpyHostToDevice,
                          k2->stream));
        CK(hipStreamSynchronize(k2->stream));
    }
    for (int b = 0; b < B; ++b) {
        frsvt_context *k2 = h->side[b % kSides];
        const UnrolledLayout<T> &u = lay[b];
        const T *Ob = O + (size_t)b * sO;
        for (int t = 0; t < steps; ++t) {
            const bool last = t + 1 == steps;
            T *X = last ? L + (size_t)b * sL : u.Lx[t];
            const int64_t ldx = last ? ldl : m;
            rc = frsvt_impl<T>(k2, m, n, u.A[t], m, tv[t], k, p, q, nullptr, 0, mh, seed + (uint64_t)b,
                               (uint64_t)t, X, ldx, nullptr, mh, nullptr, false, u.Q[t], mh, u.fac[t]);
            if (rc) return side_rc(h, k2, rc);
            if (!last) {
                rc = dual_step_impl<T>(k2, m, n, Ob, ldo, X, m, u.Y[t], m, lv[t], mus[b][t], mus[b][t + 1],
                                       nullptr, m, u.Y[t + 1], m, u.A[t + 1], m);
                if (rc) return side_rc(h, k2, rc);
            }
        }
    }
    return join_sides(h);
}

template <typename T>
int unrolled_bwd_impl(frsvt_context *h, int B, int steps, int64_t m, int64_t n, const T *O, int64_t ldo,
                      int64_t sO, const double *taus_d, const double *lams_d, int k, int p, int q,
                      uint64_t seed, const void *saved, const T *Lbar, int64_t ldlb, int64_t sLb,
                      double *tau_bar, double *lam_bar)
{
    const int64_t mh = std::min(m, n);
    const int l = (int)std::min<int64_t>(mh, (int64_t)k + p);
    std::vector<double> tv, lv;
    int rc;
    if ((rc = read_doubles(h, taus_d, steps, tv))) return rc;
    if ((rc = read_doubles(h, lams_d, steps, lv))) return rc;
    if ((rc = ensure_sides(h))) return rc;
    const size_t per = unrolled_instance_bytes<T>(steps, m, n, l);
    std::vector<UnrolledLayout<T>> lay(B);
    std::vector<std::vector<double>> mus(B);
    for (int b = 0; b < B; ++b) {
        Carver cv((char *)saved + (size_t)b * per);
        carve_unrolled<T>(cv, steps, m, n, l, lay[b]);
        if ((rc = read_doubles(h, lay[b].mus, (size_t)steps + 1, mus[b]))) return rc;
    }
    // per-(instance, step) threshold gradients, summed over the batch at the end
    const size_t gbytes = ((2 * (size_t)B * steps * sizeof(double)) + 255) & ~(size_t)255;
    if ((rc = ensure_aux(h, gbytes))) return rc;
    double *gt = (double *)h->aux;
    double *gl = gt + (size_t)B * steps;
    CK(hipMemsetAsync(gt, 0, 2 * (size_t)B * steps * sizeof(double), h->stream));
    // reverse-sweep buffers of each side context: A_bar, L_bar, Y_bar (two)
    const size_t mn = (size_t)m * n;
    for (int i = 0; i < kSides; ++i)
        if ((rc = ensure_aux(h->side[i], 4 * mn * sizeof(T) + 256))) return side_rc(h, h->side[i], rc);
    if ((rc = fork_sides(h))) return rc;
    for (int b = 0; b < B; ++b) {
        frsvt_context *k2 = h->side[b % kSides];
        const UnrolledLayout<T> &u = lay[b];
        const T *Ob = O + (size_t)b * sO;
        T *Ab = (T *)k2->aux, *Lb = Ab + mn, *Yb[2] = {Lb + mn, Lb + 2 * mn};
        int cur = 0;  // Yb[cur]: gradient of Y_{t+1}
        for (int t = steps - 1; t >= 0; --t) {
            const T *Lin;
            int64_t ldin;
            if (t == steps - 1) {
                Lin = Lbar + (size_t)b * sLb;
                ldin = ldlb;
            } else {
                // Y_{T-1} feeds no later step: its gradient is zero
                const T *Ynb = t == steps - 2 ? nullptr : Yb[cur];
                rc = dual_step_vjp_impl<T>(k2, m, n, Ob, ldo, u.Lx[t], m, u.Y[t], m, lv[t], mus[b][t],
                                           mus[b][t + 1], nullptr, m, Ynb, m, Ab, m, Lb, m, Yb[cur ^ 1], m,
                                           gl + (size_t)b * steps + t);
                if (rc) return side_rc(h, k2, rc);
                cur ^= 1;
                Lin = Lb;
                ldin = m;
            }
            rc = frsvt_vjp_impl<T>(k2, m, n, u.A[t], m, tv[t], l, q, seed + (uint64_t)b, (uint64_t)t, u.Q[t],
                                   mh, u.fac[t], Lin, ldin, Ab, m, gt + (size_t)b * steps + t);
            if (rc) return side_rc(h, k2, rc);
        }
    }
    if ((rc = join_sides(h))) return rc;
    // sums over the batch in a fixed order
    CKT(FRSVT_K_REDUCE, launch_reduce<double>(gt, steps, B, tau_bar, h->stream));
    CKT(FRSVT_K_REDUCE, launch_reduce<double>(gl, steps, B, lam_bar, h->stream));
    return FRSVT_OK;
}

// ---------------------------------------------------------------------------
// Semi-online decomposition (Type B of Table 6, Sec. 4): consecutive windows
// of `window` frames, each by the partial-SVT iALM with FRSVT (the keep
// largest singular values unshrunk), sketch widths by adaptive prediction
// bounded by l (a = l - keep, b = ceil((l / window) mhat)), q power
// iterations; window w draws with seed + w and starts from window w - 1's
// last propagated basis.
// ---------------------------------------------------------------------------
template <typename T>
int sliding_impl(frsvt_context *h, int64_t m, int64_t frames, const T *F, int64_t ldf, int window,
                 double lambda, int keep, int l, int q, uint64_t seed, double tol, int max_iter, double rho,
                 T *L, int64_t ldl, T *S, int64_t lds, frsvt_rpca_stats *stats, T *bases)
{
    const int64_t nw = frames / window;
    const int64_t mh = std::min<int64_t>(m, window);
    int rc;
    // two propagated-basis buffers (handed over from window to window)
    if ((rc = ensure_aux(h, 2 * (size_t)mh * mh * sizeof(T) + 512))) return rc;
    T *Qb[2] = {(T *)h->aux, (T *)((char *)h->aux + (((size_t)mh * mh * sizeof(T) + 255) & ~(size_t)255))};
    int r = 0, cur = 0;
    for (int64_t w = 0; w < nw; ++w) {
        frsvt_rpca_opts op;
        frsvt_rpca_default_opts(&op);
        op.tol = tol;
        op.max_iter = max_iter;
        op.rho = rho;
        op.use_frsvt = 1;
        op.q = q;
        op.seed = seed + (uint64_t)w;
        op.ap = 1;
        op.ap_a = l - keep;
        op.ap_gamma = (double)l / (double)window;
        op.keep = keep;
        op.q_init = r > 0 ? Qb[cur] : nullptr;
        op.r_init = r;
        op.q_final = Qb[cur ^ 1];
        frsvt_rpca_stats st;
        memset(&st, 0, sizeof(st));
        const int64_t c0 = w * window;
        rc = rpca_impl<T>(h, m, window, F + c0 * ldf, ldf, lambda, op, L + c0 * ldl, ldl, S + c0 * lds, lds, &st);
        if (rc != FRSVT_OK && rc != FRSVT_MAX_ITER) return rc;
        if (stats) stats[w] = st;
        // the last iteration's rank is the width of the basis handed over
        r = st.iters > 0 ? st.ranks[std::min(st.iters, 64) - 1] : 0;
        if (bases && r > 0)
            CK(hipMemcpyAsync(bases + (size_t)w * mh * l, Qb[cur ^ 1], (size_t)mh * r * sizeof(T),
                              hipMemcpyDeviceToDevice, h->stream));
        cur ^= 1;
    }
    CK(hipStreamSynchronize(h->stream));
    return FRSVT_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int frsvt_create(frsvt_handle *handle, int device, void *hip_stream)
{
    if (!handle) return -1;
    *handle = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return FRSVT_ERR_HIP;
    if (device < 0 || device >= count) return -2;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return FRSVT_ERR_HIP;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return FRSVT_ERR_UNSUPPORTED;
    frsvt_context *h = new frsvt_context();
    h->device = device;
    h->stream = (hipStream_t)hip_stream;
    h->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    int dev_prev = 0;
    (void)hipGetDevice(&dev_prev);
    (void)hipSetDevice(device);
    hipError_t e = hipMalloc(&h->dstatus, kStatusInts * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&h->dscalars, kScalarDoubles * sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc(&h->pinned, 1 << 20, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMemset(h->dstatus, 0, kStatusInts * sizeof(int));
    if (e == hipSuccess) h->scratch_dev = scratch_address(device);
    (void)hipSetDevice(dev_prev);
    if (e != hipSuccess) {
        if (h->dstatus) (void)hipFree(h->dstatus);
        if (h->dscalars) (void)hipFree(h->dscalars);
        if (h->pinned) (void)hipHostFree(h->pinned);
        delete h;
        return e == hipErrorOutOfMemory ? FRSVT_ERR_OOM : FRSVT_ERR_HIP;
    }
    *handle = h;
    return FRSVT_OK;
}

int frsvt_destroy(frsvt_handle h)
{
    if (!h) return -1;
    (void)hipStreamSynchronize(h->stream);
    for (auto &k : h->side)
        if (k) {
            (void)frsvt_destroy(k);
            k = nullptr;
        }
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    if (h->aux) (void)hipFree(h->aux);
    for (auto &r : h->recs) {
        (void)hipEventDestroy(r.second.first);
        (void)hipEventDestroy(r.second.second);
    }
    for (auto e : h->pool) (void)hipEventDestroy(e);
    if (h->host_iter) (void)hipHostFree(h->host_iter);
    if (h->wb_exec) (void)hipGraphExecDestroy(h->wb_exec);
    if (h->wb_capture) (void)hipStreamDestroy(h->wb_capture);
    if (h->wb_queue) (void)hipFree(h->wb_queue);
    if (h->wb_gs_dev) (void)hipFree(h->wb_gs_dev);
    if (h->wb_order) (void)hipFree(h->wb_order);
    if (h->ws) (void)hipFree(h->ws);
    if (h->dstatus) (void)hipFree(h->dstatus);
    if (h->dscalars) (void)hipFree(h->dscalars);
    if (h->pinned) (void)hipHostFree(h->pinned);
    if (h->owns_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
    return FRSVT_OK;
}

int frsvt_set_option(frsvt_handle h, int option, int value)
{
    if (!h) return -1;
    if (option != FRSVT_OPT_QRCP_TRUNCATE) return -2;
    if (value != 0 && value != 1) return -3;
    h->opt_truncate = value;
    return FRSVT_OK;
}

int frsvt_set_stream(frsvt_handle h, void *hip_stream)
{
    if (!h) return -1;
    h->stream = (hipStream_t)hip_stream;
    return FRSVT_OK;
}

const char *frsvt_status_string(int status)
{
    switch (status) {
    case FRSVT_OK: return "success";
    case FRSVT_NOT_CONVERGED: return "Jacobi sweep limit reached (result written)";
    case FRSVT_MAX_ITER: return "RPCA reached max_iter before the tolerance";
    case FRSVT_ERR_HIP: return "HIP runtime error";
    case FRSVT_ERR_OOM: return "out of device memory";
    case FRSVT_ERR_NONFINITE: return "non-finite input";
    case FRSVT_ERR_CHOLESKY: return "Cholesky factorisation failed after the shifted fallback";
    case FRSVT_ERR_UNSUPPORTED: return "unsupported device or configuration";
    case FRSVT_ERR_HANDLE: return "invalid handle";
    case FRSVT_ERR_SCRATCH: return "problem too large for the fixed scratch of frsvt_noalloc";
    default: break;
    }
    if (status < 0 && status > -100) return "invalid argument";
    return "unknown status";
}

const char *frsvt_last_error(frsvt_handle h) { return h ? h->last_error : "invalid handle"; }

int64_t frsvt_workspace_bytes(frsvt_handle h) { return h ? (int64_t)h->ws_bytes : -1; }

static void trace_flush(frsvt_context *h)
{
    if (h->recs.empty()) return;
    (void)hipStreamSynchronize(h->stream);
    for (auto &r : h->recs) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.second.first, r.second.second) == hipSuccess &&
            r.first >= 0 && r.first < FRSVT_K_COUNT) {
            h->trace_ms[r.first] += ms;
            h->trace_n[r.first] += 1;
        }
        h->pool.push_back(r.second.first);
        h->pool.push_back(r.second.second);
    }
    h->recs.clear();
}

int frsvt_trace_enable(frsvt_handle h, int enable)
{
    if (!h) return -1;
    trace_flush(h);
    if (enable) {
        for (int k = 0; k < FRSVT_K_COUNT; ++k) {
            h->trace_ms[k] = 0.0;
            h->trace_n[k] = 0;
        }
    }
    h->tracing = enable != 0;
    return FRSVT_OK;
}

int frsvt_trace_read(frsvt_handle h, int kernel_class, double *total_ms, int64_t *launches)
{
    if (!h) return -1;
    if (kernel_class < 0 || kernel_class >= FRSVT_K_COUNT) return -2;
    trace_flush(h);
    if (total_ms) *total_ms = h->trace_ms[kernel_class];
    if (launches) *launches = h->trace_n[kernel_class];
    return FRSVT_OK;
}

int frsvt_last_info(frsvt_handle h, int32_t *info, int count)
{
    if (!h) return -1;
    if (!info) return -2;
    if (count < 0 || count > 8) return -3;
    if (count == 0) return FRSVT_OK;
    hipError_t e = hipMemcpyAsync(h->pinned, h->dstatus, 8 * sizeof(int), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(h, e, "frsvt_last_info");
    memcpy(info, h->pinned, (size_t)count * sizeof(int32_t));
    return FRSVT_OK;
}

const char *frsvt_trace_name(int k)
{
    static const char *names[FRSVT_K_COUNT] = {"sketch", "power", "project", "reduce", "orth",
                                                "small_svd", "recon", "epilogue", "gemm", "other",
                                                "gemm_bf16", "wsvt_batched", "adjoint"};
    return (k >= 0 && k < FRSVT_K_COUNT) ? names[k] : "unknown";
}

void frsvt_rpca_default_opts(frsvt_rpca_opts *op)
{
    if (!op) return;
    op->tol = 1e-7;
    op->max_iter = 60;
    op->mu0 = 0.0;
    op->rho = 1.5;
    op->mu_bar_factor = 1e7;
    op->use_frsvt = 1;
    op->p = 5;
    op->q = 1;
    op->l0 = 0;
    op->seed = 0;
    op->ap = 0;
    op->ap_a = 2;
    op->ap_rho = 0.05;
    op->ap_gamma = 1.0;
    op->keep = 0;
    op->q_init = nullptr;
    op->r_init = 0;
    op->q_final = nullptr;
    op->resid_check = 0;
}

int svt(frsvt_handle h, frsvt_precision prec, int64_t m, int64_t n, const void *A, int64_t lda,
        double tau, void *X, int64_t ldx, int32_t *rank)
{
    if (!h) return -1;
    if (prec != FRSVT_F64 && prec != FRSVT_F32 && prec != FRSVT_MIXED_BF16) return -2;
    if (m < 1) return -3;
    if (n < 1) return -4;
    if (bad_ptr(A)) return -5;
    if (lda < m) return -6;
    if (!(tau >= 0.0) || !std::isfinite(tau)) return -7;
    if (bad_ptr(X)) return -8;
    if (ldx < m) return -9;
    if (std::min(m, n) > 1024) return FRSVT_ERR_UNSUPPORTED;
    if (prec == FRSVT_F64)
        return exact_svt_impl<double>(h, m, n, (const double *)A, lda, tau, nullptr, (double *)X, ldx, rank);
    return exact_svt_impl<float>(h, m, n, (const float *)A, lda, tau, nullptr, (float *)X, ldx, rank);
}

int wsvt(frsvt_handle h, frsvt_precision prec, int64_t m, int64_t n, const void *A, int64_t lda,
         const double *w, void *X, int64_t ldx, int32_t *rank)
{
    if (!h) return -1;
    if (prec != FRSVT_F64 && prec != FRSVT_F32 && prec != FRSVT_MIXED_BF16) return -2;
    if (m < 1) return -3;
    if (n < 1) return -4;
    if (bad_ptr(A)) return -5;
    if (lda < m) return -6;
    if (bad_ptr(w)) return -7;
    if (bad_ptr(X)) return -8;
    if (ldx < m) return -9;
    if (std::min(m, n) > 1024) return FRSVT_ERR_UNSUPPORTED;
    if (prec == FRSVT_F64)
        return exact_svt_impl<double>(h, m, n, (const double *)A, lda, 0.0, w, (double *)X, ldx, rank);
    return exact_svt_impl<float>(h, m, n, (const float *)A, lda, 0.0, w, (float *)X, ldx, rank);
}

static int frsvt_entry(frsvt_handle h, frsvt_precision prec, int64_t m, int64_t n, const void *A,
                       int64_t lda, double tau, int32_t k, int32_t p, int32_t q, const void *Q_prev,
                       int32_t r_prev, int64_t ldq_prev, uint64_t seed, uint64_t counter, void *X,
                       int64_t ldx, void *Q_out, int64_t ldq_out, int32_t *r_out, const FixedWs *fixed)
{
    if (!h) return -1;
    if (prec != FRSVT_F64 && prec != FRSVT_F32 && prec != FRSVT_MIXED_BF16) return -2;
    if (m < 1) return -3;
    if (n < 1) return -4;
    if (bad_ptr(A)) return -5;
    if (lda < m) return -6;
    if (!(tau >= 0.0) || !std::isfinite(tau)) return -7;
    const bool rp = Q_prev != nullptr && r_prev > 0;
    if (!rp && (k < 0 || k + p < 1)) return -8;
    if (p < 0) return -9;
    if (q < 0 || q > 64) return -10;
    const int64_t mh = std::min(m, n);
    if (Q_prev && (r_prev < 0 || r_prev > mh)) return -12;
    if (rp && ldq_prev < mh) return -13;
    if (bad_ptr(X)) return -16;
    if (ldx < m) return -17;
    if (Q_out && ldq_out < mh) return -19;
    // the large path's orthonormalisation takes at most 256 columns
    if (std::min<int64_t>(mh, (int64_t)(Q_prev && r_prev > 0 ? r_prev + p : k + p)) > 256)
        return FRSVT_ERR_UNSUPPORTED;
    if (prec == FRSVT_MIXED_BF16)
        return frsvt_impl<float>(h, m, n, (const float *)A, lda, tau, k, p, q, (const float *)Q_prev,
                                 r_prev, ldq_prev, seed, counter, (float *)X, ldx, (float *)Q_out,
                                 ldq_out, r_out, true, nullptr, 0, nullptr, fixed);
    if (prec == FRSVT_F64)
        return frsvt_impl<double>(h, m, n, (const double *)A, lda, tau, k, p, q,
                                  (const double *)Q_prev, r_prev, ldq_prev, seed, counter,
                                  (double *)X, ldx, (double *)Q_out, ldq_out, r_out, false, nullptr, 0,
                                  nullptr, fixed);
    return frsvt_impl<float>(h, m, n, (const float *)A, lda, tau, k, p, q, (const float *)Q_prev,
                             r_prev, ldq_prev, seed, counter, (float *)X, ldx, (float *)Q_out,
                             ldq_out, r_out, false, nullptr, 0, nullptr, fixed);
}

int frsvt(frsvt_handle h, frsvt_precision prec, int64_t m, int64_t n, const void *A, int64_t lda,
          double tau, int32_t k, int32_t p, int32_t q, const void *Q_prev, int32_t r_prev,
          int64_t ldq_prev, uint64_t seed, uint64_t counter, void *X, int64_t ldx, void *Q_out,
          int64_t ldq_out, int32_t *r_out)
{
    return frsvt_entry(h, prec, m, n, A, lda, tau, k, p, q, Q_prev, r_prev, ldq_prev, seed, counter, X, ldx,
                       Q_out, ldq_out, r_out, nullptr);
}

int frsvt_noalloc(frsvt_handle h, frsvt_precision prec, int64_t m, int64_t n, const void *A, int64_t lda,
                  double tau, int32_t k, int32_t p, int32_t q, const void *Q_prev, int32_t r_prev,
                  int64_t ldq_prev, uint64_t seed, uint64_t counter, void *X, int64_t ldx, void *Q_out,
                  int64_t ldq_out, int32_t *r_out)
{
    if (!h) return -1;
    // the device's own copy of the fixed scratch, looked up at frsvt_create
    const FixedWs fx{h->scratch_dev, (size_t)FRSVT_NOALLOC_SCRATCH_BYTES};
    return frsvt_entry(h, prec, m, n, A, lda, tau, k, p, q, Q_prev, r_prev, ldq_prev, seed, counter, X, ldx,
                       Q_out, ldq_out, r_out, &fx);
}

int rpca_ialm(frsvt_handle h, frsvt_precision prec, int64_t m, int64_t n, const void *O,
              int64_t ldo, double lambda, const frsvt_rpca_opts *opts, void *L, int64_t ldl,
              void *S, int64_t lds, frsvt_rpca_stats *stats)
{
    if (!h) return -1;
    if (prec != FRSVT_F64 && prec != FRSVT_F32 && prec != FRSVT_MIXED_BF16) return -2;
    if (m < 1) return -3;
    if (n < 1) return -4;
    if (bad_ptr(O)) return -5;
    if (ldo < m) return -6;
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return -7;
    frsvt_rpca_opts op;
    frsvt_rpca_default_opts(&op);
    if (opts) op = *opts;
    if (!(op.tol > 0.0) || op.max_iter < 1 || !(op.rho >= 1.0) || op.p < 1 || op.q < 0 ||
        !(op.mu_bar_factor >= 1.0))
        return -8;
    if (op.ap != 0 && op.ap != 1) return -8;
    if (op.resid_check != 0 && op.resid_check != 1) return -8;
    if (op.keep < 0 || op.r_init < 0 || op.r_init > std::min(m, n) || (op.r_init > 0 && bad_ptr(op.q_init)))
        return -8;
    if (op.ap && (op.ap_a < 1 || !(op.ap_rho > 0.0) || !(op.ap_rho <= 1.0) || !(op.ap_gamma > 0.0) ||
                  !(op.ap_gamma <= 1.0)))
        return -8;
    if (bad_ptr(L)) return -9;
    if (ldl < m) return -10;
    if (bad_ptr(S)) return -11;
    if (lds < m) return -12;
    // exact SVT: the one-workgroup small SVD of the short side (<= 1024);
    // FRSVT: up to 8192 (the propagated basis is kept as a short-side square)
    if (std::min(m, n) > (op.use_frsvt ? 8192 : 1024)) return FRSVT_ERR_UNSUPPORTED;
    if (prec == FRSVT_MIXED_BF16) return FRSVT_ERR_UNSUPPORTED;
    if (prec == FRSVT_F64)
        return rpca_impl<double>(h, m, n, (const double *)O, ldo, lambda, op, (double *)L, ldl,
                                 (double *)S, lds, stats);
    return rpca_impl<float>(h, m, n, (const float *)O, ldo, lambda, op, (float *)L, ldl,
                            (float *)S, lds, stats);
}

int frsvt_wsvt_tuning(frsvt_handle h, int32_t group_size[3])
{
    if (!h) return -1;
    if (!group_size) return -2;
    for (int b = 0; b < 3; ++b) group_size[b] = h->wb_tuned ? h->wb_gs[b] : 0;
    return FRSVT_OK;
}

int frsvt_wsvt_work(frsvt_handle h, int64_t work[3])
{
    if (!h) return -1;
    if (!work) return -2;
    for (int b = 0; b < 3; ++b) work[b] = 0;
    if (!h->wb_queue) return FRSVT_OK;
    CK(hipSetDevice(h->device));
    CK(hipMemcpyAsync(h->pinned, h->wb_queue + 16, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                      h->stream));
    CK(hipStreamSynchronize(h->stream));
    for (int b = 0; b < 3; ++b) work[b] = (int64_t)((const unsigned long long *)h->pinned)[b];
    return FRSVT_OK;
}

int wsvt_batched(frsvt_handle h, int64_t count, const int32_t *rows, const int32_t *cols,
                 const int64_t *offsets, const float *A_packed, float *X_packed,
                 const frsvt_wsvt_rule *rule, int32_t *ranks)
{
    if (!h) return -1;
    if (count < 0) return -2;
    if (count > 0 && bad_ptr(rows)) return -3;
    if (count > 0 && bad_ptr(cols)) return -4;
    if (count > 0 && bad_ptr(offsets)) return -5;
    if (count > 0 && bad_ptr(A_packed)) return -6;
    if (count > 0 && bad_ptr(X_packed)) return -7;
    if (bad_ptr(rule)) return -8;
    if (count == 0) return FRSVT_OK;
    if (count > (int64_t)1 << 30) return FRSVT_ERR_UNSUPPORTED;
    return wsvt_batched_impl(h, count, rows, cols, offsets, A_packed, X_packed, *rule, ranks);
}

int frsvt_fwd(frsvt_handle h, frsvt_precision prec, int64_t m, int64_t n, const void *A,
              int64_t lda, double tau, int32_t k, int32_t p, int32_t q, uint64_t seed,
              uint64_t counter, void *X, int64_t ldx, void *Q, int64_t ldq, double *factors)
{
    if (!h) return -1;
    if (prec != FRSVT_F64 && prec != FRSVT_F32) return -2;
    if (m < 1) return -3;
    if (n < 1) return -4;
    if (bad_ptr(A)) return -5;
    if (lda < m) return -6;
    if (!(tau >= 0.0) || !std::isfinite(tau)) return -7;
    if (k < 0 || p < 0 || k + p < 1) return -8;
    if (p < 0) return -9;
    if (q < 0 || q > 64) return -10;
    if (bad_ptr(X)) return -13;
    if (ldx < m) return -14;
    const int64_t mh = std::min(m, n);
    if (bad_ptr(Q)) return -15;
    if (ldq < mh) return -16;
    if (bad_ptr(factors)) return -17;
    if (std::min<int64_t>(mh, (int64_t)k + p) > 64) return FRSVT_ERR_UNSUPPORTED;
    if (prec == FRSVT_F64)
        return frsvt_impl<double>(h, m, n, (const double *)A, lda, tau, k, p, q, nullptr, 0, mh, seed,
                                  counter, (double *)X, ldx, nullptr, mh, nullptr, false, (double *)Q,
                                  ldq, factors);
    return frsvt_impl<float>(h, m, n, (const float *)A, lda, tau, k, p, q, nullptr, 0, mh, seed, counter,
                             (float *)X, ldx, nullptr, mh, nullptr, false, (float *)Q, ldq, factors);
}

int frsvt_vjp(frsvt_handle h, frsvt_precision prec, int64_t m, int64_t n, const void *A,
              int64_t lda, double tau, int32_t k, int32_t p, int32_t q, uint64_t seed,
              uint64_t counter, const void *Q, int64_t ldq, const double *factors,
              const void *X_bar, int64_t ldxb, void *A_bar, int64_t ldab, double *tau_bar)
{
    if (!h) return -1;
    if (prec != FRSVT_F64 && prec != FRSVT_F32) return -2;
    if (m < 1) return -3;
    if (n < 1) return -4;
    if (bad_ptr(A)) return -5;
    if (lda < m) return -6;
    if (!(tau >= 0.0) || !std::isfinite(tau)) return -7;
    if (k < 0 || p < 0 || k + p < 1) return -8;
    if (p < 0) return -9;
    if (q < 0 || q > 64) return -10;
    const int64_t mh = std::min(m, n);
    if (bad_ptr(Q)) return -13;
    if (ldq < mh) return -14;
    if (bad_ptr(factors)) return -15;
    if (bad_ptr(X_bar)) return -16;
    if (ldxb < m) return -17;
    if (bad_ptr(A_bar)) return -18;
    if (ldab < m) return -19;
    const int l = (int)std::min<int64_t>(mh, (int64_t)k + p);
    if (l > 64) return FRSVT_ERR_UNSUPPORTED;
    if (prec == FRSVT_F64)
        return frsvt_vjp_impl<double>(h, m, n, (const double *)A, lda, tau, l, q, seed, counter,
                                      (const double *)Q, ldq, factors, (const double *)X_bar, ldxb,
                                      (double *)A_bar, ldab, tau_bar);
    return frsvt_vjp_impl<float>(h, m, n, (const float *)A, lda, tau, l, q, seed, counter,
                                 (const float *)Q, ldq, factors, (const float *)X_bar, ldxb,
                                 (float *)A_bar, ldab, tau_bar);
}

int rpca_dual_step(frsvt_handle h, frsvt_precision prec, int64_t m, int64_t n, const void *O,
                   int64_t ldo, const void *L, int64_t ldl, const void *Y, int64_t ldy, double lam,
                   double mu, double mu_next, void *S, int64_t lds, void *Y_next, int64_t ldyn,
                   void *A_next, int64_t ldan)
{
    if (!h) return -1;
    if (prec != FRSVT_F64 && prec != FRSVT_F32) return -2;
    if (m < 1) return -3;
    if (n < 1) return -4;
    if (bad_ptr(O)) return -5;
    if (ldo < m) return -6;
    if (bad_ptr(L)) return -7;
    if (ldl < m) return -8;
    if (bad_ptr(Y)) return -9;
    if (ldy < m) return -10;
    if (!(lam >= 0.0) || !std::isfinite(lam)) return -11;
    if (!(mu > 0.0) || !std::isfinite(mu)) return -12;
    if (!(mu_next > 0.0) || !std::isfinite(mu_next)) return -13;
    if (S && lds < m) return -15;
    if (Y_next && ldyn < m) return -17;
    if (A_next && ldan < m) return -19;
    if (prec == FRSVT_F64)
        return dual_step_impl<double>(h, m, n, (const double *)O, ldo, (const double *)L, ldl,
                                      (const double *)Y, ldy, lam, mu, mu_next, (double *)S, lds,
                                      (double *)Y_next, ldyn, (double *)A_next, ldan);
    return dual_step_impl<float>(h, m, n, (const float *)O, ldo, (const float *)L, ldl,
                                 (const float *)Y, ldy, lam, mu, mu_next, (float *)S, lds,
                                 (float *)Y_next, ldyn, (float *)A_next, ldan);
}

int rpca_dual_step_vjp(frsvt_handle h, frsvt_precision prec, int64_t m, int64_t n, const void *O,
                       int64_t ldo, const void *L, int64_t ldl, const void *Y, int64_t ldy,
                       double lam, double mu, double mu_next, const void *S_bar, int64_t ldsb,
                       const void *Y_next_bar, int64_t ldynb, const void *A_next_bar,
                       int64_t ldanb, void *L_bar, int64_t ldlb, void *Y_bar, int64_t ldyb,
                       double *lam_bar)
{
    if (!h) return -1;
    if (prec != FRSVT_F64 && prec != FRSVT_F32) return -2;
    if (m < 1) return -3;
    if (n < 1) return -4;
    if (bad_ptr(O)) return -5;
    if (ldo < m) return -6;
    if (bad_ptr(L)) return -7;
    if (ldl < m) return -8;
    if (bad_ptr(Y)) return -9;
    if (ldy < m) return -10;
    if (!(lam >= 0.0) || !std::isfinite(lam)) return -11;
    if (!(mu > 0.0) || !std::isfinite(mu)) return -12;
    if (!(mu_next > 0.0) || !std::isfinite(mu_next)) return -13;
    if (S_bar && ldsb < m) return -15;
    if (Y_next_bar && ldynb < m) return -17;
    if (A_next_bar && ldanb < m) return -19;
    if (bad_ptr(L_bar)) return -20;
    if (ldlb < m) return -21;
    if (bad_ptr(Y_bar)) return -22;
    if (ldyb < m) return -23;
    if (prec == FRSVT_F64)
        return dual_step_vjp_impl<double>(h, m, n, (const double *)O, ldo, (const double *)L, ldl,
                                          (const double *)Y, ldy, lam, mu, mu_next,
                                          (const double *)S_bar, ldsb, (const double *)Y_next_bar,
                                          ldynb, (const double *)A_next_bar, ldanb,
                                          (double *)L_bar, ldlb, (double *)Y_bar, ldyb, lam_bar);
    return dual_step_vjp_impl<float>(h, m, n, (const float *)O, ldo, (const float *)L, ldl,
                                     (const float *)Y, ldy, lam, mu, mu_next, (const float *)S_bar,
                                     ldsb, (const float *)Y_next_bar, ldynb,
                                     (const float *)A_next_bar, ldanb, (float *)L_bar, ldlb,
                                     (float *)Y_bar, ldyb, lam_bar);
}

int rpca_init(frsvt_handle h, frsvt_precision prec, int64_t m, int64_t n, const void *O,
              int64_t ldo, double lambda, double mu0, void *Y0, int64_t ldy, void *A0,
              int64_t lda0, double *out)
{
    if (!h) return -1;
    if (prec != FRSVT_F64 && prec != FRSVT_F32) return -2;
    if (m < 1) return -3;
    if (n < 1) return -4;
    if (bad_ptr(O)) return -5;
    if (ldo < m) return -6;
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return -7;
    if (!std::isfinite(mu0)) return -8;
    if (bad_ptr(Y0)) return -9;
    if (ldy < m) return -10;
    if (bad_ptr(A0)) return -11;
    if (lda0 < m) return -12;
    if (std::min(m, n) > 1024) return FRSVT_ERR_UNSUPPORTED;
    if (prec == FRSVT_F64)
        return rpca_init_impl<double>(h, m, n, (const double *)O, ldo, lambda, mu0, (double *)Y0, ldy,
                                      (double *)A0, lda0, out);
    return rpca_init_impl<float>(h, m, n, (const float *)O, ldo, lambda, mu0, (float *)Y0, ldy,
                                 (float *)A0, lda0, out);
}


int64_t rpca_unrolled_saved_bytes(frsvt_precision prec, int32_t batch, int32_t steps, int64_t m, int64_t n,
                                  int32_t k, int32_t p)
{
    if (prec != FRSVT_F64 && prec != FRSVT_F32) return -1;
    if (batch < 1 || steps < 1 || m < 1 || n < 1 || k < 0 || p < 0 || k + p < 1) return -1;
    const int l = (int)std::min<int64_t>(std::min(m, n), (int64_t)k + p);
    const size_t per = prec == FRSVT_F64 ? unrolled_instance_bytes<double>(steps, m, n, l)
                                         : unrolled_instance_bytes<float>(steps, m, n, l);
    return (int64_t)(per * (size_t)batch);
}

int rpca_unrolled_schedule(frsvt_handle h, frsvt_precision prec, int64_t m, int64_t n, const void *O,
                           int64_t ldo, double lambda, double rho, double mu_bar_factor, int32_t steps,
                           double *taus, double *lams)
{
    if (!h) return -1;
    if (prec != FRSVT_F64 && prec != FRSVT_F32) return -2;
    if (m < 1) return -3;
    if (n < 1) return -4;
    if (bad_ptr(O)) return -5;
    if (ldo < m) return -6;
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return -7;
    if (!(rho >= 1.0) || !std::isfinite(rho)) return -8;
    if (!(mu_bar_factor >= 1.0)) return -9;
    if (steps < 1) return -10;
    if (bad_ptr(taus)) return -11;
    if (bad_ptr(lams)) return -12;
    if (std::min(m, n) > 1024) return FRSVT_ERR_UNSUPPORTED;
    double normF = 0.0, mx = 0.0, norm2 = 0.0;
    const Orient o = orient(m, n, ldo);
    int rc = prec == FRSVT_F64 ? input_norms<double>(h, m, n, (const double *)O, ldo, &normF, &mx)
                               : input_norms<float>(h, m, n, (const float *)O, ldo, &normF, &mx);
    if (rc) return rc;
    rc = prec == FRSVT_F64 ? spectral_norm<double>(h, (const double *)O, ldo, o, &norm2)
                           : spectral_norm<float>(h, (const float *)O, ldo, o, &norm2);
    if (rc) return rc;
    const double mu0 = norm2 > 0.0 ? 1.25 / norm2 : 1.0;
    const std::vector<double> mus = mu_schedule(mu0, rho, mu_bar_factor, steps);
    for (int t = 0; t < steps; ++t) {
        taus[t] = 1.0 / mus[t];
        lams[t] = lambda / mus[t];
    }
    return FRSVT_OK;
}

static int unrolled_check(frsvt_handle h, frsvt_precision prec, int32_t batch, int32_t steps, int64_t m,
                          int64_t n, const void *O, int64_t ldo, int64_t strideO, const double *taus,
                          const double *lams, int32_t k, int32_t p, int32_t q, int kpos)
{
    if (!h) return -1;
    if (prec != FRSVT_F64 && prec != FRSVT_F32) return -2;
    if (batch < 1) return -3;
    if (steps < 1) return -4;
    if (m < 1) return -5;
    if (n < 1) return -6;
    if (bad_ptr(O)) return -7;
    if (ldo < m) return -8;
    if (batch > 1 && strideO < ldo * n) return -9;
    if (bad_ptr(taus)) return -10;
    if (bad_ptr(lams)) return -11;
    if (k < 0 || k + p < 1) return -kpos;
    if (p < 0) return -(kpos + 1);
    if (q < 0 || q > 64) return -(kpos + 2);
    if (std::min<int64_t>(std::min(m, n), (int64_t)k + p) > 64) return FRSVT_ERR_UNSUPPORTED;
    if (std::min(m, n) > 1024) return FRSVT_ERR_UNSUPPORTED;
    return FRSVT_OK;
}

int rpca_unrolled_fwd(frsvt_handle h, frsvt_precision prec, int32_t batch, int32_t steps, int64_t m, int64_t n,
                      const void *O, int64_t ldo, int64_t strideO, const double *taus, const double *lams,
                      double lambda, double rho, double mu_bar_factor, int32_t k, int32_t p, int32_t q,
                      uint64_t seed, void *L, int64_t ldl, int64_t strideL, void *saved, int64_t saved_bytes)
{
    int rc = unrolled_check(h, prec, batch, steps, m, n, O, ldo, strideO, taus, lams, k, p, q, 15);
    if (rc) return rc;
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return -12;
    if (!(rho >= 1.0) || !std::isfinite(rho)) return -13;
    if (!(mu_bar_factor >= 1.0)) return -14;
    if (bad_ptr(L)) return -19;
    if (ldl < m) return -20;
    if (batch > 1 && strideL < ldl * n) return -21;
    if (bad_ptr(saved)) return -22;
    if (saved_bytes < rpca_unrolled_saved_bytes(prec, batch, steps, m, n, k, p)) return -23;
    if (prec == FRSVT_F64)
        return unrolled_fwd_impl<double>(h, batch, steps, m, n, (const double *)O, ldo, strideO, taus, lams, lambda,
                                         rho, mu_bar_factor, k, p, q, seed, (double *)L, ldl, strideL, saved);
    return unrolled_fwd_impl<float>(h, batch, steps, m, n, (const float *)O, ldo, strideO, taus, lams, lambda, rho,
                                    mu_bar_factor, k, p, q, seed, (float *)L, ldl, strideL, saved);
}

int rpca_unrolled_bwd(frsvt_handle h, frsvt_precision prec, int32_t batch, int32_t steps, int64_t m, int64_t n,
                      const void *O, int64_t ldo, int64_t strideO, const double *taus, const double *lams,
                      int32_t k, int32_t p, int32_t q, uint64_t seed, const void *saved, int64_t saved_bytes,
                      const void *L_bar, int64_t ldlb, int64_t strideLb, double *tau_bar, double *lam_bar)
{
    int rc = unrolled_check(h, prec, batch, steps, m, n, O, ldo, strideO, taus, lams, k, p, q, 12);
    if (rc) return rc;
    if (bad_ptr(saved)) return -16;
    if (saved_bytes < rpca_unrolled_saved_bytes(prec, batch, steps, m, n, k, p)) return -17;
    if (bad_ptr(L_bar)) return -18;
    if (ldlb < m) return -19;
    if (batch > 1 && strideLb < ldlb * n) return -20;
    if (bad_ptr(tau_bar)) return -21;
    if (bad_ptr(lam_bar)) return -22;
    if (prec == FRSVT_F64)
        return unrolled_bwd_impl<double>(h, batch, steps, m, n, (const double *)O, ldo, strideO, taus, lams, k, p,
                                         q, seed, saved, (const double *)L_bar, ldlb, strideLb, tau_bar, lam_bar);
    return unrolled_bwd_impl<float>(h, batch, steps, m, n, (const float *)O, ldo, strideO, taus, lams, k, p, q,
                                    seed, saved, (const float *)L_bar, ldlb, strideLb, tau_bar, lam_bar);
}

int rpca_sliding(frsvt_handle h, frsvt_precision prec, int64_t m, int64_t frames, const void *F, int64_t ldf,
                 int32_t window, double lambda, int32_t keep, int32_t l, int32_t q, uint64_t seed, double tol,
                 int32_t max_iter, double rho, void *L, int64_t ldl, void *S, int64_t lds,
                 frsvt_rpca_stats *stats, void *bases)
{
    if (!h) return -1;
    if (prec != FRSVT_F64 && prec != FRSVT_F32) return -2;
    if (m < 1) return -3;
    if (frames < 1) return -4;
    if (bad_ptr(F)) return -5;
    if (ldf < m) return -6;
    if (window < 2 || window > frames) return -7;
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return -8;
    if (keep < 1) return -9;
    if (l <= keep || l > window || l > m) return -10;
    if (q < 0 || q > 64) return -11;
    if (!(tol > 0.0)) return -13;
    if (max_iter < 1 || max_iter > 64) return -14;
    if (!(rho >= 1.0) || !std::isfinite(rho)) return -15;
    if (bad_ptr(L)) return -16;
    if (ldl < m) return -17;
    if (bad_ptr(S)) return -18;
    if (lds < m) return -19;
    if (prec == FRSVT_F64)
        return sliding_impl<double>(h, m, frames, (const double *)F, ldf, window, lambda, keep, l, q, seed, tol,
                                    max_iter, rho, (double *)L, ldl, (double *)S, lds, stats, (double *)bases);
    return sliding_impl<float>(h, m, frames, (const float *)F, ldf, window, lambda, keep, l, q, seed, tol, max_iter,
                               rho, (float *)L, ldl, (float *)S, lds, stats, (float *)bases);
}

}  // extern "C"

void frsvt_lrr_default_opts(frsvt_lrr_opts *op)
{
    if (!op) return;
    op->tol = 1e-8;
    op->max_iter = 1000;
    op->mu0 = 1e-6;
    op->rho = 1.1;
    op->mu_max = 1e10;
    op->use_frsvt = 1;
    op->p = 5;
    op->q = 1;
    op->seed = 0;
}

int lrr_ialm(frsvt_handle h, frsvt_precision prec, int64_t d, int64_t n, const void *X, int64_t ldx, double lambda,
             const frsvt_lrr_opts *opts, void *Z, int64_t ldz, void *E, int64_t lde, frsvt_lrr_stats *stats)
{
    if (!h) return -1;
    if (prec != FRSVT_F64 && prec != FRSVT_F32 && prec != FRSVT_MIXED_BF16) return -2;
    if (d < 1) return -3;
    if (n < 1) return -4;
    if (bad_ptr(X)) return -5;
    if (ldx < d) return -6;
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return -7;
    frsvt_lrr_opts op;
    frsvt_lrr_default_opts(&op);
    if (opts) op = *opts;
    if (!(op.tol > 0.0) || op.max_iter < 1 || !(op.mu0 > 0.0) || !(op.rho >= 1.0) || !(op.mu_max >= op.mu0) ||
        op.p < 1 || op.q < 0 || (op.use_frsvt != 0 && op.use_frsvt != 1))
        return -8;
    if (bad_ptr(Z)) return -9;
    if (ldz < n) return -10;
    if (bad_ptr(E)) return -11;
    if (lde < d) return -12;
    if (prec != FRSVT_F64 || n > 1024) return FRSVT_ERR_UNSUPPORTED;
    return lrr_impl(h, d, n, (const double *)X, ldx, lambda, op, (double *)Z, ldz, (double *)E, lde, stats);
}

void frsvt_tensor_default_opts(frsvt_tensor_opts *op)
{
    if (!op) return;
    memset(op, 0, sizeof(*op));
    op->tol = 1e-7;
    op->max_iter = 100;
    op->mu0 = 0.0;
    op->rho = 1.5;
    op->mu_max = 1e10;
    op->use_frsvt = 1;
    op->p = 5;
    op->q = 1;
    op->seed = 0;
}

int tensor_rpca(frsvt_handle h, frsvt_precision prec, int64_t I1, int64_t I2, int64_t I3, const void *O,
                const double *alpha, double lambda, const frsvt_tensor_opts *opts, void *L, void *E,
                frsvt_tensor_stats *stats)
{
    if (!h) return -1;
    if (prec != FRSVT_F64 && prec != FRSVT_F32 && prec != FRSVT_MIXED_BF16) return -2;
    if (I1 < 1) return -3;
    if (I2 < 1) return -4;
    if (I3 < 1) return -5;
    if (bad_ptr(O)) return -6;
    if (!alpha) return -7;
    for (int i = 0; i < 3; ++i)
        if (!(alpha[i] >= 0.0) || !std::isfinite(alpha[i])) return -7;
    if (!(lambda > 0.0) || !std::isfinite(lambda)) return -8;
    frsvt_tensor_opts op;
    frsvt_tensor_default_opts(&op);
    if (opts) op = *opts;
    if (!(op.tol > 0.0) || op.max_iter < 1 || !(op.mu0 >= 0.0) || !(op.rho >= 1.0) || !(op.mu_max > 0.0) ||
        (op.mu0 > 0.0 && op.mu_max < op.mu0) || op.p < 1 || op.q < 0 || (op.use_frsvt != 0 && op.use_frsvt != 1))
        return -9;
    if (bad_ptr(L)) return -10;
    if (bad_ptr(E)) return -11;
    if (L == E || L == O || E == O) return -11;
    if (prec != FRSVT_F64) return FRSVT_ERR_UNSUPPORTED;
    if (I1 > (int64_t)1 << 20 || I2 > (int64_t)1 << 20 || I3 > (int64_t)1 << 20) return FRSVT_ERR_UNSUPPORTED;
    if (std::min(I1, I2 * I3) > 1024 || std::min(I2, I1 * I3) > 1024 || std::min(I1 * I2, I3) > 1024)
        return FRSVT_ERR_UNSUPPORTED;
    return tensor_impl(h, I1, I2, I3, (const double *)O, alpha, lambda, op, (double *)L, (double *)E, stats);
}
