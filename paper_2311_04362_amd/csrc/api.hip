// Host side of libls: the C ABI declared in include/ls.h.  Validates arguments synchronously,
// sizes the context workspace, and enqueues the kernels of sketch.hip, qr.hip and iterate.hip on
// the caller's stream.  Device-detected conditions accumulate in a status word read by ls_sync.
#include <cmath>
#include <cstring>
#include <new>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "common.hpp"

namespace {

const char *kNullCtx = "null context";

// A named host-side range around the enqueueing of one phase, for profilers that record roctx
// markers (rocprofv3 --marker-trace); without such a profiler the calls do nothing.
struct Range {
    explicit Range(const char *name) { roctxRangePush(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range &) = delete;
    Range &operator=(const Range &) = delete;
};

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Makes the context's device current for the duration of a call and restores the caller's.
struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

ls_status check_embedding(ls_ctx *ctx, int64_t m, int64_t d, int32_t zeta)
{
    if (m < 1) return ls_fail(ctx, LS_ERR_ARG, "m must be >= 1");
    if (d < 1 || d >= (int64_t(1) << 31)) return ls_fail(ctx, LS_ERR_ARG, "d must be in [1, 2^31)");
    if (zeta < 1 || zeta > LS_MAX_ZETA || zeta > d)
        return ls_fail(ctx, LS_ERR_ARG, "zeta must be in [1, min(d, LS_MAX_ZETA)]");
    if (m * (int64_t)zeta >= (int64_t(1) << 31))
        return ls_fail(ctx, LS_ERR_UNSUPPORTED, "m*zeta must be < 2^31");
    return LS_OK;
}

ls_status check_mat(ls_ctx *ctx, const void *p, int64_t ld, int64_t n, const char *name, size_t align = 8)
{
    if (!p) return ls_fail(ctx, LS_ERR_ARG, std::string(name) + " is NULL");
    if (!aligned(p, align))
        return ls_fail(ctx, LS_ERR_ARG, std::string(name) + " is not " + std::to_string(align) + "-byte aligned");
    if (ld < n) return ls_fail(ctx, LS_ERR_ARG, std::string("leading dimension of ") + name + " < n");
    return LS_OK;
}

ls_status check_vec(ls_ctx *ctx, const void *p, const char *name, bool nullable = false, size_t align = 8)
{
    if (!p) return nullable ? LS_OK : ls_fail(ctx, LS_ERR_ARG, std::string(name) + " is NULL");
    if (!aligned(p, align))
        return ls_fail(ctx, LS_ERR_ARG, std::string(name) + " is not " + std::to_string(align) + "-byte aligned");
    return LS_OK;
}

ls_status check_n(ls_ctx *ctx, int64_t n)
{
    if (n < 1) return ls_fail(ctx, LS_ERR_ARG, "n must be >= 1");
    if (n > LS_MAX_N) return ls_fail(ctx, LS_ERR_UNSUPPORTED, "n exceeds LS_MAX_N");
    return LS_OK;
}

#define LS_TRY(expr)                   \
    do {                               \
        ls_status st_ = (expr);        \
        if (st_ != LS_OK) return st_;  \
    } while (0)

#define HIP_TRY(ctx, expr, what)                              \
    do {                                                      \
        ls_status st_ = ls_hip_check((ctx), (expr), (what));  \
        if (st_ != LS_OK) return st_;                         \
    } while (0)

ls_status need_device(ls_ctx *ctx)
{
    if (ctx->device < 0) return ls_fail(ctx, LS_ERR_DEVICE, "host-only context: no device work");
    return LS_OK;
}

// Two-pass arena: size with base == nullptr, grow the workspace, then carve for real.
template <class F>
ls_status with_arena(ls_ctx *ctx, F &&carve)
{
    Arena sizing;
    carve(sizing);
    LS_TRY(ls_ensure_ws(ctx, sizing.off + 256));
    Arena real;
    real.base = static_cast<char *>(ctx->ws);
    carve(real);
    return LS_OK;
}

ls_status do_embedding(ls_ctx *ctx, hipStream_t s, int64_t m, int64_t d, int32_t zeta, uint64_t seed,
                       const SketchBufs &sb, bool csr)
{
    HIP_TRY(ctx, launch_sparse_sign(s, m, d, zeta, seed, sb), "sparse-sign kernel");
    if (csr) HIP_TRY(ctx, launch_csr(s, m, d, zeta, sb), "CSR kernels");
    return LS_OK;
}

// Next start/end event pair for a timed pass launch (nullptr pair when profiling is off).
ls_status pass_events(ls_ctx *ctx, hipEvent_t &e0, hipEvent_t &e1)
{
    e0 = e1 = nullptr;
    if (!ctx->profile) return LS_OK;
    while (ctx->ev_pool.size() < ctx->ev_used + 2) {
        hipEvent_t e;
        // timestamps only: no system-scope fence at each record (about 5.6 us per record with it)
        HIP_TRY(ctx, hipEventCreateWithFlags(&e, hipEventDisableSystemFence), "create event");
        ctx->ev_pool.push_back(e);
    }
    e0 = ctx->ev_pool[ctx->ev_used];
    e1 = ctx->ev_pool[ctx->ev_used + 1];
    ctx->ev_used += 2;
    return LS_OK;
}

ls_status timed_gradient(ls_ctx *ctx, hipStream_t s, int64_t m, int64_t n, const double *A,
                         int64_t lda, const double *b, const double *x, const IterBufs &ib,
                         double *c, double *rnorm2)
{
    hipEvent_t e0, e1;
    LS_TRY(pass_events(ctx, e0, e1));
    HIP_TRY(ctx, launch_gradient(s, m, n, A, lda, b, x, ib, c, rnorm2, e0, e1), "pass kernels");
    return LS_OK;
}

// Principal branch of Lambert's W for y >= 0 by Halley's iteration on f(w) = w e^w - y.
double lambert_w0(double y)
{
    double w = std::log1p(y);
    for (int it = 0; it < 64; ++it) {
        const double ew = std::exp(w);
        const double f = w * ew - y;
        const double fp = ew * (w + 1.0);
        const double step = f / (fp - (w + 2.0) * f / (2.0 * w + 2.0));
        w -= step;
        if (std::fabs(step) <= 1e-15 * (1.0 + std::fabs(w))) break;
    }
    return w;
}

// Embedding dimension of eq. (dimension), u = 2^-53.
int64_t dimension_rule(int64_t m, int64_t n)
{
    const double a = 6.0 + 4.0 * std::sqrt(2.0), c = 6.0 - 4.0 * std::sqrt(2.0);
    const double y = c * ((double)m / ((double)n * (double)n)) * (53.0 * std::log(2.0));
    const int64_t d = (int64_t)std::ceil(a * (double)n * std::exp(lambert_w0(y)));
    return d > 20 * n ? d : 20 * n;
}

void update_params(const ls_ctx *ctx, int64_t n, int64_t d, int &mode, double &alpha, double &beta)
{
    mode = 1;
    alpha = 1.0;
    beta = 0.0;
    if (ctx->update == 0) return;
    const double eps2 = (d > 0) ? (double)n / (double)d : 0.0;   // eps = sqrt(n/d)
    mode = 2;
    if (ctx->update == 1) {            // damping, eq. (damping)
        alpha = (ctx->alpha > 0.0) ? ctx->alpha : (1.0 - eps2) * (1.0 - eps2) / (1.0 + eps2);
        beta = 0.0;
    } else {                           // momentum, eq. (momentum)
        alpha = (ctx->alpha > 0.0) ? ctx->alpha : (1.0 - eps2) * (1.0 - eps2);
        beta = (ctx->beta >= 0.0) ? ctx->beta : eps2;
    }
}

}  // namespace

ls_status ls_fail(ls_ctx *ctx, ls_status st, const std::string &msg)
{
    if (ctx) ctx->err = msg;
    return st;
}

ls_status ls_hip_check(ls_ctx *ctx, hipError_t e, const char *what)
{
    if (e == hipSuccess) return LS_OK;
    return ls_fail(ctx, LS_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

ls_status ls_ensure_ws(ls_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->ws_bytes) return LS_OK;
    // The old block may still be read by queued work: drain the device before releasing it.
    HIP_TRY(ctx, hipDeviceSynchronize(), "synchronize before workspace growth");
    if (ctx->ws) (void)hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    const size_t want = bytes + bytes / 4;
    void *p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return ls_fail(ctx, LS_ERR_ALLOC, "workspace allocation of " + std::to_string(bytes) + " bytes failed");
        }
        ctx->ws_bytes = bytes;
    } else {
        ctx->ws_bytes = want;
    }
    ctx->ws = p;
    return LS_OK;
}

// Refinement steps of Algorithm 2 in FP64 from x = x_0 with R (n x n, ld n) and RT = R^T: at most q
// steps (ended on the device by the stopping rule when LS_OPT_STOP is set), then waits and returns
// the deferred status.  ib must be sized for (m, n); est_work holds 3 n doubles.
static ls_status iterate_fp64(ls_ctx *ctx, hipStream_t s, int64_t m, int64_t n, const double *A,
                              int64_t lda, const double *b, int64_t d, int32_t q, double *x,
                              const double *R, const double *RT, const IterBufs &ib, double *est_work)
{
    int mode;
    double alpha, beta;
    update_params(ctx, n, d, mode, alpha, beta);
    StopArgs st;
    if (ctx->stop) {
        HIP_TRY(ctx, launch_estimators(s, n, R, n, RT, ctx->seed + kEstimatorSeedOffset, est_work, ib.scal), "estimators");
        HIP_TRY(ctx, launch_stop_init(s, ib.state), "stop init");
        st.state = ib.state;
        st.scal = ib.scal;
        st.dx = ib.dx;
        st.gamma = ctx->gamma;
        st.rho = ctx->rho;
    }
    if (mode == 2 && q > 0)
        HIP_TRY(ctx, hipMemcpyAsync(ib.xprev, x, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s), "copy x");
    for (int32_t i = 0; i < q; ++i) {
        if (ctx->stop) {
            st.check = (i >= 1);
            hipEvent_t e0, e1;
            LS_TRY(pass_events(ctx, e0, e1));
            HIP_TRY(ctx, launch_gradient(s, m, n, A, lda, b, x, ib, ib.c, ib.scal, e0, e1,
                                         i >= 1 ? ib.dx : nullptr, ib.scal + 1, ib.state), "pass kernels");
        } else {
            LS_TRY(timed_gradient(ctx, s, m, n, A, lda, b, x, ib, ib.c, nullptr));
        }
        HIP_TRY(ctx, launch_solve_update(s, n, R, n, RT, ib.c, x, ib.xprev, nullptr, mode, alpha, beta, ctx->status, st), "solve kernel");
    }
    const ls_status status = ls_sync(ctx, s);
    if (ctx->stop) {
        int32_t stv[2];
        double scv[4];
        HIP_TRY(ctx, hipMemcpy(stv, ib.state, sizeof(stv), hipMemcpyDeviceToHost), "read steps");
        HIP_TRY(ctx, hipMemcpy(scv, ib.scal, sizeof(scv), hipMemcpyDeviceToHost), "read estimates");
        ctx->last_steps = stv[1];
        ctx->last_normest = scv[2];
        ctx->last_condest = scv[3];
    }
    return status;
}

static void release_aside(QrAside &la)
{
    if (la.panel_done) (void)hipEventDestroy(la.panel_done);
    if (la.side_done) (void)hipEventDestroy(la.side_done);
    if (la.side) (void)hipStreamDestroy(la.side);
    la = QrAside{};
}

// The context's QR look-ahead for a d x n factorization, or null: on the per-column panel path,
// where it does not pay, or if its stream cannot be made.  The side stream (default priority) and
// its two events are created on the first factorization that uses them, so contexts that never
// factor a large sketch hold no second stream (a process has few hardware queues to share).
static const QrAside *qr_aside(ls_ctx *ctx, int64_t d, int64_t n)
{
    if (ctx->qr_panel == 1 || !qr_lookahead_pays(d, n) || ctx->device < 0) return nullptr;
    if (!ctx->qla.side) {
        DeviceGuard g(ctx->device);
        if (!g.ok || hipStreamCreateWithFlags(&ctx->qla.side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ctx->qla.panel_done, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&ctx->qla.side_done, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            release_aside(ctx->qla);
            return nullptr;
        }
    }
    return &ctx->qla;
}

// Algorithm 2 in FP64 (the body of ls_solve).
static ls_status solve_fp64(ls_ctx *ctx, hipStream_t s, int64_t m, int64_t n, const double *A, int64_t lda,
                            const double *b, int64_t d, int32_t q, double *x)
{
    const int32_t zeta = ctx->zeta;
    SketchBufs sb{};
    QrBufs qb{};
    IterBufs ib{};
    double *R = nullptr, *est_work = nullptr;
    const QrAside *la = qr_aside(ctx, d, n);   // decided once: sizing and carve agree
    LS_TRY(with_arena(ctx, [&](Arena &ar) {
        sketch_bufs(ar, m, d, zeta, sb, n, ctx->gather);
        qr_bufs(ar, d, n, qb, la != nullptr);
        iter_bufs(ar, m, n, ib, false);
        R = ar.take<double>((size_t)n * (size_t)n);
        est_work = ar.take<double>((size_t)3 * (size_t)n);
    }));
    // (a) sketch straight into the QR work matrix: B in columns 0..n-1, S b in column n.
    {
        Range r("ls_solve: sketch");
        LS_TRY(do_embedding(ctx, s, m, d, zeta, ctx->seed, sb, true));
        const double scale = 1.0 / std::sqrt((double)zeta);
        HIP_TRY(ctx, launch_gather(s, d, n, A, lda, b, sb.rowptr, sb.cols, scale, qb.W, qb.ldw, qb.W + n, qb.ldw, &sb.win), "gather kernel");
    }
    // (b) QR of [B | S b], R and Q^T S b, x0 = R^{-1} (Q^T S b)[0:n].
    {
        Range r("ls_solve: QR and x0");
        HIP_TRY(ctx, launch_qr(s, d, n, qb, ctx->status, ctx->qr_panel == 1, la), "QR kernels");
        HIP_TRY(ctx, launch_extract_r(s, n, qb, R, n, ctx->status), "extract R");
        HIP_TRY(ctx, launch_back_substitution(s, n, R, n, qb.RT, qb.qtb, x, ctx->status), "x0 solve");
    }
    // (c) q refinement steps (with the stopping rule: at most q, ended on the device).
    Range r("ls_solve: refinement");
    return iterate_fp64(ctx, s, m, n, A, lda, b, d, q, x, R, qb.RT, ib, est_work);
}

// Refinement steps of the mixed-precision sketch-and-solve start: the contraction of
// x <- x + R32^{-1} R32^{-T} B^T (S b - B x) on the FP64 sketch is about 2 condest u_32, so
// ceil(ln(1e-9) / ln(2 condest u_32)) steps, clamped to [2, 8], take the FP32 solution (about
// 1e-7 relative) to FP64 accuracy.
int32_t mixed_start_steps(double condest)
{
    const double rho = 2.0 * condest * 0x1p-24;
    if (!(rho > 0.0)) return 2;
    if (rho >= 0.5) return 8;
    const double k = std::ceil(std::log(1e-9) / std::log(rho));
    return k < 2.0 ? 2 : (k > 8.0 ? 8 : (int32_t)k);
}

// Algorithm 2 with the FP32 sketch, QR and R-solves of the mixed-precision variant; the A^T (b-Ax)
// pass and the update stay FP64.  The sketch is formed once in FP64 and rounded for the FP32 QR, so
// the sketch-and-solve start can be refined on it in FP64 (eq. sketched_ls defines x_0 exactly) and
// a fallback factors it in FP64 without sketching again.  Falls back when condest(R32) u_32 > 0.05
// or the FP32 QR flags R (after the QR, on the host: one wait), or when ||r||^2 grows three steps
// in a row (on the device, read at the end).  Sets `used` and leaves the final status to the caller.
static ls_status solve_mixed(ls_ctx *ctx, hipStream_t s, int64_t m, int64_t n, const double *A,
                             int64_t lda, const double *b, int64_t d, int32_t q, double *x, int32_t &used)
{
    const int32_t zeta = ctx->zeta;
    SketchBufs sb{};
    QrBufs qb64{};
    QrBufs32 qb{};
    IterBufs ib{}, ibs{};
    float *R = nullptr, *est_work = nullptr;
    double *Sb = nullptr, *R64 = nullptr, *est64 = nullptr;
    const QrAside *la = qr_aside(ctx, d, n);   // decided once: sizing and carve agree
    LS_TRY(with_arena(ctx, [&](Arena &ar) {
        sketch_bufs(ar, m, d, zeta, sb, n, ctx->gather);
        qr_bufs(ar, d, n, qb64, la != nullptr);
        qr_bufs(ar, d, n, qb, la != nullptr);
        iter_bufs(ar, m, n, ib, false);
        iter_bufs(ar, d, n, ibs, false);
        R = ar.take<float>((size_t)n * (size_t)n);
        est_work = ar.take<float>((size_t)3 * (size_t)n);
        Sb = ar.take<double>((size_t)d);
        R64 = ar.take<double>((size_t)n * (size_t)n);
        est64 = ar.take<double>((size_t)3 * (size_t)n);
    }));
    // (a) FP64 sketch: B in the FP64 work matrix, S b contiguous; rounded copy for the FP32 QR.
    Range r_all("ls_solve: mixed precision");
    LS_TRY(do_embedding(ctx, s, m, d, zeta, ctx->seed, sb, true));
    const double scale = 1.0 / std::sqrt((double)zeta);
    HIP_TRY(ctx, launch_gather(s, d, n, A, lda, b, sb.rowptr, sb.cols, scale, qb64.W, qb64.ldw, Sb, 1, &sb.win), "gather kernel");
    HIP_TRY(ctx, launch_round_sketch(s, d, n, qb64, Sb, qb), "round sketch");
    // (b) FP32 QR, R, the FP32 start, FP32 estimators; the fallback decision on the host.
    HIP_TRY(ctx, launch_qr(s, d, n, qb, ctx->status, ctx->qr_panel == 1, la), "QR kernels");
    HIP_TRY(ctx, launch_extract_r(s, n, qb, R, n, ctx->status), "extract R");
    HIP_TRY(ctx, launch_back_substitution(s, n, R, n, qb.RT, qb.qtb, x, ctx->status), "x0 solve");
    HIP_TRY(ctx, launch_estimators(s, n, R, n, qb.RT, ctx->seed + kEstimatorSeedOffset, est_work, ib.scal), "estimators");
    double scv[4];
    HIP_TRY(ctx, hipMemcpyAsync(ctx->status_host, ctx->status, sizeof(int32_t), hipMemcpyDeviceToHost, s), "read status");
    HIP_TRY(ctx, hipMemcpyAsync(scv, ib.scal, sizeof(scv), hipMemcpyDeviceToHost, s), "read estimates");
    HIP_TRY(ctx, hipStreamSynchronize(s), "stream synchronize");
    ctx->last_normest = scv[2];
    ctx->last_condest = scv[3];
    const int32_t st0 = *ctx->status_host;
    // FP64 solve from the FP64 sketch (the fallback): set S b as column n, factor, iterate.
    auto fallback = [&](int32_t why) -> ls_status {
        used = why;
        ctx->last_steps = q;
        HIP_TRY(ctx, hipMemsetAsync(ctx->status, 0, sizeof(int32_t), s), "clear status");
        HIP_TRY(ctx, launch_set_rhs(s, d, n, Sb, qb64), "set rhs");
        HIP_TRY(ctx, launch_qr(s, d, n, qb64, ctx->status, ctx->qr_panel == 1, la), "QR kernels");
        HIP_TRY(ctx, launch_extract_r(s, n, qb64, R64, n, ctx->status), "extract R");
        HIP_TRY(ctx, launch_back_substitution(s, n, R64, n, qb64.RT, qb64.qtb, x, ctx->status), "x0 solve");
        return iterate_fp64(ctx, s, m, n, A, lda, b, d, q, x, R64, qb64.RT, ib, est64);
    };
    if ((st0 & (ST_RANK | ST_NONFINITE)) || !(scv[3] * 0x1p-24 <= 0.05)) return fallback(LS_PRECISION_FELL_BACK_COND);
    // (c) the start to FP64 accuracy on the FP64 sketch (B still intact in qb64.W).
    const int32_t k0 = mixed_start_steps(scv[3]);
    for (int32_t k = 0; k < k0; ++k) {
        HIP_TRY(ctx, launch_gradient(s, d, n, qb64.W, qb64.ldw, Sb, x, ibs, ibs.c, nullptr), "start pass");
        HIP_TRY(ctx, launch_solve_update(s, n, R, n, qb.RT, ibs.c, x, nullptr, nullptr, 1, 1.0, 0.0, ctx->status), "start solve");
    }
    // (d) q refinement steps: FP64 pass, FP32 solves, FP64 update, growth monitor on the device.
    int mode;
    double alpha, beta;
    update_params(ctx, n, d, mode, alpha, beta);
    HIP_TRY(ctx, launch_stop_init(s, ib.state), "stop init");
    StopArgs st;
    st.state = ib.state;
    st.scal = ib.scal;
    st.dx = ib.dx;
    st.gamma = ctx->gamma;
    st.rho = ctx->rho;
    st.grow = 1;
    if (mode == 2 && q > 0)
        HIP_TRY(ctx, hipMemcpyAsync(ib.xprev, x, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s), "copy x");
    for (int32_t i = 0; i < q; ++i) {
        const bool check = ctx->stop && i >= 1;
        st.check = check;
        hipEvent_t e0, e1;
        LS_TRY(pass_events(ctx, e0, e1));
        HIP_TRY(ctx, launch_gradient(s, m, n, A, lda, b, x, ib, ib.c, ib.scal, e0, e1,
                                     check ? ib.dx : nullptr, ib.scal + 1, ib.state), "pass kernels");
        HIP_TRY(ctx, launch_solve_update(s, n, R, n, qb.RT, ib.c, x, ib.xprev, nullptr, mode, alpha, beta, ctx->status, st), "solve kernel");
    }
    int32_t stv[4];
    HIP_TRY(ctx, hipMemcpyAsync(stv, ib.state, sizeof(stv), hipMemcpyDeviceToHost, s), "read steps");
    HIP_TRY(ctx, hipStreamSynchronize(s), "stream synchronize");
    ctx->last_steps = stv[1];
    if (stv[2]) return fallback(LS_PRECISION_FELL_BACK_GROWTH);
    used = LS_PRECISION_MIXED;
    return ls_sync(ctx, s);
}

extern "C" {

ls_status ls_limits(int32_t *max_zeta, int32_t *max_n)
{
    if (max_zeta) *max_zeta = LS_MAX_ZETA;
    if (max_n) *max_n = LS_MAX_N;
    return LS_OK;
}

ls_status ls_create(int device, ls_ctx **out)
{
    if (!out) return LS_ERR_ARG;
    *out = nullptr;
    ls_ctx *ctx = new (std::nothrow) ls_ctx;
    if (!ctx) return LS_ERR_ALLOC;
    if (device == -1) {
        *out = ctx;
        return LS_OK;
    }
    int count = 0;
    if (device < 0 || hipGetDeviceCount(&count) != hipSuccess || device >= count) {
        (void)hipGetLastError();
        delete ctx;
        return LS_ERR_DEVICE;
    }
    ctx->device = device;
    DeviceGuard g(device);
    if (!g.ok || hipMalloc(&ctx->status, sizeof(int32_t)) != hipSuccess ||
        hipMemset(ctx->status, 0, sizeof(int32_t)) != hipSuccess ||
        hipHostMalloc(&ctx->status_host, sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        if (ctx->status) (void)hipFree(ctx->status);
        delete ctx;
        return LS_ERR_DEVICE;
    }
    if (pass_scratch_attach(ctx) != LS_OK) {
        (void)hipFree(ctx->status);
        (void)hipHostFree(ctx->status_host);
        delete ctx;
        return LS_ERR_DEVICE;
    }
    *out = ctx;
    return LS_OK;
}

void ls_destroy(ls_ctx *ctx)
{
    if (!ctx) return;
    if (ctx->device >= 0) {
        DeviceGuard g(ctx->device);
        (void)hipDeviceSynchronize();
        if (ctx->ws) (void)hipFree(ctx->ws);
        if (ctx->status) (void)hipFree(ctx->status);
        if (ctx->status_host) (void)hipHostFree(ctx->status_host);
        for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
        release_aside(ctx->qla);
    }
    delete ctx;
}

const char *ls_last_error(const ls_ctx *ctx)
{
    if (!ctx) return kNullCtx;
    return ctx->err.c_str();
}

ls_status ls_set_option(ls_ctx *ctx, int key, int64_t ival, double dval)
{
    if (!ctx) return LS_ERR_ARG;
    switch (key) {
    case LS_OPT_ZETA:
        if (ival < 1 || ival > LS_MAX_ZETA) return ls_fail(ctx, LS_ERR_ARG, "zeta out of range");
        ctx->zeta = (int32_t)ival;
        return LS_OK;
    case LS_OPT_SEED: ctx->seed = (uint64_t)ival; return LS_OK;
    case LS_OPT_UPDATE:
        if (ival < 0 || ival > 2) return ls_fail(ctx, LS_ERR_ARG, "update must be 0, 1 or 2");
        ctx->update = (int32_t)ival;
        return LS_OK;
    case LS_OPT_ALPHA:
        if (!std::isfinite(dval)) return ls_fail(ctx, LS_ERR_ARG, "alpha must be finite");
        ctx->alpha = dval;
        return LS_OK;
    case LS_OPT_BETA:
        if (!std::isfinite(dval)) return ls_fail(ctx, LS_ERR_ARG, "beta must be finite");
        ctx->beta = dval;
        return LS_OK;
    case LS_OPT_PRECISION:
        if (ival != 0 && ival != 1) return ls_fail(ctx, LS_ERR_ARG, "precision must be 0 (FP64) or 1 (mixed)");
        ctx->precision = (int32_t)ival;
        return LS_OK;
    case LS_OPT_PROFILE:
        if (ival != 0 && ival != 1) return ls_fail(ctx, LS_ERR_ARG, "profile must be 0 or 1");
        ctx->profile = (int32_t)ival;
        return LS_OK;
    case LS_OPT_QR_PANEL:
        if (ival != 0 && ival != 1) return ls_fail(ctx, LS_ERR_ARG, "QR panel mode must be 0 or 1");
        ctx->qr_panel = (int32_t)ival;
        return LS_OK;
    case LS_OPT_GATHER:
        if (ival != 0 && ival != 1) return ls_fail(ctx, LS_ERR_ARG, "gather mode must be 0 or 1");
        ctx->gather = (int32_t)ival;
        return LS_OK;
    case LS_OPT_STOP:
        if (ival != 0 && ival != 1) return ls_fail(ctx, LS_ERR_ARG, "stop must be 0 or 1");
        ctx->stop = (int32_t)ival;
        return LS_OK;
    case LS_OPT_GAMMA:
        if (!(dval >= 0.0) || !std::isfinite(dval)) return ls_fail(ctx, LS_ERR_ARG, "gamma must be finite and >= 0");
        ctx->gamma = dval;
        return LS_OK;
    case LS_OPT_RHO:
        if (!(dval >= 0.0) || !std::isfinite(dval)) return ls_fail(ctx, LS_ERR_ARG, "rho must be finite and >= 0");
        ctx->rho = dval;
        return LS_OK;
    default: return ls_fail(ctx, LS_ERR_ARG, "unknown option key");
    }
}

ls_status ls_get_option(const ls_ctx *ctx, int key, int64_t *ival, double *dval)
{
    if (!ctx) return LS_ERR_ARG;
    int64_t iv = 0;
    double dv = 0.0;
    switch (key) {
    case LS_OPT_ZETA: iv = ctx->zeta; break;
    case LS_OPT_SEED: iv = (int64_t)ctx->seed; break;
    case LS_OPT_UPDATE: iv = ctx->update; break;
    case LS_OPT_ALPHA: dv = ctx->alpha; break;
    case LS_OPT_BETA: dv = ctx->beta; break;
    case LS_OPT_PRECISION: iv = ctx->precision; break;
    case LS_OPT_PROFILE: iv = ctx->profile; break;
    case LS_OPT_QR_PANEL: iv = ctx->qr_panel; break;
    case LS_OPT_GATHER: iv = ctx->gather; break;
    case LS_OPT_STOP: iv = ctx->stop; break;
    case LS_OPT_GAMMA: dv = ctx->gamma; break;
    case LS_OPT_RHO: dv = ctx->rho; break;
    default: return LS_ERR_ARG;
    }
    if (ival) *ival = iv;
    if (dval) *dval = dv;
    return LS_OK;
}

ls_status ls_sketch_embedding(ls_ctx *ctx, void *stream, int64_t m, int64_t d, int32_t zeta,
                              uint64_t seed, int32_t *rows, int8_t *signs)
{
    if (!ctx) return LS_ERR_ARG;
    Range range_("ls_sketch_embedding");
    LS_TRY(check_embedding(ctx, m, d, zeta));
    if (!rows || !signs || !aligned(rows, 4)) return ls_fail(ctx, LS_ERR_ARG, "rows/signs NULL or misaligned");
    LS_TRY(need_device(ctx));
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    SketchBufs sb{};
    LS_TRY(with_arena(ctx, [&](Arena &ar) { sketch_bufs(ar, m, d, zeta, sb); }));
    LS_TRY(do_embedding(ctx, s, m, d, zeta, seed, sb, false));
    HIP_TRY(ctx, launch_unpack_embedding(s, m, zeta, sb.ent, rows, signs), "unpack kernel");
    return LS_OK;
}

ls_status ls_sketch_csr(ls_ctx *ctx, void *stream, int64_t m, int64_t d, int32_t zeta, uint64_t seed,
                        int32_t *rowptr, int32_t *cols)
{
    if (!ctx) return LS_ERR_ARG;
    Range range_("ls_sketch_csr");
    LS_TRY(check_embedding(ctx, m, d, zeta));
    if (!rowptr || !cols || !aligned(rowptr, 4) || !aligned(cols, 4))
        return ls_fail(ctx, LS_ERR_ARG, "rowptr/cols NULL or misaligned");
    LS_TRY(need_device(ctx));
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    SketchBufs sb{};
    LS_TRY(with_arena(ctx, [&](Arena &ar) { sketch_bufs(ar, m, d, zeta, sb); }));
    LS_TRY(do_embedding(ctx, s, m, d, zeta, seed, sb, true));
    HIP_TRY(ctx, hipMemcpyAsync(rowptr, sb.rowptr, sizeof(int32_t) * (size_t)(d + 1), hipMemcpyDeviceToDevice, s), "copy rowptr");
    HIP_TRY(ctx, hipMemcpyAsync(cols, sb.cols, sizeof(int32_t) * (size_t)(m * zeta), hipMemcpyDeviceToDevice, s), "copy cols");
    return LS_OK;
}

ls_status ls_sketch(ls_ctx *ctx, void *stream, int64_t m, int64_t n, const double *A, int64_t lda,
                    const double *b, int64_t d, int32_t zeta, uint64_t seed, double *B, int64_t ldb,
                    double *Sb)
{
    if (!ctx) return LS_ERR_ARG;
    Range range_("ls_sketch");
    LS_TRY(check_n(ctx, n));
    LS_TRY(check_embedding(ctx, m, d, zeta));
    LS_TRY(check_mat(ctx, A, lda, n, "A"));
    LS_TRY(check_mat(ctx, B, ldb, n, "B"));
    if ((b == nullptr) != (Sb == nullptr)) return ls_fail(ctx, LS_ERR_ARG, "b and Sb must both be given or both NULL");
    LS_TRY(check_vec(ctx, b, "b", true));
    LS_TRY(check_vec(ctx, Sb, "Sb", true));
    LS_TRY(need_device(ctx));
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    SketchBufs sb{};
    LS_TRY(with_arena(ctx, [&](Arena &ar) { sketch_bufs(ar, m, d, zeta, sb, n, ctx->gather); }));
    LS_TRY(do_embedding(ctx, s, m, d, zeta, seed, sb, true));
    const double scale = 1.0 / std::sqrt((double)zeta);
    HIP_TRY(ctx, launch_gather(s, d, n, A, lda, b, sb.rowptr, sb.cols, scale, B, ldb, Sb, 1, &sb.win), "gather kernel");
    return LS_OK;
}

ls_status ls_qr_sketch(ls_ctx *ctx, void *stream, int64_t d, int64_t n, const double *B, int64_t ldb,
                       const double *Sb, double *R, int64_t ldr, double *x0)
{
    if (!ctx) return LS_ERR_ARG;
    Range range_("ls_qr_sketch");
    LS_TRY(check_n(ctx, n));
    if (d < n) return ls_fail(ctx, LS_ERR_ARG, "d must be >= n");
    LS_TRY(check_mat(ctx, B, ldb, n, "B"));
    LS_TRY(check_vec(ctx, Sb, "Sb"));
    LS_TRY(check_mat(ctx, R, ldr, n, "R"));
    LS_TRY(check_vec(ctx, x0, "x0", true));
    LS_TRY(need_device(ctx));
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    QrBufs qb{};
    const QrAside *la = qr_aside(ctx, d, n);   // decided once: sizing and carve agree
    LS_TRY(with_arena(ctx, [&](Arena &ar) { qr_bufs(ar, d, n, qb, la != nullptr); }));
    HIP_TRY(ctx, launch_copy_sketch(s, d, n, B, ldb, Sb, qb), "copy sketch");
    HIP_TRY(ctx, launch_qr(s, d, n, qb, ctx->status, ctx->qr_panel == 1, la), "QR kernels");
    HIP_TRY(ctx, launch_extract_r(s, n, qb, R, ldr, ctx->status), "extract R");
    if (x0) HIP_TRY(ctx, launch_back_substitution(s, n, R, ldr, qb.RT, qb.qtb, x0, ctx->status), "x0 solve");
    return LS_OK;
}

ls_status ls_gradient(ls_ctx *ctx, void *stream, int64_t m, int64_t n, const double *A, int64_t lda,
                      const double *b, const double *x, double *c, double *rnorm2)
{
    if (!ctx) return LS_ERR_ARG;
    Range range_("ls_gradient");
    LS_TRY(check_n(ctx, n));
    if (m < 1) return ls_fail(ctx, LS_ERR_ARG, "m must be >= 1");
    LS_TRY(check_mat(ctx, A, lda, n, "A"));
    LS_TRY(check_vec(ctx, b, "b"));
    LS_TRY(check_vec(ctx, x, "x"));
    LS_TRY(check_vec(ctx, c, "c"));
    LS_TRY(check_vec(ctx, rnorm2, "rnorm2", true));
    LS_TRY(need_device(ctx));
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    IterBufs ib{};
    LS_TRY(with_arena(ctx, [&](Arena &ar) { iter_bufs(ar, m, n, ib, false); }));
    LS_TRY(timed_gradient(ctx, s, m, n, A, lda, b, x, ib, c, rnorm2));
    return LS_OK;
}

ls_status ls_gradient_noalloc(ls_ctx *ctx, void *stream, int64_t m, int64_t n, const double *A,
                              int64_t lda, const double *b, const double *x, double *c, double *rnorm2)
{
    if (!ctx) return LS_ERR_ARG;
    LS_TRY(check_n(ctx, n));
    if (m < 1) return ls_fail(ctx, LS_ERR_ARG, "m must be >= 1");
    LS_TRY(check_mat(ctx, A, lda, n, "A"));
    LS_TRY(check_vec(ctx, b, "b"));
    LS_TRY(check_vec(ctx, x, "x"));
    LS_TRY(check_vec(ctx, c, "c"));
    LS_TRY(check_vec(ctx, rnorm2, "rnorm2", true));
    LS_TRY(need_device(ctx));
    if (!ctx->scratch) return ls_fail(ctx, LS_ERR_DEVICE, "no scratch address for this device");
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    // The same carve as ls_gradient (same P, hence the same kernels and bits), over the fixed array.
    IterBufs ib{};
    Arena sizing;
    iter_bufs(sizing, m, n, ib, false);
    if (sizing.off > kNoAllocScratchBytes)
        return ls_fail(ctx, LS_ERR_UNSUPPORTED, "pass partials of " + std::to_string(sizing.off) +
                                                    " bytes exceed the " + std::to_string(kNoAllocScratchBytes) +
                                                    "-byte scratch");
    Arena real;
    real.base = static_cast<char *>(ctx->scratch);
    iter_bufs(real, m, n, ib, false);
    HIP_TRY(ctx, launch_gradient(s, m, n, A, lda, b, x, ib, c, rnorm2), "pass kernels");
    return LS_OK;
}

ls_status ls_precond_solve(ls_ctx *ctx, void *stream, int64_t n, const double *R, int64_t ldr,
                           const double *c, double *d)
{
    if (!ctx) return LS_ERR_ARG;
    Range range_("ls_precond_solve");
    LS_TRY(check_n(ctx, n));
    LS_TRY(check_mat(ctx, R, ldr, n, "R"));
    LS_TRY(check_vec(ctx, c, "c"));
    LS_TRY(check_vec(ctx, d, "d"));
    LS_TRY(need_device(ctx));
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    double *RT = nullptr, *Rc = nullptr;
    LS_TRY(with_arena(ctx, [&](Arena &ar) {
        RT = ar.take<double>((size_t)n * (size_t)n);
        Rc = ar.take<double>((size_t)n * (size_t)n);
    }));
    // R^T for the back substitution, and R again with leading dimension n (the substitution
    // kernels address 32 rows of R from one descriptor)
    HIP_TRY(ctx, launch_transpose(s, n, R, ldr, RT), "transpose R");
    HIP_TRY(ctx, launch_compact_upper(s, n, R, ldr, Rc), "compact R");
    HIP_TRY(ctx, launch_solve_update(s, n, Rc, n, RT, c, nullptr, nullptr, d, 0, 0.0, 0.0, ctx->status), "solve kernel");
    return LS_OK;
}

ls_status ls_sketch_f32(ls_ctx *ctx, void *stream, int64_t m, int64_t n, const double *A, int64_t lda,
                        const double *b, int64_t d, int32_t zeta, uint64_t seed, float *B, int64_t ldb,
                        float *Sb)
{
    if (!ctx) return LS_ERR_ARG;
    Range range_("ls_sketch_f32");
    LS_TRY(check_n(ctx, n));
    LS_TRY(check_embedding(ctx, m, d, zeta));
    LS_TRY(check_mat(ctx, A, lda, n, "A"));
    LS_TRY(check_mat(ctx, B, ldb, n, "B", 4));
    if ((b == nullptr) != (Sb == nullptr)) return ls_fail(ctx, LS_ERR_ARG, "b and Sb must both be given or both NULL");
    LS_TRY(check_vec(ctx, b, "b", true));
    LS_TRY(check_vec(ctx, Sb, "Sb", true, 4));
    LS_TRY(need_device(ctx));
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    SketchBufs sb{};
    LS_TRY(with_arena(ctx, [&](Arena &ar) { sketch_bufs(ar, m, d, zeta, sb, n, ctx->gather); }));
    LS_TRY(do_embedding(ctx, s, m, d, zeta, seed, sb, true));
    const double scale = 1.0 / std::sqrt((double)zeta);
    HIP_TRY(ctx, launch_gather(s, d, n, A, lda, b, sb.rowptr, sb.cols, scale, B, ldb, Sb, 1, &sb.win), "gather kernel");
    return LS_OK;
}

ls_status ls_qr_sketch_f32(ls_ctx *ctx, void *stream, int64_t d, int64_t n, const float *B,
                           int64_t ldb, const float *Sb, float *R, int64_t ldr, double *x0)
{
    if (!ctx) return LS_ERR_ARG;
    Range range_("ls_qr_sketch_f32");
    LS_TRY(check_n(ctx, n));
    if (d < n) return ls_fail(ctx, LS_ERR_ARG, "d must be >= n");
    LS_TRY(check_mat(ctx, B, ldb, n, "B", 4));
    LS_TRY(check_vec(ctx, Sb, "Sb", false, 4));
    LS_TRY(check_mat(ctx, R, ldr, n, "R", 4));
    LS_TRY(check_vec(ctx, x0, "x0", true));
    LS_TRY(need_device(ctx));
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    QrBufs32 qb{};
    const QrAside *la = qr_aside(ctx, d, n);   // decided once: sizing and carve agree
    LS_TRY(with_arena(ctx, [&](Arena &ar) { qr_bufs(ar, d, n, qb, la != nullptr); }));
    HIP_TRY(ctx, launch_copy_sketch(s, d, n, B, ldb, Sb, qb), "copy sketch");
    HIP_TRY(ctx, launch_qr(s, d, n, qb, ctx->status, ctx->qr_panel == 1, la), "QR kernels");
    HIP_TRY(ctx, launch_extract_r(s, n, qb, R, ldr, ctx->status), "extract R");
    if (x0) HIP_TRY(ctx, launch_back_substitution(s, n, (const float *)R, ldr, qb.RT, qb.qtb, x0, ctx->status), "x0 solve");
    return LS_OK;
}

ls_status ls_precond_solve_f32(ls_ctx *ctx, void *stream, int64_t n, const float *R, int64_t ldr,
                               const double *c, double *d)
{
    if (!ctx) return LS_ERR_ARG;
    Range range_("ls_precond_solve_f32");
    LS_TRY(check_n(ctx, n));
    LS_TRY(check_mat(ctx, R, ldr, n, "R", 4));
    LS_TRY(check_vec(ctx, c, "c"));
    LS_TRY(check_vec(ctx, d, "d"));
    LS_TRY(need_device(ctx));
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    float *RT = nullptr, *Rc = nullptr;
    LS_TRY(with_arena(ctx, [&](Arena &ar) {
        RT = ar.take<float>((size_t)n * (size_t)n);
        Rc = ar.take<float>((size_t)n * (size_t)n);
    }));
    HIP_TRY(ctx, launch_transpose(s, n, R, ldr, RT), "transpose R");
    HIP_TRY(ctx, launch_compact_upper(s, n, R, ldr, Rc), "compact R");
    HIP_TRY(ctx, launch_solve_update(s, n, (const float *)Rc, n, (const float *)RT, c, nullptr, nullptr, d, 0, 0.0, 0.0, ctx->status), "solve kernel");
    return LS_OK;
}

ls_status ls_iterate(ls_ctx *ctx, void *stream, int64_t m, int64_t n, const double *A, int64_t lda,
                     const double *b, const double *R, int64_t ldr, double *x, int32_t q,
                     double *rnorm2)
{
    if (!ctx) return LS_ERR_ARG;
    Range range_("ls_iterate");
    LS_TRY(check_n(ctx, n));
    if (m < 1) return ls_fail(ctx, LS_ERR_ARG, "m must be >= 1");
    if (q < 0) return ls_fail(ctx, LS_ERR_ARG, "q must be >= 0");
    LS_TRY(check_mat(ctx, A, lda, n, "A"));
    LS_TRY(check_vec(ctx, b, "b"));
    LS_TRY(check_mat(ctx, R, ldr, n, "R"));
    LS_TRY(check_vec(ctx, x, "x"));
    LS_TRY(check_vec(ctx, rnorm2, "rnorm2", true));
    if (ctx->update != 0 && !(ctx->alpha > 0.0))
        return ls_fail(ctx, LS_ERR_ARG, "damping/momentum in ls_iterate needs LS_OPT_ALPHA (and LS_OPT_BETA)");
    LS_TRY(need_device(ctx));
    if (q == 0) return LS_OK;
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    IterBufs ib{};
    double *Rc = nullptr;
    LS_TRY(with_arena(ctx, [&](Arena &ar) {
        iter_bufs(ar, m, n, ib, true);
        Rc = ar.take<double>((size_t)n * (size_t)n);
    }));
    int mode;
    double alpha, beta;
    update_params(ctx, n, 0, mode, alpha, beta);
    if (ctx->update == 2 && ctx->beta < 0.0) return ls_fail(ctx, LS_ERR_ARG, "momentum in ls_iterate needs LS_OPT_BETA");
    HIP_TRY(ctx, launch_transpose(s, n, R, ldr, ib.RT), "transpose R");
    HIP_TRY(ctx, launch_compact_upper(s, n, R, ldr, Rc), "compact R");
    if (mode == 2)
        HIP_TRY(ctx, hipMemcpyAsync(ib.xprev, x, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s), "copy x");
    for (int32_t i = 0; i < q; ++i) {
        LS_TRY(timed_gradient(ctx, s, m, n, A, lda, b, x, ib, ib.c, rnorm2 ? rnorm2 + i : nullptr));
        HIP_TRY(ctx, launch_solve_update(s, n, (const double *)Rc, n, ib.RT, ib.c, x, ib.xprev, nullptr, mode, alpha, beta, ctx->status), "solve kernel");
    }
    return LS_OK;
}

ls_status ls_solve(ls_ctx *ctx, void *stream, int64_t m, int64_t n, const double *A, int64_t lda,
                   const double *b, int64_t d, int32_t q, double *x)
{
    if (!ctx) return LS_ERR_ARG;
    Range range_("ls_solve");
    LS_TRY(check_n(ctx, n));
    if (m < n) return ls_fail(ctx, LS_ERR_ARG, "m must be >= n");
    if (d <= 0) d = dimension_rule(m, n);
    if (d < n) return ls_fail(ctx, LS_ERR_ARG, "d must be >= n");
    if (q < 0) return ls_fail(ctx, LS_ERR_ARG, "q must be >= 0");
    LS_TRY(check_embedding(ctx, m, d, ctx->zeta));
    LS_TRY(check_mat(ctx, A, lda, n, "A"));
    LS_TRY(check_vec(ctx, b, "b"));
    LS_TRY(check_vec(ctx, x, "x"));
    LS_TRY(need_device(ctx));
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    ctx->last_d = d;
    ctx->last_q = q;
    ctx->last_steps = q;
    ctx->last_normest = ctx->last_condest = NAN;
    ctx->last_precision = LS_PRECISION_FP64;
    if (ctx->precision == 1) {
        int32_t used = LS_PRECISION_MIXED;
        const ls_status st = solve_mixed(ctx, s, m, n, A, lda, b, d, q, x, used);
        ctx->last_precision = used;
        return st;
    }
    return solve_fp64(ctx, s, m, n, A, lda, b, d, q, x);
}

ls_status ls_solve_info(ls_ctx *ctx, int64_t *d_used, int32_t *steps, double *normest, double *condest,
                        int32_t *precision)
{
    if (!ctx) return LS_ERR_ARG;
    if (precision) *precision = ctx->last_precision;
    if (d_used) *d_used = ctx->last_d;
    if (steps) *steps = ctx->last_steps;
    if (normest) *normest = ctx->last_normest;
    if (condest) *condest = ctx->last_condest;
    return LS_OK;
}

ls_status ls_sync(ls_ctx *ctx, void *stream)
{
    if (!ctx) return LS_ERR_ARG;
    LS_TRY(need_device(ctx));
    DeviceGuard g(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(ctx, hipMemcpyAsync(ctx->status_host, ctx->status, sizeof(int32_t), hipMemcpyDeviceToHost, s), "read status");
    HIP_TRY(ctx, hipStreamSynchronize(s), "stream synchronize");
    const int32_t st = *ctx->status_host;
    if (st != 0) {
        HIP_TRY(ctx, hipMemsetAsync(ctx->status, 0, sizeof(int32_t), s), "clear status");
        HIP_TRY(ctx, hipStreamSynchronize(s), "stream synchronize");
        if (st & ST_RANK) return ls_fail(ctx, LS_ERR_RANK, "R is numerically singular (rank-deficient A or sketch)");
        if (st & ST_NONFINITE) return ls_fail(ctx, LS_ERR_NONFINITE, "NaN or Inf in B, R or x");
        if (st & ST_DIVERGED) return ls_fail(ctx, LS_ERR_DIVERGED, "the residual grew without bound");
        if (st & ST_TIMEOUT) return ls_fail(ctx, LS_ERR_DEVICE, "a grid barrier timed out (results invalid)");
    }
    return LS_OK;
}

ls_status ls_profile(ls_ctx *ctx, double *pass_ms, int64_t *pass_launches, int32_t reset)
{
    if (!ctx) return LS_ERR_ARG;
    LS_TRY(need_device(ctx));
    DeviceGuard g(ctx->device);
    double total = 0.0;
    for (size_t k = 0; k + 1 < ctx->ev_used; k += 2) {
        HIP_TRY(ctx, hipEventSynchronize(ctx->ev_pool[k + 1]), "event synchronize");
        float ms = 0.0f;
        HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->ev_pool[k], ctx->ev_pool[k + 1]), "event elapsed");
        total += ms;
    }
    if (pass_ms) *pass_ms = total;
    if (pass_launches) *pass_launches = (int64_t)(ctx->ev_used / 2);
    if (reset) ctx->ev_used = 0;
    return LS_OK;
}

}  // extern "C"
