// Internal declarations of libls shared by its translation units (host side + kernel launchers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "ls.h"

// Deferred device status bits, OR-ed into the context's status word by kernels.
enum : int32_t { ST_RANK = 1, ST_NONFINITE = 2, ST_DIVERGED = 4, ST_TIMEOUT = 8,
                 // served mixed precision only (a request's own status word, never a context's):
                 // the growth monitor froze x, the server repeats the request in FP64
                 ST_GROWTH = 16 };

// Look-ahead of the blocked QR: a second stream of the context and two events.  After each panel
// the next panel's columns are updated on the caller's stream, which then factors that panel,
// while the rest of the trailing matrix is updated on the side stream.
struct QrAside {
    hipStream_t side = nullptr;
    hipEvent_t panel_done = nullptr;   // recorded on the caller's stream after each panel
    hipEvent_t side_done = nullptr;    // recorded on the side stream after each trailing update
};

struct ls_ctx {
    int device = -1;                // -1: host-only context (argument checks only)
    // options
    int32_t zeta = 8;
    uint64_t seed = 0;
    int32_t update = 0;             // 0 plain, 1 damping, 2 momentum
    double alpha = 0.0;             // <= 0: derived from eps = sqrt(n/d)
    double beta = -1.0;             // < 0: derived from eps
    int32_t precision = 0;          // 0 FP64, 1 mixed (FP32 sketch/QR/solves, FP64 pass/update)
    int32_t profile = 0;            // 1: bracket each fused-pass launch with events
    int32_t qr_panel = 0;           // 1: force the per-column panel path
    int32_t gather = 0;             // 1: force the per-row sketch gather
    int32_t stop = 0;               // 1: Section 3.3 stopping rule in ls_solve
    double gamma = 1.0, rho = 0.04;
    // what the last ls_solve used (for ls_solve_info)
    int64_t last_d = 0;
    int32_t last_q = 0;
    int32_t last_steps = 0;         // refinement steps made
    double last_normest = 0.0, last_condest = 0.0;
    int32_t last_precision = 0;     // LS_PRECISION_* of the last ls_solve
    std::vector<hipEvent_t> ev_pool; // start/end pairs, reused
    size_t ev_used = 0;             // events recorded since the last reset (even count)
    // device memory owned by the library
    void *ws = nullptr;
    size_t ws_bytes = 0;
    int32_t *status = nullptr;      // device status word
    int32_t *status_host = nullptr; // pinned host copy
    void *scratch = nullptr;        // this device's copy of the fixed scratch (ls_gradient_noalloc)
    QrAside qla;                    // QR look-ahead stream and events (null: no look-ahead)
    std::string err;
};

// Bump allocator over the context workspace: first a sizing pass (base == nullptr), then the real
// pass over the allocated block.
struct Arena {
    char *base = nullptr;
    size_t off = 0;
    template <class T>
    T *take(size_t count, size_t align = 256) {
        off = (off + align - 1) / align * align;
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// Sum of count values p[0], p[stride], ... added in ascending order, U loads in flight at a time.
// The last count % U values are also loaded together before they are added (a loop of one load at
// a time would put a memory round trip per value on the path: the panel reductions sum 2 to 5
// values per thread).
template <int U, typename T>
__device__ __forceinline__ T strided_sum(const T *__restrict__ p, int count, int64_t stride)
{
    T acc = T(0);
    int g = 0;
    for (; g + U <= count; g += U) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = p[(int64_t)(g + u) * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) acc += v[u];
    }
    if (g < count) {
        T v[U - 1];
#pragma unroll
        for (int u = 0; u < U - 1; ++u) v[u] = (g + u < count) ? p[(int64_t)(g + u) * stride] : T(0);
#pragma unroll
        for (int u = 0; u < U - 1; ++u)
            if (g + u < count) acc += v[u];
    }
    return acc;
}

// sum_i p[i * stride] * w[i] for i < count, accumulated in ascending i, U loads in flight.
template <int U, typename T>
__device__ __forceinline__ T strided_dot(const T *__restrict__ p, int64_t stride, const T *w, int count)
{
    T acc = T(0);
    int i = 0;
    for (; i + U <= count; i += U) {
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = p[(int64_t)(i + u) * stride];
#pragma unroll
        for (int u = 0; u < U; ++u) acc += v[u] * w[i + u];
    }
    if (i < count) {
        T v[U - 1];
#pragma unroll
        for (int u = 0; u < U - 1; ++u) v[u] = (i + u < count) ? p[(int64_t)(i + u) * stride] : T(0);
#pragma unroll
        for (int u = 0; u < U - 1; ++u)
            if (i + u < count) acc += v[u] * w[i + u];
    }
    return acc;
}

ls_status ls_fail(ls_ctx *ctx, ls_status st, const std::string &msg);
ls_status ls_ensure_ws(ls_ctx *ctx, size_t bytes);
ls_status ls_hip_check(ls_ctx *ctx, hipError_t e, const char *what);

// ---- sketch (sketch.hip) -------------------------------------------------------------------------
// Entry lists of the column-sliced gather (k_gather_win).  Sketch rows are grouped by `rw`; the list
// of a group holds its rows' CSR entries reordered window by window (windows of kWinLen rows of A),
// rows in order inside a window, ascending j inside a row, so each row's terms keep their order.
struct WinLists {
    bool active = false;
    int32_t rw = 0;        // sketch rows per group (one wave's accumulators)
    int32_t nwl = 0;       // windows: ceil(m / kWinLen)
    int32_t nstep = 0;     // barrier steps: ceil(nwl / kWinPerStep)
    int32_t cus = 0;       // work-groups per XCD and launch (compute units per XCD)
    int32_t zeta = 0;      // nonzeros per column of S (list entries per row of A)
    uint32_t *lst = nullptr;   // m*zeta entries (j | row in group << 26 | sign << 31), group lists back to back
    int32_t *ctab = nullptr;   // (nwl+1) x d: entries of row k in windows < w
    int32_t *stab = nullptr;   // nwl x d: list offsets (k_win_scan)
    int32_t *woff = nullptr;   // groups x (nstep+1): where each barrier step starts in a list
    // Lists built from the embedding without the CSR (k_wl_*; d <= 40960, short segments):
    bool direct = false;
    int32_t *cnt = nullptr;    // nwl x d: entries of row k in window w
    int32_t *rel = nullptr;    // groups x nwl: entries of group g in window w, then their scan
    int32_t *gtot = nullptr;   // groups: list length of each group
    int32_t *gstart = nullptr; // groups + 1: where each group's list starts
};
struct SketchBufs {
    uint32_t *ent = nullptr;       // m*zeta packed (row | sign<<31), column-major by j
    int32_t *rowcount = nullptr;   // d
    int32_t *rowptr = nullptr;     // d+1
    int32_t *fill = nullptr;       // d
    uint32_t *cols = nullptr;      // m*zeta packed (j | sign<<31), by sketch row, ascending j (null when win.direct)
    int32_t *chunk_cnt = nullptr;  // ceil(m / chunk_cols) x d per-chunk row counts (chunk path), else null
    int32_t chunk_cols = 0;        // columns of S per chunk: 8192, halved while chunk_cols zeta > 8 d (>= 256)
    WinLists win;        // built by launch_csr when active (without the CSR when win.direct)
};
// n > 0 and win_mode == 0: also carve the lists of the column-sliced gather when the shape suits it.
void sketch_bufs(Arena &ar, int64_t m, int64_t d, int32_t zeta, SketchBufs &sb, int64_t n = 0,
                 int32_t win_mode = 1);
hipError_t launch_sparse_sign(hipStream_t s, int64_t m, int64_t d, int32_t zeta, uint64_t seed,
                              const SketchBufs &sb);
hipError_t launch_unpack_embedding(hipStream_t s, int64_t m, int32_t zeta, const uint32_t *ent,
                                   int32_t *rows, int8_t *signs);
hipError_t launch_csr(hipStream_t s, int64_t m, int64_t d, int32_t zeta, const SketchBufs &sb);
// With active lists (win) the column-sliced gather runs, else one wave per sketch row; both add
// the same terms in the same order and give the same bits.
hipError_t launch_gather(hipStream_t s, int64_t d, int64_t n, const double *A, int64_t lda,
                         const double *b, const int32_t *rowptr, const uint32_t *cols, double scale,
                         double *B, int64_t ldb, double *Sb, int64_t ldsb,
                         const WinLists *win = nullptr);
// The same sums (FP64) stored rounded once to FP32, for the mixed-precision path.
hipError_t launch_gather(hipStream_t s, int64_t d, int64_t n, const double *A, int64_t lda,
                         const double *b, const int32_t *rowptr, const uint32_t *cols, double scale,
                         float *B, int64_t ldb, float *Sb, int64_t ldsb,
                         const WinLists *win = nullptr);

// ---- QR (qr.hip) ---------------------------------------------------------------------------------
// Buffers of the blocked Householder QR in element type E (double; float on the mixed path).
template <typename E>
struct QrBufsT {
    E *W;                // d x ldw : [B | Sb]
    int64_t ldw;
    E *V;                // d x NB  : Householder vectors of the current panel
    E *red;              // panel reduction partials
    E *tau;              // n
    E *Yp;               // chunk partials of V^T [V | C]
    E *Z;                // NB x ldw
    E *qtb;              // n
    E *RT;               // n x n  (R^T, row-major)
    unsigned *bar;       // grid-barrier counter of the cooperative panel kernel
    // look-ahead only (null otherwise): the other panel's Householder vectors (panels alternate
    // between V and V2) and the side stream's chunk partials and Z
    E *V2 = nullptr;
    E *Yp2 = nullptr;
    E *Z2 = nullptr;
};
using QrBufs = QrBufsT<double>;
using QrBufs32 = QrBufsT<float>;
// The look-ahead pays when the trailing updates it overlaps with the panels are large: measured with
// cooperative panels, 40.2 -> 35.4 ms at d = 4e4, n = 2000 and 19.7 -> 19.0 ms at d = 3e4, n = 1500,
// but 4.20 -> 4.32 ms at d = 1e4, n = 500 and 9.77 -> 9.90 ms at d = 2e4, n = 1000 (stream and
// event costs per panel).
inline bool qr_lookahead_pays(int64_t d, int64_t n) { return (double)d * (double)n >= 3e7; }
void qr_bufs(Arena &ar, int64_t d, int64_t n, QrBufs &qb, bool lookahead = false);
void qr_bufs(Arena &ar, int64_t d, int64_t n, QrBufs32 &qb, bool lookahead = false);
hipError_t launch_copy_sketch(hipStream_t s, int64_t d, int64_t n, const double *B, int64_t ldb,
                              const double *Sb, const QrBufs &qb);
hipError_t launch_copy_sketch(hipStream_t s, int64_t d, int64_t n, const float *B, int64_t ldb,
                              const float *Sb, const QrBufs32 &qb);
// Mixed path: qb32.W = [fl32(B) | fl32(Sb)] with B in qb64.W's first n columns and Sb contiguous;
// launch_set_rhs puts Sb into column n of qb64.W (the FP64 fallback).
hipError_t launch_round_sketch(hipStream_t s, int64_t d, int64_t n, const QrBufs &qb64, const double *Sb,
                               const QrBufs32 &qb32);
hipError_t launch_set_rhs(hipStream_t s, int64_t d, int64_t n, const double *Sb, const QrBufs &qb);
// With la (and buffers from qr_bufs(.., lookahead = true)) the trailing updates are split between s
// and la->side as QrAside describes; the factorization's bits are the same either way.
hipError_t launch_qr(hipStream_t s, int64_t d, int64_t n, const QrBufs &qb, int32_t *status,
                     bool per_column = false, const QrAside *la = nullptr);
hipError_t launch_qr(hipStream_t s, int64_t d, int64_t n, const QrBufs32 &qb, int32_t *status,
                     bool per_column = false, const QrAside *la = nullptr);
hipError_t launch_extract_r(hipStream_t s, int64_t n, const QrBufs &qb, double *R, int64_t ldr,
                            int32_t *status);
hipError_t launch_extract_r(hipStream_t s, int64_t n, const QrBufs32 &qb, float *R, int64_t ldr,
                            int32_t *status);

// ---- iteration (iterate.hip) ---------------------------------------------------------------------
struct IterBufs {
    double *part;        // P x n gradient partials
    double *part_rr;     // P
    double *part_ad;     // P partials of ||A dx||^2 (stopping rule)
    double *dx;          // n: x_i - x_{i-1}
    double *scal;        // [0] ||r||^2, [1] ||A dx||^2, [2] normest, [3] condest, [4] ||r_1||^2
    int32_t *state;      // [0] done flag, [1] updates made
    double *c;           // n
    double *xprev;       // n
    double *RT;          // n x n (R^T row-major)
    int32_t P;
};
int32_t iter_partials(int64_t m, int64_t n);
// Size of the fixed per-device scratch array of ls_gradient_noalloc (33 MiB: the partials of the
// widest pass, 2048 x 2048 doubles, and the small vectors of an IterBufs carve).
constexpr size_t kNoAllocScratchBytes = (size_t)33 << 20;
// Looks up this device's address of that array (once per device; the device must be current) and
// stores it in ctx->scratch.
ls_status pass_scratch_attach(ls_ctx *ctx);

// ---- served rounds (pass.hip, solve.hip; driven by server.hip) ----------------------------------
// One resident problem of a served round.  Its pass runs as virtual work-groups 0..P-1 (P =
// iter_partials(m, n)), its reduction as column blocks 0..ceil(n/64)-1, its solve as one
// work-group, with exactly the arithmetic of ls_iterate on it alone.
struct ServeSlot {
    const double *A, *b;
    double *x;                  // x_i in, x_{i+1} out (the caller's buffer)
    const void *R, *RT;         // n x n, ld n, zero strict lower triangle; RT = R^T (FP64, or FP32
                                // when r32)
    double *part, *part_rr;     // P x n, P
    double *c, *rr;             // n, 1
    int64_t m, n, lda;
    int32_t P, pass_base, red_base, cls;
    int32_t *status;            // the problem's own status word
    int32_t r32;                // 1: mixed precision (FP32 factor, growth monitor)
    int32_t *gstate;            // r32: [0] frozen, [1] steps made, [2] monitor fired, [3] growth run
    double *gprev;              // r32: ||r||^2 of the previous step
};
int32_t pass_class(int64_t n);  // pass variant of a problem with n columns (0..8)
// Pass of every slot of class `cls` (work-groups listed in wg_slot, total_wg of them), reductions of
// every slot, and the solve + update x += d of every slot (one work-group each).
hipError_t launch_served_pass(hipStream_t s, int cls, int total_wg, const ServeSlot *slots,
                              const int32_t *wg_slot);
hipError_t launch_served_reduce(hipStream_t s, int total_wg, const ServeSlot *slots, const int32_t *wg_slot);
hipError_t launch_served_solve(hipStream_t s, int nslots, int64_t max_n, const ServeSlot *slots);
void iter_bufs(Arena &ar, int64_t m, int64_t n, IterBufs &ib, bool need_rt);
hipError_t launch_transpose(hipStream_t s, int64_t n, const double *R, int64_t ldr, double *RT);
hipError_t launch_transpose(hipStream_t s, int64_t n, const float *R, int64_t ldr, float *RT);
// Upper triangle of R copied with leading dimension n, zero below the diagonal.
hipError_t launch_compact_upper(hipStream_t s, int64_t n, const double *R, int64_t ldr, double *Rc);
hipError_t launch_compact_upper(hipStream_t s, int64_t n, const float *R, int64_t ldr, float *Rc);
hipError_t launch_gradient(hipStream_t s, int64_t m, int64_t n, const double *A, int64_t lda,
                           const double *b, const double *x, const IterBufs &ib, double *c,
                           double *rnorm2, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr,
                           const double *dx = nullptr, double *ad_out = nullptr,
                           const int32_t *done = nullptr);
// The Section 3.3 estimators draw their start vector from the stream seed + this offset.
constexpr uint64_t kEstimatorSeedOffset = 0x632BE59BD9B4E019ULL;
// Refinement steps on the FP64 sketch that take the FP32 sketch-and-solve start of the mixed
// path to FP64 accuracy, from condest of the FP32 factor (2 to 8).
int32_t mixed_start_steps(double condest);
// Stopping rule of Section 3.3 evaluated on the device (see k_solve).
struct StopArgs {
    int32_t *state = nullptr;   // [0] done flag, [1] updates made, [2] fall back to FP64, [3] growth run
                                // (nullptr: no done flag, no stopping rule, no growth monitor)
    double *scal = nullptr;     // [0] ||r_i||^2, [1] ||A dx||^2, [2] normest, [3] condest,
                                // [4] ||r_0||^2, [5] previous ||r||^2
    double *dx = nullptr;       // n: x_i - x_{i-1}, written by each update
    double gamma = 1.0, rho = 0.04;
    int check = 0;              // 1 when scal[1] holds ||A (x_i - x_{i-1})||^2 for this step
    int grow = 0;               // 1: monitor the growth of ||r_i|| (mixed precision)
};
// d = R^{-1} R^{-T} c; mode 0: write d to dout; mode 1: x += d; mode 2: x += alpha d + beta (x - xprev).
// With an FP32 factor the solves run in FP32 on c scaled by a power of two; c, x and d stay FP64.
hipError_t launch_solve_update(hipStream_t s, int64_t n, const double *R, int64_t ldr,
                               const double *RT, const double *c, double *x, double *xprev,
                               double *dout, int mode, double alpha, double beta, int32_t *status,
                               const StopArgs &st = StopArgs());
hipError_t launch_solve_update(hipStream_t s, int64_t n, const float *R, int64_t ldr,
                               const float *RT, const double *c, double *x, double *xprev,
                               double *dout, int mode, double alpha, double beta, int32_t *status,
                               const StopArgs &st = StopArgs());
// normest (power method from a SplitMix64 start, ceil(ln n) steps) -> scal[2]; condest (Hager's
// 1-norm estimate of ||R^{-1}||_1 times ||R||_1) -> scal[3], in the factor's arithmetic.
// work: 3 n entries.
hipError_t launch_estimators(hipStream_t s, int64_t n, const double *R, int64_t ldr,
                             const double *RT, uint64_t seed, double *work, double *scal);
hipError_t launch_estimators(hipStream_t s, int64_t n, const float *R, int64_t ldr,
                             const float *RT, uint64_t seed, float *work, double *scal);
hipError_t launch_stop_init(hipStream_t s, int32_t *state);
hipError_t launch_back_substitution(hipStream_t s, int64_t n, const double *R, int64_t ldr,
                                    const double *RT, const double *y, double *x, int32_t *status);
hipError_t launch_back_substitution(hipStream_t s, int64_t n, const float *R, int64_t ldr,
                                    const float *RT, const float *y, double *x, int32_t *status);
