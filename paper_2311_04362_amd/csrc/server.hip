// Served stream of least-squares solves: many independent problems min ||b - A x|| resident on one
// GPU, admitted by HBM footprint, set up (sketch, QR, sketch-and-solve start) on a few setup lanes
// (a stream and a workspace each), and iterated together in rounds on a serve stream.  A round is one refinement
// step (Algorithm 2 loop body) of every resident problem: one batched pass launch per pass class,
// one batched reduction and one batched solve + update (pass.hip, solve.hip).  Problems join at the
// next round after their setup and leave after their q-th (continuous batching), so the launch cost
// of a round is shared by everything resident.  Each problem's arithmetic is that of ls_solve on it
// alone: its result does not depend on what else is resident.
//
// Mixed precision (ls_server_set_precision): a request's setup runs in two parts on its lane.  The
// first forms the FP64 sketch, factors its FP32 rounding and takes the FP32 start and condest; the
// scheduler then reads the status word and condest and enqueues either the FP64 factorization of
// the same sketch (the condest fallback) or the refinement steps of the start on the FP64 sketch.
// Rounds solve with the FP32 factor under the growth monitor; a request whose monitor fires is
// queued again as an FP64 request.  Each outcome is ls_solve's with LS_OPT_PRECISION = 1.
//
// A scheduler thread owned by the server does all device work; ls_server_submit and ls_server_wait
// may be called from any host thread.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cmath>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "common.hpp"

namespace {

using Clock = std::chrono::steady_clock;

constexpr int kRoundsInFlight = 3;     // rounds enqueued ahead of the host
// Setups in flight at once, each on its own stream.  Setups are chains of small latency-bound
// launches, so more of them overlap better: 8 lanes measured 925-947 solves/s at saturation against
// 886-899 for 4 under HIP's default four hardware queues (839 with eight queues; 12 lanes 890-918,
// 16 lanes 860-873).
constexpr int kSetupLanes = 8;
constexpr int kClasses = 9;            // pass classes (pass_class)

enum class St { Queued, Setup, Active, Finishing, Done };

struct Req {
    int64_t ticket = 0;
    int64_t m = 0, n = 0, lda = 0, d = 0;
    int32_t q = 0;
    uint64_t seed = 0;
    const double *A = nullptr, *b = nullptr;
    double *x = nullptr;
    int64_t footprint = 0;             // resident bytes (resident_bytes)
    int64_t setup = 0;                 // setup-lane workspace it needs (setup_bytes)
    St st = St::Queued;
    int32_t rounds = 0;
    double t_submit = 0, t_admit = 0, t_start = 0, t_done = 0;
    ls_status result = LS_OK;
    // device buffers (one block from the server's cache)
    void *mem = nullptr;
    size_t mem_bytes = 0;
    double *R = nullptr, *RT = nullptr, *part = nullptr, *part_rr = nullptr, *c = nullptr, *rr = nullptr;
    int32_t *status = nullptr;
    int32_t P = 1;
    int32_t *status_host = nullptr;    // pinned: [0] status word (setup, last round), [2..3] condest
    int32_t prec = LS_PRECISION_FP64;  // arithmetic of the next setup: FP64 or mixed
    int32_t used = LS_PRECISION_FP64;  // what the result comes from (LS_PRECISION_*)
    int32_t phase = 0;                 // mixed setup: 1 FP32 factor enqueued, 2 start or fallback
    int32_t *gstate = nullptr;         // growth monitor of the FP32 rounds (ServeSlot::gstate)
    double *gprev = nullptr;
    hipEvent_t ev = nullptr;           // end of setup, then end of the last round
    int lane = -1;                     // setup lane while in setup
};

}  // namespace

struct ls_server {
    int device = -1;
    int64_t budget = 0;
    int32_t max_active = 0;
    int32_t zeta = 8;
    std::atomic<int32_t> precision{LS_PRECISION_FP64};   // of requests submitted from now on
    Clock::time_point t0;
    hipStream_t s_serve = nullptr;
    // setup lanes: a stream and a workspace (sketch and QR of one problem at a time) each
    struct Lane {
        hipStream_t s = nullptr;
        void *ws = nullptr;
        size_t ws_bytes = 0;
        bool busy = false;
    };
    std::vector<Lane> lanes;
    // device slot table and work-group maps, and their pinned staging ring
    ServeSlot *d_slots = nullptr;
    int32_t *d_wgmap = nullptr;
    size_t wgmap_cap = 0;
    struct Stage {
        ServeSlot *slots = nullptr;
        int32_t *wgmap = nullptr;
        hipEvent_t ev = nullptr;       // the copy out of this buffer has been consumed
        bool used = false;
    };
    std::vector<Stage> stage;
    size_t stage_next = 0;
    std::vector<hipEvent_t> round_ev;  // ring of round-end events
    std::deque<hipEvent_t> inflight;
    size_t round_next = 0;
    // device memory cache (blocks are reused, released at destroy)
    std::vector<std::pair<size_t, void *>> free_blocks;
    std::vector<void *> all_blocks;
    std::vector<int32_t *> pinned_status;   // every pinned status word made (freed at destroy)
    std::vector<int32_t *> pin_pool;        // status words of finished requests, for reuse
    std::vector<hipEvent_t> ev_pool;        // events of finished requests, for reuse
    int64_t lanes_ws = 0;                   // bytes held by the setup lanes' workspaces
    // requests
    std::mutex mu;
    std::condition_variable cv_done, cv_work;
    std::deque<Req *> queue;
    std::map<int64_t, std::unique_ptr<Req>> reqs;
    std::vector<Req *> setup, active, finishing;
    bool table_dirty = true;
    int64_t next_ticket = 1;
    int64_t footprint_now = 0, footprint_peak = 0;
    int64_t submitted = 0, completed = 0, rounds = 0;
    int32_t admitted_live = 0;
    bool stopping = false;
    ls_status fatal = LS_OK;
    std::string err;
    std::thread thr;
};

namespace {

double seconds_since(const ls_server *sv) { return std::chrono::duration<double>(Clock::now() - sv->t0).count(); }

// The per-problem device block (R, R^T, pass partials, c, ||r||^2, status word, growth monitor),
// carved from `base` (nullptr: sizing only).  R and R^T have room for an FP64 factor; an FP32 one
// uses the first half of each.  Returns its size in bytes.
size_t carve_req(Req *r, char *base)
{
    Arena ar;
    ar.base = base;
    r->R = ar.take<double>((size_t)(r->n * r->n));
    r->RT = ar.take<double>((size_t)(r->n * r->n));
    r->part = ar.take<double>((size_t)r->P * (size_t)r->n);
    r->part_rr = ar.take<double>((size_t)r->P);
    r->c = ar.take<double>((size_t)r->n);
    r->rr = ar.take<double>(1);
    r->status = ar.take<int32_t>(1);
    r->gstate = ar.take<int32_t>(4);
    r->gprev = ar.take<double>(1);
    return ar.off + 256;
}

// Bytes a problem holds while resident: its A and b (the caller's, but kept on the device while it
// is served) and its device block.
int64_t resident_bytes(Req *r)
{
    r->P = iter_partials(r->m, r->n);
    return 8 * r->m * r->n + 8 * r->m + (int64_t)carve_req(r, nullptr);
}

// A setup lane's workspace for one problem: embedding and CSR, the FP64 QR work matrix; for mixed
// precision also the FP32 work matrix, S b apart, the sketch-sized pass buffers of the start's
// refinement steps and the estimators' work vectors.
struct SetupBufs {
    SketchBufs sb{};
    QrBufs qb{};
    QrBufs32 qb32{};
    IterBufs ib{};
    double *Sb = nullptr;
    float *est = nullptr;
};

void carve_setup(Arena &ar, int64_t m, int64_t n, int64_t d, int32_t zeta, int32_t prec, SetupBufs &w)
{
    sketch_bufs(ar, m, d, zeta, w.sb);
    qr_bufs(ar, d, n, w.qb);
    if (prec == LS_PRECISION_MIXED) {
        qr_bufs(ar, d, n, w.qb32);
        iter_bufs(ar, d, n, w.ib, false);
        w.Sb = ar.take<double>((size_t)d);
        w.est = ar.take<float>((size_t)3 * (size_t)n);
    }
}

// Workspace a setup lane needs for a problem (the same carve enqueue_setup makes).
int64_t setup_bytes(int64_t m, int64_t n, int64_t d, int32_t zeta, int32_t prec)
{
    SetupBufs w;
    Arena ar;
    carve_setup(ar, m, n, d, zeta, prec, w);
    return (int64_t)ar.off + 256;
}

double *condest_host(Req *r) { return reinterpret_cast<double *>(r->status_host + 2); }

bool hip_ok(ls_server *sv, hipError_t e, const char *what)
{
    if (e == hipSuccess) return true;
    if (sv->fatal == LS_OK) {
        sv->fatal = LS_ERR_DEVICE;
        sv->err = std::string(what) + ": " + hipGetErrorString(e);
    }
    return false;
}

void *take_block(ls_server *sv, size_t bytes)
{
    for (size_t i = 0; i < sv->free_blocks.size(); ++i)
        if (sv->free_blocks[i].first >= bytes) {
            void *p = sv->free_blocks[i].second;
            sv->free_blocks.erase(sv->free_blocks.begin() + (long)i);
            return p;
        }
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    sv->all_blocks.push_back(p);
    return p;
}

void give_block(ls_server *sv, void *p, size_t bytes)
{
    if (p) sv->free_blocks.emplace_back(bytes, p);
}

// Per-problem device buffers: R, R^T, pass partials, c, ||r||^2, status word.
bool alloc_req(ls_server *sv, Req *r)
{
    r->P = iter_partials(r->m, r->n);
    r->mem_bytes = carve_req(r, nullptr);
    r->mem = take_block(sv, r->mem_bytes);
    if (!r->mem) return false;
    carve_req(r, static_cast<char *>(r->mem));
    return true;
}

// Frees an idle lane's workspace (its stream is drained first) and stops charging it.
void release_lane_ws(ls_server *sv, ls_server::Lane &ln)
{
    if (!ln.ws) return;
    (void)hip_ok(sv, hipStreamSynchronize(ln.s), "setup stream synchronize");
    (void)hipFree(ln.ws);
    sv->lanes_ws -= (int64_t)ln.ws_bytes;
    sv->footprint_now -= (int64_t)ln.ws_bytes;
    ln.ws = nullptr;
    ln.ws_bytes = 0;
}

// A lane's workspace large enough for the sketch and QR of one problem (the lane is idle here).
// The workspace is charged to the footprint; `room` is what the budget still allows beyond the
// lane's present workspace, and growth takes a quarter of slack only where it fits.
bool ensure_setup_ws(ls_server *sv, ls_server::Lane &ln, size_t bytes, int64_t room)
{
    if (bytes <= ln.ws_bytes) return true;
    release_lane_ws(sv, ln);
    size_t want = bytes + bytes / 4;
    if ((int64_t)want > room) want = bytes;
    if (hipMalloc(&ln.ws, want) != hipSuccess) {
        (void)hipGetLastError();
        ln.ws = nullptr;
        return false;
    }
    ln.ws_bytes = want;
    sv->lanes_ws += (int64_t)want;
    sv->footprint_now += (int64_t)want;
    sv->footprint_peak = std::max(sv->footprint_peak, sv->footprint_now);
    return true;
}

int free_lane(const ls_server *sv)
{
    for (size_t i = 0; i < sv->lanes.size(); ++i)
        if (!sv->lanes[i].busy) return (int)i;
    return -1;
}

// The idle lane for a setup needing `need` bytes of workspace: the smallest workspace that holds it,
// else the largest one (least growth); -1 if every lane is busy.
int pick_lane(const ls_server *sv, int64_t need)
{
    int best = -1;
    for (size_t i = 0; i < sv->lanes.size(); ++i) {
        const auto &ln = sv->lanes[i];
        if (ln.busy) continue;
        if (best < 0) { best = (int)i; continue; }
        const int64_t wb = (int64_t)sv->lanes[best].ws_bytes, wi = (int64_t)ln.ws_bytes;
        const bool fits_b = wb >= need, fits_i = wi >= need;
        if (fits_i && (!fits_b || wi < wb)) best = (int)i;
        else if (!fits_i && !fits_b && wi > wb) best = (int)i;
    }
    return best;
}

// Enqueue the setup of one problem on a free setup lane, then the copy of its status word and the
// event the scheduler waits for.  FP64: sketch, QR, R, R^T and x_0 (as ls_solve does).  Mixed: the
// FP64 sketch (S b apart), the FP32 QR of its rounding, R, R^T, the FP32 start and the estimators,
// with condest copied out beside the status word; enqueue_mixed_rest follows.
bool enqueue_setup(ls_server *sv, Req *r, int lane)
{
    ls_server::Lane &ln = sv->lanes[lane];
    hipStream_t s = ln.s;
    SetupBufs w;
    Arena sizing;
    carve_setup(sizing, r->m, r->n, r->d, sv->zeta, r->prec, w);
    const int64_t room = sv->budget - sv->footprint_now + (int64_t)ln.ws_bytes;
    if (!ensure_setup_ws(sv, ln, sizing.off + 256, room)) {
        r->result = LS_ERR_ALLOC;
        return false;
    }
    Arena real;
    real.base = static_cast<char *>(ln.ws);
    carve_setup(real, r->m, r->n, r->d, sv->zeta, r->prec, w);
    const int64_t n = r->n, d = r->d;
    const double scale = 1.0 / std::sqrt((double)sv->zeta);
    bool ok = hip_ok(sv, hipMemsetAsync(r->status, 0, sizeof(int32_t), s), "clear status") &&
              hip_ok(sv, launch_sparse_sign(s, r->m, d, sv->zeta, r->seed, w.sb), "sparse-sign kernel") &&
              hip_ok(sv, launch_csr(s, r->m, d, sv->zeta, w.sb), "CSR kernels");
    // per-column panels: a cooperative grid barrier would have to share the device with the rounds
    // running on the serve stream (both paths give the same bits)
    if (r->prec == LS_PRECISION_MIXED) {
        float *R = reinterpret_cast<float *>(r->R), *RT = reinterpret_cast<float *>(r->RT);
        ok = ok &&
             hip_ok(sv, launch_gather(s, d, n, r->A, r->lda, r->b, w.sb.rowptr, w.sb.cols, scale, w.qb.W,
                                      w.qb.ldw, w.Sb, 1), "gather kernel") &&
             hip_ok(sv, launch_round_sketch(s, d, n, w.qb, w.Sb, w.qb32), "round sketch") &&
             hip_ok(sv, launch_qr(s, d, n, w.qb32, r->status, true), "QR kernels") &&
             hip_ok(sv, launch_extract_r(s, n, w.qb32, R, n, r->status), "extract R") &&
             hip_ok(sv, hipMemcpyAsync(RT, w.qb32.RT, sizeof(float) * (size_t)(n * n), hipMemcpyDeviceToDevice, s), "copy R^T") &&
             hip_ok(sv, launch_back_substitution(s, n, R, n, RT, w.qb32.qtb, r->x, r->status), "x0 solve") &&
             hip_ok(sv, launch_estimators(s, n, R, n, RT, r->seed + kEstimatorSeedOffset, w.est, w.ib.scal), "estimators") &&
             hip_ok(sv, hipMemcpyAsync(condest_host(r), w.ib.scal + 3, sizeof(double), hipMemcpyDeviceToHost, s), "read condest");
        r->phase = 1;
    } else {
        ok = ok &&
             hip_ok(sv, launch_gather(s, d, n, r->A, r->lda, r->b, w.sb.rowptr, w.sb.cols, scale, w.qb.W,
                                      w.qb.ldw, w.qb.W + n, w.qb.ldw), "gather kernel") &&
             hip_ok(sv, launch_qr(s, d, n, w.qb, r->status, true), "QR kernels") &&
             hip_ok(sv, launch_extract_r(s, n, w.qb, r->R, n, r->status), "extract R") &&
             hip_ok(sv, hipMemcpyAsync(r->RT, w.qb.RT, sizeof(double) * (size_t)(n * n), hipMemcpyDeviceToDevice, s), "copy R^T") &&
             hip_ok(sv, launch_back_substitution(s, n, r->R, n, w.qb.RT, w.qb.qtb, r->x, r->status), "x0 solve");
        r->phase = 0;
    }
    return ok && hip_ok(sv, hipMemcpyAsync(r->status_host, r->status, sizeof(int32_t), hipMemcpyDeviceToHost, s), "read status") &&
           hip_ok(sv, hipEventRecord(r->ev, s), "record setup event");
}

// Second part of a mixed setup, on the same lane once the first has finished (its workspace still
// holds the FP64 sketch): ls_solve's decision from the FP32 factor's status word and condest.  Falls
// back (FP64 QR of the same sketch, R, R^T, x_0) when the FP32 QR flagged R or condest u_32 > 0.05;
// otherwise refines the FP32 start on the FP64 sketch (mixed_start_steps) and clears the growth
// monitor.
bool enqueue_mixed_rest(ls_server *sv, Req *r)
{
    ls_server::Lane &ln = sv->lanes[r->lane];
    hipStream_t s = ln.s;
    SetupBufs w;
    Arena real;
    real.base = static_cast<char *>(ln.ws);
    carve_setup(real, r->m, r->n, r->d, sv->zeta, LS_PRECISION_MIXED, w);
    const int64_t n = r->n, d = r->d;
    const int32_t st0 = r->status_host[0];
    const double cond = *condest_host(r);
    bool ok;
    if ((st0 & (ST_RANK | ST_NONFINITE)) || !(cond * 0x1p-24 <= 0.05)) {
        r->used = LS_PRECISION_FELL_BACK_COND;
        ok = hip_ok(sv, hipMemsetAsync(r->status, 0, sizeof(int32_t), s), "clear status") &&
             hip_ok(sv, launch_set_rhs(s, d, n, w.Sb, w.qb), "set rhs") &&
             hip_ok(sv, launch_qr(s, d, n, w.qb, r->status, true), "QR kernels") &&
             hip_ok(sv, launch_extract_r(s, n, w.qb, r->R, n, r->status), "extract R") &&
             hip_ok(sv, hipMemcpyAsync(r->RT, w.qb.RT, sizeof(double) * (size_t)(n * n), hipMemcpyDeviceToDevice, s), "copy R^T") &&
             hip_ok(sv, launch_back_substitution(s, n, r->R, n, w.qb.RT, w.qb.qtb, r->x, r->status), "x0 solve");
    } else {
        r->used = LS_PRECISION_MIXED;
        const float *R = reinterpret_cast<const float *>(r->R), *RT = reinterpret_cast<const float *>(r->RT);
        const int32_t k0 = mixed_start_steps(cond);
        ok = hip_ok(sv, hipMemsetAsync(r->gstate, 0, 4 * sizeof(int32_t), s), "clear growth monitor");
        for (int32_t k = 0; k < k0 && ok; ++k)
            ok = hip_ok(sv, launch_gradient(s, d, n, w.qb.W, w.qb.ldw, w.Sb, r->x, w.ib, w.ib.c, nullptr), "start pass") &&
                 hip_ok(sv, launch_solve_update(s, n, R, n, RT, w.ib.c, r->x, nullptr, nullptr, 1, 1.0, 0.0, r->status), "start solve");
    }
    r->phase = 2;
    return ok && hip_ok(sv, hipMemcpyAsync(r->status_host, r->status, sizeof(int32_t), hipMemcpyDeviceToHost, s), "read status") &&
           hip_ok(sv, hipEventRecord(r->ev, s), "record setup event");
}

ls_status status_of(int32_t st)
{
    if (st & ST_RANK) return LS_ERR_RANK;
    if (st & ST_NONFINITE) return LS_ERR_NONFINITE;
    if (st & ST_DIVERGED) return LS_ERR_DIVERGED;
    if (st & ST_TIMEOUT) return LS_ERR_DEVICE;
    return LS_OK;
}

// Called with the lock held: a request leaves the server.  Its device block goes back to the cache;
// with `recycle` (no device work of the request can still be pending) its event and pinned status
// word go back to the pools for later requests.  Only the host record (result and times) stays.
void finish(ls_server *sv, Req *r, ls_status result, bool recycle = true)
{
    r->result = result;
    r->st = St::Done;
    r->t_done = seconds_since(sv);
    give_block(sv, r->mem, r->mem_bytes);
    r->mem = nullptr;
    sv->footprint_now -= r->footprint;
    sv->admitted_live -= 1;
    sv->completed += 1;
    if (recycle) {
        if (r->ev) sv->ev_pool.push_back(r->ev);
        if (r->status_host) sv->pin_pool.push_back(r->status_host);
        r->ev = nullptr;
        r->status_host = nullptr;
    }
    sv->cv_done.notify_all();
}

// Called with the lock held: the growth monitor of a mixed request fired (its x is frozen).  As
// ls_solve falls back to FP64, the request gives its device block back and queues again, first, as
// an FP64 request; its result will be reported as LS_PRECISION_FELL_BACK_GROWTH.
void requeue_fp64(ls_server *sv, Req *r)
{
    give_block(sv, r->mem, r->mem_bytes);
    r->mem = nullptr;
    sv->footprint_now -= r->footprint;
    sv->admitted_live -= 1;
    r->prec = LS_PRECISION_FP64;
    r->used = LS_PRECISION_FELL_BACK_GROWTH;
    r->setup = setup_bytes(r->m, r->n, r->d, sv->zeta, LS_PRECISION_FP64);
    r->rounds = 0;
    r->st = St::Queued;
    sv->queue.push_front(r);
}

// Slot table and work-group maps of the current active set into the next staging buffer, copied to
// the device on the serve stream.  Returns false on a device error.
bool upload_table(ls_server *sv, int32_t class_wg[kClasses], int32_t class_off[kClasses], int32_t &red_wg,
                  int32_t &red_off, int64_t &max_n)
{
    ls_server::Stage &stg = sv->stage[sv->stage_next];
    sv->stage_next = (sv->stage_next + 1) % sv->stage.size();
    if (stg.used && !hip_ok(sv, hipEventSynchronize(stg.ev), "staging reuse")) return false;
    const int ns = (int)sv->active.size();
    for (int k = 0; k < kClasses; ++k) class_wg[k] = 0;
    max_n = 1;
    // pass work-groups grouped by class, then the reduction work-groups
    size_t off = 0;
    for (int k = 0; k < kClasses; ++k) {
        class_off[k] = (int32_t)off;
        for (int i = 0; i < ns; ++i) {
            Req *r = sv->active[i];
            if (pass_class(r->n) != k) continue;
            ServeSlot &sl = stg.slots[i];
            sl.pass_base = class_wg[k];
            for (int32_t p = 0; p < r->P; ++p) stg.wgmap[off++] = i;
            class_wg[k] += r->P;
        }
    }
    red_off = (int32_t)off;
    red_wg = 0;
    for (int i = 0; i < ns; ++i) {
        Req *r = sv->active[i];
        ServeSlot &sl = stg.slots[i];
        sl.A = r->A;
        sl.b = r->b;
        sl.x = r->x;
        sl.R = r->R;
        sl.RT = r->RT;
        sl.part = r->part;
        sl.part_rr = r->part_rr;
        sl.c = r->c;
        sl.rr = r->rr;
        sl.m = r->m;
        sl.n = r->n;
        sl.lda = r->lda;
        sl.P = r->P;
        sl.cls = pass_class(r->n);
        sl.status = r->status;
        sl.r32 = r->used == LS_PRECISION_MIXED ? 1 : 0;
        sl.gstate = r->gstate;
        sl.gprev = r->gprev;
        sl.red_base = red_wg;
        const int32_t blocks = (int32_t)((r->n + 63) / 64);
        for (int32_t k2 = 0; k2 < blocks; ++k2) stg.wgmap[off++] = i;
        red_wg += blocks;
        max_n = std::max<int64_t>(max_n, r->n);
    }
    hipStream_t s = sv->s_serve;
    if (!hip_ok(sv, hipMemcpyAsync(sv->d_slots, stg.slots, sizeof(ServeSlot) * (size_t)ns, hipMemcpyHostToDevice, s), "upload slots") ||
        !hip_ok(sv, hipMemcpyAsync(sv->d_wgmap, stg.wgmap, sizeof(int32_t) * off, hipMemcpyHostToDevice, s), "upload map") ||
        !hip_ok(sv, hipEventRecord(stg.ev, s), "record staging event"))
        return false;
    stg.used = true;
    return true;
}

void scheduler(ls_server *sv)
{
    if (hipSetDevice(sv->device) != hipSuccess) {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->fatal = LS_ERR_DEVICE;
        sv->err = "scheduler: cannot select the device";
        sv->cv_done.notify_all();
        return;
    }
    int32_t class_wg[kClasses] = {0}, class_off[kClasses] = {0};
    int32_t red_wg = 0, red_off = 0;
    int64_t max_n = 1;
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        bool progress = false;
        if (sv->fatal != LS_OK) {             // fail everything still pending
            for (auto &kv : sv->reqs)     // device work may still be pending: keep their events
                if (kv.second->st != St::Done) finish(sv, kv.second.get(), sv->fatal, false);
            sv->queue.clear();
            sv->setup.clear();
            sv->active.clear();
            sv->finishing.clear();
        }
        // (1) admission: FIFO while the footprint budget, the slot table and a setup lane allow.
        // The footprint counts every resident problem and the setup lanes' workspaces; a problem
        // is admitted when its resident bytes and its lane's workspace growth fit the budget.  When
        // the front problem does not fit, idle lanes give their workspaces back first.
        while (!sv->queue.empty() && sv->admitted_live < sv->max_active && free_lane(sv) >= 0) {
            Req *r = sv->queue.front();
            const int lane = pick_lane(sv, r->setup);
            const int64_t grow = std::max<int64_t>(0, r->setup - (int64_t)sv->lanes[lane].ws_bytes);
            if (sv->footprint_now + r->footprint + grow > sv->budget) {
                bool freed = false;
                for (auto &ln : sv->lanes)
                    if (!ln.busy && ln.ws && &ln != &sv->lanes[lane]) {
                        release_lane_ws(sv, ln);
                        freed = true;
                    }
                if (freed) continue;
                if (sv->lanes[lane].ws && grow > 0) {        // start the lane afresh at this size
                    release_lane_ws(sv, sv->lanes[lane]);
                    continue;
                }
                break;
            }
            sv->queue.pop_front();
            r->t_admit = seconds_since(sv);
            if (!alloc_req(sv, r)) {
                r->result = LS_ERR_ALLOC;
                r->st = St::Done;
                r->t_done = r->t_admit;
                sv->completed += 1;
                if (r->ev) sv->ev_pool.push_back(r->ev);
                if (r->status_host) sv->pin_pool.push_back(r->status_host);
                r->ev = nullptr;
                r->status_host = nullptr;
                sv->cv_done.notify_all();
                continue;
            }
            sv->footprint_now += r->footprint;
            sv->footprint_peak = std::max(sv->footprint_peak, sv->footprint_now);
            sv->admitted_live += 1;
            if (!enqueue_setup(sv, r, lane)) {
                finish(sv, r, r->result != LS_OK ? r->result : LS_ERR_DEVICE);
                continue;
            }
            sv->lanes[lane].busy = true;
            r->lane = lane;
            r->st = St::Setup;
            sv->setup.push_back(r);
            progress = true;
        }
        // (2) finished setups join the active set (or leave: error, or q = 0); the first part of a
        // mixed setup is followed by its second on the same lane
        for (size_t i = 0; i < sv->setup.size();) {
            Req *r = sv->setup[i];
            const hipError_t e = hipEventQuery(r->ev);
            if (e == hipErrorNotReady) { ++i; continue; }
            if (e == hipSuccess && r->phase == 1) {
                progress = true;
                if (enqueue_mixed_rest(sv, r)) { ++i; continue; }
                // a device error (sv->fatal is set): device work may still be pending
                sv->setup.erase(sv->setup.begin() + (long)i);
                sv->lanes[r->lane].busy = false;
                r->lane = -1;
                finish(sv, r, LS_ERR_DEVICE, false);
                continue;
            }
            sv->setup.erase(sv->setup.begin() + (long)i);
            sv->lanes[r->lane].busy = false;
            r->lane = -1;
            progress = true;
            if (!hip_ok(sv, e, "setup event")) break;
            const ls_status st = status_of(*r->status_host);
            if (st != LS_OK || r->q == 0) {
                finish(sv, r, st);
                continue;
            }
            r->st = St::Active;
            r->t_start = seconds_since(sv);
            sv->active.push_back(r);
            sv->table_dirty = true;
        }
        // (3) retire finished requests and rounds
        while (!sv->inflight.empty() && hipEventQuery(sv->inflight.front()) == hipSuccess) {
            sv->inflight.pop_front();
            progress = true;
        }
        for (size_t i = 0; i < sv->finishing.size();) {
            Req *r = sv->finishing[i];
            const hipError_t e = hipEventQuery(r->ev);
            if (e == hipErrorNotReady) { ++i; continue; }
            sv->finishing.erase(sv->finishing.begin() + (long)i);
            progress = true;
            if (!hip_ok(sv, e, "round event")) {
                finish(sv, r, LS_ERR_DEVICE);
                continue;
            }
            if (*r->status_host & ST_GROWTH) {
                requeue_fp64(sv, r);
                continue;
            }
            finish(sv, r, status_of(*r->status_host));
        }
        // (4) one more round of every active problem, if fewer than kRoundsInFlight are queued
        if (!sv->active.empty() && (int)sv->inflight.size() < kRoundsInFlight && sv->fatal == LS_OK) {
            if (sv->table_dirty) {
                if (!upload_table(sv, class_wg, class_off, red_wg, red_off, max_n)) continue;
                sv->table_dirty = false;
            }
            hipStream_t s = sv->s_serve;
            bool ok = true;
            for (int k = 0; k < kClasses && ok; ++k)
                ok = hip_ok(sv, launch_served_pass(s, k, class_wg[k], sv->d_slots, sv->d_wgmap + class_off[k]), "served pass");
            ok = ok && hip_ok(sv, launch_served_reduce(s, red_wg, sv->d_slots, sv->d_wgmap + red_off), "served reduce") &&
                 hip_ok(sv, launch_served_solve(s, (int)sv->active.size(), max_n, sv->d_slots), "served solve");
            if (!ok) continue;
            sv->rounds += 1;
            for (size_t i = 0; i < sv->active.size();) {
                Req *r = sv->active[i];
                if (++r->rounds < r->q) { ++i; continue; }
                // last round of this problem: its status word, then its completion event
                ok = hip_ok(sv, hipMemcpyAsync(r->status_host, r->status, sizeof(int32_t), hipMemcpyDeviceToHost, s), "read status") &&
                     hip_ok(sv, hipEventRecord(r->ev, s), "record last round");
                r->st = St::Finishing;
                sv->finishing.push_back(r);
                sv->active.erase(sv->active.begin() + (long)i);
                sv->table_dirty = true;
            }
            hipEvent_t ev = sv->round_ev[sv->round_next];
            sv->round_next = (sv->round_next + 1) % sv->round_ev.size();
            if (hip_ok(sv, hipEventRecord(ev, s), "record round")) sv->inflight.push_back(ev);
            progress = true;
        }
        const bool idle = sv->queue.empty() && sv->setup.empty() && sv->active.empty() && sv->finishing.empty();
        if (idle && sv->stopping) break;
        if (!progress) {
            // nothing to do right now: wait for a submission; while rounds run, poll the device
            // again at once (a sleep would add its wake-up delay to every round); while only setups
            // run, poll every few microseconds
            if (idle) sv->cv_work.wait(lk, [&] { return sv->stopping || !sv->queue.empty(); });
            else {
                const bool rounds_running = !sv->active.empty() || !sv->finishing.empty();
                lk.unlock();
                if (rounds_running) std::this_thread::yield();
                else std::this_thread::sleep_for(std::chrono::microseconds(5));
                lk.lock();
            }
        }
    }
    // drain the device before the streams and buffers go away
    lk.unlock();
    (void)hipStreamSynchronize(sv->s_serve);
    for (auto &ln : sv->lanes) (void)hipStreamSynchronize(ln.s);
}

ls_status check_solve_args(ls_server *sv, int64_t m, int64_t n, const double *A, int64_t lda,
                           const double *b, int64_t d, int32_t q, const double *x)
{
    auto fail = [&](ls_status st, const char *msg) {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->err = msg;
        return st;
    };
    if (n < 1) return fail(LS_ERR_ARG, "n must be >= 1");
    if (n > LS_MAX_N) return fail(LS_ERR_UNSUPPORTED, "n exceeds LS_MAX_N");
    if (m < n) return fail(LS_ERR_ARG, "m must be >= n");
    if (d < n) return fail(LS_ERR_ARG, "d must be >= n");
    if (d >= (int64_t(1) << 31)) return fail(LS_ERR_ARG, "d must be < 2^31");
    if (q < 0) return fail(LS_ERR_ARG, "q must be >= 0");
    if (sv->zeta > d) return fail(LS_ERR_ARG, "zeta must be <= d");
    if (m * (int64_t)sv->zeta >= (int64_t(1) << 31)) return fail(LS_ERR_UNSUPPORTED, "m*zeta must be < 2^31");
    auto aligned8 = [](const void *p) { return p && (reinterpret_cast<uintptr_t>(p) % 8) == 0; };
    if (!aligned8(A) || !aligned8(b) || !aligned8(x)) return fail(LS_ERR_ARG, "A, b and x must be non-NULL and 8-byte aligned");
    if (lda < n) return fail(LS_ERR_ARG, "leading dimension of A < n");
    return LS_OK;
}

}  // namespace

extern "C" {

ls_status ls_server_create(int device, int64_t budget_bytes, int32_t max_active, ls_server **out)
{
    if (!out) return LS_ERR_ARG;
    *out = nullptr;
    if (budget_bytes <= 0 || max_active < 1 || max_active > 4096) return LS_ERR_ARG;
    auto sv = std::unique_ptr<ls_server>(new (std::nothrow) ls_server);
    if (!sv) return LS_ERR_ALLOC;
    sv->budget = budget_bytes;
    sv->max_active = max_active;
    sv->t0 = Clock::now();
    if (device == -1) {                    // host-only: argument checks, no device work
        *out = sv.release();
        return LS_OK;
    }
    int count = 0;
    if (device < 0 || hipGetDeviceCount(&count) != hipSuccess || device >= count) {
        (void)hipGetLastError();
        return LS_ERR_DEVICE;
    }
    sv->device = device;
    int prev = -1;
    (void)hipGetDevice(&prev);
    bool ok = hipSetDevice(device) == hipSuccess;
    // map capacity: pass work-groups of max_active problems (at most 2048 each) plus their
    // reduction blocks (at most LS_MAX_N / 64 each)
    sv->wgmap_cap = (size_t)max_active * (2048 + LS_MAX_N / 64);
    sv->lanes.resize(kSetupLanes);
    for (auto &ln : sv->lanes) ok = ok && hipStreamCreateWithFlags(&ln.s, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipStreamCreateWithFlags(&sv->s_serve, hipStreamNonBlocking) == hipSuccess &&
         hipMalloc(&sv->d_slots, sizeof(ServeSlot) * (size_t)max_active) == hipSuccess &&
         hipMalloc(&sv->d_wgmap, sizeof(int32_t) * sv->wgmap_cap) == hipSuccess;
    sv->stage.resize(3);
    for (auto &st : sv->stage)
        ok = ok && hipHostMalloc(&st.slots, sizeof(ServeSlot) * (size_t)max_active, hipHostMallocDefault) == hipSuccess &&
             hipHostMalloc(&st.wgmap, sizeof(int32_t) * sv->wgmap_cap, hipHostMallocDefault) == hipSuccess &&
             hipEventCreateWithFlags(&st.ev, hipEventDisableTiming) == hipSuccess;
    sv->round_ev.resize(kRoundsInFlight + 2);
    for (auto &e : sv->round_ev) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    if (prev >= 0) (void)hipSetDevice(prev);
    if (!ok) {
        (void)hipGetLastError();
        ls_server_destroy(sv.release());
        return LS_ERR_DEVICE;
    }
    sv->thr = std::thread(scheduler, sv.get());
    *out = sv.release();
    return LS_OK;
}

void ls_server_destroy(ls_server *sv)
{
    if (!sv) return;
    if (sv->thr.joinable()) {
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->stopping = true;
        }
        sv->cv_work.notify_all();
        sv->thr.join();
    }
    if (sv->device >= 0) {
        int prev = -1;
        (void)hipGetDevice(&prev);
        (void)hipSetDevice(sv->device);
        if (sv->s_serve) (void)hipStreamSynchronize(sv->s_serve);
        for (auto &ln : sv->lanes)
            if (ln.s) (void)hipStreamSynchronize(ln.s);
        for (auto &kv : sv->reqs) {
            if (kv.second->ev) (void)hipEventDestroy(kv.second->ev);
        }
        for (hipEvent_t e : sv->ev_pool) (void)hipEventDestroy(e);
        for (int32_t *p : sv->pinned_status) (void)hipHostFree(p);
        for (void *p : sv->all_blocks) (void)hipFree(p);
        for (auto &st : sv->stage) {
            if (st.slots) (void)hipHostFree(st.slots);
            if (st.wgmap) (void)hipHostFree(st.wgmap);
            if (st.ev) (void)hipEventDestroy(st.ev);
        }
        for (auto &e : sv->round_ev) if (e) (void)hipEventDestroy(e);
        for (auto &ln : sv->lanes)
            if (ln.ws) (void)hipFree(ln.ws);
        if (sv->d_slots) (void)hipFree(sv->d_slots);
        if (sv->d_wgmap) (void)hipFree(sv->d_wgmap);
        for (auto &ln : sv->lanes)
            if (ln.s) (void)hipStreamDestroy(ln.s);
        if (sv->s_serve) (void)hipStreamDestroy(sv->s_serve);
        if (prev >= 0) (void)hipSetDevice(prev);
    }
    delete sv;
}

ls_status ls_server_submit(ls_server *sv, int64_t m, int64_t n, const double *A, int64_t lda,
                           const double *b, int64_t d, int32_t q, uint64_t seed, double *x,
                           int64_t *ticket)
{
    if (!sv || !ticket) return LS_ERR_ARG;
    {
        const ls_status st = check_solve_args(sv, m, n, A, lda, b, d, q, x);
        if (st != LS_OK) return st;
    }
    auto r = std::unique_ptr<Req>(new (std::nothrow) Req);
    if (!r) return LS_ERR_ALLOC;
    r->m = m;
    r->n = n;
    r->d = d;
    const int32_t prec = sv->precision.load();
    const int64_t fp = (sv->device >= 0) ? resident_bytes(r.get()) : 8 * m * n + 8 * m;
    const int64_t su = setup_bytes(m, n, d, sv->zeta, prec);
    std::unique_lock<std::mutex> lk(sv->mu);
    if (fp + su > sv->budget) {
        sv->err = "the problem's footprint (resident bytes and setup workspace) exceeds the server's HBM budget";
        return LS_ERR_ALLOC;
    }
    if (sv->device < 0) {
        sv->err = "host-only server: no device work";
        return LS_ERR_DEVICE;
    }
    if (sv->fatal != LS_OK) return sv->fatal;
    int32_t *pin = nullptr;
    if (!sv->pin_pool.empty()) {
        pin = sv->pin_pool.back();
        sv->pin_pool.pop_back();
    } else if (hipHostMalloc(&pin, 4 * sizeof(int32_t), hipHostMallocDefault) == hipSuccess) {
        sv->pinned_status.push_back(pin);
    } else {
        (void)hipGetLastError();
        sv->err = "cannot allocate the request's pinned status word";
        return LS_ERR_DEVICE;
    }
    if (!sv->ev_pool.empty()) {
        r->ev = sv->ev_pool.back();
        sv->ev_pool.pop_back();
    } else if (hipEventCreateWithFlags(&r->ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        sv->pin_pool.push_back(pin);
        sv->err = "cannot create the request's event";
        return LS_ERR_DEVICE;
    }
    *pin = 0;
    r->status_host = pin;
    r->ticket = sv->next_ticket++;
    r->lda = lda;
    r->q = q;
    r->seed = seed;
    r->prec = prec;
    r->used = prec;
    r->A = A;
    r->b = b;
    r->x = x;
    r->footprint = fp;
    r->setup = su;
    r->t_submit = seconds_since(sv);
    *ticket = r->ticket;
    sv->queue.push_back(r.get());
    sv->reqs[r->ticket] = std::move(r);
    sv->submitted += 1;
    lk.unlock();
    sv->cv_work.notify_all();
    return LS_OK;
}

ls_status ls_server_wait(ls_server *sv, int64_t ticket, double timeout_s, ls_status *result)
{
    if (!sv) return LS_ERR_ARG;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) {
        sv->err = "unknown ticket";
        return LS_ERR_ARG;
    }
    Req *r = it->second.get();
    auto done = [&] { return r->st == St::Done; };
    if (timeout_s < 0) sv->cv_done.wait(lk, done);
    else if (!sv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) return LS_ERR_TIMEOUT;
    if (result) *result = r->result;
    return LS_OK;
}

ls_status ls_server_footprint(ls_server *sv, int64_t m, int64_t n, int64_t d, int64_t *resident,
                              int64_t *setup)
{
    if (!sv || !resident || !setup) return LS_ERR_ARG;
    if (n < 1 || n > LS_MAX_N || m < n || d < n || d >= (int64_t(1) << 31) || m * (int64_t)sv->zeta >= (int64_t(1) << 31))
        return LS_ERR_ARG;
    Req r;
    r.m = m;
    r.n = n;
    r.d = d;
    *resident = (sv->device >= 0) ? resident_bytes(&r) : 8 * m * n + 8 * m;
    *setup = setup_bytes(m, n, d, sv->zeta, sv->precision.load());
    return LS_OK;
}

ls_status ls_server_request_info(ls_server *sv, int64_t ticket, double *times)
{
    if (!sv || !times) return LS_ERR_ARG;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return LS_ERR_ARG;
    const Req *r = it->second.get();
    times[0] = r->t_submit;
    times[1] = r->t_admit;
    times[2] = r->t_start;
    times[3] = r->t_done;
    return LS_OK;
}

ls_status ls_server_stats(ls_server *sv, int64_t *stats)
{
    if (!sv || !stats) return LS_ERR_ARG;
    std::lock_guard<std::mutex> lk(sv->mu);
    stats[0] = sv->submitted;
    stats[1] = sv->completed;
    stats[2] = (int64_t)sv->queue.size();
    stats[3] = sv->admitted_live;
    stats[4] = sv->footprint_now;
    stats[5] = sv->footprint_peak;
    stats[6] = sv->rounds;
    stats[7] = sv->lanes_ws;
    return LS_OK;
}

ls_status ls_server_set_precision(ls_server *sv, int32_t precision)
{
    if (!sv || (precision != LS_PRECISION_FP64 && precision != LS_PRECISION_MIXED)) return LS_ERR_ARG;
    sv->precision.store(precision);
    return LS_OK;
}

ls_status ls_server_request_precision(ls_server *sv, int64_t ticket, int32_t *used)
{
    if (!sv || !used) return LS_ERR_ARG;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end()) return LS_ERR_ARG;
    *used = it->second->used;
    return LS_OK;
}

const char *ls_server_last_error(ls_server *sv)
{
    if (!sv) return "null server";
    std::lock_guard<std::mutex> lk(sv->mu);
    return sv->err.c_str();
}

}  // extern "C"
