// Fused refinement pass of iterative sketching on gfx950 (Algorithm 2 loop body; stable form of
// Section 3.2): c = A^T (b - A x) and ||b - A x||^2.
//
//   k_pass     for each row block, r = b - A x in registers (never stored), then acc += A^T r; each
//              work-group writes one partial of c and of ||r||^2.  A is read exactly once, as
//              coalesced segments of its rows; the grid is one wave of co-resident work-groups.
//   k_reduce   sums the partials in a fixed order (deterministic c and ||r||^2).
#include <mutex>

#include "common.hpp"

namespace {

constexpr int kPassThreads = 256;     // 4 waves per work-group
constexpr int kMaxPartials = 2048;

template <int G>
__device__ __forceinline__ double group_sum(double v)
{
    // Sum over the G consecutive lanes holding one row (G a power of two, <= 64).
#pragma unroll
    for (int off = 1; off < G; off <<= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// G lanes share one row; a wave holds 64/G rows at once and RT such row groups per tile.
// Lane sub (= lane % G) owns columns sub + G*c, c < CPL, so each load instruction of a row group
// reads G consecutive doubles.  Tiles are dealt round-robin over all waves of the grid, so at any
// moment the grid streams one contiguous window of A; A and b are read with non-temporal loads
// (each byte is used once, so they need not displace anything in the caches).
// With DX, the same row loads also give t = A_row . dx and the partial of ||A dx||^2 (part_ad): for
// dx = x_i - x_{i-1} that is ||r(x_{i-1}) - r(x_i)||^2, the left side of the stopping rule.
// A non-null `done` flag that is set makes the launch a no-op (the stopping rule has fired).
template <int G, int CPL, int RT, bool DX>
__device__ __forceinline__ void
pass_body(int vblock, int vgrid, int64_t m, int64_t n, const double *__restrict__ A, int64_t lda,
          const double *__restrict__ b, const double *__restrict__ x, double *__restrict__ part,
          double *__restrict__ part_rr, const double *__restrict__ dx, double *__restrict__ part_ad)
{
    constexpr int RPW = 64 / G;
    constexpr int TILE = RPW * RT;                   // rows per wave per tile
    constexpr int WAVES = kPassThreads / 64;
    __shared__ double s_acc[64 * CPL];
    __shared__ double s_rr[WAVES];
    __shared__ double s_ad[WAVES];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sub = lane % G, grp = lane / G;

    double xr[CPL], dr[CPL];
    bool cok[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int64_t col = sub + (int64_t)G * c;
        cok[c] = col < n;
        xr[c] = cok[c] ? x[col] : 0.0;
        dr[c] = (DX && cok[c]) ? dx[col] : 0.0;
    }
    double acc[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) acc[c] = 0.0;
    double rr = 0.0, ad = 0.0;

    const int64_t step = (int64_t)vgrid * WAVES * TILE;
    for (int64_t t0 = ((int64_t)vblock * WAVES + wave) * TILE; t0 < m; t0 += step) {
        double a[RT][CPL];
        double bb[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const int64_t row = t0 + (int64_t)t * RPW + grp;
            const bool rok = row < m;
            const double *ar = A + row * lda + sub;
#pragma unroll
            for (int c = 0; c < CPL; ++c)
                a[t][c] = (rok && cok[c]) ? __builtin_nontemporal_load(ar + G * c) : 0.0;
            bb[t] = rok ? __builtin_nontemporal_load(b + row) : 0.0;
        }
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            double dot = 0.0;
#pragma unroll
            for (int c = 0; c < CPL; ++c) dot = fma(a[t][c], xr[c], dot);
            dot = group_sum<G>(dot);
            const double r = bb[t] - dot;            // residual entry, FP64, before A^T
            if (sub == 0) rr = fma(r, r, rr);
            if (DX) {
                double td = 0.0;
#pragma unroll
                for (int c = 0; c < CPL; ++c) td = fma(a[t][c], dr[c], td);
                td = group_sum<G>(td);
                if (sub == 0) ad = fma(td, td, ad);
            }
#pragma unroll
            for (int c = 0; c < CPL; ++c) acc[c] = fma(a[t][c], r, acc[c]);
        }
    }
    // Sum the RPW row groups of the wave (lanes with equal sub), then the waves in fixed order.
#pragma unroll
    for (int off = G; off < 64; off <<= 1) {
#pragma unroll
        for (int c = 0; c < CPL; ++c) acc[c] += __shfl_xor(acc[c], off, 64);
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) rr += __shfl_xor(rr, off, 64);
    if (lane == 0) s_rr[wave] = rr;
    if (DX) {
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) ad += __shfl_xor(ad, off, 64);
        if (lane == 0) s_ad[wave] = ad;
    }
#pragma unroll
    for (int w = 0; w < WAVES; ++w) {
        if (wave == w && grp == 0) {
#pragma unroll
            for (int c = 0; c < CPL; ++c)
                s_acc[sub + G * c] = (w == 0) ? acc[c] : s_acc[sub + G * c] + acc[c];
        }
        __syncthreads();
    }
    for (int col = threadIdx.x; col < G * CPL; col += kPassThreads)
        if (col < n) part[(int64_t)vblock * n + col] = s_acc[col];
    if (threadIdx.x == 0) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < WAVES; ++w) s += s_rr[w];
        part_rr[vblock] = s;
        if (DX) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) t += s_ad[w];
            part_ad[vblock] = t;
        }
    }
}

template <int G, int CPL, int RT, bool DX>
__global__ void __launch_bounds__(kPassThreads)
k_pass(int64_t m, int64_t n, const double *__restrict__ A, int64_t lda, const double *__restrict__ b,
       const double *__restrict__ x, double *__restrict__ part, double *__restrict__ part_rr,
       const double *__restrict__ dx, double *__restrict__ part_ad, const int32_t *__restrict__ done)
{
    if (done && *done) return;
    pass_body<G, CPL, RT, DX>(blockIdx.x, gridDim.x, m, n, A, lda, b, x, part, part_rr, dx, part_ad);
}

// Served rounds: the pass of many resident problems in one launch.  Work-group w runs virtual
// work-group w - pass_base of problem wg_slot[w], out of that problem's own P partials, so each
// problem's arithmetic is exactly that of k_pass on it alone (ls_solve / ls_iterate).
template <int G, int CPL, int RT>
__global__ void __launch_bounds__(kPassThreads)
k_pass_served(const ServeSlot *__restrict__ slots, const int32_t *__restrict__ wg_slot)
{
    const ServeSlot &sl = slots[wg_slot[blockIdx.x]];
    pass_body<G, CPL, RT, false>((int)blockIdx.x - sl.pass_base, sl.P, sl.m, sl.n, sl.A, sl.lda, sl.b,
                                 sl.x, sl.part, sl.part_rr, nullptr, nullptr);
}

// c[col] = sum_p part[p][col] in a fixed order: 16 contiguous groups of partials, each summed in
// ascending p, then the 16 group sums in order.  Work-group 0 also reduces ||r||^2 likewise.
constexpr int kRedGroups = 16;

__device__ __forceinline__ void
reduce_body(int vblock, int32_t P, int64_t n, const double *__restrict__ part,
            const double *__restrict__ part_rr, double *__restrict__ c, double *__restrict__ rr_out,
            const double *__restrict__ part_ad, double *__restrict__ ad_out)
{
    __shared__ double s[kRedGroups][64];
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int64_t col = (int64_t)vblock * 64 + lane;
    const int32_t per = (P + kRedGroups - 1) / kRedGroups;
    const int32_t p_lo = g * per;
    const int32_t cnt = (p_lo + per < P) ? per : (P > p_lo ? P - p_lo : 0);
    s[g][lane] = (col < n) ? strided_sum<8>(part + (int64_t)p_lo * n + col, cnt, n) : 0.0;
    __syncthreads();
    if (g == 0 && col < n) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < kRedGroups; ++q) t += s[q][lane];
        c[col] = t;
    }
    if (vblock == 0 && rr_out) {
        __syncthreads();
        if (lane == 0) s[g][0] = strided_sum<8>(part_rr + p_lo, cnt, 1);
        if (lane == 1 && part_ad) s[g][1] = strided_sum<8>(part_ad + p_lo, cnt, 1);
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0, a = 0.0;
            for (int q = 0; q < kRedGroups; ++q) t += s[q][0];
            *rr_out = t;
            if (part_ad) {
                for (int q = 0; q < kRedGroups; ++q) a += s[q][1];
                *ad_out = a;
            }
        }
    }
}

__global__ void __launch_bounds__(64 * kRedGroups)
k_reduce(int32_t P, int64_t n, const double *__restrict__ part, const double *__restrict__ part_rr,
         double *__restrict__ c, double *__restrict__ rr_out, const double *__restrict__ part_ad,
         double *__restrict__ ad_out, const int32_t *__restrict__ done)
{
    if (done && *done) return;
    reduce_body(blockIdx.x, P, n, part, part_rr, c, rr_out, part_ad, ad_out);
}

// Served rounds: the reductions of many problems in one launch (work-group w does column block
// w - red_base of problem wg_slot[w]).
__global__ void __launch_bounds__(64 * kRedGroups)
k_reduce_served(const ServeSlot *__restrict__ slots, const int32_t *__restrict__ wg_slot)
{
    const ServeSlot &sl = slots[wg_slot[blockIdx.x]];
    reduce_body((int)blockIdx.x - sl.red_base, sl.P, sl.n, sl.part, sl.part_rr, sl.c, sl.rr, nullptr, nullptr);
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// The pass variant for a given n: G lanes per row, CPL columns per lane, RT row groups per tile.
struct PassVariant {
    const void *fn;
    int id;
};

template <int G, int CPL, int RT>
const void *pass_fn() { return reinterpret_cast<const void *>(&k_pass<G, CPL, RT, true>); }

PassVariant pass_variant(int64_t n)
{
    if (n <= 8) return {pass_fn<8, 1, 4>(), 0};
    if (n <= 16) return {pass_fn<16, 1, 4>(), 1};
    if (n <= 32) return {pass_fn<16, 2, 4>(), 2};
    if (n <= 64) return {pass_fn<16, 4, 4>(), 3};
    if (n <= 128) return {pass_fn<64, 2, 4>(), 4};
    if (n <= 256) return {pass_fn<64, 4, 4>(), 5};
    if (n <= 512) return {pass_fn<64, 8, 4>(), 6};
    if (n <= 1024) return {pass_fn<64, 16, 2>(), 7};
    return {pass_fn<64, 32, 1>(), 8};
}

// Work-groups that fit on the device at once for a variant (cached per device and variant).  The
// 257..512-column variant (id 6) takes one work-group per CU instead: with fewer row streams open at
// once it reads A at 7.1 TB/s, against 7.0 TB/s with all three that fit.  The variant for 2000
// columns measured faster with every resident work-group, so the others keep the full count.
int resident_wgs(int id, const void *fn)
{
    static int cache[64][9];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cache[dev][id] > 0) return cache[dev][id];
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kPassThreads, 0) != hipSuccess ||
        cus <= 0 || per_cu <= 0) {
        (void)hipGetLastError();
        return 256;
    }
    if (id == 6) per_cu = 1;
    cache[dev][id] = cus * per_cu;
    return cache[dev][id];
}

template <int G, int CPL, int RT>
void pass_launch(hipStream_t s, int P, int64_t m, int64_t n, const double *A, int64_t lda,
                 const double *b, const double *x, double *part, double *part_rr, const double *dx,
                 double *part_ad, const int32_t *done)
{
    if (dx)
        hipLaunchKernelGGL((k_pass<G, CPL, RT, true>), dim3(P), dim3(kPassThreads), 0, s, m, n, A, lda,
                           b, x, part, part_rr, dx, part_ad, done);
    else
        hipLaunchKernelGGL((k_pass<G, CPL, RT, false>), dim3(P), dim3(kPassThreads), 0, s, m, n, A, lda,
                           b, x, part, part_rr, dx, part_ad, done);
}

}  // namespace

int32_t pass_class(int64_t n) { return pass_variant(n).id; }

namespace {

template <int G, int CPL, int RT>
void served_pass_launch(hipStream_t s, int total_wg, const ServeSlot *slots, const int32_t *wg_slot)
{
    hipLaunchKernelGGL((k_pass_served<G, CPL, RT>), dim3(total_wg), dim3(kPassThreads), 0, s, slots, wg_slot);
}

}  // namespace

hipError_t launch_served_pass(hipStream_t s, int cls, int total_wg, const ServeSlot *slots,
                              const int32_t *wg_slot)
{
    if (total_wg <= 0) return hipSuccess;
    switch (cls) {                        // the classes of pass_variant
    case 0: served_pass_launch<8, 1, 4>(s, total_wg, slots, wg_slot); break;
    case 1: served_pass_launch<16, 1, 4>(s, total_wg, slots, wg_slot); break;
    case 2: served_pass_launch<16, 2, 4>(s, total_wg, slots, wg_slot); break;
    case 3: served_pass_launch<16, 4, 4>(s, total_wg, slots, wg_slot); break;
    case 4: served_pass_launch<64, 2, 4>(s, total_wg, slots, wg_slot); break;
    case 5: served_pass_launch<64, 4, 4>(s, total_wg, slots, wg_slot); break;
    case 6: served_pass_launch<64, 8, 4>(s, total_wg, slots, wg_slot); break;
    case 7: served_pass_launch<64, 16, 2>(s, total_wg, slots, wg_slot); break;
    default: served_pass_launch<64, 32, 1>(s, total_wg, slots, wg_slot); break;
    }
    return hipGetLastError();
}

hipError_t launch_served_reduce(hipStream_t s, int total_wg, const ServeSlot *slots, const int32_t *wg_slot)
{
    if (total_wg <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_served, dim3(total_wg), dim3(64 * kRedGroups), 0, s, slots, wg_slot);
    return hipGetLastError();
}

// Scratch of ls_gradient_noalloc: the P x n partials of c and the P partials of ||r||^2 (with the
// rest of an IterBufs carve) for any n <= LS_MAX_N, P <= kMaxPartials.  One copy per GPU, held until
// the process ends.  Host code never uses this name as an address: its device address on each GPU
// comes from hipGetSymbolAddress (pass_scratch_attach).
static_assert(kNoAllocScratchBytes >= (size_t)kMaxPartials * LS_MAX_N * sizeof(double) + (64u << 10),
              "scratch must hold the partials of the widest pass");
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

ls_status pass_scratch_attach(ls_ctx *ctx)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    if (ctx->device < 0 || ctx->device >= kMaxDevices)
        return ls_fail(ctx, LS_ERR_DEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[ctx->device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));   // the current device's copy
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return ls_fail(ctx, LS_ERR_DEVICE, std::string("scratch address: ") + hipGetErrorString(e));
        }
        addr[ctx->device] = p;
    }
    ctx->scratch = addr[ctx->device];
    return LS_OK;
}

int32_t iter_partials(int64_t m, int64_t n)
{
    // One wave of co-resident work-groups (at most one per 256 rows), or one per CU (id 6).
    const PassVariant v = pass_variant(n);
    int64_t P = resident_wgs(v.id, v.fn);
    if (P > kMaxPartials) P = kMaxPartials;
    const int64_t by_rows = ceil_div(m, 256);
    if (P > by_rows) P = by_rows;
    if (P < 1) P = 1;
    return (int32_t)P;
}

void iter_bufs(Arena &ar, int64_t m, int64_t n, IterBufs &ib, bool need_rt)
{
    ib.P = iter_partials(m, n);
    ib.part = ar.take<double>((size_t)ib.P * (size_t)n);
    ib.part_rr = ar.take<double>((size_t)ib.P);
    ib.part_ad = ar.take<double>((size_t)ib.P);
    ib.dx = ar.take<double>((size_t)n);
    ib.scal = ar.take<double>(8);
    ib.state = ar.take<int32_t>(8);
    ib.c = ar.take<double>((size_t)n);
    ib.xprev = ar.take<double>((size_t)n);
    ib.RT = need_rt ? ar.take<double>((size_t)n * (size_t)n) : nullptr;
}

hipError_t launch_gradient(hipStream_t s, int64_t m, int64_t n, const double *A, int64_t lda,
                           const double *b, const double *x, const IterBufs &ib, double *c,
                           double *rnorm2, hipEvent_t ev0, hipEvent_t ev1, const double *dx,
                           double *ad_out, const int32_t *done)
{
    const int P = ib.P;
    if (ev0) {
        hipError_t e0 = hipEventRecord(ev0, s);
        if (e0 != hipSuccess) return e0;
    }
    if (n <= 8) pass_launch<8, 1, 4>(s, P, m, n, A, lda, b, x, ib.part, ib.part_rr, dx, ib.part_ad, done);
    else if (n <= 16) pass_launch<16, 1, 4>(s, P, m, n, A, lda, b, x, ib.part, ib.part_rr, dx, ib.part_ad, done);
    else if (n <= 32) pass_launch<16, 2, 4>(s, P, m, n, A, lda, b, x, ib.part, ib.part_rr, dx, ib.part_ad, done);
    else if (n <= 64) pass_launch<16, 4, 4>(s, P, m, n, A, lda, b, x, ib.part, ib.part_rr, dx, ib.part_ad, done);
    else if (n <= 128) pass_launch<64, 2, 4>(s, P, m, n, A, lda, b, x, ib.part, ib.part_rr, dx, ib.part_ad, done);
    else if (n <= 256) pass_launch<64, 4, 4>(s, P, m, n, A, lda, b, x, ib.part, ib.part_rr, dx, ib.part_ad, done);
    else if (n <= 512) pass_launch<64, 8, 4>(s, P, m, n, A, lda, b, x, ib.part, ib.part_rr, dx, ib.part_ad, done);
    else if (n <= 1024) pass_launch<64, 16, 2>(s, P, m, n, A, lda, b, x, ib.part, ib.part_rr, dx, ib.part_ad, done);
    else if (n <= 2048) pass_launch<64, 32, 1>(s, P, m, n, A, lda, b, x, ib.part, ib.part_rr, dx, ib.part_ad, done);
    else return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev1) {
        e = hipEventRecord(ev1, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)ceil_div(n, 64)), dim3(64 * kRedGroups), 0, s, P, n, ib.part,
                       ib.part_rr, c, rnorm2, dx ? ib.part_ad : nullptr, ad_out, done);
    return hipGetLastError();
}

