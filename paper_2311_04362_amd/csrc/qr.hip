// Blocked Householder QR of the sketch [B | S b] (d x (n+1)) on gfx950 (Algorithm 2, third and
// fourth lines; eq. it-sk-qr; sketch-and-solve start eq. sketched_ls).
//
// Panels of kNB columns.  Inside a panel the reflectors are computed one column per launch
// (k_panel_step): every work-group owns RB consecutive rows held in registers; each launch
// (1) reduces, in a fixed order, the partial sums the previous launch left for this column,
// (2) forms the reflector H = I - tau v v^T with beta = -sign(alpha) ||column||, sign(0) = +1,
// (3) applies it to the rest of the panel, and (4) leaves the partial sums for the next column.
// No grid-wide barrier and no spin-wait: launch boundaries order the steps.
//
// After the panel, the compact-WY form Q_p = I - V T V^T (T upper triangular) is built and the
// trailing columns -- including the S b column, so Q is never formed -- are updated as
// C <- C - V (T^T (V^T C)) by four launches: V^T [V | C] over row chunks (k_vx_partial), the chunk
// sums (k_sum_partials), T and Z = T^T V^T C (k_tz), and C -= V Z (k_update_c).  Both products run on the matrix
// cores (v_mfma_f64_16x16x4f64, or v_mfma_f32_16x16x4f32 for the single-precision factorization of
// the mixed-precision path); every reduction has a fixed order, so the factorization is
// deterministic.  Every kernel is instantiated for FP64 and FP32.
//
// Look-ahead (large d n): after panel p the caller's stream updates only panel p+1's columns and
// factors panel p+1, while a second stream of the context updates the other trailing columns, so
// the latency-bound panel overlaps the bandwidth-bound update.  A column's update does not depend on
// which other columns share its launch, so the factorization's bits do not change.
#include <algorithm>
#include <type_traits>
#include <utility>

#include "common.hpp"

namespace {

constexpr int kNB = 32;     // panel width
// Rows per work-group in the panel kernels (one per thread), chosen from d alone so that both panel
// paths factor a given matrix alike: 512 rows (8 waves) for d >= kRBLargeFrom, where it measured
// fastest (205 -> 182 us per panel at d = 10^4), else 128 (2 waves), which gives the one-column
// launches of the served stream's small sketches more work-groups (687 -> 750 solves/s against 256).
constexpr int kRBSmall = 128;
constexpr int kRBLarge = 512;
constexpr int64_t kRBLargeFrom = 8192;
inline int panel_rows(int64_t d) { return d >= kRBLargeFrom ? kRBLarge : kRBSmall; }

// 16x16x4 MFMA per element type.  Operand layout (checked on gfx950 for both): A[i][kk] from lane
// i + 16 kk, B[kk][j] from lane j + 16 kk.  The accumulator layouts differ: element q of a lane's
// accumulator holds D[4 q + lane/16][lane % 16] for f64 and D[4 (lane/16) + q][lane % 16] for f32.
template <typename T> struct Mfma;
template <> struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(double a, double b, v4 c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int q, int lane) { return 4 * q + (lane >> 4); }
    static constexpr double kUnit = 0x1p-53;
};
template <> struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 mma(float a, float b, v4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int q, int lane) { return 4 * (lane >> 4) + q; }
    static constexpr float kUnit = 0x1p-24f;
};


// Exchanges between two registers across lane halves: with x, y on entry, lane l ends with
// x = (own x, or the partner's y) and y = (the partner's x, or own y), the partner being l ^ 32
// (v_permlane32_swap) or l ^ 16 (v_permlane16_swap), so x + y is what a lane of the lower half
// (lane & off == 0) gets by adding its x to the partner's x, and a lane of the upper half by
// adding its y to the partner's y.  (Lane layout of both instructions checked on gfx950.)
template <bool k32>
__device__ __forceinline__ void lane_swap(double &x, double &y)
{
    const uint64_t a = __builtin_bit_cast(uint64_t, x), b = __builtin_bit_cast(uint64_t, y);
    const unsigned alo = (unsigned)a, ahi = (unsigned)(a >> 32), blo = (unsigned)b, bhi = (unsigned)(b >> 32);
    const auto lo = k32 ? __builtin_amdgcn_permlane32_swap(alo, blo, false, false)
                        : __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
    const auto hi = k32 ? __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false)
                        : __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
    x = __builtin_bit_cast(double, ((uint64_t)(unsigned)hi[0] << 32) | (unsigned)lo[0]);
    y = __builtin_bit_cast(double, ((uint64_t)(unsigned)hi[1] << 32) | (unsigned)lo[1]);
}

template <bool k32>
__device__ __forceinline__ void lane_swap(float &x, float &y)
{
    const auto r = k32 ? __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, x), __builtin_bit_cast(unsigned, y), false, false)
                       : __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, x), __builtin_bit_cast(unsigned, y), false, false);
    x = __builtin_bit_cast(float, (unsigned)r[0]);
    y = __builtin_bit_cast(float, (unsigned)r[1]);
}

// Sums v[0..kNB) across the 64 lanes of a wave by recursive halving: at each step a lane keeps half
// of its values and adds the partner's copy of them (partner lane ^ 32, ^ 16, ..., ^ 1), so 32
// values need 16+8+4+2+1+1 exchanges.  The first two steps, which carry 24 of the 31 exchanges, are
// register swaps on the VALU (lane_swap); the rest go through ds_bpermute.
// On return lane l holds the wave total of value (l >> 1) & 31 (both lanes of a pair agree).
template <typename E>
__device__ __forceinline__ E wave_transpose_sum(E (&v)[kNB], int lane)
{
    static_assert(kNB == 32, "the swap steps take the partner offsets 32 and 16");
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        E x = v[i], y = v[i + 16];
        lane_swap<true>(x, y);
        v[i] = x + y;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        E x = v[i], y = v[i + 8];
        lane_swap<false>(x, y);
        v[i] = x + y;
    }
#pragma unroll
    for (int half = 4, off = 8; half >= 1; half >>= 1, off >>= 1) {
        const bool upper = (lane & off) != 0;
        E send[4], keep[4], recv[4];
        // A stage selects all its values first, then exchanges them all, then adds: the exchanges
        // of a stage are in flight together (one wait per stage, not one per value).  The empty
        // asm keeps each pair opaque: otherwise the compiler folds the selects into one load with
        // a lane-dependent index, which moves v to scratch memory.
#pragma unroll
        for (int i = 0; i < half; ++i) {
            E lo = v[i], hi = v[i + half];
            asm volatile("" : "+v"(lo), "+v"(hi));
            send[i] = upper ? lo : hi;
            keep[i] = upper ? hi : lo;
        }
#pragma unroll
        for (int i = 0; i < half; ++i) recv[i] = __shfl_xor(send[i], off, 64);
#pragma unroll
        for (int i = 0; i < half; ++i) v[i] = keep[i] + recv[i];
    }
    return v[0] + __shfl_xor(v[0], 1, 64);
}

// Value index held by lane l after wave_transpose_sum: the bits of l above bit 0, reversed over
// the five halving steps (the step with partner offset 32 decides the highest index bit).
__device__ __forceinline__ int transpose_sum_index(int lane)
{
    int idx = 0;
#pragma unroll
    for (int b = 0, off = 32; off >= 2; ++b, off >>= 1)
        if (lane & off) idx |= (kNB / 2) >> b;
    return idx;
}

// Panel step for column k = p0 + jc (jc = -1: no reflector yet, only the partial sums for the
// panel's first column).  red_in/piv_in hold what the previous launch left for column k:
//   red_in[w * kNB + l] = sum over rows of w (rows >= k) of W[i,k] W[i,p0+l]
//   piv_in[l]           = W[k, p0+l] (the pivot row, before this step)
// The launch writes the same quantities for column k+1 into red_out/piv_out.
template <typename E, int RB, bool FULL>
__global__ void __launch_bounds__(RB)
k_panel_step(int64_t d, int64_t p0, int nbp, int jc, int nwg, E *__restrict__ W, int64_t ldw,
             E *__restrict__ V, const E *__restrict__ red_in,
             const E *__restrict__ piv_in, E *__restrict__ red_out,
             E *__restrict__ piv_out, E *__restrict__ tau, int32_t *__restrict__ status)
{
    const int nb = FULL ? kNB : nbp;          // panel width (kNB for every panel but the last)
    __shared__ E s_tl[kNB];
    __shared__ E s_f[kNB];
    __shared__ E s_red[RB / kNB][kNB];
    __shared__ E s_part[RB / 64][kNB];
    __shared__ E s_scal[2];                       // beta, v_k
    const int tid = threadIdx.x;
    const int64_t k = p0 + jc;
    const int64_t i = p0 + (int64_t)blockIdx.x * RB + tid;   // this thread's row
    const bool row_ok = i < d;

    E w[kNB];
#pragma unroll
    for (int l = 0; l < kNB; ++l) w[l] = (row_ok && l < nb) ? W[i * ldw + p0 + l] : E(0);

    if (jc >= 0) {
        {   // reduce the partials: 8 contiguous groups of work-groups, then the groups in order
            constexpr int NS = RB / kNB;
            const int l = tid % kNB, sl = tid / kNB;
            const int per = (nwg + NS - 1) / NS;
            const int g0 = sl * per;
            const int cnt = (g0 + per < nwg) ? per : (nwg > g0 ? nwg - g0 : 0);
            s_red[sl][l] = strided_sum<8>(red_in + (int64_t)g0 * kNB + l, cnt, kNB);
            __syncthreads();
            if (tid < kNB) {
                E acc = E(0);
#pragma unroll
                for (int q = 0; q < NS; ++q) acc += s_red[q][tid];
                s_tl[tid] = acc;
            }
        }
        __syncthreads();
        if (tid == 0) {
            const E alpha = piv_in[jc];
            const E ss = s_tl[jc];
            const E sigma = sqrt(ss);
            E beta, t;
            if (sigma == E(0)) {               // exactly zero column: no reflection
                beta = E(0);
                t = E(0);
                atomicOr(status, ST_RANK);
            } else {
                beta = (alpha >= E(0)) ? -sigma : sigma;
                t = E(1) / (sigma * (sigma + fabs(alpha)));   // 2 / (v^T v)
            }
            if (!isfinite(sigma) || !isfinite(alpha)) atomicOr(status, ST_NONFINITE);
            s_scal[0] = beta;
            s_scal[1] = alpha - beta;
            if (blockIdx.x == 0) tau[k] = t;
            for (int l = 0; l < kNB; ++l)
                s_f[l] = (l > jc && l < nb) ? t * (s_tl[l] - beta * piv_in[l]) : E(0);
        }
        __syncthreads();
        if (row_ok) {
            E *vrow = V + (i - p0) * kNB;
            if (i >= k) {
                E wjc = E(0);
#pragma unroll
                for (int l = 0; l < kNB; ++l)
                    if (l == jc) wjc = w[l];
                const E vi = (i == k) ? s_scal[1] : wjc;
#pragma unroll
                for (int l = 0; l < kNB; ++l)
                    if (l > jc && l < nb) w[l] -= s_f[l] * vi;
                vrow[jc] = vi;
#pragma unroll
                for (int l = 0; l < kNB; ++l)
                    if (l == jc) w[l] = (i == k) ? s_scal[0] : E(0);
#pragma unroll
                for (int l = 0; l < kNB; ++l)
                    if (l >= jc && l < nb) W[i * ldw + p0 + l] = w[l];
            } else {
                vrow[jc] = E(0);
            }
        }
    } else if (row_ok) {
        E *vrow = V + (i - p0) * kNB;
#pragma unroll
        for (int l = 0; l < kNB; ++l) vrow[l] = E(0);
    }

    // Partial sums for column k+1 over rows >= k+1, and its pivot row.
    const int jn = jc + 1;
    if (jn < nb) {
        const bool part = row_ok && i >= k + 1;
        E wn = E(0);
#pragma unroll
        for (int l = 0; l < kNB; ++l)
            if (l == jn && part) wn = w[l];
        const int wave = tid >> 6, lane = tid & 63;
        E pv[kNB];
#pragma unroll
        for (int l = 0; l < kNB; ++l) pv[l] = (l >= jn && l < nb) ? wn * w[l] : E(0);
        const E tot = wave_transpose_sum(pv, lane);
        if ((lane & 1) == 0) s_part[wave][transpose_sum_index(lane)] = tot;
        if (i == k + 1) {
#pragma unroll
            for (int l = 0; l < kNB; ++l) piv_out[l] = w[l];
        }
        __syncthreads();
        if (tid < kNB) {
            E acc = E(0);
#pragma unroll
            for (int g = 0; g < RB / 64; ++g) acc += s_part[g][tid];
            red_out[blockIdx.x * kNB + tid] = acc;
        }
    }
}

// ---- Cooperative panel: one launch factors all kNB columns of a panel --------------------------
// Each work-group keeps RPT * RB rows of the panel in registers for the whole panel; a column step
// is local arithmetic plus one grid-wide exchange of kNB partial sums.  All work-groups are
// co-resident (cooperative launch), and each grid barrier spins a bounded number of times: if the
// bound is ever reached the kernel flags ST_TIMEOUT and runs to completion, so it always exits.
constexpr unsigned kSpinLimit = 1u << 20;
constexpr int kBarFlags = 1024;             // step flags: at most this many work-groups per panel
constexpr int kCounterBarrierWgs = 64;      // up to this many work-groups: one arrival counter
constexpr int kBarCounters = (LS_MAX_N + kNB - 1) / kNB;   // one counter per panel, after the flags
constexpr int kBarWords = kBarFlags + kBarCounters;         // zeroed once per factorization

// Calls f(std::integral_constant<int, J>{}) for J = 0, 1, ... in order.
template <class F, int... J>
__device__ __forceinline__ void for_each_column(F &f, std::integer_sequence<int, J...>)
{
    (f(std::integral_constant<int, J>{}), ...);
}

// Grid barrier by per-work-group step flags: after publishing its data, work-group g stores
// flag[g] = epoch with release semantics; the barrier waits until every flag has reached epoch.
// Flags only grow (epochs rise over the panels of a factorization), so they need no reset between
// panels.  The wait is bounded: past kSpinLimit polls the kernel flags ST_TIMEOUT and continues,
// so every work-group always finishes.
__device__ __forceinline__ void flag_barrier(unsigned *flags, int nwg, unsigned epoch, int32_t *status)
{
    __syncthreads();
    if (threadIdx.x < 64) {
        if (threadIdx.x == 0)
            __hip_atomic_store(flags + blockIdx.x, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        unsigned spins = 0;
        for (;;) {
            // a lane polls the flags of work-groups lane, lane + 64, ..., four loads in flight
            bool mine = true;
            for (int g0 = threadIdx.x; g0 < nwg; g0 += 256) {
                unsigned f[4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    f[u] = (g0 + 64 * u < nwg)
                               ? __hip_atomic_load(flags + g0 + 64 * u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                               : epoch;
#pragma unroll
                for (int u = 0; u < 4; ++u) mine &= f[u] >= epoch;
            }
            if (__all(mine)) break;
            if (++spins > kSpinLimit) {
                if (threadIdx.x == 0) atomicOr(status, ST_TIMEOUT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// Grid barrier by one arrival counter per panel: thread 0 of each work-group adds 1 with release
// semantics, then polls until the counter reaches `target` (nwg arrivals per barrier) and acquires.
// It measured faster than the step flags up to 40 work-groups (QR 4.02 -> 3.85 ms at d = 1e4,
// n = 500; 10.20 -> 9.93 ms at d = 2e4, n = 1000) and slower at 79 (33.7 -> 34.2 ms at d = 4e4,
// n = 2000), so the panel takes it up to kCounterBarrierWgs work-groups.  Same wait bound.
__device__ __forceinline__ void counter_barrier(unsigned *ctr, unsigned target, int32_t *status)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        unsigned spins = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > kSpinLimit) {
                atomicOr(status, ST_TIMEOUT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

template <typename E, int RPT, int RB, bool FULL>
__global__ void __launch_bounds__(RB)
k_panel_coop(int64_t d, int64_t p0, int nbp, int nwg, E *__restrict__ W, int64_t ldw,
             E *__restrict__ V, E *__restrict__ red, E *__restrict__ tau,
             unsigned *__restrict__ bar, unsigned epoch0, int32_t *__restrict__ status)
{
    const int nb = FULL ? kNB : nbp;          // panel width (kNB for every panel but the last)
    __shared__ E s_tl[kNB];
    __shared__ E s_f[kNB];
    __shared__ E s_part[RB / 64][kNB];
    __shared__ E s_red[RB / kNB][kNB];
    __shared__ E s_scal[2];
    __shared__ E s_piv[kNB];
    __shared__ int s_haspiv;
    // The panel's Householder vectors for this work-group's rows, column-major (conflict-free):
    // written to V once after the last column, so the barriers' release fences do not also push
    // V stores out of L2 at every column.
    __shared__ E s_v[kNB][RPT * RB];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    E *piv = red + 2 * (int64_t)nwg * kNB;            // 2 x kNB pivot rows
    const int tidx = transpose_sum_index(lane);
    int64_t row[RPT];
    bool ok[RPT];
    E w[RPT][kNB];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        row[r] = p0 + ((int64_t)blockIdx.x * RPT + r) * RB + tid;
        ok[r] = row[r] < d;
#pragma unroll
        for (int l = 0; l < kNB; ++l) w[r][l] = (ok[r] && l < nb) ? W[row[r] * ldw + p0 + l] : E(0);
    }
    // One column step.  The steps are expanded at compile time (for_each_column below, always
    // inlined), so every register index is static -- a runtime index would put the row arrays in
    // scratch memory or behind select chains.
    auto column = [&](auto jcc) __attribute__((always_inline)) {
        constexpr int jc = decltype(jcc)::value;
        if (jc >= nb) return;
        const int64_t k = p0 + jc;
        const int pb = jc & 1;
        E *rb = red + (int64_t)pb * nwg * kNB;
        // (1) partial sums of column jc over my rows >= k, and the pivot row
        {
            E pv[kNB];
#pragma unroll
            for (int l = 0; l < kNB; ++l) pv[l] = E(0);
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                const bool use = ok[r] && row[r] >= k;
#pragma unroll
                for (int l = jc; l < kNB; ++l)
                    if (use && l < nb) pv[l] += w[r][jc] * w[r][l];
            }
            const E tot = wave_transpose_sum(pv, lane);
            if ((lane & 1) == 0) s_part[wave][tidx] = tot;
        }
        if (tid == 0) s_haspiv = 0;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RPT; ++r)
            if (row[r] == k) {
#pragma unroll
                for (int l = 0; l < kNB; ++l) s_piv[l] = w[r][l];
                s_haspiv = 1;
            }
        __syncthreads();
        // wave 0 publishes the partials (and the pivot row, from its owner): the barrier's release
        // fence, issued by thread 0, then covers every store the other work-groups will read
        if (tid < kNB) {
            E acc = E(0);
#pragma unroll
            for (int g = 0; g < RB / 64; ++g) acc += s_part[g][tid];
            rb[(int64_t)blockIdx.x * kNB + tid] = acc;
            if (s_haspiv) piv[pb * kNB + tid] = s_piv[tid];
        }
        if (nwg <= kCounterBarrierWgs)        // panel p's counter: bar[kBarFlags + p], apart from the flags
            counter_barrier(bar + kBarFlags + epoch0 / (kNB + 1), (unsigned)nwg * (unsigned)(jc + 1), status);
        else
            flag_barrier(bar, nwg, epoch0 + (unsigned)(jc + 1), status);
        // (2) every work-group reduces the partials in the same fixed order
        {
            constexpr int NS = RB / kNB;
            const int l = tid % kNB, sl = tid / kNB;
            const int per = (nwg + NS - 1) / NS;
            const int g0 = sl * per;
            const int cnt = (g0 + per < nwg) ? per : (nwg > g0 ? nwg - g0 : 0);
            s_red[sl][l] = strided_sum<8>(rb + (int64_t)g0 * kNB + l, cnt, kNB);
            if (tid < kNB) s_piv[tid] = piv[pb * kNB + tid];
            __syncthreads();
            if (tid < kNB) {
                E acc = E(0);
#pragma unroll
                for (int q = 0; q < NS; ++q) acc += s_red[q][tid];
                s_tl[tid] = acc;
            }
            __syncthreads();
        }
        // (3) reflector H = I - tau v v^T, beta = -sign(alpha) sigma (every one of the first kNB
        // threads forms the same scalars), then the update coefficients of the panel columns
        if (tid < kNB) {
            const E alpha = s_piv[jc];
            const E sigma = sqrt(s_tl[jc]);
            E beta, t;
            if (sigma == E(0)) {
                beta = E(0);
                t = E(0);
            } else {
                beta = (alpha >= E(0)) ? -sigma : sigma;
                t = E(1) / (sigma * (sigma + fabs(alpha)));   // 2 / (v^T v)
            }
            const int l = tid;
            s_f[l] = (l > jc && l < nb) ? t * (s_tl[l] - beta * s_piv[l]) : E(0);
            if (tid == 0) {
                if (sigma == E(0)) atomicOr(status, ST_RANK);
                if (!isfinite(sigma) || !isfinite(alpha)) atomicOr(status, ST_NONFINITE);
                s_scal[0] = beta;
                s_scal[1] = alpha - beta;
                if (blockIdx.x == 0) tau[k] = t;
            }
        }
        __syncthreads();
        // (4) apply the reflector to my rows; entry jc of each row's Householder vector goes to V
        // (zero for rows above the pivot)
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            if (!ok[r]) continue;
            const bool below = row[r] >= k;
            const E vi = (row[r] == k) ? s_scal[1] : w[r][jc];
            s_v[jc][r * RB + tid] = below ? vi : E(0);
            if (!below) continue;
#pragma unroll
            for (int l = jc + 1; l < kNB; ++l)
                if (l < nb) w[r][l] -= s_f[l] * vi;
            w[r][jc] = (row[r] == k) ? s_scal[0] : E(0);
        }
    };
    for_each_column(column, std::make_integer_sequence<int, kNB>{});
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        if (!ok[r]) continue;
#pragma unroll
        for (int l = 0; l < kNB; ++l)
            if (l < nb) W[row[r] * ldw + p0 + l] = w[r][l];
        E *vrow = V + (row[r] - p0) * kNB;
#pragma unroll
        for (int l = 0; l < kNB; ++l) vrow[l] = (l < nb) ? s_v[l][r * RB + tid] : E(0);
    }
}

__global__ void k_zero_u32(unsigned *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Work-group id -> (major, minor) tile for a grid of 8 ceil(nmajor / 8) nminor work-groups: every
// tile of one major index (a row block or chunk, which shares its rows of V) runs on one XCD
// (work-group i runs on XCD i mod 8), minor indices in order.  False for the padding past nmajor.
__device__ __forceinline__ bool xcd_tile(int64_t id, int64_t nmajor, int64_t nminor, int64_t &major, int64_t &minor)
{
    const int64_t j = id / 8;
    major = id % 8 + 8 * (j / nminor);
    minor = j % nminor;
    return major < nmajor;
}

// P[ch][a][c] = sum over the rows r of chunk ch of V[r][a] X[r][c], for X = [V | C] (column c < kNB
// of X is column c of V, column c >= kNB is column c - kNB of C), a < kNB, c < nx = kNB + nc.
// Work-group: 64 columns of X.  Its four waves take interleaved groups of 4 rows of the chunk
// (split-K), each wave 32 x 64 in eight MFMA accumulators; the waves' results are added in wave
// order through LDS, so the partial is deterministic.  Operand and accumulator rows as in Mfma<E>.
template <typename E>
__global__ void __launch_bounds__(256)
k_vx_partial(int64_t rows, int64_t chunk, const E *__restrict__ V, const E *__restrict__ C,
             int64_t ldc, int64_t nx, int64_t ldo, E *__restrict__ P, int64_t nch)
{
    __shared__ E s_acc[4][kNB][64 + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t ch, cblk;
    if (!xcd_tile(blockIdx.x, nch, (nx + 63) / 64, ch, cblk)) return;
    const int64_t r_lo = ch * chunk;
    const int64_t r_hi = (r_lo + chunk < rows) ? r_lo + chunk : rows;
    const int kk = lane >> 4, ii = lane & 15;
    // Column 16 s + ii of this block, s < 4: its source array, leading dimension and validity.
    const E *src[4];
    int64_t lds[4];
    bool cok[4];
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) {
        const int64_t col = cblk * 64 + 16 * sb + ii;
        cok[sb] = col < nx;
        src[sb] = (col < kNB) ? V + col : C + (col - kNB);
        lds[sb] = (col < kNB) ? (int64_t)kNB : ldc;
    }
    typename Mfma<E>::v4 acc[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) acc[h][sb] = (typename Mfma<E>::v4){E(0), E(0), E(0), E(0)};
    // Rows r, r + 16, r + 32, r + 48 of this wave are loaded together, then applied in that order.
    for (int64_t r = r_lo + 4 * wave; r < r_hi; r += 64) {
        E a0[4], a1[4], bv[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t rr = r + 16 * u + kk;
            const bool ok = rr < r_hi;
            a0[u] = ok ? V[rr * kNB + ii] : E(0);
            a1[u] = ok ? V[rr * kNB + 16 + ii] : E(0);
#pragma unroll
            for (int sb = 0; sb < 4; ++sb) bv[u][sb] = (ok && cok[sb]) ? src[sb][rr * lds[sb]] : E(0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int sb = 0; sb < 4; ++sb) {
                acc[0][sb] = Mfma<E>::mma(a0[u], bv[u][sb], acc[0][sb]);
                acc[1][sb] = Mfma<E>::mma(a1[u], bv[u][sb], acc[1][sb]);
            }
    }
#pragma unroll
    for (int sb = 0; sb < 4; ++sb)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int a = Mfma<E>::row(q, lane);
            s_acc[wave][a][16 * sb + ii] = acc[0][sb][q];
            s_acc[wave][16 + a][16 * sb + ii] = acc[1][sb][q];
        }
    __syncthreads();
    for (int e = threadIdx.x; e < kNB * 64; e += blockDim.x) {
        const int a = e / 64, c = e % 64;
        const int64_t col = cblk * 64 + c;
        if (col >= nx) continue;
        const E t = ((s_acc[0][a][c] + s_acc[1][a][c]) + s_acc[2][a][c]) + s_acc[3][a][c];
        P[(ch * kNB + a) * ldo + col] = t;
    }
}

// P[0][a][c] <- sum over chunks ch of P[ch][a][c], added in chunk order, for a < kNB, c < nx.
// Work-group (64-column block, 4 rows of the 32): one entry per thread, so the chunk partials of a
// panel are summed by many compute units at once.  Each thread reads its entry of every chunk
// before writing the sum over chunk 0's.
template <typename E>
__global__ void __launch_bounds__(256)
k_sum_partials(int nch, int64_t ldo, int64_t nx, E *__restrict__ P)
{
    const int a = blockIdx.y * 4 + (threadIdx.x >> 6);
    const int64_t c = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
    if (c >= nx) return;
    E *p = P + (int64_t)a * ldo + c;
    p[0] = strided_sum<8>(p, nch, (int64_t)kNB * ldo);
}

// For one 64-column block of the trailing columns: G = V^T V and Y = V^T C are the chunk sums of P
// (added in chunk order); T is the compact-WY factor, T[j][j] = tau_j and T[0:j, j] =
// -tau_j T[0:j, 0:j] G[0:j, j], formed by every work-group in its first wave; then
// Z[:, c] = T^T Y[:, c].
template <typename E>
__global__ void __launch_bounds__(1024)
k_tz(int nch, int64_t ldo, const E *__restrict__ P, const E *__restrict__ tau, int64_t p0, int nbp,
     int64_t nc, E *__restrict__ Z, int64_t ldz)
{
    __shared__ E G[kNB][kNB + 1];
    __shared__ E Ts[kNB][kNB + 1];
    __shared__ E Y[kNB][64 + 1];
    __shared__ E s_tau[kNB];
    const int tid = threadIdx.x;
    const int64_t pstride = (int64_t)kNB * ldo;
    if (tid < kNB) s_tau[tid] = (tid < nbp) ? tau[p0 + tid] : E(0);
    {
        // Three chunk sums per thread (one entry of G, two of Y), each added in ascending chunk
        // order; their loads are interleaved so that 24 are in flight at a time.
        const int ga = tid / kNB, gc = tid % kNB;
        const E *pg = P + (int64_t)ga * ldo + gc;
        const E *py[2];
        bool yok[2];
        int ya[2], ycl[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int e = tid + h * 1024;
            ya[h] = e / 64;
            ycl[h] = e % 64;
            const int64_t c = (int64_t)blockIdx.x * 64 + ycl[h];
            yok[h] = c < nc;
            py[h] = P + (int64_t)ya[h] * ldo + kNB + (yok[h] ? c : 0);
        }
        E g = E(0), y[2] = {E(0), E(0)};
        for (int c0 = 0; c0 < nch; c0 += 8) {
            E vg[8], vy[2][8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const bool in = c0 + u < nch;
                const int64_t off = (int64_t)(c0 + u) * pstride;
                vg[u] = in ? pg[off] : E(0);
#pragma unroll
                for (int h = 0; h < 2; ++h) vy[h][u] = (in && yok[h]) ? py[h][off] : E(0);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (c0 + u >= nch) break;
                g += vg[u];
#pragma unroll
                for (int h = 0; h < 2; ++h) y[h] += vy[h][u];
            }
        }
        G[ga][gc] = g;
        Ts[ga][gc] = E(0);
#pragma unroll
        for (int h = 0; h < 2; ++h) Y[ya[h]][ycl[h]] = y[h];
    }
    __syncthreads();
    // Row i of T needs only its own earlier entries: T[i][j] = -tau_j sum_{q=i}^{j-1} T[i][q] G[q][j],
    // summed in ascending q.  Lane i of the first wave forms row i (it reads back only its own row).
    if (tid < nbp) {
        const int i = tid;
        Ts[i][i] = s_tau[i];
        for (int j = i + 1; j < nbp; ++j) {
            E acc = E(0);
#pragma unroll 8
            for (int q = i; q < j; ++q) acc += Ts[i][q] * G[q][j];
            Ts[i][j] = -s_tau[j] * acc;
        }
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int e = tid + h * 1024;
        const int a = e / 64, cl = e % 64;
        const int64_t c = (int64_t)blockIdx.x * 64 + cl;
        if (c >= nc) continue;
        E z = E(0);
        for (int b2 = 0; b2 <= a; ++b2) z += Ts[b2][a] * Y[b2][cl];
        Z[(int64_t)a * ldz + c] = z;
    }
}

// C[r][c] -= sum_a V[r][a] Z[a][c] over rows r < rows, columns c < nc.
// Work-group tile 256 x 64: wave w owns rows 64w..64w+63 in four 16-row blocks and four 16-column
// MFMA blocks.  The wave loads its 32 x 64 slice of Z once and keeps it in registers for its four
// row blocks (Z was reloaded for every 16 rows before: more load instructions than C itself).  Each
// entry's products are accumulated over a in the same order as before, so the bits are the same.
constexpr int kUpdRows = 256;

template <typename E>
__global__ void __launch_bounds__(256)
k_update_c(int64_t rows, int64_t nc, const E *__restrict__ V, const E *__restrict__ Z,
           int64_t ldz, E *__restrict__ C, int64_t ldc)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t rblk, cblk;
    if (!xcd_tile(blockIdx.x, (rows + kUpdRows - 1) / kUpdRows, (nc + 63) / 64, rblk, cblk)) return;
    const int64_t c0 = cblk * 64;
    const int kk = lane >> 4, ii = lane & 15;
    // this lane's operands of Z: row a + kk, column c0 + 16 cb + ii, for a = 0, 4, ..., kNB - 4
    E zv[kNB / 4][4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        const int64_t cc = c0 + 16 * cb + ii;
#pragma unroll
        for (int a4 = 0; a4 < kNB / 4; ++a4)
            zv[a4][cb] = (cc < nc) ? Z[(int64_t)(4 * a4 + kk) * ldz + cc] : E(0);
    }
    for (int rb = 0; rb < 4; ++rb) {
        const int64_t r0 = rblk * kUpdRows + 64 * wave + 16 * rb;
        if (r0 >= rows) break;
        const int64_t ra = r0 + ii;
        const bool ra_ok = ra < rows;
        // this lane's 16 entries of C, loaded first so that their latency overlaps the products
        E cv[4][4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const int64_t cc = c0 + 16 * cb + ii;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t r = r0 + Mfma<E>::row(q, lane);
                cv[cb][q] = (cc < nc && r < rows) ? C[r * ldc + cc] : E(0);
            }
        }
        typename Mfma<E>::v4 acc[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[cb] = (typename Mfma<E>::v4){E(0), E(0), E(0), E(0)};
#pragma unroll
        for (int a4 = 0; a4 < kNB / 4; ++a4) {
            const E av = ra_ok ? V[ra * kNB + 4 * a4 + kk] : E(0);
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) acc[cb] = Mfma<E>::mma(av, zv[a4][cb], acc[cb]);
        }
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            const int64_t cc = c0 + 16 * cb + ii;
            if (cc >= nc) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t r = r0 + Mfma<E>::row(q, lane);
                if (r < rows) C[r * ldc + cc] = cv[cb][q] - acc[cb][q];
            }
        }
    }
}

// Mixed path: W32 = [fl32(B) | fl32(Sb)] from the FP64 sketch (B in W64's first n columns, Sb
// contiguous), each entry rounded once.
__global__ void __launch_bounds__(256)
k_round_sketch(int64_t d, int64_t n, const double *__restrict__ B, int64_t ldb,
               const double *__restrict__ Sb, float *__restrict__ W, int64_t ldw)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t w = n + 1;
    if (e >= d * w) return;
    const int64_t i = e / w, c = e % w;
    W[i * ldw + c] = (float)((c < n) ? B[i * ldb + c] : Sb[i]);
}

// Column n of the FP64 work matrix = Sb (the mixed path's fallback to the FP64 QR).
__global__ void __launch_bounds__(256)
k_set_rhs(int64_t d, int64_t n, const double *__restrict__ Sb, double *__restrict__ W, int64_t ldw)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d) W[i * ldw + n] = Sb[i];
}

template <typename E>
__global__ void __launch_bounds__(256)
k_copy_sketch(int64_t d, int64_t n, const E *__restrict__ B, int64_t ldb,
              const E *__restrict__ Sb, E *__restrict__ W, int64_t ldw)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t w = n + 1;
    if (e >= d * w) return;
    const int64_t i = e / w, c = e % w;
    W[i * ldw + c] = (c < n) ? B[i * ldb + c] : Sb[i];
}

// R (upper triangle of W), R^T, Q^T Sb; flags NaN/Inf.
template <typename E>
__global__ void __launch_bounds__(256)
k_extract_r(int64_t n, const E *__restrict__ W, int64_t ldw, E *__restrict__ R,
            int64_t ldr, E *__restrict__ RT, E *__restrict__ qtb,
            int32_t *__restrict__ status)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n) return;
    const int64_t i = e / n, c = e % n;
    const E v = (c >= i) ? W[i * ldw + c] : E(0);
    if (R) R[i * ldr + c] = v;
    RT[c * n + i] = v;
    if (c == 0) {
        const E q = W[i * ldw + n];
        qtb[i] = q;
        if (!isfinite(q)) atomicOr(status, ST_NONFINITE);
    }
    if (!isfinite(v)) atomicOr(status, ST_NONFINITE);
}

// Rank test on diag(R): |R_kk| <= n u max_j |R_jj|.
template <typename E>
__global__ void __launch_bounds__(256)
k_rank_check(int64_t n, const E *__restrict__ RT, int32_t *__restrict__ status)
{
    __shared__ E smax[4];
    E mx = E(0);
    for (int64_t k = threadIdx.x; k < n; k += blockDim.x) mx = fmax(mx, fabs(RT[k * n + k]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = mx;
    __syncthreads();
    mx = fmax(fmax(smax[0], smax[1]), fmax(smax[2], smax[3]));
    const E tol = (E)n * Mfma<E>::kUnit * mx;
    for (int64_t k = threadIdx.x; k < n; k += blockDim.x)
        if (!(fabs(RT[k * n + k]) > tol)) atomicOr(status, ST_RANK);
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

int64_t panel_wgs_max(int64_t d) { return ceil_div(d, kRBSmall); }

int64_t chunk_rows(int64_t rows)
{
    int64_t ch = ceil_div(rows, 64);
    if (ch < 256) ch = 256;
    return ceil_div(ch, 4) * 4;
}

}  // namespace

template <typename E>
static void qr_bufs_impl(Arena &ar, int64_t d, int64_t n, QrBufsT<E> &qb, bool lookahead)
{
    qb.ldw = ceil_div(n + 1, 8) * 8;
    qb.W = ar.take<E>((size_t)d * (size_t)qb.ldw);
    qb.V = ar.take<E>((size_t)d * kNB);
    qb.red = ar.take<E>((size_t)2 * (size_t)(panel_wgs_max(d) * kNB + kNB));
    qb.tau = ar.take<E>((size_t)n);
    // every panel uses at most min(64, ceil(rows/256)) chunks (see chunk_rows)
    const int64_t nch = std::min<int64_t>(64, ceil_div(d, 256));
    const int64_t ldo = ceil_div(n + 1, 64) * 64 + 64;
    qb.Yp = ar.take<E>((size_t)nch * kNB * (size_t)ldo);
    qb.Z = ar.take<E>((size_t)kNB * (size_t)qb.ldw);
    qb.qtb = ar.take<E>((size_t)n);
    qb.RT = ar.take<E>((size_t)n * (size_t)n);
    qb.bar = ar.take<unsigned>(kBarWords);
    if (lookahead) {
        qb.V2 = ar.take<E>((size_t)d * kNB);
        qb.Yp2 = ar.take<E>((size_t)nch * kNB * (size_t)ldo);
        qb.Z2 = ar.take<E>((size_t)kNB * (size_t)qb.ldw);
    }
}

void qr_bufs(Arena &ar, int64_t d, int64_t n, QrBufs &qb, bool lookahead) { qr_bufs_impl(ar, d, n, qb, lookahead); }
void qr_bufs(Arena &ar, int64_t d, int64_t n, QrBufs32 &qb, bool lookahead) { qr_bufs_impl(ar, d, n, qb, lookahead); }

template <typename E>
static hipError_t copy_sketch_impl(hipStream_t s, int64_t d, int64_t n, const E *B, int64_t ldb,
                                   const E *Sb, const QrBufsT<E> &qb)
{
    const int64_t total = d * (n + 1);
    hipLaunchKernelGGL(k_copy_sketch<E>, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s, d, n,
                       B, ldb, Sb, qb.W, qb.ldw);
    return hipGetLastError();
}

hipError_t launch_copy_sketch(hipStream_t s, int64_t d, int64_t n, const double *B, int64_t ldb,
                              const double *Sb, const QrBufs &qb)
{
    return copy_sketch_impl(s, d, n, B, ldb, Sb, qb);
}

hipError_t launch_copy_sketch(hipStream_t s, int64_t d, int64_t n, const float *B, int64_t ldb,
                              const float *Sb, const QrBufs32 &qb)
{
    return copy_sketch_impl(s, d, n, B, ldb, Sb, qb);
}

hipError_t launch_round_sketch(hipStream_t s, int64_t d, int64_t n, const QrBufs &qb64, const double *Sb,
                               const QrBufs32 &qb32)
{
    const int64_t total = d * (n + 1);
    hipLaunchKernelGGL(k_round_sketch, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, s, d, n,
                       (const double *)qb64.W, qb64.ldw, Sb, qb32.W, qb32.ldw);
    return hipGetLastError();
}

hipError_t launch_set_rhs(hipStream_t s, int64_t d, int64_t n, const double *Sb, const QrBufs &qb)
{
    hipLaunchKernelGGL(k_set_rhs, dim3((unsigned)ceil_div(d, 256)), dim3(256), 0, s, d, n, Sb, qb.W, qb.ldw);
    return hipGetLastError();
}

namespace {

// Work-groups of k_panel_coop<E, RPT> that can be co-resident on the current device (0: cooperative
// launch unavailable).  Cached per device.
template <typename E, int RPT, int RB, bool FULL>
int coop_capacity()
{
    static int cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (cache[dev] != 0) return cache[dev] > 0 ? cache[dev] : 0;
    int coop = 0, cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(&k_panel_coop<E, RPT, RB, FULL>), RB, 0) != hipSuccess ||
        per_cu <= 0) {
        (void)hipGetLastError();
        cache[dev] = -1;
        return 0;
    }
    cache[dev] = cus * per_cu;
    return cache[dev];
}

// The step flags carry epochs that grow over all panels of one factorization (panel p uses
// p (kNB + 1) + 1 ... p (kNB + 1) + kNB), and each panel has its own arrival counter, so flags and
// counters are cleared once, before the factorization's first cooperative panel (zero_flags), not
// before every panel.
template <typename E, int RPT, int RB, bool FULL>
hipError_t launch_panel_coop(hipStream_t s, int64_t d, int64_t p0, int nbp, int nwg, E *W,
                             int64_t ldw, E *V, E *red, E *tau, unsigned *bar, bool zero_flags,
                             int32_t *status)
{
    if (zero_flags) hipLaunchKernelGGL(k_zero_u32, dim3((kBarWords + 255) / 256), dim3(256), 0, s, bar, kBarWords);
    unsigned epoch0 = (unsigned)(p0 / kNB) * (unsigned)(kNB + 1);
    void *args[] = {&d, &p0, &nbp, &nwg, &W, &ldw, &V, &red, &tau, &bar, &epoch0, &status};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(&k_panel_coop<E, RPT, RB, FULL>), dim3(nwg),
                                      dim3(RB), args, 0, s);
}

// One panel by the cooperative kernel if the device can hold its grid; returns false to request
// the per-column path.
template <typename E, int RB>
bool panel_cooperative(hipStream_t s, int64_t d, int64_t p0, int nbp, const QrBufsT<E> &qb, E *V,
                       bool &flags_zeroed, int32_t *status, hipError_t &err)
{
    // One row per thread, as in k_panel_step: the work-groups' partial sums are then grouped exactly
    // as the per-column path groups them, so the two paths give the same bits.  A grid too large
    // to be co-resident takes the per-column path.
    const int64_t rows = d - p0;
    err = hipSuccess;
    const int nwg = (int)ceil_div(rows, RB);
    const bool full = nbp == kNB;
    if (nwg > kBarFlags || nwg > (full ? coop_capacity<E, 1, RB, true>() : coop_capacity<E, 1, RB, false>()))
        return false;
    err = full ? launch_panel_coop<E, 1, RB, true>(s, d, p0, nbp, nwg, qb.W, qb.ldw, V, qb.red, qb.tau, qb.bar,
                                                   !flags_zeroed, status)
               : launch_panel_coop<E, 1, RB, false>(s, d, p0, nbp, nwg, qb.W, qb.ldw, V, qb.red, qb.tau, qb.bar,
                                                    !flags_zeroed, status);
    flags_zeroed = true;
    return true;
}

// Trailing update C <- Q_p^T C of columns [c0, c1) of the work matrix by panel p0's reflectors V
// (the four launches described at the top), with chunk partials Yp and Z.  Each column's arithmetic
// depends only on V, tau and that column, so splitting the columns over launches keeps the bits.
template <typename E>
void trailing_update(hipStream_t s, int64_t d, int64_t n, const QrBufsT<E> &qb, int64_t p0, int nbp,
                     const E *V, E *Yp, E *Z, int64_t c0, int64_t c1)
{
    const int64_t ldw = qb.ldw;
    const int64_t rows = d - p0;
    const int64_t nc = c1 - c0;
    const int64_t chunk = chunk_rows(rows);
    const int nch = (int)ceil_div(rows, chunk);
    const int64_t ldo = ceil_div(n + 1, 64) * 64 + 64;
    const E *C0 = qb.W + p0 * ldw + c0;
    hipLaunchKernelGGL(k_vx_partial<E>, dim3((unsigned)(8 * ceil_div(nch, 8) * ceil_div(kNB + nc, 64))), dim3(256), 0,
                       s, rows, chunk, V, C0, ldw, (int64_t)kNB + nc, ldo, Yp, (int64_t)nch);
    hipLaunchKernelGGL(k_sum_partials<E>, dim3((unsigned)ceil_div(kNB + nc, 64), kNB / 4), dim3(256), 0, s,
                       nch, ldo, (int64_t)kNB + nc, Yp);
    hipLaunchKernelGGL(k_tz<E>, dim3((unsigned)ceil_div(nc, 64)), dim3(1024), 0, s, 1, ldo, Yp,
                       qb.tau, p0, nbp, nc, Z, ldw);
    hipLaunchKernelGGL(k_update_c<E>, dim3((unsigned)(8 * ceil_div(ceil_div(rows, kUpdRows), 8) * ceil_div(nc, 64))),
                       dim3(256), 0, s, rows, nc, V, Z, ldw, qb.W + p0 * ldw + c0, ldw);
}

// The factorization, panel by panel.  With look-ahead (la and qb.V2), after panel p the caller's
// stream s updates panel p+1's columns and factors panel p+1 while la->side updates the remaining
// columns; s waits for the side stream before it touches columns the side stream updated, and panels
// alternate between V and V2 so that panel p+1 never overwrites vectors the side stream still reads.
template <typename E>
hipError_t qr_impl(hipStream_t s, int64_t d, int64_t n, const QrBufsT<E> &qb, int32_t *status,
                   bool per_column, const QrAside *la)
{
    const int64_t ldw = qb.ldw;
    const int64_t red_stride = panel_wgs_max(d) * kNB + kNB;
    E *redA = qb.red, *redB = qb.red + red_stride;
    const bool ahead = la && la->side && qb.V2 && !per_column && n > kNB;
    bool flags_zeroed = false;
    if (ahead) {
        // the side stream starts after everything before the factorization on s
        if (hipEventRecord(la->panel_done, s) != hipSuccess ||
            hipStreamWaitEvent(la->side, la->panel_done, 0) != hipSuccess ||
            hipEventRecord(la->side_done, la->side) != hipSuccess)
            return hipGetLastError();
    }
    for (int64_t p0 = 0; p0 < n; p0 += kNB) {
        const int nbp = (int)((n - p0 < kNB) ? n - p0 : kNB);
        const int64_t rows = d - p0;
        E *V = (ahead && ((p0 / kNB) & 1)) ? qb.V2 : qb.V;
        hipError_t err = hipSuccess;
        const int rb = panel_rows(d);
        const bool coop = !per_column && (rb == kRBLarge
                                              ? panel_cooperative<E, kRBLarge>(s, d, p0, nbp, qb, V, flags_zeroed, status, err)
                                              : panel_cooperative<E, kRBSmall>(s, d, p0, nbp, qb, V, flags_zeroed, status, err));
        if (!coop) {
            const int nwg = (int)ceil_div(rows, rb);
            E *rin = redA, *rout = redB;
            const bool full = nbp == kNB;
            for (int jc = -1; jc < nbp; ++jc) {
#define LS_PANEL_STEP(RBV, FULLV)                                                                              \
    hipLaunchKernelGGL((k_panel_step<E, RBV, FULLV>), dim3(nwg), dim3(RBV), 0, s, d, p0, nbp, jc, nwg, qb.W, ldw, V, \
                       rin, rin + (int64_t)nwg * kNB, rout, rout + (int64_t)nwg * kNB, qb.tau, status)
                if (rb == kRBLarge) {
                    if (full) LS_PANEL_STEP(kRBLarge, true);
                    else LS_PANEL_STEP(kRBLarge, false);
                } else {
                    if (full) LS_PANEL_STEP(kRBSmall, true);
                    else LS_PANEL_STEP(kRBSmall, false);
                }
#undef LS_PANEL_STEP
                E *t = rin;
                rin = rout;
                rout = t;
            }
        }
        if (err != hipSuccess) return err;
        const int64_t c_first = p0 + nbp;                      // trailing columns c_first..n (S b last)
        const int64_t next = (n - c_first < kNB) ? n - c_first : kNB;   // the next panel's columns
        if (ahead && next > 0) {
            // order: s records the panel, waits for the side stream's last update (it updated the
            // next panel's columns), then updates them; the side stream waits for the panel only
            if (hipEventRecord(la->panel_done, s) != hipSuccess ||
                hipStreamWaitEvent(s, la->side_done, 0) != hipSuccess ||
                hipStreamWaitEvent(la->side, la->panel_done, 0) != hipSuccess)
                return hipGetLastError();
            trailing_update(la->side, d, n, qb, p0, nbp, V, qb.Yp2, qb.Z2, c_first + next, n + 1);
            if (hipEventRecord(la->side_done, la->side) != hipSuccess) return hipGetLastError();
            trailing_update(s, d, n, qb, p0, nbp, V, qb.Yp, qb.Z, c_first, c_first + next);
        } else {
            if (ahead && hipStreamWaitEvent(s, la->side_done, 0) != hipSuccess) return hipGetLastError();
            trailing_update(s, d, n, qb, p0, nbp, V, qb.Yp, qb.Z, c_first, n + 1);
        }
    }
    return hipGetLastError();
}

template <typename E>
hipError_t extract_r_impl(hipStream_t s, int64_t n, const QrBufsT<E> &qb, E *R, int64_t ldr,
                          int32_t *status)
{
    hipLaunchKernelGGL(k_extract_r<E>, dim3((unsigned)ceil_div(n * n, 256)), dim3(256), 0, s, n, qb.W,
                       qb.ldw, R, ldr, qb.RT, qb.qtb, status);
    hipLaunchKernelGGL(k_rank_check<E>, dim3(1), dim3(256), 0, s, n, qb.RT, status);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_qr(hipStream_t s, int64_t d, int64_t n, const QrBufs &qb, int32_t *status,
                     bool per_column, const QrAside *la)
{
    return qr_impl(s, d, n, qb, status, per_column, la);
}

hipError_t launch_qr(hipStream_t s, int64_t d, int64_t n, const QrBufs32 &qb, int32_t *status,
                     bool per_column, const QrAside *la)
{
    return qr_impl(s, d, n, qb, status, per_column, la);
}

hipError_t launch_extract_r(hipStream_t s, int64_t n, const QrBufs &qb, double *R, int64_t ldr,
                            int32_t *status)
{
    return extract_r_impl(s, n, qb, R, ldr, status);
}

hipError_t launch_extract_r(hipStream_t s, int64_t n, const QrBufs32 &qb, float *R, int64_t ldr,
                            int32_t *status)
{
    return extract_r_impl(s, n, qb, R, ldr, status);
}
