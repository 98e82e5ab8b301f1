// Triangular solves and update of iterative sketching on gfx950 (Algorithm 2: d_i = R^{-1} (R^{-T} c_i),
// x_{i+1} = x_i + d_i; the damping / momentum update of eq. damping_momentum; the sketch-and-solve
// start x_0 = R^{-1} (Q^T S b)).
//
//   k_solve       one work-group: R^T y = c by forward substitution, R d = y by back substitution
//                 (32-wide diagonal blocks by one wave while the other waves apply earlier blocks
//                 as coalesced GEMV updates; no inverse matrix is ever formed), then the update.
//                 One CU streams R twice, so the GEMV waves read 16 bytes per load (two doubles,
//                 or four floats) when the rows allow it: one CU's read rate rises from about 76
//                 to 114 GB/s, and each unknown's sum keeps its order and its bits.
//   k_back        back substitution alone (x_0).
//   k_transpose   R^T for the column reads of the back substitution.
//
// Every kernel is instantiated for FP64 and for FP32 factors.  With an FP32 factor (mixed precision)
// the right-hand side is scaled by a power of two that brings its largest entry into [1/2, 1),
// rounded once to FP32, solved in FP32, and scaled back exactly in FP64; the update stays FP64.
#include "common.hpp"

namespace {

__device__ __forceinline__ double readlane(double v, int l)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)(u & 0xFFFFFFFFull), l);
    const int hi = __builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ float readlane(float v, int l)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// Buffer-descriptor loads for the GEMV updates: the lane's byte offset travels in a VGPR and the
// row's byte offset, uniform across the wave, in an SGPR, so 32 loads in flight cost no address
// registers.  The descriptor covers `bytes` bytes from `base` (at most 2^31 - 1).  The hardware
// range check is not relied on: callers load only rows that exist and clamp the column index of
// lanes that have nothing to load into the matrix.
template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rows_rsrc(const T *base, int64_t bytes)
{
    const int nb = (int)(bytes <= 0 ? 0 : (bytes < 0x7FFFFFFF ? bytes : 0x7FFFFFFF));
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(base), (short)0, nb, 0x00020000);
}

__device__ __forceinline__ double rows_load(__amdgpu_buffer_rsrc_t rs, double *, uint32_t vbytes, uint32_t sbytes)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)vbytes, (int)sbytes, 0));
}

__device__ __forceinline__ float rows_load(__amdgpu_buffer_rsrc_t rs, float *, uint32_t vbytes, uint32_t sbytes)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)vbytes, (int)sbytes, 0));
}

// sum over u < kSB of M[u][j] w[u] in ascending u (M row-major with leading dimension ld, behind
// the descriptor rs), all loads issued first.  Rows from `count` on repeat row count-1 and must meet
// zeros in w.
template <typename T, int kSB>
__device__ __forceinline__ T rows_dot(__amdgpu_buffer_rsrc_t rs, int64_t ld, int64_t j, const T *w, int count)
{
    T v[kSB];
#pragma unroll
    for (int u = 0; u < kSB; ++u)
        v[u] = rows_load(rs, (T *)nullptr, (uint32_t)(j * (int64_t)sizeof(T)),
                         (uint32_t)((u < count ? u : count - 1) * ld * (int64_t)sizeof(T)));
    T acc = T(0);
#pragma unroll
    for (int u = 0; u < kSB; ++u) acc += v[u] * w[u];
    return acc;
}

// VW consecutive entries of one row (VW = 1: rows_load; otherwise one 16-byte load of two doubles
// or four floats, the byte offsets 16-byte aligned).
template <typename T, int VW>
__device__ __forceinline__ void rows_loadw(__amdgpu_buffer_rsrc_t rs, uint32_t vbytes, uint32_t sbytes, T (&out)[VW])
{
    if constexpr (VW == 1) {
        out[0] = rows_load(rs, (T *)nullptr, vbytes, sbytes);
    } else {
        static_assert(VW * sizeof(T) == 16, "16-byte loads take two doubles or four floats");
        const auto q = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)vbytes, (int)sbytes, 0);
        if constexpr (sizeof(T) == 8) {
            out[0] = __builtin_bit_cast(double, ((uint64_t)(uint32_t)q[1] << 32) | (uint32_t)q[0]);
            out[1] = __builtin_bit_cast(double, ((uint64_t)(uint32_t)q[3] << 32) | (uint32_t)q[2]);
        } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) out[v] = __builtin_bit_cast(float, (uint32_t)q[v]);
        }
    }
}

// rows_dot for the VW unknowns j .. j+VW-1: acc[v] = sum over u < kSB of M[u][j+v] w[u] in ascending
// u (so each unknown's sum is rows_dot's, bit for bit).  The rows go in kSB / VW at a time, all loads
// of a group issued first: the same bytes in flight as rows_dot, in the same registers.
template <typename T, int kSB, int VW>
__device__ __forceinline__ void rows_dotw(__amdgpu_buffer_rsrc_t rs, int64_t ld, int64_t j, const T *w, int count,
                                          T (&acc)[VW])
{
    constexpr int kG = kSB / VW;
#pragma unroll
    for (int q = 0; q < VW; ++q) acc[q] = T(0);
#pragma unroll
    for (int u0 = 0; u0 < kSB; u0 += kG) {
        T v[kG][VW];
#pragma unroll
        for (int u = 0; u < kG; ++u)
            rows_loadw<T, VW>(rs, (uint32_t)(j * (int64_t)sizeof(T)),
                              (uint32_t)((u0 + u < count ? u0 + u : count - 1) * ld * (int64_t)sizeof(T)), v[u]);
#pragma unroll
        for (int u = 0; u < kG; ++u)
#pragma unroll
            for (int q = 0; q < VW; ++q) acc[q] += v[u][q] * w[u0 + u];
    }
}

// Diagonal block of the substitutions used by the library, and the solve kernels' work-group size.
constexpr int kSolveBlock = 32;
constexpr int kSolveThreads = 512;

// LDS of the substitution kernels: double-buffered diagonal block, the reciprocals of its diagonal,
// and the block of R that couples the current block of unknowns to the next one.
template <typename T, int kSB>
struct SubstLds {
    T diag[2][kSB][kSB + 1];
    T rdiag[2][kSB];
    T off[2][kSB][kSB + 1];
};

// The LDS data of diagonal block b, numbered e < 2 kSB^2 + kSB: the diagonal block, the coupling
// block (forward: R[b, b+1], the terms of block b in the equations of block b+1; backward:
// R[b-1, b]) and the reciprocals of the diagonal.  Zero (reciprocal one) outside the n x n matrix.
// The load always reads a valid address (clamped into the matrix) and the value is fixed up when it
// is stored, so a wave issues all its loads without waiting on any of them.
template <typename T, int kSB>
struct BlockData {
    static constexpr int kCount = 2 * kSB * kSB + kSB;

    template <bool kForward>
    static __device__ __forceinline__ void where(int64_t n, int b, int e, int64_t &r, int64_t &c, bool &inside)
    {
        const int64_t b0 = (int64_t)b * kSB;
        if (e < kSB * kSB) {
            r = b0 + e / kSB;
            c = b0 + e % kSB;
        } else if (e < 2 * kSB * kSB) {
            const int f = e - kSB * kSB;
            r = (kForward ? b0 : b0 - kSB) + f / kSB;
            c = (kForward ? b0 + kSB : b0) + f % kSB;
        } else {
            r = c = b0 + (e - 2 * kSB * kSB);
        }
        inside = r >= 0 && r < n && c >= 0 && c < n;
    }

    template <bool kForward>
    static __device__ __forceinline__ T load(const T *__restrict__ R, int64_t ldr, int64_t n, int b, int e)
    {
        int64_t r, c;
        bool inside;
        where<kForward>(n, b, e, r, c, inside);
        r = r < 0 ? 0 : (r < n ? r : n - 1);
        c = c < 0 ? 0 : (c < n ? c : n - 1);
        return R[r * ldr + c];
    }

    template <bool kForward>
    static __device__ __forceinline__ void store(SubstLds<T, kSB> &L, int buf, int64_t n, int b, int e, T raw)
    {
        int64_t r, c;
        bool inside;
        where<kForward>(n, b, e, r, c, inside);
        if (e < kSB * kSB) L.diag[buf][e / kSB][e % kSB] = inside ? raw : T(0);
        else if (e < 2 * kSB * kSB) L.off[buf][(e - kSB * kSB) / kSB][(e - kSB * kSB) % kSB] = inside ? raw : T(0);
        else L.rdiag[buf][e - 2 * kSB * kSB] = inside ? T(1) / raw : T(1);
    }
};

// One block's LDS data staged in the registers of wave 1 (the stager): loaded a step before it is
// needed, written to the idle LDS buffer the step after.  Element e = lane + 64 p of BlockData's
// numbering sits in v[p]: p < 16 the diagonal block (row 2p + lane/32, column lane%32), p < 32 the
// coupling block (same pattern), p = 32 the diagonal entries (lanes < 32).  Away from the edges of
// the matrix the loads go through two buffer descriptors with the row offsets in SGPRs, so a step
// costs 33 loads and 33 LDS writes; blocks that touch an edge take the clamped element-wise path.
template <typename T, int kSB>
struct Stage {
    static_assert(kSB == 32, "two rows of a 32-wide block per 64-lane access");
    static constexpr int kPer = 33;
    T v[kPer];

    template <bool kForward>
    static __device__ __forceinline__ bool edge(int64_t n, int b)
    {
        const int64_t b0 = (int64_t)b * kSB;
        return kForward ? (b0 + 2 * kSB > n) : (b < 1 || b0 + kSB > n);
    }

    template <bool kForward>
    __device__ __forceinline__ void load(const T *__restrict__ R, int64_t ldr, int64_t n, int b, int lane)
    {
        const int64_t b0 = (int64_t)b * kSB;
        if (edge<kForward>(n, b)) {
#pragma unroll
            for (int p = 0; p < kPer; ++p) {
                const int e = lane + p * 64;
                v[p] = BlockData<T, kSB>::template load<kForward>(R, ldr, n, b, e < BlockData<T, kSB>::kCount ? e : 0);
            }
            return;
        }
        const int64_t span = ((int64_t)(kSB - 1) * ldr + kSB) * (int64_t)sizeof(T);
        const auto rd = rows_rsrc(R + b0 * ldr + b0, span);
        const auto ro = rows_rsrc(kForward ? R + b0 * ldr + b0 + kSB : R + (b0 - kSB) * ldr + b0, span);
        const uint32_t vo = (uint32_t)(((int64_t)(lane >> 5) * ldr + (lane & 31)) * (int64_t)sizeof(T));
#pragma unroll
        for (int p = 0; p < 16; ++p) {
            const uint32_t so = (uint32_t)(2 * p * ldr * (int64_t)sizeof(T));
            v[p] = rows_load(rd, (T *)nullptr, vo, so);
            v[16 + p] = rows_load(ro, (T *)nullptr, vo, so);
        }
        v[32] = rows_load(rd, (T *)nullptr, (uint32_t)((int64_t)(lane & 31) * (ldr + 1) * (int64_t)sizeof(T)), 0u);
    }

    template <bool kForward>
    __device__ __forceinline__ void store(SubstLds<T, kSB> &L, int buf, int64_t n, int b, int lane) const
    {
        if (edge<kForward>(n, b)) {
#pragma unroll
            for (int p = 0; p < kPer; ++p) {
                const int e = lane + p * 64;
                if (e < BlockData<T, kSB>::kCount) BlockData<T, kSB>::template store<kForward>(L, buf, n, b, e, v[p]);
            }
            return;
        }
        const int r = lane >> 5, c = lane & 31;
#pragma unroll
        for (int p = 0; p < 16; ++p) {
            L.diag[buf][2 * p + r][c] = v[p];
            L.off[buf][2 * p + r][c] = v[16 + p];
        }
        if (lane < 32) L.rdiag[buf][lane] = T(1) / v[32];
    }
};

// Rows of R (forward) or R^T (backward) that each GEMV wave prefetches for the next step's update:
// 32 entries of one unknown per slot, 128 VGPRs either way (the 512-thread work-group leaves 256
// VGPRs per wave; the estimators, which keep more state, use one slot).
template <typename T>
struct Prefetch {
    static constexpr int kSlots = sizeof(T) == 8 ? 2 : 4;
};

// Solves one diagonal block in wave 0: lane l holds unknown l (v) and column l of the block
// (col[li] = T[li][l] of the triangular factor being applied, T = R^T forward or R backward).
// Each lane scales its equation by the rounded reciprocal of its diagonal entry first, so unknown
// li is lane li's value itself: it is broadcast with readlane and removed from every lane.  (This
// is substitution on the system with unit diagonal; every entry carries one extra rounding.)  The
// factor's other triangle is zero (the library only hands the kernels R with a zero lower
// triangle), so lanes already solved or not yet reached keep their value, and lane li's own entry
// goes to the result.  A partial last block is padded (zero entries, unit reciprocals, zero
// unknowns), so the loop has no branch; the column is read from LDS before the loop.  Lanes
// 32..63 compute values nobody reads.
template <typename T, int kSB, bool kForward>
__device__ __forceinline__ T block_solve(T v, const T (*diag)[kSB + 1], const T *rdiag, int lane)
{
    const int lc = lane & (kSB - 1);
    const T rd = rdiag[lc];
    T col[kSB];
#pragma unroll
    for (int li = 0; li < kSB; ++li) col[li] = (kForward ? diag[li][lc] : diag[lc][li]) * rd;
    v *= rd;
    T res = T(0);
#pragma unroll
    for (int q = 0; q < kSB; ++q) {
        const int li = kForward ? q : kSB - 1 - q;
        const T yi = readlane(v, li);
        v -= col[li] * yi;
        res = (lane == li) ? yi : res;
    }
    return res;
}

// Contribution of the solved block (y, one unknown per lane) to the next block's unknowns:
// lane l gets sum over li of cpl(li, l) y_li, in four interleaved partial sums added pairwise.
template <typename T, int kSB, bool kForward>
__device__ __forceinline__ T block_carry(T y, const T (*off)[kSB + 1], int lane)
{
    const int lc = lane & (kSB - 1);
    T o[kSB];
#pragma unroll
    for (int li = 0; li < kSB; ++li) o[li] = kForward ? off[li][lc] : off[lc][li];
    T a[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int li = 0; li < kSB; ++li) a[li & 3] += o[li] * readlane(y, li);
    return (a[0] + a[1]) + (a[2] + a[3]);
}

// Forward substitution R^T y = v in place on s[] (R upper triangular with a zero lower triangle,
// row-major; s holds n unknowns followed by zeros up to a multiple of kSB), by a work-group of
// kThreads threads in three roles.  Each role runs its own loop with one barrier per block (the
// barrier counts waves, so the loops stay in step), which keeps their registers and their
// outstanding loads apart.
//   wave 0 (solver), step k:  solves block k (block_solve) and forms its contribution to block k+1
//                             (the "carry", block_carry).
//   wave 1 (stager), step k:  writes the LDS data of block k+1, loaded during step k-1, into the
//                             idle buffer, then loads block k+2's.
//   waves 2.. (GEMV), step k: apply block k-1 to every unknown past block k+1, over rows of R loaded
//                             during step k-1 (unknowns beyond the prefetch slots load theirs in the
//                             step), then load the rows of block k for step k+1.
// So no load of R waits on the solver's critical path.  Each unknown receives the terms of earlier
// blocks in a fixed order, and no two waves write one entry in one phase.  Unknowns are divided by
// R_ii as multiplication by the rounded reciprocal.
template <typename T, int kSB, int kThreads, int kPF = Prefetch<T>::kSlots, int VW = 1>
__device__ __forceinline__ void fwd_subst(int64_t n, const T *__restrict__ R, int64_t ldr, T *s,
                                          SubstLds<T, kSB> &L)
{
    constexpr int kG = kThreads - 128;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nblk = (int)((n + kSB - 1) / kSB);
    for (int e = tid; e < BlockData<T, kSB>::kCount; e += kThreads)
        BlockData<T, kSB>::template store<true>(L, 0, n, 0, e, BlockData<T, kSB>::template load<true>(R, ldr, n, 0, e));
    if (wave == 0) {
        __syncthreads();
        T carry = T(0);
        for (int k = 0; k < nblk; ++k) {
            const int64_t i0 = (int64_t)k * kSB;
            const int nb = (int)((i0 + kSB < n) ? kSB : n - i0);
            const int buf = k & 1;
            T v = (lane < nb) ? s[i0 + lane] - carry : T(0);
            v = block_solve<T, kSB, true>(v, L.diag[buf], L.rdiag[buf], lane);
            if (lane < nb) s[i0 + lane] = v;
            if (k + 1 < nblk) carry = block_carry<T, kSB, true>(v, L.off[buf], lane);
            __syncthreads();
        }
        return;
    }
    if (wave == 1) {
        Stage<T, kSB> stage;
        if (nblk > 1) stage.template load<true>(R, ldr, n, 1, lane);
        __syncthreads();
        for (int k = 0; k < nblk; ++k) {
            if (k + 1 < nblk) stage.template store<true>(L, (k & 1) ^ 1, n, k + 1, lane);
            if (k + 2 < nblk) stage.template load<true>(R, ldr, n, k + 2, lane);
            __syncthreads();
        }
        return;
    }
    // GEMV waves: a thread takes VW consecutive unknowns per slot (VW = 2: 16-byte loads; n and ldr
    // even), so kPF / VW slots fill the same registers.
    constexpr int kS = kPF / VW > 0 ? kPF / VW : 1;
    const int th = tid - 128;
    T pr[kS][kSB][VW];
    __syncthreads();
    for (int k = 0; k < nblk; ++k) {
        const int64_t i0 = (int64_t)k * kSB;
        const int64_t lo = i0 + kSB;                    // first unknown past block k
        if (k >= 1) {                                   // block k-1 (always full) -> unknowns lo..n-1
            const int64_t p0 = i0 - kSB;
#pragma unroll
            for (int r = 0; r < kS; ++r) {
                const int64_t j = lo + (int64_t)VW * (th + (int64_t)r * kG);
                if (j < n) {
#pragma unroll
                    for (int q = 0; q < VW; ++q) {
                        T acc = T(0);
#pragma unroll
                        for (int u = 0; u < kSB; ++u) acc += pr[r][u][q] * s[p0 + u];
                        s[j + q] -= acc;
                    }
                }
            }
            if (lo + (int64_t)VW * ((int64_t)kS * kG + th) < n) {
                const auto rs = rows_rsrc(R + p0 * ldr, ((int64_t)(kSB - 1) * ldr + n) * (int64_t)sizeof(T));
                for (int64_t j = lo + (int64_t)VW * ((int64_t)kS * kG + th); j < n; j += (int64_t)VW * kG) {
                    T acc[VW];
                    rows_dotw<T, kSB, VW>(rs, ldr, j, s + p0, kSB, acc);
#pragma unroll
                    for (int q = 0; q < VW; ++q) s[j + q] -= acc[q];
                }
            }
        }
        if (k + 1 < nblk) {                             // rows of block k (full) for unknowns lo+kSB..
            const auto rs = rows_rsrc(R + i0 * ldr, ((int64_t)(kSB - 1) * ldr + n) * (int64_t)sizeof(T));
#pragma unroll
            for (int r = 0; r < kS; ++r) {
                const int64_t q0 = (int64_t)VW * ((int64_t)(wave - 2) * 64 + (int64_t)r * kG);   // first unknown of the wave
                if (lo + kSB + q0 < n) {                // wave-uniform
                    const int64_t j = lo + kSB + (int64_t)VW * (th + (int64_t)r * kG);
                    const int64_t jc = j < n ? j : n - VW;
#pragma unroll
                    for (int u = 0; u < kSB; ++u)
                        rows_loadw<T, VW>(rs, (uint32_t)(jc * (int64_t)sizeof(T)),
                                          (uint32_t)(u * ldr * (int64_t)sizeof(T)), pr[r][u]);
                }
            }
        }
        __syncthreads();
    }
}

// Back substitution R z = v in place on s[] (padded as in fwd_subst); RT = R^T (row-major, ld n)
// gives the columns of R contiguously for the GEMV updates.  Same roles as fwd_subst, blocks taken
// from the last; the GEMV waves apply block B+1 to unknowns 0..B*kSB-1.
template <typename T, int kSB, int kThreads, int kPF = Prefetch<T>::kSlots, int VW = 1>
__device__ __forceinline__ void back_subst(int64_t n, const T *__restrict__ R, int64_t ldr,
                                           const T *__restrict__ RT, T *s, SubstLds<T, kSB> &L)
{
    constexpr int kG = kThreads - 128;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nblk = (int)((n + kSB - 1) / kSB);
    for (int e = tid; e < BlockData<T, kSB>::kCount; e += kThreads)
        BlockData<T, kSB>::template store<false>(L, 0, n, nblk - 1, e,
                                                 BlockData<T, kSB>::template load<false>(R, ldr, n, nblk - 1, e));
    if (wave == 0) {
        __syncthreads();
        T carry = T(0);
        for (int t = 0; t < nblk; ++t) {
            const int B = nblk - 1 - t;
            const int64_t i0 = (int64_t)B * kSB;
            const int nb = (int)((i0 + kSB < n) ? kSB : n - i0);
            const int buf = t & 1;
            T v = (lane < nb) ? s[i0 + lane] - carry : T(0);
            v = block_solve<T, kSB, false>(v, L.diag[buf], L.rdiag[buf], lane);
            if (lane < nb) s[i0 + lane] = v;
            if (B >= 1) carry = block_carry<T, kSB, false>(v, L.off[buf], lane);
            __syncthreads();
        }
        return;
    }
    if (wave == 1) {
        Stage<T, kSB> stage;
        if (nblk > 1) stage.template load<false>(R, ldr, n, nblk - 2, lane);
        __syncthreads();
        for (int t = 0; t < nblk; ++t) {
            const int B = nblk - 1 - t;
            if (B >= 1) stage.template store<false>(L, (t & 1) ^ 1, n, B - 1, lane);
            if (B >= 2) stage.template load<false>(R, ldr, n, B - 2, lane);
            __syncthreads();
        }
        return;
    }
    constexpr int kS = kPF / VW > 0 ? kPF / VW : 1;
    const int th = tid - 128;
    T pr[kS][kSB][VW];
    __syncthreads();
    for (int t = 0; t < nblk; ++t) {
        const int B = nblk - 1 - t;
        const int64_t i0 = (int64_t)B * kSB;
        if (t >= 1) {                                   // block B+1 -> unknowns 0..i0-1
            const int64_t p0 = i0 + kSB;
#pragma unroll
            for (int r = 0; r < kS; ++r) {
                const int64_t j = (int64_t)VW * (th + (int64_t)r * kG);
                if (j < i0) {
#pragma unroll
                    for (int q = 0; q < VW; ++q) {
                        T acc = T(0);
#pragma unroll
                        for (int u = 0; u < kSB; ++u) acc += pr[r][u][q] * s[p0 + u];   // padded s: zero past n
                        s[j + q] -= acc;
                    }
                }
            }
            if ((int64_t)VW * ((int64_t)kS * kG + th) < i0) {
                const int pb = (int)((p0 + kSB < n) ? kSB : n - p0);
                const auto rs = rows_rsrc(RT + p0 * n, (n - p0) * n * (int64_t)sizeof(T));
                for (int64_t j = (int64_t)VW * ((int64_t)kS * kG + th); j < i0; j += (int64_t)VW * kG) {
                    T acc[VW];
                    rows_dotw<T, kSB, VW>(rs, n, j, s + p0, pb, acc);
#pragma unroll
                    for (int q = 0; q < VW; ++q) s[j + q] -= acc[q];
                }
            }
        }
        if (B >= 1) {                                   // columns of block B for unknowns 0..i0-kSB-1
            const int nb = (int)((i0 + kSB < n) ? kSB : n - i0);
            const auto rs = rows_rsrc(RT + i0 * n, (n - i0) * n * (int64_t)sizeof(T));
#pragma unroll
            for (int r = 0; r < kS; ++r) {
                const int64_t q0 = (int64_t)VW * ((int64_t)(wave - 2) * 64 + (int64_t)r * kG);
                if (q0 < i0 - kSB) {                    // wave-uniform
                    const int64_t j = (int64_t)VW * (th + (int64_t)r * kG);
                    const int64_t jc = j < n ? j : n - VW;
                    // rows past n (partial last block) repeat row n-1: they meet zeros in s
#pragma unroll
                    for (int u = 0; u < kSB; ++u)
                        rows_loadw<T, VW>(rs, (uint32_t)(jc * (int64_t)sizeof(T)),
                                          (uint32_t)((u < nb ? u : nb - 1) * n * (int64_t)sizeof(T)), pr[r][u]);
                }
            }
        }
        __syncthreads();
    }
}

// Block-wide sum in a fixed order (wave reductions, then the waves in order); all threads get it.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *red)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    T t = T(0);
    for (int w = 0; w < nw; ++w) t += red[w];
    return t;
}

// Block-wide maximum; all threads get it.
__device__ __forceinline__ double block_max(double v, double *red)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t = fmax(t, red[w]);
    return t;
}

// Unknowns of the substitutions live in LDS padded to a multiple of the block (zeros past n).
template <int kSB>
__host__ __device__ constexpr int64_t padded(int64_t n) { return (n + kSB - 1) / kSB * kSB; }

template <typename T, int kSB>
__device__ __forceinline__ void zero_pad(int64_t n, T *s)
{
    for (int64_t j = n + threadIdx.x; j < padded<kSB>(n); j += blockDim.x) s[j] = T(0);
}

// Right-hand side c (FP64) into the solve type: unchanged for FP64; for FP32, scaled by 2^-e with
// e the exponent of max |c| (frexp: max |c| 2^-e in [1/2, 1)) and rounded once.  Returns e.
template <typename T>
__device__ __forceinline__ int load_rhs(int64_t n, const double *__restrict__ c, T *s, double *red)
{
    if (sizeof(T) == 8) {
        for (int64_t j = threadIdx.x; j < n; j += blockDim.x) s[j] = (T)c[j];
        return 0;
    }
    double mx = 0.0;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) mx = fmax(mx, fabs(c[j]));
    mx = block_max(mx, red);
    int e = 0;
    if (mx > 0.0 && isfinite(mx)) (void)frexp(mx, &e);
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) s[j] = (T)ldexp(c[j], -e);
    return e;
}

// d = R^{-1} (R^{-T} c), then the update selected by mode (see launch_solve_update).  With a
// stopping rule (st.state != nullptr): once the done flag is set the launch is a no-op; when
// st.check is set the rule of Section 3.3,
//   ||r(x_i) - r(x_{i-1})|| <= u (gamma normest ||x_i|| + rho condest ||r(x_i)||),  u = 2^-53,
// is evaluated first (||r(x_i)||^2 and ||A (x_i - x_{i-1})||^2 come from this step's pass) and, if it
// holds, x_i is kept and the done flag raised.  A residual that grew beyond 100 ||r(x_0)|| also
// stops the iteration and flags ST_DIVERGED.  With st.grow set (mixed precision), a residual that
// grew three steps in a row, each time by more than a relative 2^-20, raises the done flag and
// state[2] = 1: the caller then falls back to FP64.
template <typename T, int kSB, int VW>
__global__ void __launch_bounds__(kSolveThreads)
k_solve(int64_t n, const T *__restrict__ R, int64_t ldr, const T *__restrict__ RT,
        const double *__restrict__ c, double *__restrict__ x, double *__restrict__ xprev,
        double *__restrict__ dout, int mode, double alpha, double beta, int32_t *__restrict__ status,
        int32_t *__restrict__ st_state, double *__restrict__ st_scal, double *__restrict__ st_dx,
        double st_gamma, double st_rho, int st_check, int st_grow)
{
    extern __shared__ __align__(16) unsigned char smem[];
    T *s = reinterpret_cast<T *>(smem);
    __shared__ SubstLds<T, kSB> L;
    __shared__ double red[kSolveThreads / 64];
    if (st_state) {
        if (st_state[0]) return;
        if (st_check) {
            double xx = 0.0;
            for (int64_t j = threadIdx.x; j < n; j += blockDim.x) xx += x[j] * x[j];
            xx = block_sum(xx, red);
            const double rr = st_scal[0], ad = st_scal[1];
            const double u = 0x1p-53;
            const bool stop = sqrt(ad) <= u * (st_gamma * st_scal[2] * sqrt(xx) + st_rho * st_scal[3] * sqrt(rr));
            const bool diverged = !(rr <= 1e4 * st_scal[4]);
            if (stop || diverged) {
                if (threadIdx.x == 0) {
                    st_state[0] = 1;
                    if (diverged) atomicOr(status, ST_DIVERGED);
                }
                return;
            }
        } else if (threadIdx.x == 0 && st_state[1] == 0) {
            st_scal[4] = st_scal[0];                       // ||r(x_0)||^2
        }
        if (st_grow) {
            const double rr = st_scal[0];
            const bool first = st_state[1] == 0;
            const int run = (!first && rr > st_scal[5] * (1.0 + 0x1p-20)) ? st_state[3] + 1 : 0;
            if (run >= 3 || !isfinite(rr)) {
                if (threadIdx.x == 0) {
                    st_state[0] = 1;
                    st_state[2] = 1;
                }
                return;
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                st_state[3] = run;
                st_scal[5] = rr;
            }
        }
    }
    const int e = load_rhs<T>(n, c, s, red);
    zero_pad<T, kSB>(n, s);
    __syncthreads();
    fwd_subst<T, kSB, kSolveThreads, Prefetch<T>::kSlots, VW>(n, R, ldr, s, L);
    back_subst<T, kSB, kSolveThreads, Prefetch<T>::kSlots, VW>(n, R, ldr, RT, s, L);
    bool bad = false;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
        const double dj = (sizeof(T) == 8) ? (double)s[j] : ldexp((double)s[j], e);
        if (mode == 0) {
            dout[j] = dj;
            bad |= !isfinite(dj);
        } else if (mode == 1) {
            const double xo = x[j];
            const double xn = xo + dj;
            x[j] = xn;
            if (st_state) st_dx[j] = xn - xo;
            bad |= !isfinite(xn);
        } else {
            const double xo = x[j];
            const double xn = xo + alpha * dj + beta * (xo - xprev[j]);
            xprev[j] = xo;
            x[j] = xn;
            if (st_state) st_dx[j] = xn - xo;
            bad |= !isfinite(xn);
        }
    }
    if (bad) atomicOr(status, ST_NONFINITE);
    if (st_state && threadIdx.x == 0) st_state[1] += 1;
}

// One served problem's step with the arithmetic of k_solve on it alone: FP64 factor, plain update;
// or FP32 factor (mixed precision) with k_solve's growth monitor, where a residual that grew three
// rounds in a row by more than a relative 2^-20 (or a non-finite one) freezes x for the rest of the
// request's rounds and raises ST_GROWTH, so that the server repeats the request in FP64.
template <typename T, int kSB>
__device__ __forceinline__ void served_step(const ServeSlot &sl, T *s, SubstLds<T, kSB> &L, double *red)
{
    const int64_t n = sl.n;
    if (sizeof(T) == 4) {
        int32_t *g = sl.gstate;
        if (g[0]) return;
        const double rr = *sl.rr;
        const int run = (g[1] != 0 && rr > sl.gprev[0] * (1.0 + 0x1p-20)) ? g[3] + 1 : 0;
        if (run >= 3 || !isfinite(rr)) {
            if (threadIdx.x == 0) {
                g[0] = 1;
                g[2] = 1;
                atomicOr(sl.status, ST_GROWTH);
            }
            return;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            g[3] = run;
            sl.gprev[0] = rr;
        }
    }
    const T *R = static_cast<const T *>(sl.R), *RT = static_cast<const T *>(sl.RT);
    const int e = load_rhs<T>(n, sl.c, s, red);
    zero_pad<T, kSB>(n, s);
    __syncthreads();
    fwd_subst<T, kSB, kSolveThreads>(n, R, n, s, L);
    back_subst<T, kSB, kSolveThreads>(n, R, n, RT, s, L);
    bool bad = false;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
        const double dj = (sizeof(T) == 8) ? (double)s[j] : ldexp((double)s[j], e);
        const double xn = sl.x[j] + dj;
        sl.x[j] = xn;
        bad |= !isfinite(xn);
    }
    if (bad) atomicOr(sl.status, ST_NONFINITE);
    if (sizeof(T) == 4 && threadIdx.x == 0) sl.gstate[1] += 1;
}

// Served rounds: d = R^{-1} (R^{-T} c) and x += d for every resident problem, one work-group each.
// The FP64 and FP32 substitutions share one LDS block.
template <int kSB>
__global__ void __launch_bounds__(kSolveThreads)
k_solve_served(const ServeSlot *__restrict__ slots)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ __align__(16) unsigned char lds[sizeof(SubstLds<double, kSB>)];
    __shared__ double red[kSolveThreads / 64];
    const ServeSlot &sl = slots[blockIdx.x];
    if (sl.r32)
        served_step<float, kSB>(sl, reinterpret_cast<float *>(smem), *reinterpret_cast<SubstLds<float, kSB> *>(lds), red);
    else
        served_step<double, kSB>(sl, reinterpret_cast<double *>(smem), *reinterpret_cast<SubstLds<double, kSB> *>(lds), red);
}

// w = R v for upper triangular R, read through RT = R^T (ld n, zero above its diagonal): w_i is the
// sum over j >= i of R[i][j] v_j, added in ascending j into one accumulator.  The lanes of a wave
// own 64 consecutive outputs and walk the rows of RT together, so every load instruction reads 64
// consecutive entries (a walk down R's rows or RT's columns would give each lane its own cache
// line).  A wave starts at the row its lowest output needs; for a lane whose diagonal comes later,
// the zero entries before it add +0 * v_j and leave its accumulator +0, so every sum is the one a
// walk from j = i gives.  Blocks of 64 outputs are dealt to the waves in a zigzag (block w, then
// the block mirrored from the end), which evens out the rows each wave walks.  v is in LDS.
template <typename T, int U>
__device__ __forceinline__ void upper_matvec(int64_t n, const T *__restrict__ RT, const T *v, T *__restrict__ w)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int64_t nblk = (n + 63) / 64;
    for (int64_t r = 0;; ++r) {
        const int64_t blk = (r & 1) ? (r + 1) * nw - 1 - wave : r * nw + wave;
        if (r * nw >= nblk) break;
        if (blk >= nblk) continue;
        const int64_t i0 = blk * 64, i = i0 + lane;
        const T *col = RT + (i < n ? i : i0);       // the lane's column of RT (kept in the matrix)
        T acc = T(0);
        int64_t j = i0;
        for (; j + U <= n; j += U) {
            T a[U];
#pragma unroll
            for (int u = 0; u < U; ++u) a[u] = col[(j + u) * n];
#pragma unroll
            for (int u = 0; u < U; ++u) acc += a[u] * v[j + u];
        }
        for (; j < n; ++j) acc += col[j * n] * v[j];
        if (i < n) w[i] = acc;
    }
}

// v = R^T w for upper triangular R (ld ldr, zero below its diagonal): v_k is the sum over i <= k of
// R[i][k] w_i, added in ascending i into one accumulator.  As in upper_matvec the lanes own 64
// consecutive outputs and walk R's rows together, here up to the last row the block's highest
// output needs; the zero entries after a lane's diagonal add +-0 and leave its sum unchanged (but
// for the sign of an exactly zero sum).  w is in LDS.
template <typename T, int U>
__device__ __forceinline__ void lower_matvec(int64_t n, const T *__restrict__ R, int64_t ldr, const T *w, T *__restrict__ v)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int64_t nblk = (n + 63) / 64;
    for (int64_t r = 0;; ++r) {
        const int64_t blk = (r & 1) ? (r + 1) * nw - 1 - wave : r * nw + wave;
        if (r * nw >= nblk) break;
        if (blk >= nblk) continue;
        const int64_t k0 = blk * 64, k = k0 + lane;
        const int64_t iend = (k0 + 64 < n) ? k0 + 64 : n;   // rows 0 .. iend - 1
        const T *col = R + (k < n ? k : k0);
        T acc = T(0);
        int64_t i = 0;
        for (; i + U <= iend; i += U) {
            T a[U];
#pragma unroll
            for (int u = 0; u < U; ++u) a[u] = col[(i + u) * ldr];
#pragma unroll
            for (int u = 0; u < U; ++u) acc += a[u] * w[i + u];
        }
        for (; i < iend; ++i) acc += col[i * ldr] * w[i];
        if (k < n) v[k] = acc;
    }
}

// Section 3.3 estimators, one work-group, in the arithmetic of the factor (T).
//   normest: v = g/||g|| with g_i uniform on [-1, 1) (53 high bits of SplitMix64 output i of the
//            stream `seed`); ceil(ln n) times: w = R v, est = ||w||, v = R^T w / ||R^T w||.
//   condest: ||R||_1 times Hager's estimate of ||R^{-1}||_1 (Higham, Ch. 15): x = e/n; up to five
//            times: y = R^{-1} x, est = ||y||_1, xi = sign(y), z = R^{-T} xi; stop when
//            ||z||_inf <= z^T x, else x = e_j for the first j maximising |z_j|.
constexpr int kEstThreads = 512;

template <typename T, int kSB>
__global__ void __launch_bounds__(kEstThreads)
k_estimators(int64_t n, const T *__restrict__ R, int64_t ldr, const T *__restrict__ RT,
             uint64_t seed, T *__restrict__ work, double *__restrict__ scal)
{
    extern __shared__ __align__(16) unsigned char smem[];
    T *s = reinterpret_cast<T *>(smem);
    __shared__ SubstLds<T, kSB> L;
    __shared__ T red[kEstThreads / 64];
    __shared__ int64_t s_arg[kEstThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    T *v = work, *w = work + n, *xv = work + 2 * n;
    // ---- normest
    T gg = T(0);
    for (int64_t i = tid; i < n; i += blockDim.x) {
        uint64_t z = seed + ((uint64_t)i + 1ULL) * 0x9E3779B97F4A7C15ULL;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        z ^= z >> 31;
        const T g = (T)(2.0 * ((double)(z >> 11) * 0x1p-53) - 1.0);
        v[i] = g;
        gg += g * g;
    }
    gg = sqrt(block_sum(gg, red));
    for (int64_t i = tid; i < n; i += blockDim.x) v[i] /= gg;
    __syncthreads();
    int steps = (int)ceil(log((double)n));
    if (steps < 1) steps = 1;
    T est = T(0);
    for (int it = 0; it < steps; ++it) {
        for (int64_t i = tid; i < n; i += blockDim.x) s[i] = v[i];
        __syncthreads();
        upper_matvec<T, 16>(n, RT, s, w);                   // w = R v
        __syncthreads();
        T ww = T(0);
        for (int64_t i = tid; i < n; i += blockDim.x) ww += w[i] * w[i];
        est = sqrt(block_sum(ww, red));
        for (int64_t i = tid; i < n; i += blockDim.x) s[i] = w[i];
        __syncthreads();
        lower_matvec<T, 16>(n, R, ldr, s, v);               // v = R^T w
        __syncthreads();
        T vv = T(0);
        for (int64_t k = tid; k < n; k += blockDim.x) vv += v[k] * v[k];
        vv = sqrt(block_sum(vv, red));
        if (vv == T(0)) break;
        for (int64_t k = tid; k < n; k += blockDim.x) v[k] /= vv;
        __syncthreads();
    }
    // ---- condest
    T n1 = T(0);
    for (int64_t k = tid; k < n; k += blockDim.x) {        // column 1-norms, 8 loads in flight
        T a = T(0);
        int64_t i = 0;
        for (; i + 8 <= k + 1; i += 8) {
            T t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = R[(i + u) * ldr + k];
#pragma unroll
            for (int u = 0; u < 8; ++u) a += fabs(t[u]);
        }
        for (; i <= k; ++i) a += fabs(R[i * ldr + k]);
        n1 = fmax(n1, a);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) n1 = fmax(n1, __shfl_xor(n1, off, 64));
    __syncthreads();
    if (lane == 0) red[wave] = n1;
    __syncthreads();
    n1 = T(0);
    for (int q = 0; q < nw; ++q) n1 = fmax(n1, red[q]);
    for (int64_t i = tid; i < n; i += blockDim.x) xv[i] = T(1) / (T)n;
    zero_pad<T, kSB>(n, s);
    __syncthreads();
    T inv1 = T(0);
    for (int it = 0; it < 5; ++it) {
        for (int64_t i = tid; i < n; i += blockDim.x) s[i] = xv[i];
        __syncthreads();
        back_subst<T, kSB, kEstThreads, 1>(n, R, ldr, RT, s, L);     // y = R^{-1} x
        T e1 = T(0);
        for (int64_t i = tid; i < n; i += blockDim.x) e1 += fabs(s[i]);
        inv1 = block_sum(e1, red);
        for (int64_t i = tid; i < n; i += blockDim.x) s[i] = (s[i] >= T(0)) ? T(1) : T(-1);
        __syncthreads();
        fwd_subst<T, kSB, kEstThreads, 1>(n, R, ldr, s, L);          // z = R^{-T} xi
        T zmax = T(-1), ztx = T(0);
        int64_t jmax = n;
        for (int64_t i = tid; i < n; i += blockDim.x) {
            const T az = fabs(s[i]);
            if (az > zmax) { zmax = az; jmax = i; }
            ztx += s[i] * xv[i];
        }
        ztx = block_sum(ztx, red);
        // first index of the largest |z|: wave-level then block-level argmax
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const T oz = __shfl_xor(zmax, off, 64);
            const int64_t oj = __shfl_xor(jmax, off, 64);
            if (oz > zmax || (oz == zmax && oj < jmax)) { zmax = oz; jmax = oj; }
        }
        __syncthreads();
        if (lane == 0) { red[wave] = zmax; s_arg[wave] = jmax; }
        __syncthreads();
        zmax = T(-1);
        jmax = n;
        for (int q = 0; q < nw; ++q)
            if (red[q] > zmax || (red[q] == zmax && s_arg[q] < jmax)) { zmax = red[q]; jmax = s_arg[q]; }
        __syncthreads();
        if (zmax <= ztx) break;
        for (int64_t i = tid; i < n; i += blockDim.x) xv[i] = (i == jmax) ? T(1) : T(0);
        __syncthreads();
    }
    if (tid == 0) {
        scal[2] = (double)est;
        scal[3] = (double)n1 * (double)inv1;
    }
}

__global__ void k_stop_init(int32_t *state)
{
    if (threadIdx.x < 4) state[threadIdx.x] = 0;
}

// x = R^{-1} y (sketch-and-solve start), y in the factor's type, x in FP64.
template <typename T, int kSB, int VW>
__global__ void __launch_bounds__(kSolveThreads)
k_back(int64_t n, const T *__restrict__ R, int64_t ldr, const T *__restrict__ RT,
       const T *__restrict__ y, double *__restrict__ x, int32_t *__restrict__ status)
{
    extern __shared__ __align__(16) unsigned char smem[];
    T *s = reinterpret_cast<T *>(smem);
    __shared__ SubstLds<T, kSB> L;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) s[j] = y[j];
    zero_pad<T, kSB>(n, s);
    __syncthreads();
    back_subst<T, kSB, kSolveThreads, Prefetch<T>::kSlots, VW>(n, R, ldr, RT, s, L);
    bool bad = false;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
        x[j] = (double)s[j];
        bad |= !isfinite(s[j]);
    }
    if (bad) atomicOr(status, ST_NONFINITE);
}

template <typename T>
__global__ void __launch_bounds__(256)
k_transpose(int64_t n, const T *__restrict__ R, int64_t ldr, T *__restrict__ RT)
{
    __shared__ T tile[32][33];
    const int64_t bx = (int64_t)blockIdx.x * 32, by = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = by + r, j = bx + tx;
        tile[r][tx] = (i < n && j < n) ? ((j >= i) ? R[i * ldr + j] : T(0)) : T(0);
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = bx + r, j = by + tx;     // RT[i][j] = R[j][i]
        if (i < n && j < n) RT[i * n + j] = tile[tx][r];
    }
}

// Rc = upper triangle of R with leading dimension n (zero below the diagonal).
template <typename T>
__global__ void __launch_bounds__(256)
k_compact_upper(int64_t n, const T *__restrict__ R, int64_t ldr, T *__restrict__ Rc)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * n) return;
    const int64_t i = e / n, j = e % n;
    Rc[e] = (j >= i) ? R[i * ldr + j] : T(0);
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <typename T>
hipError_t transpose_impl(hipStream_t s, int64_t n, const T *R, int64_t ldr, T *RT)
{
    hipLaunchKernelGGL(k_transpose<T>, dim3((unsigned)ceil_div(n, 32), (unsigned)ceil_div(n, 32)),
                       dim3(256), 0, s, n, R, ldr, RT);
    return hipGetLastError();
}

// The GEMV waves read 16 bytes per load (two doubles or four floats) when every row of R and R^T
// starts 16-byte aligned (n and ldr multiples of 16 / sizeof(T), aligned bases); the sums are the
// same either way.  FP32 factors take it above n = 512 only: ls_precond_solve_f32 measured 340 ->
// 286 us at n = 2000 and 114 -> 106 us at n = 1000, but 47.3 -> 50.8 us at n = 500 (FP64: faster
// at every n measured, 500 to 2000).
template <typename T>
bool wide_rows(int64_t n, const T *R, int64_t ldr, const T *RT)
{
    constexpr int64_t k = 16 / sizeof(T);
    return (sizeof(T) == 8 || n > 512) && n % k == 0 && ldr % k == 0 && (uintptr_t)R % 16 == 0 &&
           (uintptr_t)RT % 16 == 0;
}

template <typename T>
hipError_t solve_update_impl(hipStream_t s, int64_t n, const T *R, int64_t ldr, const T *RT,
                             const double *c, double *x, double *xprev, double *dout, int mode,
                             double alpha, double beta, int32_t *status, const StopArgs &st)
{
    const size_t lds = (size_t)padded<kSolveBlock>(n) * sizeof(T);
    if (wide_rows(n, R, ldr, RT))
        hipLaunchKernelGGL((k_solve<T, kSolveBlock, 16 / sizeof(T)>), dim3(1), dim3(kSolveThreads), lds, s, n, R,
                           ldr, RT, c, x, xprev, dout, mode, alpha, beta, status, st.state, st.scal, st.dx,
                           st.gamma, st.rho, st.check, st.grow);
    else
        hipLaunchKernelGGL((k_solve<T, kSolveBlock, 1>), dim3(1), dim3(kSolveThreads), lds, s, n, R,
                           ldr, RT, c, x, xprev, dout, mode, alpha, beta, status, st.state, st.scal, st.dx,
                           st.gamma, st.rho, st.check, st.grow);
    return hipGetLastError();
}

template <typename T>
hipError_t estimators_impl(hipStream_t s, int64_t n, const T *R, int64_t ldr, const T *RT,
                           uint64_t seed, T *work, double *scal)
{
    hipLaunchKernelGGL((k_estimators<T, kSolveBlock>), dim3(1), dim3(kEstThreads), (size_t)padded<kSolveBlock>(n) * sizeof(T), s,
                       n, R, ldr, RT, seed, work, scal);
    return hipGetLastError();
}

template <typename T>
hipError_t back_impl(hipStream_t s, int64_t n, const T *R, int64_t ldr, const T *RT, const T *y,
                     double *x, int32_t *status)
{
    const size_t lds = (size_t)padded<kSolveBlock>(n) * sizeof(T);
    if (wide_rows(n, R, ldr, RT))
        hipLaunchKernelGGL((k_back<T, kSolveBlock, 16 / sizeof(T)>), dim3(1), dim3(kSolveThreads), lds, s, n, R,
                           ldr, RT, y, x, status);
    else
        hipLaunchKernelGGL((k_back<T, kSolveBlock, 1>), dim3(1), dim3(kSolveThreads), lds, s, n, R, ldr, RT, y, x,
                           status);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_transpose(hipStream_t s, int64_t n, const double *R, int64_t ldr, double *RT)
{
    return transpose_impl(s, n, R, ldr, RT);
}

hipError_t launch_compact_upper(hipStream_t s, int64_t n, const double *R, int64_t ldr, double *Rc)
{
    hipLaunchKernelGGL(k_compact_upper<double>, dim3((unsigned)ceil_div(n * n, 256)), dim3(256), 0, s, n, R, ldr, Rc);
    return hipGetLastError();
}

hipError_t launch_compact_upper(hipStream_t s, int64_t n, const float *R, int64_t ldr, float *Rc)
{
    hipLaunchKernelGGL(k_compact_upper<float>, dim3((unsigned)ceil_div(n * n, 256)), dim3(256), 0, s, n, R, ldr, Rc);
    return hipGetLastError();
}

hipError_t launch_transpose(hipStream_t s, int64_t n, const float *R, int64_t ldr, float *RT)
{
    return transpose_impl(s, n, R, ldr, RT);
}

hipError_t launch_solve_update(hipStream_t s, int64_t n, const double *R, int64_t ldr,
                               const double *RT, const double *c, double *x, double *xprev,
                               double *dout, int mode, double alpha, double beta, int32_t *status,
                               const StopArgs &st)
{
    return solve_update_impl(s, n, R, ldr, RT, c, x, xprev, dout, mode, alpha, beta, status, st);
}

hipError_t launch_solve_update(hipStream_t s, int64_t n, const float *R, int64_t ldr,
                               const float *RT, const double *c, double *x, double *xprev,
                               double *dout, int mode, double alpha, double beta, int32_t *status,
                               const StopArgs &st)
{
    return solve_update_impl(s, n, R, ldr, RT, c, x, xprev, dout, mode, alpha, beta, status, st);
}

hipError_t launch_estimators(hipStream_t s, int64_t n, const double *R, int64_t ldr,
                             const double *RT, uint64_t seed, double *work, double *scal)
{
    return estimators_impl(s, n, R, ldr, RT, seed, work, scal);
}

hipError_t launch_estimators(hipStream_t s, int64_t n, const float *R, int64_t ldr,
                             const float *RT, uint64_t seed, float *work, double *scal)
{
    return estimators_impl(s, n, R, ldr, RT, seed, work, scal);
}

hipError_t launch_served_solve(hipStream_t s, int nslots, int64_t max_n, const ServeSlot *slots)
{
    if (nslots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_solve_served<kSolveBlock>, dim3(nslots), dim3(kSolveThreads),
                       (size_t)padded<kSolveBlock>(max_n) * sizeof(double), s, slots);
    return hipGetLastError();
}

hipError_t launch_stop_init(hipStream_t s, int32_t *state)
{
    hipLaunchKernelGGL(k_stop_init, dim3(1), dim3(64), 0, s, state);
    return hipGetLastError();
}

hipError_t launch_back_substitution(hipStream_t s, int64_t n, const double *R, int64_t ldr,
                                    const double *RT, const double *y, double *x, int32_t *status)
{
    return back_impl(s, n, R, ldr, RT, y, x, status);
}

hipError_t launch_back_substitution(hipStream_t s, int64_t n, const float *R, int64_t ldr,
                                    const float *RT, const float *y, double *x, int32_t *status)
{
    return back_impl(s, n, R, ldr, RT, y, x, status);
}
