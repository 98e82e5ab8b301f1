// Sparse-sign sketch B = S A, S b on gfx950 (eq. sparse_sign; Algorithm 2, "B <- S A").
//
//   k_sparse_sign   one thread per column j of S: zeta distinct rows + signs from the counter-based
//                   SplitMix64 stream, packed as (row | sign << 31); integer histogram of rows.
//   k_scan_rows     exclusive scan of the row histogram -> CSR row pointers.
//   k_csr_scatter   places each nonzero in its sketch row (slot order within a row is arbitrary).
//   k_csr_sort      sorts every sketch row by column index j, making the CSR unique: ascending j.
//   k_chunk_*       the same CSR from per-chunk LDS histograms, without global atomics and without
//                   the row sort, when d <= kLdsRows and the (chunk, row) segments are short (below);
//                   k_sparse_sign then skips its histogram.
//   k_gather        one wave per (sketch row, 64*CPL-column tile): B[k,:] = sum of +-A[j,:] over the
//                   row's columns in ascending j, times fl(1/sqrt(zeta)).  Rows of A are read as
//                   coalesced 512-byte segments (non-temporal); no atomics on floating-point data.
//                   Every row of A is fetched from HBM once per nonzero of its column of S (zeta x).
//   k_wl_hist, k_wl_wscan, k_wl_place
//                   the entry lists of k_gather_win straight from the embedding (no CSR), when
//                   d <= kLdsRows and d >= 512 zeta: each group of sketch rows' entries, window by
//                   window, rows in order, ascending j (below).
//   k_win_count, k_win_scan, k_win_scatter
//                   the same lists from the CSR, for the other shapes.
//   k_gather_win    the same sums with each row of A fetched from HBM once or twice, not zeta times:
//                   a work-group owns a 64-column slice of 16*rw sketch rows, accumulated in LDS;
//                   when one XCD's compute units hold all sketch rows of a slice, the eight slices
//                   that share rows of A run on the eight XCDs at the same time (one slice per
//                   XCD), else each launch takes every row block of a few slices (row-major), so
//                   A's columns are read once over all launches; a work-group barrier every
//                   kWinPerStep windows (kWinRowMajorSync times that in row-major launches) keeps
//                   the 16 waves of a CU within a few thousand rows of A of each other, so the
//                   other nonzeros of a row of A find it in that XCD's L2.  Each accumulator has one
//                   owner (its wave) and receives its terms in ascending j, so the bits equal
//                   k_gather's.
#include <algorithm>

#include "common.hpp"

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ULL;
constexpr uint64_t kDrawsPerColumn = 65536ULL;

__device__ __forceinline__ uint64_t splitmix_out(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + (k + 1ULL) * kGamma;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__global__ void __launch_bounds__(256)
k_sparse_sign(int64_t m, uint64_t d, int32_t zeta, uint64_t seed, uint32_t *__restrict__ ent,
              int32_t *__restrict__ rowcount)   // rowcount == nullptr: no histogram
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    uint32_t taken[LS_MAX_ZETA];
    int got = 0;
    uint32_t *out = ent + j * zeta;
    for (uint64_t t = 0; got < zeta && t < kDrawsPerColumn; ++t) {
        const uint64_t z = splitmix_out(seed, (uint64_t)j * kDrawsPerColumn + t);
        const uint32_t row = (uint32_t)((z >> 11) % d);
        bool dup = false;
#pragma unroll
        for (int e = 0; e < LS_MAX_ZETA; ++e) dup |= (e < got) && (taken[e] == row);
        if (dup) continue;
#pragma unroll
        for (int e = 0; e < LS_MAX_ZETA; ++e)
            if (e == got) taken[e] = row;
        out[got] = row | ((uint32_t)(z & 1ULL) << 31);
        if (rowcount) atomicAdd(&rowcount[row], 1);
        ++got;
    }
    for (uint32_t row = 0; got < zeta; ++row) {   // exhausted draws: smallest free rows, sign +1
        bool dup = false;
#pragma unroll
        for (int e = 0; e < LS_MAX_ZETA; ++e) dup |= (e < got) && (taken[e] == row);
        if (dup) continue;
#pragma unroll
        for (int e = 0; e < LS_MAX_ZETA; ++e)
            if (e == got) taken[e] = row;
        out[got] = row;
        if (rowcount) atomicAdd(&rowcount[row], 1);
        ++got;
    }
}

__global__ void __launch_bounds__(256)
k_unpack(int64_t nnz, const uint32_t *__restrict__ ent, int32_t *__restrict__ rows,
         int8_t *__restrict__ signs)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nnz) return;
    const uint32_t v = ent[i];
    rows[i] = (int32_t)(v & 0x7FFFFFFFu);
    signs[i] = (v >> 31) ? -1 : 1;
}

// Single work-group exclusive scan (d is at most a few hundred thousand).
__global__ void __launch_bounds__(1024)
k_scan_rows(int64_t d, const int32_t *__restrict__ count, int32_t *__restrict__ rowptr,
            int32_t *__restrict__ fill)
{
    __shared__ int32_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (d + 1023) / 1024;
    const int64_t lo = t * per, hi = (lo + per < d) ? lo + per : d;
    int32_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += count[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int32_t v = (t >= off) ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int32_t base = (t == 0) ? 0 : part[t - 1];
    for (int64_t i = lo; i < hi; ++i) {
        rowptr[i] = base;
        base += count[i];
        fill[i] = 0;
    }
    if (t == 1023) rowptr[d] = part[1023];
}

__global__ void __launch_bounds__(256)
k_csr_scatter(int64_t nnz, int32_t zeta, const uint32_t *__restrict__ ent,
              const int32_t *__restrict__ rowptr, int32_t *__restrict__ fill,
              uint32_t *__restrict__ cols)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nnz) return;
    const uint32_t v = ent[i];
    const uint32_t row = v & 0x7FFFFFFFu;
    const uint32_t j = (uint32_t)(i / zeta);
    const int32_t pos = rowptr[row] + atomicAdd(&fill[row], 1);
    cols[pos] = j | (v & 0x80000000u);
}

__device__ __forceinline__ void cmp_swap(uint32_t *a, int i, int l)
{
    const uint32_t x = a[i], y = a[l];
    if ((x & 0x7FFFFFFFu) > (y & 0x7FFFFFFFu)) {
        a[i] = y;
        a[l] = x;
    }
}

// Bitonic sort of one sketch row, all comparators ascending (the first step of each stage
// compares mirrored positions).  Positions >= L act as +infinity and never move, so comparators
// reaching past the row end are skipped and no padding is stored.  Rows up to kSortCap entries are
// sorted in LDS; longer rows are sorted in place in global memory by the same network.
constexpr int kSortCap = 8192;

__global__ void __launch_bounds__(256)
k_csr_sort(int64_t d, const int32_t *__restrict__ rowptr, uint32_t *__restrict__ cols)
{
    __shared__ uint32_t buf[kSortCap];
    const int64_t k = blockIdx.x;
    if (k >= d) return;
    const int32_t lo = rowptr[k];
    const int L = rowptr[k + 1] - lo;
    if (L <= 1) return;
    const bool in_lds = L <= kSortCap;
    uint32_t *a = in_lds ? buf : cols + lo;
    if (in_lds) {
        for (int i = threadIdx.x; i < L; i += blockDim.x) buf[i] = cols[lo + i];
    }
    __syncthreads();
    int P = 1;
    while (P < L) P <<= 1;
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const bool flip = (stride == (size >> 1));
            for (int t = threadIdx.x; t < (P >> 1); t += blockDim.x) {
                int i, l;
                if (flip) {
                    const int blk = t / stride, off = t % stride;
                    i = blk * size + off;
                    l = blk * size + size - 1 - off;
                } else {
                    const int blk = t / stride, off = t % stride;
                    i = blk * 2 * stride + off;
                    l = i + stride;
                }
                if (l < L) cmp_swap(a, i, l);
            }
            __syncthreads();
        }
    }
    if (in_lds) {
        for (int i = threadIdx.x; i < L; i += blockDim.x) cols[lo + i] = buf[i];
    }
}

// ---- CSR by chunk histograms (d <= kLdsRows) -------------------------------------------------------
// The columns of S are cut into chunks of cc columns (cc = kChunkCols, halved while a (chunk, row)
// segment would hold more than 8 entries on average, down to kMinChunkCols, so that small d keep
// short segments too).  A work-group counts its chunk's nonzeros per
// sketch row in LDS; the counts are summed over chunks (row lengths, then rowptr by k_scan_rows) and
// turned in place into each (chunk, row) segment's start; a work-group then places its chunk's
// nonzeros in their segments (LDS counters) and sorts each segment, a handful of entries, by j.
// Segments of one row follow chunk order, so every row ends in ascending j: the CSR of k_csr_sort.
constexpr int kChunkCols = 8192;
constexpr int kMinChunkCols = 256;
constexpr int64_t kLdsRows = 40960;      // 160 KiB of int32 counters

__global__ void __launch_bounds__(1024)
k_chunk_hist(int64_t m, int64_t d, int32_t zeta, int64_t cc, const uint32_t *__restrict__ ent,
             int32_t *__restrict__ cnt)
{
    __shared__ int32_t h[kLdsRows];
    const int64_t c = blockIdx.x;
    for (int64_t k = threadIdx.x; k < d; k += blockDim.x) h[k] = 0;
    __syncthreads();
    const int64_t j1 = ((c + 1) * cc < m) ? (c + 1) * cc : m;
    for (int64_t i = c * cc * zeta + threadIdx.x; i < j1 * zeta; i += blockDim.x)
        atomicAdd(&h[ent[i] & 0x7FFFFFFFu], 1);
    __syncthreads();
    for (int64_t k = threadIdx.x; k < d; k += blockDim.x) cnt[c * d + k] = h[k];
}

// rowcount[k] = sum over chunks of cnt[c][k], in chunk order.  One thread per row.
__global__ void __launch_bounds__(256)
k_chunk_total(int64_t d, int32_t nchunk, const int32_t *__restrict__ cnt, int32_t *__restrict__ rowcount)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= d) return;
    rowcount[k] = strided_sum<8>(cnt + k, nchunk, d);
}

// cnt[c][k] <- rowptr[k] + sum over chunks c' < c of cnt[c'][k] (start of the chunk's segment).
__global__ void __launch_bounds__(256)
k_chunk_base(int64_t d, int32_t nchunk, const int32_t *__restrict__ rowptr, int32_t *__restrict__ cnt)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= d) return;
    int32_t run = rowptr[k];
    int32_t c = 0;
    for (; c + 8 <= nchunk; c += 8) {
        int32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = cnt[(int64_t)(c + u) * d + k];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            cnt[(int64_t)(c + u) * d + k] = run;
            run += v[u];
        }
    }
    for (; c < nchunk; ++c) {
        const int32_t v = cnt[(int64_t)c * d + k];
        cnt[(int64_t)c * d + k] = run;
        run += v;
    }
}

__global__ void __launch_bounds__(1024)
k_chunk_place(int64_t m, int64_t d, int32_t zeta, int64_t cc, const uint32_t *__restrict__ ent,
              const int32_t *__restrict__ base, uint32_t *__restrict__ cols)
{
    __shared__ int32_t pos[kLdsRows];
    const int64_t c = blockIdx.x;
    const int32_t *b = base + c * d;
    for (int64_t k = threadIdx.x; k < d; k += blockDim.x) pos[k] = b[k];
    __syncthreads();
    const int64_t j1 = ((c + 1) * cc < m) ? (c + 1) * cc : m;
    for (int64_t i = c * cc * zeta + threadIdx.x; i < j1 * zeta; i += blockDim.x) {
        const uint32_t v = ent[i];
        const int32_t p = atomicAdd(&pos[v & 0x7FFFFFFFu], 1);
        cols[p] = (uint32_t)(i / zeta) | (v & 0x80000000u);
    }
    __syncthreads();   // this work-group's entries are in place (visible to the work-group)
    for (int64_t k = threadIdx.x; k < d; k += blockDim.x) {
        const int32_t lo = b[k], hi = pos[k];
        if (hi - lo <= 1) continue;
        if (hi - lo <= 16) {
            // in registers: pad with the largest key (j <= 2^31 - 2), bitonic network, write back
            uint32_t x[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) x[i] = (lo + i < hi) ? cols[lo + i] : 0xFFFFFFFFu;
#pragma unroll
            for (int kk = 2; kk <= 16; kk <<= 1)
#pragma unroll
                for (int jj = kk >> 1; jj > 0; jj >>= 1)
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const int l = i ^ jj;
                        if (l <= i) continue;
                        const bool up = (i & kk) == 0;
                        const uint32_t a = x[i], c = x[l];
                        const bool swap = up ? ((a & 0x7FFFFFFFu) > (c & 0x7FFFFFFFu))
                                             : ((a & 0x7FFFFFFFu) < (c & 0x7FFFFFFFu));
                        x[i] = swap ? c : a;
                        x[l] = swap ? a : c;
                    }
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (lo + i < hi) cols[lo + i] = x[i];
            continue;
        }
        for (int32_t i = lo + 1; i < hi; ++i) {      // longer segments: insertion sort by j
            const uint32_t x = cols[i];
            int32_t q = i - 1;
            while (q >= lo && (cols[q] & 0x7FFFFFFFu) > (x & 0x7FFFFFFFu)) {
                cols[q + 1] = cols[q];
                --q;
            }
            cols[q + 1] = x;
        }
    }
}

// One wave per (sketch row k, column tile).  Lane l owns columns c0 + l + 64 c, c < CPL, so every
// load instruction reads 64 consecutive doubles of a row of A.  Terms are added in ascending j;
// four rows are loaded before they are added so that several rows are in flight per wave.
// The sums are FP64; OT is the stored type (float on the mixed path: each entry rounded once).
template <int CPL, typename OT>
__global__ void __launch_bounds__(64)
k_gather(int64_t n, int32_t ntiles, const double *__restrict__ A, int64_t lda,
         const double *__restrict__ b, const int32_t *__restrict__ rowptr,
         const uint32_t *__restrict__ cols, double scale, OT *__restrict__ B, int64_t ldb,
         OT *__restrict__ Sb, int64_t ldsb)
{
    const int64_t k = blockIdx.x / ntiles;
    const int tile = blockIdx.x % ntiles;
    const int lane = threadIdx.x;
    const int64_t c0 = (int64_t)tile * 64 * CPL + lane;
    bool ok[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) ok[c] = (c0 + 64 * c) < n;
    double acc[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) acc[c] = 0.0;
    double sb = 0.0;
    const bool do_b = (b != nullptr) && tile == 0 && lane == 0;
    const int32_t lo = rowptr[k], hi = rowptr[k + 1];
    int32_t e = lo;
    for (; e + 4 <= hi; e += 4) {
        uint32_t v[4];
        double a[4][CPL];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = cols[e + u];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double *row = A + (int64_t)(v[u] & 0x7FFFFFFFu) * lda + c0;
#pragma unroll
            for (int c = 0; c < CPL; ++c) a[u][c] = ok[c] ? __builtin_nontemporal_load(row + 64 * c) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool neg = (v[u] >> 31) != 0;
#pragma unroll
            for (int c = 0; c < CPL; ++c) acc[c] = neg ? acc[c] - a[u][c] : acc[c] + a[u][c];
            if (do_b) {
                const double bj = b[v[u] & 0x7FFFFFFFu];
                sb = neg ? sb - bj : sb + bj;
            }
        }
    }
    for (; e < hi; ++e) {
        const uint32_t v = cols[e];
        const bool neg = (v >> 31) != 0;
        const double *row = A + (int64_t)(v & 0x7FFFFFFFu) * lda + c0;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const double a = ok[c] ? row[64 * c] : 0.0;
            acc[c] = neg ? acc[c] - a : acc[c] + a;
        }
        if (do_b) {
            const double bj = b[v & 0x7FFFFFFFu];
            sb = neg ? sb - bj : sb + bj;
        }
    }
    OT *out = B + k * ldb + c0;
#pragma unroll
    for (int c = 0; c < CPL; ++c)
        if (ok[c]) out[64 * c] = (OT)(acc[c] * scale);
    if (do_b) Sb[k * ldsb] = (OT)(sb * scale);
}

// ---- column-sliced gather -------------------------------------------------------------------------
constexpr int kWinWaves = 16;          // waves per work-group (one group of rw sketch rows each)
constexpr int kWinMaxRows = 20;        // rw at most: 16 x 20 x 64 doubles = 160 KiB of LDS
constexpr int64_t kWinLen = 4096;      // rows of A per list window
constexpr int kWinPerStep = 4;         // windows between two work-group barriers
// Row-major launches (below) with fewer than 128 list entries per group and step (d above about
// 2.5e4) meet at a barrier only every kWinRowMajorSync steps: each barrier waits on the group with
// the most entries, which weighs more the fewer there are.  Measured at m = 4e6, n = 2000,
// d = 4e4 (row blocks over all XCDs): 59.1 ms every step, 57.9 every 4, 63.5 every 16, 69.8 never;
// with each slice on its own XCDs: 50.9 every step, 49.5 every 2, 48.6 every 4.
constexpr int kWinRowMajorSync = 4;
constexpr int kWinBatch = 8;           // rows of A in flight per wave (16 in flight fetch 1.8x the bytes)
// A list entry packs the column j of S (bits 0..25), the entry's row within its group (26..30) and
// the sign (31), so the column-sliced gather takes m < 2^26.
constexpr int kListJBits = 26;
constexpr uint32_t kListJMask = (1u << kListJBits) - 1u;
constexpr int64_t kListMaxRows = (int64_t)1 << kListJBits;

// ctab[w*d + k] = entries of sketch row k in windows < w, for w = 0..nwl: entry p of the row
// writes the windows (window of entry p-1, window of entry p], and p = L closes up to nwl, so every
// (w, k) is written once.  One wave per row.
__global__ void __launch_bounds__(256)
k_win_count(int64_t d, int32_t nwl, const int32_t *__restrict__ rowptr,
            const uint32_t *__restrict__ cols, int32_t *__restrict__ ctab)
{
    const int64_t k = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (k >= d) return;
    const int32_t lo = rowptr[k], L = rowptr[k + 1] - lo;
    for (int32_t p = lane; p <= L; p += 64) {
        const int32_t w = (p < L) ? (int32_t)((cols[lo + p] & 0x7FFFFFFFu) / kWinLen) : nwl;
        const int32_t wp = (p > 0) ? (int32_t)((cols[lo + p - 1] & 0x7FFFFFFFu) / kWinLen) : -1;
        for (int32_t ww = wp + 1; ww <= w; ++ww) ctab[(int64_t)ww * d + k] = p;
    }
}

// For group g (rows g*RW ..) and window w, the window-w entries of the group's row r start in the
// group's list at  sum_{r' < r} ctab[w+1][r'] + sum_{r' > r} ctab[w][r']  plus the row's own entries
// before window w; stab[w*d + k] holds the two sums.  woff[g][t] = where window t*kWinPerStep
// starts in the list (absolute position in the entry arrays), woff[g][nstep] = the group's end.
// One wave per (g, w); lanes are the group's rows.
template <int RW>
__global__ void __launch_bounds__(256)
k_win_scan(int64_t d, int32_t nwl, int32_t nstep, const int32_t *__restrict__ rowptr,
           const int32_t *__restrict__ ctab, int32_t *__restrict__ stab, int32_t *__restrict__ woff)
{
    const int64_t pair = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t ngroups = (d + RW - 1) / RW;
    if (pair >= ngroups * (int64_t)nwl) return;
    const int64_t g = pair / nwl;
    const int32_t w = (int32_t)(pair % nwl);
    const int64_t k = g * RW + lane;
    const bool row = lane < RW && k < d;
    const int32_t c0 = row ? ctab[(int64_t)w * d + k] : 0;
    const int32_t c1 = row ? ctab[(int64_t)(w + 1) * d + k] : 0;
    int32_t pre = c1, suf = c0;      // inclusive prefix of c1, inclusive suffix of c0
#pragma unroll
    for (int off = 1; off < 32; off <<= 1) {
        const int32_t up = __shfl_up(pre, off);
        const int32_t dn = __shfl_down(suf, off);
        if (lane >= off) pre += up;
        if (lane + off < 64) suf += dn;
    }
    if (row) stab[(int64_t)w * d + k] = (pre - c1) + (suf - c0);
    const int32_t *gp = rowptr + g * RW;
    if (lane == 0 && w % kWinPerStep == 0) woff[g * (nstep + 1) + w / kWinPerStep] = gp[0] + suf;
    if (lane == 0 && w == 0) {
        const int64_t end = (g * RW + RW < d) ? g * RW + RW : d;
        woff[g * (nstep + 1) + nstep] = rowptr[end];
    }
}

// Places every CSR entry in its group's list, with its row within the group packed in.
template <int RW>
__global__ void __launch_bounds__(256)
k_win_scatter(int64_t d, const int32_t *__restrict__ rowptr, const uint32_t *__restrict__ cols,
              const int32_t *__restrict__ stab, uint32_t *__restrict__ lst)
{
    const int64_t k = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (k >= d) return;
    const int64_t g = k / RW;
    const int32_t gs = rowptr[g * RW];
    const int32_t lo = rowptr[k], L = rowptr[k + 1] - lo;
    for (int32_t p = lane; p < L; p += 64) {
        const uint32_t v = cols[lo + p];
        const int32_t w = (int32_t)((v & 0x7FFFFFFFu) / kWinLen);
        const int32_t dst = gs + p + stab[(int64_t)w * d + k];
        lst[dst] = v | ((uint32_t)(k - g * RW) << kListJBits);
    }
}

// ---- window lists straight from the embedding (d <= kLdsRows, short segments) --------------------
// Window w of the lists is columns [w kWinLen, (w+1) kWinLen) of S, i.e. a contiguous range of the
// embedding, so the lists can be built without the CSR: a row histogram per window, a scan over the
// windows of each group, a scan over the groups, then each window places its entries in their
// (group, window) segments by LDS counters and sorts every (window, row) segment by j.  The lists
// equal those of k_win_count / k_win_scan / k_win_scatter entry for entry.

// cnt[w][k] = entries of sketch row k in window w; tot[g][w] = entries of group g in window w.
template <int RW>
__global__ void __launch_bounds__(1024)
k_wl_hist(int64_t m, int64_t d, int32_t zeta, int32_t nwl, const uint32_t *__restrict__ ent,
          int32_t *__restrict__ cnt, int32_t *__restrict__ tot)
{
    __shared__ int32_t h[kLdsRows];
    const int64_t w = blockIdx.x;
    for (int64_t k = threadIdx.x; k < d; k += blockDim.x) h[k] = 0;
    __syncthreads();
    const int64_t j1 = ((w + 1) * kWinLen < m) ? (w + 1) * kWinLen : m;
    for (int64_t i = w * kWinLen * zeta + threadIdx.x; i < j1 * zeta; i += blockDim.x)
        atomicAdd(&h[ent[i] & 0x7FFFFFFFu], 1);
    __syncthreads();
    for (int64_t k = threadIdx.x; k < d; k += blockDim.x) cnt[w * d + k] = h[k];
    const int64_t ngroups = (d + RW - 1) / RW;
    for (int64_t g = threadIdx.x; g < ngroups; g += blockDim.x) {
        int32_t t = 0;
#pragma unroll
        for (int r = 0; r < RW; ++r)
            if (g * RW + r < d) t += h[g * RW + r];
        tot[g * nwl + w] = t;
    }
}

// One wave per group: tot[g][:] becomes its exclusive scan over the windows (the group-relative
// start of each window's segment), and gtot[g] the group's length.
__global__ void __launch_bounds__(256)
k_wl_wscan(int64_t ngroups, int32_t nwl, int32_t *__restrict__ tot, int32_t *__restrict__ gtot)
{
    const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (g >= ngroups) return;
    int32_t *t = tot + g * nwl;
    int32_t carry = 0;
    for (int32_t w0 = 0; w0 < nwl; w0 += 64) {
        const int32_t w = w0 + lane;
        const int32_t v = (w < nwl) ? t[w] : 0;
        int32_t x = v;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (w < nwl) t[w] = carry + x - v;
        carry += __shfl(x, 63, 64);
    }
    if (lane == 0) gtot[g] = carry;
}

// Window w places its entries: row k's entries of the window go to gstart[g] + rel[g][w] plus the
// entries of the group's earlier rows in the window; the window also records where its barrier
// step starts in each group's list (woff).  Each (window, row) segment is then sorted by j.
template <int RW>
__global__ void __launch_bounds__(1024)
k_wl_place(int64_t m, int64_t d, int32_t zeta, int32_t nwl, int32_t nstep,
           const uint32_t *__restrict__ ent, const int32_t *__restrict__ cnt,
           const int32_t *__restrict__ rel, const int32_t *__restrict__ gstart,
           const int32_t *__restrict__ gtot, int32_t *__restrict__ woff, uint32_t *__restrict__ lst)
{
    __shared__ int32_t h[kLdsRows];
    const int64_t w = blockIdx.x;
    const int64_t ngroups = (d + RW - 1) / RW;
    const int32_t *c = cnt + w * d;
    for (int64_t g = threadIdx.x; g < ngroups; g += blockDim.x) {
        int32_t run = gstart[g] + rel[g * nwl + w];
        if (w % kWinPerStep == 0) woff[g * (nstep + 1) + w / kWinPerStep] = run;
        if (w == nwl - 1) woff[g * (nstep + 1) + nstep] = gstart[g] + gtot[g];
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const int64_t k = g * RW + r;
            if (k < d) {
                h[k] = run;
                run += c[k];
            }
        }
    }
    __syncthreads();
    const int64_t j1 = ((w + 1) * kWinLen < m) ? (w + 1) * kWinLen : m;
    for (int64_t i = w * kWinLen * zeta + threadIdx.x; i < j1 * zeta; i += blockDim.x) {
        const uint32_t v = ent[i];
        const uint32_t k = v & 0x7FFFFFFFu;
        const int32_t p = atomicAdd(&h[k], 1);
        lst[p] = (uint32_t)(i / zeta) | ((k % RW) << kListJBits) | (v & 0x80000000u);
    }
    __syncthreads();   // this work-group's entries are in place (visible to the work-group)
    for (int64_t k = threadIdx.x; k < d; k += blockDim.x) {
        const int32_t hi = h[k], lo = hi - c[k];
        if (hi - lo <= 1) continue;
        if (hi - lo <= 16) {
            uint32_t x[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) x[i] = (lo + i < hi) ? lst[lo + i] : 0xFFFFFFFFu;
#pragma unroll
            for (int kk = 2; kk <= 16; kk <<= 1)
#pragma unroll
                for (int jj = kk >> 1; jj > 0; jj >>= 1)
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const int l = i ^ jj;
                        if (l <= i) continue;
                        const bool up = (i & kk) == 0;
                        const uint32_t a = x[i], b = x[l];
                        const bool swap = up ? ((a & kListJMask) > (b & kListJMask))
                                             : ((a & kListJMask) < (b & kListJMask));
                        x[i] = swap ? b : a;
                        x[l] = swap ? a : b;
                    }
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (lo + i < hi) lst[lo + i] = x[i];
            continue;
        }
        for (int32_t i = lo + 1; i < hi; ++i) {      // longer segments: insertion sort by j
            const uint32_t x = lst[i];
            int32_t q = i - 1;
            while (q >= lo && (lst[q] & kListJMask) > (x & kListJMask)) {
                lst[q + 1] = lst[q];
                --q;
            }
            lst[q + 1] = x;
        }
    }
}

// k_wl_place with the window staged in LDS (zeta <= 8, d <= kStageRows): the window's entries are
// placed at window-local positions (16-bit row counters, two to an LDS word), each (window, row)
// segment is sorted there by j, and each group's segment then goes to its list with contiguous
// stores.  Same lists as k_wl_place.
constexpr int kStageEntries = (int)kWinLen * 8;          // a window's entries for zeta <= 8 (128 KiB)
constexpr int64_t kStageRows = 15360;                    // 16-bit counters in the remaining LDS

template <int RW>
__global__ void __launch_bounds__(1024)
k_wl_place_lds(int64_t m, int64_t d, int32_t zeta, int32_t nwl, int32_t nstep,
               const uint32_t *__restrict__ ent, const int32_t *__restrict__ cnt,
               const int32_t *__restrict__ rel, const int32_t *__restrict__ gstart,
               const int32_t *__restrict__ gtot, int32_t *__restrict__ woff, uint32_t *__restrict__ lst)
{
    __shared__ uint32_t loc[kStageEntries];
    __shared__ uint32_t h2[kStageRows / 2];              // row k's counter: half (k & 1) of word k / 2
    const int64_t w = blockIdx.x;
    const int tid = threadIdx.x;
    const int64_t ngroups = (d + RW - 1) / RW;
    const int32_t *c = cnt + w * d;
    for (int64_t q = tid; q < (d + 1) / 2; q += blockDim.x) h2[q] = 0u;
    for (int64_t g = tid; g < ngroups; g += blockDim.x) {
        if (w % kWinPerStep == 0) woff[g * (nstep + 1) + w / kWinPerStep] = gstart[g] + rel[g * nwl + w];
        if (w == nwl - 1) woff[g * (nstep + 1) + nstep] = gstart[g] + gtot[g];
    }
    // Window-local start of each row: exclusive scan of the row counts in row order (rows of a
    // group are consecutive, so each group's entries form one local segment).  Thread t takes
    // rows [t per, (t+1) per); the 1024 partial sums are scanned in loc[] before it holds entries.
    int32_t *part = reinterpret_cast<int32_t *>(loc);
    const int64_t per = (d + 1023) / 1024;
    const int64_t r0 = tid * per, r1 = (r0 + per < d) ? r0 + per : d;
    int32_t sum = 0;
    for (int64_t k = r0; k < r1; ++k) sum += c[k];
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int32_t v = (tid >= off) ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int32_t run = part[tid] - sum;
    __syncthreads();                                     // part[] is read; loc[] is free again
    for (int64_t k = r0; k < r1; ++k) {                  // two threads may share a word: atomics
        atomicAdd(&h2[k >> 1], (uint32_t)run << (16 * (k & 1)));
        run += c[k];
    }
    __syncthreads();
    const int64_t j1 = ((w + 1) * kWinLen < m) ? (w + 1) * kWinLen : m;
    for (int64_t i = w * kWinLen * zeta + tid; i < j1 * zeta; i += blockDim.x) {
        const uint32_t v = ent[i];
        const uint32_t k = v & 0x7FFFFFFFu;
        const uint32_t sh = 16u * (k & 1u);
        const uint32_t p = (atomicAdd(&h2[k >> 1], 1u << sh) >> sh) & 0xFFFFu;
        loc[p] = (uint32_t)(i / zeta) | ((k % RW) << kListJBits) | (v & 0x80000000u);
    }
    __syncthreads();
    // sort each (window, row) segment by j in LDS
    for (int64_t k = tid; k < d; k += blockDim.x) {
        const int32_t hi = (int32_t)((h2[k >> 1] >> (16 * (k & 1))) & 0xFFFFu), lo = hi - c[k];
        if (hi - lo <= 1) continue;
        if (hi - lo <= 16) {
            uint32_t x[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) x[i] = (lo + i < hi) ? loc[lo + i] : 0xFFFFFFFFu;
#pragma unroll
            for (int kk = 2; kk <= 16; kk <<= 1)
#pragma unroll
                for (int jj = kk >> 1; jj > 0; jj >>= 1)
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const int l = i ^ jj;
                        if (l <= i) continue;
                        const bool up = (i & kk) == 0;
                        const uint32_t a = x[i], b = x[l];
                        const bool swap = up ? ((a & kListJMask) > (b & kListJMask))
                                             : ((a & kListJMask) < (b & kListJMask));
                        x[i] = swap ? b : a;
                        x[l] = swap ? a : b;
                    }
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (lo + i < hi) loc[lo + i] = x[i];
            continue;
        }
        for (int32_t i = lo + 1; i < hi; ++i) {
            const uint32_t x = loc[i];
            int32_t q = i - 1;
            while (q >= lo && (loc[q] & kListJMask) > (x & kListJMask)) {
                loc[q + 1] = loc[q];
                --q;
            }
            loc[q + 1] = x;
        }
    }
    __syncthreads();
    // each group's segment to its list, one wave per group, 64 consecutive entries per store
    const int wave = tid >> 6, lane = tid & 63;
    for (int64_t g = wave; g < ngroups; g += blockDim.x / 64) {
        const int64_t kl = g * RW + RW - 1 < d ? g * RW + RW - 1 : d - 1;   // last row of the group
        const int32_t end = (int32_t)((h2[kl >> 1] >> (16 * (kl & 1))) & 0xFFFFu);
        int32_t beg = 0;
        if (g > 0) {
            const int64_t kp = g * RW - 1;                                  // last row of group g-1
            beg = (int32_t)((h2[kp >> 1] >> (16 * (kp & 1))) & 0xFFFFu);
        }
        uint32_t *dst = lst + gstart[g] + rel[g * nwl + w];
        for (int32_t e = beg + lane; e < end; e += 64) dst[e - beg] = loc[e];
    }
}

// Work-group (XCD x = blockIdx % 8, block blockIdx / 8) takes column slice slice0 + x and row block
// rb0 + blockIdx / 8 (16 groups of RW sketch rows, one per wave).  Lane l of a wave owns column
// 64*slice + l of its RW rows in LDS; column n is S b (lane reads b).  The wave walks its group's
// list: 64 entries are read per vector load and broadcast by readlane, kWinBatch rows of A are in
// flight, and each term goes to its row's accumulator by an LDS add in list order (one writer per
// accumulator, so the order of each row's terms is the list's: ascending j).
template <int RW, typename OT>
__global__ void __launch_bounds__(kWinWaves * 64)
k_gather_win(int64_t d, int64_t n, int32_t nslice, int32_t slice0, int64_t rb0, int64_t nrb_all,
             const double *__restrict__ A, int64_t lda, const double *__restrict__ b,
             const int32_t *__restrict__ woff, int32_t nstep, const uint32_t *__restrict__ lst,
             double scale, OT *__restrict__ B, int64_t ldb,
             OT *__restrict__ Sb, int64_t ldsb, int32_t sync_every, int32_t xgroups)
{
    __shared__ double acc[kWinWaves * kWinMaxRows * 64];   // full size: one work-group per CU
    // Slice-per-XCD launches (nrb_all == 0): work-group i takes slice slice0 + i % 8 (XCD i mod 8)
    // and row block rb0 + i / 8.  Row-major launches (nrb_all > 0): work-group i takes row block
    // i % nrb_all of slice slice0 + i / nrb_all, so one launch covers every sketch row of a few
    // slices and A's columns are read once over all launches.  With xgroups > 0 (a divisor of 8,
    // the launch's slices) the row-major launch keeps each slice on its own XCDs: slice j of the
    // launch on the XCDs x with x % xgroups == j, its row blocks dealt over them, so the nonzeros
    // of a row of A meet in fewer L2s.
    int slice;
    int64_t rb;
    if (nrb_all == 0) {
        slice = slice0 + (int)(blockIdx.x % 8);
        rb = rb0 + blockIdx.x / 8;
    } else if (xgroups > 0) {
        const int x = (int)(blockIdx.x % 8);
        slice = slice0 + x % xgroups;
        rb = (int64_t)(blockIdx.x / 8) * (8 / xgroups) + x / xgroups;
        if (rb >= nrb_all) return;
    } else {
        slice = slice0 + (int)(blockIdx.x / nrb_all);
        rb = (int64_t)(blockIdx.x % nrb_all);
    }
    if (slice >= nslice) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t ngroups = (d + RW - 1) / RW;
    const int64_t g = rb * kWinWaves + wave;
    const bool live = g < ngroups;
    const int64_t r0 = g * RW;
    const int64_t r1 = live ? ((r0 + RW < d) ? r0 + RW : d) : r0;
    const int64_t col = (int64_t)slice * 64 + lane;
    const bool is_a = col < n;
    const bool is_b = (col == n) && (b != nullptr);
    // This lane's source column: A[:, col], b, or (no column) A[0, 0] read and never stored.
    const double *src = is_a ? A + col : (is_b ? b : A);
    const int64_t stride = is_a ? lda : (is_b ? 1 : 0);
    double *my = acc + wave * RW * 64 + lane;
#pragma unroll
    for (int r = 0; r < RW; ++r) my[r * 64] = 0.0;
    const int32_t *wo = woff + (live ? g : 0) * (int64_t)(nstep + 1);
    for (int32_t t = 0; t < nstep; ++t) {
        const int32_t lo = live ? wo[t] : 0, hi = live ? wo[t + 1] : 0;
        for (int32_t e0 = lo; e0 < hi; e0 += 64) {
            const int cnt = (hi - e0 < 64) ? hi - e0 : 64;
            const uint32_t vd = lane < cnt ? lst[e0 + lane] : 0u;
            int u0 = 0;
            for (; u0 + kWinBatch <= cnt; u0 += kWinBatch) {
                uint32_t v[kWinBatch];
                double a[kWinBatch];
#pragma unroll
                for (int u = 0; u < kWinBatch; ++u) {
                    v[u] = __builtin_amdgcn_readlane(vd, u0 + u);
                    a[u] = src[(int64_t)(v[u] & kListJMask) * stride];
                }
#pragma unroll
                for (int u = 0; u < kWinBatch; ++u) {
                    const int r = (int)((v[u] >> kListJBits) & 31u);
                    atomicAdd(my + r * 64, (v[u] >> 31) ? -a[u] : a[u]);
                }
            }
            for (; u0 < cnt; ++u0) {
                const uint32_t v = __builtin_amdgcn_readlane(vd, u0);
                const int r = (int)((v >> kListJBits) & 31u);
                const double a = src[(int64_t)(v & kListJMask) * stride];
                atomicAdd(my + r * 64, (v >> 31) ? -a : a);
            }
        }
        if ((t + 1) % sync_every == 0) __syncthreads();
    }
    if (is_a || is_b) {
        OT *out = is_a ? B + col : Sb;
        const int64_t ld = is_a ? ldb : ldsb;
        for (int64_t r = r0; r < r1; ++r) out[r * ld] = (OT)(my[(r - r0) * 64] * scale);
    }
}

inline unsigned blocks_for(int64_t count, int per) { return (unsigned)((count + per - 1) / per); }

// Compute units per XCD of the current device (work-groups per XCD in one k_gather_win launch).
int cus_per_xcd()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus >= 8 ? cus / 8 : 0;
}

// Rows per group for d sketch rows: the fewest launches of (8 XCDs x cus work-groups x 16 groups),
// then the smallest multiple of 4 rows that covers d in that many launches.
int32_t win_rows(int64_t d, int cus)
{
    const int64_t per = (int64_t)cus * kWinWaves;
    const int64_t launches = (d + per * kWinMaxRows - 1) / (per * kWinMaxRows);
    const int64_t rows = (d + launches * per - 1) / (launches * per);
    return (int32_t)((rows + 3) / 4 * 4);
}

}  // namespace

void sketch_bufs(Arena &ar, int64_t m, int64_t d, int32_t zeta, SketchBufs &sb, int64_t n,
                 int32_t win_mode)
{
    const size_t nnz = (size_t)m * (size_t)zeta;
    sb = SketchBufs{};
    sb.ent = ar.take<uint32_t>(nnz);
    sb.rowcount = ar.take<int32_t>((size_t)d);
    sb.rowptr = ar.take<int32_t>((size_t)d + 1);
    sb.fill = ar.take<int32_t>((size_t)d);
    // The column-sliced gather pays for its lists and its fixed grid when at least seven 64-column
    // slices keep the eight XCDs busy and A is large.
    const int cus = (win_mode == 0 && n >= 448 && m >= 65536 && m < kListMaxRows && d >= 64) ? cus_per_xcd() : 0;
    WinLists &w = sb.win;
    if (cus > 0) {
        w.active = true;
        w.cus = cus;
        w.rw = win_rows(d, cus);
        w.zeta = zeta;
        w.nwl = (int32_t)((m + kWinLen - 1) / kWinLen);
        w.nstep = (w.nwl + kWinPerStep - 1) / kWinPerStep;
        const int64_t ngroups = (d + w.rw - 1) / w.rw;
        w.lst = ar.take<uint32_t>(nnz);
        w.woff = ar.take<int32_t>((size_t)ngroups * (size_t)(w.nstep + 1));
        // Straight from the embedding, with no CSR at all, when the row counters fit in LDS, a
        // (window, row) segment holds kWinLen zeta / d <= 8 entries on average (the register sort
        // takes nearly all of them) and the count matrix is bounded.
        const size_t win_cells = (size_t)w.nwl * (size_t)d;
        w.direct = d <= kLdsRows && 8 * d >= kWinLen * zeta && win_cells <= ((size_t)1 << 26);
        if (w.direct) {
            w.cnt = ar.take<int32_t>(win_cells);
            w.rel = ar.take<int32_t>((size_t)ngroups * (size_t)w.nwl);
            w.gtot = ar.take<int32_t>((size_t)ngroups);
            w.gstart = ar.take<int32_t>((size_t)ngroups + 1);
            return;                                   // sb.cols and sb.chunk_cnt stay null
        }
        w.ctab = ar.take<int32_t>((size_t)(w.nwl + 1) * (size_t)d);
        w.stab = ar.take<int32_t>((size_t)w.nwl * (size_t)d);
    }
    sb.cols = ar.take<uint32_t>(nnz);
    // The chunk path needs the counters in LDS (d <= kLdsRows), short segments (a (chunk, row)
    // segment holds cc zeta / d entries on average: at most 8, so the register sort takes nearly
    // all of them) and a bounded count matrix.
    int64_t cc = kChunkCols;
    while (cc > kMinChunkCols && cc * zeta > 8 * d) cc >>= 1;
    const size_t chunk_cells = (size_t)((m + cc - 1) / cc) * (size_t)d;
    const bool chunk_path = d <= kLdsRows && 8 * d >= cc * zeta && chunk_cells <= ((size_t)1 << 26);
    sb.chunk_cnt = chunk_path ? ar.take<int32_t>(chunk_cells) : nullptr;
    sb.chunk_cols = chunk_path ? (int32_t)cc : 0;
}

hipError_t launch_sparse_sign(hipStream_t s, int64_t m, int64_t d, int32_t zeta, uint64_t seed,
                              const SketchBufs &sb)
{
    int32_t *count = nullptr;          // the chunk and direct paths count rows themselves
    if (!sb.chunk_cnt && !sb.win.direct) {
        hipError_t e = hipMemsetAsync(sb.rowcount, 0, sizeof(int32_t) * (size_t)d, s);
        if (e != hipSuccess) return e;
        count = sb.rowcount;
    }
    hipLaunchKernelGGL(k_sparse_sign, dim3(blocks_for(m, 256)), dim3(256), 0, s, m, (uint64_t)d,
                       zeta, seed, sb.ent, count);
    return hipGetLastError();
}

hipError_t launch_unpack_embedding(hipStream_t s, int64_t m, int32_t zeta, const uint32_t *ent,
                                   int32_t *rows, int8_t *signs)
{
    const int64_t nnz = m * zeta;
    hipLaunchKernelGGL(k_unpack, dim3(blocks_for(nnz, 256)), dim3(256), 0, s, nnz, ent, rows, signs);
    return hipGetLastError();
}

hipError_t launch_csr(hipStream_t s, int64_t m, int64_t d, int32_t zeta, const SketchBufs &sb)
{
    const int64_t nnz = m * zeta;
    if (sb.win.active && sb.win.direct) {            // the gather's lists only, no CSR
        const WinLists &w = sb.win;
        const int64_t ngroups = (d + w.rw - 1) / w.rw;
        switch (w.rw) {
#define LS_WL_CASE(R)                                                                                     \
        case R:                                                                                           \
            hipLaunchKernelGGL(k_wl_hist<R>, dim3((unsigned)w.nwl), dim3(1024), 0, s, m, d, zeta, w.nwl,   \
                               sb.ent, w.cnt, w.rel);                                                     \
            hipLaunchKernelGGL(k_wl_wscan, dim3(blocks_for(ngroups, 4)), dim3(256), 0, s, ngroups, w.nwl,  \
                               w.rel, w.gtot);                                                            \
            hipLaunchKernelGGL(k_scan_rows, dim3(1), dim3(1024), 0, s, ngroups, w.gtot, w.gstart, sb.fill); \
            if (zeta <= 8 && d <= kStageRows)                                                             \
                hipLaunchKernelGGL(k_wl_place_lds<R>, dim3((unsigned)w.nwl), dim3(1024), 0, s, m, d, zeta,  \
                                   w.nwl, w.nstep, sb.ent, w.cnt, w.rel, w.gstart, w.gtot, w.woff, w.lst); \
            else                                                                                          \
                hipLaunchKernelGGL(k_wl_place<R>, dim3((unsigned)w.nwl), dim3(1024), 0, s, m, d, zeta,      \
                                   w.nwl, w.nstep, sb.ent, w.cnt, w.rel, w.gstart, w.gtot, w.woff, w.lst); \
            break;
        LS_WL_CASE(4) LS_WL_CASE(8) LS_WL_CASE(12) LS_WL_CASE(16) LS_WL_CASE(20)
#undef LS_WL_CASE
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    if (sb.chunk_cnt) {
        const int64_t cc = sb.chunk_cols;
        const int32_t nchunk = (int32_t)((m + cc - 1) / cc);
        hipLaunchKernelGGL(k_chunk_hist, dim3((unsigned)nchunk), dim3(1024), 0, s, m, d, zeta, cc, sb.ent, sb.chunk_cnt);
        hipLaunchKernelGGL(k_chunk_total, dim3(blocks_for(d, 256)), dim3(256), 0, s, d, nchunk, sb.chunk_cnt, sb.rowcount);
        hipLaunchKernelGGL(k_scan_rows, dim3(1), dim3(1024), 0, s, d, sb.rowcount, sb.rowptr, sb.fill);
        hipLaunchKernelGGL(k_chunk_base, dim3(blocks_for(d, 256)), dim3(256), 0, s, d, nchunk, sb.rowptr, sb.chunk_cnt);
        hipLaunchKernelGGL(k_chunk_place, dim3((unsigned)nchunk), dim3(1024), 0, s, m, d, zeta, cc, sb.ent, sb.chunk_cnt, sb.cols);
    } else {
        hipLaunchKernelGGL(k_scan_rows, dim3(1), dim3(1024), 0, s, d, sb.rowcount, sb.rowptr, sb.fill);
        hipLaunchKernelGGL(k_csr_scatter, dim3(blocks_for(nnz, 256)), dim3(256), 0, s, nnz, zeta, sb.ent,
                           sb.rowptr, sb.fill, sb.cols);
        hipLaunchKernelGGL(k_csr_sort, dim3((unsigned)d), dim3(256), 0, s, d, sb.rowptr, sb.cols);
    }
    if (!sb.win.active) return hipGetLastError();
    const WinLists &w = sb.win;
    const int64_t ngroups = (d + w.rw - 1) / w.rw;
    const unsigned row_blocks = blocks_for(d, 4), pair_blocks = blocks_for(ngroups * w.nwl, 4);
    hipLaunchKernelGGL(k_win_count, dim3(row_blocks), dim3(256), 0, s, d, w.nwl, sb.rowptr, sb.cols, w.ctab);
    switch (w.rw) {
#define LS_WIN_CASE(R)                                                                                   \
    case R:                                                                                              \
        hipLaunchKernelGGL(k_win_scan<R>, dim3(pair_blocks), dim3(256), 0, s, d, w.nwl, w.nstep,        \
                           sb.rowptr, w.ctab, w.stab, w.woff);                                           \
        hipLaunchKernelGGL(k_win_scatter<R>, dim3(row_blocks), dim3(256), 0, s, d, sb.rowptr, sb.cols,   \
                           w.stab, w.lst);                                                               \
        break;
    LS_WIN_CASE(4) LS_WIN_CASE(8) LS_WIN_CASE(12) LS_WIN_CASE(16) LS_WIN_CASE(20)
#undef LS_WIN_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

namespace {

template <typename OT>
hipError_t gather_win_launch(hipStream_t s, dim3 grid, int64_t d, int64_t n, int32_t nslice,
                             int32_t s0, int64_t rb0, int64_t nrb_all, const double *A, int64_t lda,
                             const double *b, double scale, OT *B, int64_t ldb, OT *Sb, int64_t ldsb,
                             const WinLists &w, int32_t xgroups = 0, int32_t sync_every = 1)
{
    switch (w.rw) {
#define LS_WIN_CASE(R)                                                                                   \
    case R:                                                                                              \
        hipLaunchKernelGGL((k_gather_win<R, OT>), grid, dim3(kWinWaves * 64), 0, s, d, n, nslice, s0,   \
                           rb0, nrb_all, A, lda, b, w.woff, w.nstep, w.lst, scale, B, ldb, Sb, ldsb,     \
                           sync_every, xgroups);                                                         \
        break;
    LS_WIN_CASE(4) LS_WIN_CASE(8) LS_WIN_CASE(12) LS_WIN_CASE(16) LS_WIN_CASE(20)
#undef LS_WIN_CASE
    default: return hipErrorInvalidValue;
    }
    return hipSuccess;
}

// Slice-per-XCD launches, when one XCD's CUs hold every sketch row of a slice: each XCD takes its
// own slice of a group of eight, so a row of A is fetched into each XCD's L2 once and shared there
// by the CUs that need it.  Larger d takes row-major launches -- all row blocks of as many slices
// as the device holds -- so A's columns are read once over all launches.  When the launch's slice
// count divides 8 and each XCD can hold its share, the slices are kept apart by XCD (slice j on the
// XCDs x with x % ns == j), so the nonzeros of a row of A still meet in one of a few L2s: at
// m = 4e6, n = 2000, d = 4e4 (two slices per launch, each on four XCDs) the sketch took 48.6 ms
// against 58.1 ms with the row blocks of both slices dealt over all eight XCDs, at m = 1e6,
// n = 1000, d = 2e4 (four slices, two XCDs each) 5.73 ms against 6.46 ms with two slice-per-XCD
// launches per group of eight slices.  Row-major launches meet at a work-group barrier every
// step when a group has at least 128 list entries per step (d = 2e4), else every kWinRowMajorSync
// steps (d = 3e4 and 4e4: 11.10 and 48.6 ms, against 11.65 and 50.9 every step).
template <typename OT>
hipError_t gather_win(hipStream_t s, int64_t d, int64_t n, const double *A, int64_t lda,
                      const double *b, double scale, OT *B, int64_t ldb, OT *Sb, int64_t ldsb,
                      const WinLists &w)
{
    const int32_t nslice = (int32_t)((n + (b ? 1 : 0) + 63) / 64);
    const int64_t ngroups = (d + w.rw - 1) / w.rw;
    const int64_t nrb = (ngroups + kWinWaves - 1) / kWinWaves;
    hipError_t e = hipSuccess;
    if (nrb <= (int64_t)w.cus) {
        for (int32_t s0 = 0; s0 < nslice && e == hipSuccess; s0 += 8)
            e = gather_win_launch(s, dim3((unsigned)(8 * nrb)), d, n, nslice, s0, 0, 0, A, lda, b, scale, B, ldb,
                                  Sb, ldsb, w);
    } else {
        // list entries of one group per barrier step: rw rows x (kWinPerStep kWinLen zeta / d)
        const int64_t per_step = (int64_t)w.rw * kWinPerStep * kWinLen * w.zeta / d;
        const int32_t sync_every = per_step >= 128 ? 1 : kWinRowMajorSync;
        const int64_t per_launch = std::max<int64_t>(1, (int64_t)8 * w.cus / nrb);   // slices
        for (int32_t s0 = 0; s0 < nslice && e == hipSuccess; s0 += (int32_t)per_launch) {
            const int64_t ns = std::min<int64_t>(per_launch, nslice - s0);
            const int64_t per_xcd = (ns == 1 || ns == 2 || ns == 4 || ns == 8) ? (nrb + 8 / ns - 1) / (8 / ns) : 0;
            if (per_xcd > 0 && per_xcd <= (int64_t)w.cus)
                e = gather_win_launch(s, dim3((unsigned)(8 * per_xcd)), d, n, nslice, s0, 0, nrb, A, lda, b, scale,
                                      B, ldb, Sb, ldsb, w, (int32_t)ns, sync_every);
            else
                e = gather_win_launch(s, dim3((unsigned)(ns * nrb)), d, n, nslice, s0, 0, nrb, A, lda, b, scale,
                                      B, ldb, Sb, ldsb, w, 0, sync_every);
        }
    }
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

template <typename OT>
hipError_t gather_impl(hipStream_t s, int64_t d, int64_t n, const double *A, int64_t lda,
                       const double *b, const int32_t *rowptr, const uint32_t *cols, double scale,
                       OT *B, int64_t ldb, OT *Sb, int64_t ldsb, const WinLists *win)
{
    if (win && win->active) return gather_win(s, d, n, A, lda, b, scale, B, ldb, Sb, ldsb, *win);
    // Columns per lane: the smallest of 1, 2, 4, 8 covering n in one tile, else tiles of 512.
    int cpl = 8;
    if (n <= 64) cpl = 1;
    else if (n <= 128) cpl = 2;
    else if (n <= 256) cpl = 4;
    const int32_t ntiles = (int32_t)((n + 64 * cpl - 1) / (64 * cpl));
    const dim3 grid((unsigned)(d * ntiles));
    switch (cpl) {
    case 1: hipLaunchKernelGGL((k_gather<1, OT>), grid, dim3(64), 0, s, n, ntiles, A, lda, b, rowptr, cols, scale, B, ldb, Sb, ldsb); break;
    case 2: hipLaunchKernelGGL((k_gather<2, OT>), grid, dim3(64), 0, s, n, ntiles, A, lda, b, rowptr, cols, scale, B, ldb, Sb, ldsb); break;
    case 4: hipLaunchKernelGGL((k_gather<4, OT>), grid, dim3(64), 0, s, n, ntiles, A, lda, b, rowptr, cols, scale, B, ldb, Sb, ldsb); break;
    default: hipLaunchKernelGGL((k_gather<8, OT>), grid, dim3(64), 0, s, n, ntiles, A, lda, b, rowptr, cols, scale, B, ldb, Sb, ldsb); break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_gather(hipStream_t s, int64_t d, int64_t n, const double *A, int64_t lda,
                         const double *b, const int32_t *rowptr, const uint32_t *cols, double scale,
                         double *B, int64_t ldb, double *Sb, int64_t ldsb, const WinLists *win)
{
    return gather_impl(s, d, n, A, lda, b, rowptr, cols, scale, B, ldb, Sb, ldsb, win);
}

hipError_t launch_gather(hipStream_t s, int64_t d, int64_t n, const double *A, int64_t lda,
                         const double *b, const int32_t *rowptr, const uint32_t *cols, double scale,
                         float *B, int64_t ldb, float *Sb, int64_t ldsb, const WinLists *win)
{
    return gather_impl(s, d, n, A, lda, b, rowptr, cols, scale, B, ldb, Sb, ldsb, win);
}
