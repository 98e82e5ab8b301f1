// Sparse-sign sketch B = S A, S b on gfx950 (eq. sparse_sign; Algorithm 2, "B <- S A").
//
//   k_sparse_sign   one thread per column j of S: zeta distinct rows + signs from the counter-based
//                   SplitMix64 stream, packed as (row | sign << 31); integer histogram of rows.
//   k_scan_rows     exclusive scan of the row histogram -> CSR row pointers.
//   k_csr_scatter   places each nonzero in its sketch row (slot order within a row is arbitrary).
//   k_csr_sort      sorts every sketch row by column index j, making the CSR unique: ascending j.
//   k_gather        one wave per (sketch row, 64*CPL-column tile): B[k,:] = sum of +-A[j,:] over the
//                   row's columns in ascending j, times fl(1/sqrt(zeta)).  Rows of A are read as
//                   coalesced 512-byte segments (non-temporal); no atomics on floating-point data.
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
              int32_t *__restrict__ rowcount)
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
        atomicAdd(&rowcount[row], 1);
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
        atomicAdd(&rowcount[row], 1);
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

inline unsigned blocks_for(int64_t count, int per) { return (unsigned)((count + per - 1) / per); }

}  // namespace

void sketch_bufs(Arena &ar, int64_t m, int64_t d, int32_t zeta, SketchBufs &sb)
{
    const size_t nnz = (size_t)m * (size_t)zeta;
    sb.ent = ar.take<uint32_t>(nnz);
    sb.rowcount = ar.take<int32_t>((size_t)d);
    sb.rowptr = ar.take<int32_t>((size_t)d + 1);
    sb.fill = ar.take<int32_t>((size_t)d);
    sb.cols = ar.take<uint32_t>(nnz);
}

hipError_t launch_sparse_sign(hipStream_t s, int64_t m, int64_t d, int32_t zeta, uint64_t seed,
                              const SketchBufs &sb)
{
    hipError_t e = hipMemsetAsync(sb.rowcount, 0, sizeof(int32_t) * (size_t)d, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sparse_sign, dim3(blocks_for(m, 256)), dim3(256), 0, s, m, (uint64_t)d,
                       zeta, seed, sb.ent, sb.rowcount);
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
    hipLaunchKernelGGL(k_scan_rows, dim3(1), dim3(1024), 0, s, d, sb.rowcount, sb.rowptr, sb.fill);
    hipLaunchKernelGGL(k_csr_scatter, dim3(blocks_for(nnz, 256)), dim3(256), 0, s, nnz, zeta, sb.ent,
                       sb.rowptr, sb.fill, sb.cols);
    hipLaunchKernelGGL(k_csr_sort, dim3((unsigned)d), dim3(256), 0, s, d, sb.rowptr, sb.cols);
    return hipGetLastError();
}

namespace {

template <typename OT>
hipError_t gather_impl(hipStream_t s, int64_t d, int64_t n, const double *A, int64_t lda,
                       const double *b, const int32_t *rowptr, const uint32_t *cols, double scale,
                       OT *B, int64_t ldb, OT *Sb, int64_t ldsb)
{
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
                         double *B, int64_t ldb, double *Sb, int64_t ldsb)
{
    return gather_impl(s, d, n, A, lda, b, rowptr, cols, scale, B, ldb, Sb, ldsb);
}

hipError_t launch_gather(hipStream_t s, int64_t d, int64_t n, const double *A, int64_t lda,
                         const double *b, const int32_t *rowptr, const uint32_t *cols, double scale,
                         float *B, int64_t ldb, float *Sb, int64_t ldsb)
{
    return gather_impl(s, d, n, A, lda, b, rowptr, cols, scale, B, ldb, Sb, ldsb);
}
