// Refinement step of iterative sketching on gfx950 (Algorithm 2 loop; eq. it-sk-it-ref; stable
// form of Section 3.2).
//
//   k_pass        fused pass over A: for each row block, r = b - A x in registers (never stored),
//                 then acc += A^T r; each work-group writes one partial of c = A^T r and of ||r||^2.
//                 A is read exactly once, as coalesced 64-lane segments of its rows.
//   k_reduce      sums the partials in a fixed order (deterministic c and ||r||^2).
//   k_solve       one work-group: R^T y = c by forward substitution, R d = y by back
//                 substitution (64-wide diagonal blocks by one wave, off-diagonal blocks as
//                 coalesced GEMV updates; no inverse is ever formed), then the update of x.
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
// reads G consecutive doubles.
template <int G, int CPL, int RT>
__global__ void __launch_bounds__(kPassThreads)
k_pass(int64_t m, int64_t n, const double *__restrict__ A, int64_t lda, const double *__restrict__ b,
       const double *__restrict__ x, int64_t rows_per_wg, double *__restrict__ part,
       double *__restrict__ part_rr)
{
    constexpr int RPW = 64 / G;
    constexpr int TILE = RPW * RT;                   // rows per wave per tile
    __shared__ double s_acc[64 * CPL];
    __shared__ double s_rr[kPassThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sub = lane % G, grp = lane / G;

    double xr[CPL];
    bool cok[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int64_t col = sub + (int64_t)G * c;
        cok[c] = col < n;
        xr[c] = cok[c] ? x[col] : 0.0;
    }
    double acc[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) acc[c] = 0.0;
    double rr = 0.0;

    const int64_t r_begin = (int64_t)blockIdx.x * rows_per_wg;
    const int64_t r_end = (r_begin + rows_per_wg < m) ? r_begin + rows_per_wg : m;
    for (int64_t t0 = r_begin + (int64_t)wave * TILE; t0 < r_end; t0 += (int64_t)(kPassThreads / 64) * TILE) {
        double a[RT][CPL];
        double bb[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            const int64_t row = t0 + (int64_t)t * RPW + grp;
            const bool rok = row < r_end;
            const double *ar = A + row * lda + sub;
#pragma unroll
            for (int c = 0; c < CPL; ++c) a[t][c] = (rok && cok[c]) ? ar[G * c] : 0.0;
            bb[t] = rok ? b[row] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < RT; ++t) {
            double dot = 0.0;
#pragma unroll
            for (int c = 0; c < CPL; ++c) dot = fma(a[t][c], xr[c], dot);
            dot = group_sum<G>(dot);
            const double r = bb[t] - dot;            // residual entry, FP64, before A^T
            if (sub == 0) rr = fma(r, r, rr);
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
#pragma unroll
    for (int w = 0; w < kPassThreads / 64; ++w) {
        if (wave == w && grp == 0) {
#pragma unroll
            for (int c = 0; c < CPL; ++c)
                s_acc[sub + G * c] = (w == 0) ? acc[c] : s_acc[sub + G * c] + acc[c];
        }
        __syncthreads();
    }
    for (int col = threadIdx.x; col < G * CPL; col += kPassThreads)
        if (col < n) part[(int64_t)blockIdx.x * n + col] = s_acc[col];
    if (threadIdx.x == 0) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kPassThreads / 64; ++w) s += s_rr[w];
        part_rr[blockIdx.x] = s;
    }
}

// c[col] = sum_p part[p][col] in a fixed order: 4 groups of partials, each summed sequentially,
// then the 4 group sums in order.  Work-group 0 also reduces ||r||^2.
__global__ void __launch_bounds__(256)
k_reduce(int32_t P, int64_t n, const double *__restrict__ part, const double *__restrict__ part_rr,
         double *__restrict__ c, double *__restrict__ rr_out)
{
    __shared__ double s[4][64];
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int64_t col = (int64_t)blockIdx.x * 64 + lane;
    const int32_t per = (P + 3) / 4;
    const int32_t p_lo = g * per, p_hi = (p_lo + per < P) ? p_lo + per : P;
    double acc = 0.0;
    if (col < n)
        for (int32_t p = p_lo; p < p_hi; ++p) acc += part[(int64_t)p * n + col];
    s[g][lane] = acc;
    __syncthreads();
    if (g == 0 && col < n) c[col] = ((s[0][lane] + s[1][lane]) + s[2][lane]) + s[3][lane];
    if (blockIdx.x == 0 && rr_out) {
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int32_t p = 0; p < P; ++p) t += part_rr[p];
            *rr_out = t;
        }
    }
}

// Forward substitution R^T y = v in place on s[0:n] (R upper, row-major: R^T's column i is R's
// row i, read contiguously).  Diagonal 64-blocks by wave 0; the rest as a GEMV per block.
__device__ void fwd_subst(int64_t n, const double *__restrict__ R, int64_t ldr, double *s)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int64_t i0 = 0; i0 < n; i0 += 64) {
        const int64_t i1 = (i0 + 64 < n) ? i0 + 64 : n;
        if (wave == 0) {
            const int64_t me = i0 + lane;
            double v = (me < n) ? s[me] : 0.0;
            for (int64_t i = i0; i < i1; ++i) {
                const int li = (int)(i - i0);
                const double yi = __shfl(v, li, 64) / R[i * ldr + i];
                if (lane == li) v = yi;
                else if (lane > li && me < i1) v -= R[i * ldr + me] * yi;
            }
            if (me < i1) s[me] = v;
        }
        __syncthreads();
        for (int64_t j = i1 + tid; j < n; j += blockDim.x) {
            double acc = 0.0;
            for (int64_t i = i0; i < i1; ++i) acc += R[i * ldr + j] * s[i];
            s[j] -= acc;
        }
        __syncthreads();
    }
}

// Back substitution R z = v in place on s[0:n], using RT = R^T (row-major) so that column i of R
// is read contiguously.
__device__ void back_subst(int64_t n, const double *__restrict__ R, int64_t ldr,
                           const double *__restrict__ RT, double *s)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t nb = (n + 63) / 64;
    for (int64_t blk = nb - 1; blk >= 0; --blk) {
        const int64_t i0 = blk * 64;
        const int64_t i1 = (i0 + 64 < n) ? i0 + 64 : n;
        if (wave == 0) {
            const int64_t me = i0 + lane;
            double v = (me < i1) ? s[me] : 0.0;
            for (int64_t i = i1 - 1; i >= i0; --i) {
                const int li = (int)(i - i0);
                const double zi = __shfl(v, li, 64) / R[i * ldr + i];
                if (lane == li) v = zi;
                else if (lane < li) v -= RT[i * n + me] * zi;
            }
            if (me < i1) s[me] = v;
        }
        __syncthreads();
        for (int64_t j = tid; j < i0; j += blockDim.x) {
            double acc = 0.0;
            for (int64_t i = i0; i < i1; ++i) acc += RT[i * n + j] * s[i];
            s[j] -= acc;
        }
        __syncthreads();
    }
}

// d = R^{-1} (R^{-T} c), then the update selected by mode (see launch_solve_update).
__global__ void __launch_bounds__(1024)
k_solve(int64_t n, const double *__restrict__ R, int64_t ldr, const double *__restrict__ RT,
        const double *__restrict__ c, double *__restrict__ x, double *__restrict__ xprev,
        double *__restrict__ dout, int mode, double alpha, double beta, int32_t *__restrict__ status)
{
    extern __shared__ double s[];
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) s[j] = c[j];
    __syncthreads();
    fwd_subst(n, R, ldr, s);
    back_subst(n, R, ldr, RT, s);
    bool bad = false;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
        const double dj = s[j];
        if (mode == 0) {
            dout[j] = dj;
            bad |= !isfinite(dj);
        } else if (mode == 1) {
            const double xn = x[j] + dj;
            x[j] = xn;
            bad |= !isfinite(xn);
        } else {
            const double xo = x[j];
            const double xn = xo + alpha * dj + beta * (xo - xprev[j]);
            xprev[j] = xo;
            x[j] = xn;
            bad |= !isfinite(xn);
        }
    }
    if (bad) atomicOr(status, ST_NONFINITE);
}

// x = R^{-1} y (sketch-and-solve start).
__global__ void __launch_bounds__(1024)
k_back(int64_t n, const double *__restrict__ R, int64_t ldr, const double *__restrict__ RT,
       const double *__restrict__ y, double *__restrict__ x, int32_t *__restrict__ status)
{
    extern __shared__ double s[];
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) s[j] = y[j];
    __syncthreads();
    back_subst(n, R, ldr, RT, s);
    bool bad = false;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
        x[j] = s[j];
        bad |= !isfinite(s[j]);
    }
    if (bad) atomicOr(status, ST_NONFINITE);
}

__global__ void __launch_bounds__(256)
k_transpose(int64_t n, const double *__restrict__ R, int64_t ldr, double *__restrict__ RT)
{
    __shared__ double tile[32][33];
    const int64_t bx = (int64_t)blockIdx.x * 32, by = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = by + r, j = bx + tx;
        tile[r][tx] = (i < n && j < n) ? ((j >= i) ? R[i * ldr + j] : 0.0) : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = bx + r, j = by + tx;     // RT[i][j] = R[j][i]
        if (i < n && j < n) RT[i * n + j] = tile[tx][r];
    }
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// The pass variant for a given n: G lanes per row, CPL columns per lane, RT row groups per tile.
struct PassVariant {
    const void *fn;
    int id;
};

template <int G, int CPL, int RT>
const void *pass_fn() { return reinterpret_cast<const void *>(&k_pass<G, CPL, RT>); }

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

// Work-groups that fit on the device at once for a variant (cached per device and variant).
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
    cache[dev][id] = cus * per_cu;
    return cache[dev][id];
}

template <int G, int CPL, int RT>
void pass_launch(hipStream_t s, int P, int64_t rows_per_wg, int64_t m, int64_t n, const double *A,
                 int64_t lda, const double *b, const double *x, double *part, double *part_rr)
{
    hipLaunchKernelGGL((k_pass<G, CPL, RT>), dim3(P), dim3(kPassThreads), 0, s, m, n, A, lda, b, x,
                       rows_per_wg, part, part_rr);
}

}  // namespace

int32_t iter_partials(int64_t m, int64_t n)
{
    // One wave of co-resident work-groups, each over a contiguous block of at least 256 rows.
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
    ib.c = ar.take<double>((size_t)n);
    ib.xprev = ar.take<double>((size_t)n);
    ib.RT = need_rt ? ar.take<double>((size_t)n * (size_t)n) : nullptr;
}

hipError_t launch_transpose(hipStream_t s, int64_t n, const double *R, int64_t ldr, double *RT)
{
    hipLaunchKernelGGL(k_transpose, dim3((unsigned)ceil_div(n, 32), (unsigned)ceil_div(n, 32)),
                       dim3(256), 0, s, n, R, ldr, RT);
    return hipGetLastError();
}

hipError_t launch_gradient(hipStream_t s, int64_t m, int64_t n, const double *A, int64_t lda,
                           const double *b, const double *x, const IterBufs &ib, double *c,
                           double *rnorm2, hipEvent_t ev0, hipEvent_t ev1)
{
    const int P = ib.P;
    const int64_t rpw = ceil_div(m, P);
    if (ev0) {
        hipError_t e0 = hipEventRecord(ev0, s);
        if (e0 != hipSuccess) return e0;
    }
    if (n <= 8) pass_launch<8, 1, 4>(s, P, rpw, m, n, A, lda, b, x, ib.part, ib.part_rr);
    else if (n <= 16) pass_launch<16, 1, 4>(s, P, rpw, m, n, A, lda, b, x, ib.part, ib.part_rr);
    else if (n <= 32) pass_launch<16, 2, 4>(s, P, rpw, m, n, A, lda, b, x, ib.part, ib.part_rr);
    else if (n <= 64) pass_launch<16, 4, 4>(s, P, rpw, m, n, A, lda, b, x, ib.part, ib.part_rr);
    else if (n <= 128) pass_launch<64, 2, 4>(s, P, rpw, m, n, A, lda, b, x, ib.part, ib.part_rr);
    else if (n <= 256) pass_launch<64, 4, 4>(s, P, rpw, m, n, A, lda, b, x, ib.part, ib.part_rr);
    else if (n <= 512) pass_launch<64, 8, 4>(s, P, rpw, m, n, A, lda, b, x, ib.part, ib.part_rr);
    else if (n <= 1024) pass_launch<64, 16, 2>(s, P, rpw, m, n, A, lda, b, x, ib.part, ib.part_rr);
    else if (n <= 2048) pass_launch<64, 32, 1>(s, P, rpw, m, n, A, lda, b, x, ib.part, ib.part_rr);
    else return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev1) {
        e = hipEventRecord(ev1, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)ceil_div(n, 64)), dim3(256), 0, s, P, n, ib.part,
                       ib.part_rr, c, rnorm2);
    return hipGetLastError();
}

hipError_t launch_solve_update(hipStream_t s, int64_t n, const double *R, int64_t ldr,
                               const double *RT, const double *c, double *x, double *xprev,
                               double *dout, int mode, double alpha, double beta, int32_t *status)
{
    hipLaunchKernelGGL(k_solve, dim3(1), dim3(1024), (size_t)n * sizeof(double), s, n, R, ldr, RT, c,
                       x, xprev, dout, mode, alpha, beta, status);
    return hipGetLastError();
}

hipError_t launch_back_substitution(hipStream_t s, int64_t n, const double *R, int64_t ldr,
                                    const double *RT, const double *y, double *x, int32_t *status)
{
    hipLaunchKernelGGL(k_back, dim3(1), dim3(1024), (size_t)n * sizeof(double), s, n, R, ldr, RT, y,
                       x, status);
    return hipGetLastError();
}
