// Triangular solves and update of iterative sketching on gfx950 (Algorithm 2: d_i = R^{-1} (R^{-T} c_i),
// x_{i+1} = x_i + d_i; the damping / momentum update of eq. damping_momentum; the sketch-and-solve
// start x_0 = R^{-1} (Q^T S b)).
//
//   k_solve       one work-group: R^T y = c by forward substitution, R d = y by back substitution
//                 (32-wide diagonal blocks by one wave while the other waves apply earlier blocks
//                 as coalesced GEMV updates; no inverse matrix is ever formed), then the update.
//   k_back        back substitution alone (x_0).
//   k_transpose   R^T for the column reads of the back substitution.
#include "common.hpp"

namespace {

__device__ __forceinline__ double readlane_f64(double v, int l)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(unsigned)(u & 0xFFFFFFFFull), l);
    const int hi = __builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

// Diagonal block of the substitutions used by the library, and the solve kernels' work-group size.
constexpr int kSolveBlock = 32;
constexpr int kSolveThreads = 1024;

// LDS of the substitution kernels: double-buffered diagonal block, the reciprocals of its diagonal,
// and the block of R that couples the current block of unknowns to the next one.
template <int kSB>
struct SubstLds {
    double diag[2][kSB][kSB + 1];
    double rdiag[2][kSB];
    double off[2][kSB][kSB + 1];
};

// dst = R[r0:r0+kSB, c0:c0+kSB] (zero outside the n x n matrix), read by threads t.. of the WG.
template <int kSB>
__device__ __forceinline__ void load_block(double (*dst)[kSB + 1], const double *__restrict__ R,
                                           int64_t ldr, int64_t n, int64_t r0, int64_t c0, int t,
                                           int nt)
{
    for (int e = t; e < kSB * kSB; e += nt) {
        const int r = e / kSB, c = e % kSB;
        const int64_t gr = r0 + r, gc = c0 + c;
        dst[r][c] = (gr >= 0 && gr < n && gc >= 0 && gc < n) ? R[gr * ldr + gc] : 0.0;
    }
}

// Reciprocals of R[i0+l, i0+l] (1 outside R), by threads t.. of the WG.
template <int kSB>
__device__ __forceinline__ void load_rdiag(double *dst, const double *__restrict__ R, int64_t ldr,
                                           int64_t n, int64_t i0, int t, int nt)
{
    for (int l = t; l < kSB; l += nt) {
        const int64_t g = i0 + l;
        dst[l] = (g >= 0 && g < n) ? 1.0 / R[g * ldr + g] : 1.0;
    }
}

// Solves one diagonal block in wave 0: lane l holds unknown l (v) and column l of the block
// (colv[li] = T[li][l] of the triangular factor being applied, T = R^T forward or R backward);
// unknown li = v_li * (1 / T[li][li]) is broadcast with readlane and removed from the others.
template <int kSB, bool kForward>
__device__ __forceinline__ double block_solve(double v, const double (*diag)[kSB + 1],
                                              const double *rdiag, int nb, int lane)
{
    const int lc = (lane < kSB) ? lane : 0;
    const double rd = rdiag[lc];
#define colv(li) (kForward ? diag[li][lc] : diag[lc][li])
    if (kForward) {
#pragma unroll
        for (int li = 0; li < kSB; ++li) {
            if (li < nb) {
                const double yi = readlane_f64(v * rd, li);
                if (lane == li) v = yi;
                else if (lane > li && lane < nb) v -= colv(li) * yi;
            }
        }
    } else {
#pragma unroll
        for (int li = kSB - 1; li >= 0; --li) {
            if (li < nb) {
                const double zi = readlane_f64(v * rd, li);
                if (lane == li) v = zi;
                else if (lane < li) v -= colv(li) * zi;
            }
        }
    }
#undef colv
    return v;
}

// Forward substitution R^T y = v in place on s[0:n] (R upper triangular, row-major).
// Block k of unknowns is solved by wave 0 alone (block_solve); wave 0 then forms the contribution
// of block k to block k+1 in registers (the "carry").  Meanwhile waves 1.. apply block k-1 to every
// unknown past block k+1 (coalesced reads of rows of R, 32 loads in flight per thread) and load the
// next diagonal, reciprocal and coupling blocks into the other LDS buffer.  Each unknown therefore
// receives the terms of earlier blocks in a fixed order, and no two waves write one entry in one
// phase.  Unknowns are divided by R_ii as multiplication by the rounded reciprocal.
template <int kSB>
__device__ __forceinline__ void fwd_subst(int64_t n, const double *__restrict__ R, int64_t ldr, double *s,
                                          SubstLds<kSB> &L)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nblk = (int)((n + kSB - 1) / kSB);
    load_block<kSB>(L.diag[0], R, ldr, n, 0, 0, tid, blockDim.x);
    load_rdiag<kSB>(L.rdiag[0], R, ldr, n, 0, tid, blockDim.x);
    load_block<kSB>(L.off[0], R, ldr, n, 0, kSB, tid, blockDim.x);
    __syncthreads();
    double carry = 0.0;
    for (int k = 0; k < nblk; ++k) {
        const int64_t i0 = (int64_t)k * kSB;
        const int nb = (int)((i0 + kSB < n) ? kSB : n - i0);
        const int buf = k & 1;
        double next = 0.0;
        if (wave == 0) {
            double v = (lane < nb) ? s[i0 + lane] - carry : 0.0;
            v = block_solve<kSB, true>(v, L.diag[buf], L.rdiag[buf], nb, lane);
            if (lane < nb) s[i0 + lane] = v;
            if (k + 1 < nblk) {
                const int lc = (lane < kSB) ? lane : 0;
#pragma unroll
                for (int li = 0; li < kSB; ++li)
                    if (li < nb) next += L.off[buf][li][lc] * readlane_f64(v, li);
            }
        } else {
            const int t = tid - 64, nt = blockDim.x - 64;
            if (k >= 1) {                               // block k-1 (always full) -> past block k+1
                const int64_t p0 = i0 - kSB;
                for (int64_t j = i0 + kSB + t; j < n; j += nt)
                    s[j] -= strided_dot<kSB>(R + p0 * ldr + j, ldr, s + p0, kSB);
            }
            if (k + 1 < nblk) {
                load_block<kSB>(L.diag[buf ^ 1], R, ldr, n, i0 + kSB, i0 + kSB, t, nt);
                load_rdiag<kSB>(L.rdiag[buf ^ 1], R, ldr, n, i0 + kSB, t, nt);
                load_block<kSB>(L.off[buf ^ 1], R, ldr, n, i0 + kSB, i0 + 2 * kSB, t, nt);
            }
        }
        __syncthreads();
        carry = next;
    }
}

// Back substitution R z = v in place on s[0:n]; RT = R^T (row-major, ld n) gives the columns of R
// contiguously for the far updates.  Same schedule as fwd_subst, blocks taken from the last.
template <int kSB>
__device__ __forceinline__ void back_subst(int64_t n, const double *__restrict__ R, int64_t ldr,
                                           const double *__restrict__ RT, double *s, SubstLds<kSB> &L)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nblk = (int)((n + kSB - 1) / kSB);
    const int64_t last0 = (int64_t)(nblk - 1) * kSB;
    load_block<kSB>(L.diag[0], R, ldr, n, last0, last0, tid, blockDim.x);
    load_rdiag<kSB>(L.rdiag[0], R, ldr, n, last0, tid, blockDim.x);
    load_block<kSB>(L.off[0], R, ldr, n, last0 - kSB, last0, tid, blockDim.x);  // rows of block B-1
    __syncthreads();
    double carry = 0.0;
    for (int t = 0; t < nblk; ++t) {
        const int B = nblk - 1 - t;
        const int64_t i0 = (int64_t)B * kSB;
        const int nb = (int)((i0 + kSB < n) ? kSB : n - i0);
        const int buf = t & 1;
        double next = 0.0;
        if (wave == 0) {
            double v = (lane < nb) ? s[i0 + lane] - carry : 0.0;
            v = block_solve<kSB, false>(v, L.diag[buf], L.rdiag[buf], nb, lane);
            if (lane < nb) s[i0 + lane] = v;
            if (B >= 1) {
                const int lc = (lane < kSB) ? lane : 0;
#pragma unroll
                for (int li = 0; li < kSB; ++li)
                    if (li < nb) next += L.off[buf][lc][li] * readlane_f64(v, li);
            }
        } else {
            const int th = tid - 64, nt = blockDim.x - 64;
            if (t >= 1) {                               // block B+1 -> blocks B-1, B-2, ...
                const int64_t p0 = i0 + kSB;
                const int pb = (int)((p0 + kSB < n) ? kSB : n - p0);
                for (int64_t j = th; j < i0; j += nt)
                    s[j] -= strided_dot<kSB>(RT + p0 * n + j, n, s + p0, pb);
            }
            if (B >= 1) {
                load_block<kSB>(L.diag[buf ^ 1], R, ldr, n, i0 - kSB, i0 - kSB, th, nt);
                load_rdiag<kSB>(L.rdiag[buf ^ 1], R, ldr, n, i0 - kSB, th, nt);
                load_block<kSB>(L.off[buf ^ 1], R, ldr, n, i0 - 2 * kSB, i0 - kSB, th, nt);
            }
        }
        __syncthreads();
        carry = next;
    }
}

// Block-wide sum in a fixed order (wave reductions, then the waves in order); all threads get it.
__device__ __forceinline__ double block_sum(double v, double *red)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += red[w];
    return t;
}

// d = R^{-1} (R^{-T} c), then the update selected by mode (see launch_solve_update).  With a
// stopping rule (st.state != nullptr): once the done flag is set the launch is a no-op; when
// st.check is set the rule of Section 3.3,
//   ||r(x_i) - r(x_{i-1})|| <= u (gamma normest ||x_i|| + rho condest ||r(x_i)||),  u = 2^-53,
// is evaluated first (||r(x_i)||^2 and ||A (x_i - x_{i-1})||^2 come from this step's pass) and, if it
// holds, x_i is kept and the done flag raised.  A residual that grew beyond 100 ||r(x_0)|| also
// stops the iteration and flags ST_DIVERGED.
template <int kSB>
__global__ void __launch_bounds__(kSolveThreads)
k_solve(int64_t n, const double *__restrict__ R, int64_t ldr, const double *__restrict__ RT,
        const double *__restrict__ c, double *__restrict__ x, double *__restrict__ xprev,
        double *__restrict__ dout, int mode, double alpha, double beta, int32_t *__restrict__ status,
        int32_t *__restrict__ st_state, double *__restrict__ st_scal, double *__restrict__ st_dx,
        double st_gamma, double st_rho, int st_check)
{
    struct {
        int32_t *state;
        double *scal, *dx;
        double gamma, rho;
        int check;
    } st = {st_state, st_scal, st_dx, st_gamma, st_rho, st_check};
    extern __shared__ double s[];
    __shared__ SubstLds<kSB> L;
    __shared__ double red[kSolveThreads / 64];
    if (st.state) {
        if (st.state[0]) return;
        if (st.check) {
            double xx = 0.0;
            for (int64_t j = threadIdx.x; j < n; j += blockDim.x) xx += x[j] * x[j];
            xx = block_sum(xx, red);
            const double rr = st.scal[0], ad = st.scal[1];
            const double u = 0x1p-53;
            const bool stop = sqrt(ad) <= u * (st.gamma * st.scal[2] * sqrt(xx) + st.rho * st.scal[3] * sqrt(rr));
            const bool diverged = !(rr <= 1e4 * st.scal[4]);
            if (stop || diverged) {
                if (threadIdx.x == 0) {
                    st.state[0] = 1;
                    if (diverged) atomicOr(status, ST_DIVERGED);
                }
                return;
            }
        } else if (threadIdx.x == 0 && st.state[1] == 0) {
            st.scal[4] = st.scal[0];                       // ||r(x_0)||^2
        }
    }
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) s[j] = c[j];
    __syncthreads();
    fwd_subst<kSB>(n, R, ldr, s, L);
    back_subst<kSB>(n, R, ldr, RT, s, L);
    bool bad = false;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
        const double dj = s[j];
        if (mode == 0) {
            dout[j] = dj;
            bad |= !isfinite(dj);
        } else if (mode == 1) {
            const double xo = x[j];
            const double xn = xo + dj;
            x[j] = xn;
            if (st.state) st.dx[j] = xn - xo;
            bad |= !isfinite(xn);
        } else {
            const double xo = x[j];
            const double xn = xo + alpha * dj + beta * (xo - xprev[j]);
            xprev[j] = xo;
            x[j] = xn;
            if (st.state) st.dx[j] = xn - xo;
            bad |= !isfinite(xn);
        }
    }
    if (bad) atomicOr(status, ST_NONFINITE);
    if (st.state && threadIdx.x == 0) st.state[1] += 1;
}

// Section 3.3 estimators, one work-group.
//   normest: v = g/||g|| with g_i uniform on [-1, 1) (53 high bits of SplitMix64 output i of the
//            stream `seed`); ceil(ln n) times: w = R v, est = ||w||, v = R^T w / ||R^T w||.
//   condest: ||R||_1 times Hager's estimate of ||R^{-1}||_1 (Higham, Ch. 15): x = e/n; up to five
//            times: y = R^{-1} x, est = ||y||_1, xi = sign(y), z = R^{-T} xi; stop when
//            ||z||_inf <= z^T x, else x = e_j for the first j maximising |z_j|.
constexpr int kEstThreads = 512;

template <int kSB>
__global__ void __launch_bounds__(kEstThreads)
k_estimators(int64_t n, const double *__restrict__ R, int64_t ldr, const double *__restrict__ RT,
             uint64_t seed, double *__restrict__ work, double *__restrict__ scal)
{
    extern __shared__ double s[];
    __shared__ SubstLds<kSB> L;
    __shared__ double red[kSolveThreads / 64];
    __shared__ int64_t s_arg[kSolveThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    double *v = work, *w = work + n, *xv = work + 2 * n;
    // ---- normest
    double gg = 0.0;
    for (int64_t i = tid; i < n; i += blockDim.x) {
        uint64_t z = seed + ((uint64_t)i + 1ULL) * 0x9E3779B97F4A7C15ULL;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        z ^= z >> 31;
        const double g = 2.0 * ((double)(z >> 11) * 0x1p-53) - 1.0;
        v[i] = g;
        gg += g * g;
    }
    gg = sqrt(block_sum(gg, red));
    for (int64_t i = tid; i < n; i += blockDim.x) v[i] /= gg;
    __syncthreads();
    int steps = (int)ceil(log((double)n));
    if (steps < 1) steps = 1;
    double est = 0.0;
    for (int it = 0; it < steps; ++it) {
        for (int64_t i = wave; i < n; i += nw) {            // w = R v, one row per wave
            double a = 0.0;
            for (int64_t k = i + lane; k < n; k += 64) a += R[i * ldr + k] * v[k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
            if (lane == 0) w[i] = a;
        }
        __syncthreads();
        double ww = 0.0;
        for (int64_t i = tid; i < n; i += blockDim.x) ww += w[i] * w[i];
        est = sqrt(block_sum(ww, red));
        double vv = 0.0;
        for (int64_t k = tid; k < n; k += blockDim.x) {      // v = R^T w, one column per thread
            double a = 0.0;
            for (int64_t i = 0; i <= k; ++i) a += R[i * ldr + k] * w[i];
            v[k] = a;
            vv += a * a;
        }
        vv = sqrt(block_sum(vv, red));
        if (vv == 0.0) break;
        for (int64_t k = tid; k < n; k += blockDim.x) v[k] /= vv;
        __syncthreads();
    }
    // ---- condest
    double n1 = 0.0;
    for (int64_t k = tid; k < n; k += blockDim.x) {
        double a = 0.0;
        for (int64_t i = 0; i <= k; ++i) a += fabs(R[i * ldr + k]);
        n1 = fmax(n1, a);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) n1 = fmax(n1, __shfl_xor(n1, off, 64));
    __syncthreads();
    if (lane == 0) red[wave] = n1;
    __syncthreads();
    n1 = 0.0;
    for (int q = 0; q < nw; ++q) n1 = fmax(n1, red[q]);
    for (int64_t i = tid; i < n; i += blockDim.x) xv[i] = 1.0 / (double)n;
    __syncthreads();
    double inv1 = 0.0;
    for (int it = 0; it < 5; ++it) {
        for (int64_t i = tid; i < n; i += blockDim.x) s[i] = xv[i];
        __syncthreads();
        back_subst<kSB>(n, R, ldr, RT, s, L);                 // y = R^{-1} x
        double e1 = 0.0;
        for (int64_t i = tid; i < n; i += blockDim.x) e1 += fabs(s[i]);
        inv1 = block_sum(e1, red);
        for (int64_t i = tid; i < n; i += blockDim.x) s[i] = (s[i] >= 0.0) ? 1.0 : -1.0;
        __syncthreads();
        fwd_subst<kSB>(n, R, ldr, s, L);                      // z = R^{-T} xi
        double zmax = -1.0, ztx = 0.0;
        int64_t jmax = n;
        for (int64_t i = tid; i < n; i += blockDim.x) {
            const double az = fabs(s[i]);
            if (az > zmax) { zmax = az; jmax = i; }
            ztx += s[i] * xv[i];
        }
        ztx = block_sum(ztx, red);
        // first index of the largest |z|: wave-level then block-level argmax
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double oz = __shfl_xor(zmax, off, 64);
            const int64_t oj = __shfl_xor(jmax, off, 64);
            if (oz > zmax || (oz == zmax && oj < jmax)) { zmax = oz; jmax = oj; }
        }
        __syncthreads();
        if (lane == 0) { red[wave] = zmax; s_arg[wave] = jmax; }
        __syncthreads();
        zmax = -1.0;
        jmax = n;
        for (int q = 0; q < nw; ++q)
            if (red[q] > zmax || (red[q] == zmax && s_arg[q] < jmax)) { zmax = red[q]; jmax = s_arg[q]; }
        __syncthreads();
        if (zmax <= ztx) break;
        for (int64_t i = tid; i < n; i += blockDim.x) xv[i] = (i == jmax) ? 1.0 : 0.0;
        __syncthreads();
    }
    if (tid == 0) {
        scal[2] = est;
        scal[3] = n1 * inv1;
    }
}

__global__ void k_stop_init(int32_t *state)
{
    if (threadIdx.x < 2) state[threadIdx.x] = 0;
}

// x = R^{-1} y (sketch-and-solve start).
template <int kSB>
__global__ void __launch_bounds__(kSolveThreads)
k_back(int64_t n, const double *__restrict__ R, int64_t ldr, const double *__restrict__ RT,
       const double *__restrict__ y, double *__restrict__ x, int32_t *__restrict__ status)
{
    extern __shared__ double s[];
    __shared__ SubstLds<kSB> L;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) s[j] = y[j];
    __syncthreads();
    back_subst<kSB>(n, R, ldr, RT, s, L);
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

}  // namespace

hipError_t launch_transpose(hipStream_t s, int64_t n, const double *R, int64_t ldr, double *RT)
{
    hipLaunchKernelGGL(k_transpose, dim3((unsigned)ceil_div(n, 32), (unsigned)ceil_div(n, 32)),
                       dim3(256), 0, s, n, R, ldr, RT);
    return hipGetLastError();
}

hipError_t launch_solve_update(hipStream_t s, int64_t n, const double *R, int64_t ldr,
                               const double *RT, const double *c, double *x, double *xprev,
                               double *dout, int mode, double alpha, double beta, int32_t *status,
                               const StopArgs &st)
{
    hipLaunchKernelGGL(k_solve<kSolveBlock>, dim3(1), dim3(kSolveThreads), (size_t)n * sizeof(double), s, n, R,
                       ldr, RT, c, x, xprev, dout, mode, alpha, beta, status, st.state, st.scal, st.dx,
                       st.gamma, st.rho, st.check);
    return hipGetLastError();
}

hipError_t launch_estimators(hipStream_t s, int64_t n, const double *R, int64_t ldr,
                             const double *RT, uint64_t seed, double *work, double *scal)
{
    hipLaunchKernelGGL(k_estimators<kSolveBlock>, dim3(1), dim3(kEstThreads), (size_t)n * sizeof(double), s,
                       n, R, ldr, RT, seed, work, scal);
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
    hipLaunchKernelGGL(k_back<kSolveBlock>, dim3(1), dim3(kSolveThreads), (size_t)n * sizeof(double), s, n, R, ldr, RT, y,
                       x, status);
    return hipGetLastError();
}
