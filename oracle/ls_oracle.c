/*
 * ls_oracle.c -- plain, slow CPU reference ("the oracle") for iterative sketching, the randomized
 * least-squares solver of E. N. Epperly, "Fast and forward stable randomized algorithms for linear
 * least-squares problems" (arXiv 2311.04362).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this library.  It shares no code, header or constant table with the GPU library;
 * the two meet only in the seeded input arrays they are both given.
 *
 * Everything is IEEE double (single precision only in the mixed-precision functions at the end),
 * straight loops in the order the definitions state them, compiled
 * with -ffp-contract=off so that no multiply-add is fused behind the reader's back.  Matrices are
 * row-major with an explicit leading dimension (elements between two rows).
 *
 * Functions and the passages they follow:
 *   orc_splitmix64          SplitMix64 output (Steele, Lea & Flood, OOPSLA 2014) -- the random
 *                           source of the sparse-sign embedding (the paper leaves it open)
 *   orc_sparse_sign         sparse-sign embedding S, eq. (sparse_sign), Section 2.2
 *   orc_sketch              B = S A and S b, Algorithm 2 (second line)
 *   orc_householder_lstsq   Householder-QR least squares, Section 2.1 (backward-stable reference,
 *                           eq. ls_backward); also the sketch-and-solve start, eq. (sketched_ls)
 *   orc_tsqr_lstsq          the same method in TSQR form (a reduction tree of Householder
 *                           factorizations over row blocks, on host threads) for large m
 *   orc_residual_gradient   r_i = b - A x_i and c_i = A^T r_i, Algorithm 2 loop body
 *   orc_solve_rt/orc_solve_r the two triangular solves of Algorithm 2, Section 3.2
 *   orc_iterative_sketching Algorithm 2 end to end
 *   orc_iterative_sketching_dm  Algorithm 2 with damping / momentum, eq. (damping_momentum)
 *   orc_normest / orc_condest_1 / orc_dimension   Section 3.3 implementation guidance
 *   orc_iterative_sketching_stop  Algorithm 2 with the Section 3.3 stopping rule
 *   *_f32, orc_precond_f32, orc_iterative_sketching_mixed   the mixed-precision reading (single-
 *                           precision sketch, QR and solves; double pass and update), with its
 *                           fallback rule -- the paper is silent on precision; see the comment
 *                           above these functions
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------------------------ */
/* SplitMix64 (Steele, Lea & Flood 2014).  The generator's state advances by the odd constant
 * 0x9E3779B97F4A7C15 per output and each output is the state passed through the finalizer below
 * (the published "mix64" with shifts 30/27/31).  Output k (k = 0, 1, ...) of the stream seeded
 * with `seed` is therefore mix64(seed + (k+1) * gamma): the stream is counter-based. */
static uint64_t orc_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t orc_splitmix64(uint64_t seed, uint64_t k)
{
    return orc_mix64(seed + (k + 1ULL) * 0x9E3779B97F4A7C15ULL);
}

/* ------------------------------------------------------------------------------------------ */
/* Sparse-sign embedding, eq. (sparse_sign): S = zeta^{-1/2} [s_1 ... s_m], each column s_j of
 * length d holding exactly zeta nonzeros equal to +-1 at uniformly random (distinct) positions.
 *
 * Bit-level reading of "uniformly random positions" and "uniform +-1":
 *   column j consumes outputs k = j*2^16 + t, t = 0, 1, 2, ... of the SplitMix64 stream `seed`;
 *   a draw z proposes row (z >> 11) mod d; a row already taken by this column is rejected and the
 *   next draw is used; an accepted draw fixes that entry's sign: -1 if bit 0 of z is set, else +1.
 *   Should all 2^16 draws of a column be spent (only conceivable when d is close to zeta), the
 *   column is completed with the smallest free rows, sign +1.
 * Output: rows[j*zeta + e], signs[j*zeta + e] for the e-th accepted entry of column j. */
#define ORC_DRAWS_PER_COLUMN 65536ULL

int orc_sparse_sign(int64_t m, int64_t d, int32_t zeta, uint64_t seed, int32_t *rows, int8_t *signs)
{
    if (m < 0 || d < 1 || zeta < 1 || zeta > d) return 1;
    for (int64_t j = 0; j < m; ++j) {
        int32_t *rj = rows + j * zeta;
        int8_t *sj = signs + j * zeta;
        int32_t got = 0;
        for (uint64_t t = 0; got < zeta && t < ORC_DRAWS_PER_COLUMN; ++t) {
            uint64_t z = orc_splitmix64(seed, (uint64_t)j * ORC_DRAWS_PER_COLUMN + t);
            int32_t row = (int32_t)((z >> 11) % (uint64_t)d);
            int dup = 0;
            for (int32_t e = 0; e < got; ++e) dup |= (rj[e] == row);
            if (dup) continue;
            rj[got] = row;
            sj[got] = (z & 1ULL) ? -1 : 1;
            ++got;
        }
        for (int32_t row = 0; got < zeta; ++row) {
            int dup = 0;
            for (int32_t e = 0; e < got; ++e) dup |= (rj[e] == row);
            if (!dup) { rj[got] = row; sj[got] = 1; ++got; }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Sketch, Algorithm 2 ("B <- S A"), together with S b (the same S embeds range([A b]),
 * Section 2.3).  By the definition of the product, B[k,:] = sum_j S[k,j] A[j,:].  The loop runs
 * over j in ascending order, so each row of B receives its terms in ascending j.  The entries of S
 * are +-zeta^{-1/2}; the common factor fl(1/sqrt(zeta)) is applied once to each finished sum
 * (adding +-A[j,:] is exact, so the only roundings are the additions and that one product). */
int orc_sketch(int64_t m, int64_t n, const double *A, int64_t lda, const double *b, int64_t d,
               int32_t zeta, uint64_t seed, double *B, int64_t ldb, double *Sb)
{
    if (n < 1 || lda < n || ldb < n || d < 1 || zeta < 1 || zeta > d) return 1;
    int32_t *rows = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1) * (size_t)zeta);
    int8_t *signs = (int8_t *)malloc(sizeof(int8_t) * (size_t)(m > 0 ? m : 1) * (size_t)zeta);
    if (!rows || !signs) { free(rows); free(signs); return 2; }
    orc_sparse_sign(m, d, zeta, seed, rows, signs);
    for (int64_t k = 0; k < d; ++k) {
        for (int64_t c = 0; c < n; ++c) B[k * ldb + c] = 0.0;
        if (Sb) Sb[k] = 0.0;
    }
    for (int64_t j = 0; j < m; ++j) {
        for (int32_t e = 0; e < zeta; ++e) {
            int64_t k = rows[j * zeta + e];
            double s = (double)signs[j * zeta + e];
            for (int64_t c = 0; c < n; ++c) B[k * ldb + c] += s * A[j * lda + c];
            if (Sb && b) Sb[k] += s * b[j];
        }
    }
    double scale = 1.0 / sqrt((double)zeta);
    for (int64_t k = 0; k < d; ++k) {
        for (int64_t c = 0; c < n; ++c) B[k * ldb + c] *= scale;
        if (Sb) Sb[k] *= scale;
    }
    free(rows);
    free(signs);
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Back substitution R x = y for upper-triangular R (n x n). */
void orc_solve_r(int64_t n, const double *R, int64_t ldr, const double *y, double *x)
{
    for (int64_t i = n - 1; i >= 0; --i) {
        double s = y[i];
        for (int64_t k = i + 1; k < n; ++k) s -= R[i * ldr + k] * x[k];
        x[i] = s / R[i * ldr + i];
    }
}

/* Forward substitution R^T y = c (R^T is lower triangular; its row i is column i of R). */
void orc_solve_rt(int64_t n, const double *R, int64_t ldr, const double *c, double *y)
{
    for (int64_t i = 0; i < n; ++i) {
        double s = c[i];
        for (int64_t k = 0; k < i; ++k) s -= R[k * ldr + i] * y[k];
        y[i] = s / R[i * ldr + i];
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Householder-QR least squares (the textbook method of Section 2.1, backward stable):
 * factor W = [M | rhs] (rows x (n+1)) by Householder reflections H_0 ... H_{n-1},
 *   for k = 0..n-1:  alpha = W[k,k];  sigma = ||W[k:rows, k]||;  beta = -sign(alpha) sigma
 *                    (sign(0) = +1);  v = W[k:rows, k] - beta e_1;
 *                    apply H = I - 2 v v^T / (v^T v) to columns k+1..n (rhs included);
 *                    R[k,k] = beta, R[k,k+1:n] = the updated row k,
 * then (Q^T rhs)[0:n] = W[0:n, n] and x solves R x = (Q^T rhs)[0:n] by back substitution.
 * The norm of (Q^T rhs)[n:rows] is ||rhs - M x||.  Q is never formed.
 * Returns 0, 1 on bad arguments, 2 on allocation failure, 3 + k if column k is exactly zero
 * after the previous reflections (rank deficient).  R, qtb, x and resid may be NULL. */
int orc_householder_lstsq(int64_t rows, int64_t n, const double *M, int64_t ldm, const double *rhs,
                          double *R, int64_t ldr, double *qtb, double *x, double *resid)
{
    if (n < 1 || rows < n || ldm < n || (R && ldr < n)) return 1;
    int64_t w = n + 1;
    double *W = (double *)malloc(sizeof(double) * (size_t)rows * (size_t)w);
    double *v = (double *)malloc(sizeof(double) * (size_t)rows);
    double *wt = (double *)malloc(sizeof(double) * (size_t)w);
    double *Rl = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
    if (!W || !v || !wt || !Rl) { free(W); free(v); free(wt); free(Rl); return 2; }
    for (int64_t i = 0; i < rows; ++i) {
        for (int64_t c = 0; c < n; ++c) W[i * w + c] = M[i * ldm + c];
        W[i * w + n] = rhs ? rhs[i] : 0.0;
    }
    memset(Rl, 0, sizeof(double) * (size_t)n * (size_t)n);
    int rc = 0;
    for (int64_t k = 0; k < n; ++k) {
        double alpha = W[k * w + k];
        double ss = 0.0;
        for (int64_t i = k; i < rows; ++i) ss += W[i * w + k] * W[i * w + k];
        double sigma = sqrt(ss);
        if (sigma == 0.0) { rc = 3 + (int)k; break; }
        double beta = (alpha >= 0.0) ? -sigma : sigma;
        v[k] = alpha - beta;
        for (int64_t i = k + 1; i < rows; ++i) v[i] = W[i * w + k];
        double vtv = 0.0;
        for (int64_t i = k; i < rows; ++i) vtv += v[i] * v[i];
        /* w_l = v^T W[k:rows, l] for l = k+1..n, accumulated in row order */
        for (int64_t l = k + 1; l < w; ++l) wt[l] = 0.0;
        for (int64_t i = k; i < rows; ++i)
            for (int64_t l = k + 1; l < w; ++l) wt[l] += v[i] * W[i * w + l];
        for (int64_t l = k + 1; l < w; ++l) wt[l] = 2.0 * wt[l] / vtv;
        for (int64_t i = k; i < rows; ++i)
            for (int64_t l = k + 1; l < w; ++l) W[i * w + l] -= wt[l] * v[i];
        Rl[k * n + k] = beta;
        for (int64_t l = k + 1; l < n; ++l) Rl[k * n + l] = W[k * w + l];
        W[k * w + k] = beta;
        for (int64_t i = k + 1; i < rows; ++i) W[i * w + k] = 0.0;
    }
    if (rc == 0) {
        for (int64_t l = 0; l < n; ++l) wt[l] = W[l * w + n];
        if (qtb) for (int64_t l = 0; l < n; ++l) qtb[l] = wt[l];
        if (resid) {
            double s = 0.0;
            for (int64_t i = n; i < rows; ++i) s += W[i * w + n] * W[i * w + n];
            *resid = sqrt(s);
        }
        if (x) orc_solve_r(n, Rl, n, wt, x);
        if (R)
            for (int64_t i = 0; i < n; ++i)
                for (int64_t c = 0; c < n; ++c) R[i * ldr + c] = Rl[i * n + c];
    }
    free(W); free(v); free(wt); free(Rl);
    return rc;
}

/* ------------------------------------------------------------------------------------------ */
/* Householder least squares in TSQR form ("tall-skinny QR": Demmel, Grigori, Hoemmen & Langou,
 * SIAM J. Sci. Comput. 34, 2012), the same backward-stable method as orc_householder_lstsq
 * (Section 2.1) organised as a reduction tree so that it reaches m in the millions on host cores.
 *
 * The augmented matrix [A | b] (m x (n+1)) is cut into row blocks of block_rows rows (the last block
 * takes the remainder, so it has block_rows .. 2 block_rows - 1 rows).  Each block is factored by
 * orc_householder_lstsq, which yields its triangular factor R_i, (Q_i^T b_i)[0:n] and the norm
 * rho_i of the rest of Q_i^T b_i: together the (n+1) x (n+1) upper-triangular factor
 *     T_i = [[R_i, (Q_i^T b_i)[0:n]], [0, rho_i]]
 * of [A_i | b_i] (T_i^T T_i = [A_i | b_i]^T [A_i | b_i]).  The T_i are stacked in groups of
 * f = max(2, floor(block_rows / (n+1))) and each stacked group is factored the same way (a group of
 * one is passed on unchanged), level after level, until one T remains.  Its leading n x n block is
 * the R of [A | b] up to row signs, and x solves R x = T[0:n, n] by back substitution;
 * |T[n, n]| = ||b - A x|| is a by-product (the last reflection's norm).
 *
 * Blocks of one level are independent and run on up to nthreads host threads (OpenMP); the tree
 * does not depend on the thread count, so neither do the bits of the result.
 * Every block must have full column rank (true with probability one for data drawn from a
 * continuous distribution); returns 0, 1 on bad arguments (block_rows < n + 1, m < n), 2 on
 * allocation failure, 3 + k when the final R has R[k,k] == 0, 4 + n when a block is rank deficient.
 * R (nullable, n x n, ldr) receives the final R, resid (nullable) |T[n, n]|. */
int orc_tsqr_lstsq(int64_t m, int64_t n, const double *A, int64_t lda, const double *b,
                   int64_t block_rows, int32_t nthreads, double *x, double *R, int64_t ldr,
                   double *resid)
{
    if (n < 1 || m < n || lda < n || block_rows < n + 1 || (R && ldr < n) || nthreads < 1) return 1;
    const int64_t w = n + 1;
    int64_t nblk = m / block_rows;
    if (nblk < 1) nblk = 1;
    double *T = (double *)malloc(sizeof(double) * (size_t)nblk * (size_t)w * (size_t)w);
    int *brc = (int *)malloc(sizeof(int) * (size_t)nblk);
    if (!T || !brc) { free(T); free(brc); return 2; }

    /* level 0: row blocks of [A | b] */
    #pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int64_t i = 0; i < nblk; ++i) {
        const int64_t r0 = i * block_rows;
        const int64_t r1 = (i == nblk - 1) ? m : r0 + block_rows;
        double *Ti = T + (size_t)i * (size_t)w * (size_t)w;
        double *qtb = (double *)malloc(sizeof(double) * (size_t)n);
        double rho = 0.0;
        int rc = qtb ? orc_householder_lstsq(r1 - r0, n, A + r0 * lda, lda, b + r0, Ti, w, qtb, NULL, &rho) : 2;
        if (rc == 0) {
            for (int64_t k = 0; k < n; ++k) Ti[k * w + n] = qtb[k];
            for (int64_t c = 0; c < w; ++c) Ti[n * w + c] = 0.0;
            Ti[n * w + n] = rho;
        }
        brc[i] = rc;
        free(qtb);
    }
    int rc = 0;
    for (int64_t i = 0; i < nblk; ++i)
        if (brc[i]) rc = (brc[i] == 2) ? 2 : 4 + (int)n;
    /* upper levels: groups of f stacked factors */
    const int64_t f = (block_rows / w) > 2 ? block_rows / w : 2;
    int64_t cnt = nblk;
    while (rc == 0 && cnt > 1) {
        const int64_t ng = (cnt + f - 1) / f;
        double *Tn = (double *)malloc(sizeof(double) * (size_t)ng * (size_t)w * (size_t)w);
        if (!Tn) { rc = 2; break; }
        #pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
        for (int64_t g = 0; g < ng; ++g) {
            const int64_t k0 = g * f;
            const int64_t k1 = (k0 + f < cnt) ? k0 + f : cnt;
            const double *Y = T + (size_t)k0 * (size_t)w * (size_t)w;   /* (k1-k0) w x w, ld w */
            double *Tg = Tn + (size_t)g * (size_t)w * (size_t)w;
            int grc = 0;
            if (k1 - k0 == 1) {
                memcpy(Tg, Y, sizeof(double) * (size_t)w * (size_t)w);
            } else {
                const int64_t rows = (k1 - k0) * w;
                double *rhs = (double *)malloc(sizeof(double) * (size_t)rows);
                double *qtb = (double *)malloc(sizeof(double) * (size_t)n);
                double rho = 0.0;
                if (!rhs || !qtb) grc = 2;
                if (!grc) {
                    for (int64_t r = 0; r < rows; ++r) rhs[r] = Y[r * w + n];
                    grc = orc_householder_lstsq(rows, n, Y, w, rhs, Tg, w, qtb, NULL, &rho);
                }
                if (!grc) {
                    for (int64_t k = 0; k < n; ++k) Tg[k * w + n] = qtb[k];
                    for (int64_t c = 0; c < w; ++c) Tg[n * w + c] = 0.0;
                    Tg[n * w + n] = rho;
                }
                free(rhs);
                free(qtb);
            }
            brc[g] = grc;
        }
        for (int64_t g = 0; g < ng; ++g)
            if (brc[g]) rc = (brc[g] == 2) ? 2 : 4 + (int)n;
        free(T);
        T = Tn;
        cnt = ng;
    }
    if (rc == 0) {
        for (int64_t k = 0; k < n; ++k)
            if (T[k * w + k] == 0.0) { rc = 3 + (int)k; break; }
    }
    if (rc == 0) {
        double *y = (double *)malloc(sizeof(double) * (size_t)n);
        if (!y) rc = 2;
        else {
            for (int64_t k = 0; k < n; ++k) y[k] = T[k * w + n];
            if (x) orc_solve_r(n, T, w, y, x);
            if (resid) *resid = fabs(T[n * w + n]);
            if (R)
                for (int64_t i = 0; i < n; ++i)
                    for (int64_t c = 0; c < n; ++c) R[i * ldr + c] = (c >= i) ? T[i * w + c] : 0.0;
            free(y);
        }
    }
    free(T);
    free(brc);
    return rc;
}

/* ------------------------------------------------------------------------------------------ */
/* One evaluation of the right-hand side of the refinement step, Algorithm 2 loop body, in the
 * stable form of Section 3.2: first the residual r = b - A x (each (A x)_i summed over columns in
 * order, then subtracted from b_i), then c = A^T r (each c_l summed over rows in order).  The
 * algebraically equal A^T b - A^T (A x) is the unstable "bad residual" variant and is not used.
 * rnorm2 (nullable) receives sum_i r_i^2. */
void orc_residual_gradient(int64_t m, int64_t n, const double *A, int64_t lda, const double *b,
                           const double *x, double *c, double *rnorm2)
{
    double rr = 0.0;
    for (int64_t l = 0; l < n; ++l) c[l] = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        double ax = 0.0;
        for (int64_t l = 0; l < n; ++l) ax += A[i * lda + l] * x[l];
        double r = b[i] - ax;
        rr += r * r;
        for (int64_t l = 0; l < n; ++l) c[l] += A[i * lda + l] * r;
    }
    if (rnorm2) *rnorm2 = rr;
}

/* ------------------------------------------------------------------------------------------ */
/* Iterative sketching, Algorithm 2:
 *   S <- d x m sparse-sign embedding;  B <- S A;  (Q, R) <- QR(B, 'econ');
 *   x_0 <- R^{-1} (Q^T (S b))                      (sketch-and-solve start, eq. sketched_ls)
 *   for i = 0..q-1:  r_i <- b - A x_i;  c_i <- A^T r_i;  d_i <- R^{-1} (R^{-T} c_i);
 *                    x_{i+1} <- x_i + d_i.
 * Outputs x (= x_q); optional x_hist ((q+1) x n: x_0..x_q), R (n x n, ldr), rnorm2_hist (q
 * entries: ||r_i||^2).  Return codes as orc_householder_lstsq. */
int orc_iterative_sketching(int64_t m, int64_t n, const double *A, int64_t lda, const double *b,
                            int64_t d, int32_t zeta, uint64_t seed, int32_t q, double *x,
                            double *x_hist, double *R_out, int64_t ldr, double *rnorm2_hist)
{
    if (n < 1 || m < n || d < n || q < 0 || lda < n) return 1;
    double *B = (double *)malloc(sizeof(double) * (size_t)d * (size_t)n);
    double *Sb = (double *)malloc(sizeof(double) * (size_t)d);
    double *R = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
    double *c = (double *)malloc(sizeof(double) * (size_t)n);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    double *dv = (double *)malloc(sizeof(double) * (size_t)n);
    int rc = 2;
    if (!B || !Sb || !R || !c || !y || !dv) goto done;
    rc = orc_sketch(m, n, A, lda, b, d, zeta, seed, B, n, Sb);
    if (rc) goto done;
    rc = orc_householder_lstsq(d, n, B, n, Sb, R, n, NULL, x, NULL);
    if (rc) goto done;
    if (x_hist) memcpy(x_hist, x, sizeof(double) * (size_t)n);
    for (int32_t i = 0; i < q; ++i) {
        orc_residual_gradient(m, n, A, lda, b, x, c, rnorm2_hist ? &rnorm2_hist[i] : NULL);
        orc_solve_rt(n, R, n, c, y);
        orc_solve_r(n, R, n, y, dv);
        for (int64_t l = 0; l < n; ++l) x[l] = x[l] + dv[l];
        if (x_hist) memcpy(x_hist + (size_t)(i + 1) * (size_t)n, x, sizeof(double) * (size_t)n);
    }
    if (R_out)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t l = 0; l < n; ++l) R_out[i * ldr + l] = R[i * n + l];
done:
    free(B); free(Sb); free(R); free(c); free(y); free(dv);
    return rc;
}

/* Iterative sketching with damping or momentum, eq. (damping_momentum): the same loop with the
 * update x_{i+1} = x_i + alpha d_i + beta (x_i - x_{i-1}); the first step takes x_{-1} = x_0.
 * Damping (eq. damping): alpha = (1-eps^2)^2/(1+eps^2), beta = 0; momentum (eq. momentum):
 * alpha = (1-eps^2)^2, beta = eps^2 (the caller passes alpha and beta). */
int orc_iterative_sketching_dm(int64_t m, int64_t n, const double *A, int64_t lda, const double *b,
                               int64_t d, int32_t zeta, uint64_t seed, int32_t q, double alpha,
                               double beta, double *x, double *x_hist)
{
    if (n < 1 || m < n || d < n || q < 0 || lda < n) return 1;
    double *B = (double *)malloc(sizeof(double) * (size_t)d * (size_t)n);
    double *Sb = (double *)malloc(sizeof(double) * (size_t)d);
    double *R = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
    double *c = (double *)malloc(sizeof(double) * (size_t)n);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    double *dv = (double *)malloc(sizeof(double) * (size_t)n);
    double *xprev = (double *)malloc(sizeof(double) * (size_t)n);
    int rc = 2;
    if (!B || !Sb || !R || !c || !y || !dv || !xprev) goto done;
    rc = orc_sketch(m, n, A, lda, b, d, zeta, seed, B, n, Sb);
    if (rc) goto done;
    rc = orc_householder_lstsq(d, n, B, n, Sb, R, n, NULL, x, NULL);
    if (rc) goto done;
    memcpy(xprev, x, sizeof(double) * (size_t)n);
    if (x_hist) memcpy(x_hist, x, sizeof(double) * (size_t)n);
    for (int32_t i = 0; i < q; ++i) {
        orc_residual_gradient(m, n, A, lda, b, x, c, NULL);
        orc_solve_rt(n, R, n, c, y);
        orc_solve_r(n, R, n, y, dv);
        for (int64_t l = 0; l < n; ++l) {
            double xn = x[l] + alpha * dv[l] + beta * (x[l] - xprev[l]);
            xprev[l] = x[l];
            x[l] = xn;
        }
        if (x_hist) memcpy(x_hist + (size_t)(i + 1) * (size_t)n, x, sizeof(double) * (size_t)n);
    }
done:
    free(B); free(Sb); free(R); free(c); free(y); free(dv); free(xprev);
    return rc;
}

/* ------------------------------------------------------------------------------------------ */
/* Section 3.3 guidance, used by the stopping rule.
 * normest: ||R|| estimated by `steps` steps of the power method on R^T R from the start vector g
 * (the caller passes a Gaussian g): v <- g/||g||; repeat: w = R v, v' = R^T w, est = ||w||,
 * v = v'/||v'||.  Returns the last ||R v||. */
double orc_normest(int64_t n, const double *R, int64_t ldr, const double *g, int32_t steps)
{
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    double est = 0.0, s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += g[i] * g[i];
    s = sqrt(s);
    for (int64_t i = 0; i < n; ++i) v[i] = g[i] / s;
    for (int32_t it = 0; it < steps; ++it) {
        double ww = 0.0;
        for (int64_t i = 0; i < n; ++i) {          /* w = R v (R upper) */
            double a = 0.0;
            for (int64_t k = i; k < n; ++k) a += R[i * ldr + k] * v[k];
            w[i] = a;
            ww += a * a;
        }
        est = sqrt(ww);
        double vv = 0.0;
        for (int64_t k = 0; k < n; ++k) {          /* v = R^T w */
            double a = 0.0;
            for (int64_t i = 0; i <= k; ++i) a += R[i * ldr + k] * w[i];
            v[k] = a;
            vv += a * a;
        }
        vv = sqrt(vv);
        if (vv == 0.0) break;
        for (int64_t k = 0; k < n; ++k) v[k] /= vv;
    }
    free(v); free(w);
    return est;
}

/* ||T^{-1}||_1 estimate for T in {R, R^T} by Hager's method (Higham, Accuracy and Stability,
 * Ch. 15, Alg. 15.3 without the extra vector): start x = e/n; repeat: y = T^{-1} x;
 * xi = sign(y); z = T^{-T} xi; if ||z||_inf <= z^T x stop; else x = e_j, j = argmax |z_j|.
 * Used as condest(R) = ||R||_1 * est(||R^{-1}||_1). */
static double orc_inv_norm1_est(int64_t n, const double *R, int64_t ldr)
{
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) x[i] = 1.0 / (double)n;
    double est = 0.0;
    for (int it = 0; it < 5; ++it) {
        orc_solve_r(n, R, ldr, x, y);               /* y = R^{-1} x */
        est = 0.0;
        for (int64_t i = 0; i < n; ++i) est += fabs(y[i]);
        for (int64_t i = 0; i < n; ++i) y[i] = (y[i] >= 0.0) ? 1.0 : -1.0;
        orc_solve_rt(n, R, ldr, y, z);              /* z = R^{-T} xi */
        int64_t jmax = 0;
        double zmax = 0.0, ztx = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (fabs(z[i]) > zmax) { zmax = fabs(z[i]); jmax = i; }
            ztx += z[i] * x[i];
        }
        if (zmax <= ztx) break;
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        x[jmax] = 1.0;
    }
    free(x); free(y); free(z);
    return est;
}

double orc_condest_1(int64_t n, const double *R, int64_t ldr)
{
    double n1 = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        double s = 0.0;
        for (int64_t i = 0; i <= k; ++i) s += fabs(R[i * ldr + k]);
        if (s > n1) n1 = s;
    }
    return n1 * orc_inv_norm1_est(n, R, ldr);
}

/* Principal branch W_0 of the Lambert W function for x >= 0 by Newton's method on w e^w = x. */
static double orc_lambert_w0(double x)
{
    double w = (x < 1.0) ? x : log(x) - log(log(x) + 1.0);
    if (w < 0.0) w = 0.0;
    for (int it = 0; it < 100; ++it) {
        double ew = exp(w);
        double f = w * ew - x;
        double wn = w - f / (ew * (w + 1.0));
        if (fabs(wn - w) <= 1e-15 * (1.0 + fabs(wn))) { w = wn; break; }
        w = wn;
    }
    return w;
}

/* Embedding dimension of eq. (dimension):
 *   d = max(ceil((6+4 sqrt 2) n exp(W((6-4 sqrt 2) (m/n^2) log(1/u)))), 20 n). */
int64_t orc_dimension(int64_t m, int64_t n, double u)
{
    double a = 6.0 + 4.0 * sqrt(2.0), c = 6.0 - 4.0 * sqrt(2.0);
    double arg = c * ((double)m / ((double)n * (double)n)) * log(1.0 / u);
    double dd = ceil(a * (double)n * exp(orc_lambert_w0(arg)));
    int64_t d = (int64_t)dd;
    return d > 20 * n ? d : 20 * n;
}

/* One row of the sketch from its terms: out = fl(1/sqrt(zeta)) * sum_t sign_t * rows[t, :], summed
 * in the order given (the caller passes the terms of sketch row k in ascending column j of S, as
 * the full product orc_sketch accumulates them).  Lets a test check sampled rows of a sketch whose
 * A is too large to sketch on the CPU. */
void orc_sketch_row(int64_t cnt, int64_t n, const double *rows, int64_t ldr, const int8_t *signs,
                    int32_t zeta, double *out)
{
    for (int64_t c = 0; c < n; ++c) out[c] = 0.0;
    for (int64_t t = 0; t < cnt; ++t) {
        double s = (double)signs[t];
        for (int64_t c = 0; c < n; ++c) out[c] += s * rows[t * ldr + c];
    }
    double scale = 1.0 / sqrt((double)zeta);
    for (int64_t c = 0; c < n; ++c) out[c] *= scale;
}

/* ------------------------------------------------------------------------------------------ */
/* Algorithm 2 with the stopping rule of Section 3.3: normest = orc_normest(R, g, ceil(ln n)),
 * condest = orc_condest_1(R); after each update, stop and return x_{i+1} as soon as
 *   ||r(x_{i+1}) - r(x_i)|| <= u (gamma normest ||x_{i+1}|| + rho condest ||r(x_{i+1})||),
 * u = 2^-53, with at most qmax updates.  Both residual norms are evaluated from their definition
 * (r(x) = b - A x for each iterate).  *iters receives the number of updates made; est (nullable,
 * 2 doubles) receives normest and condest.  Return codes as orc_iterative_sketching. */
int orc_iterative_sketching_stop(int64_t m, int64_t n, const double *A, int64_t lda, const double *b,
                                 int64_t d, int32_t zeta, uint64_t seed, int32_t qmax, double gamma,
                                 double rho, const double *g, double *x, int32_t *iters, double *est)
{
    if (n < 1 || m < n || d < n || qmax < 0 || lda < n) return 1;
    const double u = ldexp(1.0, -53);
    double *B = (double *)malloc(sizeof(double) * (size_t)d * (size_t)n);
    double *Sb = (double *)malloc(sizeof(double) * (size_t)d);
    double *R = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
    double *c = (double *)malloc(sizeof(double) * (size_t)n);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    double *dv = (double *)malloc(sizeof(double) * (size_t)n);
    double *xn = (double *)malloc(sizeof(double) * (size_t)n);
    int rc = 2;
    *iters = 0;
    if (!B || !Sb || !R || !c || !y || !dv || !xn) goto done;
    rc = orc_sketch(m, n, A, lda, b, d, zeta, seed, B, n, Sb);
    if (rc) goto done;
    rc = orc_householder_lstsq(d, n, B, n, Sb, R, n, NULL, x, NULL);
    if (rc) goto done;
    {
        int32_t steps = (int32_t)ceil(log((double)n));
        if (steps < 1) steps = 1;
        double normest = orc_normest(n, R, n, g, steps);
        double condest = orc_condest_1(n, R, n);
        if (est) { est[0] = normest; est[1] = condest; }
        for (int32_t i = 0; i < qmax; ++i) {
            orc_residual_gradient(m, n, A, lda, b, x, c, NULL);
            orc_solve_rt(n, R, n, c, y);
            orc_solve_r(n, R, n, y, dv);
            for (int64_t l = 0; l < n; ++l) xn[l] = x[l] + dv[l];
            /* ||r(x_{i+1}) - r(x_i)|| = ||A (x_{i+1} - x_i)||, ||r(x_{i+1})||, ||x_{i+1}|| */
            double dr = 0.0, rr = 0.0, xx = 0.0;
            for (int64_t l = 0; l < n; ++l) xx += xn[l] * xn[l];
            for (int64_t j = 0; j < m; ++j) {
                double ad = 0.0, ax = 0.0;
                for (int64_t l = 0; l < n; ++l) {
                    ad += A[j * lda + l] * (xn[l] - x[l]);
                    ax += A[j * lda + l] * xn[l];
                }
                double r = b[j] - ax;
                dr += ad * ad;
                rr += r * r;
            }
            for (int64_t l = 0; l < n; ++l) x[l] = xn[l];
            *iters = i + 1;
            if (sqrt(dr) <= u * (gamma * normest * sqrt(xx) + rho * condest * sqrt(rr))) break;
        }
    }
done:
    free(B); free(Sb); free(R); free(c); free(y); free(dv); free(xn);
    return rc;
}

/* ------------------------------------------------------------------------------------------ */
/* Mixed precision.  The paper computes everything in double.  This is the reading in which the
 * sketch is kept in single precision (the double sketch of orc_sketch, rounded once), its
 * Householder QR and the two triangular solves of every step run in single precision, and the
 * residual/gradient pass and the update stay in double, so the iteration is an iterative
 * refinement whose preconditioner is a single-precision R.  Single-precision code below keeps every
 * intermediate in IEEE binary32 (x86-64 SSE evaluates float expressions in float). */

/* Back and forward substitution in single precision (as orc_solve_r / orc_solve_rt). */
void orc_solve_r_f32(int64_t n, const float *R, int64_t ldr, const float *y, float *x)
{
    for (int64_t i = n - 1; i >= 0; --i) {
        float s = y[i];
        for (int64_t k = i + 1; k < n; ++k) s -= R[i * ldr + k] * x[k];
        x[i] = s / R[i * ldr + i];
    }
}

void orc_solve_rt_f32(int64_t n, const float *R, int64_t ldr, const float *c, float *y)
{
    for (int64_t i = 0; i < n; ++i) {
        float s = c[i];
        for (int64_t k = 0; k < i; ++k) s -= R[k * ldr + i] * y[k];
        y[i] = s / R[i * ldr + i];
    }
}

/* Householder-QR least squares in single precision: the steps of orc_householder_lstsq with every
 * quantity a float (sigma by sqrtf of the float sum of squares).  x (double, nullable) receives the
 * float back-substitution solution R x = (Q^T rhs)[0:n], widened.  Return codes as the double
 * version. */
int orc_householder_lstsq_f32(int64_t rows, int64_t n, const float *M, int64_t ldm, const float *rhs,
                              float *R, int64_t ldr, float *qtb, double *x)
{
    if (n < 1 || rows < n || ldm < n || (R && ldr < n)) return 1;
    int64_t w = n + 1;
    float *W = (float *)malloc(sizeof(float) * (size_t)rows * (size_t)w);
    float *v = (float *)malloc(sizeof(float) * (size_t)rows);
    float *wt = (float *)malloc(sizeof(float) * (size_t)w);
    float *Rl = (float *)malloc(sizeof(float) * (size_t)n * (size_t)n);
    float *xs = (float *)malloc(sizeof(float) * (size_t)n);
    if (!W || !v || !wt || !Rl || !xs) { free(W); free(v); free(wt); free(Rl); free(xs); return 2; }
    for (int64_t i = 0; i < rows; ++i) {
        for (int64_t c = 0; c < n; ++c) W[i * w + c] = M[i * ldm + c];
        W[i * w + n] = rhs ? rhs[i] : 0.0f;
    }
    memset(Rl, 0, sizeof(float) * (size_t)n * (size_t)n);
    int rc = 0;
    for (int64_t k = 0; k < n; ++k) {
        float alpha = W[k * w + k];
        float ss = 0.0f;
        for (int64_t i = k; i < rows; ++i) ss += W[i * w + k] * W[i * w + k];
        float sigma = sqrtf(ss);
        if (sigma == 0.0f) { rc = 3 + (int)k; break; }
        float beta = (alpha >= 0.0f) ? -sigma : sigma;
        v[k] = alpha - beta;
        for (int64_t i = k + 1; i < rows; ++i) v[i] = W[i * w + k];
        float vtv = 0.0f;
        for (int64_t i = k; i < rows; ++i) vtv += v[i] * v[i];
        for (int64_t l = k + 1; l < w; ++l) wt[l] = 0.0f;
        for (int64_t i = k; i < rows; ++i)
            for (int64_t l = k + 1; l < w; ++l) wt[l] += v[i] * W[i * w + l];
        for (int64_t l = k + 1; l < w; ++l) wt[l] = 2.0f * wt[l] / vtv;
        for (int64_t i = k; i < rows; ++i)
            for (int64_t l = k + 1; l < w; ++l) W[i * w + l] -= wt[l] * v[i];
        Rl[k * n + k] = beta;
        for (int64_t l = k + 1; l < n; ++l) Rl[k * n + l] = W[k * w + l];
        W[k * w + k] = beta;
        for (int64_t i = k + 1; i < rows; ++i) W[i * w + k] = 0.0f;
    }
    if (rc == 0) {
        for (int64_t l = 0; l < n; ++l) wt[l] = W[l * w + n];
        if (qtb) for (int64_t l = 0; l < n; ++l) qtb[l] = wt[l];
        if (x) {
            orc_solve_r_f32(n, Rl, n, wt, xs);
            for (int64_t l = 0; l < n; ++l) x[l] = (double)xs[l];
        }
        if (R)
            for (int64_t i = 0; i < n; ++i)
                for (int64_t c = 0; c < n; ++c) R[i * ldr + c] = Rl[i * n + c];
    }
    free(W); free(v); free(wt); free(Rl); free(xs);
    return rc;
}

/* d = R^{-1} (R^{-T} c) for a double c and a single-precision R: c is scaled by 2^-e, e the binary
 * exponent of max_i |c_i| in the frexp convention (so the largest entry lands in [1/2, 1)), rounded
 * to float, both substitutions run in float, and the result is scaled back by 2^e in double.  Both
 * scalings are exact; the scaling keeps the float solves clear of underflow and overflow. */
void orc_precond_f32(int64_t n, const float *R, int64_t ldr, const double *c, double *d)
{
    float *cs = (float *)malloc(sizeof(float) * (size_t)n);
    float *y = (float *)malloc(sizeof(float) * (size_t)n);
    float *z = (float *)malloc(sizeof(float) * (size_t)n);
    double mx = 0.0;
    for (int64_t i = 0; i < n; ++i) if (fabs(c[i]) > mx) mx = fabs(c[i]);
    int e = 0;
    if (mx > 0.0 && isfinite(mx)) (void)frexp(mx, &e);
    for (int64_t i = 0; i < n; ++i) cs[i] = (float)ldexp(c[i], -e);
    orc_solve_rt_f32(n, R, ldr, cs, y);
    orc_solve_r_f32(n, R, ldr, y, z);
    for (int64_t i = 0; i < n; ++i) d[i] = ldexp((double)z[i], e);
    free(cs); free(y); free(z);
}

/* Section 3.3 estimators evaluated in single precision on a single-precision R (the steps of
 * orc_normest and orc_condest_1 with float quantities; the start vector g is rounded to float). */
double orc_normest_f32(int64_t n, const float *R, int64_t ldr, const double *g, int32_t steps)
{
    float *v = (float *)malloc(sizeof(float) * (size_t)n);
    float *w = (float *)malloc(sizeof(float) * (size_t)n);
    float est = 0.0f, s = 0.0f;
    for (int64_t i = 0; i < n; ++i) { v[i] = (float)g[i]; s += v[i] * v[i]; }
    s = sqrtf(s);
    for (int64_t i = 0; i < n; ++i) v[i] = v[i] / s;
    for (int32_t it = 0; it < steps; ++it) {
        float ww = 0.0f;
        for (int64_t i = 0; i < n; ++i) {
            float a = 0.0f;
            for (int64_t k = i; k < n; ++k) a += R[i * ldr + k] * v[k];
            w[i] = a;
            ww += a * a;
        }
        est = sqrtf(ww);
        float vv = 0.0f;
        for (int64_t k = 0; k < n; ++k) {
            float a = 0.0f;
            for (int64_t i = 0; i <= k; ++i) a += R[i * ldr + k] * w[i];
            v[k] = a;
            vv += a * a;
        }
        vv = sqrtf(vv);
        if (vv == 0.0f) break;
        for (int64_t k = 0; k < n; ++k) v[k] /= vv;
    }
    free(v); free(w);
    return (double)est;
}

double orc_condest_1_f32(int64_t n, const float *R, int64_t ldr)
{
    float n1 = 0.0f;
    for (int64_t k = 0; k < n; ++k) {
        float s = 0.0f;
        for (int64_t i = 0; i <= k; ++i) s += fabsf(R[i * ldr + k]);
        if (s > n1) n1 = s;
    }
    float *x = (float *)malloc(sizeof(float) * (size_t)n);
    float *y = (float *)malloc(sizeof(float) * (size_t)n);
    float *z = (float *)malloc(sizeof(float) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) x[i] = 1.0f / (float)n;
    float est = 0.0f;
    for (int it = 0; it < 5; ++it) {
        orc_solve_r_f32(n, R, ldr, x, y);
        est = 0.0f;
        for (int64_t i = 0; i < n; ++i) est += fabsf(y[i]);
        for (int64_t i = 0; i < n; ++i) y[i] = (y[i] >= 0.0f) ? 1.0f : -1.0f;
        orc_solve_rt_f32(n, R, ldr, y, z);
        int64_t jmax = 0;
        float zmax = 0.0f, ztx = 0.0f;
        for (int64_t i = 0; i < n; ++i) {
            if (fabsf(z[i]) > zmax) { zmax = fabsf(z[i]); jmax = i; }
            ztx += z[i] * x[i];
        }
        if (zmax <= ztx) break;
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0f;
        x[jmax] = 1.0f;
    }
    free(x); free(y); free(z);
    return (double)n1 * (double)est;
}

/* Refinement steps of the sketch-and-solve start in the mixed reading: the single-precision QR
 * solution x_0 is only single-precision accurate, while eq. (sketched_ls) defines x_0 as the exact
 * minimizer of ||S b - S A x||; k0 steps of x <- x + orc_precond_f32(R, B^T (S b - B x)) on the
 * double sketch (residual and update in double, as in the main loop) bring it to double accuracy.
 * The contraction of these steps is about 2 condest(R) u_32, hence
 *   k0 = ceil(ln(1e-9) / ln(2 condest u_32)), clamped to [2, 8]
 * (from single-precision accuracy, about 1e-7, down to about 1e-16). */
int32_t orc_mixed_start_steps(double condest)
{
    double rho = 2.0 * condest * ldexp(1.0, -24);
    if (!(rho > 0.0)) return 2;
    if (rho >= 0.5) return 8;
    double k = ceil(log(1e-9) / log(rho));
    return k < 2.0 ? 2 : (k > 8.0 ? 8 : (int32_t)k);
}

/* Algorithm 2 in mixed precision, with the fallback rule of this reading:
 *   B, S b (double, orc_sketch) -> rounded to float; single-precision Householder QR gives R and
 *   x_0; if condest(R) (orc_condest_1_f32) times u_32 = 2^-24 exceeds 0.05 (or is not finite), the
 *   single-precision factor is not trusted and the whole solve is redone in double
 *   (orc_iterative_sketching), *used = 2;
 *   otherwise x_0 is refined on the double sketch (orc_mixed_start_steps), then q steps
 *   x <- x + orc_precond_f32(R, A^T (b - A x)) with the pass and the update in double; if
 *   ||r(x_i)||^2 grows three steps in a row, each time by more than a relative 2^-20 (well above its
 *   rounding noise), or is not finite, the solve is redone in double, *used = 3; else *used = 1.
 * R_out (nullable, float, ldr) receives the single-precision R; rnorm2_hist (nullable, q) the
 * ||r_i||^2 of the mixed steps made.  Return codes as orc_iterative_sketching. */
int orc_iterative_sketching_mixed(int64_t m, int64_t n, const double *A, int64_t lda, const double *b,
                                  int64_t d, int32_t zeta, uint64_t seed, int32_t q, double *x,
                                  float *R_out, int64_t ldr, double *rnorm2_hist, int32_t *used)
{
    if (n < 1 || m < n || d < n || q < 0 || lda < n) return 1;
    double *B = (double *)malloc(sizeof(double) * (size_t)d * (size_t)n);
    double *Sb = (double *)malloc(sizeof(double) * (size_t)d);
    float *B32 = (float *)malloc(sizeof(float) * (size_t)d * (size_t)n);
    float *Sb32 = (float *)malloc(sizeof(float) * (size_t)d);
    float *R = (float *)malloc(sizeof(float) * (size_t)n * (size_t)n);
    double *c = (double *)malloc(sizeof(double) * (size_t)n);
    double *dv = (double *)malloc(sizeof(double) * (size_t)n);
    int rc = 2;
    *used = 1;
    if (!B || !Sb || !B32 || !Sb32 || !R || !c || !dv) goto done;
    rc = orc_sketch(m, n, A, lda, b, d, zeta, seed, B, n, Sb);
    if (rc) goto done;
    for (int64_t i = 0; i < d * n; ++i) B32[i] = (float)B[i];
    for (int64_t i = 0; i < d; ++i) Sb32[i] = (float)Sb[i];
    rc = orc_householder_lstsq_f32(d, n, B32, n, Sb32, R, n, NULL, x);
    if (rc) goto done;
    if (R_out)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t l = 0; l < n; ++l) R_out[i * ldr + l] = R[i * n + l];
    {
        double ce = orc_condest_1_f32(n, R, n);
        if (!(ce * ldexp(1.0, -24) <= 0.05)) {
            *used = 2;
            rc = orc_iterative_sketching(m, n, A, lda, b, d, zeta, seed, q, x, NULL, NULL, 0, NULL);
            goto done;
        }
        int32_t k0 = orc_mixed_start_steps(ce);
        for (int32_t k = 0; k < k0; ++k) {
            orc_residual_gradient(d, n, B, n, Sb, x, c, NULL);
            orc_precond_f32(n, R, n, c, dv);
            for (int64_t l = 0; l < n; ++l) x[l] = x[l] + dv[l];
        }
    }
    {
        double prev = 0.0;
        int run = 0;
        for (int32_t i = 0; i < q; ++i) {
            double rr;
            orc_residual_gradient(m, n, A, lda, b, x, c, &rr);
            if (rnorm2_hist) rnorm2_hist[i] = rr;
            run = (i >= 1 && rr > prev * (1.0 + ldexp(1.0, -20))) ? run + 1 : 0;
            if (run >= 3 || !isfinite(rr)) {
                *used = 3;
                rc = orc_iterative_sketching(m, n, A, lda, b, d, zeta, seed, q, x, NULL, NULL, 0, NULL);
                goto done;
            }
            prev = rr;
            orc_precond_f32(n, R, n, c, dv);
            for (int64_t l = 0; l < n; ++l) x[l] = x[l] + dv[l];
        }
    }
done:
    free(B); free(Sb); free(B32); free(Sb32); free(R); free(c); free(dv);
    return rc;
}
