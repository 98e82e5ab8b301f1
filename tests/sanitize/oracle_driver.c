/* Runs every entry point of the oracle (oracle/ls_oracle.c) once on small inputs, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer: any out-of-bounds access, use after free, leak or
 * undefined operation aborts the run.  Inputs are filled by a small linear congruential generator;
 * the checks here are only that each call succeeds and returns finite numbers (the oracle's values
 * are pinned by the Python tests). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

uint64_t orc_splitmix64(uint64_t seed, uint64_t k);
int orc_sparse_sign(int64_t m, int64_t d, int32_t zeta, uint64_t seed, int32_t *rows, int8_t *signs);
int orc_sketch(int64_t m, int64_t n, const double *A, int64_t lda, const double *b, int64_t d,
               int32_t zeta, uint64_t seed, double *B, int64_t ldb, double *Sb);
void orc_solve_r(int64_t n, const double *R, int64_t ldr, const double *y, double *x);
void orc_solve_rt(int64_t n, const double *R, int64_t ldr, const double *c, double *y);
int orc_householder_lstsq(int64_t rows, int64_t n, const double *M, int64_t ldm, const double *rhs,
                          double *R, int64_t ldr, double *qtb, double *x, double *resid);
int orc_tsqr_lstsq(int64_t m, int64_t n, const double *A, int64_t lda, const double *b,
                   int64_t block_rows, int32_t nthreads, double *x, double *R, int64_t ldr, double *resid);
void orc_residual_gradient(int64_t m, int64_t n, const double *A, int64_t lda, const double *b,
                           const double *x, double *c, double *rnorm2);
int orc_iterative_sketching(int64_t m, int64_t n, const double *A, int64_t lda, const double *b,
                            int64_t d, int32_t zeta, uint64_t seed, int32_t q, double *x,
                            double *x_hist, double *R_out, int64_t ldr, double *rnorm2_hist);
int orc_iterative_sketching_dm(int64_t m, int64_t n, const double *A, int64_t lda, const double *b,
                               int64_t d, int32_t zeta, uint64_t seed, int32_t q, double alpha,
                               double beta, double *x, double *x_hist);
double orc_normest(int64_t n, const double *R, int64_t ldr, const double *g, int32_t steps);
double orc_condest_1(int64_t n, const double *R, int64_t ldr);
int64_t orc_dimension(int64_t m, int64_t n, double u);
void orc_sketch_row(int64_t cnt, int64_t n, const double *rows, int64_t ldr, const int8_t *signs,
                    int32_t zeta, double *out);
int orc_iterative_sketching_stop(int64_t m, int64_t n, const double *A, int64_t lda, const double *b,
                                 int64_t d, int32_t zeta, uint64_t seed, int32_t qmax, double gamma,
                                 double rho, const double *g, double *x, int32_t *iters, double *est);
int orc_householder_lstsq_f32(int64_t rows, int64_t n, const float *M, int64_t ldm, const float *rhs,
                              float *R, int64_t ldr, float *qtb, double *x);
void orc_precond_f32(int64_t n, const float *R, int64_t ldr, const double *c, double *d);
double orc_normest_f32(int64_t n, const float *R, int64_t ldr, const double *g, int32_t steps);
double orc_condest_1_f32(int64_t n, const float *R, int64_t ldr);
int32_t orc_mixed_start_steps(double condest);
int orc_iterative_sketching_mixed(int64_t m, int64_t n, const double *A, int64_t lda, const double *b,
                                  int64_t d, int32_t zeta, uint64_t seed, int32_t q, double *x,
                                  float *R_out, int64_t ldr, double *rnorm2_hist, int32_t *used);

static uint64_t lcg = 12345;
static double uni(void)
{
    lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
    return (double)(lcg >> 11) * 0x1p-53 - 0.5;
}

static int failures = 0;
static void check(int ok, const char *what)
{
    if (!ok) {
        fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

static int finite_all(const double *v, int64_t k)
{
    for (int64_t i = 0; i < k; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

int main(void)
{
    const int64_t m = 300, n = 12, lda = 13, d = 100, q = 6;
    const int32_t zeta = 8;
    double *A = calloc((size_t)(m * lda), sizeof(double));
    double *b = calloc((size_t)m, sizeof(double));
    float *Af = calloc((size_t)(d * n), sizeof(float));
    float *bf = calloc((size_t)d, sizeof(float));
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) A[i * lda + j] = uni();
        b[i] = uni();
    }
    check(orc_splitmix64(0, 0) != 0, "splitmix64");
    int32_t *rows = calloc((size_t)(m * zeta), sizeof(int32_t));
    int8_t *signs = calloc((size_t)(m * zeta), 1);
    check(orc_sparse_sign(m, d, zeta, 7, rows, signs) == 0, "sparse_sign");
    check(orc_sparse_sign(m, 3, 3, 7, rows, signs) == 0, "sparse_sign, zeta = d");
    double *B = calloc((size_t)(d * n), sizeof(double)), *Sb = calloc((size_t)d, sizeof(double));
    check(orc_sketch(m, n, A, lda, b, d, zeta, 7, B, n, Sb) == 0 && finite_all(B, d * n), "sketch");
    double *R = calloc((size_t)(n * n), sizeof(double)), *qtb = calloc((size_t)n, sizeof(double));
    double *x = calloc((size_t)n, sizeof(double)), *y = calloc((size_t)n, sizeof(double));
    double res = 0.0;
    check(orc_householder_lstsq(m, n, A, lda, b, R, n, qtb, x, &res) == 0 && finite_all(x, n), "householder");
    check(orc_tsqr_lstsq(m, n, A, lda, b, 64, 2, x, R, n, &res) == 0 && finite_all(x, n), "tsqr");
    check(orc_tsqr_lstsq(m, n, A, lda, b, m, 1, x, NULL, n, NULL) == 0, "tsqr, one block");
    check(orc_tsqr_lstsq(m, n, A, lda, b, n, 1, x, R, n, &res) == 1, "tsqr, block too small");
    double c[12], rr = 0.0;
    orc_residual_gradient(m, n, A, lda, b, x, c, &rr);
    check(finite_all(c, n) && isfinite(rr), "residual_gradient");
    orc_solve_rt(n, R, n, c, y);
    orc_solve_r(n, R, n, y, x);
    check(finite_all(x, n), "substitutions");
    double *xh = calloc((size_t)((q + 1) * n), sizeof(double)), *rh = calloc((size_t)(q + 1), sizeof(double));
    check(orc_iterative_sketching(m, n, A, lda, b, d, zeta, 9, (int32_t)q, x, xh, R, n, rh) == 0 &&
              finite_all(x, n), "iterative_sketching");
    check(orc_iterative_sketching_dm(m, n, A, lda, b, d, zeta, 9, (int32_t)q, 0.5, 0.1, x, xh) == 0, "damping/momentum");
    double g[12];
    for (int64_t i = 0; i < n; ++i) g[i] = uni();
    check(isfinite(orc_normest(n, R, n, g, 3)) && isfinite(orc_condest_1(n, R, n)), "estimators");
    check(orc_dimension(m, n, 0x1p-53) >= n, "dimension");
    double row[12];
    orc_sketch_row(3, n, A, lda, signs, zeta, row);
    check(finite_all(row, n), "sketch_row");
    int32_t iters = 0;
    double est[4];
    check(orc_iterative_sketching_stop(m, n, A, lda, b, d, zeta, 9, 50, 1.0, 0.04, g, x, &iters, est) == 0 &&
              iters >= 1, "stopping rule");
    for (int64_t i = 0; i < d * n; ++i) Af[i] = (float)B[i];
    for (int64_t i = 0; i < d; ++i) bf[i] = (float)Sb[i];
    float *Rf = calloc((size_t)(n * n), sizeof(float)), *qtbf = calloc((size_t)n, sizeof(float));
    check(orc_householder_lstsq_f32(d, n, Af, n, bf, Rf, n, qtbf, x) == 0 && finite_all(x, n), "householder f32");
    orc_precond_f32(n, Rf, n, c, y);
    check(finite_all(y, n), "precond f32");
    check(isfinite(orc_normest_f32(n, Rf, n, g, 3)) && isfinite(orc_condest_1_f32(n, Rf, n)), "estimators f32");
    check(orc_mixed_start_steps(10.0) >= 2, "mixed start steps");
    int32_t used = -1;
    double *rh2 = calloc((size_t)(q + 1), sizeof(double));
    check(orc_iterative_sketching_mixed(m, n, A, lda, b, d, zeta, 9, (int32_t)q, x, Rf, n, rh2, &used) == 0 &&
              used >= 0, "mixed");
    free(A); free(b); free(Af); free(bf); free(rows); free(signs); free(B); free(Sb); free(R); free(qtb);
    free(x); free(y); free(xh); free(rh); free(Rf); free(qtbf); free(rh2);
    if (failures) return 1;
    printf("oracle driver: all calls clean\n");
    return 0;
}
