/*
 * FP64 reference for the l1 regressions of l1 filtering -- TEST INFRASTRUCTURE.
 *
 * This file is part of the oracle: a plain, slow, obviously correct CPU
 * implementation used only by the tests, by the smoke check and by the CPU
 * baseline of the benchmark.  The GPU library never links or calls it and it
 * shares no code with the GPU library.
 *
 * What it computes (Liu, Lin, Wei, Su, "Solving Principal Component Pursuit
 * in Linear Time via l1 Filtering", Sec. 3.2):
 *   the column problem (eq. l1c') and the row problem (eq. l1r') are both of
 *   the form (eq. l1g)
 *        min_{E,Z} ||E||_1   s.t.   X = A Z + E,   A^T A = I,
 *   and decompose into one independent regression per column of X.  Each is
 *   solved by the ADM of Algorithm 1:
 *        E_{k+1} = S_{1/beta_k}( X - A Z_k + Y_k / beta_k )
 *        Z_{k+1} = A^T ( X - E_{k+1} + Y_k / beta_k )
 *        Y_{k+1} = Y_k + beta_k ( X - A Z_{k+1} - E_{k+1} )
 *        beta_{k+1} = min( rho beta_k, beta_bar )
 *   looping while ||X - A Z_k - E_k||_inf / ||X||_inf >= eps, starting from
 *   E_0 = Z_0 = Y_0 = 0.  S_tau is the soft-thresholding operator
 *   S_tau(t) = sgn(t) max(|t| - tau, 0) (Sec. 2, eq. SVT).
 *
 * Readings where the paper is silent (each listed in the design notes):
 *   - beta, the stopping test and ||X||_inf are taken per regression (the
 *     regressions are independent, Sec. 3.2, last paragraph);
 *   - beta_0 = beta0_scale / ||x||_2 and beta_bar = beta_max_scale * beta_0;
 *   - an all-zero x returns z = 0, e = 0, y = 0 after 0 iterations;
 *   - the output is the last iterate; a regression that has not met the test
 *     after max_iter iterations returns -max_iter as its iteration count.
 *
 * oracle_alg1_clip() is an algebraically identical rewrite of the same
 * iteration (valid because A^T A = I), kept here only so that the tests can
 * check the rewrite against the literal form in FP64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Soft-thresholding S_tau(t) = sgn(t) max(|t| - tau, 0). */
static double soft_threshold(double t, double tau)
{
    if (t > tau) return t - tau;
    if (t < -tau) return t + tau;
    return 0.0;
}

/* out = A z, A is p x r column-major with leading dimension lda. */
static void mat_vec(int p, int r, const double *A, int lda, const double *z, double *out)
{
    for (int i = 0; i < p; ++i) out[i] = 0.0;
    for (int c = 0; c < r; ++c) {
        const double zc = z[c];
        const double *col = A + (size_t)c * lda;
        for (int i = 0; i < p; ++i) out[i] += col[i] * zc;
    }
}

/* out = A^T v. */
static void mat_t_vec(int p, int r, const double *A, int lda, const double *v, double *out)
{
    for (int c = 0; c < r; ++c) {
        const double *col = A + (size_t)c * lda;
        double s = 0.0;
        for (int i = 0; i < p; ++i) s += col[i] * v[i];
        out[c] = s;
    }
}

/*
 * Algorithm 1, literal form, on one regression x (length p) against A (p x r).
 * Outputs z (r), e (p), y (p); returns the iteration count K (>= 0) or
 * -max_iter if the stopping test was not met.
 */
int oracle_alg1(int p, int r, const double *x, const double *A, int lda,
                double eps, double rho, double beta0_scale, double beta_max_scale,
                int max_iter, double *z, double *e, double *y)
{
    double xinf = 0.0, xx = 0.0;
    for (int i = 0; i < p; ++i) {
        xinf = fmax(xinf, fabs(x[i]));
        xx += x[i] * x[i];
    }
    for (int c = 0; c < r; ++c) z[c] = 0.0;
    for (int i = 0; i < p; ++i) { e[i] = 0.0; y[i] = 0.0; }
    if (xinf == 0.0) return 0;

    double beta = beta0_scale / sqrt(xx);
    const double beta_bar = beta_max_scale * beta;

    double *az = (double *)malloc(sizeof(double) * (size_t)p);
    double *res = (double *)malloc(sizeof(double) * (size_t)p);
    double *tmp = (double *)malloc(sizeof(double) * (size_t)p);
    /* residual of the starting point: X - A Z_0 - E_0 = X */
    for (int i = 0; i < p; ++i) res[i] = x[i];

    int k = 0;
    for (;;) {
        double rinf = 0.0;
        for (int i = 0; i < p; ++i) rinf = fmax(rinf, fabs(res[i]));
        if (!(rinf / xinf >= eps)) break;          /* loop condition of Alg. 1 */
        if (k == max_iter) { k = -max_iter; break; }

        /* Step 1: E_{k+1} = S_{1/beta}(X - A Z_k + Y_k/beta) */
        mat_vec(p, r, A, lda, z, az);
        for (int i = 0; i < p; ++i)
            e[i] = soft_threshold(x[i] - az[i] + y[i] / beta, 1.0 / beta);

        /* Step 2: Z_{k+1} = A^T (X - E_{k+1} + Y_k/beta) */
        for (int i = 0; i < p; ++i) tmp[i] = x[i] - e[i] + y[i] / beta;
        mat_t_vec(p, r, A, lda, tmp, z);

        /* Step 3: Y_{k+1} = Y_k + beta (X - A Z_{k+1} - E_{k+1}) */
        mat_vec(p, r, A, lda, z, az);
        for (int i = 0; i < p; ++i) {
            res[i] = x[i] - az[i] - e[i];
            y[i] += beta * res[i];
        }
        beta = fmin(rho * beta, beta_bar);
        ++k;
    }
    free(az);
    free(res);
    free(tmp);
    return k;
}

/*
 * The same iteration rewritten with G_k = clip(beta_k (X - A Z_k) + Y_k, -1, 1):
 *   Z_{k+1} = Z_k + A^T G_k / beta_k,   Y_{k+1} = G_k - A A^T G_k,
 *   E_{k+1} = X - A Z_k + (Y_k - G_k)/beta_k,
 *   X - A Z_{k+1} - E_{k+1} = (Y_{k+1} - Y_k)/beta_k.
 * It follows from S_tau(t) = t - clip(t, -tau, tau) and A^T A = I.
 */
int oracle_alg1_clip(int p, int r, const double *x, const double *A, int lda,
                     double eps, double rho, double beta0_scale, double beta_max_scale,
                     int max_iter, double *z, double *e, double *y)
{
    double xinf = 0.0, xx = 0.0;
    for (int i = 0; i < p; ++i) {
        xinf = fmax(xinf, fabs(x[i]));
        xx += x[i] * x[i];
    }
    for (int c = 0; c < r; ++c) z[c] = 0.0;
    for (int i = 0; i < p; ++i) { e[i] = 0.0; y[i] = 0.0; }
    if (xinf == 0.0) return 0;

    double beta = beta0_scale / sqrt(xx);
    const double beta_bar = beta_max_scale * beta;
    double *u = (double *)malloc(sizeof(double) * (size_t)p);  /* X - A Z_k */
    double *g = (double *)malloc(sizeof(double) * (size_t)p);
    double *v = (double *)malloc(sizeof(double) * (size_t)p);
    double *w = (double *)malloc(sizeof(double) * (size_t)(r > 0 ? r : 1));
    for (int i = 0; i < p; ++i) u[i] = x[i];

    int k = 0;
    for (;;) {
        if (k == max_iter) { k = -max_iter; break; }
        for (int i = 0; i < p; ++i) {
            double t = beta * u[i] + y[i];
            g[i] = t > 1.0 ? 1.0 : (t < -1.0 ? -1.0 : t);
        }
        mat_t_vec(p, r, A, lda, g, w);
        for (int c = 0; c < r; ++c) z[c] += w[c] / beta;
        mat_vec(p, r, A, lda, w, v);
        double rinf = 0.0;
        for (int i = 0; i < p; ++i) {
            double ynew = g[i] - v[i];
            e[i] = u[i] + (y[i] - g[i]) / beta;
            rinf = fmax(rinf, fabs(ynew - y[i]) / beta);
            u[i] -= v[i] / beta;
            y[i] = ynew;
        }
        beta = fmin(rho * beta, beta_bar);
        ++k;
        if (!(rinf / xinf >= eps)) break;
    }
    free(u);
    free(g);
    free(v);
    free(w);
    return k;
}

/*
 * Independent regressions: column j of X (p x nreg, leading dimension ldx) is
 * regressed on A.  Z is r x nreg (leading dimension r); E and Y, when not
 * NULL, are p x nreg (leading dimension p).  iters gets one count per
 * regression.  nthreads <= 0 uses the OpenMP default.  form 0 = literal,
 * form 1 = clip rewrite.
 */
void oracle_alg1_batch(int p, int r, int nreg, const double *X, int64_t ldx,
                       const double *A, int lda, double eps, double rho,
                       double beta0_scale, double beta_max_scale, int max_iter,
                       double *Z, double *E, double *Y, int *iters, int nthreads, int form)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        double *e_loc = (double *)malloc(sizeof(double) * (size_t)p);
        double *y_loc = (double *)malloc(sizeof(double) * (size_t)p);
#pragma omp for schedule(dynamic, 16)
        for (int j = 0; j < nreg; ++j) {
            const double *x = X + (size_t)j * (size_t)ldx;
            double *z = Z + (size_t)j * (size_t)r;
            int k = form == 0
                ? oracle_alg1(p, r, x, A, lda, eps, rho, beta0_scale, beta_max_scale,
                              max_iter, z, e_loc, y_loc)
                : oracle_alg1_clip(p, r, x, A, lda, eps, rho, beta0_scale, beta_max_scale,
                                   max_iter, z, e_loc, y_loc);
            if (E) memcpy(E + (size_t)j * p, e_loc, sizeof(double) * (size_t)p);
            if (Y) memcpy(Y + (size_t)j * p, y_loc, sizeof(double) * (size_t)p);
            iters[j] = k;
        }
        free(e_loc);
        free(y_loc);
    }
}

/* Number of threads the OpenMP runtime would use (for reporting). */
int oracle_num_threads(int requested)
{
#ifdef _OPENMP
    if (requested > 0) return requested;
    return omp_get_max_threads();
#else
    (void)requested;
    return 1;
#endif
}
