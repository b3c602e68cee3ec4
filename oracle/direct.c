/*
 * oracle/direct.c -- plain FP64 CPU evaluation of the additive-kernel
 * matrix-vector products, computed straight from their definitions.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent checker for the
 * GPU library: only the tests, the smoke check and the benchmark's CPU
 * baseline may load it.  It shares no code, header or table with the GPU
 * path.
 *
 * What is computed (O(P * N * rows) work, no approximation):
 *
 *   Windowed additive kernel (eq. (3), "windowed ANOVA kernel" section, and
 *   its implementation form eqs. (7)-(8) in "Implementing the NFFT approach"):
 *       K(x_i, x_j) = sum_w sigma_w^2 kappa(||x_i^{W_w} - x_j^{W_w}||; l_w)
 *   with a separate amplitude sigma_w per window as in the feature-grouping
 *   optimisation of the feature-arrangement section (one shared sigma_f is
 *   the all-equal case) and a separate length scale l_w per window.
 *
 *   Gaussian   kappa(r) = exp(-r^2 / (2 l^2)),  d kappa/d l = r^2 / l^3 * kappa
 *              (derivative from the "Implementing the NFFT approach" section)
 *   Matern-1/2 kappa(r) = exp(-r / l),          d kappa/d l = r / l^2 * kappa
 *              (section "Extension to other kernels")
 *   Matern-3/2 kappa(r) = (1 + a r) exp(-a r),  a = sqrt(3) / l,
 *              d kappa/d l = 3 r^2 / l^3 * exp(-a r)
 *              (the further kernel that section names; the standard
 *              Matern form with smoothness 3/2, differentiated in l)
 *
 *   Y[i, r]          = sum_w sigma_w^2 sum_j kappa_w(i, j) V[j, r]
 *   dY_dl[w][i, r]   = sigma_w^2 sum_j d kappa_w(i, j)/d l_w V[j, r]
 *   dY_ds[w][i, r]   = 2 sigma_w sum_j kappa_w(i, j) V[j, r]
 *
 * The diagonal term j = i is included (the fast summation sums over all j).
 *
 * Summation: terms are added in blocks of ORACLE_BLOCK consecutive j in
 * plain double precision, and block sums are combined with Neumaier's
 * compensated summation, so the rounding error stays near a few ulps of
 * the result even for N = 10^6 terms.
 *
 * Matrices are column-major with a leading dimension: V[j + r * ldv],
 * Y[i + r * ldy].  X is row-major: X[j * ldx + f].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_BLOCK 256
#define ORACLE_MAXD 8

enum { ORACLE_GAUSSIAN = 1, ORACLE_MATERN12 = 3, ORACLE_MATERN32 = 5 };

typedef struct {
    double s;
    double c;
} neumaier_t;

static inline void neumaier_add(neumaier_t *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

/* kappa and d kappa / d l for squared distance r2 */
static inline void kernel_eval(int kernel, double r2, double ell, double *k, double *dk)
{
    if (kernel == ORACLE_GAUSSIAN) {
        double e = exp(-r2 / (2.0 * ell * ell));
        *k = e;
        *dk = r2 / (ell * ell * ell) * e;
    } else if (kernel == ORACLE_MATERN12) {
        double r = sqrt(r2);
        double e = exp(-r / ell);
        *k = e;
        *dk = r / (ell * ell) * e;
    } else {
        double ar = sqrt(3.0 * r2) / ell;
        double e = exp(-ar);
        *k = (1.0 + ar) * e;
        *dk = ar * ar / ell * e;
    }
}

/*
 * Returns 0 on success, a negative value on invalid arguments.
 * rows: indices of the output rows to evaluate (NULL = all N rows, in order).
 * Y, dY_dl, dY_ds may each be NULL.  dY_dl and dY_ds hold P consecutive
 * blocks, block w starting at w * ldy * R.
 */
int oracle_direct(int64_t N, int32_t D, const double *X, int64_t ldx,
                  int32_t P, const int32_t *win_off, const int32_t *win_feat,
                  int32_t kernel, const double *ell, const double *sigma,
                  int32_t R, const double *V, int64_t ldv,
                  int64_t nrows, const int64_t *rows,
                  double *Y, int64_t ldy, double *dY_dl, double *dY_ds)
{
    if (N < 0 || D <= 0 || P <= 0 || R <= 0 || nrows < 0 || ldx < D || ldv < N || ldy < nrows)
        return -1;
    if (kernel != ORACLE_GAUSSIAN && kernel != ORACLE_MATERN12 && kernel != ORACLE_MATERN32)
        return -2;
    for (int32_t w = 0; w < P; ++w) {
        int32_t dw = win_off[w + 1] - win_off[w];
        if (dw <= 0 || dw > ORACLE_MAXD || !(ell[w] > 0.0))
            return -3;
        for (int32_t q = win_off[w]; q < win_off[w + 1]; ++q)
            if (win_feat[q] < 0 || win_feat[q] >= D)
                return -4;
    }

#pragma omp parallel
    {
        neumaier_t *accK = (neumaier_t *)malloc(sizeof(neumaier_t) * (size_t)R);
        neumaier_t *accD = (neumaier_t *)malloc(sizeof(neumaier_t) * (size_t)R);
        double *blkK = (double *)malloc(sizeof(double) * (size_t)R);
        double *blkD = (double *)malloc(sizeof(double) * (size_t)R);

#pragma omp for schedule(dynamic, 4)
        for (int64_t ii = 0; ii < nrows; ++ii) {
            int64_t i = rows ? rows[ii] : ii;
            const double *xi = X + i * ldx;
            for (int32_t r = 0; r < R && Y; ++r)
                Y[ii + r * ldy] = 0.0;
            for (int32_t w = 0; w < P; ++w) {
                const int32_t f0 = win_off[w], dw = win_off[w + 1] - win_off[w];
                double xw[ORACLE_MAXD];
                for (int32_t q = 0; q < dw; ++q)
                    xw[q] = xi[win_feat[f0 + q]];
                memset(accK, 0, sizeof(neumaier_t) * (size_t)R);
                memset(accD, 0, sizeof(neumaier_t) * (size_t)R);
                for (int64_t j0 = 0; j0 < N; j0 += ORACLE_BLOCK) {
                    int64_t j1 = j0 + ORACLE_BLOCK < N ? j0 + ORACLE_BLOCK : N;
                    for (int32_t r = 0; r < R; ++r) {
                        blkK[r] = 0.0;
                        blkD[r] = 0.0;
                    }
                    for (int64_t j = j0; j < j1; ++j) {
                        const double *xj = X + j * ldx;
                        double r2 = 0.0;
                        for (int32_t q = 0; q < dw; ++q) {
                            double t = xw[q] - xj[win_feat[f0 + q]];
                            r2 += t * t;
                        }
                        double k, dk;
                        kernel_eval(kernel, r2, ell[w], &k, &dk);
                        for (int32_t r = 0; r < R; ++r) {
                            double v = V[j + r * ldv];
                            blkK[r] += k * v;
                            blkD[r] += dk * v;
                        }
                    }
                    for (int32_t r = 0; r < R; ++r) {
                        neumaier_add(&accK[r], blkK[r]);
                        neumaier_add(&accD[r], blkD[r]);
                    }
                }
                const double s = sigma[w];
                for (int32_t r = 0; r < R; ++r) {
                    double kv = accK[r].s + accK[r].c;
                    double dv = accD[r].s + accD[r].c;
                    if (Y)
                        Y[ii + r * ldy] += s * s * kv;
                    if (dY_dl)
                        dY_dl[(int64_t)w * ldy * R + ii + r * ldy] = s * s * dv;
                    if (dY_ds)
                        dY_ds[(int64_t)w * ldy * R + ii + r * ldy] = 2.0 * s * kv;
                }
            }
        }
        free(accK);
        free(accD);
        free(blkK);
        free(blkD);
    }
    return 0;
}

/* Number of OpenMP threads the oracle runs with (for reporting). */
int oracle_num_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}
