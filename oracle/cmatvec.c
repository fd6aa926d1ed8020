/* FP64 CPU oracle: the covariance-kernel product Z = diag(rs) Gamma diag(cs) Y
 * with Gamma[i][c] = sigma^2 k(xr_i - xc_c) generated on the fly.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  This is the kernel
 * product of step 5 of the nine-step Galerkin operator (paper Sec. 3.1, the
 * matrix Gamma applied with rows computed on the fly) and of step 3 of
 * Algorithm 1 (paper Sec. 3.2).  Plain loops, one row per OpenMP iteration,
 * FP64 throughout.
 *
 * kernel 0: Gaussian     sigma^2 exp(-|x - y|_2^2 / ell^2)
 * kernel 1: exponential  sigma^2 exp(-|x - y|_1 / ell)
 *
 * xr: nr x 3 row points (row-major), xc: nc x 3 column points,
 * Y: nc x b (row-major), Z: nr x b (row-major, overwritten),
 * rs / cs: optional row / column scalings (NULL means 1).
 */
#include <math.h>
#include <stdlib.h>
#include <omp.h>

void ka_oracle_gamma_apply(int kernel, double sigma, double ell,
                           const double* xr, long nr, const double* xc, long nc,
                           const double* Y, int b, double* Z,
                           const double* rs, const double* cs, int nthreads)
{
    const double s2 = sigma * sigma;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
    {
        double* acc = (double*)malloc(sizeof(double) * (size_t)b);
#pragma omp for schedule(dynamic, 16)
        for (long i = 0; i < nr; ++i) {
            for (int j = 0; j < b; ++j) acc[j] = 0.0;
            const double x0 = xr[3 * i], x1 = xr[3 * i + 1], x2 = xr[3 * i + 2];
            for (long c = 0; c < nc; ++c) {
                const double d0 = x0 - xc[3 * c], d1 = x1 - xc[3 * c + 1], d2 = x2 - xc[3 * c + 2];
                double g;
                if (kernel == 0)
                    g = s2 * exp(-(d0 * d0 + d1 * d1 + d2 * d2) / (ell * ell));
                else
                    g = s2 * exp(-(fabs(d0) + fabs(d1) + fabs(d2)) / ell);
                if (cs) g *= cs[c];
                const double* y = Y + (size_t)c * b;
                for (int j = 0; j < b; ++j) acc[j] += g * y[j];
            }
            const double r = rs ? rs[i] : 1.0;
            for (int j = 0; j < b; ++j) Z[(size_t)i * b + j] = r * acc[j];
        }
        free(acc);
    }
}

int ka_oracle_max_threads(void) { return omp_get_max_threads(); }
