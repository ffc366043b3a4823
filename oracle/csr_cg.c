/*
 * Plain conjugate gradients on a symmetric CSR matrix, FP64, OpenMP.
 *
 * TEST INFRASTRUCTURE ONLY: part of the CPU oracle.  Solves K u = f for the
 * canonical periodic linear-FE stiffness assembled by oracle/fe.py (the plain
 * definition the FE-projection scheme is equivalent to), without a
 * preconditioner, from u = 0, until ||f - K u|| <= tol ||f|| or maxit.
 *
 * Returns the number of iterations; *relres receives the final recursive
 * residual norm relative to ||f||.  K must be symmetric positive
 * semi-definite with f in its range.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

static void spmv(int64_t n, const int64_t *ip, const int32_t *ix, const double *a,
                 const double *x, double *y)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t k = ip[i]; k < ip[i + 1]; ++k) s += a[k] * x[ix[k]];
        y[i] = s;
    }
}

static double dot(int64_t n, const double *x, const double *y)
{
    double s = 0.0;
    #pragma omp parallel for reduction(+:s) schedule(static)
    for (int64_t i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}

int64_t oracle_csr_cg(int64_t n, const int64_t *ip, const int32_t *ix, const double *a,
                      const double *f, double *u, double *r, double *p, double *q,
                      double tol, int64_t maxit, double *relres)
{
    memset(u, 0, sizeof(double) * (size_t)n);
    memcpy(r, f, sizeof(double) * (size_t)n);
    memcpy(p, f, sizeof(double) * (size_t)n);
    double nf = sqrt(dot(n, f, f));
    double rr = nf * nf;
    *relres = 0.0;
    if (nf == 0.0) return 0;
    int64_t it = 0;
    while (it < maxit) {
        spmv(n, ip, ix, a, p, q);
        double alpha = rr / dot(n, p, q);
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            u[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        ++it;
        double rr_new = dot(n, r, r);
        *relres = sqrt(rr_new) / nf;
        if (*relres <= tol) break;
        double beta = rr_new / rr;
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        rr = rr_new;
    }
    return it;
}

/* Fixed number of CG iterations (no convergence test), for timing. */
int64_t oracle_csr_cg_fixed(int64_t n, const int64_t *ip, const int32_t *ix, const double *a,
                            const double *f, double *u, double *r, double *p, double *q,
                            int64_t iters, double *relres)
{
    return oracle_csr_cg(n, ip, ix, a, f, u, r, p, q, 0.0, iters, relres);
}
