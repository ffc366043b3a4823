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
#include <omp.h>
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

/* The CG iteration; t_iter (nullable) receives the wall time of each iteration. */
static int64_t cg_core(int64_t n, const int64_t *ip, const int32_t *ix, const double *a,
                       const double *f, double *u, double *r, double *p, double *q,
                       double tol, int64_t maxit, double *relres, double *t_iter)
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
        const double t0 = omp_get_wtime();
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
        if (*relres <= tol) {
            if (t_iter) t_iter[it - 1] = omp_get_wtime() - t0;
            break;
        }
        double beta = rr_new / rr;
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        rr = rr_new;
        if (t_iter) t_iter[it - 1] = omp_get_wtime() - t0;
    }
    return it;
}

int64_t oracle_csr_cg(int64_t n, const int64_t *ip, const int32_t *ix, const double *a,
                      const double *f, double *u, double *r, double *p, double *q,
                      double tol, int64_t maxit, double *relres)
{
    return cg_core(n, ip, ix, a, f, u, r, p, q, tol, maxit, relres, 0);
}

/* Fixed number of CG iterations with the wall time of each (timing). */
int64_t oracle_csr_cg_timed(int64_t n, const int64_t *ip, const int32_t *ix, const double *a,
                            const double *f, double *u, double *r, double *p, double *q,
                            int64_t iters, double *t_iter)
{
    double relres = 0.0;
    return cg_core(n, ip, ix, a, f, u, r, p, q, 0.0, iters, &relres, t_iter);
}

/* Fixed number of CG iterations (no convergence test), for timing. */
int64_t oracle_csr_cg_fixed(int64_t n, const int64_t *ip, const int32_t *ix, const double *a,
                            const double *f, double *u, double *r, double *p, double *q,
                            int64_t iters, double *relres)
{
    return oracle_csr_cg(n, ip, ix, a, f, u, r, p, q, 0.0, iters, relres);
}

/*
 * Periodic linear-FE stiffness in CSR form, assembled per node from
 * node-neighbour coefficient blocks (for grids too large for a triplet list).
 *
 * Node n (grid coordinates x) couples to the nb nodes x + slot_off[k]; row
 * (n, i) holds, for k = 0..nb-1 and j = 0..D-1, the column (x + slot_off[k]) D + j
 * with value sum over the terms t of slot k of
 *     A_t[i][j] lambda(x - vc_t) + B_t[i][j] mu(x - vc_t),
 * i.e. the element blocks of every element having node n as its vertex at
 * position vc_t in its voxel (the terms are formed by oracle/fe.py from the
 * shape-function gradients).  Indices are periodic.  indices and data hold
 * N D nb D entries (every row nb D long); the row pointer is implicit.
 */
void oracle_structured_csr(int dim, const int64_t *shape, int nb, const int32_t *slot_off, int nterm,
                           const int32_t *term_slot, const int32_t *term_vc, const double *term_A,
                           const double *term_B, const double *lam, const double *mu,
                           int32_t *indices, double *data)
{
    const int64_t n0 = shape[0], n1 = dim == 3 ? shape[1] : 1, n2 = dim == 3 ? shape[2] : shape[1];
    const int64_t N = n0 * n1 * n2;
    const int64_t rowlen = (int64_t)nb * dim;
    #pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        const int64_t x0 = n / (n1 * n2), x1 = (n / n2) % n1, x2 = n % n2;
        int32_t *ix = indices + n * dim * rowlen;
        double *a = data + n * dim * rowlen;
        for (int64_t e = 0; e < dim * rowlen; ++e) a[e] = 0.0;
        for (int k = 0; k < nb; ++k) {
            const int32_t *o = slot_off + 3 * k;
            const int64_t y0 = ((x0 + o[0]) % n0 + n0) % n0;
            const int64_t y1 = dim == 3 ? ((x1 + o[1]) % n1 + n1) % n1 : 0;
            const int64_t y2 = ((x2 + o[dim == 3 ? 2 : 1]) % n2 + n2) % n2;
            const int64_t m = (y0 * n1 + y1) * n2 + y2;
            for (int i = 0; i < dim; ++i)
                for (int j = 0; j < dim; ++j) ix[i * rowlen + k * dim + j] = (int32_t)(m * dim + j);
        }
        for (int t = 0; t < nterm; ++t) {
            const int32_t *v = term_vc + 3 * t;
            const int64_t y0 = ((x0 - v[0]) % n0 + n0) % n0;
            const int64_t y1 = dim == 3 ? ((x1 - v[1]) % n1 + n1) % n1 : 0;
            const int64_t y2 = ((x2 - v[dim == 3 ? 2 : 1]) % n2 + n2) % n2;
            const int64_t vox = (y0 * n1 + y1) * n2 + y2;
            const double l = lam[vox], u = mu[vox];
            const int k = term_slot[t];
            for (int i = 0; i < dim; ++i)
                for (int j = 0; j < dim; ++j)
                    a[i * rowlen + k * dim + j] += term_A[(t * dim + i) * dim + j] * l + term_B[(t * dim + i) * dim + j] * u;
        }
    }
}
