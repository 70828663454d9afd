/*
 * Plain FP64 Jacobi-preconditioned conjugate gradient on a CSR matrix.
 *
 * TEST INFRASTRUCTURE ONLY: part of the CPU oracle.  It computes the unique
 * solution of the SPD system of the paper's Section 3.2 on grids too large for
 * a direct solve, and it is the timed CPU baseline.  It shares nothing with the
 * GPU library.
 *
 * The iteration is the textbook PCG of the paper's Algorithm 1 with the
 * diagonal (Jacobi) preconditioner; the stopping test is on the recursive
 * residual, ||r_k||_2 <= rtol * ||b||_2, followed by one explicit residual
 * b - A x whose norm is returned.  Loops are OpenMP-parallel with static
 * schedules, so results are reproducible for a fixed thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

static void csr_mv(int64_t n, const int64_t *ip, const int32_t *ix, const double *a,
                   const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t p = ip[i]; p < ip[i + 1]; ++p)
            s += a[p] * x[ix[p]];
        y[i] = s;
    }
}

static double dot(int64_t n, const double *u, const double *v)
{
    double s = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : s)
    for (int64_t i = 0; i < n; ++i)
        s += u[i] * v[i];
    return s;
}

int oracle_threads(void) { return omp_get_max_threads(); }

/* Threads of the following solves (the one-core timing of the baseline). */
void oracle_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }

/* Returns 0 on convergence, 1 if maxit was reached, 2 on breakdown, 3 on bad input. */
int oracle_jacobi_cg(int64_t n, const int64_t *ip, const int32_t *ix, const double *a,
                     const double *b, double *x, double rtol, int64_t maxit,
                     int64_t *iters_out, double *relres_out)
{
    if (n <= 0 || !ip || !ix || !a || !b || !x)
        return 3;
    double *r = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n);
    double *p = malloc(sizeof(double) * n), *q = malloc(sizeof(double) * n);
    double *dinv = malloc(sizeof(double) * n);
    if (!r || !z || !p || !q || !dinv) {
        free(r); free(z); free(p); free(q); free(dinv);
        return 3;
    }
    int status = 0;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int64_t k = ip[i]; k < ip[i + 1]; ++k)
            if (ix[k] == i) d = a[k];
        dinv[i] = 1.0 / d;
    }
    csr_mv(n, ip, ix, a, x, q);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        r[i] = b[i] - q[i];
        z[i] = dinv[i] * r[i];
        p[i] = z[i];
    }
    double bnorm = sqrt(dot(n, b, b));
    if (bnorm == 0.0) bnorm = 1.0;
    double rz = dot(n, r, z);
    double rr = dot(n, r, r);
    int64_t it = 0;
    while (sqrt(rr) > rtol * bnorm && it < maxit) {
        csr_mv(n, ip, ix, a, p, q);
        double pq = dot(n, p, q);
        if (!(pq > 0.0)) { status = 2; break; }
        double alpha = rz / pq;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * q[i];
            z[i] = dinv[i] * r[i];
        }
        double rz_new = dot(n, r, z);
        rr = dot(n, r, r);
        double beta = rz_new / rz;
        rz = rz_new;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            p[i] = z[i] + beta * p[i];
        ++it;
    }
    if (status == 0 && it >= maxit && sqrt(rr) > rtol * bnorm)
        status = 1;
    csr_mv(n, ip, ix, a, x, q);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        r[i] = b[i] - q[i];
    *relres_out = sqrt(dot(n, r, r)) / bnorm;
    *iters_out = it;
    free(r); free(z); free(p); free(q); free(dinv);
    return status;
}
