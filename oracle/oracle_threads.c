/*
 * oracle_threads.c -- the oracle's Jacobi-PCG with its row loops spread
 * over host threads, for timing the CPU on all of its cores.
 *
 * TEST INFRASTRUCTURE ONLY (the CPU-baseline leg of the benchmark and the
 * tests).  It is the loop of or_pcg in apcg_oracle.c (Hestenes & Stiefel;
 * step order of the paper's PCG loop, Section 3.3; Jacobi preconditioning,
 * Section 4.1) with x0 = 0, the unpreconditioned stopping norm and no
 * history: every row loop (product, updates, preconditioner) is an OpenMP
 * loop with a static schedule, and every inner product is a sum of
 * per-thread partials (each thread's rows in index order) added in thread
 * order, so a given thread count always gives the same result.  With one
 * thread every sum is the serial one, bit for bit.  Parity checks use the
 * serial oracle; this file only exists to time the host fairly.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>

#define OT_CONVERGED 1
#define OT_MAXIT 2
#define OT_BREAKDOWN_PAP 4
#define OT_BREAKDOWN_RZ 8
#define OT_NAN 16
#define OT_SETUP_ERROR 128

/* x . y as the sum over threads (in thread order) of each thread's rows
 * summed in index order; part holds one slot per thread. */
static double tdot(int32_t n, const double *x, const double *y, int nt, double *part)
{
#pragma omp parallel num_threads(nt)
    {
        int t = omp_get_thread_num();
        int T = omp_get_num_threads();
        int64_t lo = (int64_t)n * t / T, hi = (int64_t)n * (t + 1) / T;
        double s = 0.0;
        for (int64_t i = lo; i < hi; ++i) s += x[i] * y[i];
        part[t] = s;
        if (t == 0)
            for (int u = T; u < nt; ++u) part[u] = 0.0;
    }
    double s = 0.0;
    for (int t = 0; t < nt; ++t) s += part[t];
    return s;
}

static void tspmv(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val, const double *x,
                  double *y, int nt)
{
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int32_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) s += val[k] * x[col[k]];
        y[i] = s;
    }
}

/* Jacobi-PCG from x0 = 0 on nthreads threads; x receives the iterate.
 * Returns the status bits (the oracle's numbering); *its the number of
 * products with p, *res the final ||r||, *ref = ||b||. */
int32_t or_pcg_threads(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                       const double *b, double *x, double rtol, int32_t maxit, int32_t nthreads,
                       int32_t *its, double *res, double *ref)
{
    int nt = nthreads > 0 ? nthreads : 1;
    size_t nb = (size_t)(n > 0 ? n : 1) * sizeof(double);
    double *dinv = malloc(nb), *r = malloc(nb), *z = malloc(nb), *p = malloc(nb), *w = malloc(nb);
    double *part = malloc((size_t)nt * sizeof(double));
    int32_t status = 0, k = 0, bad = 0;
    *its = 0;
    *res = 0.0;
    *ref = 0.0;
    if (!dinv || !r || !z || !p || !w || !part) { status = OT_SETUP_ERROR; goto done; }

#pragma omp parallel for schedule(static) num_threads(nt) reduction(+ : bad)
    for (int32_t i = 0; i < n; ++i) {
        double d = 0.0;
        int found = 0;
        for (int32_t q = rowptr[i]; q < rowptr[i + 1]; ++q)
            if (col[q] == i) { d = val[q]; found = 1; }
        if (!found || !(d > 0.0)) bad += 1;
        else dinv[i] = 1.0 / d;
        x[i] = 0.0;
        r[i] = b[i];
    }
    if (bad) { status = OT_SETUP_ERROR; goto done; }
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int32_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
    *ref = sqrt(tdot(n, b, b, nt, part));
    *res = sqrt(tdot(n, r, r, nt, part));
    if (*ref == 0.0) { *res = 0.0; status = OT_CONVERGED; goto done; }
    if (!isfinite(*res)) { status = OT_NAN; goto done; }
    if (*res <= rtol * *ref) { status = OT_CONVERGED; goto done; }
    double rho = tdot(n, z, r, nt, part);
    if (!(rho > 0.0)) { status = isfinite(rho) ? OT_BREAKDOWN_RZ : OT_NAN; goto done; }
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int32_t i = 0; i < n; ++i) p[i] = z[i];

    for (k = 1; k <= maxit; ++k) {
        tspmv(n, rowptr, col, val, p, w, nt);
        double delta = tdot(n, p, w, nt, part);
        if (!(delta > 0.0)) {
            status = isfinite(delta) ? OT_BREAKDOWN_PAP : OT_NAN;
            k -= 1;
            break;
        }
        double alpha = rho / delta;
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int32_t i = 0; i < n; ++i) {
            x[i] += alpha * p[i];
            r[i] -= alpha * w[i];
            z[i] = dinv[i] * r[i];
        }
        double rho_new = tdot(n, z, r, nt, part);
        *res = sqrt(tdot(n, r, r, nt, part));
        if (!isfinite(*res) || !isfinite(rho_new)) { status = OT_NAN; break; }
        if (*res <= rtol * *ref) { status = OT_CONVERGED; break; }
        if (!(rho_new > 0.0)) { status = OT_BREAKDOWN_RZ; break; }
        double beta = rho_new / rho;
        rho = rho_new;
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int32_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    if (k > maxit) { k = maxit; status = OT_MAXIT; }
    *its = k;

done:
    free(dinv); free(r); free(z); free(p); free(w); free(part);
    return status;
}
