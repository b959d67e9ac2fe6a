/*
 * apcg_oracle.c -- plain, serial, FP64 CPU reference for the asynchronous
 * PCG hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file: only the test suite, the package smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header or
 * constant with the HIP library.
 *
 * Every loop runs serially in index order, in IEEE double precision with no
 * blocking, fusion or reordering beyond what the cited definition states.
 *
 * Sources:
 *   - Preconditioned CG: Hestenes & Stiefel (1952), cited by the paper in
 *     Section 4.2; step order follows the paper's mixed sync/async PCG loop
 *     (Section 3.3): alpha from p.w, x and r updates, preconditioner apply,
 *     norm of the new residual, convergence test, beta from z.r, then the
 *     direction update p = z + beta p.  Initialisation (omitted in the
 *     paper) is the textbook one: r0 = b - A x0, z0 = B r0, p0 = z0.
 *   - Jacobi preconditioner B = D^{-1}: Section 4.1 ("Jacobi (diagonal
 *     scaling) preconditioning").
 *   - Flexible CG, FCG(1) (Notay, SIAM J. Sci. Comput. 22, 2000; equivalently
 *     Golub & Ye 1999, Polak-Ribiere form): identical to PCG except
 *     beta = -(z_{k+1} . w_k) / (p_k . w_k).
 *   - Chebyshev polynomial preconditioner: z = sum_j c_j T_j(Y) D^{-1} r with
 *     Y = (2/lmax) D^{-1} A - I, evaluated by the forward three-term
 *     recurrence T_{j+1} = 2 Y T_j - T_{j-1}.
 *   - Gershgorin discs of D^{-1} A: centre 1, radius sum_{j!=i} |a_ij|/|a_ii|.
 *   - TFQMR (the paper's second benchmark method): Freund (1993), two
 *     products per iteration as in Saad (2nd ed., Section 7.4.3) and Kelley
 *     (1995, Section 3.6.3), left-preconditioned by D^{-1}.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Solve status bits (the oracle's own numbering). */
#define OR_CONVERGED 1
#define OR_MAXIT 2
#define OR_BREAKDOWN_PAP 4
#define OR_BREAKDOWN_RZ 8
#define OR_NAN 16
#define OR_STALL 32
#define OR_FALLBACK 64
#define OR_SETUP_ERROR 128

/* Preconditioner kinds and stopping-norm kinds. */
#define OR_PC_NONE 0
#define OR_PC_JACOBI 1
#define OR_NORM_UNPRECONDITIONED 0
#define OR_NORM_PRECONDITIONED 1

/* y = A x (row by row, each row summed in column-storage order). */
void or_spmv(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
             const double *x, double *y)
{
    for (int32_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) s += val[k] * x[col[k]];
        y[i] = s;
    }
}

/* x . y summed in index order. */
double or_dot(int64_t n, const double *x, const double *y)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += x[i] * y[i];
    return s;
}

/* Euclidean norm sqrt(x . x). */
double or_norm2(int64_t n, const double *x) { return sqrt(or_dot(n, x, x)); }

/* dinv_i = 1 / a_ii.  Returns 0, or -1 when a diagonal entry is missing or
 * not strictly positive (the Jacobi preconditioner is then undefined for an
 * SPD solve). */
int32_t or_jacobi_inverse(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                          double *dinv)
{
    for (int32_t i = 0; i < n; ++i) {
        double d = 0.0;
        int found = 0;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (col[k] == i) { d = val[k]; found = 1; }
        if (!found || !(d > 0.0)) return -1;
        dinv[i] = 1.0 / d;
    }
    return 0;
}

/* Gershgorin bounds of D^{-1} A: lo = min_i (1 - R_i), hi = max_i (1 + R_i). */
int32_t or_gershgorin(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                      double *lo, double *hi)
{
    double l = INFINITY, h = -INFINITY;
    for (int32_t i = 0; i < n; ++i) {
        double d = 0.0, off = 0.0;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            if (col[k] == i) d = val[k];
            else off += fabs(val[k]);
        }
        if (d == 0.0) return -1;
        double R = off / fabs(d);
        if (1.0 - R < l) l = 1.0 - R;
        if (1.0 + R > h) h = 1.0 + R;
    }
    *lo = l;
    *hi = h;
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Jacobi-PCG / CG                                                         */
/* ---------------------------------------------------------------------- */

/*
 * Solves A x = b from the initial guess held in x.  Returns the status bits.
 *
 *   pc         OR_PC_NONE or OR_PC_JACOBI
 *   norm_type  OR_NORM_UNPRECONDITIONED: stop when ||r_k|| <= rtol ||b||
 *              OR_NORM_PRECONDITIONED:   stop when ||z_k|| <= rtol ||B b||
 *   its        number of products A p (iterations) performed
 *   res, ref   final stopping norm and its reference (||b|| or ||B b||)
 *   alpha_hist, beta_hist (may be NULL): alpha_k, beta_k per iteration
 *   res_hist   (may be NULL): stopping norm after each iteration
 *   dir_hist   (may be NULL): the first ndir search directions p_0.. (n each)
 *
 * Iteration k (k = 1..maxit):
 *   w = A p; delta = p.w; stop with BREAKDOWN_PAP unless delta > 0
 *   alpha = rho / delta; x += alpha p; r -= alpha w
 *   z = B r; rho' = z.r; res = ||r|| (or ||z||)
 *   NAN if res or rho' is not finite; CONVERGED if res <= rtol ref
 *   BREAKDOWN_RZ unless rho' > 0
 *   beta = rho' / rho; rho = rho'; p = z + beta p
 */
int32_t or_pcg(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
               const double *b, double *x, double rtol, int32_t maxit, int32_t pc, int32_t norm_type,
               int32_t *its, double *res, double *ref, double *alpha_hist, double *beta_hist,
               double *res_hist, double *dir_hist, int32_t ndir)
{
    size_t nb = (size_t)(n > 0 ? n : 1) * sizeof(double);
    double *dinv = malloc(nb), *r = malloc(nb), *z = malloc(nb), *p = malloc(nb), *w = malloc(nb);
    int32_t status = 0, k = 0;
    *its = 0;
    *res = 0.0;
    *ref = 0.0;
    if (!dinv || !r || !z || !p || !w) { status = OR_SETUP_ERROR; goto done; }

    if (pc == OR_PC_JACOBI) {
        if (or_jacobi_inverse(n, rowptr, col, val, dinv) != 0) { status = OR_SETUP_ERROR; goto done; }
    } else {
        for (int32_t i = 0; i < n; ++i) dinv[i] = 1.0;
    }

    /* r0 = b - A x0; z0 = B r0 */
    or_spmv(n, rowptr, col, val, x, w);
    for (int32_t i = 0; i < n; ++i) r[i] = b[i] - w[i];
    for (int32_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];

    if (norm_type == OR_NORM_PRECONDITIONED) {
        double s = 0.0;
        for (int32_t i = 0; i < n; ++i) s += (dinv[i] * b[i]) * (dinv[i] * b[i]);
        *ref = sqrt(s);
        *res = or_norm2(n, z);
    } else {
        *ref = or_norm2(n, b);
        *res = or_norm2(n, r);
    }
    if (*ref == 0.0) {
        /* b = 0: the solution is x = 0 */
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        *res = 0.0;
        status = OR_CONVERGED;
        goto done;
    }
    if (!isfinite(*res) || !isfinite(*ref)) { status = OR_NAN; goto done; }
    if (*res <= rtol * *ref) { status = OR_CONVERGED; goto done; }

    double rho = or_dot(n, z, r);
    if (!(rho > 0.0)) { status = isfinite(rho) ? OR_BREAKDOWN_RZ : OR_NAN; goto done; }
    for (int32_t i = 0; i < n; ++i) p[i] = z[i];

    for (k = 1; k <= maxit; ++k) {
        if (dir_hist && k - 1 < ndir) memcpy(dir_hist + (size_t)(k - 1) * n, p, nb);
        or_spmv(n, rowptr, col, val, p, w);
        double delta = or_dot(n, p, w);
        if (!(delta > 0.0)) {
            status = isfinite(delta) ? OR_BREAKDOWN_PAP : OR_NAN;
            k -= 1;
            break;
        }
        double alpha = rho / delta;
        if (alpha_hist) alpha_hist[k - 1] = alpha;
        for (int32_t i = 0; i < n; ++i) x[i] += alpha * p[i];
        for (int32_t i = 0; i < n; ++i) r[i] -= alpha * w[i];
        for (int32_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
        double rho_new = or_dot(n, z, r);
        *res = (norm_type == OR_NORM_PRECONDITIONED) ? or_norm2(n, z) : or_norm2(n, r);
        if (res_hist) res_hist[k - 1] = *res;
        if (!isfinite(*res) || !isfinite(rho_new)) { status = OR_NAN; break; }
        if (*res <= rtol * *ref) { status = OR_CONVERGED; break; }
        if (!(rho_new > 0.0)) { status = OR_BREAKDOWN_RZ; break; }
        double beta = rho_new / rho;
        if (beta_hist) beta_hist[k - 1] = beta;
        rho = rho_new;
        for (int32_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    if (k > maxit) { k = maxit; status = OR_MAXIT; }
    *its = k;

done:
    free(dinv); free(r); free(z); free(p); free(w);
    return status;
}

/* ---------------------------------------------------------------------- */
/* Chebyshev polynomial preconditioner                                     */
/* ---------------------------------------------------------------------- */

/* out = Y u with Y = (2/lmax) D^{-1} A - I; tmp is scratch of length n. */
static void cheb_arg(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                     const double *dinv, double lmax, const double *u, double *out, double *tmp)
{
    or_spmv(n, rowptr, col, val, u, tmp);
    for (int32_t i = 0; i < n; ++i) out[i] = (2.0 / lmax) * (dinv[i] * tmp[i]) - u[i];
}

/*
 * z = P r = sum_{j=0..deg} c_j T_j(Y) v,  v = D^{-1} r,
 * Y = (2/lmax) D^{-1} A - I, by T_0 v = v, T_1 v = Y v,
 * T_{j+1} v = 2 Y T_j v - T_{j-1} v.  Uses deg products with A.
 */
int32_t or_poly_apply(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                      const double *dinv, double lmax, int32_t deg, const double *c,
                      const double *r, double *z)
{
    size_t m = (size_t)(n > 0 ? n : 1);
    double *tp = calloc(m, sizeof(double)), *tc = calloc(m, sizeof(double));
    double *tn = calloc(m, sizeof(double)), *tmp = calloc(m, sizeof(double));
    if (!tp || !tc || !tn || !tmp) { free(tp); free(tc); free(tn); free(tmp); return -1; }
    for (int32_t i = 0; i < n; ++i) tp[i] = dinv[i] * r[i];
    for (int32_t i = 0; i < n; ++i) z[i] = c[0] * tp[i];
    if (deg >= 1) {
        cheb_arg(n, rowptr, col, val, dinv, lmax, tp, tc, tmp);
        for (int32_t i = 0; i < n; ++i) z[i] += c[1] * tc[i];
    }
    for (int32_t j = 2; j <= deg; ++j) {
        cheb_arg(n, rowptr, col, val, dinv, lmax, tc, tn, tmp);
        for (int32_t i = 0; i < n; ++i) tn[i] = 2.0 * tn[i] - tp[i];
        for (int32_t i = 0; i < n; ++i) z[i] += c[j] * tn[i];
        double *t = tp; tp = tc; tc = tn; tn = t;
    }
    free(tp); free(tc); free(tn); free(tmp);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Flexible CG, FCG(1), with the polynomial preconditioner and a fallback  */
/* to Jacobi-PCG                                                           */
/* ---------------------------------------------------------------------- */

/*
 * Solves A x = b from x with z = P r (or_poly_apply).  Iteration k:
 *   w = A p; delta = p.w                       (BREAKDOWN_PAP unless > 0)
 *   alpha = rho / delta; x += alpha p; r -= alpha w; res = ||r||
 *   NAN if not finite; CONVERGED if res <= rtol ||b||
 *   z = P r; rho' = r.z; zeta = z.w            (BREAKDOWN_RZ unless rho' > 0)
 *   beta = -zeta / delta; rho = rho'; p = z + beta p
 *   stall: no new minimum of res during the last
 *          max(stall_min, stall_frac * k) iterations
 * With fallback != 0 a breakdown or stall restarts plain Jacobi-PCG from the
 * current x for the remaining iteration budget (FALLBACK is then set and the
 * iteration counts add up).  The stopping norm is the unpreconditioned one.
 * With precheck != 0, p(t) = sum_j c_j T_j(2t/lmax - 1) is evaluated first at
 * t = lmax q / 1023, q = 0..1023; a value <= 0 means the preconditioner is
 * not SPD on the spectrum's enclosure [0, lmax], which counts as a
 * BREAKDOWN_RZ before the first iteration.
 */
static int poly_positive(int32_t deg, const double *c, double lmax)
{
    for (int q = 0; q < 1024; ++q) {
        double y = 2.0 * (lmax * q / 1023.0) / lmax - 1.0;
        double t0 = 1.0, t1 = y, p = c[0];
        if (deg >= 1) p += c[1] * t1;
        for (int32_t j = 2; j <= deg; ++j) {
            double t2 = 2.0 * y * t1 - t0;
            p += c[j] * t2;
            t0 = t1;
            t1 = t2;
        }
        if (!(p > 0.0)) return 0;
    }
    return 1;
}

int32_t or_fcg_poly(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                    const double *b, double *x, double rtol, int32_t maxit, int32_t deg,
                    const double *c, double lmax, int32_t stall_min, double stall_frac,
                    int32_t fallback, int32_t precheck, int32_t *its, double *res, double *ref,
                    int32_t *fcg_its)
{
    size_t nb = (size_t)(n > 0 ? n : 1) * sizeof(double);
    double *dinv = malloc(nb), *r = malloc(nb), *z = malloc(nb), *p = malloc(nb), *w = malloc(nb);
    int32_t status = 0, k = 0, failed = 0;
    *its = 0;
    *fcg_its = 0;
    *res = 0.0;
    *ref = 0.0;
    if (!dinv || !r || !z || !p || !w) { status = OR_SETUP_ERROR; goto done; }
    if (or_jacobi_inverse(n, rowptr, col, val, dinv) != 0) { status = OR_SETUP_ERROR; goto done; }

    or_spmv(n, rowptr, col, val, x, w);
    for (int32_t i = 0; i < n; ++i) r[i] = b[i] - w[i];
    *ref = or_norm2(n, b);
    *res = or_norm2(n, r);
    if (*ref == 0.0) {
        for (int32_t i = 0; i < n; ++i) x[i] = 0.0;
        *res = 0.0;
        status = OR_CONVERGED;
        goto done;
    }
    if (!isfinite(*res) || !isfinite(*ref)) { status = OR_NAN; goto done; }
    if (*res <= rtol * *ref) { status = OR_CONVERGED; goto done; }
    double rho = 0.0;
    if (precheck && !poly_positive(deg, c, lmax)) {
        failed = OR_BREAKDOWN_RZ;
    } else {
        if (or_poly_apply(n, rowptr, col, val, dinv, lmax, deg, c, r, z) != 0) { status = OR_SETUP_ERROR; goto done; }
        rho = or_dot(n, r, z);
        if (!(rho > 0.0)) {
            if (!isfinite(rho)) { status = OR_NAN; goto done; }
            failed = OR_BREAKDOWN_RZ;
        }
    }
    for (int32_t i = 0; i < n; ++i) p[i] = z[i];
    double best = *res;
    int32_t best_k = 0;

    for (k = (failed ? 0 : 1); !failed && k <= maxit; ++k) {
        or_spmv(n, rowptr, col, val, p, w);
        double delta = or_dot(n, p, w);
        if (!(delta > 0.0)) {
            k -= 1;
            if (!isfinite(delta)) { status = OR_NAN; goto finish; }
            failed = OR_BREAKDOWN_PAP;
            break;
        }
        double alpha = rho / delta;
        for (int32_t i = 0; i < n; ++i) x[i] += alpha * p[i];
        for (int32_t i = 0; i < n; ++i) r[i] -= alpha * w[i];
        *res = or_norm2(n, r);
        if (!isfinite(*res)) { status = OR_NAN; goto finish; }
        if (*res <= rtol * *ref) { status = OR_CONVERGED; goto finish; }
        if (*res < best) { best = *res; best_k = k; }
        else {
            double win = stall_frac * (double)k;
            if (win < (double)stall_min) win = (double)stall_min;
            if ((double)(k - best_k) >= win) { failed = OR_STALL; break; }
        }
        or_poly_apply(n, rowptr, col, val, dinv, lmax, deg, c, r, z);
        double rho_new = or_dot(n, r, z);
        double zeta = or_dot(n, z, w);
        if (!isfinite(rho_new) || !isfinite(zeta)) { status = OR_NAN; goto finish; }
        if (!(rho_new > 0.0)) { failed = OR_BREAKDOWN_RZ; break; }
        double beta = -zeta / delta;
        rho = rho_new;
        for (int32_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    if (!failed) { k = maxit; status = OR_MAXIT; goto finish; }

    /* breakdown or stall */
    *fcg_its = k;
    if (!fallback) { status = failed; *its = k; goto done; }
    {
        int32_t its2 = 0;
        double res2 = 0.0, ref2 = 0.0;
        int32_t left = maxit - k;
        int32_t st2 = or_pcg(n, rowptr, col, val, b, x, rtol, left, OR_PC_JACOBI, OR_NORM_UNPRECONDITIONED,
                             &its2, &res2, &ref2, NULL, NULL, NULL, NULL, 0);
        *its = k + its2;
        *res = res2;
        status = st2 | OR_FALLBACK | failed;
    }
    goto done;

finish:
    *its = k;
    *fcg_its = k;
done:
    free(dinv); free(r); free(z); free(p); free(w);
    return status;
}

/* ---------------------------------------------------------------------- */
/* TFQMR                                                                   */
/* ---------------------------------------------------------------------- */

/*
 * Transpose-free QMR, the paper's second benchmark method (Section 4,
 * "Transpose-Free Quasi-Minimal Residual"; Freund, SIAM J. Sci. Comput. 14,
 * 1993), in the arrangement with two products per iteration (Saad, Iterative
 * Methods for Sparse Linear Systems, 2nd ed., Section 7.4.3; Kelley,
 * Iterative Methods for Linear and Nonlinear Equations, 1995, Section 3.6.3),
 * applied to the left-preconditioned system B A x = B b with B = D^{-1}
 * (pc = Jacobi, every a_ii nonzero) or B = I:
 *
 *   r0 = B (b - A x0);  w = y1 = r0;  u1 = B A y1;  v = u1;  d = 0
 *   tau = ref = ||r0||;  theta = eta = 0;  rho = r0 . r0
 *   iteration k = 1, 2, ...:
 *     sigma = r0 . v (0: breakdown);  alpha = rho / sigma
 *     y2 = y1 - alpha v;  u2 = B A y2
 *     half-steps j = 1, 2 (m = 2k - 2 + j) with (y, u) = (y1, u1), (y2, u2):
 *       w = w - alpha u
 *       d = y + (theta^2 eta / alpha) d
 *       theta = ||w|| / tau;  c = 1 / sqrt(1 + theta^2);  tau = tau theta c
 *       eta = c^2 alpha;  x = x + eta d
 *       converged when tau sqrt(m + 1) <= rtol ref
 *     rho' = r0 . w (0: breakdown);  beta = rho' / rho;  rho = rho'
 *     y1 = w + beta y2;  u1 = B A y1;  v = u1 + beta (u2 + beta v)
 *
 * tau sqrt(m + 1) bounds ||B (b - A x_m)|| (Freund's estimate); it is the
 * reported residual (*bound) and the tested one.  *its counts iterations k
 * (two products each), *halfsteps the last m.  tau_hist (optional, 2 maxit
 * doubles) receives tau after every half-step.  Returns the status bits.
 */
int32_t or_tfqmr(int32_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                 const double *b, double *x, int32_t x0_zero, double rtol, int32_t maxit, int32_t pc,
                 int32_t *its, int32_t *halfsteps, double *bound, double *ref_out, double *tau_hist)
{
    double *bd = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *r0 = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *w = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *y1 = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *y2 = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *u1 = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *u2 = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *v = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *d = malloc(sizeof(double) * (n > 0 ? n : 1));
    int32_t status = 0, k = 0, m = 0;
    double tau = 0.0, ref = 0.0;
    *its = 0;
    *halfsteps = 0;
    *bound = 0.0;
    *ref_out = 0.0;

    /* B = D^{-1}: every diagonal entry present and nonzero */
    for (int32_t i = 0; i < n; ++i) {
        if (pc == OR_PC_NONE) { bd[i] = 1.0; continue; }
        double a = 0.0;
        int found = 0;
        for (int32_t q = rowptr[i]; q < rowptr[i + 1]; ++q)
            if (col[q] == i) { a = val[q]; found = 1; }
        if (!found || a == 0.0 || !isfinite(a)) { status = OR_SETUP_ERROR; goto done; }
        bd[i] = 1.0 / a;
    }
    /* r0 = B (b - A x0) */
    if (x0_zero) {
        for (int32_t i = 0; i < n; ++i) { x[i] = 0.0; r0[i] = bd[i] * b[i]; }
    } else {
        or_spmv(n, rowptr, col, val, x, w);
        for (int32_t i = 0; i < n; ++i) r0[i] = bd[i] * (b[i] - w[i]);
    }
    ref = or_norm2(n, r0);
    *ref_out = ref;
    if (!isfinite(ref)) { status = OR_NAN; goto done; }
    if (ref == 0.0) { status = OR_CONVERGED; goto done; }
    if (maxit <= 0) { status = OR_MAXIT; *bound = ref; goto done; }
    for (int32_t i = 0; i < n; ++i) { w[i] = r0[i]; y1[i] = r0[i]; d[i] = 0.0; }
    or_spmv(n, rowptr, col, val, y1, u1);
    for (int32_t i = 0; i < n; ++i) { u1[i] *= bd[i]; v[i] = u1[i]; }
    tau = ref;
    double theta = 0.0, eta = 0.0, rho = or_dot(n, r0, r0);

    for (k = 1; k <= maxit; ++k) {
        const double sigma = or_dot(n, r0, v);
        if (!isfinite(sigma)) { status = OR_NAN; --k; goto finish; }
        if (sigma == 0.0) { status = OR_BREAKDOWN_PAP; --k; goto finish; }
        const double alpha = rho / sigma;
        for (int32_t i = 0; i < n; ++i) y2[i] = y1[i] - alpha * v[i];
        or_spmv(n, rowptr, col, val, y2, u2);
        for (int32_t i = 0; i < n; ++i) u2[i] *= bd[i];
        for (int j = 1; j <= 2; ++j) {
            const double *y = j == 1 ? y1 : y2, *u = j == 1 ? u1 : u2;
            m = 2 * k - 2 + j;
            const double f = theta * theta * eta / alpha;
            for (int32_t i = 0; i < n; ++i) {
                w[i] = w[i] - alpha * u[i];
                d[i] = y[i] + f * d[i];
            }
            theta = or_norm2(n, w) / tau;
            const double c = 1.0 / sqrt(1.0 + theta * theta);
            tau = tau * theta * c;
            eta = c * c * alpha;
            for (int32_t i = 0; i < n; ++i) x[i] = x[i] + eta * d[i];
            if (tau_hist) tau_hist[m - 1] = tau;
            *bound = tau * sqrt((double)m + 1.0);
            if (!isfinite(*bound)) { status = OR_NAN; goto finish; }
            if (*bound <= rtol * ref) { status = OR_CONVERGED; goto finish; }
        }
        const double rho_new = or_dot(n, r0, w);
        if (!isfinite(rho_new)) { status = OR_NAN; goto finish; }
        if (rho_new == 0.0) { status = OR_BREAKDOWN_RZ; goto finish; }
        const double beta = rho_new / rho;
        rho = rho_new;
        for (int32_t i = 0; i < n; ++i) y1[i] = w[i] + beta * y2[i];
        or_spmv(n, rowptr, col, val, y1, u1);
        for (int32_t i = 0; i < n; ++i) {
            u1[i] *= bd[i];
            v[i] = u1[i] + beta * (u2[i] + beta * v[i]);
        }
    }
    k = maxit;
    status = OR_MAXIT;
finish:
    *its = k;
    *halfsteps = m;
done:
    free(bd); free(r0); free(w); free(y1); free(y2); free(u1); free(u2); free(v); free(d);
    return status;
}
