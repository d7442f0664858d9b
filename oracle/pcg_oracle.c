/*
 * Oracle for the preconditioned conjugate-gradient solve -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, single-threaded FP64 C.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or constant with the GPU library and must be built with
 * -ffp-contract=off so that no multiply-add is fused.
 *
 * What it computes (paper, Section IV): the conjugate-gradient method of
 * Golub and Van Loan for a symmetric positive-definite matrix stored in CSR,
 * with a continue-condition that ends the loop early, at tolerance 1e-10
 * (Table I caption), with at most N iterations (the "132651 loop").  The
 * paper does not print the algorithm; the readings taken here are:
 *   - tolerance is on the unpreconditioned 2-norm  ||b - A x|| / ||b||;
 *   - x0 defaults to zero (the caller passes it in x);
 *   - preconditioner M = diag(A) (Jacobi) or M = I ("none", the paper's
 *     flop accounting);
 *   - when the recurrence residual passes the test, the true residual
 *     b - A x is computed; if it also passes the solve has converged,
 *     otherwise r is replaced by it and the iteration continues;
 *   - "iterations" counts products A p inside the loop;
 *   - breakdown (p'Ap <= 0, r'z <= 0, or a non-finite scalar) ends the
 *     solve with a status instead of a result: CG needs an SPD system.
 * Sums run sequentially from index 0 upward (or pairwise, as a second
 * rounding order for self-consistency checks); a CSR row is summed in
 * stored column order.
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

/* Built plainly, the oracle is single-threaded and these expand to nothing.
 * A second build with -fopenmp (used only to time the CPU on all its cores)
 * splits the row loop of the product and the element-wise loops across
 * threads, which leaves their results unchanged, and the sequential dot
 * product into per-thread partial sums, which changes its rounding order. */
#ifdef _OPENMP
#include <omp.h>
#define ORC_PAR _Pragma("omp parallel for schedule(static)")
#define ORC_PAR_SUM _Pragma("omp parallel for schedule(static) reduction(+:s)")
#else
#define ORC_PAR
#define ORC_PAR_SUM
#endif

/* Threads a solve uses: 1 in the plain build. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

#define ORC_CONVERGED 0
#define ORC_MAXIT 1
#define ORC_BREAKDOWN 2
#define ORC_EINVAL (-1)
#define ORC_EDIAG (-2)
#define ORC_ENOMEM (-3)

typedef struct {
    int iters;
    int status;
    int replacements;
    int pad;
    double relres_recur; /* ||r_k|| / ||b|| from the recurrence at exit */
    double relres_true;  /* ||b - A x|| / ||b|| for the returned x      */
} oracle_info;

/* y = A x, each row summed in stored column order. */
int oracle_spmv(int n, const int *rowptr, const int *col, const double *val,
                const double *x, double *y)
{
    if (n < 0 || !rowptr || !col || !val || !x || !y) return ORC_EINVAL;
    ORC_PAR
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) s += val[k] * x[col[k]];
        y[i] = s;
    }
    return 0;
}

static double sum_pairwise(const double *a, const double *b, size_t lo, size_t hi)
{
    if (hi - lo <= 8) {
        double s = 0.0;
        for (size_t i = lo; i < hi; ++i) s += a[i] * b[i];
        return s;
    }
    size_t mid = lo + (hi - lo) / 2;
    return sum_pairwise(a, b, lo, mid) + sum_pairwise(a, b, mid, hi);
}

/* a . b ; mode 0 = sequential from index 0, mode 1 = pairwise halving. */
double oracle_dot(int n, const double *a, const double *b, int mode)
{
    if (n <= 0) return 0.0;
    if (mode == 1) return sum_pairwise(a, b, 0, (size_t)n);
    double s = 0.0;
    ORC_PAR_SUM
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* r = b - A x ; returns ||r||_2 (sequential sum), or -1 on bad arguments. */
double oracle_residual(int n, const int *rowptr, const int *col, const double *val,
                       const double *b, const double *x, double *r)
{
    if (oracle_spmv(n, rowptr, col, val, x, r) != 0) return -1.0;
    ORC_PAR
    for (int i = 0; i < n; ++i) r[i] = b[i] - r[i];
    return sqrt(oracle_dot(n, r, r, 0));
}

static void snapshot(double *trace, int n, int k, const double *x, const double *r,
                     const double *z, const double *p)
{
    if (!trace) return;
    double *t = trace + (size_t)k * 4 * (size_t)n;
    memcpy(t, x, sizeof(double) * (size_t)n);
    memcpy(t + n, r, sizeof(double) * (size_t)n);
    if (z) memcpy(t + 2 * (size_t)n, z, sizeof(double) * (size_t)n);
    if (p) memcpy(t + 3 * (size_t)n, p, sizeof(double) * (size_t)n);
}

/*
 * Solve A x = b.  x holds x0 on entry and the result on exit.
 *   precond  : 0 = none (M = I), 1 = Jacobi (M = diag A)
 *   sum_mode : 0 = sequential dot products, 1 = pairwise
 *   maxit    : <= 0 means n
 *   hist     : optional, maxit+1 doubles: hist[0] = ||r_0||/||b||, hist[k] =
 *              recurrence ||r_k||/||b|| after iteration k (before any
 *              replacement)
 *   trace    : optional, (maxit+1) * 4n doubles: x_k, r_k, z_k, p_k after
 *              iteration k (z_k, p_k left untouched when the loop ends at k)
 */
int oracle_pcg(int n, const int *rowptr, const int *col, const double *val,
               const double *b, double *x, double tol, int maxit, int precond,
               int sum_mode, oracle_info *info, double *hist, double *trace)
{
    if (n <= 0 || !rowptr || !col || !val || !b || !x || !info || !(tol >= 0.0))
        return ORC_EINVAL;
    if (maxit <= 0) maxit = n;
    memset(info, 0, sizeof(*info));

    double *diag = malloc(sizeof(double) * (size_t)n);
    double *r = malloc(sizeof(double) * (size_t)n);
    double *z = malloc(sizeof(double) * (size_t)n);
    double *p = malloc(sizeof(double) * (size_t)n);
    double *q = malloc(sizeof(double) * (size_t)n);
    if (!diag || !r || !z || !p || !q) {
        free(diag); free(r); free(z); free(p); free(q);
        return ORC_ENOMEM;
    }
    int status = ORC_MAXIT;

    /* M = diag(A) for Jacobi; every diagonal entry must be present and > 0. */
    for (int i = 0; i < n; ++i) {
        diag[i] = 1.0;
        if (precond == 1) {
            double d = 0.0;
            int found = 0;
            for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
                if (col[k] == i) { d += val[k]; found = 1; }
            if (!found || !(d > 0.0)) { status = ORC_EDIAG; goto out; }
            diag[i] = d;
        }
    }

    double nb = sqrt(oracle_dot(n, b, b, sum_mode));
    if (nb == 0.0) {
        ORC_PAR
        for (int i = 0; i < n; ++i) x[i] = 0.0;
        info->relres_recur = 0.0;
        info->relres_true = 0.0;
        if (hist) hist[0] = 0.0;
        status = ORC_CONVERGED;
        goto out;
    }
    double thr = tol * nb;

    /* r0 = b - A x0 */
    oracle_spmv(n, rowptr, col, val, x, r);
    ORC_PAR
    for (int i = 0; i < n; ++i) r[i] = b[i] - r[i];
    double rn = sqrt(oracle_dot(n, r, r, sum_mode));
    if (hist) hist[0] = rn / nb;
    info->relres_recur = rn / nb;
    if (rn <= thr) {
        info->relres_true = rn / nb;
        snapshot(trace, n, 0, x, r, NULL, NULL);
        status = ORC_CONVERGED;
        goto out;
    }
    /* z0 = M^{-1} r0, p0 = z0, rho0 = r0' z0 */
    ORC_PAR
    for (int i = 0; i < n; ++i) z[i] = r[i] / diag[i];
    memcpy(p, z, sizeof(double) * (size_t)n);
    double rho = oracle_dot(n, r, z, sum_mode);
    snapshot(trace, n, 0, x, r, z, p);

    int k = 0;
    while (k < maxit) {
        oracle_spmv(n, rowptr, col, val, p, q);           /* q = A p       */
        double sigma = oracle_dot(n, p, q, sum_mode);       /* sigma = p'q   */
        if (!(sigma > 0.0) || !isfinite(sigma)) { status = ORC_BREAKDOWN; break; }
        double alpha = rho / sigma;
        ORC_PAR
        for (int i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
        ORC_PAR
        for (int i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
        ++k;
        rn = sqrt(oracle_dot(n, r, r, sum_mode));
        if (hist) hist[k] = rn / nb;
        info->relres_recur = rn / nb;
        if (rn <= thr) {                                    /* continue-condition */
            oracle_spmv(n, rowptr, col, val, x, q);
            ORC_PAR
            for (int i = 0; i < n; ++i) q[i] = b[i] - q[i];
            double tn = sqrt(oracle_dot(n, q, q, sum_mode));
            if (tn <= thr) {
                snapshot(trace, n, k, x, r, NULL, NULL);
                status = ORC_CONVERGED;
                break;
            }
            memcpy(r, q, sizeof(double) * (size_t)n);       /* residual replacement */
            info->replacements += 1;
        }
        ORC_PAR
        for (int i = 0; i < n; ++i) z[i] = r[i] / diag[i];
        double rho_new = oracle_dot(n, r, z, sum_mode);
        if (!(rho_new > 0.0) || !isfinite(rho_new)) {
            snapshot(trace, n, k, x, r, z, NULL);
            status = ORC_BREAKDOWN;
            break;
        }
        double beta = rho_new / rho;
        rho = rho_new;
        ORC_PAR
        for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        snapshot(trace, n, k, x, r, z, p);
    }
    info->iters = k;
    {
        /* Reported, not part of the method: the true residual of the returned x. */
        oracle_spmv(n, rowptr, col, val, x, q);
        ORC_PAR
        for (int i = 0; i < n; ++i) q[i] = b[i] - q[i];
        info->relres_true = sqrt(oracle_dot(n, q, q, sum_mode)) / nb;
    }

out:
    info->status = status;
    free(diag); free(r); free(z); free(p); free(q);
    return status;
}

/*
 * The same solve in the single-reduction form of Chronopoulos and Gear
 * (J. Comput. Appl. Math. 25, 1989): s = A p is carried by the recurrence
 * s = w + beta s with w = A u, u = M^{-1} r, so the iteration needs one
 * product, that of u.  In exact arithmetic the iterates are those of
 * oracle_pcg.  Stopping rules, statuses, history and trace follow oracle_pcg
 * (trace slots hold x, r, u, p).
 *
 * p'Ap is taken as sigma = p's, the inner product of the direction with the
 * recurred s.  (A parallel code obtains the same number from the one
 * reduction that yields r'u, because p's expands into inner products of u,
 * w, the previous p and the previous s.)  Chronopoulos and Gear's scalar
 * recurrence sigma = w'u - beta r'u / alpha is not used: it assumes that the
 * new residual is M^{-1}-orthogonal to the previous one, which a residual
 * replacement near the attainable accuracy destroys, and the recurred sigma
 * then turns negative for an SPD matrix.
 *
 * After a residual replacement the auxiliary vectors are recomputed as well
 * (the replacement strategy for this family of forms analysed by Cools,
 * Yetkin, Agullo, Giraud and Vanroose, SIAM J. Matrix Anal. Appl. 39, 2018):
 * w = A u for the replaced residual, and s = A p for the new direction.
 */
int oracle_pcg_sr(int n, const int *rowptr, const int *col, const double *val,
                  const double *b, double *x, double tol, int maxit, int precond,
                  int sum_mode, oracle_info *info, double *hist, double *trace)
{
    if (n <= 0 || !rowptr || !col || !val || !b || !x || !info || !(tol >= 0.0))
        return ORC_EINVAL;
    if (maxit <= 0) maxit = n;
    memset(info, 0, sizeof(*info));

    double *diag = malloc(sizeof(double) * (size_t)n);
    double *r = malloc(sizeof(double) * (size_t)n);
    double *u = malloc(sizeof(double) * (size_t)n);
    double *w = malloc(sizeof(double) * (size_t)n);
    double *p = malloc(sizeof(double) * (size_t)n);
    double *sv = malloc(sizeof(double) * (size_t)n);
    double *t = malloc(sizeof(double) * (size_t)n);
    if (!diag || !r || !u || !w || !p || !sv || !t) {
        free(diag); free(r); free(u); free(w); free(p); free(sv); free(t);
        return ORC_ENOMEM;
    }
    int status = ORC_MAXIT;
    for (int i = 0; i < n; ++i) {
        diag[i] = 1.0;
        if (precond == 1) {
            double d = 0.0;
            int found = 0;
            for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
                if (col[k] == i) { d += val[k]; found = 1; }
            if (!found || !(d > 0.0)) { status = ORC_EDIAG; goto out; }
            diag[i] = d;
        }
    }

    double nb = sqrt(oracle_dot(n, b, b, sum_mode));
    if (nb == 0.0) {
        ORC_PAR
        for (int i = 0; i < n; ++i) x[i] = 0.0;
        if (hist) hist[0] = 0.0;
        status = ORC_CONVERGED;
        goto out;
    }
    double thr = tol * nb;
    oracle_spmv(n, rowptr, col, val, x, r);
    ORC_PAR
    for (int i = 0; i < n; ++i) r[i] = b[i] - r[i];
    double rn = sqrt(oracle_dot(n, r, r, sum_mode));
    if (hist) hist[0] = rn / nb;
    info->relres_recur = rn / nb;
    if (rn <= thr) {
        info->relres_true = rn / nb;
        snapshot(trace, n, 0, x, r, NULL, NULL);
        status = ORC_CONVERGED;
        goto out;
    }
    /* u0 = M^{-1} r0, w0 = A u0, p0 = u0, s0 = w0, sigma0 = p0's0 */
    ORC_PAR
    for (int i = 0; i < n; ++i) u[i] = r[i] / diag[i];
    oracle_spmv(n, rowptr, col, val, u, w);
    double gamma = oracle_dot(n, r, u, sum_mode);
    memcpy(p, u, sizeof(double) * (size_t)n);
    memcpy(sv, w, sizeof(double) * (size_t)n);
    double sigma = oracle_dot(n, p, sv, sum_mode);
    snapshot(trace, n, 0, x, r, u, p);

    int k = 0, replaced = 0;
    while (k < maxit) {
        if (!(sigma > 0.0) || !isfinite(sigma)) { status = ORC_BREAKDOWN; break; }
        double alpha = gamma / sigma;
        ORC_PAR
        for (int i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
        ORC_PAR
        for (int i = 0; i < n; ++i) r[i] = r[i] - alpha * sv[i];
        ++k;
        rn = sqrt(oracle_dot(n, r, r, sum_mode));
        if (hist) hist[k] = rn / nb;
        info->relres_recur = rn / nb;
        if (rn <= thr) {                                    /* continue-condition */
            oracle_spmv(n, rowptr, col, val, x, t);
            ORC_PAR
            for (int i = 0; i < n; ++i) t[i] = b[i] - t[i];
            double tn = sqrt(oracle_dot(n, t, t, sum_mode));
            if (tn <= thr) {
                snapshot(trace, n, k, x, r, NULL, NULL);
                status = ORC_CONVERGED;
                break;
            }
            memcpy(r, t, sizeof(double) * (size_t)n);       /* residual replacement */
            info->replacements += 1;
            replaced = 1;
        }
        ORC_PAR
        for (int i = 0; i < n; ++i) u[i] = r[i] / diag[i];
        oracle_spmv(n, rowptr, col, val, u, w);             /* w = A u */
        double gamma_new = oracle_dot(n, r, u, sum_mode);
        if (!(gamma_new > 0.0) || !isfinite(gamma_new)) {
            snapshot(trace, n, k, x, r, u, NULL);
            status = ORC_BREAKDOWN;
            break;
        }
        double beta = gamma_new / gamma;
        gamma = gamma_new;
        ORC_PAR
        for (int i = 0; i < n; ++i) p[i] = u[i] + beta * p[i];
        if (replaced) {
            oracle_spmv(n, rowptr, col, val, p, sv);        /* s = A p, recomputed */
            replaced = 0;
        } else {
            ORC_PAR
            for (int i = 0; i < n; ++i) sv[i] = w[i] + beta * sv[i];
        }
        sigma = oracle_dot(n, p, sv, sum_mode);             /* sigma = p's */
        snapshot(trace, n, k, x, r, u, p);
    }
    info->iters = k;
    oracle_spmv(n, rowptr, col, val, x, t);
    ORC_PAR
    for (int i = 0; i < n; ++i) t[i] = b[i] - t[i];
    info->relres_true = sqrt(oracle_dot(n, t, t, sum_mode)) / nb;

out:
    info->status = status;
    free(diag); free(r); free(u); free(w); free(p); free(sv); free(t);
    return status;
}

/*
 * The same Jacobi-PCG solve with the FP32 matrix stream: the products inside
 * the loop use the values rounded to single precision, in the row-sum-
 * preserving evaluation
 *     y_i = sum_k fl32(a_ik) (x[col_k] - x_i) + s_i x_i,   s_i = sum_k a_ik,
 * (s_i summed in double, in stored order; the terms added in stored order),
 * with every vector, dot product and scalar in double.  Reliable updates
 * (Sleijpen and van der Vorst): besides the ordinary continue-condition, the
 * true residual b - A x with the double values is formed whenever ||r|| has
 * fallen to `drop` times its value after the last replacement (drop > 0), and
 * either confirms convergence or replaces r.  Statuses and info as
 * oracle_pcg; replacements counts every replaced residual.
 */
static void spmv_f32_rowsum(int n, const int *rowptr, const int *col, const double *v32, const double *s64,
                            const double *x, double *y)
{
    ORC_PAR
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) s += v32[k] * (x[col[k]] - x[i]);
        y[i] = s + s64[i] * x[i];
    }
}

int oracle_pcg_m32(int n, const int *rowptr, const int *col, const double *val,
                   const double *b, double *x, double tol, int maxit, int precond,
                   double drop, oracle_info *info)
{
    if (n <= 0 || !rowptr || !col || !val || !b || !x || !info || !(tol >= 0.0) || !(drop >= 0.0))
        return ORC_EINVAL;
    if (maxit <= 0) maxit = n;
    memset(info, 0, sizeof(*info));
    const int nnz = rowptr[n];
    double *diag = malloc(sizeof(double) * (size_t)n);
    double *r = malloc(sizeof(double) * (size_t)n);
    double *z = malloc(sizeof(double) * (size_t)n);
    double *p = malloc(sizeof(double) * (size_t)n);
    double *q = malloc(sizeof(double) * (size_t)n);
    double *s64 = malloc(sizeof(double) * (size_t)n);
    double *v32 = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    if (!diag || !r || !z || !p || !q || !s64 || !v32) {
        free(diag); free(r); free(z); free(p); free(q); free(s64); free(v32);
        return ORC_ENOMEM;
    }
    int status = ORC_MAXIT;
    for (int k = 0; k < nnz; ++k) v32[k] = (double)(float)val[k];
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) s += val[k];
        s64[i] = s;
        diag[i] = 1.0;
        if (precond == 1) {
            double d = 0.0;
            int found = 0;
            for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
                if (col[k] == i) { d += val[k]; found = 1; }
            if (!found || !(d > 0.0)) { status = ORC_EDIAG; goto out; }
            diag[i] = d;
        }
    }
    double nb = sqrt(oracle_dot(n, b, b, 0));
    if (nb == 0.0) {
        for (int i = 0; i < n; ++i) x[i] = 0.0;
        status = ORC_CONVERGED;
        goto out;
    }
    double thr = tol * nb;
    oracle_spmv(n, rowptr, col, val, x, r);                 /* r0 = b - A x0 with the double values */
    for (int i = 0; i < n; ++i) r[i] = b[i] - r[i];
    double rn = sqrt(oracle_dot(n, r, r, 0));
    info->relres_recur = rn / nb;
    if (rn <= thr) {
        info->relres_true = rn / nb;
        status = ORC_CONVERGED;
        goto out;
    }
    for (int i = 0; i < n; ++i) z[i] = r[i] / diag[i];
    memcpy(p, z, sizeof(double) * (size_t)n);
    double rho = oracle_dot(n, r, z, 0);
    double rref = rn;                                         /* ||r|| after the last replacement */
    int k = 0;
    while (k < maxit) {
        spmv_f32_rowsum(n, rowptr, col, v32, s64, p, q);   /* q = A~ p */
        double sigma = oracle_dot(n, p, q, 0);
        if (!(sigma > 0.0) || !isfinite(sigma)) { status = ORC_BREAKDOWN; break; }
        double alpha = rho / sigma;
        for (int i = 0; i < n; ++i) x[i] = x[i] + alpha * p[i];
        for (int i = 0; i < n; ++i) r[i] = r[i] - alpha * q[i];
        ++k;
        rn = sqrt(oracle_dot(n, r, r, 0));
        info->relres_recur = rn / nb;
        if (rn <= thr || rn <= drop * rref) {
            oracle_spmv(n, rowptr, col, val, x, q);        /* true residual, double values */
            for (int i = 0; i < n; ++i) q[i] = b[i] - q[i];
            double tn = sqrt(oracle_dot(n, q, q, 0));
            if (tn <= thr) { status = ORC_CONVERGED; break; }
            memcpy(r, q, sizeof(double) * (size_t)n);       /* residual replacement */
            info->replacements += 1;
            rref = tn;
        }
        for (int i = 0; i < n; ++i) z[i] = r[i] / diag[i];
        double rho_new = oracle_dot(n, r, z, 0);
        if (!(rho_new > 0.0) || !isfinite(rho_new)) { status = ORC_BREAKDOWN; break; }
        double beta = rho_new / rho;
        rho = rho_new;
        for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    }
    info->iters = k;
    oracle_spmv(n, rowptr, col, val, x, q);
    for (int i = 0; i < n; ++i) q[i] = b[i] - q[i];
    info->relres_true = sqrt(oracle_dot(n, q, q, 0)) / nb;
out:
    info->status = status;
    free(diag); free(r); free(z); free(p); free(q); free(s64); free(v32);
    return status;
}
