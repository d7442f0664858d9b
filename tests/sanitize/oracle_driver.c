/* Runs the oracle's C solvers on small systems under AddressSanitizer and
 * UndefinedBehaviorSanitizer (built by tests/test_sanitizers.py).  The oracle
 * source is included whole so that its types and constants are the ones it
 * defines.  Exit status: the number of failed checks. */
#include "pcg_oracle.c"

#include <stdio.h>

/* 5-point Laplacian plus c times the identity on an m x m grid, CSR with
 * columns in ascending order. */
static int lap2d(int m, double c, int **rowptr, int **col, double **val)
{
    const int n = m * m;
    *rowptr = malloc(sizeof(int) * (size_t)(n + 1));
    *col = malloc(sizeof(int) * (size_t)(5 * n));
    *val = malloc(sizeof(double) * (size_t)(5 * n));
    int k = 0;
    for (int i = 0; i < n; ++i) {
        const int y = i / m, x = i % m;
        (*rowptr)[i] = k;
        const int nb[5] = {y > 0 ? i - m : -1, x > 0 ? i - 1 : -1, i, x < m - 1 ? i + 1 : -1,
                           y < m - 1 ? i + m : -1};
        for (int t = 0; t < 5; ++t) {
            if (nb[t] < 0) continue;
            (*col)[k] = nb[t];
            (*val)[k] = nb[t] == i ? 4.0 + c : -1.0;
            ++k;
        }
    }
    (*rowptr)[n] = k;
    return n;
}

static int check(int cond, const char *what, int m)
{
    if (!cond) printf("FAIL %s (m = %d)\n", what, m);
    return cond ? 0 : 1;
}

int main(void)
{
    int fails = 0;
    const int sizes[3] = {1, 2, 16};
    for (int s = 0; s < 3; ++s) {
        const int m = sizes[s];
        int *rp, *ci;
        double *v;
        const int n = lap2d(m, 1e-2, &rp, &ci, &v);
        double *xs = malloc(sizeof(double) * (size_t)n), *b = malloc(sizeof(double) * (size_t)n);
        double *x = malloc(sizeof(double) * (size_t)n), *hist = malloc(sizeof(double) * (size_t)(n + 1));
        for (int i = 0; i < n; ++i) xs[i] = 1.0 + 0.25 * (double)(i % 7);
        fails += check(oracle_spmv(n, rp, ci, v, xs, b) == 0, "spmv", m);
        for (int pc = 0; pc < 2; ++pc)
            for (int mode = 0; mode < 2; ++mode) {
                oracle_info info;
                memset(x, 0, sizeof(double) * (size_t)n);
                int rc = oracle_pcg(n, rp, ci, v, b, x, 1e-10, 0, pc, mode, &info, hist, NULL);
                fails += check(rc == 0 && info.status == ORC_CONVERGED && info.relres_true <= 1e-10, "pcg", m);
                memset(x, 0, sizeof(double) * (size_t)n);
                rc = oracle_pcg_sr(n, rp, ci, v, b, x, 1e-10, 0, pc, mode, &info, hist, NULL);
                fails += check(rc == 0 && info.status == ORC_CONVERGED && info.relres_true <= 1e-10, "pcg_sr", m);
            }
        oracle_info info;
        memset(x, 0, sizeof(double) * (size_t)n);
        int rc = oracle_pcg_m32(n, rp, ci, v, b, x, 1e-10, 0, 1, 1e-2, &info);
        fails += check(rc == 0 && info.status == ORC_CONVERGED && info.relres_true <= 1e-10, "pcg_m32", m);
        fails += check(oracle_dot(n, xs, xs, 0) > 0.0 && oracle_dot(n, xs, xs, 1) > 0.0, "dot", m);
        /* Rejected inputs and a zero diagonal. */
        fails += check(oracle_pcg(0, rp, ci, v, b, x, 1e-10, 0, 1, 0, &info, NULL, NULL) == ORC_EINVAL, "n = 0", m);
        fails += check(oracle_pcg(n, rp, ci, v, NULL, x, 1e-10, 0, 1, 0, &info, NULL, NULL) == ORC_EINVAL, "b = NULL",
                       m);
        v[rp[0]] = 0.0;  /* row 0's first entry is its diagonal when y = 0 and x = 0 */
        memset(x, 0, sizeof(double) * (size_t)n);
        fails += check(oracle_pcg(n, rp, ci, v, b, x, 1e-10, 0, 1, 0, &info, NULL, NULL) == ORC_EDIAG, "zero diagonal",
                       m);
        free(rp); free(ci); free(v); free(xs); free(b); free(x); free(hist);
    }
    printf("oracle driver: %d failed checks\n", fails);
    return fails;
}
