/*
 * Oracle (test infrastructure only): plain incomplete LU with zero fill,
 * ILU(0), of one sparse matrix in CSR form, computed in place in FP64.
 *
 * This is the level-0 incomplete factorisation the paper uses as an inexact
 * local solver (Sec. V-B, "Incomplete Local Solver"): the factors keep exactly
 * the sparsity pattern of the input, L unit lower triangular, U upper
 * triangular.  The rows are taken in the matrix's own order (the paper keeps
 * the original ordering for ILU, Table IV discussion).
 *
 * Row-by-row ("IKJ") form: for row i and each k < i in its pattern, in
 * ascending order, l_ik = a_ik / u_kk, then a_ij -= l_ik * u_kj for every
 * j > k that lies in both row i and row k.
 *
 * Only the test suite, the smoke check and the CPU timing leg of the
 * benchmark may load this file's library.
 */
#include <stdint.h>
#include <stdlib.h>

/* Returns 0 on success, 1 + row index of the first zero pivot, or -1 if a
 * row has no diagonal entry.  Column indices of each row must be sorted. */
int oracle_ilu0(int64_t n, const int64_t *rowptr, const int32_t *col, double *val)
{
    int64_t *where = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *diag = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!where || !diag) { free(where); free(diag); return -2; }
    for (int64_t j = 0; j < n; ++j) { where[j] = -1; diag[j] = -1; }
    int rc = 0;
    for (int64_t i = 0; i < n && rc == 0; ++i) {
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            where[col[p]] = p;
            if (col[p] == i) diag[i] = p;
        }
        if (diag[i] < 0) { rc = -1; }
        for (int64_t p = rowptr[i]; p < rowptr[i + 1] && rc == 0; ++p) {
            int64_t k = col[p];
            if (k >= i) break;
            double lik = val[p] / val[diag[k]];
            val[p] = lik;
            for (int64_t q = diag[k] + 1; q < rowptr[k + 1]; ++q) {
                int64_t pos = where[col[q]];
                if (pos >= 0) val[pos] -= lik * val[q];
            }
        }
        if (rc == 0 && val[diag[i]] == 0.0) rc = (int)(1 + i);
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) where[col[p]] = -1;
    }
    free(where);
    free(diag);
    return rc;
}
