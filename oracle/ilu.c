/*
 * Oracle (test infrastructure only): plain level-based incomplete LU of one
 * sparse matrix in CSR form, in FP64.
 *
 * These are the incomplete factorisations the paper uses as inexact local
 * solvers (Sec. V-B, "Incomplete Local Solver"; ILU(k) in Sec. VII-C):
 * L unit lower triangular and U upper triangular on a prescribed pattern,
 * rows taken in the matrix's own order (the paper keeps the original
 * ordering for ILU, Table IV discussion).
 *
 * oracle_iluk_pattern: the level-of-fill pattern of ILU(p).  Entries of A
 * have level 0; eliminating row k from row i creates (i, j) for j > k in
 * row k with level lev(i,k) + lev(k,j) + 1, the smallest level over all
 * such k is kept, and only entries of level <= p are part of the pattern.
 *
 * oracle_ilu0 (named for its first use; it factors on whatever pattern it
 * is given, so with the ILU(p) pattern and zero fill values it computes
 * ILU(p)): row-by-row ("IKJ") form: for row i and each k < i in its
 * pattern, in ascending order, l_ik = a_ik / u_kk, then a_ij -= l_ik * u_kj
 * for every j > k that lies in both row i and row k.
 *
 * Only the test suite, the smoke check and the CPU timing leg of the
 * benchmark may load this file's library.
 */
#include <limits.h>
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

/* Level-of-fill pattern of ILU(p) for a matrix with sorted rows that all hold
 * their diagonal.  Writes out_rowptr[n+1], out_col[nnz], out_lev[nnz] (rows
 * sorted) and returns nnz; if a row does not fit in cap entries it stops
 * there (the rows after it would read the rows not stored) and returns
 * -(a larger capacity to try: at least the entries up to that row, at least
 * twice cap); -2 on allocation failure. */
int64_t oracle_iluk_pattern(int64_t n, const int64_t *rowptr, const int32_t *col, int p,
                            int64_t *out_rowptr, int32_t *out_col, int32_t *out_lev, int64_t cap)
{
    /* row i is kept as a sorted linked list of its columns: nxt[c] is the
     * next column after c, n terminates the list */
    int64_t *nxt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t *lev = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!nxt || !lev) { free(nxt); free(lev); return -2; }
    for (int64_t c = 0; c < n; ++c) lev[c] = INT_MAX;
    int64_t nnz = 0;
    out_rowptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t head = n;
        /* the pattern of A's row i, level 0 (built back to front) */
        for (int64_t q = rowptr[i + 1] - 1; q >= rowptr[i]; --q) {
            nxt[col[q]] = head;
            head = col[q];
            lev[col[q]] = 0;
        }
        for (int64_t k = head; k < i; k = nxt[k]) {
            /* eliminate row k (its final pattern is known: k < i) */
            int64_t prev = k;
            for (int64_t q = out_rowptr[k]; q < out_rowptr[k + 1]; ++q) {
                const int64_t j = out_col[q];
                if (j <= k) continue;
                const int64_t nl = (int64_t)lev[k] + out_lev[q] + 1;
                if (nl > p) continue;
                if (lev[j] == INT_MAX) {
                    /* insert j after prev (columns of row k ascend, so the
                     * search resumes where the last one stopped) */
                    while (nxt[prev] < j) prev = nxt[prev];
                    nxt[j] = nxt[prev];
                    nxt[prev] = j;
                    lev[j] = (int32_t)nl;
                } else if (nl < lev[j]) {
                    lev[j] = (int32_t)nl;
                }
                if (j > prev) prev = j;
            }
        }
        int64_t len = 0;
        for (int64_t c = head; c < n; c = nxt[c]) ++len;
        if (nnz + len > cap) {
            const int64_t need = nnz + len > 2 * cap ? nnz + len : 2 * cap;
            free(nxt);
            free(lev);
            return -need;
        }
        for (int64_t c = head; c < n; c = nxt[c]) {
            out_col[nnz] = (int32_t)c;
            out_lev[nnz] = lev[c];
            ++nnz;
            lev[c] = INT_MAX;
        }
        out_rowptr[i + 1] = nnz;
    }
    free(nxt);
    free(lev);
    return nnz;
}
