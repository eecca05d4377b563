/*
 * Oracle numeric core: plain right-looking sparse LU on the filled pattern S.
 *
 * TEST INFRASTRUCTURE ONLY.  Compiled with gcc, loaded by the oracle's Python
 * wrapper; the product library neither links nor calls it.
 *
 * What it computes (the scalar form of the right-looking blocked LU of
 * Algorithm 1, Section 2.2, with every block of size 1): for the permuted
 * matrix A' = A[perm][:, perm], the unique LU factorization without row
 * exchanges, A' = L U with L unit lower triangular, stored on the symmetric
 * filled pattern S (entries of S that A' lacks start at 0.0).  For
 * k = 0 .. n-1:
 *     fail if a_kk is zero or not finite;
 *     a_ik <- a_ik / a_kk               for i in L(k)   (fp64 division)
 *     a_ij <- a_ij - a_ik * a_kj        for i in L(k), j in U(k).
 * The paper never mentions pivoting and credits stability to the reordering
 * phase (Section 1); diagonal pivots are used as they come.
 *
 * Storage: S's lower triangle in CSC, diagonal first in every column,
 * rows sorted.  For entry e of column k at row r:
 *     lval[e] = L(r, k)  (r > k),   lval[colptr[k]] = U(k, k),
 *     uval[e] = U(k, r)  (r > k)    (the mirror entry of the upper triangle).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

/* position of row r in column c, or -1 */
static int64_t find_row(const int64_t *colptr, const int32_t *rowidx, int64_t c, int64_t r) {
    int64_t lo = colptr[c], hi = colptr[c + 1] - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        int64_t v = rowidx[mid];
        if (v == r) return mid;
        if (v < r) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* Place A's values (CSR of the original matrix) on S.  inv[old] = new.
 * Returns 0, or -1 if an entry of A is missing from S. */
int oracle_scatter(int64_t n, const int64_t *rowptr, const int32_t *colidx, const double *vals,
                   const int32_t *inv, const int64_t *colptr, const int32_t *rowidx,
                   double *lval, double *uval) {
    int64_t nnzS = colptr[n];
    for (int64_t e = 0; e < nnzS; ++e) { lval[e] = 0.0; uval[e] = 0.0; }
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
            int64_t r = inv[i], c = inv[colidx[q]];
            if (r >= c) {
                int64_t e = find_row(colptr, rowidx, c, r);
                if (e < 0) return -1;
                lval[e] += vals[q];
            } else {
                int64_t e = find_row(colptr, rowidx, r, c);
                if (e < 0) return -1;
                uval[e] += vals[q];
            }
        }
    }
    return 0;
}

/* Right-looking elimination of columns 0 .. kmax-1.  Returns 0 on success,
 * 1 + k for the first zero / non-finite pivot k, -2 if S is not closed under
 * fill (a caller error). */
int64_t oracle_factor(int64_t n, int64_t kmax, const int64_t *colptr, const int32_t *rowidx,
                      double *lval, double *uval) {
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!pos) return -1;
    for (int64_t i = 0; i < n; ++i) pos[i] = -1;
    if (kmax > n) kmax = n;
    for (int64_t k = 0; k < kmax; ++k) {
        int64_t d = colptr[k];
        double piv = lval[d];
        if (piv == 0.0 || !isfinite(piv)) { free(pos); return 1 + k; }
        for (int64_t e = d + 1; e < colptr[k + 1]; ++e) lval[e] = lval[e] / piv;
        /* m runs over L(k) == U(k) (S is symmetric) */
        for (int64_t em = d + 1; em < colptr[k + 1]; ++em) {
            int64_t m = rowidx[em];
            double lmk = lval[em];   /* L(m, k) */
            double ukm = uval[em];   /* U(k, m) */
            for (int64_t q = colptr[m]; q < colptr[m + 1]; ++q) pos[rowidx[q]] = q;
            /* column m of L: rows i > m with i in L(k) */
            /* row m of U: columns j > m with j in U(k) */
            for (int64_t e = em + 1; e < colptr[k + 1]; ++e) {
                int64_t i = rowidx[e];
                int64_t q = pos[i];
                /* (i, m) is in S: both are neighbours of k in S and k < min(i, m) */
                if (q < 0) { free(pos); return -2; }
                lval[q] -= lval[e] * ukm;   /* a_im -= l_ik * u_km */
                uval[q] -= lmk * uval[e];   /* a_mi -= l_mk * u_ki */
            }
            lval[colptr[m]] -= lmk * ukm;  /* diagonal a_mm */
            for (int64_t q = colptr[m]; q < colptr[m + 1]; ++q) pos[rowidx[q]] = -1;
        }
    }
    free(pos);
    return 0;
}

/* Solve on the permuted system, in place on x (n x nrhs, column-major, ld).
 * trans = 0:  x <- U^{-1} L^{-1} x ;  trans = 1:  x <- L^{-T} U^{-T} x. */
void oracle_solve(int64_t n, const int64_t *colptr, const int32_t *rowidx,
                  const double *lval, const double *uval, double *x, int64_t nrhs,
                  int64_t ld, int trans) {
    for (int64_t c = 0; c < nrhs; ++c) {
        double *v = x + c * ld;
        if (!trans) {
            for (int64_t k = 0; k < n; ++k) {          /* L y = x, by columns */
                double yk = v[k];
                for (int64_t e = colptr[k] + 1; e < colptr[k + 1]; ++e) v[rowidx[e]] -= lval[e] * yk;
            }
            for (int64_t k = n - 1; k >= 0; --k) {     /* U x = y, by rows */
                double s = v[k];
                for (int64_t e = colptr[k] + 1; e < colptr[k + 1]; ++e) s -= uval[e] * v[rowidx[e]];
                v[k] = s / lval[colptr[k]];
            }
        } else {
            for (int64_t k = 0; k < n; ++k) {          /* U^T z = x, by columns of U^T */
                double zk = v[k] / lval[colptr[k]];
                v[k] = zk;
                for (int64_t e = colptr[k] + 1; e < colptr[k + 1]; ++e) v[rowidx[e]] -= uval[e] * zk;
            }
            for (int64_t k = n - 1; k >= 0; --k) {     /* L^T w = z, by rows of L^T */
                double s = v[k];
                for (int64_t e = colptr[k] + 1; e < colptr[k + 1]; ++e) s -= lval[e] * v[rowidx[e]];
                v[k] = s;
            }
        }
    }
}
