/*
 * FP64 CPU oracle for the local FusedMM path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load or call this library.  The GPU library never links, includes or calls it,
 * and it shares no code with the GPU kernels.
 *
 * Every routine is the plain definition from the paper, written as loops in
 * double precision, over a canonical CSR pattern (int32 rowptr[m+1], int32
 * colidx[nnz], columns of a row strictly increasing):
 *
 *   SDDMM(A, B, S) = S * (A . B^T)      Section II, Eq. (1); per-entry form in
 *                                         Section IV-A: R_ij = S_ij <A_i:, B_j:>,
 *                                         only at stored entries of S.
 *   SpMMA(S, B)    = S . B              Section II (m x r output).
 *   SpMMB(S, A)    = S^T . A            Section II (n x r output).
 *   transpose      CSR -> CSC           Section IV-B: FusedMMB runs on a stored
 *                                         transposed copy of S.
 *
 * FusedMMA / FusedMMB and the adjoints are compositions of these, assembled in
 * the Python wrapper next to this file.
 *
 * Summation order: the dot product runs over k ascending, the SpMM sums over the
 * stored entries of a row in ascending position order.  Rows are independent,
 * so the row loops are split across OpenMP threads without changing any sum.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no FMA contraction,
 * so every product and sum is rounded once, as written).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* Rows to visit: rows[t] for t < nrows, or every row 0..m-1 when rows == NULL. */
static inline int64_t pick_row(const int64_t *rows, int64_t t) { return rows ? rows[t] : t; }

/*
 * SDDMM (Eq. (1)): for every stored entry p = (i, j) of the visited rows,
 *   R[p] = val[p] * sum_{k<r} A[i,k] * B[j,k].
 * val == NULL means every stored value is 1 (the pattern alone).
 * R is indexed by CSR position; entries of rows that are not visited are left as they are.
 */
void oracle_sddmm(int64_t m, int64_t r, const int32_t *rowptr, const int32_t *colidx,
                  const double *val, const double *A, const double *B, double *R,
                  const int64_t *rows, int64_t nrows)
{
    int64_t count = rows ? nrows : m;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < count; ++t) {
        int64_t i = pick_row(rows, t);
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int64_t j = colidx[p];
            double dot = 0.0;
            for (int64_t k = 0; k < r; ++k)
                dot += A[i * r + k] * B[j * r + k];
            R[p] = (val ? val[p] : 1.0) * dot;
        }
    }
}

/*
 * SpMMA (Section II): C = W . B, with W the sparse matrix whose stored values are w
 * (CSR order).  Row t of C (t-th visited row i) is
 *   C[t,:] = sum over stored p of row i, ascending, of w[p] * B[colidx[p], :].
 * C has one r-vector per visited row and is overwritten.
 */
void oracle_spmm_a(int64_t m, int64_t r, const int32_t *rowptr, const int32_t *colidx,
                   const double *w, const double *B, double *C,
                   const int64_t *rows, int64_t nrows)
{
    int64_t count = rows ? nrows : m;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < count; ++t) {
        int64_t i = pick_row(rows, t);
        double *c = C + t * r;
        for (int64_t k = 0; k < r; ++k) c[k] = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            const double *b = B + (int64_t)colidx[p] * r;
            double s = w[p];
            for (int64_t k = 0; k < r; ++k)
                c[k] += s * b[k];
        }
    }
}

/*
 * SpMMB (Section II): C = W^T . A, an n x r output.  Written as the scatter
 * C[j,:] += w[p] * A[i,:] over the stored entries in CSR order, which is the
 * definition of the transposed product without forming W^T.  Sequential, so every
 * column receives its terms in ascending row order.
 */
void oracle_spmm_b(int64_t m, int64_t n, int64_t r, const int32_t *rowptr, const int32_t *colidx,
                   const double *w, const double *A, double *C)
{
    memset(C, 0, (size_t)(n * r) * sizeof(double));
    for (int64_t i = 0; i < m; ++i) {
        const double *a = A + i * r;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            double *c = C + (int64_t)colidx[p] * r;
            double s = w[p];
            for (int64_t k = 0; k < r; ++k)
                c[k] += s * a[k];
        }
    }
}

/*
 * Transpose of the pattern (the stored transposed copy of Section IV-B):
 * colptr[n+1], rowidx[nnz] and perm[nnz] with perm[q] = CSR position of the q-th
 * CSC entry.  Counting sort by column, then a scatter that walks rows in ascending
 * order, so the rows inside a column come out ascending.  valT[q] = val[perm[q]]
 * when both are non-NULL.
 */
void oracle_csr_to_csc(int64_t m, int64_t n, const int32_t *rowptr, const int32_t *colidx,
                       const double *val, int32_t *colptr, int32_t *rowidx, double *valT,
                       int32_t *perm)
{
    int64_t *next = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t nnz = rowptr[m];
    for (int64_t p = 0; p < nnz; ++p) next[colidx[p] + 1] += 1;
    for (int64_t j = 0; j < n; ++j) next[j + 1] += next[j];
    for (int64_t j = 0; j <= n; ++j) colptr[j] = (int32_t)next[j];
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int64_t q = next[colidx[p]]++;
            rowidx[q] = (int32_t)i;
            perm[q] = (int32_t)p;
            if (val && valT) valT[q] = val[p];
        }
    }
    free(next);
}

/* Threads for the routines above (n >= 1; for timing at a fixed thread count). */
void oracle_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Number of OpenMP threads the routines above use (for reporting). */
int oracle_num_threads(void)
{
    int t = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            t = omp_get_num_threads();
#endif
        }
    }
    return t;
}

/*
 * Graph attention edge scores (Section VI-E): the attention product of row i and row j
 * is a^T (H_i: || H_j:) = a1 . H_i + a2 . H_j, with a = (a1 || a2).  Per node:
 *   s[i] = sum_k a1[k] H[i,k],   t[i] = sum_k a2[k] H[i,k].
 */
void oracle_gat_scores(int64_t n, int64_t r, const double *H, const double *a1, const double *a2, double *s, double *t)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double x = 0.0, y = 0.0;
        for (int64_t k = 0; k < r; ++k) {
            x += a1[k] * H[i * r + k];
            y += a2[k] * H[i * r + k];
        }
        s[i] = x;
        t[i] = y;
    }
}

/*
 * Edge values S'_ij = LeakyReLU(S_ij (s_i + t_j)) at the stored entries (Section VI-E:
 * the sampled attention product followed by LeakyReLU), and, when softmax != 0, the
 * softmax of each row's values over its stored entries:
 *   w[p] = exp(e[p] - max_row) / sum_{q in row} exp(e[q] - max_row).
 * val == NULL means a 0/1 adjacency (every stored value 1).
 */
void oracle_gat_edges(int64_t m, const int32_t *rowptr, const int32_t *colidx, const double *val, const double *s,
                      const double *t, double slope, int softmax, double *w)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < m; ++i) {
        const int64_t b = rowptr[i], e = rowptr[i + 1];
        for (int64_t p = b; p < e; ++p) {
            const double x = (val ? val[p] : 1.0) * (s[i] + t[colidx[p]]);
            w[p] = x >= 0.0 ? x : slope * x;
        }
        if (softmax && e > b) {
            double mx = w[b];
            for (int64_t p = b + 1; p < e; ++p)
                if (w[p] > mx) mx = w[p];
            double sum = 0.0;
            for (int64_t p = b; p < e; ++p) {
                w[p] = exp(w[p] - mx);
                sum += w[p];
            }
            for (int64_t p = b; p < e; ++p) w[p] /= sum;
        }
    }
}
