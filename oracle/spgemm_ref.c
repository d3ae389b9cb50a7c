/*
 * CPU oracle for C = A * B on row-major compressed (CSR) FP64 matrices.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the tests, the smoke check and the bench's CPU
 * baseline do.  It shares no code with the GPU path.
 *
 * What it computes (paper, Section IV-A, the row-major algorithm attributed to
 * Gustavson, and the listing of the row-major computation kernel):
 *   for every row r of A, every stored a(r,c) of that row in stored order, and
 *   every stored b(c,x) of row c of B, add a(r,c) * b(c,x) into a dense
 *   temporary row vector at position x; the vector starts out filled with
 *   zeros.  After the row is done, the vector is a dense picture of row r of C.
 *
 * How the dense row becomes a sparse row (paper, Section IV-B, the "Sort"
 * storing strategy): the indices touched in the row are kept in a separate
 * list, the list is sorted, and only those positions are emitted, in
 * increasing column order (the append/finalize contract of Section IV-B).
 * First touches are detected with a separate byte marker array (one of the
 * paper's lookup vectors), so an entry whose value cancels to 0.0 is still
 * stored: the structure of C is the union of the column sets of the B rows
 * that a row of A selects, independent of the values.
 *
 * Arithmetic: every update is one FP64 multiply followed by one FP64 add,
 * each rounded to nearest (this file is compiled with -ffp-contract=off, so no
 * fused multiply-add), accumulated in A's stored (ascending column) order,
 * starting from +0.0.
 *
 * Index widths: row pointers are int64, column indices int32.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Number of stored entries of rows r0..r1-1 of C = A*B, written to
 * counts[0..r1-r0).  Returns 0, or -1 if scratch could not be allocated. */
int oracle_row_counts(int64_t r0, int64_t r1,
                      const int64_t *a_ptr, const int32_t *a_col,
                      int64_t b_cols, const int64_t *b_ptr, const int32_t *b_col,
                      int64_t *counts)
{
    unsigned char *mark = calloc((size_t)(b_cols > 0 ? b_cols : 1), 1);
    int32_t *touched = malloc(sizeof(int32_t) * (size_t)(b_cols > 0 ? b_cols : 1));
    if (!mark || !touched) { free(mark); free(touched); return -1; }
    for (int64_t r = r0; r < r1; ++r) {
        int64_t n = 0;
        for (int64_t e = a_ptr[r]; e < a_ptr[r + 1]; ++e) {
            int32_t c = a_col[e];
            for (int64_t f = b_ptr[c]; f < b_ptr[c + 1]; ++f) {
                int32_t x = b_col[f];
                if (!mark[x]) { mark[x] = 1; touched[n++] = x; }
            }
        }
        for (int64_t t = 0; t < n; ++t) mark[touched[t]] = 0;
        counts[r - r0] = n;
    }
    free(mark);
    free(touched);
    return 0;
}

/* Rows r0..r1-1 of C = A*B.  c_ptr[0..r1-r0] must already hold the output
 * offsets (c_ptr[0] is where row r0 starts in c_col/c_val); the caller sizes
 * them from oracle_row_counts.  Returns 0, or -1 on allocation failure. */
int oracle_rows(int64_t r0, int64_t r1,
                const int64_t *a_ptr, const int32_t *a_col, const double *a_val,
                int64_t b_cols, const int64_t *b_ptr, const int32_t *b_col, const double *b_val,
                const int64_t *c_ptr, int32_t *c_col, double *c_val)
{
    size_t w = (size_t)(b_cols > 0 ? b_cols : 1);
    double *temp = malloc(sizeof(double) * w);
    unsigned char *mark = calloc(w, 1);
    int32_t *touched = malloc(sizeof(int32_t) * w);
    if (!temp || !mark || !touched) { free(temp); free(mark); free(touched); return -1; }
    for (size_t x = 0; x < w; ++x) temp[x] = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
        int64_t n = 0;
        for (int64_t e = a_ptr[r]; e < a_ptr[r + 1]; ++e) {
            int32_t c = a_col[e];
            double va = a_val[e];
            for (int64_t f = b_ptr[c]; f < b_ptr[c + 1]; ++f) {
                int32_t x = b_col[f];
                if (!mark[x]) { mark[x] = 1; touched[n++] = x; }
                double prod = va * b_val[f];
                temp[x] = temp[x] + prod;
            }
        }
        qsort(touched, (size_t)n, sizeof(int32_t), cmp_i32);
        int64_t out = c_ptr[r - r0];
        for (int64_t t = 0; t < n; ++t) {
            int32_t x = touched[t];
            c_col[out] = x;
            c_val[out] = temp[x];
            ++out;
            temp[x] = 0.0;
            mark[x] = 0;
        }
    }
    free(temp);
    free(mark);
    free(touched);
    return 0;
}
