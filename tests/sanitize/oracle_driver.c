/*
 * Sanitizer driver for the CPU oracle (test infrastructure): builds small
 * CSR operands (empty rows, a dense row, duplicate-free random columns),
 * calls oracle_row_counts and oracle_rows on whole and partial row ranges,
 * and checks them against a dense brute-force product computed here.  Built
 * with AddressSanitizer and UndefinedBehaviorSanitizer; exit status 0 when
 * every check passes.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_row_counts(int64_t r0, int64_t r1, const int64_t *a_ptr, const int32_t *a_col, int64_t b_cols,
                      const int64_t *b_ptr, const int32_t *b_col, int64_t *counts);
int oracle_rows(int64_t r0, int64_t r1, const int64_t *a_ptr, const int32_t *a_col, const double *a_val,
                int64_t b_cols, const int64_t *b_ptr, const int32_t *b_col, const double *b_val,
                const int64_t *c_ptr, int32_t *c_col, double *c_val);

static uint64_t state = 0x9e3779b97f4a7c15ull;
static uint64_t next(void) {
    uint64_t z = (state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

/* rows x cols CSR with each entry present with probability num/den; row
 * `dense_row` (if >= 0) full, row `empty_row` empty */
static void make(int64_t rows, int64_t cols, int num, int den, int64_t dense_row, int64_t empty_row,
                 int64_t **ptr, int32_t **col, double **val) {
    *ptr = calloc((size_t)rows + 1, sizeof(int64_t));
    *col = malloc(sizeof(int32_t) * (size_t)(rows * cols + 1));
    *val = malloc(sizeof(double) * (size_t)(rows * cols + 1));
    int64_t n = 0;
    for (int64_t r = 0; r < rows; ++r) {
        for (int64_t c = 0; c < cols; ++c) {
            int take = r == dense_row || (r != empty_row && (int)(next() % (uint64_t)den) < num);
            if (take) {
                (*col)[n] = (int32_t)c;
                (*val)[n] = (double)(int)(next() % 7) - 3.0;
                ++n;
            }
        }
        (*ptr)[r + 1] = n;
    }
}

static int check(int64_t m, int64_t k, int64_t n, int num, int den) {
    int64_t *ap, *bp;
    int32_t *ac, *bc;
    double *av, *bv;
    make(m, k, num, den, m > 2 ? 1 : -1, m > 3 ? 2 : -1, &ap, &ac, &av);
    make(k, n, num, den, -1, k > 1 ? 0 : -1, &bp, &bc, &bv);
    /* dense brute force: structure and values, products added in A's order */
    double *dv = calloc((size_t)(m * n + 1), sizeof(double));
    unsigned char *ds = calloc((size_t)(m * n + 1), 1);
    for (int64_t r = 0; r < m; ++r)
        for (int64_t e = ap[r]; e < ap[r + 1]; ++e)
            for (int64_t f = bp[ac[e]]; f < bp[ac[e] + 1]; ++f) {
                double p = av[e] * bv[f];
                dv[r * n + bc[f]] = dv[r * n + bc[f]] + p;
                ds[r * n + bc[f]] = 1;
            }
    int bad = 0;
    for (int64_t r0 = 0; r0 <= m; r0 += (m / 3 > 0 ? m / 3 : 1)) {
        const int64_t r1 = m;
        int64_t *cnt = malloc(sizeof(int64_t) * (size_t)(r1 - r0 + 1));
        if (oracle_row_counts(r0, r1, ap, ac, n, bp, bc, cnt) != 0) return 1;
        int64_t *cp = calloc((size_t)(r1 - r0 + 1), sizeof(int64_t));
        for (int64_t r = r0; r < r1; ++r) cp[r - r0 + 1] = cp[r - r0] + cnt[r - r0];
        int32_t *cc = malloc(sizeof(int32_t) * (size_t)(cp[r1 - r0] + 1));
        double *cv = malloc(sizeof(double) * (size_t)(cp[r1 - r0] + 1));
        if (oracle_rows(r0, r1, ap, ac, av, n, bp, bc, bv, cp, cc, cv) != 0) return 1;
        for (int64_t r = r0; r < r1; ++r) {
            int64_t q = cp[r - r0];
            for (int64_t x = 0; x < n; ++x) {
                if (!ds[r * n + x]) continue;
                if (q >= cp[r - r0 + 1] || cc[q] != x || memcmp(&cv[q], &dv[r * n + x], sizeof(double)) != 0) bad = 1;
                ++q;
            }
            if (q != cp[r - r0 + 1]) bad = 1;
        }
        free(cnt);
        free(cp);
        free(cc);
        free(cv);
        if (r0 == m) break;
    }
    free(dv);
    free(ds);
    free(ap); free(ac); free(av); free(bp); free(bc); free(bv);
    return bad;
}

int main(void) {
    int bad = 0;
    bad |= check(0, 0, 0, 1, 2);
    bad |= check(5, 0, 4, 1, 2);
    bad |= check(7, 6, 0, 1, 2);
    bad |= check(1, 1, 1, 1, 1);
    for (int t = 0; t < 12; ++t) bad |= check(3 + t * 5, 2 + t * 7, 4 + t * 3, 1 + t % 3, 4);
    printf(bad ? "oracle driver: MISMATCH\n" : "oracle driver: ok\n");
    return bad;
}
