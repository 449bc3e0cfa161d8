/*
 * CPU oracle for row-wise sparse matrix-matrix product C = A*B.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or table with the HIP library; it is a plain, slow, obviously
 * correct restatement of what the paper defines:
 *
 *   - Gustavson's row-wise product (Section 2, Fig. 1): row i of C is built by
 *     scanning every stored a_ik of row i and every stored b_kj of row k and
 *     either inserting c_ij = a_ik*b_kj or adding it to the existing c_ij.
 *   - The accumulator is the sparse accumulator (SPA) of Section 2: a dense
 *     value vector over the columns of C plus a list of the columns touched.
 *   - Row flop (Fig. 4, part 1): flop_i = sum over a_ik of nnz(b_k*).
 *   - Row partition over threads (Fig. 4, part 2): exclusive prefix sum of
 *     flop, ave = total/tnum, thread t starts at the first row whose prefix is
 *     at least ave*t.
 *   - Two phases (Section 2; Fig. 5): a symbolic pass counts nnz(c_i*), the
 *     counts are prefix-summed into the row pointers of C, then a numeric pass
 *     fills columns and values; rows are sorted by column if asked (Section
 *     4.2.1, output step).
 *   - Masked sum for triangle counting (Section 5.6): sum of c_ij over the
 *     positions (i,j) stored in a mask matrix.
 *
 * Conventions (readings where the paper is silent):
 *   - The pattern is structural: an entry exists as soon as one product
 *     reaches it, whatever its value; zero sums are kept.
 *   - int64 values use wrap-around (mod 2^64) multiply and add.
 *   - Floating point is IEEE binary64; each c_ij is summed in the order
 *     (p over row i of A in storage order, q over row k of B in storage order).
 *   - Unsorted mode emits each row in first-touch order.
 *   - Row pointers are int64 everywhere; column ids are int32.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define OR_F64 0
#define OR_I64 1

/* -------------------------------------------------------------- validate */

/* Structure check of a CSR operand before any product (the CSR layout of
 * Section 2: row i holds positions rpts[i] .. rpts[i+1]-1 of cols/vals).
 * Returns 0 if well formed, else the first failed rule:
 *   1  rpts[0] != 0          2  rpts decreases somewhere
 *   3  rpts[nrows] != nnz    4  a column id outside [0, ncols)
 *   5  a column repeated within a row (checked only if check_dup)
 *   6  scratch memory unavailable for the repeat check */
int oracle_validate_csr(int64_t nrows, int64_t ncols, int64_t nnz, const int64_t *rpts,
                        const int32_t *cols, int check_dup)
{
    if (rpts[0] != 0) return 1;
    for (int64_t i = 0; i < nrows; ++i)
        if (rpts[i + 1] < rpts[i]) return 2;
    if (rpts[nrows] != nnz) return 3;
    for (int64_t p = 0; p < nnz; ++p)
        if (cols[p] < 0 || (int64_t)cols[p] >= ncols) return 4;
    if (!check_dup) return 0;
    int64_t *seen = (int64_t *)malloc((size_t)(ncols > 0 ? ncols : 1) * sizeof(int64_t));
    if (!seen) return 6;
    for (int64_t j = 0; j < ncols; ++j) seen[j] = -1;
    int bad = 0;
    for (int64_t i = 0; i < nrows && !bad; ++i)
        for (int64_t p = rpts[i]; p < rpts[i + 1]; ++p) {
            if (seen[cols[p]] == i) { bad = 5; break; }
            seen[cols[p]] = i;
        }
    free(seen);
    return bad;
}

/* ------------------------------------------------------------------ flop */

/* Per-row flop (Fig. 4 part 1) for the selected rows; returns the total. */
int64_t oracle_row_flop(int64_t nsel, const int64_t *rows, const int64_t *rptsA,
                        const int32_t *colsA, const int64_t *rptsB, int64_t *flop_out,
                        int nthreads)
{
    int64_t total = 0;
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) reduction(+ : total) num_threads(nthreads)
    for (int64_t s = 0; s < nsel; ++s) {
        int64_t i = rows ? rows[s] : s;
        int64_t f = 0;
        for (int64_t p = rptsA[i]; p < rptsA[i + 1]; ++p) {
            int64_t k = colsA[p];
            f += rptsB[k + 1] - rptsB[k];
        }
        if (flop_out) flop_out[s] = f;
        total += f;
    }
    return total;
}

/* Fig. 4 part 2.  offset has tnum+1 entries.  flop_ps is the exclusive prefix
 * sum (length n+1), and offset[t] = first id with flop_ps[id] >= total*t/tnum,
 * compared exactly as flop_ps[id]*tnum >= total*t. */
void oracle_rows_to_threads(int64_t n, const int64_t *flop, int tnum, int64_t *offset)
{
    int64_t *ps = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    ps[0] = 0;
    for (int64_t i = 0; i < n; ++i) ps[i + 1] = ps[i] + flop[i];
    const __int128 total = ps[n];
    offset[0] = 0;
    for (int t = 1; t < tnum; ++t) {
        const __int128 target = total * t;
        int64_t lo = 0, hi = n + 1; /* lower_bound over ps[0..n] */
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if ((__int128)ps[mid] * tnum >= target) hi = mid; else lo = mid + 1;
        }
        offset[t] = lo;
    }
    offset[tnum] = n;
    free(ps);
}

/* Thread partition of the selected rows by their flop. */
static int64_t *partition_rows(int64_t nsel, const int64_t *rows, const int64_t *rptsA,
                               const int32_t *colsA, const int64_t *rptsB, int tnum)
{
    int64_t *flop = (int64_t *)malloc((size_t)(nsel > 0 ? nsel : 1) * sizeof(int64_t));
    int64_t *offset = (int64_t *)malloc((size_t)(tnum + 1) * sizeof(int64_t));
    oracle_row_flop(nsel, rows, rptsA, colsA, rptsB, flop, tnum);
    oracle_rows_to_threads(nsel, flop, tnum, offset);
    free(flop);
    return offset;
}

/* -------------------------------------------------------------- symbolic */

/* nnz of each selected row of C, prefix-summed into rpts_out[nsel+1].
 * Returns nnz of the selection, or -1 if scratch memory is unavailable. */
int64_t oracle_symbolic(int64_t nsel, const int64_t *rows, int64_t ncolsB,
                        const int64_t *rptsA, const int32_t *colsA,
                        const int64_t *rptsB, const int32_t *colsB,
                        int64_t *rpts_out, int nthreads)
{
    int tnum = nthreads > 0 ? nthreads : omp_get_max_threads();
    int64_t *offset = partition_rows(nsel, rows, rptsA, colsA, rptsB, tnum);
    int failed = 0;
#pragma omp parallel num_threads(tnum)
    {
        int tid = omp_get_thread_num();
        int64_t *mark = (int64_t *)malloc((size_t)(ncolsB > 0 ? ncolsB : 1) * sizeof(int64_t));
        if (!mark) {
#pragma omp atomic write
            failed = 1;
        } else {
            for (int64_t j = 0; j < ncolsB; ++j) mark[j] = -1;
            for (int64_t s = offset[tid]; s < offset[tid + 1]; ++s) {
                int64_t i = rows ? rows[s] : s;
                int64_t cnt = 0;
                for (int64_t p = rptsA[i]; p < rptsA[i + 1]; ++p) {
                    int64_t k = colsA[p];
                    for (int64_t q = rptsB[k]; q < rptsB[k + 1]; ++q) {
                        int64_t j = colsB[q];
                        if (mark[j] != s) { mark[j] = s; ++cnt; }
                    }
                }
                rpts_out[s + 1] = cnt; /* count for now; scanned below */
            }
            free(mark);
        }
    }
    free(offset);
    if (failed) return -1;
    rpts_out[0] = 0;
    for (int64_t s = 0; s < nsel; ++s) rpts_out[s + 1] += rpts_out[s];
    return rpts_out[nsel];
}

/* --------------------------------------------------------------- numeric */

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

#define DEFINE_NUMERIC(NAME, T, MUL, ADD)                                                     \
static int NAME(int sorted, int64_t nsel, const int64_t *rows, int64_t ncolsB,                \
                const int64_t *rptsA, const int32_t *colsA, const T *valsA,                   \
                const int64_t *rptsB, const int32_t *colsB, const T *valsB,                   \
                const int64_t *rpts_out, int32_t *cols_out, T *vals_out, int tnum)            \
{                                                                                             \
    int64_t *offset = partition_rows(nsel, rows, rptsA, colsA, rptsB, tnum);                  \
    int failed = 0;                                                                           \
    _Pragma("omp parallel num_threads(tnum)")                                                 \
    {                                                                                         \
        int tid = omp_get_thread_num();                                                       \
        size_t w = (size_t)(ncolsB > 0 ? ncolsB : 1);                                         \
        int64_t *mark = (int64_t *)malloc(w * sizeof(int64_t));                               \
        T *val = (T *)malloc(w * sizeof(T));                                                  \
        int32_t *list = (int32_t *)malloc(w * sizeof(int32_t));                               \
        if (!mark || !val || !list) {                                                         \
            _Pragma("omp atomic write")                                                       \
            failed = 1;                                                                       \
        } else {                                                                              \
            for (int64_t j = 0; j < ncolsB; ++j) mark[j] = -1;                                \
            for (int64_t s = offset[tid]; s < offset[tid + 1]; ++s) {                         \
                int64_t i = rows ? rows[s] : s;                                               \
                int64_t len = 0;                                                              \
                for (int64_t p = rptsA[i]; p < rptsA[i + 1]; ++p) {                           \
                    int64_t k = colsA[p];                                                     \
                    T a = valsA[p];                                                           \
                    for (int64_t q = rptsB[k]; q < rptsB[k + 1]; ++q) {                       \
                        int32_t j = colsB[q];                                                 \
                        T x = MUL(a, valsB[q]);                                               \
                        if (mark[j] != s) { mark[j] = s; val[j] = x; list[len++] = j; }       \
                        else val[j] = ADD(val[j], x);                                         \
                    }                                                                         \
                }                                                                             \
                if (len != rpts_out[s + 1] - rpts_out[s]) {                                   \
                    _Pragma("omp atomic write")                                               \
                    failed = 2;                                                               \
                    continue;                                                                 \
                }                                                                             \
                if (sorted) qsort(list, (size_t)len, sizeof(int32_t), cmp_i32);               \
                int64_t o = rpts_out[s];                                                      \
                for (int64_t t = 0; t < len; ++t) {                                           \
                    cols_out[o + t] = list[t];                                                \
                    vals_out[o + t] = val[list[t]];                                           \
                }                                                                             \
            }                                                                                 \
        }                                                                                     \
        free(mark); free(val); free(list);                                                    \
    }                                                                                         \
    free(offset);                                                                             \
    return failed ? -failed : 0;                                                              \
}

#define F64_MUL(a, b) ((a) * (b))
#define F64_ADD(a, b) ((a) + (b))
#define I64_MUL(a, b) ((int64_t)((uint64_t)(a) * (uint64_t)(b)))
#define I64_ADD(a, b) ((int64_t)((uint64_t)(a) + (uint64_t)(b)))

DEFINE_NUMERIC(numeric_f64, double, F64_MUL, F64_ADD)
DEFINE_NUMERIC(numeric_i64, int64_t, I64_MUL, I64_ADD)

/* Fill columns/values of the selected rows.  rpts_out must come from
 * oracle_symbolic on the same selection.  Returns 0, or a negative code if
 * scratch memory is unavailable (-1) or a row count disagrees (-2). */
int oracle_numeric(int dtype, int sorted, int64_t nsel, const int64_t *rows, int64_t ncolsB,
                   const int64_t *rptsA, const int32_t *colsA, const void *valsA,
                   const int64_t *rptsB, const int32_t *colsB, const void *valsB,
                   const int64_t *rpts_out, int32_t *cols_out, void *vals_out, int nthreads)
{
    int tnum = nthreads > 0 ? nthreads : omp_get_max_threads();
    if (dtype == OR_F64)
        return numeric_f64(sorted, nsel, rows, ncolsB, rptsA, colsA, (const double *)valsA,
                           rptsB, colsB, (const double *)valsB, rpts_out, cols_out,
                           (double *)vals_out, tnum);
    if (dtype == OR_I64)
        return numeric_i64(sorted, nsel, rows, ncolsB, rptsA, colsA, (const int64_t *)valsA,
                           rptsB, colsB, (const int64_t *)valsB, rpts_out, cols_out,
                           (int64_t *)vals_out, tnum);
    return -3;
}

/* ----------------------------------------------------------- masked sum */

/* sum over stored (i,j) of M of C_ij (int64, wrap-around).  Section 5.6 uses
 * it with C = L*U and M = A: each triangle is counted twice. */
int64_t oracle_masked_sum_i64(int64_t m, int64_t ncols,
                              const int64_t *rptsC, const int32_t *colsC, const int64_t *valsC,
                              const int64_t *rptsM, const int32_t *colsM, int nthreads)
{
    int tnum = nthreads > 0 ? nthreads : omp_get_max_threads();
    uint64_t total = 0;
#pragma omp parallel num_threads(tnum) reduction(+ : total)
    {
        int64_t *mark = (int64_t *)malloc((size_t)(ncols > 0 ? ncols : 1) * sizeof(int64_t));
        for (int64_t j = 0; j < ncols; ++j) mark[j] = -1;
#pragma omp for schedule(static)
        for (int64_t i = 0; i < m; ++i) {
            for (int64_t p = rptsM[i]; p < rptsM[i + 1]; ++p) mark[colsM[p]] = i;
            for (int64_t q = rptsC[i]; q < rptsC[i + 1]; ++q)
                if (mark[colsC[q]] == i) total += (uint64_t)valsC[q];
        }
        free(mark);
    }
    return (int64_t)total;
}

int oracle_max_threads(void) { return omp_get_max_threads(); }
