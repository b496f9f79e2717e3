/*
 * Plain CPU oracle for sparse-matrix permutation, extraction and assignment.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file.  Only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header or table with the GPU
 * library.
 *
 * Every routine writes out the definition given in the paper's problem
 * formulation (Section 2, "Problem Formulation"), in the slowest obvious way:
 *
 *   permute   (Sec. 2.1):  A'[i,j] = A[pvec[i], qvec[j]]   for all i < m, j < n
 *   extract   (Sec. 2.2):  B[i,j]  = A[pvec[i], qvec[j]]   for all (i,j) in pvec x qvec
 *             (also on column-compressed CSC/DCSC storage, walking the
 *             selected columns as the appendix's Alg. 5 does)
 *   assign    (Sec. 2.3, and the Add step of Sec. 4.7):
 *                          B'[pvec[i], qvec[j]] = B[i,j]   for stored entries of B
 *                          A_new = A (+) B'   with a user-chosen addition
 *
 * Conventions (each is a reading of the paper; the design notes list them):
 *   - 0-based indices (the paper counts from 1);
 *   - CSR with columns strictly ascending inside each row;
 *   - values are moved as raw bytes (4 or 8 per value), never re-rounded;
 *   - PLUS adds in the value's own type with round-to-nearest-even.  For
 *     4-byte values the sum is formed in double and rounded once to float:
 *     double has 53 >= 2*24+2 significand bits, so this equals a single
 *     correctly rounded float addition (double rounding is innocuous for +).
 *
 * Two routines per operation family:
 *   - orc_permute, orc_spref, orc_spref_dcsc search every (i, j) pair of the
 *     definition (slow, literal; for small inputs and sampled rows);
 *   - orc_permute_map and orc_spref_map compute the same result from the
 *     stored entries with inverse index tables, as the definition can be
 *     restated: permute copies row p[i] and renames each column c to
 *     qinv[c]; extract builds, for every column c, the ascending list of
 *     positions j with J[j] = c and emits (j, value) for every stored entry
 *     of row I[i] and every j in its column's list.  Each output row is then
 *     sorted by column.  Their cost is the number of stored entries read,
 *     so they finish whole outputs at full benchmark sizes.  The assignment
 *     (orc_spasgn) is a merge of the stored entries already.
 *
 * Output rows may be restricted to a list `rows` (the sampled-row mode used
 * at full benchmark sizes); rows == NULL means every output row.  Outputs use
 * the two-call protocol: with cap smaller than the needed count nothing is
 * written beyond out_ptr and *need receives the count.
 *
 * The map routines and the assignment take a thread count: output rows are
 * independent, so they are counted, then filled, in parallel over rows
 * (OpenMP); the result does not depend on the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "hp_oracle.h"

/* ---- small helpers --------------------------------------------------- */

/* Position of column c in row r of a canonical CSR, or -1. */
static int64_t find_in_row(const int64_t *rowptr, const int32_t *col, int64_t r, int32_t c)
{
    int64_t lo = rowptr[r], hi = rowptr[r + 1];
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (col[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    if (lo < rowptr[r + 1] && col[lo] == c) return lo;
    return -1;
}

static void copy_val(void *dst, int64_t di, const void *src, int64_t si, int vsize)
{
    memcpy((char *)dst + di * vsize, (const char *)src + si * vsize, (size_t)vsize);
}

int orc_check_csr(int64_t m, int64_t n, const int64_t *rowptr, const int32_t *col)
{
    if (m < 0 || n < 0 || !rowptr) return ORC_INVALID_ARG;
    if (rowptr[0] != 0) return ORC_NOT_CANONICAL;
    for (int64_t r = 0; r < m; r++) {
        if (rowptr[r + 1] < rowptr[r]) return ORC_NOT_CANONICAL;
        for (int64_t k = rowptr[r]; k < rowptr[r + 1]; k++) {
            if (col[k] < 0 || col[k] >= n) return ORC_INDEX_RANGE;
            if (k > rowptr[r] && col[k] <= col[k - 1]) return ORC_NOT_CANONICAL;
        }
    }
    return ORC_OK;
}

/* v is a permutation of [0, len): every value in range, none repeated. */
static int check_permutation(const int32_t *v, int64_t len)
{
    unsigned char *seen = (unsigned char *)calloc((size_t)(len > 0 ? len : 1), 1);
    if (!seen) return ORC_INVALID_ARG;
    int st = ORC_OK;
    for (int64_t i = 0; i < len; i++) {
        if (v[i] < 0 || v[i] >= len) { st = ORC_INDEX_RANGE; break; }
        if (seen[v[i]]) { st = ORC_NOT_PERMUTATION; break; }
        seen[v[i]] = 1;
    }
    free(seen);
    return st;
}

static int check_range(const int32_t *v, int64_t len, int64_t hi)
{
    for (int64_t i = 0; i < len; i++)
        if (v[i] < 0 || v[i] >= hi) return ORC_INDEX_RANGE;
    return ORC_OK;
}

/* Values in range and pairwise distinct (assignment vectors, Sec. 2.3). */
static int check_distinct(const int32_t *v, int64_t len, int64_t hi)
{
    int st = check_range(v, len, hi);
    if (st != ORC_OK) return st;
    unsigned char *seen = (unsigned char *)calloc((size_t)(hi > 0 ? hi : 1), 1);
    if (!seen) return ORC_INVALID_ARG;
    for (int64_t i = 0; i < len; i++) {
        if (seen[v[i]]) { st = ORC_DUPLICATE_INDEX; break; }
        seen[v[i]] = 1;
    }
    free(seen);
    return st;
}

/* ---- permutation, Sec. 2.1 -------------------------------------------- */

int orc_permute(int64_t m, int64_t n, const int64_t *rowptr, const int32_t *col,
                const void *val, int vsize, const int32_t *p, const int32_t *q,
                const int64_t *rows, int64_t ns,
                int64_t *out_ptr, int32_t *out_col, void *out_val, int64_t cap, int64_t *need)
{
    if (vsize != 4 && vsize != 8) return ORC_INVALID_ARG;
    if (!q) {                       /* symmetric form P A P^T */
        if (m != n) return ORC_SHAPE;
        q = p;
    }
    int st = check_permutation(p, m);
    if (st != ORC_OK) return st;
    st = check_permutation(q, n);
    if (st != ORC_OK) return st;
    if (!rows) ns = m;
    int64_t cnt = 0;
    out_ptr[0] = 0;
    for (int64_t s = 0; s < ns; s++) {
        int64_t i = rows ? rows[s] : s;
        if (i < 0 || i >= m) return ORC_INDEX_RANGE;
        int64_t src = p[i];
        /* A'[i, j] = A[p[i], q[j]] for every j, in increasing j. */
        for (int64_t j = 0; j < n; j++) {
            int64_t k = find_in_row(rowptr, col, src, q[j]);
            if (k < 0) continue;
            if (cnt < cap) {
                out_col[cnt] = (int32_t)j;
                copy_val(out_val, cnt, val, k, vsize);
            }
            cnt++;
        }
        out_ptr[s + 1] = cnt;
    }
    *need = cnt;
    return ORC_OK;
}

/* ---- extraction, Sec. 2.2 --------------------------------------------- */

int orc_spref(int64_t m, int64_t n, const int64_t *rowptr, const int32_t *col,
              const void *val, int vsize, const int32_t *I, int64_t nI,
              const int32_t *J, int64_t nJ, const int64_t *rows, int64_t ns,
              int64_t *out_ptr, int32_t *out_col, void *out_val, int64_t cap, int64_t *need)
{
    if (vsize != 4 && vsize != 8) return ORC_INVALID_ARG;
    if (nI < 0 || nJ < 0) return ORC_INVALID_ARG;
    int st = check_range(I, nI, m);
    if (st != ORC_OK) return st;
    st = check_range(J, nJ, n);
    if (st != ORC_OK) return st;
    if (!rows) ns = nI;
    int64_t cnt = 0;
    out_ptr[0] = 0;
    for (int64_t s = 0; s < ns; s++) {
        int64_t i = rows ? rows[s] : s;
        if (i < 0 || i >= nI) return ORC_INDEX_RANGE;
        /* C[i, j] = A[I[i], J[j]] over the whole Cartesian product row i x J. */
        for (int64_t j = 0; j < nJ; j++) {
            int64_t k = find_in_row(rowptr, col, I[i], J[j]);
            if (k < 0) continue;
            if (cnt < cap) {
                out_col[cnt] = (int32_t)j;
                copy_val(out_val, cnt, val, k, vsize);
            }
            cnt++;
        }
        out_ptr[s + 1] = cnt;
    }
    *need = cnt;
    return ORC_OK;
}

/* ---- extraction on column-compressed storage (Sec. 2.2, appendix Alg. 5) */

/* Stored column holding column id c: with jc (doubly compressed, Sec. 4.1)
 * the k with jc[k] == c, by binary search over the nzc stored ids, or -1;
 * without jc (plain CSC) every column is stored and k = c. */
static int64_t find_stored_col(const int32_t *jc, int64_t nzc, int32_t c)
{
    if (!jc) return c;
    int64_t lo = 0, hi = nzc - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (jc[mid] == c) return mid;
        if (jc[mid] < c) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

/* Position of row r among the row indices of stored column k, by binary
 * search (the membership test of Alg. 5), or -1. */
static int64_t find_in_col(const int64_t *colptr, const int32_t *row, int64_t k, int32_t r)
{
    int64_t lo = colptr[k], hi = colptr[k + 1] - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (row[mid] == r) return mid;
        if (row[mid] < r) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

/* C = A(I, J) with A and C column-compressed: for every selected column
 * J[j] and every selected row I[i], C[i, j] = A[I[i], J[j]] when the binary
 * search finds I[i] in that column.  Output in CSC: out_ptr over the output
 * columns (all nJ, or the listed `cols`), out_row holds positions i in I,
 * ascending within a column.  jc == NULL: A is plain CSC (colptr has n+1
 * entries, nzc ignored). */
int orc_spref_dcsc(int64_t m, int64_t n, int64_t nzc, const int32_t *jc, const int64_t *colptr,
                   const int32_t *row, const void *val, int vsize, const int32_t *I, int64_t nI,
                   const int32_t *J, int64_t nJ, const int64_t *cols, int64_t ns,
                   int64_t *out_ptr, int32_t *out_row, void *out_val, int64_t cap, int64_t *need)
{
    if (vsize != 4 && vsize != 8) return ORC_INVALID_ARG;
    if (nI < 0 || nJ < 0 || (jc && (nzc < 0 || nzc > n))) return ORC_INVALID_ARG;
    int st = check_range(I, nI, m);
    if (st != ORC_OK) return st;
    st = check_range(J, nJ, n);
    if (st != ORC_OK) return st;
    if (!cols) ns = nJ;
    int64_t cnt = 0;
    out_ptr[0] = 0;
    for (int64_t s = 0; s < ns; s++) {
        int64_t j = cols ? cols[s] : s;
        if (j < 0 || j >= nJ) return ORC_INDEX_RANGE;
        int64_t k = find_stored_col(jc, nzc, J[j]);
        if (k >= 0) {
            for (int64_t i = 0; i < nI; i++) {
                int64_t p = find_in_col(colptr, row, k, I[i]);
                if (p < 0) continue;
                if (cnt < cap) {
                    out_row[cnt] = (int32_t)i;
                    copy_val(out_val, cnt, val, p, vsize);
                }
                cnt++;
            }
        }
        out_ptr[s + 1] = cnt;
    }
    *need = cnt;
    return ORC_OK;
}

/* ---- row-parallel driver ----------------------------------------------- */

/* A stored entry on its way to an output row: new column c, index k of its
 * value in the source array.  Keys are unique inside an output row, so the
 * order qsort gives equal keys never matters. */
typedef struct { int32_t c; int64_t k; } ent_t;

static int cmp_ent(const void *a, const void *b)
{
    const ent_t *x = (const ent_t *)a, *y = (const ent_t *)b;
    return (x->c > y->c) - (x->c < y->c);
}

/* One output row of a routine: returns its entry count and, when oc is not
 * NULL, writes its columns (ascending) and values at oc / ov.  `work` holds
 * at least the larger of the row's entry count and the routine's own bound
 * (rowfn_t.work_elems) of ent_t. */
typedef int64_t (*row_fn)(const void *ctx, int64_t i, int32_t *oc, void *ov, ent_t *work);

typedef struct {
    row_fn row;
    const void *ctx;
    int64_t nout;        /* number of output rows                        */
    int64_t work_elems;  /* scratch entries a count-only call may need   */
    int vsize;
} rowfn_t;

/* Output row of the s-th requested row: rows[s], or s when every row is
 * requested. */
static int64_t pick_row(const int64_t *rows, int64_t s)
{
    return rows ? rows[s] : s;
}

/* Counts every requested output row, sums the counts into out_ptr, and, if
 * the arrays are given and cap holds the total, fills the rows.  Rows are
 * independent, so both passes split them over nthreads threads. */
static int drive_rows(const rowfn_t *f, const int64_t *rows, int64_t ns, int64_t *out_ptr,
                      int32_t *out_col, void *out_val, int64_t cap, int64_t *need, int nthreads)
{
    if (!rows) ns = f->nout;
    if (rows)
        for (int64_t s = 0; s < ns; s++)
            if (rows[s] < 0 || rows[s] >= f->nout) return ORC_INDEX_RANGE;
    if (nthreads < 1) nthreads = 1;
#ifndef _OPENMP
    nthreads = 1;
#endif
    const int64_t w0 = f->work_elems > 0 ? f->work_elems : 1;
    ent_t *work = (ent_t *)malloc(sizeof(ent_t) * (size_t)w0 * (size_t)nthreads);
    if (!work) return ORC_INVALID_ARG;
    int64_t maxlen = 0;
    out_ptr[0] = 0;
#pragma omp parallel for schedule(dynamic, 1024) num_threads(nthreads) reduction(max : maxlen)
    for (int64_t s = 0; s < ns; s++) {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        const int64_t c = f->row(f->ctx, pick_row(rows, s), NULL, NULL, work + (size_t)t * (size_t)w0);
        out_ptr[s + 1] = c;
        if (c > maxlen) maxlen = c;
    }
    free(work);
    for (int64_t s = 0; s < ns; s++) out_ptr[s + 1] += out_ptr[s];
    *need = out_ptr[ns];
    if (!out_col || !out_val || cap < *need) return ORC_OK;
    const int64_t w1 = maxlen > w0 ? maxlen : w0;
    work = (ent_t *)malloc(sizeof(ent_t) * (size_t)w1 * (size_t)nthreads);
    if (!work) return ORC_INVALID_ARG;
#pragma omp parallel for schedule(dynamic, 1024) num_threads(nthreads)
    for (int64_t s = 0; s < ns; s++) {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        f->row(f->ctx, pick_row(rows, s), out_col + out_ptr[s], (char *)out_val + out_ptr[s] * f->vsize,
               work + (size_t)t * (size_t)w1);
    }
    free(work);
    return ORC_OK;
}

/* Writes the n entries of e, sorted by column, to oc / ov. */
static void sort_and_write(ent_t *e, int64_t n, int32_t *oc, void *ov, const void *val, int vsize)
{
    qsort(e, (size_t)n, sizeof(ent_t), cmp_ent);
    for (int64_t t = 0; t < n; t++) {
        oc[t] = e[t].c;
        copy_val(ov, t, val, e[t].k, vsize);
    }
}

/* ---- permutation through the inverse column map (Sec. 2.1) -------------- */

typedef struct {
    const int64_t *rowptr;
    const int32_t *col;
    const void *val;
    int vsize;
    const int32_t *p;
    const int32_t *qinv;
} perm_ctx_t;

/* Output row i is row p[i] of A with every column c renamed qinv[c]. */
static int64_t perm_row(const void *ctx, int64_t i, int32_t *oc, void *ov, ent_t *work)
{
    const perm_ctx_t *x = (const perm_ctx_t *)ctx;
    const int64_t src = x->p[i];
    const int64_t a = x->rowptr[src], b = x->rowptr[src + 1];
    if (!oc) return b - a;
    for (int64_t k = a; k < b; k++) {
        work[k - a].c = x->qinv[x->col[k]];
        work[k - a].k = k;
    }
    sort_and_write(work, b - a, oc, ov, x->val, x->vsize);
    return b - a;
}

int orc_permute_map(int64_t m, int64_t n, const int64_t *rowptr, const int32_t *col,
                    const void *val, int vsize, const int32_t *p, const int32_t *q,
                    const int64_t *rows, int64_t ns,
                    int64_t *out_ptr, int32_t *out_col, void *out_val, int64_t cap, int64_t *need,
                    int nthreads)
{
    if (vsize != 4 && vsize != 8) return ORC_INVALID_ARG;
    if (!q) {                       /* symmetric form P A P^T */
        if (m != n) return ORC_SHAPE;
        q = p;
    }
    int st = check_permutation(p, m);
    if (st != ORC_OK) return st;
    st = check_permutation(q, n);
    if (st != ORC_OK) return st;
    /* qinv[q[j]] = j: A'[i, j] = A[p[i], q[j]] holds the entry of column c =
     * q[j] of row p[i] at column j = qinv[c]. */
    int32_t *qinv = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!qinv) return ORC_INVALID_ARG;
    for (int64_t j = 0; j < n; j++) qinv[q[j]] = (int32_t)j;
    perm_ctx_t ctx = {rowptr, col, val, vsize, p, qinv};
    rowfn_t f = {perm_row, &ctx, m, 0, vsize};
    st = drive_rows(&f, rows, ns, out_ptr, out_col, out_val, cap, need, nthreads);
    free(qinv);
    return st;
}

/* ---- extraction through the column multimap (Sec. 2.2) ------------------ */

typedef struct {
    const int64_t *rowptr;
    const int32_t *col;
    const void *val;
    int vsize;
    const int32_t *I;
    const int64_t *lstart;   /* n+1 offsets into list, by column */
    const int32_t *list;     /* positions j of J, grouped by column J[j], ascending */
} spref_ctx_t;

/* Output row i: every stored entry (I[i], c) of A appears once at every
 * position j with J[j] = c. */
static int64_t spref_row(const void *ctx, int64_t i, int32_t *oc, void *ov, ent_t *work)
{
    const spref_ctx_t *x = (const spref_ctx_t *)ctx;
    const int64_t r = x->I[i];
    int64_t cnt = 0;
    for (int64_t k = x->rowptr[r]; k < x->rowptr[r + 1]; k++) {
        const int32_t c = x->col[k];
        for (int64_t t = x->lstart[c]; t < x->lstart[c + 1]; t++) {
            if (oc) {
                work[cnt].c = x->list[t];
                work[cnt].k = k;
            }
            cnt++;
        }
    }
    if (oc) sort_and_write(work, cnt, oc, ov, x->val, x->vsize);
    return cnt;
}

int orc_spref_map(int64_t m, int64_t n, const int64_t *rowptr, const int32_t *col,
                  const void *val, int vsize, const int32_t *I, int64_t nI,
                  const int32_t *J, int64_t nJ, const int64_t *rows, int64_t ns,
                  int64_t *out_ptr, int32_t *out_col, void *out_val, int64_t cap, int64_t *need,
                  int nthreads)
{
    if (vsize != 4 && vsize != 8) return ORC_INVALID_ARG;
    if (nI < 0 || nJ < 0) return ORC_INVALID_ARG;
    int st = check_range(I, nI, m);
    if (st != ORC_OK) return st;
    st = check_range(J, nJ, n);
    if (st != ORC_OK) return st;
    /* list[c]: the positions j with J[j] = c, ascending (a counting sort of
     * the positions by their column). */
    int64_t *lstart = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *fillp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int32_t *list = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nJ > 0 ? nJ : 1));
    if (!lstart || !fillp || !list) {
        free(lstart);
        free(fillp);
        free(list);
        return ORC_INVALID_ARG;
    }
    for (int64_t j = 0; j < nJ; j++) lstart[J[j] + 1]++;
    for (int64_t c = 0; c < n; c++) lstart[c + 1] += lstart[c];
    for (int64_t c = 0; c < n; c++) fillp[c] = lstart[c];
    for (int64_t j = 0; j < nJ; j++) list[fillp[J[j]]++] = (int32_t)j;
    free(fillp);
    spref_ctx_t ctx = {rowptr, col, val, vsize, I, lstart, list};
    rowfn_t f = {spref_row, &ctx, nI, 0, vsize};
    st = drive_rows(&f, rows, ns, out_ptr, out_col, out_val, cap, need, nthreads);
    free(lstart);
    free(list);
    return st;
}

/* ---- assignment, Sec. 2.3 / Sec. 4.7 ---------------------------------- */

static void add_vals(void *dst, int64_t di, const void *a, int64_t ai,
                     const void *b, int64_t bi, int vsize)
{
    if (vsize == 8) {
        double x, y, z;
        memcpy(&x, (const char *)a + ai * 8, 8);
        memcpy(&y, (const char *)b + bi * 8, 8);
        z = x + y;
        memcpy((char *)dst + di * 8, &z, 8);
    } else {
        float x, y, z;
        memcpy(&x, (const char *)a + ai * 4, 4);
        memcpy(&y, (const char *)b + bi * 4, 4);
        z = (float)((double)x + (double)y);
        memcpy((char *)dst + di * 4, &z, 4);
    }
}

typedef struct {
    const int64_t *rowptr;
    const int32_t *col;
    const void *val;
    int vsize;
    const int64_t *browptr;
    const int32_t *bcol;
    const void *bval;
    const int32_t *J;
    const int64_t *rowpos;   /* position of each row of A in I, or -1    */
    const int64_t *colpos;   /* position of each column of A in J, or -1 */
    int op;
} asgn_ctx_t;

/* Row r of A_new: the entry-wise union of row r of A and row r of B'. */
static int64_t asgn_row(const void *ctx, int64_t r, int32_t *out_col, void *out_val, ent_t *bp)
{
    const asgn_ctx_t *x = (const asgn_ctx_t *)ctx;
    const int64_t *rowptr = x->rowptr, *browptr = x->browptr, *colpos = x->colpos;
    const int32_t *col = x->col, *bcol = x->bcol, *J = x->J;
    const void *val = x->val, *bval = x->bval;
    const int vsize = x->vsize, op = x->op;
    const int64_t i = x->rowpos[r];
    int64_t nb = 0;
    if (i >= 0) {
        /* Row r of B' = row i of B with each column cb moved to J[cb]. */
        for (int64_t k = browptr[i]; k < browptr[i + 1]; k++) {
            bp[nb].c = J[bcol[k]];
            bp[nb].k = k;
            nb++;
        }
        qsort(bp, (size_t)nb, sizeof(ent_t), cmp_ent);
    }
    int64_t cnt = 0;
    int64_t ka = rowptr[r], ea = rowptr[r + 1], kb = 0;
    while (ka < ea || kb < nb) {
        if (ka < ea && i >= 0 && op == ORC_OP_REPLACE && colpos[col[ka]] >= 0) {
            ka++;               /* block replace: A entries inside I x J are removed */
            continue;
        }
        int take_a = 0, take_b = 0;
        if (ka < ea && kb < nb) {
            if (col[ka] < bp[kb].c) take_a = 1;
            else if (col[ka] > bp[kb].c) take_b = 1;
            else take_a = take_b = 1;
        } else if (ka < ea) take_a = 1;
        else take_b = 1;
        if (out_col) {
            if (take_a && take_b) {
                out_col[cnt] = col[ka];
                if (op == ORC_OP_PLUS) add_vals(out_val, cnt, val, ka, bval, bp[kb].k, vsize);
                else copy_val(out_val, cnt, bval, bp[kb].k, vsize);   /* select-second */
            } else if (take_a) {
                out_col[cnt] = col[ka];
                copy_val(out_val, cnt, val, ka, vsize);
            } else {
                out_col[cnt] = bp[kb].c;
                copy_val(out_val, cnt, bval, bp[kb].k, vsize);
            }
        }
        cnt++;
        if (take_a) ka++;
        if (take_b) kb++;
    }
    return cnt;
}

int orc_spasgn(int64_t m, int64_t n, const int64_t *rowptr, const int32_t *col, const void *val,
               int vsize, int64_t bm, int64_t bn, const int64_t *browptr, const int32_t *bcol,
               const void *bval, const int32_t *I, int64_t nI, const int32_t *J, int64_t nJ,
               int op, const int64_t *rows, int64_t ns,
               int64_t *out_ptr, int32_t *out_col, void *out_val, int64_t cap, int64_t *need,
               int nthreads)
{
    if (vsize != 4 && vsize != 8) return ORC_INVALID_ARG;
    if (op != ORC_OP_SECOND && op != ORC_OP_PLUS && op != ORC_OP_REPLACE) return ORC_INVALID_ARG;
    if (bm != nI || bn != nJ) return ORC_SHAPE;
    int st = check_distinct(I, nI, m);
    if (st != ORC_OK) return st;
    st = check_distinct(J, nJ, n);
    if (st != ORC_OK) return st;
    /* Position of each row / column of A inside pvec / qvec (or -1). */
    int64_t *rowpos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    int64_t *colpos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!rowpos || !colpos) { free(rowpos); free(colpos); return ORC_INVALID_ARG; }
    int64_t maxb = 0;
    for (int64_t i = 0; i < bm; i++)
        if (browptr[i + 1] - browptr[i] > maxb) maxb = browptr[i + 1] - browptr[i];
    for (int64_t r = 0; r < m; r++) rowpos[r] = -1;
    for (int64_t c = 0; c < n; c++) colpos[c] = -1;
    for (int64_t i = 0; i < nI; i++) rowpos[I[i]] = i;
    for (int64_t j = 0; j < nJ; j++) colpos[J[j]] = j;
    asgn_ctx_t ctx = {rowptr, col, val, vsize, browptr, bcol, bval, J, rowpos, colpos, op};
    rowfn_t f = {asgn_row, &ctx, m, maxb, vsize};
    st = drive_rows(&f, rows, ns, out_ptr, out_col, out_val, cap, need, nthreads);
    free(rowpos);
    free(colpos);
    return st;
}
