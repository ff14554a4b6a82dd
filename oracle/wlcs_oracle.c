/*
 * Test infrastructure: the CPU oracle for alignment plots.
 *
 * Only the test suite, the smoke entry point and the CPU-baseline leg of the
 * benchmark load this library.  The product path never calls it, and this file
 * shares no code, header, table or helper with the HIP path.
 *
 * What it computes (Section 2 of Krusche & Tiskin, "Computing alignment plots
 * efficiently"): for strings x (length m) and y (length n) and a window length
 * w, the alignment plot is the matrix
 *
 *     WLCS(i, j) = LLCS(x_i .. x_{i+w-1}, y_j .. y_{j+w-1})
 *
 * for i in 1..m-w and j in 1..n-w (1-based, as the paper defines the plot), that
 * is, the length of a longest common subsequence of every pair of w-windows.
 * Stored 0-based: out[i*ld + j] holds WLCS(i+1, j+1) for 0 <= i < m-w,
 * 0 <= j < n-w.  With full_range != 0 the plot covers every window,
 * 0 <= i <= m-w and 0 <= j <= n-w.
 *
 * How: the paper's baseline, the standard dynamic program (Wagner-Fischer /
 * Needleman-Wunsch with LCS scores: match 1, mismatch 0, gap 0; Section 2),
 * run independently for every window pair, O(m n w^2) in total.  Nothing here
 * uses seaweeds: the oracle is the plain definition written out.
 *
 *     L[p][0] = L[0][q] = 0
 *     L[p][q] = L[p-1][q-1] + 1                  if a[p-1] == b[q-1]
 *             = max(L[p-1][q], L[p][q-1])        otherwise
 *     LLCS(a, b) = L[|a|][|b|]
 *
 * With step sizes hx, hy (Section 3: only windows starting at multiples of a
 * step are compared), oracle_wlcs_strided evaluates the same definition at the
 * x-windows r*hx and the y-windows c*hy only.
 *
 * Characters are compared as raw bytes.  Parallelism is over independent rows
 * of the plot only (plain POSIX threads, static partition); each entry is
 * evaluated by the recurrence above in its textbook order.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL -1
#define ORACLE_ENOMEM -2

/* LLCS of a (length la) and b (length lb) by the full (la+1) x (lb+1) table.
 * tab must hold (la+1)*(lb+1) ints.  Standard dynamic program, Section 2. */
static int llcs_table(const uint8_t *a, int la, const uint8_t *b, int lb, int *tab)
{
    const int cols = lb + 1;
    for (int q = 0; q <= lb; ++q) tab[q] = 0;          /* L[0][q] = 0 */
    for (int p = 1; p <= la; ++p) {
        tab[p * cols] = 0;                               /* L[p][0] = 0 */
        for (int q = 1; q <= lb; ++q) {
            int v;
            if (a[p - 1] == b[q - 1]) {
                v = tab[(p - 1) * cols + (q - 1)] + 1;
            } else {
                int up = tab[(p - 1) * cols + q];
                int left = tab[p * cols + (q - 1)];
                v = up > left ? up : left;
            }
            tab[p * cols + q] = v;
        }
    }
    return tab[la * cols + lb];
}

int oracle_llcs(const uint8_t *a, int64_t la, const uint8_t *b, int64_t lb)
{
    if (la < 0 || lb < 0 || (la > 0 && !a) || (lb > 0 && !b)) return ORACLE_EINVAL;
    if (la > 4096 || lb > 4096) return ORACLE_EINVAL;
    int *tab = (int *)malloc(sizeof(int) * (size_t)(la + 1) * (size_t)(lb + 1));
    if (!tab) return ORACLE_ENOMEM;
    int r = llcs_table(a, (int)la, b, (int)lb, tab);
    free(tab);
    return r;
}

/* Number of windows along a string of length len for window w: the paper's
 * plot takes len - w of them (i in 1..len-w); full_range takes all len - w + 1. */
static int64_t n_windows(int64_t len, int32_t w, int full_range)
{
    int64_t k = len - w + (full_range ? 1 : 0);
    return k > 0 ? k : 0;
}

typedef struct {
    const uint8_t *x, *y;
    int32_t w;
    int64_t rows, cols;
    const int64_t *row_ids;   /* NULL: rows 0..rows-1; else the listed x-windows */
    int64_t hx, hy;           /* steps: output (r, c) is x-window r*hx (or row_ids[r]), y-window c*hy */
    uint8_t *out;
    int64_t ld;
    int64_t r0, r1;           /* this worker's range of output rows */
} rows_job;

static void *rows_worker(void *arg)
{
    rows_job *jb = (rows_job *)arg;
    const int w = jb->w;
    int *tab = (int *)malloc(sizeof(int) * (size_t)(w + 1) * (size_t)(w + 1));
    if (!tab) return (void *)1;
    for (int64_t r = jb->r0; r < jb->r1; ++r) {
        int64_t i = jb->row_ids ? jb->row_ids[r] : r * jb->hx;
        for (int64_t c = 0; c < jb->cols; ++c)
            jb->out[r * jb->ld + c] = (uint8_t)llcs_table(jb->x + i, w, jb->y + c * jb->hy, w, tab);
    }
    free(tab);
    return NULL;
}

static int run_rows(const uint8_t *x, const uint8_t *y, int32_t w, int64_t rows, int64_t cols,
                    const int64_t *row_ids, int64_t hx, int64_t hy, uint8_t *out, int64_t ld,
                    int nthreads)
{
    if (rows == 0 || cols == 0) return ORACLE_OK;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (nthreads > rows) nthreads = (int)rows;
    rows_job jobs[256];
    pthread_t th[256];
    int started[256];
    int status = ORACLE_OK;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = (rows_job){x, y, w, rows, cols, row_ids, hx, hy, out, ld,
                             rows * t / nthreads, rows * (t + 1) / nthreads};
        started[t] = (t > 0) && pthread_create(&th[t], NULL, rows_worker, &jobs[t]) == 0;
        if (t > 0 && !started[t]) status = ORACLE_ENOMEM;
    }
    if (rows_worker(&jobs[0]) != NULL) status = ORACLE_ENOMEM;
    for (int t = 1; t < nthreads; ++t) {
        if (!started[t]) {
            if (rows_worker(&jobs[t]) != NULL) status = ORACLE_ENOMEM;
            continue;
        }
        void *ret = NULL;
        pthread_join(th[t], &ret);
        if (ret != NULL) status = ORACLE_ENOMEM;
    }
    return status;
}

/* Whole alignment plot into host memory out (rows x cols, row stride ld). */
int oracle_wlcs(const uint8_t *x, int64_t m, const uint8_t *y, int64_t n, int32_t w,
                int32_t full_range, uint8_t *out, int64_t ld, int32_t nthreads)
{
    if (m < 0 || n < 0 || w < 1 || w > 255) return ORACLE_EINVAL;
    int64_t rows = n_windows(m, w, full_range), cols = n_windows(n, w, full_range);
    if (rows == 0 || cols == 0) return ORACLE_OK;
    if (!x || !y || !out || ld < cols) return ORACLE_EINVAL;
    return run_rows(x, y, w, rows, cols, NULL, 1, 1, out, ld, nthreads);
}

/* The plot with step sizes (Section 3: only windows starting at multiples of
 * a step are compared): out[r*ld + c] = WLCS of x-window r*hx and y-window
 * c*hy (0-based starts), for the ceil(rows/hx) x ceil(cols/hy) such pairs,
 * rows and cols counted as in oracle_wlcs. */
int oracle_wlcs_strided(const uint8_t *x, int64_t m, const uint8_t *y, int64_t n, int32_t w,
                        int64_t hx, int64_t hy, int32_t full_range, uint8_t *out, int64_t ld,
                        int32_t nthreads)
{
    if (m < 0 || n < 0 || w < 1 || w > 255 || hx < 1 || hy < 1) return ORACLE_EINVAL;
    int64_t rows = n_windows(m, w, full_range), cols = n_windows(n, w, full_range);
    int64_t orows = (rows + hx - 1) / hx, ocols = (cols + hy - 1) / hy;
    if (orows == 0 || ocols == 0) return ORACLE_OK;
    if (!x || !y || !out || ld < ocols) return ORACLE_EINVAL;
    return run_rows(x, y, w, orows, ocols, NULL, hx, hy, out, ld, nthreads);
}

/* Selected rows of the plot: out row r holds x-window row_ids[r] against every
 * y-window (cols entries, stride ld). */
int oracle_wlcs_rows(const uint8_t *x, int64_t m, const uint8_t *y, int64_t n, int32_t w,
                     int32_t full_range, const int64_t *row_ids, int64_t nrows,
                     uint8_t *out, int64_t ld, int32_t nthreads)
{
    if (m < 0 || n < 0 || w < 1 || w > 255 || nrows < 0) return ORACLE_EINVAL;
    int64_t rows = n_windows(m, w, full_range), cols = n_windows(n, w, full_range);
    if (nrows == 0 || cols == 0) return ORACLE_OK;
    if (!x || !y || !out || !row_ids || ld < cols) return ORACLE_EINVAL;
    for (int64_t r = 0; r < nrows; ++r)
        if (row_ids[r] < 0 || row_ids[r] >= rows) return ORACLE_EINVAL;
    return run_rows(x, y, w, nrows, cols, row_ids, 1, 1, out, ld, nthreads);
}

/* Individual entries: out[k] = WLCS at (ii[k], jj[k]) (0-based window starts). */
int oracle_wlcs_at(const uint8_t *x, int64_t m, const uint8_t *y, int64_t n, int32_t w,
                   const int64_t *ii, const int64_t *jj, int64_t count, uint8_t *out)
{
    if (m < 0 || n < 0 || w < 1 || w > 255 || count < 0) return ORACLE_EINVAL;
    if (count == 0) return ORACLE_OK;
    if (!x || !y || !ii || !jj || !out) return ORACLE_EINVAL;
    int *tab = (int *)malloc(sizeof(int) * (size_t)(w + 1) * (size_t)(w + 1));
    if (!tab) return ORACLE_ENOMEM;
    for (int64_t k = 0; k < count; ++k) {
        if (ii[k] < 0 || jj[k] < 0 || ii[k] + w > m || jj[k] + w > n) {
            free(tab);
            return ORACLE_EINVAL;
        }
        out[k] = (uint8_t)llcs_table(x + ii[k], w, y + jj[k], w, tab);
    }
    free(tab);
    return ORACLE_OK;
}

/* ---- O-batch: the same recurrence for 64 neighbouring y-windows at once ----
 * oracle_wlcs_batch computes what oracle_wlcs computes, with the same dynamic
 * program for every window pair; only the loops over independent windows are
 * interchanged.  For one x-window a = x[i..i+w) and the y-windows
 * b_k = y[j0+k .. j0+k+w) (k < 64), the 64 tables are filled together, cell
 * by cell in the textbook order (row p = 1..w, then column q = 1..w), one
 * byte per window (every entry is at most w <= 255):
 *
 *     L_k[p][q] = L_k[p-1][q-1] + 1             if a[p-1] == b_k[q-1]
 *               = max(L_k[p-1][q], L_k[p][q-1])  otherwise
 *
 * Only the previous row of each table is kept (row p overwrites row p-1 from
 * left to right, the textbook space-saving form), with the entries
 * L_k[p-1][q-1] and L_k[p][q-1] carried along the row.  Letter q-1 of the 64
 * windows is y[j0+q-1 .. j0+q+63): one contiguous load, so the compiler turns
 * the loop over k into vector instructions.  The tests pin this function
 * equal to oracle_wlcs entry by entry. */
#define OB_LANES 64

__attribute__((target_clones("avx2", "default")))
static void batch_windows(const uint8_t *a, int w, const uint8_t *y, uint8_t *row, uint8_t *res)
{
    for (int q = 0; q <= w; ++q)
        for (int k = 0; k < OB_LANES; ++k) row[q * OB_LANES + k] = 0;  /* L[0][q] = 0 */
    for (int p = 1; p <= w; ++p) {
        const uint8_t ap = a[p - 1];
        uint8_t diag[OB_LANES], left[OB_LANES];
        for (int k = 0; k < OB_LANES; ++k) diag[k] = left[k] = 0;     /* L[p-1][0] = L[p][0] = 0 */
        for (int q = 1; q <= w; ++q) {
            uint8_t *up = row + q * OB_LANES;                           /* L[p-1][q], becomes L[p][q] */
            const uint8_t *bq = y + q - 1;                              /* b_k[q-1] = y[j0+k+q-1] */
            for (int k = 0; k < OB_LANES; ++k) {
                const uint8_t u = up[k];
                const uint8_t v = bq[k] == ap ? (uint8_t)(diag[k] + 1) : (u > left[k] ? u : left[k]);
                diag[k] = u;
                left[k] = v;
                up[k] = v;
            }
        }
    }
    for (int k = 0; k < OB_LANES; ++k) res[k] = row[w * OB_LANES + k];
}

typedef struct {
    const uint8_t *x, *ypad;
    int32_t w;
    int64_t cols;
    const int64_t *row_ids;
    uint8_t *out;
    int64_t ld;
    int64_t r0, r1;
    int status;
} batch_job;

static void *batch_worker(void *arg)
{
    batch_job *jb = (batch_job *)arg;
    const int w = jb->w;
    uint8_t *row = (uint8_t *)malloc((size_t)(w + 1) * OB_LANES);
    if (!row) {
        jb->status = ORACLE_ENOMEM;
        return NULL;
    }
    uint8_t res[OB_LANES];
    for (int64_t r = jb->r0; r < jb->r1; ++r) {
        const int64_t i = jb->row_ids ? jb->row_ids[r] : r;
        for (int64_t j0 = 0; j0 < jb->cols; j0 += OB_LANES) {
            batch_windows(jb->x + i, w, jb->ypad + j0, row, res);
            const int64_t nk = jb->cols - j0 < OB_LANES ? jb->cols - j0 : OB_LANES;
            memcpy(jb->out + r * jb->ld + j0, res, (size_t)nk);
        }
    }
    free(row);
    return NULL;
}

/* The plot rows of oracle_wlcs (row_ids NULL: every x-window; else out row r
 * holds x-window row_ids[r]) by O-batch. */
int oracle_wlcs_batch(const uint8_t *x, int64_t m, const uint8_t *y, int64_t n, int32_t w,
                      int32_t full_range, const int64_t *row_ids, int64_t nrows, uint8_t *out, int64_t ld,
                      int32_t nthreads)
{
    if (m < 0 || n < 0 || w < 1 || w > 255 || nrows < 0) return ORACLE_EINVAL;
    int64_t rows = n_windows(m, w, full_range), cols = n_windows(n, w, full_range);
    if (!row_ids) nrows = rows;
    if (nrows == 0 || cols == 0) return ORACLE_OK;
    if (!x || !y || !out || ld < cols) return ORACLE_EINVAL;
    if (row_ids)
        for (int64_t r = 0; r < nrows; ++r)
            if (row_ids[r] < 0 || row_ids[r] >= rows) return ORACLE_EINVAL;
    /* y with room for the last group's 64 lanes (their results are dropped) */
    uint8_t *ypad = (uint8_t *)calloc((size_t)n + OB_LANES, 1);
    if (!ypad) return ORACLE_ENOMEM;
    memcpy(ypad, y, (size_t)n);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (nthreads > nrows) nthreads = (int)nrows;
    batch_job jobs[256];
    pthread_t th[256];
    int started[256];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = (batch_job){x, ypad, w, cols, row_ids, out, ld, nrows * t / nthreads,
                              nrows * (t + 1) / nthreads, ORACLE_OK};
        started[t] = (t > 0) && pthread_create(&th[t], NULL, batch_worker, &jobs[t]) == 0;
    }
    batch_worker(&jobs[0]);
    int status = jobs[0].status;
    for (int t = 1; t < nthreads; ++t) {
        if (started[t]) pthread_join(th[t], NULL);
        else batch_worker(&jobs[t]);
        if (jobs[t].status != ORACLE_OK) status = jobs[t].status;
    }
    free(ypad);
    return status;
}

/* ---- alignment-score plots ----------------------------------------------
 * Section 2 also scores alignments with match 1, mismatch 0 and gap -1/2.  The
 * oracle computes that score directly by the standard dynamic program, kept in
 * half units so that everything stays integral:
 *     T[p][0] = -p,  T[0][q] = -q,
 *     T[p][q] = max(T[p-1][q-1] + 2 [a_p == b_q], T[p-1][q] - 1, T[p][q-1] - 1),
 *     score(a, b) = T[|a|][|b|] / 2.
 * (It does not use the '$' blow-up the paper reduces this score to.) */
static int score2_table(const uint8_t *a, int la, const uint8_t *b, int lb, int *tab)
{
    const int cols = lb + 1;
    for (int q = 0; q <= lb; ++q) tab[q] = -q;
    for (int p = 1; p <= la; ++p) {
        tab[p * cols] = -p;
        for (int q = 1; q <= lb; ++q) {
            int diag = tab[(p - 1) * cols + (q - 1)] + (a[p - 1] == b[q - 1] ? 2 : 0);
            int up = tab[(p - 1) * cols + q] - 1;
            int left = tab[p * cols + (q - 1)] - 1;
            int v = diag;
            if (up > v) v = up;
            if (left > v) v = left;
            tab[p * cols + q] = v;
        }
    }
    return tab[la * cols + lb];
}

/* Twice the alignment score of a and b (lengths <= 4096). */
int oracle_score2(const uint8_t *a, int64_t la, const uint8_t *b, int64_t lb, int32_t *out)
{
    if (la < 0 || lb < 0 || la > 4096 || lb > 4096 || !out || (la > 0 && !a) || (lb > 0 && !b))
        return ORACLE_EINVAL;
    int *tab = (int *)malloc(sizeof(int) * (size_t)(la + 1) * (size_t)(lb + 1));
    if (!tab) return ORACLE_ENOMEM;
    *out = score2_table(a, (int)la, b, (int)lb, tab);
    free(tab);
    return ORACLE_OK;
}

typedef struct {
    const uint8_t *x, *y;
    int32_t w, step;
    int64_t cols;
    int8_t *out;
    int64_t ld;
    int64_t r0, r1;
    int status;
} score_job;

static void *score_worker(void *arg)
{
    score_job *jb = (score_job *)arg;
    const int w = jb->w;
    int *tab = (int *)malloc(sizeof(int) * (size_t)(w + 1) * (size_t)(w + 1));
    if (!tab) {
        jb->status = ORACLE_ENOMEM;
        return NULL;
    }
    for (int64_t r = jb->r0; r < jb->r1; ++r) {
        const int64_t i = r * jb->step;
        for (int64_t j = 0; j < jb->cols; ++j)
            jb->out[r * jb->ld + j] = (int8_t)(score2_table(jb->x + i, w, jb->y + j, w, tab) / 2);
    }
    free(tab);
    return NULL;
}

/* Alignment-score plot with a vertical step: out row r holds the scores of the
 * x-window starting at r*step against every y-window (score of two w-windows
 * is an integer in [-w, w]; w <= 127).  Rows: the windows 0, step, 2*step, ...
 * below m - w (m - w + 1 with full_range); columns: n - w (n - w + 1). */
int oracle_score_plot(const uint8_t *x, int64_t m, const uint8_t *y, int64_t n, int32_t w, int32_t step,
                      int32_t full_range, int8_t *out, int64_t ld, int32_t nthreads)
{
    if (m < 0 || n < 0 || w < 1 || w > 127 || step < 1) return ORACLE_EINVAL;
    int64_t rows_all = n_windows(m, w, full_range), cols = n_windows(n, w, full_range);
    int64_t rows = rows_all > 0 ? (rows_all + step - 1) / step : 0;
    if (rows == 0 || cols == 0) return ORACLE_OK;
    if (!x || !y || !out || ld < cols) return ORACLE_EINVAL;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (nthreads > rows) nthreads = (int)rows;
    score_job jobs[256];
    pthread_t th[256];
    int started[256];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = (score_job){x, y, w, step, cols, out, ld, rows * t / nthreads, rows * (t + 1) / nthreads,
                              ORACLE_OK};
        started[t] = (t > 0) && pthread_create(&th[t], NULL, score_worker, &jobs[t]) == 0;
    }
    score_worker(&jobs[0]);
    int status = jobs[0].status;
    for (int t = 1; t < nthreads; ++t) {
        if (started[t]) pthread_join(th[t], NULL);
        else score_worker(&jobs[t]);
        if (jobs[t].status != ORACLE_OK) status = jobs[t].status;
    }
    return status;
}

